// Capture of two iterations as a HIP graph for ffd_iterate_graph.  Part of the
// single translation unit capi.hip.
#pragma once

#include "create.hpp"

namespace {

// Captures two iterations (so the two map buffers return to their roles) on
// the handle's own stream; history records are addressed through the device
// counter.  Host bookkeeping changed by the capture is restored.
ffd_status capture_graph(ffd_ctx* h) {
  if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  h->graph_exec = nullptr;
  h->graph = nullptr;
  h->graph_valid = false;
  if (!h->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  if (!h->k_dev) HIP_TRY(h->alloc(&h->k_dev, 1));
  const int cur0 = h->cur;
  const int64_t k0 = h->k;
  HIP_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  // the rotation (3D, h = 0: not read by the next iteration) is stored by the
  // second iteration only, so U is current after every replay
  one_iteration(h, h->cap_stream, nullptr, true, false, true);
  one_iteration(h, h->cap_stream, nullptr, true, true, true);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
  h->cur = cur0;
  h->k = k0;
  if (e != hipSuccess || !g) return fail(FFD_ERR_DEVICE, "graph capture failed");
  h->graph = g;
  HIP_TRY(hipGraphInstantiate(&h->graph_exec, g, nullptr, nullptr, 0));
  h->graph_cur = cur0;
  h->graph_hist = h->hist;
  h->graph_valid = true;
  return FFD_OK;
}

}  // namespace
