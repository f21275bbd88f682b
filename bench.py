"""Benchmark of the flip-free ADMM iteration on one MI355X.

Default workload: the twisted tet cube, 64^3 cells x 6 Kuhn tets
(1,572,864 tets, 274,625 vertices), symmetric Dirichlet, rho = 10, float32
element steps and float64 factor / solve / sums.  One "step" is one full
ADMM iteration (W-step right-hand side, both triangular solves, fused
U/P/Lambda step, residual reduction) with all inputs resident in HBM.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "ADMM iters/s + local-step elems/s at 1.5M tets; fwd+bwd s/iter vs plain"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3  # MI355X published FP32 vector peak (packed / dual-issue)
FP32_NONPACKED_TFLOPS = 78.6  # 256 CUs x 64 lanes x 2 flop (FMA) x 2.4 GHz, one FP32 op per lane per cycle

# HBM bytes per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE runs
# (scaled by a plain copy of known size) on the benchmark workload, keyed by a
# hash of the kernel sources they were measured on: a changed kernel reports
# no traffic until it is measured again.
MEASURED_TRAFFIC = {
    # (source hash, element-step precision): per-iteration bytes and counters
    # (profiles/twisted_cube_64_hbm_traffic.md, profiles/twisted_cube_64_local_step_valu.md)
    ("599c8a08c6153d73", 32): {"solve": 3173.0e6, "local": 407.3e6, "local_flop_per_elem": 2258.2,
                           "local_valu_per_wave": 2628.1},
}


def kernel_source_hash() -> str:
    """Hash of every source under csrc/ (kernels, runtime and host set-up,
    which fixes the factor the solve streams)."""
    import hashlib
    h = hashlib.sha256()
    base = os.path.join(ROOT, "paper_2107_05200_amd", "csrc")
    files = sorted(os.path.relpath(os.path.join(d, f), base) for d, _, fs in os.walk(base) for f in fs
                   if f.endswith((".hip", ".hpp", ".cpp")))
    for rel in files:
        h.update(rel.encode())
        with open(os.path.join(base, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def local_step_bytes_per_element(d: int, prec: int, n: int, m: int, h_mode: int = 0, store_u: bool = False) -> float:
    """Unique HBM bytes of one fused local step per element, for the branch
    the kernel takes: reads T (d+1 int32), B (d^2), w, P (symmetric), Lambda
    (d^2), and the rotation U only where it is an input (2D: the tie rule;
    h_mode 1: the proximal term, which also reads |grad f(P)|^2); writes P,
    Lambda and the next right-hand side's corner vectors ((d+1) d), and U and
    |grad f(P)|^2 where they are stored (2D and h_mode 1 always, otherwise
    only on iterations whose state is kept: store_u); plus the two float64
    maps (W^k, W^{k-1}) read once per vertex."""
    r = prec // 8
    nU = 2 if d == 2 else 9
    nP = 3 if d == 2 else 6
    u_in = d == 2 or h_mode == 1
    u_out = u_in or store_u
    reads = 4 * (d + 1) + r * (d * d + 1 + nP + d * d) + (r * nU if u_in else 0) + (r if h_mode else 0)
    writes = r * (nP + d * d + (d + 1) * d) + (r * (nU + 1) if u_out else 0)
    maps = 2 * 8 * d * n / m
    return reads + writes + maps


def wrhs_bytes(d: int, prec: int, m: int, nF: int, n: int) -> float:
    """W-step right-hand side: CSR row pointers and (d+1) m incidence entries,
    the corner vectors once, the float64 result and the pinned-row copy."""
    r = prec // 8
    return 4 * (nF + 1) + 4 * (d + 1) * m + r * (d + 1) * d * m + 8 * d * nF + 8 * d * (n - nF)


def cpu_baseline(w, state, n_sample: int, passes: int):
    """The FP64 oracle's element steps (U, P, Lambda steps and diagnostics) on a
    sample of the workload's elements at the GPU's current state."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    import oracle as O

    rng = np.random.default_rng(0)
    start = int(rng.integers(0, max(1, w.m - n_sample)))
    sel = np.arange(start, min(w.m, start + n_sample))
    T = w.T[sel]
    verts, Tl = np.unique(T, return_inverse=True)
    Tl = Tl.reshape(T.shape).astype(np.int32)
    x = state["map"].cpu().numpy()[verts]
    U = state["U"].cpu().numpy().astype(np.float64)[sel]
    P = state["P"].cpu().numpy().astype(np.float64)[sel]
    L = state["Lam"].cpu().numpy().astype(np.float64)[sel]
    with threadpool_limits(limits=1):
        sub = O.OracleSolver(w.V[verts], Tl, w.energy, w.rho, np.array([0]), x[:1])
        times = []
        for _ in range(passes):
            sub.set_state(x, U, 0.5 * (P + np.transpose(P, (0, 2, 1))), L)
            t0 = time.perf_counter()
            sub.local_steps(x)
            times.append(time.perf_counter() - t0)
    t = min(times)
    return {"value": len(sel) / t, "unit": "local-step elems/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(sel)} contiguous elements of the {w.m:,}-element workload at the GPU state "
                      f"after the timed run; oracle element steps (U, P, Lambda, diagnostics), best of "
                      f"{passes} passes, 1 thread; factorising this L_FF takes the oracle minutes, "
                      f"beyond the benchmark budget, so whole oracle iterations are timed on smaller "
                      f"workloads (oracle_iterations; up to the tet cube at 32^3, an eighth of this one)",
            "host_cpu": _cpu_name(), "host_nproc": os.cpu_count()}


def oracle_iteration_rates():
    """The oracle's whole iterations (W-step with its factorised L_FF, element
    steps, diagnostics) beside the device's plain iterations of the same
    workloads (float64 and float32 element steps, as in the parity tests):
    the 32x32 height field, the sphere cap (501,126 triangles) and the tet
    cube at 16^3 and 32^3 (196,608 tets, an eighth of the benchmark cube).
    One thread; the oracle's first iteration (which factorises L_FF) is
    timed apart from the iterations after it."""
    import torch
    from threadpoolctl import threadpool_limits
    import oracle as O
    from paper_2107_05200_amd import binding, meshgen

    rows = {}
    for label, mk, k_cpu, k_gpu, prec in (
            ("height field UV, 1,922 triangles, SD", lambda: meshgen.height_field_uv(), 20, 200, 64),
            ("sphere cap UV, 501,126 triangles, SG", lambda: meshgen.sphere_cap_uv(), 3, 200, 32),
            ("twisted tet cube 16^3, 24,576 tets, SD", lambda: meshgen.twisted_cube(16), 5, 200, 32),
            ("twisted tet cube 32^3, 196,608 tets, SD", lambda: meshgen.twisted_cube(32), 2, 200, 32)):
        w = mk()
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            r = O.OracleSolver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos)
            r.init(w.x0)
            r.iterate(1)  # the first W-step factorises L_FF
            t1 = time.perf_counter()
            r.iterate(k_cpu)
            t2 = time.perf_counter()
        g = binding.Solver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, precision=prec)
        g.init(w.x0)
        g.iterate(5)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        g.iterate(k_gpu)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        g.close()
        cpu_it, gpu_it = (t2 - t1) / k_cpu, (t4 - t3) / k_gpu
        rows[label] = {"oracle_s_per_iter": cpu_it, "oracle_setup_and_first_iteration_s": t1 - t0,
                       "oracle_iters": k_cpu, "device_s_per_iter": gpu_it, "device_precision": prec,
                       "ratio": cpu_it / gpu_it}
        log(f"  oracle iterations, {label}: {cpu_it:.3g} s per iteration after {t1 - t0:.1f} s of set-up "
            f"and first iteration; device {gpu_it * 1e3:.3f} ms")
    return rows


def adjoint_leg(K: int = 100, every: int = 10, reps: int = 3):
    """Disk deformation (99,846 triangles, 16 handles): fwd+bwd seconds per
    iteration of the checkpointed adjoint divided by plain seconds per
    iteration (best of `reps` runs of each), both with the autotuned launch
    shapes; beside it the same with a checkpoint every iteration (every
    state kept, nothing recomputed)."""
    import torch
    from paper_2107_05200_amd import binding, meshgen
    w = meshgen.disk_deformation()
    s = binding.Solver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, precision=32)
    t0 = time.perf_counter()
    launch = s.init(w.V).autotune()
    tune = time.perf_counter() - t0
    s.init(w.V).iterate(10)
    s.init(w.V).adjoint_forward(10, every)
    s.adjoint_backward(energy_loss=True)
    torch.cuda.synchronize()
    plain, fb, fb1 = [], [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        s.init(w.V).iterate(K)
        torch.cuda.synchronize()
        plain.append((time.perf_counter() - t0) / K)
        t0 = time.perf_counter()
        s.init(w.V).adjoint_forward(K, every)
        pb, vb = s.adjoint_backward(energy_loss=True)
        torch.cuda.synchronize()
        fb.append((time.perf_counter() - t0) / K)
        # every state kept (a checkpoint per iteration): nothing recomputed
        t0 = time.perf_counter()
        s.init(w.V).adjoint_forward(K, 1)
        pb, vb = s.adjoint_backward(energy_loss=True)
        torch.cuda.synchronize()
        fb1.append((time.perf_counter() - t0) / K)
    # The dominant kernels of fwd+bwd are the triangular solves: one per
    # iteration of the forward pass, one per recomputed iteration (every - 1
    # of every `every`) and one per adjoint W-step (the same symmetric factor).  Their duration per solve
    # comes from the per-phase events of a profiled plain pass on this handle.
    ph = s.init(w.V).iterate_profiled(K)
    info = s.info()
    s.close()
    solve_ms = (ph["solve_fwd"] + ph["solve_bwd"]) / K
    solve_bytes = 2.0 * 8.0 * info["factor_nnz"]
    gbs = solve_bytes / (solve_ms * 1e-3) / 1e9
    solves_per_iter = 2.0 + (every - 1) / every  # forward, recomputed (every - 1 of every), adjoint
    roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "k_solve_fwd* + k_solve_bwd* (one solve of the disk's factor; fwd+bwd runs 2 + (every - 1) / every per iteration)",
            "algorithmic_bytes": solve_bytes, "ms_per_launch": round(solve_ms, 5),
            "solve_share_of_fwd_bwd": round(solves_per_iter * solve_ms * 1e-3 / min(fb), 4),
            "phase_ms_per_iter": {k: round(v / K, 5) for k, v in ph.items() if k != "total"}}
    return {"workload": f"disk deformation, {w.m:,} triangles, 16 handles, K={K}, checkpoint every {every}",
            "plain_s_per_iter": min(plain), "fwd_bwd_s_per_iter": min(fb), "ratio": min(fb) / min(plain),
            "fwd_bwd_s_per_iter_all_states_kept": min(fb1), "ratio_all_states_kept": min(fb1) / min(plain),
            "autotune_s": tune, "launch": launch, "factor_nnz": info["factor_nnz"], "roofline_solve": roof}


def batched_leg(iters: int = 200):
    """256 height-field charts (200..50k triangles, SD/SG mixed): one batched
    handle (autotuned, replayed graphs) vs the same charts run one handle at a
    time (default launch shapes, replayed graphs)."""
    import numpy as np
    import torch
    from paper_2107_05200_amd import binding, meshgen
    ws = meshgen.batched_charts()
    m = sum(w.m for w in ws)
    t0 = time.perf_counter()
    bs = binding.BatchSolver(ws, precision=32)
    setup = time.perf_counter() - t0
    x0 = np.concatenate([w.x0 for w in ws])
    bs.init(x0)
    t0 = time.perf_counter()
    launch = bs.autotune()
    tune = time.perf_counter() - t0
    bs.iterate(6, graph=True)
    torch.cuda.synchronize()
    bs.init(x0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bs.iterate(iters, graph=True)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    # the solve of the block-diagonal factor against HBM: per-phase events of a
    # profiled pass (each factor entry read once per pass)
    ph = bs.iterate_profiled(iters)
    info = bs.info()
    solve_ms = (ph["solve_fwd"] + ph["solve_bwd"]) / iters
    solve_bytes = 2.0 * 8.0 * info["factor_nnz"]
    gbs = solve_bytes / (solve_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": "k_solve_fwd* + k_solve_bwd* (block-diagonal factor of the 256 charts)",
            "algorithmic_bytes": solve_bytes, "ms_per_launch": round(solve_ms, 5),
            "phase_ms_per_iter": {k: round(v / iters, 5) for k, v in ph.items() if k != "total"}}
    bs.close()
    solvers = [binding.Solver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, precision=32) for w in ws]
    for s_, w in zip(solvers, ws):
        s_.init(w.x0).iterate(2, graph=True)
    torch.cuda.synchronize()
    for s_, w in zip(solvers, ws):
        s_.init(w.x0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s_ in solvers:
        s_.iterate(iters, graph=True)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    for s_ in solvers:
        s_.close()
    return {"workload": f"{len(ws)} height-field charts, {m:,} triangles total, SD/SG mixed, {iters} iterations",
            "batched_elem_iters_per_s": m * iters / tb, "plain_elem_iters_per_s": m * iters / tp,
            "speedup": tp / tb, "batched_ms_per_iter": tb / iters * 1e3, "setup_s": setup,
            "autotune_s": tune, "launch": launch, "factor_nnz": info["factor_nnz"], "roofline_solve": roof}


def uv_pipeline_leg(max_iter: int = 1000):
    """The paper's UV pipeline on the sphere cap (501,126 triangles, symmetric
    gradient): a Tutte initial map with the boundary on a circle, then
    Algorithm 2 with rescaling (rho_r = 5, refactorisation on the host) and
    the termination test every 10 iterations (1e-6, 1e-5, flip-free)."""
    import torch
    from paper_2107_05200_amd import binding, meshgen
    w = meshgen.sphere_cap_uv()
    idx, pos = meshgen.circle_boundary(w.V, w.T)
    binding.tutte_map(w.V, w.T, idx, pos)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    W0 = binding.tutte_map(w.V, w.T, idx, pos)
    torch.cuda.synchronize()
    t_tutte = time.perf_counter() - t0
    t0 = time.perf_counter()
    s = binding.Solver(w.V, w.T, w.energy, w.rho, idx[:1], pos[:1], precision=32)
    t_setup = time.perf_counter() - t0
    s.init(W0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, conv, nres = s.run(max_iter, check_every=10, eps_abs=1e-6, eps_rel=1e-5, flip_free=True, rescale_rho=5.0)
    torch.cuda.synchronize()
    t_run = time.perf_counter() - t0
    h = s.history()
    s.close()
    return {"workload": f"sphere cap UV, {w.m:,} triangles, SG, Tutte init, rescaling, max {max_iter} iterations",
            "tutte_s": t_tutte, "setup_s": t_setup, "run_s": t_run, "iterations": done, "converged": conv,
            "rescales": nres, "final_flips": int(h[-1, 5]), "final_E_map": float(h[-1, 3])}


def constraints_leg(iters: int = 200, rows: int = 48):
    """Disk deformation (99,846 triangles, 16 handles) with `rows` general
    constraint rows (vertex-on-segment, fixed-difference and centroid
    relations): seconds per replayed iteration with and without them (each
    handle autotuned)."""
    import numpy as np
    import torch
    from paper_2107_05200_amd import binding, meshgen
    w = meshgen.disk_deformation()
    rng = np.random.default_rng(48)
    v = rng.choice(np.setdiff1d(np.arange(w.n), w.pinned_idx), size=7 * (rows // 3), replace=False)
    A = np.zeros((rows, w.n))
    c = np.zeros((rows, 2))
    for i in range(rows // 3):
        a, b, c_ = v[7 * i:7 * i + 3]
        A[3 * i, [a, b, c_]] = [1.0, -0.5, -0.5]
        A[3 * i + 1, [v[7 * i + 3], v[7 * i + 4]]] = [1.0, -1.0]
        c[3 * i + 1] = w.V[v[7 * i + 3]] - w.V[v[7 * i + 4]]
        A[3 * i + 2, v[7 * i + 4:7 * i + 7]] = 1.0 / 3.0
        c[3 * i + 2] = w.V[v[7 * i + 4:7 * i + 7]].mean(axis=0)
    out = {}
    for name, con in (("plain", None), ("constrained", (A, c))):
        t0 = time.perf_counter()
        s = binding.Solver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, precision=32, constraints=con)
        setup = time.perf_counter() - t0
        s.init(w.V).autotune()
        s.init(w.V).iterate(10, graph=True)
        torch.cuda.synchronize()
        s.init(w.V)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.iterate(iters, graph=True)
        torch.cuda.synchronize()
        out[name] = {"ms_per_iter": (time.perf_counter() - t0) / iters * 1e3, "setup_s": setup}
        s.close()
    return {"workload": f"disk deformation, {w.m:,} triangles, 16 handles, {rows} constraint rows, {iters} iterations",
            **out, "ratio": out["constrained"]["ms_per_iter"] / out["plain"]["ms_per_iter"]}


def cube_leg(w, precision: int, steps: int, warmup: int, tune_cache=None, no_graph=False, leaf_size=0,
             keep=False):
    """The tet cube at one element-step precision: set-up, autotune, `warmup`
    replayed iterations, then `steps` iterations timed between two HIP events
    on the solver's stream, a second pass of `steps` iterations with per-phase
    events (the phase split and the kernels' average durations), and the
    per-level timing of the solve.  Returns (results, solver or None)."""
    import torch
    from paper_2107_05200_amd import binding
    t0 = time.perf_counter()
    s = binding.Solver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos, precision=precision,
                       leaf_size=leaf_size)
    setup_s = time.perf_counter() - t0
    info = s.info()
    log(f"[fp{precision}] setup {setup_s:.1f}s: factor nnz {info['factor_nnz']:.3e}, levels {info['n_levels']}, "
        f"numeric {info['t_numeric']:.1f}s, device {info['device_bytes'] / 2**30:.2f} GiB")
    stream = torch.cuda.current_stream()
    s.init(w.x0)
    t0 = time.perf_counter()
    launch = s.autotune(tune_cache)
    log(f"[fp{precision}] launch shapes {launch} ({time.perf_counter() - t0:.2f}s)")
    s.iterate(warmup, stream, graph=not no_graph)
    torch.cuda.synchronize()
    # timed region: K iterations between two HIP events on the solver's
    # stream (per-phase events add a few microseconds per phase, so the phase
    # split comes from a separate profiled pass)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    s.iterate(steps, stream, graph=not no_graph)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    K = steps
    total_ms = e0.elapsed_time(e1)
    ms_per_step = total_ms / K
    log(f"[fp{precision}] timed {K} iterations: {total_ms:.2f} ms events, {wall * 1e3:.2f} ms wall")
    ph = s.iterate_profiled(K, stream)
    torch.cuda.synchronize()
    log(f"[fp{precision}] profiled pass of {K} iterations: phases {ph}")
    levels = s.profile_solve_levels(10, stream)
    log(f"[fp{precision}] solve levels (fwd ms, bwd ms, MB, TB/s fwd, TB/s bwd):")
    for l, lv in enumerate(levels):
        log(f"  {l:2d} {lv['fwd_ms']:.4f} {lv['bwd_ms']:.4f} {lv['bytes'] / 1e6:8.1f} "
            f"{lv['bytes'] / lv['fwd_ms'] / 1e9:.2f} {lv['bytes'] / lv['bwd_ms'] / 1e9:.2f} nodes {int(lv['nodes'])}")
    hist = s.history()
    log(f"[fp{precision}] last history record: {dict(zip(binding.HIST_NAMES, hist[-1].tolist()))}")
    d, m, n, nF = w.d, w.m, w.n, info["n_free"]
    solve_ms = (ph["solve_fwd"] + ph["solve_bwd"]) / K
    local_ms = ph["local"] / K
    solve_bytes = 2.0 * 8.0 * info["factor_nnz"]  # each factor entry read once per pass
    # the profiled pass stores U and |grad f|^2 on its last iteration only
    lb = ((K - 1) * local_step_bytes_per_element(d, precision, n, m) +
          local_step_bytes_per_element(d, precision, n, m, store_u=True)) / K
    local_bytes = lb * m
    solve_gbs = solve_bytes / (solve_ms * 1e-3) / 1e9
    local_gbs = local_bytes / (local_ms * 1e-3) / 1e9
    standard = (w.meta.get("k"), leaf_size) == (64, 0)
    traffic = MEASURED_TRAFFIC.get((kernel_source_hash(), precision), {}) if standard else {}
    timing = "HIP events around each phase of a second pass of K iterations on the same stream"
    roof_solve = {"bound": "hbm", "achieved": round(solve_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": round(solve_gbs / HBM_PEAK_GBS, 4), "traffic": traffic.get("solve"),
                  "kernel": "k_solve_fwd* + k_solve_bwd* (one W-step solve, all levels)",
                  "algorithmic_bytes": solve_bytes, "ms_per_launch": round(solve_ms, 5), "timing": timing}
    roof_local = {"bound": "hbm", "achieved": round(local_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": round(local_gbs / HBM_PEAK_GBS, 4), "traffic": traffic.get("local"), "kernel": "k_local",
                  "algorithmic_bytes": local_bytes, "bytes_per_element": round(lb, 2),
                  "ms_per_launch": round(local_ms, 5), "timing": timing}
    roof_local_alu = None
    if traffic.get("local_flop_per_elem"):
        tf = traffic["local_flop_per_elem"] * m / (local_ms * 1e-3) / 1e12
        roof_local_alu = {"bound": "alu", "achieved": round(tf, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                          "frac": round(tf / FP32_PEAK_TFLOPS, 4),
                          "frac_nonpacked": round(tf / FP32_NONPACKED_TFLOPS, 4), "kernel": "k_local",
                          "flop_per_element": traffic["local_flop_per_elem"],
                          "valu_instructions_per_wave": traffic["local_valu_per_wave"],
                          "note": "flop = (ADD + MUL + 2 FMA + TRANS) x 64 from the SQ_INSTS_VALU_* counters; "
                                  "frac against the published 157.3 TFLOP/s, frac_nonpacked against 78.6 "
                                  "(one FP32 op per lane per cycle; packed FP32 is not generated)"}
    res = {
        "iters_per_s": round(1000.0 / ms_per_step, 2),
        "ms_per_step": round(ms_per_step, 5),
        "launch": launch,
        "free_vertices": nF,
        "local_step_elems_per_s": round(m / (local_ms * 1e-3), 1),
        "phase_ms_per_iter": {k: round(v / K, 5) for k, v in ph.items() if k != "total"},
        "setup_s": round(setup_s, 2),
        "factor": {"nnz": info["factor_nnz"], "levels": info["n_levels"], "numeric_s": round(info["t_numeric"], 2)},
        "roofline": roof_solve if solve_ms >= local_ms else roof_local,
        "roofline_local_step": roof_local,
        "roofline_local_step_alu": roof_local_alu,
        "roofline_solve": roof_solve,
        "wrhs_gbs": round(wrhs_bytes(d, precision, m, nF, n) / (ph["wrhs"] / K * 1e-3) / 1e9, 1),
        "solve_levels": [{"fwd_ms": round(lv["fwd_ms"], 5), "bwd_ms": round(lv["bwd_ms"], 5),
                          "MB": round(lv["bytes"] / 1e6, 2), "nodes": int(lv["nodes"]), "c_max": int(lv["c_max"]),
                          "r_max": int(lv["r_max"])} for lv in levels],
    }
    if not keep:
        s.close()
        s = None
    return res, s


def precision64_leg(w, steps: int, warmup: int, tune_cache=None):
    """The same cube with float64 element steps: the paper's arithmetic
    (IEEE double throughout)."""
    res, _ = cube_leg(w, 64, steps, warmup, tune_cache)
    keep = ("iters_per_s", "ms_per_step", "local_step_elems_per_s", "phase_ms_per_iter", "roofline_solve",
            "roofline_local_step", "launch")
    return {"dtype": "f64", **{k: res[k] for k in keep}}


def _oracle_fullsize_worker(k: int, iters: int, out_path: str):
    """Child process: the oracle's set-up and whole iterations (W-step with its
    factorised L_FF, element steps, diagnostics) on the k^3 tet cube, one
    thread; writes a JSON object to out_path."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    import oracle as O
    from paper_2107_05200_amd import meshgen
    w = meshgen.twisted_cube(k)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        r = O.OracleSolver(w.V, w.T, w.energy, w.rho, w.pinned_idx, w.pinned_pos)
        r.init(w.x0)
        r.iterate(1)  # the first W-step factorises L_FF
        t1 = time.perf_counter()
        r.iterate(iters)
        t2 = time.perf_counter()
    res = {"oracle_setup_and_first_iteration_s": t1 - t0, "oracle_s_per_iter": (t2 - t1) / iters,
           "oracle_iters_per_s": iters / (t2 - t1), "iterations_timed": iters, "threads": 1,
           "workload": f"twisted tet cube {k}^3 ({w.m:,} tets)", "E_P_after": float(r.history.col("E_P")[-1])}
    with open(out_path, "w") as f:
        json.dump(res, f)


def start_oracle_fullsize(k: int, iters: int = 2):
    """Start the oracle's full-size iterations in a child process (one core)
    so that its long factorisation overlaps the device legs."""
    import subprocess
    import tempfile
    path = os.path.join(tempfile.gettempdir(), f"ffd_oracle_fullsize_{os.getpid()}.json")
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    proc = subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-worker", str(k), str(iters), path],
                            env=env, stdout=subprocess.DEVNULL, stderr=subprocess.PIPE)
    log(f"oracle full-size iterations started (pid {proc.pid})")
    return proc, path, time.perf_counter()


def finish_oracle_fullsize(job, timeout_s: float):
    proc, path, t0 = job
    try:
        _, err = proc.communicate(timeout=max(1.0, timeout_s))
    except Exception:
        proc.kill()
        proc.communicate()
        return {"error": f"not finished within {timeout_s:.0f} s of waiting"}
    if proc.returncode != 0 or not os.path.exists(path):
        return {"error": f"worker exited with {proc.returncode}: {err.decode(errors='replace')[-300:]}"}
    with open(path) as f:
        res = json.load(f)
    os.remove(path)
    res["wall_s_since_start"] = time.perf_counter() - t0
    return res


def _cpu_name():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cube", type=int, default=64, help="cells per side of the tet cube")
    ap.add_argument("--precision", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=200000)
    ap.add_argument("--no-extra", action="store_true", help="skip the adjoint, batched, constraints and UV-pipeline legs")
    ap.add_argument("--tune-cache", default=None, help="launch-shape cache file (read, or written after tuning)")
    ap.add_argument("--no-graph", action="store_true", help="time direct launches instead of replayed HIP graphs")
    ap.add_argument("--leaf-size", type=int, default=0, help="nested-dissection leaf size (0: the library's default)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain elementwise copy (negation) of MIB MiB ten times (counter calibration)")
    ap.add_argument("--no-fp64", action="store_true", help="skip the float64 element-step line")
    ap.add_argument("--oracle-fullsize", action="store_true",
                    help="also time the oracle's whole iterations on the full cube (a child process on one core "
                         "started first; its factorisation takes minutes, so the run waits for it at the end)")
    ap.add_argument("--oracle-worker", nargs=3, metavar=("K", "ITERS", "OUT"), help=argparse.SUPPRESS)
    ap.add_argument("--leg", choices=("adjoint", "batched", "constraints", "uv_pipeline"), default=None,
                    help="run only this extra leg (no cube) and print its JSON (for profiling it alone)")
    args = ap.parse_args()
    if args.oracle_worker:
        _oracle_fullsize_worker(int(args.oracle_worker[0]), int(args.oracle_worker[1]), args.oracle_worker[2])
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU (the multi-GPU path is a design, not code); --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    # the oracle's child process starts before this process touches the GPU
    oracle_job = None
    if args.oracle_fullsize and not args.no_cpu_baseline and not args.calibrate_copy:
        oracle_job = start_oracle_fullsize(args.cube)

    import numpy as np
    import torch
    from paper_2107_05200_amd import binding, meshgen

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(10):
            torch.neg(src, out=dst)  # one elementwise kernel: reads and writes nbytes
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": nbytes, "calibrate_copy_bytes_written": nbytes,
                          "launches": 10}), flush=True)
        return
    if args.leg:
        fn = {"adjoint": adjoint_leg, "batched": batched_leg, "constraints": constraints_leg,
              "uv_pipeline": uv_pipeline_leg}[args.leg]
        print(json.dumps({"leg": args.leg, **fn()}), flush=True)
        return
    t0 = time.perf_counter()
    w = meshgen.twisted_cube(args.cube)
    log(f"workload {w.name}: m={w.m} n={w.n} pins={len(w.pinned_idx)} ({time.perf_counter() - t0:.1f}s)")
    main_leg, s = cube_leg(w, args.precision, args.steps, args.warmup, args.tune_cache, args.no_graph,
                           args.leaf_size, keep=True)
    K = args.steps
    m, n, nF = w.m, w.n, main_leg["free_vertices"]
    out = {
        "metric": METRIC,
        "value": main_leg["iters_per_s"],
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": main_leg["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 element steps + f64 solve" if args.precision == 32 else "f64",
        "data": "synthetic",
        "config": {"workload": f"twisted tet cube {args.cube}^3 x 6 Kuhn tets ({m:,} tets, {n:,} vertices), "
                               f"symmetric Dirichlet, rho=10, bottom fixed, top 45deg twist + 0.3 lift",
                   "elements": m, "vertices": n, "free_vertices": nF, "precision": args.precision,
                   "launch": main_leg["launch"]},
        "local_step_elems_per_s": main_leg["local_step_elems_per_s"],
        "fwd_bwd_s_per_iter_vs_plain": None,
        **{k: v for k, v in main_leg.items() if k not in ("iters_per_s", "ms_per_step", "launch", "free_vertices",
                                                            "local_step_elems_per_s")},
    }
    st = None
    if not args.no_cpu_baseline:
        st = {k: v.cpu() for k, v in s.get_state().items()}
        torch.cuda.synchronize()
    s.close()
    if not args.no_fp64:
        t0 = time.perf_counter()
        out["fp64"] = precision64_leg(w, K, args.warmup)
        log(f"fp64 line: {out['fp64']['iters_per_s']} iters/s ({time.perf_counter() - t0:.1f}s)")
    if not args.no_extra:
        t0 = time.perf_counter()
        adj = adjoint_leg()
        out["fwd_bwd_s_per_iter_vs_plain"] = round(adj["ratio"], 3)
        out["adjoint"] = adj
        log(f"adjoint leg: {adj} ({time.perf_counter() - t0:.1f}s)")
        t0 = time.perf_counter()
        out["batched"] = batched_leg()
        log(f"batched leg: {out['batched']} ({time.perf_counter() - t0:.1f}s)")
        t0 = time.perf_counter()
        out["constraints"] = constraints_leg()
        log(f"constraints leg: {out['constraints']} ({time.perf_counter() - t0:.1f}s)")
        t0 = time.perf_counter()
        out["uv_pipeline"] = uv_pipeline_leg()
        log(f"uv pipeline leg: {out['uv_pipeline']} ({time.perf_counter() - t0:.1f}s)")
    if st is not None:
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(w, st, args.cpu_sample, 3)
        log(f"cpu baseline {out['cpu_baseline']['value']:.0f} elems/s ({time.perf_counter() - t0:.1f}s)")
        t0 = time.perf_counter()
        out["cpu_baseline"]["oracle_iterations"] = oracle_iteration_rates()
        log(f"oracle iterations: {out['cpu_baseline']['oracle_iterations']} ({time.perf_counter() - t0:.1f}s)")
    if oracle_job is not None:
        t0 = time.perf_counter()
        full = finish_oracle_fullsize(oracle_job, 1800.0)
        full["device_s_per_iter"] = main_leg["ms_per_step"] * 1e-3
        if "oracle_s_per_iter" in full:
            full["ratio"] = full["oracle_s_per_iter"] / full["device_s_per_iter"]
        out.setdefault("cpu_baseline", {})["oracle_iterations_fullsize"] = full
        log(f"oracle full-size iterations: {full} (waited {time.perf_counter() - t0:.1f}s)")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
