"""torch.autograd.Function around the unrolled ADMM iterations.

``flip_free_energy(pins, V, T, ...)`` runs K iterations of the flip-free ADMM
from the identity map W^0 = V with the handles pinned at ``pins`` and returns
the final energy sum_i w_i f(P_i^K).  Its backward pass is the library's
hand-written adjoint (ffd_adjoint_backward), which recomputes the iterations
between device checkpoints taken every ``checkpoint_every`` iterations
(``checkpoint_every=1`` keeps every state and recomputes nothing).
"""
from __future__ import annotations

import numpy as np
import torch

from .binding import Solver


class FlipFreeEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pins, V, T, pinned_idx, energy, rho, K, checkpoint_every, precision):
        Vn = V.detach().to("cpu", torch.float64).numpy()
        pn = pins.detach().to("cpu", torch.float64).numpy()
        s = Solver(Vn, np.asarray(T), energy, rho, np.asarray(pinned_idx), pn, precision=precision)
        s.init(V.detach().to(s.device, torch.float64))
        s.adjoint_forward(int(K), int(checkpoint_every))
        loss = float(s.history(s.iteration() - 1, 1)[0, 2])
        ctx.solver = s
        ctx.devices = (pins.device, V.device)
        return torch.tensor(loss, dtype=torch.float64, device=V.device)

    @staticmethod
    def backward(ctx, gout):
        s = ctx.solver
        pb, vb = s.adjoint_backward(energy_loss=True)
        g = gout.to(torch.float64)
        gp = (pb * g.to(pb.device)).to(ctx.devices[0])
        gv = None if vb is None else (vb * g.to(vb.device)).to(ctx.devices[1])
        ctx.solver = None
        s.close()
        return gp, gv, None, None, None, None, None, None, None


def flip_free_energy(pins, V, T, pinned_idx, energy=0, rho=10.0, K=100, checkpoint_every=10, precision=32):
    """Final energy after K iterations; differentiable in pins and V."""
    return FlipFreeEnergy.apply(pins, V, T, pinned_idx, energy, rho, K, checkpoint_every, precision)
