"""torch.autograd front end of the transmission and its adjoint.

forward: build the operator, solve the windows, combine and evaluate T(E)
(all in libtransec_gpu); backward: tsg_transmission_vjp with dL/dT as the
energy weights.  Differentiable inputs: the potential V (N,) and the
absorber parameters (amp_L, width_L, amp_R, width_R); the absorber centres,
the grid, the windows, the energies and the solver options are fixed.
"""
from __future__ import annotations

from typing import Optional, Sequence, Tuple

import numpy as np

from .binding import Operator, TsgOpts


def _fn():
    import torch

    class TransmissionFn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, V, absorber, grid, centres, windows, energies, opts):
            nx, ny, nz, h = grid
            aL, wL, aR, wR = [float(x) for x in absorber.detach().cpu().numpy()]
            oper = Operator(nx, ny, nz, h, V.detach().cpu().numpy().astype(np.float64),
                            (aL, wL, centres[0], aR, wR, centres[1]))
            oper.solve_all_partitions(windows, opts)
            E = np.asarray(energies, dtype=np.float64)
            T = oper.transmission(E)
            ctx.oper, ctx.E = oper, E
            ctx.V_meta = (V.dtype, V.device)
            ctx.a_meta = (absorber.dtype, absorber.device)
            return torch.tensor(T, dtype=torch.float64, device=V.device)

        @staticmethod
        def backward(ctx, gT):
            dV, dab = ctx.oper.transmission_vjp(ctx.E, gT.detach().cpu().numpy().astype(np.float64))
            ctx.oper.close()
            gV = torch.tensor(dV, dtype=ctx.V_meta[0], device=ctx.V_meta[1])
            ga = torch.tensor(dab, dtype=ctx.a_meta[0], device=ctx.a_meta[1])
            return gV, ga, None, None, None, None, None

    return TransmissionFn


_FN = None


def transmission(V, absorber, grid: Tuple[int, int, int, float], centres: Tuple[float, float],
                 windows: Sequence[Tuple[float, int]], energies: Sequence[float], opts: Optional[TsgOpts] = None):
    """T(E) as a differentiable function of V (torch float64, N) and
    absorber = torch.tensor([amp_L, width_L, amp_R, width_R])."""
    global _FN
    if _FN is None:
        _FN = _fn()
    return _FN.apply(V, absorber, tuple(grid), tuple(centres), list(windows), list(energies), opts)
