"""ln Z / N of the 4D Ising model as a differentiable torch function.

Forward: hotrg_init + `nsteps` coarse-graining steps (axes x, y, z, t in
turn) + hotrg_lnZ, with per-step checkpoints kept on the device.
Backward: hotrg_backward, the hand-written reverse pass through every step
(isometries and environments included), scaled by the incoming gradient.
Energy and magnetisation per site follow as e = -d(lnZ/N)/d beta and
m = (1/beta) d(lnZ/N)/d h.
"""
import torch

from . import hotrg as H


class HotrgLnZ(torch.autograd.Function):
    @staticmethod
    def forward(ctx, beta, h, dcut: int, nsteps: int, precision: int = H.FP64):
        ctx_h = H.Context(float(beta), float(h), int(dcut), precision=precision, keep_checkpoints=True,
                          impurities=False)
        for n in range(int(nsteps)):
            ctx_h.step(n % 4)
        lnz = ctx_h.lnz()
        ctx.hotrg = ctx_h
        return torch.tensor(lnz, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad):
        ctx_h = ctx.hotrg
        try:
            db, dh = ctx_h.backward()
        finally:
            ctx_h.close()
            ctx.hotrg = None
        g = grad.to(torch.float64)
        return g * db, g * dh, None, None, None


def lnz_per_site(beta, h, dcut: int, nsteps: int, precision: int = H.FP64):
    """beta, h: 0-dim float64 tensors (requires_grad as needed)."""
    return HotrgLnZ.apply(beta, h, dcut, nsteps, precision)
