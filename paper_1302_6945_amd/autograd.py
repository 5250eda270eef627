"""torch.autograd.Function over the C ABI: forward = tikh_toeplitz_solve[_z],
backward = tikh_toeplitz_solve_backward[_z] (hand-written adjoint derived from
eq. (tiksol): one more solve of the same operator in normal form, then
FFT cross-correlations for the Toeplitz-generator gradient).  Only the
solution x is saved for backward; the recursion tree is recomputed."""
import torch

from . import _lib


class ToeplitzTikhonov(torch.autograd.Function):
    @staticmethod
    def forward(ctx, col, row, b, lam):
        lam_f = float(lam)
        x = _lib.solve(col.detach(), row.detach(), b.detach(), lam_f)
        ctx.save_for_backward(col.detach(), row.detach(), b.detach(), x)
        ctx.lam = lam_f
        ctx.lam_is_tensor = isinstance(lam, torch.Tensor)
        return x

    @staticmethod
    def backward(ctx, gx):
        col, row, b, x = ctx.saved_tensors
        g_col, g_row, g_b, g_lam = _lib.backward(col, row, b, ctx.lam, x, gx.contiguous())
        if not col.is_complex():
            g_col, g_row, g_b = g_col.real if g_col.is_complex() else g_col, g_row, g_b
        g_lam_out = g_lam.to(torch.float64) if ctx.lam_is_tensor else None
        return g_col, g_row, g_b, g_lam_out


def tikhonov_solve(col, row, b, lam):
    """Differentiable x = argmin ||T x - b||^2 + lam^2 ||x||^2 (GPU)."""
    return ToeplitzTikhonov.apply(col, row, b, lam)
