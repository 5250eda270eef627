"""torch.autograd.Function over the C ABI: forward = tikh_toeplitz_solve[_z],
backward = tikh_toeplitz_solve_backward[_z] (hand-written adjoint derived from
eq. (tiksol): one more solve of the same operator in normal form, then FFT
cross-correlations for the Toeplitz-generator gradient).  Only the solution x
is saved for backward; the recursion tree is recomputed, not stored.
Gradients follow torch's complex convention dL/dRe + i dL/dIm."""
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
        ctx.dtypes = (col.dtype, row.dtype, b.dtype)
        return x

    @staticmethod
    def backward(ctx, gx):
        col, row, b, x = ctx.saved_tensors
        g_col, g_row, g_b, g_lam = _lib.backward(col, row, b, ctx.lam, x, gx.contiguous())
        outs = []
        for g, dt in zip((g_col, g_row, g_b), ctx.dtypes):
            outs.append(g.real if (g.is_complex() and not dt.is_complex) else g)
        return outs[0], outs[1], outs[2], (g_lam if ctx.lam_is_tensor else None)


def tikhonov_solve(col, row, b, lam):
    """Differentiable x = argmin ||T x - b||^2 + lam^2 ||x||^2 on the GPU."""
    return ToeplitzTikhonov.apply(col, row, b, lam)
