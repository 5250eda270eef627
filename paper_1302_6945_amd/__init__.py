"""MI355X (gfx950) superfast Tikhonov-regularized Toeplitz least squares.

Thin Python binding of the C ABI in include/tikh.h (libtikh.so, built from
paper_1302_6945_amd/csrc by paper_1302_6945_amd/build.py).  The binding only
marshals arguments: every step of the solve runs in the HIP kernels of the
library.  PyTorch supplies device memory and the current stream.  There is no
CPU fallback: importing this package raises if the library is missing.

Paper: Turnes, Balcan, Romberg, "Superfast Tikhonov Regularization of Toeplitz
Systems" (Sec. 2 eq. (tik)/(tiksol) with L = lambda I).
"""
from ._lib import (TikhError, lib, library_path, set_options, get_options, get_stats, plan_info, fft_batched, autotune_nlim,
                   profile_kernel, profile_read,
                   tikh_toeplitz_solve, tikh_toeplitz_solve_z, tikh_toeplitz_solve_normal,
                   tikh_toeplitz_solve_normal_z, tikh_toeplitz_solve_batched,
                   tikh_toeplitz_solve_batched_noalloc, solve_batched_noalloc,
                   tikh_gramian_solve, tikh_gramian_solve_z, tikh_gramian_solve_batched, gramian_solve,
                   gramian_solve_batched,
                   tikh_toeplitz_solve_backward, tikh_toeplitz_solve_backward_z,
                   tikh_toeplitz_solve_backward_batched, solve, solve_normal, solve_batched,
                   backward, backward_batched, workspace_bytes, set_workspace,
                   PreparedBatch, prepare_batched, prepare_backward_batched,
                   tikh_prepare_batched, tikh_prepare_backward_batched, tikh_prepared_run, tikh_prepared_free)
from .autograd import ToeplitzTikhonov, tikhonov_solve
from .bilevel import BilevelTuner

__all__ = ["workspace_bytes", "set_workspace", "TikhError", "lib", "library_path", "set_options", "get_options", "get_stats", "plan_info", "fft_batched", "autotune_nlim", "profile_kernel", "profile_read",
           "tikh_toeplitz_solve", "tikh_toeplitz_solve_z", "tikh_toeplitz_solve_normal",
           "tikh_toeplitz_solve_normal_z", "tikh_toeplitz_solve_batched",
           "tikh_toeplitz_solve_batched_noalloc", "solve_batched_noalloc",
           "tikh_gramian_solve", "tikh_gramian_solve_z", "tikh_gramian_solve_batched", "gramian_solve",
           "gramian_solve_batched",
           "tikh_toeplitz_solve_backward", "tikh_toeplitz_solve_backward_z",
           "tikh_toeplitz_solve_backward_batched", "solve", "solve_normal", "solve_batched",
           "backward", "backward_batched", "ToeplitzTikhonov", "tikhonov_solve",
           "PreparedBatch", "prepare_batched", "prepare_backward_batched", "tikh_prepare_batched",
           "tikh_prepare_backward_batched", "tikh_prepared_run", "tikh_prepared_free", "BilevelTuner"]
