"""CPU oracle for the l2 Tikhonov-regularized Toeplitz least-squares solve.

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py, never by the product package.  See
oracle/tikh_oracle.c for what it computes (dense Householder QR of the stacked
system [T; lambda I], the plain definition of eq. (tiksol) with L = lambda I;
band_solve is the same least-squares problem by a banded QR, for generators of
finite support at sizes the dense QR cannot reach; gramian_solve is the
Toeplitz-Gramian problem (G + L^H L) x = y written out densely; general_solve
is the general problem min ||Tx - b||^2 + ||Lx||^2 with a Toeplitz L, the
stacked least-squares system written out densely).
"""
from .oracle import (build, solve, solve_normal, gradients, T_apply, TH_apply,
                     dense_T, normal_residual, normal_residual_fft, band_solve,
                     band_gradients, lag_sums, gramian_solve, general_solve, general_solve_normal)

__all__ = ["build", "solve", "solve_normal", "gradients", "T_apply", "TH_apply",
           "dense_T", "normal_residual", "normal_residual_fft", "band_solve",
           "band_gradients", "lag_sums", "gramian_solve", "general_solve", "general_solve_normal"]
