"""Seeded synthetic inputs shaped like the paper's experiments.

This module holds input construction only (random generators, b = T x_true +
noise, a power-iteration estimate of ||T||_2 for choosing lambda); it contains
none of the solver's arithmetic and is shared by the tests, the benchmark and
the oracle checks.  Every problem is generated on the host in FP64 from
np.random.SeedSequence([13026945, config, index]).

Toeplitz convention (paper Sec. 1, T = [a_{i-j}], m x n): col[i] = a_i for
i < m, row[j] = a_{-j} for 0 < j < n, row[0] = a_0.
"""
import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
from scipy.signal import fftconvolve

SEED = 13026945


def rng_for(config, index=0):
    return np.random.default_rng(np.random.SeedSequence([SEED, int(config), int(index)]))


def split_generator(a, m, n):
    """a holds a_s for s = -(n-1) .. m-1 (length m+n-1) -> (col, row)."""
    a = np.asarray(a)
    col = a[n - 1:].copy()
    row = a[:n][::-1].copy()
    return col, row


def toeplitz_matvec(col, row, x):
    """T x for the Toeplitz matrix given by (col, row); full-convolution slice."""
    col = np.asarray(col); row = np.asarray(row); x = np.asarray(x)
    m, n = len(col), len(row)
    g = np.concatenate([row[1:][::-1], col])        # a_{-(n-1)} .. a_{m-1}
    full = fftconvolve(g, x) if min(len(g), len(x)) > 64 else np.convolve(g, x)
    return full[n - 1:n - 1 + m]


def toeplitz_rmatvec(col, row, v):
    """T^H v (correlation)."""
    col = np.asarray(col); row = np.asarray(row); v = np.asarray(v)
    m, n = len(col), len(row)
    g = np.concatenate([row[1:][::-1], col])
    gr = np.conj(g[::-1])                            # conj(a_{m-1}) .. conj(a_{-(n-1)})
    full = fftconvolve(gr, v) if min(len(gr), len(v)) > 64 else np.convolve(gr, v)
    # (T^H v)_j = sum_i conj(a_{i-j}) v_i ; gr[q] = conj(a_{m-1-q})
    return full[m - 1:m - 1 + n]


def norm2_estimate(col, row, iters=50, seed=0):
    """||T||_2 by power iteration on T^H T (input construction for lambda paths)."""
    rng = np.random.default_rng(seed)
    n = len(row)
    v = rng.standard_normal(n)
    if np.iscomplexobj(col) or np.iscomplexobj(row):
        v = v + 1j * rng.standard_normal(n)
    v /= np.linalg.norm(v)
    s = 0.0
    for _ in range(iters):
        w = toeplitz_rmatvec(col, row, toeplitz_matvec(col, row, v))
        s = np.linalg.norm(w)
        if s == 0:
            return 0.0
        v = w / s
    return math.sqrt(s)


@dataclass
class Problem:
    col: np.ndarray
    row: np.ndarray
    b: List[np.ndarray]               # right-hand sides (each length m)
    lams: List[float]                 # regularization parameters
    x_true: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def m(self):
        return len(self.col)

    @property
    def n(self):
        return len(self.row)

    @property
    def is_complex(self):
        return np.iscomplexobj(self.col)


def envelope_generator(rng, m, n, L, cplx=False, cut=40.0):
    """a_s = z_s exp(-|s|/L), z_s ~ N(0,1) (complex: (u+iv)/sqrt 2), zero for |s| > cut*L."""
    s = np.arange(-(n - 1), m)
    if cplx:
        z = (rng.standard_normal(len(s)) + 1j * rng.standard_normal(len(s))) / math.sqrt(2.0)
    else:
        z = rng.standard_normal(len(s))
    a = z * np.exp(-np.abs(s) / L)
    a[np.abs(s) > cut * L] = 0.0
    return split_generator(a, m, n)


def config0(index=0):
    """m=384 x n=256 real T, a_s = N(0,1) exp(-|s|/32); x_true ~ N(0,1); b = T x + 0.01 N(0,1); lambda = 0.05."""
    rng = rng_for(0, index)
    m, n = 384, 256
    s = np.arange(-(n - 1), m)
    a = rng.standard_normal(len(s)) * np.exp(-np.abs(s) / 32.0)
    col, row = split_generator(a, m, n)
    x = rng.standard_normal(n)
    b = toeplitz_matvec(col, row, x) + 0.01 * rng.standard_normal(m)
    return Problem(col, row, [b], [0.05], x, dict(config=0))


def gaussian_psf(sigma, taps=None):
    taps = taps or 2 * int(math.ceil(4 * sigma)) + 1
    t = np.arange(taps)
    h = np.exp(-(t - (taps - 1) / 2.0) ** 2 / (2.0 * sigma ** 2))
    return h / h.sum()


def piecewise_constant(rng, n, jumps=64):
    x = np.zeros(n)
    pos = np.sort(rng.choice(np.arange(1, n), size=min(jumps, n - 1), replace=False))
    h = rng.standard_normal(len(pos))
    for p, v in zip(pos, h):
        x[p:] += v
    return x


def config1(n=2 ** 16, index=0, sigma=24.0, taps=193, lam=1e-2, noise=1e-3):
    """1-D deblurring: full convolution with a unit-sum Gaussian PSF (193 taps,
    sigma = 24 samples), m = n + 192; x_true piecewise constant with 64 jumps;
    b = T x + 1e-3 N(0,1); lambda = 1e-2."""
    rng = rng_for(1, index)
    h = gaussian_psf(sigma, taps)
    m = n + len(h) - 1
    col = np.zeros(m); col[:len(h)] = h
    row = np.zeros(n); row[0] = h[0]
    x = piecewise_constant(rng, n)
    b = toeplitz_matvec(col, row, x) + noise * rng.standard_normal(m)
    return Problem(col, row, [b], [lam], x, dict(config=1, sigma=sigma))


def config2(index, nrhs=4, nlam=8):
    """Batching law: n = round(2^U[9,14]), m = n + U{0..n/4}, envelope L ~ U[8,128]
    (hard cut at 40 L), 8 lambdas log-spaced 1e-4..1, 4 RHS built as in config 0."""
    rng = rng_for(2, index)
    n = int(round(2.0 ** rng.uniform(9, 14)))
    m = n + int(rng.integers(0, n // 4 + 1))
    L = rng.uniform(8, 128)
    col, row = envelope_generator(rng, m, n, L)
    x = rng.standard_normal(n)
    bs = [toeplitz_matvec(col, row, rng.standard_normal(n)) + 0.01 * rng.standard_normal(m) for _ in range(nrhs)]
    lams = [10.0 ** (-4 + 4 * j / 7.0) for j in range(nlam)]
    return Problem(col, row, bs, lams, x, dict(config=2, L=L))


def config3(n=2 ** 15, m=None, index=0, lam=0.02):
    """Complex T, a_s complex Gaussian with exp(-|s|/64) envelope (cut at 40*64),
    m = n + n/8; x_true ~ CN(0,1); b = T x + 0.01 CN(0,1); lambda = 0.02."""
    rng = rng_for(3, index)
    m = m if m is not None else n + n // 8
    col, row = envelope_generator(rng, m, n, 64.0, cplx=True)
    x = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / math.sqrt(2.0)
    e = (rng.standard_normal(m) + 1j * rng.standard_normal(m)) / math.sqrt(2.0)
    b = toeplitz_matvec(col, row, x) + 0.01 * e
    return Problem(col, row, [b], [lam], x, dict(config=3))


def config4(index):
    """Bilevel lambda tuning problem: Gaussian PSF sigma ~ U[4,48], n = round(2^U[12,16]),
    x_true and noise as in config 1, plus an independent validation draw."""
    rng = rng_for(4, index)
    sigma = rng.uniform(4, 48)
    h = gaussian_psf(sigma)
    n = int(round(2.0 ** rng.uniform(12, 16)))
    m = n + len(h) - 1
    col = np.zeros(m); col[:len(h)] = h
    row = np.zeros(n); row[0] = h[0]
    x = piecewise_constant(rng, n)
    Tx = toeplitz_matvec(col, row, x)
    b = Tx + 1e-3 * rng.standard_normal(m)
    bval = Tx + 1e-3 * rng.standard_normal(m)
    return Problem(col, row, [b, bval], [1e-2], x, dict(config=4, sigma=sigma))


def headline(index, n=2 ** 14, nrhs=4, nlam=8, m=None):
    """The n = 2^14 slice of the batching law: m = n + U{0..n/4}, envelope
    generator with L ~ U[8,128]; lambda path lam_j = s_max 10^(-3+3j/7) with
    s_max ~ ||T||_2 (power iteration, +1% margin), so that the regularized
    normal matrix has condition number <= 1 + 1e6; 4 RHS as in config 0."""
    rng = rng_for(5, index)
    m = m if m is not None else n + int(rng.integers(0, n // 4 + 1))
    L = rng.uniform(8, 128)
    col, row = envelope_generator(rng, m, n, L)
    x = rng.standard_normal(n)
    bs = [toeplitz_matvec(col, row, rng.standard_normal(n)) + 0.01 * rng.standard_normal(m) for _ in range(nrhs)]
    smax = 1.01 * norm2_estimate(col, row, iters=50, seed=index)
    lams = [smax * 10.0 ** (-3 + 3 * j / 7.0) for j in range(nlam)]
    return Problem(col, row, bs, lams, x, dict(config="H", L=L, smax=smax))


def replica(n, index=0):
    """Paper-shaped accuracy workload (Sec. 7.2): square T with complex standard
    normal generator, lambda^2 = sqrt(N) with N = 2n, known x, y = (T^H T + lambda^2 I) x."""
    rng = rng_for(6, index * 100003 + n)
    s = np.arange(-(n - 1), n)
    a = (rng.standard_normal(len(s)) + 1j * rng.standard_normal(len(s))) / math.sqrt(2.0)
    col, row = split_generator(a, n, n)
    lam = (2.0 * n) ** 0.25
    x = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) / math.sqrt(2.0)
    y = toeplitz_rmatvec(col, row, toeplitz_matvec(col, row, x)) + lam ** 2 * x
    return Problem(col, row, [y], [lam], x, dict(config="replica", normal_form=True))


def replica_gramian(n, index=0):
    """Paper-shaped accuracy workload of the Toeplitz-Gramian problem (Sec. 7.1-7.2): n x n
    Hermitian Toeplitz G with complex standard normal entries and main diagonal
    10 sqrt(N), N = 2n; L an n x n Toeplitz matrix with complex standard normal
    generator; known x; y = (G + L^H L) x."""
    rng = rng_for(7, index * 100003 + n)
    cn = lambda k: (rng.standard_normal(k) + 1j * rng.standard_normal(k)) / math.sqrt(2.0)
    gram = cn(n)
    gram[0] = 10.0 * math.sqrt(2.0 * n)
    s = np.arange(-(n - 1), n)
    lcol, lrow = split_generator(cn(len(s)), n, n)
    x = cn(n)
    grow = np.conj(gram)
    grow[0] = gram[0]
    y = toeplitz_matvec(gram, grow, x) + toeplitz_rmatvec(lcol, lrow, toeplitz_matvec(lcol, lrow, x))
    return GramianProblem(gram, lcol, lrow, [y], x, dict(config="replica_gramian"))


def replica_general(n, index=0):
    """Paper-shaped accuracy workload of the general problem (Sec. 7.1-7.2): n x n Toeplitz T
    and L with complex standard normal generators, known x, y = (T^H T + L^H L) x (normal
    form).  Returns (col, row, lcol, lrow, y, x)."""
    rng = rng_for(8, index * 100003 + n)
    cn = lambda k: (rng.standard_normal(k) + 1j * rng.standard_normal(k)) / math.sqrt(2.0)
    col, row = split_generator(cn(2 * n - 1), n, n)
    lcol, lrow = split_generator(cn(2 * n - 1), n, n)
    x = cn(n)
    y = toeplitz_rmatvec(col, row, toeplitz_matvec(col, row, x)) + \
        toeplitz_rmatvec(lcol, lrow, toeplitz_matvec(lcol, lrow, x))
    return col, row, lcol, lrow, y, x


def random_problem(rng, m, n, cplx=False, L=None):
    """Small random problem for parity sweeps (ragged sizes)."""
    s = np.arange(-(n - 1), m)
    a = rng.standard_normal(len(s)) + (1j * rng.standard_normal(len(s)) if cplx else 0.0)
    if L is not None:
        a = a * np.exp(-np.abs(s) / L)
    col, row = split_generator(a, m, n)
    b = rng.standard_normal(m) + (1j * rng.standard_normal(m) if cplx else 0.0)
    return col, row, b


@dataclass
class GramianProblem:
    """Toeplitz-Gramian problem (G + L^H L) x = y: gram = first column of the n x n Hermitian
    Toeplitz Gramian, (lcol, lrow) the p x n Toeplitz regularizer, ys right-hand sides."""
    gram: np.ndarray
    lcol: np.ndarray
    lrow: np.ndarray
    ys: List[np.ndarray]
    x_true: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def n(self):
        return len(self.gram)

    @property
    def p(self):
        return len(self.lcol)


def nufft_problem(index=0, n=4096, K=4096, lreg=1e4):
    """Reconstruction from non-uniform spectral samples (Sec. 7.4): x_true is a length-n sum of
    three real sinusoids with frequencies in [0, 0.02]; K sample frequencies f_k are drawn from the
    triangular distribution on [-1/2, 1/2) (mode 0); the Voronoi-cell widths of the sorted
    frequencies (period 1), in units of the uniform spacing 1/K (so a uniform grid has unit
    weights), weight the samples (regularized condition number about 1e7, as the paper reports
    for its example); the weighted Gramian A^H W A with
    A_{ks} = exp(-2 pi i f_k s) is Hermitian Toeplitz with first column g_d = sum_k w_k exp(2 pi i f_k d);
    L is the scaled second difference (2 lreg on the diagonal, -lreg beside it, p = n); the
    right-hand side is y = A^H W X for the exact samples X = A x_true."""
    rng = rng_for(7, index)
    fr = rng.uniform(0.0, 0.02, 3)
    ph = rng.uniform(0.0, 2 * math.pi, 3)
    amp = rng.standard_normal(3)
    s = np.arange(n)
    x = sum(a * np.cos(2 * math.pi * f * s + q) for a, f, q in zip(amp, fr, ph))
    fk = np.sort(rng.triangular(-0.5, 0.0, 0.5, K))
    fk[fk >= 0.5] -= 1.0
    fk = np.sort(fk)
    ext = np.concatenate([[fk[-1] - 1.0], fk, [fk[0] + 1.0]])
    w = 0.5 * K * (ext[2:] - ext[:-2])
    E = np.exp(-2j * math.pi * np.outer(fk, s))                 # A, K x n
    X = E @ x
    y = E.conj().T @ (w * X)
    gram = np.exp(2j * math.pi * np.outer(s, fk)) @ w           # g_d, d = 0 .. n-1
    lcol = np.zeros(n); lcol[0] = 2 * lreg; lcol[1] = -lreg
    lrow = np.zeros(n); lrow[0] = 2 * lreg; lrow[1] = -lreg
    return GramianProblem(gram, lcol, lrow, [y], x, dict(config="nufft", freqs=fr, K=K))


def random_gramian(rng, n, p, cplx=True, L=None):
    """Random Toeplitz-Gramian problem for parity sweeps: the Gramian of a random circulant
    (so that it is Toeplitz and positive semidefinite) and a random p x n Toeplitz L."""
    c = rng.standard_normal(n) + (1j * rng.standard_normal(n) if cplx else 0)
    if L is not None:
        c = c * np.exp(-np.minimum(np.arange(n), n - np.arange(n)) / L)
    ch = np.fft.fft(c)
    gram = np.fft.ifft(np.abs(ch) ** 2)                           # first column of C^H C
    if not cplx:
        gram = gram.real
    s = np.arange(-(n - 1), p)
    a = rng.standard_normal(len(s)) + (1j * rng.standard_normal(len(s)) if cplx else 0)
    if L is not None:
        a = a * np.exp(-np.abs(s) / L)
    lcol, lrow = split_generator(0.3 * a, p, n)
    y = rng.standard_normal(n) + (1j * rng.standard_normal(n) if cplx else 0)
    return GramianProblem(gram, lcol, lrow, [y], None, dict(config="gramian"))
