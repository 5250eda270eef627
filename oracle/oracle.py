"""ctypes binding of oracle/tikh_oracle.c (test infrastructure only).

Every function takes numpy arrays and works in complex FP64; real inputs are
promoted.  Toeplitz convention (paper Sec. 1, T = [a_{i-j}]): col[i] = a_i
(i < m), row[j] = a_{-j} (0 < j < n); row[0] is ignored.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tikh_oracle.c")
_LIB = os.path.join(_HERE, "libtikh_oracle.so")
_lib = None


def build(force=False):
    """Compile the C oracle with gcc (-O3 for loop vectorization, OpenMP; no target-specific flags)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.tikh_oracle_qr_solve.argtypes = [I64, I64, P, P, P, P, ctypes.c_double, P, ctypes.c_int]
        lib.tikh_oracle_qr_solve.restype = ctypes.c_int
        lib.tikh_oracle_T_apply.argtypes = [I64, I64, P, P, P, P]
        lib.tikh_oracle_TH_apply.argtypes = [I64, I64, P, P, P, P]
        lib.tikh_oracle_gradients.argtypes = [I64, I64, P, P, P, ctypes.c_double, P, P, P, P, P,
                                              ctypes.POINTER(ctypes.c_double), ctypes.c_int]
        lib.tikh_oracle_gradients.restype = ctypes.c_int
        lib.tikh_oracle_band_solve.argtypes = [I64, I64, P, P, I64, P, P, ctypes.c_double, P]
        lib.tikh_oracle_band_solve.restype = ctypes.c_int
        lib.tikh_oracle_band_solve_real.argtypes = [I64, I64, P, P, I64, P, P, ctypes.c_double, P]
        lib.tikh_oracle_band_solve_real.restype = ctypes.c_int
        lib.tikh_oracle_lag_sums.argtypes = [I64, I64, P, P, P, P, P, P]
        _lib = lib
    return _lib


def _c(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _threads(nthreads):
    return int(nthreads) if nthreads else 1


def solve(col, row, b, lam, nthreads=1):
    """x = argmin ||Tx - b||^2 + lam^2 ||x||^2 by dense Householder QR of [T; lam I]."""
    col, row, b = _c(col), _c(row), _c(b)
    m, n = len(col), len(row)
    assert len(b) == m
    x = np.zeros(n, np.complex128)
    st = _load().tikh_oracle_qr_solve(m, n, _p(col), _p(row), _p(b), None, float(lam), _p(x), _threads(nthreads))
    if st != 0:
        raise RuntimeError("oracle QR failed with status %d" % st)
    return x


def solve_normal(col, row, y, lam, nthreads=1):
    """x = (T^H T + lam^2 I)^{-1} y, as least squares of [T; lam I] x ~ [0; y/lam]."""
    col, row, y = _c(col), _c(row), _c(y)
    m, n = len(col), len(row)
    assert len(y) == n
    d = _c(y / float(lam))
    x = np.zeros(n, np.complex128)
    st = _load().tikh_oracle_qr_solve(m, n, _p(col), _p(row), None, _p(d), float(lam), _p(x), _threads(nthreads))
    if st != 0:
        raise RuntimeError("oracle QR failed with status %d" % st)
    return x


def band_solve(col, row, rhs, lam, normal=False):
    """Least-squares solutions by banded QR (Givens rotations; exact for generators of finite support).

    rhs: one vector or a list of vectors sharing (T, lam): right-hand sides b (m entries), or with
    normal=True normal-form data y (n entries, x = (T^H T + lam^2 I)^{-1} y).  Returns an array
    [len(rhs)][n] (or [n] for a single vector).  Real data runs the real-arithmetic variant."""
    single = np.ndim(rhs[0]) == 0
    vecs = [rhs] if single else list(rhs)
    m, n = len(col), len(row)
    real = not (np.iscomplexobj(col) or np.iscomplexobj(row) or any(np.iscomplexobj(v) for v in vecs))
    dt = np.float64 if real else np.complex128
    colc = np.ascontiguousarray(np.asarray(col, dtype=dt))
    rowc = np.ascontiguousarray(np.asarray(row, dtype=dt))
    if normal:
        assert all(len(v) == n for v in vecs)
        top, bot = None, np.ascontiguousarray(np.stack([np.asarray(v, dtype=dt) / float(lam) for v in vecs]))
    else:
        assert all(len(v) == m for v in vecs)
        top, bot = np.ascontiguousarray(np.stack([np.asarray(v, dtype=dt) for v in vecs])), None
    x = np.zeros((len(vecs), n), dt)
    fn = _load().tikh_oracle_band_solve_real if real else _load().tikh_oracle_band_solve
    st = fn(m, n, _p(colc), _p(rowc), len(vecs), _p(top), _p(bot), float(lam), _p(x))
    if st != 0:
        raise RuntimeError("oracle banded QR failed with status %d" % st)
    return x[0] if single else x


def band_gradients(col, row, b, lam, x, gx, with_lag_sums=True):
    """Gradients of a loss through x = solve(col, row, b, lam) (eq. (tiksol)) with the banded QR:
    w = (T^H T + lam^2 I)^{-1} gx, g_b = T w, g_lam = -2 lam Re<w, x>, and (optionally, O(mn))
    the lag sums of (b - T x) w^H - (T w) x^H.  x is the forward solution the gradient is taken at."""
    col, row, b, x, gx = _c(col), _c(row), _c(b), _c(x), _c(gx)
    m, n = len(col), len(row)
    w = _c(band_solve(col, row, [gx], lam, normal=True)[0])
    Tw = T_apply(col, row, w)
    out = dict(w=w, g_b=Tw, g_lam=float(-2.0 * lam * np.vdot(w, x).real))
    if with_lag_sums:
        gcol, grow = lag_sums(col, row, b, x, w)
        out.update(g_col=gcol, g_row=grow)
    return out


def lag_sums(col, row, b, x, w):
    """Generator gradient of the adjoint: lag sums of (b - T x) w^H - (T w) x^H written out (O(mn))."""
    col, row, b, x, w = _c(col), _c(row), _c(b), _c(x), _c(w)
    m, n = len(col), len(row)
    r = b - T_apply(col, row, x)
    Tw = T_apply(col, row, w)
    gcol = np.zeros(m, np.complex128)
    grow = np.zeros(n, np.complex128)
    _load().tikh_oracle_lag_sums(m, n, _p(r), _p(w), _p(Tw), _p(x), _p(gcol), _p(grow))
    return gcol, grow


def gramian_solve(gram, lcol, lrow, y):
    """Toeplitz-Gramian problem (Sec. 2, third case; Sec. 3.4): x = (G + L^H L)^{-1} y, where G is
    the n x n Hermitian Toeplitz Gramian with first column gram (G[r][s] = gram[r-s] for r >= s,
    conj(gram[s-r]) otherwise) and L the p x n Toeplitz regularizer (lcol[i] = l_i, lrow[j] = l_{-j}).
    The matrix G + L^H L is formed densely and solved by LAPACK (numpy.linalg.solve)."""
    gram, lcol, lrow, y = _c(gram), _c(lcol), _c(lrow), _c(y)
    n = len(gram)
    assert len(lrow) == n and len(y) == n
    G = np.empty((n, n), np.complex128)
    for r in range(n):
        G[r, :r + 1] = gram[r::-1]
        G[r, r + 1:] = np.conj(gram[1:n - r])
    L = dense_T(lcol, lrow)
    return np.linalg.solve(G + L.conj().T @ L, y)


def T_apply(col, row, v):
    col, row, v = _c(col), _c(row), _c(v)
    m, n = len(col), len(row)
    y = np.zeros(m, np.complex128)
    _load().tikh_oracle_T_apply(m, n, _p(col), _p(row), _p(v), _p(y))
    return y


def TH_apply(col, row, v):
    col, row, v = _c(col), _c(row), _c(v)
    m, n = len(col), len(row)
    y = np.zeros(n, np.complex128)
    _load().tikh_oracle_TH_apply(m, n, _p(col), _p(row), _p(v), _p(y))
    return y


def gradients(col, row, b, lam, gx, nthreads=1):
    """Returns dict(x, g_b, g_col, g_row, g_lam) for loss gradient gx = dL/dRe x + i dL/dIm x."""
    col, row, b, gx = _c(col), _c(row), _c(b), _c(gx)
    m, n = len(col), len(row)
    x = np.zeros(n, np.complex128)
    gb = np.zeros(m, np.complex128)
    gcol = np.zeros(m, np.complex128)
    grow = np.zeros(n, np.complex128)
    glam = ctypes.c_double(0.0)
    st = _load().tikh_oracle_gradients(m, n, _p(col), _p(row), _p(b), float(lam), _p(gx), _p(x), _p(gb),
                                       _p(gcol), _p(grow), ctypes.byref(glam), _threads(nthreads))
    if st != 0:
        raise RuntimeError("oracle gradient failed with status %d" % st)
    return dict(x=x, g_b=gb, g_col=gcol, g_row=grow, g_lam=glam.value)


def dense_T(col, row):
    """The m x n Toeplitz matrix T = [a_{i-j}] written out (small sizes only)."""
    col, row = _c(col), _c(row)
    m, n = len(col), len(row)
    T = np.empty((m, n), np.complex128)
    for i in range(m):
        for j in range(n):
            T[i, j] = col[i - j] if i >= j else row[j - i]
    return T


def normal_residual_fft(col, row, b, lam, x):
    """The same relative residual with the products T v and T^H v formed by numpy FFT
    convolutions of the generator (for full sizes)."""
    col, row, b, x = _c(col), _c(row), _c(b), _c(x)
    m, n = len(col), len(row)
    g = np.concatenate([row[1:][::-1], col])              # a_{-(n-1)} .. a_{m-1}
    L = 1
    while L < len(g) + max(m, n):
        L *= 2
    G = np.fft.fft(g, L)
    GH = np.fft.fft(np.conj(g[::-1]), L)                   # conj(a_{m-1}) .. conj(a_{-(n-1)})

    def T(v):
        return np.fft.ifft(G * np.fft.fft(v, L))[n - 1:n - 1 + m]

    def TH(v):
        return np.fft.ifft(GH * np.fft.fft(v, L))[m - 1:m - 1 + n]

    r = TH(b - T(x)) - float(lam) ** 2 * x
    scale = np.linalg.norm(TH(b)) + float(lam) ** 2 * np.linalg.norm(x)
    return float(np.linalg.norm(r) / scale)


def normal_residual(col, row, b, lam, x):
    """Relative residual of the optimality condition T^H (b - T x) = lam^2 x."""
    r = TH_apply(col, row, _c(b) - T_apply(col, row, x)) - float(lam) ** 2 * _c(x)
    scale = np.linalg.norm(TH_apply(col, row, b)) + float(lam) ** 2 * np.linalg.norm(x)
    return float(np.linalg.norm(r) / scale)


def general_solve(col, row, lcol, lrow, b):
    """The general problem (Sec. 2 eq. (tik) with a Toeplitz Tikhonov matrix L, p x n; Sec. 3.2):
    x = argmin ||T x - b||^2 + ||L x||^2, i.e. the least-squares solution of the stacked system
    [T; L] x = [b; 0], written out densely and solved by numpy.linalg.lstsq (small sizes only).
    (lcol, lrow) follow the Toeplitz convention of T: lcol[i] = l_i (i < p), lrow[j] = l_{-j}."""
    T, L = dense_T(col, row), dense_T(lcol, lrow)
    A = np.vstack([T, L])
    rhs = np.concatenate([_c(b), np.zeros(L.shape[0], np.complex128)])
    return np.linalg.lstsq(A, rhs, rcond=None)[0]


def general_solve_normal(col, row, lcol, lrow, y):
    """Normal form of the general problem (Sec. 7.1): x = (T^H T + L^H L)^{-1} y, the Gramians
    formed densely and the system solved by numpy.linalg.solve (small sizes only)."""
    T, L = dense_T(col, row), dense_T(lcol, lrow)
    return np.linalg.solve(T.conj().T @ T + L.conj().T @ L, _c(y))
