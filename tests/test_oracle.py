"""Pins for the CPU oracle (dense Householder QR of [T; lambda I]).

Each test checks the oracle against something the paper or the mathematics
fixes independently of the oracle's own code: exact rational arithmetic on tiny
inputs, 50-digit normal equations, the circulant closed form (Fourier domain),
special cases, the scaling law, the large-lambda limit, an independent library
least-squares routine and the optimality condition of eq. (tik)/(tiksol).
"""
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle
import workloads as W


def test_T_matches_definition():
    # Sec. 1: T = [a_{i-j}]; col holds a_0..a_{m-1}, row holds a_0, a_{-1}, ...
    col = np.array([10, 11, 12, 13]); row = np.array([10, 21, 22])
    T = oracle.dense_T(col, row).real
    expect = np.array([[10, 21, 22], [11, 10, 21], [12, 11, 10], [13, 12, 11]])
    assert np.array_equal(T, expect)


def _exact_solution(T_int, b_int, lam2):
    """Exact rational solve of (T^T T + lam2 I) x = T^T b by Gaussian elimination."""
    m, n = len(T_int), len(T_int[0])
    A = [[sum(Fraction(T_int[k][i]) * T_int[k][j] for k in range(m)) + (lam2 if i == j else 0)
          for j in range(n)] for i in range(n)]
    y = [sum(Fraction(T_int[k][i]) * b_int[k] for k in range(m)) for i in range(n)]
    for c in range(n):
        p = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[p] = A[p], A[c]; y[c], y[p] = y[p], y[c]
        for r in range(n):
            if r != c and A[r][c] != 0:
                f = A[r][c] / A[c][c]
                A[r] = [A[r][k] - f * A[c][k] for k in range(n)]
                y[r] -= f * y[c]
    return [y[i] / A[i][i] for i in range(n)]


@pytest.mark.parametrize("m,n", [(3, 2), (2, 3), (5, 5), (6, 4), (4, 7), (1, 1), (1, 3), (3, 1)])
def test_exact_rational_bruteforce(m, n):
    rng = np.random.default_rng(100 * m + n)
    col = rng.integers(-5, 6, size=m); row = rng.integers(-5, 6, size=n); row[0] = col[0]
    b = rng.integers(-5, 6, size=m)
    lam2 = Fraction(3, 4)
    T = [[int(col[i - j]) if i >= j else int(row[j - i]) for j in range(n)] for i in range(m)]
    xe = np.array([float(v) for v in _exact_solution(T, [int(v) for v in b], lam2)])
    x = oracle.solve(col, row, b, float(lam2) ** 0.5)
    assert np.abs(x.imag).max() == 0.0
    np.testing.assert_allclose(x.real, xe, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("m,n", [(5, 3), (3, 5), (6, 6), (8, 2)])
def test_mpmath_complex_bruteforce(m, n):
    rng = np.random.default_rng(7 * m + n)
    col = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    row = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    b = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    lam = 0.3
    mpmath.mp.dps = 50
    T = mpmath.matrix(m, n)
    for i in range(m):
        for j in range(n):
            v = col[i - j] if i >= j else row[j - i]
            T[i, j] = mpmath.mpc(v.real, v.imag)
    TH = T.transpose_conj()
    A = TH * T + lam ** 2 * mpmath.eye(n)
    bb = mpmath.matrix([mpmath.mpc(v.real, v.imag) for v in b])
    xe = mpmath.lu_solve(A, TH * bb)
    xe = np.array([complex(xe[i]) for i in range(n)])
    x = oracle.solve(col, row, b, lam)
    np.testing.assert_allclose(x, xe, rtol=1e-12, atol=1e-13)
    # mutation check: the transposed or conjugated operand must be rejected by this pin
    x_bad = oracle.solve(np.conj(col), np.conj(row), b, lam)
    assert np.abs(x_bad - xe).max() > 1e-6


@pytest.mark.parametrize("n", [16, 64, 257])
@pytest.mark.parametrize("cplx", [False, True])
def test_circulant_closed_form(n, cplx):
    """Circulant T (m = n, a_{-j} = a_{n-j}): the Fourier-domain closed form
    x = IDFT(conj(a^) b^ / (|a^|^2 + lambda^2))."""
    rng = np.random.default_rng(n + 1000 * cplx)
    c = rng.standard_normal(n) + (1j * rng.standard_normal(n) if cplx else 0)
    col = c.copy(); row = np.array([c[(n - j) % n] for j in range(n)])
    b = rng.standard_normal(n) + (1j * rng.standard_normal(n) if cplx else 0)
    lam = 0.4
    ah = np.fft.fft(c); bh = np.fft.fft(b)
    xe = np.fft.ifft(np.conj(ah) * bh / (np.abs(ah) ** 2 + lam ** 2))
    x = oracle.solve(col, row, b, lam)
    np.testing.assert_allclose(x, xe, rtol=1e-11, atol=1e-12)


def test_scaled_identity_and_zero():
    n = 9
    rng = np.random.default_rng(3)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    c = 1.5 - 0.5j; lam = 0.8
    col = np.zeros(n, complex); col[0] = c; row = np.zeros(n, complex); row[0] = c
    np.testing.assert_allclose(oracle.solve(col, row, b, lam), np.conj(c) * b / (abs(c) ** 2 + lam ** 2), rtol=1e-13)
    z = np.zeros(n)
    assert np.abs(oracle.solve(np.zeros(12), z, rng.standard_normal(12), lam)).max() < 1e-14


def test_scaling_law_and_large_lambda():
    rng = np.random.default_rng(5)
    col, row, b = W.random_problem(rng, 20, 13, cplx=True)
    lam, alpha = 0.6, 3.7
    x1 = oracle.solve(col, row, b, lam)
    x2 = oracle.solve(alpha * col, alpha * row, b, alpha * lam)
    np.testing.assert_allclose(x2, x1 / alpha, rtol=1e-12)
    big = 1e5
    xl = oracle.solve(col, row, b, big)
    np.testing.assert_allclose(big ** 2 * xl, oracle.TH_apply(col, row, b), rtol=1e-6)


@pytest.mark.parametrize("m,n,cplx", [(40, 30, False), (30, 40, True), (64, 64, True)])
def test_lstsq_and_optimality(m, n, cplx):
    rng = np.random.default_rng(m * n)
    col, row, b = W.random_problem(rng, m, n, cplx=cplx)
    lam = 0.25
    x = oracle.solve(col, row, b, lam)
    T = oracle.dense_T(col, row)
    A = np.vstack([T, lam * np.eye(n)])
    xe = np.linalg.lstsq(A, np.concatenate([b, np.zeros(n)]), rcond=None)[0]
    np.testing.assert_allclose(x, xe, rtol=1e-10, atol=1e-12)
    assert oracle.normal_residual(col, row, b, lam, x) < 1e-13
    # T_apply / TH_apply against the dense matrix
    v = rng.standard_normal(n); w = rng.standard_normal(m)
    np.testing.assert_allclose(oracle.T_apply(col, row, v), T @ v, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(oracle.TH_apply(col, row, w), T.conj().T @ w, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("cplx", [False, True])
def test_normal_form_entry(cplx):
    rng = np.random.default_rng(11)
    col, row, _ = W.random_problem(rng, 25, 17, cplx=cplx)
    y = rng.standard_normal(17) + (1j * rng.standard_normal(17) if cplx else 0)
    lam = 0.9
    x = oracle.solve_normal(col, row, y, lam)
    T = oracle.dense_T(col, row)
    np.testing.assert_allclose((T.conj().T @ T + lam ** 2 * np.eye(17)) @ x, y, rtol=1e-11, atol=1e-12)


def _loss(col, row, b, lam, xt):
    x = oracle.solve(col, row, b, lam)
    return 0.5 * np.sum(np.abs(x - xt) ** 2)


@pytest.mark.parametrize("cplx", [False, True])
def test_gradients_central_differences(cplx):
    """Hand-derived adjoint (w = A^{-1} g, g_b = T w, g_lam = -2 lam Re<w,x>,
    G_T = (b - T x) w^H - (T w) x^H) against central differences of the oracle."""
    rng = np.random.default_rng(21 + cplx)
    m, n = 14, 9
    col, row, b = W.random_problem(rng, m, n, cplx=cplx)
    lam = 0.7
    xt = rng.standard_normal(n) + (1j * rng.standard_normal(n) if cplx else 0)
    x = oracle.solve(col, row, b, lam)
    g = oracle.gradients(col, row, b, lam, x - xt)
    np.testing.assert_allclose(g["x"], x, rtol=1e-13)
    h = 1e-6
    dirs = rng.standard_normal((6, 2 * m + 2 * n + 1))
    for d in dirs:
        d /= np.linalg.norm(d)
        dcol = d[:m] + (1j * d[m:2 * m] if cplx else 0)
        drow = np.concatenate([[0], d[2 * m:2 * m + n - 1]]) + (1j * np.concatenate([[0], d[2 * m + n - 1:2 * m + 2 * n - 2]]) if cplx else 0)
        db = d[-1 - m:-1] if not cplx else d[-1 - m:-1] * (1 + 1j)
        dl = d[-1]
        fp = _loss(col + h * dcol, row + h * drow, b + h * db, lam + h * dl, xt)
        fm = _loss(col - h * dcol, row - h * drow, b - h * db, lam - h * dl, xt)
        fd = (fp - fm) / (2 * h)
        an = (np.sum((np.conj(g["g_col"]) * dcol).real) + np.sum((np.conj(g["g_row"]) * drow).real)
              + np.sum((np.conj(g["g_b"]) * db).real) + g["g_lam"] * dl)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)
    # dx/dlambda = -2 lambda A^{-1} x
    dxdl = (oracle.solve(col, row, b, lam + h) - oracle.solve(col, row, b, lam - h)) / (2 * h)
    np.testing.assert_allclose(dxdl, -2 * lam * oracle.solve_normal(col, row, x, lam), rtol=1e-6, atol=1e-8)


# ---- banded QR (exact for generators of finite support, used at full sizes) ----

def _banded_problem(rng, m, n, wl, wu, cplx):
    col = rng.standard_normal(m) + (1j * rng.standard_normal(m) if cplx else 0)
    row = rng.standard_normal(n) + (1j * rng.standard_normal(n) if cplx else 0)
    col[wl + 1:] = 0
    row[wu + 1:] = 0
    row[0] = col[0]
    return col, row


@pytest.mark.parametrize("m,n,wl,wu,cplx", [(40, 30, 5, 3, False), (30, 40, 2, 7, True), (50, 50, 0, 0, False),
                                            (60, 20, 10, 0, True), (25, 60, 0, 9, False), (7, 5, 6, 4, True),
                                            (1, 1, 0, 0, False), (90, 64, 89, 63, True)])
def test_band_qr_against_lstsq(m, n, wl, wu, cplx):
    """Banded QR against numpy's least squares of the stacked system, several right-hand
    sides sharing one factorization, both entries (b, and normal-form y)."""
    rng = np.random.default_rng(m * 1000 + n * 10 + wl)
    col, row = _banded_problem(rng, m, n, wl, wu, cplx)
    lam = 0.3
    T = oracle.dense_T(col, row)
    A = np.vstack([T, lam * np.eye(n)])
    bs = [rng.standard_normal(m) + (1j * rng.standard_normal(m) if cplx else 0) for _ in range(3)]
    xb = oracle.band_solve(col, row, bs, lam)
    for r in range(3):
        xe = np.linalg.lstsq(A, np.concatenate([bs[r], np.zeros(n)]), rcond=None)[0]
        np.testing.assert_allclose(xb[r], xe, rtol=1e-11, atol=1e-12)
    ys = [rng.standard_normal(n) + (1j * rng.standard_normal(n) if cplx else 0) for _ in range(2)]
    xn = oracle.band_solve(col, row, ys, lam, normal=True)
    for r in range(2):
        np.testing.assert_allclose((T.conj().T @ T + lam ** 2 * np.eye(n)) @ xn[r], ys[r], rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("n,L,cplx", [(600, 6.0, False), (1500, 4.0, True), (2000, 10.0, False)])
def test_band_qr_against_dense_qr(n, L, cplx):
    """Banded QR against the dense Householder QR at n <= 2000 on envelope generators
    cut at 40 L (the inputs of the full-size workloads), tall and square."""
    rng = np.random.default_rng(n)
    m = n + n // 8
    col, row = W.envelope_generator(rng, m, n, L, cplx=cplx)
    b = rng.standard_normal(m) + (1j * rng.standard_normal(m) if cplx else 0)
    lam = 0.05
    xd = oracle.solve(col, row, b, lam, nthreads=8)
    xb = oracle.band_solve(col, row, [b], lam)[0]
    assert np.linalg.norm(xb - xd) / np.linalg.norm(xd) < 1e-11


def test_band_qr_closed_forms():
    """T = c I (bandwidth 0): x = conj(c) b / (|c|^2 + lam^2); T = 0: x = 0; the scaling law
    x(alpha T, alpha lam) = x(T, lam) / alpha on a banded operator."""
    n = 300
    rng = np.random.default_rng(9)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    c, lam = 1.5 - 0.5j, 0.8
    col = np.zeros(n, complex); col[0] = c; row = np.zeros(n, complex); row[0] = c
    np.testing.assert_allclose(oracle.band_solve(col, row, [b], lam)[0], np.conj(c) * b / (abs(c) ** 2 + lam ** 2),
                               rtol=1e-14)
    assert np.abs(oracle.band_solve(np.zeros(n + 5), np.zeros(n), [b.real[:1].repeat(n + 5)], lam)[0]).max() == 0.0
    col, row = _banded_problem(rng, n + 20, n, 12, 5, True)
    b2 = rng.standard_normal(n + 20)
    x1 = oracle.band_solve(col, row, [b2], 0.4)[0]
    x2 = oracle.band_solve(3.7 * col, 3.7 * row, [b2], 3.7 * 0.4)[0]
    np.testing.assert_allclose(x2, x1 / 3.7, rtol=1e-12)


def test_band_qr_mutation_fails():
    """A plausible slip (the conjugate generator, i.e. T^T instead of T) must fail the pin."""
    rng = np.random.default_rng(17)
    col, row = _banded_problem(rng, 30, 24, 4, 3, True)
    b = rng.standard_normal(30) + 1j * rng.standard_normal(30)
    xe = oracle.solve(col, row, b, 0.5)
    xbad = oracle.band_solve(np.conj(col), np.conj(row), [b], 0.5)[0]
    assert np.linalg.norm(xbad - xe) / np.linalg.norm(xe) > 1e-3


@pytest.mark.parametrize("cplx", [False, True])
def test_band_gradients_against_dense(cplx):
    """The banded adjoint (w by banded QR, g_b = T w, g_lam, lag sums) against the dense
    oracle's gradients, which central differences pin above."""
    rng = np.random.default_rng(31 + cplx)
    m, n = 70, 52
    col, row = _banded_problem(rng, m, n, 9, 4, cplx)
    b = rng.standard_normal(m) + (1j * rng.standard_normal(m) if cplx else 0)
    gx = rng.standard_normal(n) + (1j * rng.standard_normal(n) if cplx else 0)
    lam = 0.35
    ref = oracle.gradients(col, row, b, lam, gx)
    got = oracle.band_gradients(col, row, b, lam, ref["x"], gx)
    for k in ("g_b", "g_col", "g_row"):
        np.testing.assert_allclose(got[k], ref[k], rtol=1e-11, atol=1e-12)
    assert abs(got["g_lam"] - ref["g_lam"]) <= 1e-11 * max(1.0, abs(ref["g_lam"]))


def test_normal_residual_fft():
    """FFT-formed optimality residual: equal to the direct one on a small problem, at
    rounding level for the oracle's solution, and large for a perturbed solution."""
    rng = np.random.default_rng(41)
    col, row, b = W.random_problem(rng, 90, 70, cplx=True, L=10.0)
    lam = 0.2
    x = oracle.solve(col, row, b, lam)
    r1 = oracle.normal_residual_fft(col, row, b, lam, x)
    assert r1 < 1e-14
    xp = x * (1 + 1e-6)
    assert abs(oracle.normal_residual_fft(col, row, b, lam, xp) / oracle.normal_residual(col, row, b, lam, xp) - 1) < 1e-6
    assert oracle.normal_residual_fft(col, row, b, lam, xp) > 1e-8


# ---- Toeplitz-Gramian problem (Sec. 2, third case; Sec. 3.4) ----

def test_gramian_reduces_to_l2():
    """T circulant (so that G = T^H T is Toeplitz) with L = lambda I (a p = n Toeplitz
    regularizer) is the l2 problem's normal form: the Gramian oracle must equal the dense-QR
    normal-form solve."""
    rng = np.random.default_rng(51)
    for (n, cplx) in [(20, False), (25, True), (9, True)]:
        c = rng.standard_normal(n) + (1j * rng.standard_normal(n) if cplx else 0)
        col = c.copy(); row = np.concatenate([[c[0]], c[1:][::-1]])
        T = oracle.dense_T(col, row)
        gram = (T.conj().T @ T)[:, 0]
        lam = 0.6
        lcol = np.zeros(n); lcol[0] = lam
        lrow = np.zeros(n); lrow[0] = lam
        y = rng.standard_normal(n) + (1j * rng.standard_normal(n) if cplx else 0)
        np.testing.assert_allclose(oracle.gramian_solve(gram, lcol, lrow, y), oracle.solve_normal(col, row, y, lam),
                                   rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("n", [16, 63, 200])
def test_gramian_circulant_closed_form(n):
    """G and L circulant (Hermitian-symmetric first column c for G, first column d for L,
    p = n): x = IDFT(y^ / (c^ + |d^|^2))."""
    rng = np.random.default_rng(n + 5)
    c = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    c = 0.5 * (c + np.conj(np.roll(c[::-1], 1)))          # c_{n-s} = conj(c_s): G Hermitian
    ch = np.fft.fft(c).real
    c[0] += 1.0 - ch.min()                                   # G positive definite
    d = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    gram = c.copy()
    lcol = d.copy(); lrow = np.concatenate([[d[0]], d[1:][::-1]])
    y = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    xe = np.fft.ifft(np.fft.fft(y) / (np.fft.fft(c).real + np.abs(np.fft.fft(d)) ** 2))
    np.testing.assert_allclose(oracle.gramian_solve(gram, lcol, lrow, y), xe, rtol=1e-10, atol=1e-11)


def test_gramian_exact_rational():
    """Integer data, exact rational elimination of (G + L^T L) x = y (G symmetric Toeplitz
    with a dominant diagonal, L a 4 x 5 Toeplitz regularizer)."""
    rng = np.random.default_rng(61)
    n, p = 5, 4
    gram = rng.integers(-3, 4, size=n); gram[0] = 12
    G = [[int(gram[abs(r - s)]) for s in range(n)] for r in range(n)]
    lcol = rng.integers(-3, 4, size=p); lrow = rng.integers(-3, 4, size=n); lrow[0] = lcol[0]
    L = [[int(lcol[i - j]) if i >= j else int(lrow[j - i]) for j in range(n)] for i in range(p)]
    A = [[Fraction(G[r][s] + sum(L[k][r] * L[k][s] for k in range(p))) for s in range(n)] for r in range(n)]
    y = [Fraction(int(v)) for v in rng.integers(-5, 6, size=n)]
    M = [row[:] + [y[i]] for i, row in enumerate(A)]
    for c in range(n):
        pv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[pv] = M[pv], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [M[r][k] - f * M[c][k] for k in range(n + 1)]
    xe = np.array([float(M[i][n] / M[i][i]) for i in range(n)])
    x = oracle.gramian_solve(gram, lcol, lrow, np.array([float(v) for v in y]))
    np.testing.assert_allclose(x.real, xe, rtol=1e-12, atol=1e-13)
    assert np.abs(x.imag).max() == 0.0


def test_gramian_mutation_fails():
    """A plausible slip (G built from conj(gram), i.e. G transposed) must change the answer."""
    rng = np.random.default_rng(71)
    n = 12
    gram = rng.standard_normal(n) + 1j * rng.standard_normal(n); gram[0] = 8.0
    lcol = rng.standard_normal(n); lrow = np.concatenate([[lcol[0]], rng.standard_normal(n - 1)])
    y = rng.standard_normal(n)
    x1 = oracle.gramian_solve(gram, lcol, lrow, y)
    x2 = oracle.gramian_solve(np.conj(gram), lcol, lrow, y)
    assert np.linalg.norm(x1 - x2) / np.linalg.norm(x1) > 1e-3


def test_replica_workloads_recover_x():
    """The Table 1 replica workloads (Sec. 7.1-7.2) are consistent: the dense oracle recovers
    their known x from y (normal form for the l2 problem, (G + L^H L) x = y for the
    Toeplitz-Gramian one)."""
    for n in (16, 64):
        q = W.replica(n, 1)
        assert np.max(np.abs(oracle.solve_normal(q.col, q.row, q.b[0], q.lams[0]) - q.x_true)) <= 1e-12
        assert abs(q.lams[0] ** 2 - np.sqrt(2.0 * n)) <= 1e-12
        p = W.replica_gramian(n, 1)
        assert abs(p.gram[0] - 10.0 * np.sqrt(2.0 * n)) <= 1e-12
        assert np.max(np.abs(oracle.gramian_solve(p.gram, p.lcol, p.lrow, p.ys[0]) - p.x_true)) <= 1e-12


# ---------------------------------------------------------------- the general problem (Sec. 3.2)
def _circ(c):
    n = len(c)
    col = np.asarray(c, np.complex128)
    row = np.concatenate([[col[0]], col[1:][::-1]])
    return col, row


def test_general_reduces_to_l2_with_scaled_identity():
    """L = lambda I turns the general problem into eq. (tiksol) of the l2 problem: the
    numpy least-squares oracle must agree with the C Householder QR (O1)."""
    rng = np.random.default_rng(31)
    for (m, n, cplx) in ((9, 6, False), (5, 8, True), (20, 20, True)):
        col, row, b = W.random_problem(rng, m, n, cplx=cplx, L=4.0)
        lam = 0.37
        lcol = np.zeros(n, complex); lcol[0] = lam
        lrow = np.zeros(n, complex); lrow[0] = lam
        x = oracle.general_solve(col, row, lcol, lrow, b)
        xr = oracle.solve(col, row, b, lam)
        assert np.linalg.norm(x - xr) <= 1e-12 * np.linalg.norm(xr)


def test_general_exact_rational():
    """3 x 2 T and 2 x 2 L with integer generators: the normal equations
    (T^T T + L^T L) x = T^T b solved exactly in rational arithmetic."""
    a = {-1: 2, 0: 1, 1: -1, 2: 3}            # a_s of T (m = 3, n = 2)
    l = {-1: 1, 0: 2, 1: -1}                  # l_s of L (p = 2, n = 2)
    m, n, p = 3, 2, 2
    T = [[Fraction(a[i - j]) for j in range(n)] for i in range(m)]
    Lm = [[Fraction(l[i - j]) for j in range(n)] for i in range(p)]
    b = [Fraction(v) for v in (1, -2, 4)]
    A = [[sum(T[k][i] * T[k][j] for k in range(m)) + sum(Lm[k][i] * Lm[k][j] for k in range(p))
          for j in range(n)] for i in range(n)]
    r = [sum(T[k][i] * b[k] for k in range(m)) for i in range(n)]
    det = A[0][0] * A[1][1] - A[0][1] * A[1][0]
    xe = [(r[0] * A[1][1] - A[0][1] * r[1]) / det, (A[0][0] * r[1] - A[1][0] * r[0]) / det]
    col = np.array([a[0], a[1], a[2]], float); row = np.array([a[0], a[-1]], float)
    lcol = np.array([l[0], l[1]], float); lrow = np.array([l[0], l[-1]], float)
    x = oracle.general_solve(col, row, lcol, lrow, np.array([1.0, -2.0, 4.0]))
    assert np.max(np.abs(x - np.array([float(v) for v in xe]))) <= 1e-13


def _circulant_closed_form(t, l, b):
    th, lh, bh = np.fft.fft(t), np.fft.fft(l), np.fft.fft(b)
    return np.fft.ifft(np.conj(th) * bh / (np.abs(th) ** 2 + np.abs(lh) ** 2))


def test_general_circulant_closed_form():
    """Circulant T and L (n x n): T^H T + L^H L is diagonal in the Fourier basis, so
    x = IDFT(conj(t^) b^ / (|t^|^2 + |l^|^2))."""
    rng = np.random.default_rng(32)
    for n in (7, 16, 45):
        t = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        l = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        (tc, tr), (lc, lr) = _circ(t), _circ(l)
        x = oracle.general_solve(tc, tr, lc, lr, b)
        xr = _circulant_closed_form(t, l, b)
        assert np.linalg.norm(x - xr) <= 1e-11 * np.linalg.norm(xr)
        assert np.linalg.norm(oracle.general_solve_normal(tc, tr, lc, lr,
                                                          oracle.TH_apply(tc, tr, b)) - xr) <= 1e-11 * np.linalg.norm(xr)


def test_general_optimality_with_second_difference():
    """With L the (n-2) x n second difference (a rectangular Toeplitz L), the solution
    satisfies the optimality condition T^H (b - T x) = L^H L x."""
    rng = np.random.default_rng(33)
    m, n = 40, 30
    col, row, b = W.random_problem(rng, m, n, cplx=True, L=6.0)
    lcol = np.zeros(n - 2); lcol[0] = 1.0
    lrow = np.zeros(n); lrow[0], lrow[1], lrow[2] = 1.0, -2.0, 1.0
    x = oracle.general_solve(col, row, lcol, lrow, b)
    T, L = oracle.dense_T(col, row), oracle.dense_T(lcol, lrow)
    lhs = T.conj().T @ (b - T @ x)
    rhs = L.conj().T @ (L @ x)
    assert np.linalg.norm(lhs - rhs) <= 1e-11 * np.linalg.norm(T.conj().T @ b)


def test_general_pins_catch_a_transposed_regularizer():
    """Mutation: the normal equations formed with L^T L instead of L^H L (a dropped
    conjugate) fail the circulant closed form for complex L."""
    rng = np.random.default_rng(34)
    n = 16
    t = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    l = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    (tc, tr), (lc, lr) = _circ(t), _circ(l)
    T, L = oracle.dense_T(tc, tr), oracle.dense_T(lc, lr)
    bad = np.linalg.solve(T.conj().T @ T + L.T @ L, T.conj().T @ b)
    xr = _circulant_closed_form(t, l, b)
    assert np.linalg.norm(bad - xr) > 1e-3 * np.linalg.norm(xr)


def test_general_replica_workload_recovers_x():
    for n in (16, 64):
        col, row, lcol, lrow, y, x = W.replica_general(n, 2)
        assert np.max(np.abs(oracle.general_solve_normal(col, row, lcol, lrow, y) - x)) <= 1e-12
