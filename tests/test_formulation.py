"""The interpolation conditions the GPU path assembles, checked on the CPU against the
oracle's solutions (no GPU): the l2 problem's two condition sets per root of unity
(Sec. 3.3, eq. (ex6) with k-circulant extensions, transformed by eq. (vandprod) into the
conditions of eq. (intcond)) and those of the Toeplitz-Gramian problem (Sec. 3.4,
eq. (ex7)).

With the unknown p* = [x; sigma = T x; gamma_1; gamma_2; 1] and w = exp(+2 pi i / N),

    F_nu = [ lambda^2 w^{(m+k-1) nu},  w^{(k-1) nu} conj(c^(w^nu)),  1,  0,  -w^{(m+k-1) nu} y^(w^nu) ]
    G_nu = [ -c^(w^nu),                w^{(n+k-1) nu},               0,  1,  0 ]

where c_T[r] = a_{r-(n+k-1)} for r >= k (the k entries below are arbitrary) and y = T^H b.
Both conditions hold at every node for some gamma_1 of m+k-1 coefficients and gamma_2 of
n+k-1 exactly when x solves the normal equations: the gammas solved for from the
conditions must have no coefficients past those lengths.  Each plausible misreading (the
extension index off by one, a dropped conjugate, a wrong shift, mixed Fourier signs)
leaves such coefficients."""
import numpy as np
import pytest

import oracle
import workloads as W


def ev(c, N):
    """Evaluations sum_i c_i w^{i nu}, nu < N, w = exp(+2 pi i / N)."""
    out = np.zeros(N, np.complex128)
    out[:len(c)] = c
    return N * np.fft.ifft(out)


def coef(E):
    """Coefficients (mod z^N - 1) of the polynomial with evaluations E at the N-th roots of unity."""
    return np.fft.fft(E) / len(E)


def wp(e, N):
    return np.exp(2j * np.pi * e * np.arange(N) / N)


def l2_extension(a, m, n, k, fill, shift=0):
    """First column of the k-circulant extension of T (generator a_s, s = -(n-1)..m-1)."""
    N = m + n + k - 1
    c = np.zeros(N, np.complex128)
    for r in range(N):
        s = r - (n + k - 1) - shift
        if -(n - 1) <= s <= m - 1 and r >= k:
            c[r] = a[s + n - 1]
    c[:k] = fill[:k]
    return c


def l2_tails(c, x, sigma, y, lam, m, n, k, conj=True, fshift=None, ysign=1):
    """gamma_1, gamma_2 solved for from F and G at every node; returns the coefficients past
    their lengths (zero exactly when the conditions hold with the stated degrees)."""
    N = m + n + k - 1
    ch, xh, sh = ev(c, N), ev(x, N), ev(sigma, N)
    # ysign < 0: sum_i y_i w^{-i nu}, the other sign
    yh = ev(y, N) if ysign > 0 else np.conj(ev(np.conj(y), N))
    fs = k - 1 if fshift is None else fshift
    g2 = coef(ch * xh - wp(n + k - 1, N) * sh)
    g1 = coef(-(lam ** 2 * wp(m + k - 1, N) * xh + wp(fs, N) * (np.conj(ch) if conj else ch) * sh
                - wp(m + k - 1, N) * yh))
    return g1[m + k - 1:], g2[n + k - 1:]


CASES = [(7, 5, 3, False), (5, 9, 0, True), (12, 12, 4, True), (9, 4, 1, False), (16, 11, 6, True)]


def _problem(m, n, cplx, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(m + n - 1) + (1j * rng.standard_normal(m + n - 1) if cplx else 0)
    col, row = W.split_generator(a, m, n)
    b = rng.standard_normal(m) + (1j * rng.standard_normal(m) if cplx else 0)
    return rng, a, col, row, b


@pytest.mark.parametrize("m,n,k,cplx", CASES)
def test_l2_conditions_hold_at_the_solution(m, n, k, cplx):
    rng, a, col, row, b = _problem(m, n, cplx, 11 * m + n + k)
    lam = 0.7
    T = oracle.dense_T(col, row)
    x = oracle.solve(col, row, b, lam)
    sigma, y = T @ x, T.conj().T @ b
    scale = np.linalg.norm(x) * (lam ** 2 + np.sum(np.abs(a)) ** 2) + np.linalg.norm(y)
    # the extension's arbitrary entries do not matter: two fills
    for fill in (np.zeros(k), rng.standard_normal(k) + 1j * rng.standard_normal(k)):
        c = l2_extension(a, m, n, k, fill)
        t1, t2 = l2_tails(c, x, sigma, y, lam, m, n, k)
        assert np.max(np.abs(t1), initial=0.0) <= 1e-12 * scale
        assert np.max(np.abs(t2), initial=0.0) <= 1e-12 * scale
        # F's tail is the normal-equation residual lambda^2 x + T^H T x - T^H b, G's is T x - sigma
        xp = x + 1e-3 * rng.standard_normal(n)
        t1, t2 = l2_tails(c, xp, T @ xp, y, lam, m, n, k)
        assert np.max(np.abs(t1)) > 1e-7 * scale
        assert np.max(np.abs(t2), initial=0.0) <= 1e-12 * scale


@pytest.mark.parametrize("m,n,k,cplx", CASES)
def test_l2_misreadings_leave_tails(m, n, k, cplx):
    rng, a, col, row, b = _problem(m, n, cplx, 13 * m + n + k)
    lam = 0.7
    T = oracle.dense_T(col, row)
    x = oracle.solve(col, row, b, lam)
    sigma, y = T @ x, T.conj().T @ b
    scale = np.linalg.norm(x) * (lam ** 2 + np.sum(np.abs(a)) ** 2) + np.linalg.norm(y)
    fill = rng.standard_normal(k)
    big = lambda t: np.max(np.abs(t), initial=0.0) > 1e-6 * scale
    # the printed extension read literally: every index one further
    c1 = l2_extension(a, m, n, k, fill, shift=1)
    t1, t2 = l2_tails(c1, x, sigma, y, lam, m, n, k)
    assert big(t1) or big(t2)
    c = l2_extension(a, m, n, k, fill)
    # the adjoint's symbol without its conjugate (for real generators too:
    # conj(c^(w^nu)) = c^(w^-nu))
    t1, _ = l2_tails(c, x, sigma, y, lam, m, n, k, conj=False)
    assert big(t1)
    # the adjoint's shift k instead of k - 1
    t1, _ = l2_tails(c, x, sigma, y, lam, m, n, k, fshift=k)
    assert big(t1)
    # the right-hand side evaluated with the other Fourier sign
    t1, _ = l2_tails(c, x, sigma, y, lam, m, n, k, ysign=-1)
    assert big(t1)


def gram_tails(gram, lcol, lrow, x, y, N, fill_g, fill_l):
    """The Toeplitz-Gramian conditions: F = [g^, w^{(N-n-p)} conj(l^), 1, 0, -w^{(N-n)} y^],
    G = [-l^, w^{(N-p)}, 0, 1, 0]; c_G[N-n+s] = g_s (|s| < n), c_L[r] = l_{r-(N-p)}."""
    n, p = len(gram), len(lcol)
    cg = np.zeros(N, np.complex128)
    cg[:N - 2 * n + 1] = fill_g
    for s in range(-(n - 1), n):
        cg[N - n + s] = gram[s] if s >= 0 else np.conj(gram[-s])
    kl = N - (p + n - 1)
    cl = np.zeros(N, np.complex128)
    cl[:kl] = fill_l
    for r in range(kl, N):
        s = r - (N - p)
        cl[r] = lcol[s] if s >= 0 else lrow[-s]
    L = oracle.dense_T(lcol, lrow)
    sigma = L @ x
    gh, lh, xh, sh, yh = ev(cg, N), ev(cl, N), ev(x, N), ev(sigma, N), ev(y, N)
    g2 = coef(lh * xh - wp(N - p, N) * sh)
    g1 = coef(-(gh * xh + wp(N - n - p, N) * np.conj(lh) * sh - wp(N - n, N) * yh))
    return g1[N - n:], g2[N - p:]


@pytest.mark.parametrize("n,p,extra", [(6, 4, 0), (5, 9, 2), (8, 8, 3)])
def test_gramian_conditions_hold_at_the_solution(n, p, extra):
    rng = np.random.default_rng(100 * n + p)
    N = max(2 * n - 1, p + n - 1) + extra
    lcol = rng.standard_normal(p) + 1j * rng.standard_normal(p)
    lrow = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    gram = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    gram[0] = 4.0 * n                                # diagonally dominant: G positive definite
    y = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x = oracle.gramian_solve(gram, lcol, lrow, y)
    scale = np.linalg.norm(x) * (np.sum(np.abs(gram)) * 2 + (np.sum(np.abs(lcol)) + np.sum(np.abs(lrow))) ** 2) \
        + np.linalg.norm(y)
    fg = rng.standard_normal(N - 2 * n + 1)
    fl = rng.standard_normal(N - (p + n - 1))
    t1, t2 = gram_tails(gram, lcol, lrow, x, y, N, fg, fl)
    assert np.max(np.abs(t1)) <= 1e-12 * scale
    assert np.max(np.abs(t2)) <= 1e-12 * scale
    # another x leaves F's tail (G x + L^H L x - y)
    t1, _ = gram_tails(gram, lcol, lrow, x + 1e-3, y, N, fg, fl)
    assert np.max(np.abs(t1)) > 1e-7 * scale


def toeplitz_extension(col, row, rows, N):
    """First column of an N-circulant holding the rows x n Toeplitz block (col, row) in its
    last `rows` rows and first n columns: c[r] = a_{r-(N-rows)}; the entries below
    N-(rows+n-1) are the arbitrary ones (left zero here)."""
    n = len(row)
    c = np.zeros(N, np.complex128)
    for r in range(N - (rows + n - 1), N):
        s = r - (N - rows)
        c[r] = col[s] if s >= 0 else row[-s]
    return c


def general_tails(col, row, lcol, lrow, x, y, N, conj=True):
    """The general problem's three condition sets (Sec. 3.2 eqs. (ex2)-(ex3), transformed as
    eq. (intcond)), unknown [x; s1 = T x; s2 = L x; g1; g2; g3; 1] and one extension size N
    for both blocks:
        F = [0, w^{(N-m-n)} conj(t^), w^{(N-p-n)} conj(l^), 1, 0, 0, -w^{(N-n)} y^]
        G = [-t^, w^{(N-m)}, 0, 0, 1, 0, 0]
        H = [-l^, 0, w^{(N-p)}, 0, 0, 1, 0]
    Returns the coefficients of g1, g2, g3 past N-n, N-m and N-p."""
    m, n, p = len(col), len(row), len(lcol)
    T, L = oracle.dense_T(col, row), oracle.dense_T(lcol, lrow)
    th, lh = ev(toeplitz_extension(col, row, m, N), N), ev(toeplitz_extension(lcol, lrow, p, N), N)
    xh, s1h, s2h, yh = ev(x, N), ev(T @ x, N), ev(L @ x, N), ev(y, N)
    cj = np.conj if conj else (lambda v: v)
    g1 = coef(-(wp(N - m - n, N) * cj(th) * s1h + wp(N - p - n, N) * cj(lh) * s2h - wp(N - n, N) * yh))
    g2 = coef(th * xh - wp(N - m, N) * s1h)
    g3 = coef(lh * xh - wp(N - p, N) * s2h)
    return g1[N - n:], g2[N - m:], g3[N - p:]


@pytest.mark.parametrize("m,n,p,extra", [(7, 5, 5, 0), (6, 6, 9, 1), (10, 4, 3, 2), (5, 8, 8, 0), (6, 4, 6, 0)])
def test_general_conditions_hold_at_the_solution(m, n, p, extra):
    """The general problem's conditions (its GPU path is not built): at the oracle's solution
    of min ||T x - b||^2 + ||L x||^2 the three gammas have no coefficients past their
    lengths; with N = max(m, p) + n (one extension entry, as the paper's 1-circulant
    extensions) the lengths are the paper's degree bounds (eq. (degcon)) when m = p.  A
    perturbed x, or the adjoint symbols without their conjugates, leave F's tail."""
    rng = np.random.default_rng(7 * m + 5 * n + p)
    cn = lambda k: rng.standard_normal(k) + 1j * rng.standard_normal(k)
    col, row, lcol, lrow, b = cn(m), cn(n), cn(p), cn(n), cn(m)
    row[0] = col[0]
    lrow[0] = lcol[0]
    N = max(m, p) + n + extra
    x = oracle.general_solve(col, row, lcol, lrow, b)
    T = oracle.dense_T(col, row)
    y = T.conj().T @ b
    scale = np.linalg.norm(x) * (np.sum(np.abs(col)) + np.sum(np.abs(row)) + np.sum(np.abs(lcol))
                                 + np.sum(np.abs(lrow))) ** 2 + np.linalg.norm(y)
    tails = general_tails(col, row, lcol, lrow, x, y, N)
    for t in tails:
        assert np.max(np.abs(t)) <= 1e-12 * scale
    if m == p and extra == 0:
        # gamma lengths N - n, N - m, N - p: the paper's bounds m, n, n (eq. (degcon))
        assert (N - n, N - m, N - p) == (m, n, n)
    t1 = general_tails(col, row, lcol, lrow, x + 1e-3, y, N)[0]
    assert np.max(np.abs(t1)) > 1e-7 * scale
    t1 = general_tails(col, row, lcol, lrow, x, y, N, conj=False)[0]
    assert np.max(np.abs(t1)) > 1e-6 * scale
