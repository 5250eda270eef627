"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Small and medium problems are compared element by element with the oracle
(dense Householder QR of [T; lambda I]) at sizes the oracle finishes in
seconds, spanning several leaves, several tree levels and ragged extensions.
Full-size problems (generators of finite support) are compared element by
element with the banded QR oracle, which solves the same least-squares problem
exactly at any size, or with known solutions whose right-hand sides are formed
in long double.  Tolerance: relative
2-norm error <= 1e-9 against the oracle (the accuracy target for problems
whose regularized normal matrix has condition number <= 1e6)."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle
import workloads as W

TOL = 1e-9
LEAF_WAVE_GROUPS = int(os.environ.get("TIKH_TEST_LEAF_WAVE_GROUPS", "1536"))


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1302_6945_amd as P
    # the leaf-step variant can be forced for the whole module (1: one wavefront per group)
    P.set_options(n_lim=256, refine=1, leaf_wave_groups=LEAF_WAVE_GROUPS)
    yield P
    P.set_options(n_lim=256, refine=1)


def dev(a):
    return torch.tensor(np.asarray(a), device="cuda:0")


def relerr(x, xr):
    return np.linalg.norm(np.asarray(x) - xr) / max(np.linalg.norm(xr), 1e-300)


SIZES = [(1, 1), (1, 4), (4, 1), (2, 2), (3, 7), (7, 3), (33, 31), (64, 64), (100, 37), (37, 100), (129, 128),
         (300, 211)]


@pytest.mark.parametrize("m,n", SIZES)
@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("nlim", [64, 256])
def test_small_parity(P, m, n, cplx, nlim):
    rng = np.random.default_rng(1000 * m + n + 7 * cplx + nlim)
    col, row, b = W.random_problem(rng, m, n, cplx=cplx, L=8.0)
    lam = 0.5
    P.set_options(n_lim=nlim)
    x = P.solve(dev(col), dev(row), dev(b), lam).cpu().numpy()
    xr = oracle.solve(col, row, b, lam)
    assert relerr(x, xr) <= TOL, (m, n, cplx, nlim, relerr(x, xr), P.get_stats())
    if not cplx:
        assert x.dtype == np.float64


def test_config0_parity(P):
    pr = W.config0()
    x = P.solve(dev(pr.col), dev(pr.row), dev(pr.b[0]), pr.lams[0]).cpu().numpy()
    xr = oracle.solve(pr.col, pr.row, pr.b[0], pr.lams[0])
    assert relerr(x, xr) <= TOL
    st = P.get_stats()
    assert (st["N"], st["leaf_nodes"], st["depth"], st["k"]) == (640, 80, 3, 1)


@pytest.mark.parametrize("cplx", [False, True])
def test_normal_form_parity(P, cplx):
    rng = np.random.default_rng(5 + cplx)
    col, row, _ = W.random_problem(rng, 250, 180, cplx=cplx, L=16.0)
    y = rng.standard_normal(180) + (1j * rng.standard_normal(180) if cplx else 0)
    x = P.solve_normal(dev(col), dev(row), dev(y), 0.2).cpu().numpy()
    assert relerr(x, oracle.solve_normal(col, row, y, 0.2)) <= TOL


def test_refinement_off_still_close(P):
    pr = W.config0()
    P.set_options(refine=0)
    try:
        x = P.solve(dev(pr.col), dev(pr.row), dev(pr.b[0]), pr.lams[0]).cpu().numpy()
    finally:
        P.set_options(refine=1)
    assert relerr(x, oracle.solve(pr.col, pr.row, pr.b[0], pr.lams[0])) <= 1e-8


def test_deblurring_medium(P):
    pr = W.config1(n=2048)
    x = P.solve(dev(pr.col), dev(pr.row), dev(pr.b[0]), pr.lams[0]).cpu().numpy()
    xr = oracle.solve(pr.col, pr.row, pr.b[0], pr.lams[0], nthreads=8)
    assert relerr(x, xr) <= TOL


def test_batched_ragged(P):
    rng = np.random.default_rng(42)
    shapes = [(50, 40), (200, 150), (33, 90), (300, 300), (7, 5)]
    nlam, nrhs = 3, 2
    cols, rows, bs, lams = [], [], [], []
    probs = []
    for (m, n) in shapes:
        col, row, _ = W.random_problem(rng, m, n, L=10.0)
        B = [rng.standard_normal(m) for _ in range(nrhs)]
        L = [0.1 * (3 ** j) for j in range(nlam)]
        probs.append((col, row, B, L))
        cols.append(col); rows.append(row); bs.extend(B); lams.extend(L)
    x, info = P.solve_batched([s[0] for s in shapes], [s[1] for s in shapes], dev(np.concatenate(cols)),
                              dev(np.concatenate(rows)), lams, nrhs, dev(np.concatenate(bs)))
    torch.cuda.synchronize()
    x = x.cpu().numpy()
    assert (info.cpu().numpy() == 0).all()
    off = 0
    for (col, row, B, L) in probs:
        n = len(row)
        for lam in L:
            for b in B:
                assert relerr(x[off:off + n], oracle.solve(col, row, b, lam)) <= TOL
                off += n
    assert off == len(x)


@pytest.mark.parametrize("chunk_groups", [1, 5])
def test_chunked_batch_side_by_side(P, chunk_groups):
    """A batch split into chunks of at most chunk_groups groups (equal chunks, run side by
    side on several streams) gives the oracle's solutions, as the one-chunk batch does."""
    rng = np.random.default_rng(7)
    m, n, nlam, nrhs = 260, 200, 3, 4
    probs = [W.random_problem(rng, m, n, L=12.0)[:2] for _ in range(4)]
    B = [[rng.standard_normal(m) for _ in range(nrhs)] for _ in probs]
    lams = [0.05 * (4 ** j) for j in range(nlam)]
    args = ([m] * 4, [n] * 4, dev(np.concatenate([c for c, _ in probs])), dev(np.concatenate([r for _, r in probs])),
            lams * 4, nrhs, dev(np.concatenate([np.concatenate(b) for b in B])))
    x1, i1 = P.solve_batched(*args)
    P.set_options(chunk_groups=chunk_groups)
    try:
        x2, i2 = P.solve_batched(*args)
        torch.cuda.synchronize()
    finally:
        P.set_options(chunk_groups=0)
    assert (i1.cpu().numpy() == 0).all() and (i2.cpu().numpy() == 0).all()
    x1, x2 = x1.cpu().numpy(), x2.cpu().numpy()
    off = 0
    for (col, row), bs in zip(probs, B):
        for lam in lams:
            for b in bs:
                ref = oracle.solve(col, row, b, lam)
                assert relerr(x2[off:off + n], ref) <= TOL
                assert relerr(x2[off:off + n], x1[off:off + n]) <= TOL
                off += n
    assert off == len(x2)


def test_adaptive_refinement_batched(P):
    """Groups whose estimated error is still above the target after the
    mandatory refinement step take more steps, after being exchanged to the
    front of the batch; the others stop.  Over a lambda path (kappa from about
    1 to 1e6) a sweep of targets flags ragged subsets; the number of extra
    steps never grows as the target loosens, and every solve of every run
    must match the oracle at its own output position."""
    probs = [W.headline(i, n=1024, nrhs=2, nlam=8) for i in range(3)]
    ms = [p.m for p in probs]
    ns = [p.n for p in probs]
    args = (ms, ns, dev(np.concatenate([p.col for p in probs])), dev(np.concatenate([p.row for p in probs])),
            [l for p in probs for l in p.lams], 2, dev(np.concatenate([np.concatenate(p.b) for p in probs])))
    nsolve = 3 * 8 * 2
    ref = [oracle.solve(p.col, p.row, b, lam) for p in probs for lam in p.lams for b in p.b]
    extras = []
    for tol in (1e-10, 1e-16, 1e-20, 1e-24, 1e-28):
        P.set_options(refine=1, refine_max=3, refine_tol=tol)
        try:
            x, info = P.solve_batched(*args)
            torch.cuda.synchronize()
            extra = P.get_stats()["refine_extra"]
        finally:
            P.set_options(refine=1, refine_max=3, refine_tol=1e-10)
        x = x.cpu().numpy()
        assert (info.cpu().numpy() == 0).all()
        off = 0
        for i, xr in enumerate(ref):
            n = len(xr)
            assert relerr(x[off:off + n], xr) <= TOL, (tol, i)
            off += n
        assert off == len(x)
        extras.append(extra)
    print("extra refinement steps per target:", extras)
    assert all(a <= b for a, b in zip(extras, extras[1:])), extras
    assert any(0 < e < 2 * nsolve for e in extras), extras


def test_refinement_skipped_when_certified(P):
    """Before the first refinement step, the groups whose first solves are certified to
    refine_tol by the a-posteriori bound ||x - x*|| <= ||r|| / lambda^2 (plus the residual's
    rounding margin) take no refinement step: the large lambdas of a path from kappa ~ 1e6
    to ~2; the small ones cannot be certified and refine.  Every solve matches the oracle
    with the filter on and off."""
    probs = [W.headline(i, n=1024, nrhs=2, nlam=8) for i in range(3)]
    ms = [p.m for p in probs]
    ns = [p.n for p in probs]
    args = (ms, ns, dev(np.concatenate([p.col for p in probs])), dev(np.concatenate([p.row for p in probs])),
            [l for p in probs for l in p.lams], 2, dev(np.concatenate([np.concatenate(p.b) for p in probs])))
    nsolve = 3 * 8 * 2
    ref = [oracle.solve(p.col, p.row, b, lam) for p in probs for lam in p.lams for b in p.b]
    out = {}
    for skip in (0, 1):
        P.set_options(refine=1, refine_max=3, refine_skip=skip)
        try:
            x, info = P.solve_batched(*args)
            torch.cuda.synchronize()
            out[skip] = (x.cpu().numpy(), info.cpu().numpy(), P.get_stats()["refine_skipped"])
        finally:
            P.set_options(refine_skip=0)
    assert out[0][2] == 0
    assert 0 < out[1][2] < nsolve and out[1][2] % 2 == 0   # whole groups of 2 right-hand sides
    for skip in (0, 1):
        x, info, _ = out[skip]
        assert (info == 0).all()
        off = 0
        for i, xr in enumerate(ref):
            n = len(xr)
            assert relerr(x[off:off + n], xr) <= TOL, (skip, i)
            off += n
    assert relerr(out[1][0], out[0][0]) <= TOL


@pytest.mark.parametrize("defer_tol", [1e-3, 2e-3])
@pytest.mark.parametrize("nlim", [64, 256])
def test_difficult_points_deferred(P, defer_tol, nlim):
    """Difficult points (Sec. 5): with a deferral threshold, chosen conditions
    whose pivot entry is small relative to their row are set aside, carried
    through the products, and processed after the root against the final
    basis.  Headline-shaped problems (m - n spread, lambda path) have pivot
    ratios down to about 1e-5; every solve must still match the oracle."""
    pr = W.headline(0, n=512, nrhs=1, nlam=8)
    rng = np.random.default_rng(11)
    colc, rowc, bc = W.random_problem(rng, 300, 211, cplx=True, L=20.0)
    cases = [(pr.col, pr.row, pr.b[0], pr.lams[j]) for j in (0, 3, 7)] + [(colc, rowc, bc, 0.05)]
    P.set_options(n_lim=nlim, defer_tol=defer_tol)
    try:
        deferred = 0
        for col, row, b, lam in cases:
            x = P.solve(dev(col), dev(row), dev(b), lam).cpu().numpy()
            deferred += P.get_stats()["deferred"]
            assert relerr(x, oracle.solve(col, row, b, lam)) <= TOL, (len(col), len(row), lam)
    finally:
        P.set_options(n_lim=256, defer_tol=0.0)
    assert deferred > 0


@pytest.mark.parametrize("nlim", [128, 192, 256])
@pytest.mark.parametrize("defer_tol", [0.0, 1e-3])
def test_leaf_single_wavefront_parity(P, nlim, defer_tol):
    """The leaf steps (Alg. 1, leaf case) run either with one wavefront per 64
    conditions or, for large batches, with one wavefront per group holding
    several conditions per lane.  Forcing each path on the same batch, both
    must match the oracle and each other."""
    pr = W.headline(0, n=512, nrhs=2, nlam=4)
    args = ([pr.m], [pr.n], dev(pr.col), dev(pr.row), list(pr.lams), 2, dev(np.concatenate(pr.b)))
    ref = [oracle.solve(pr.col, pr.row, b, lam) for lam in pr.lams for b in pr.b]
    xs = []
    for wg in (1, 1 << 30):
        P.set_options(n_lim=nlim, defer_tol=defer_tol, leaf_wave_groups=wg)
        try:
            x, info = P.solve_batched(*args)
            torch.cuda.synchronize()
        finally:
            P.set_options(n_lim=256, defer_tol=0.0, leaf_wave_groups=LEAF_WAVE_GROUPS)
        x = x.cpu().numpy()
        assert (info.cpu().numpy() == 0).all(), (wg, nlim, defer_tol)
        for i, xr in enumerate(ref):
            assert relerr(x[i * pr.n:(i + 1) * pr.n], xr) <= TOL, (wg, nlim, defer_tol, i)
        xs.append(x)
    assert relerr(xs[0], xs[1]) <= 1e-12


def test_difficult_points_capacity(P):
    """More deferred conditions than a solve holds is reported (info bit 4),
    not silently dropped."""
    rng = np.random.default_rng(5)
    col, row, b = W.random_problem(rng, 300, 211, L=20.0)
    P.set_options(n_lim=256, defer_tol=0.9)
    try:
        with pytest.raises(P.TikhError):
            P.solve(dev(col), dev(row), dev(b), 0.2)
    finally:
        P.set_options(n_lim=256, defer_tol=0.0)


def _ld_T(col, row, v):
    """T v in 80-bit long double (direct sums), for constructing exact right-hand sides."""
    col = np.asarray(col, np.longdouble); row = np.asarray(row, np.longdouble); v = np.asarray(v, np.longdouble)
    m, n = len(col), len(row)
    g = np.concatenate([row[1:][::-1], col])
    return np.convolve(g, v)[n - 1:n - 1 + m]


def _ld_TH(col, row, v):
    col = np.asarray(col, np.longdouble); row = np.asarray(row, np.longdouble); v = np.asarray(v, np.longdouble)
    m, n = len(col), len(row)
    g = np.concatenate([row[1:][::-1], col])
    return np.convolve(g[::-1], v)[m - 1:m - 1 + n]


@pytest.mark.parametrize("j", [0, 7])
def test_headline_size_known_solution(P, j):
    """n = 2^14, m = n + U{0..n/4} (the headline shape), lambda from the certified
    path (kappa <= 1 + 1e6 at j = 0).  As in the paper's accuracy experiments
    (Sec. 7.1-7.2) the normal-form system (T^H T + lambda^2 I) x = y is solved
    for a known x with y formed in long double and rounded once, so the known x
    is the exact solution to within kappa * u ~ 1e-10."""
    pr = W.headline(0)
    lam = pr.lams[j]
    xt = pr.x_true
    y = (_ld_TH(pr.col, pr.row, _ld_T(pr.col, pr.row, xt)) + np.longdouble(lam) ** 2 * xt).astype(np.float64)
    x = P.solve_normal(dev(pr.col), dev(pr.row), dev(y), lam).cpu().numpy()
    assert relerr(x, xt) <= TOL, (j, relerr(x, xt))


def test_headline_size_rhs_transform(P):
    """The least-squares entry forms T^H b on the GPU by FFTs; at full size it must
    agree with the normal-form entry fed T^H b computed in long double."""
    pr = W.headline(1)
    lam = pr.lams[4]
    b = pr.b[0]
    y = _ld_TH(pr.col, pr.row, b).astype(np.float64)
    x1 = P.solve(dev(pr.col), dev(pr.row), dev(b), lam).cpu().numpy()
    x2 = P.solve_normal(dev(pr.col), dev(pr.row), dev(y), lam).cpu().numpy()
    assert relerr(x1, x2) <= TOL


@pytest.mark.parametrize("n,cplx", [(1000, False), (4096, True), (2 ** 14, False)])
def test_circulant_closed_form_gpu(P, n, cplx):
    """Circulant T (m = n, a_{-j} = a_{n-j}): the Fourier-domain closed form
    x = IDFT(conj(a^) b^ / (|a^|^2 + lambda^2)) holds at any size; lambda is set so
    that the regularized normal matrix has condition number 1e6."""
    rng = np.random.default_rng(n + 31 * cplx)
    c = rng.standard_normal(n) + (1j * rng.standard_normal(n) if cplx else 0)
    col = c.copy()
    row = np.concatenate([[c[0]], c[1:][::-1]])
    b = rng.standard_normal(n) + (1j * rng.standard_normal(n) if cplx else 0)
    ah = np.fft.fft(c)
    lam = float(np.abs(ah).max()) * 1e-3
    xe = np.fft.ifft(np.conj(ah) * np.fft.fft(b) / (np.abs(ah) ** 2 + lam ** 2))
    if not cplx:
        xe = xe.real
    x = P.solve(dev(col), dev(row), dev(b), lam).cpu().numpy()
    assert relerr(x, xe) <= TOL, (n, cplx, relerr(x, xe))


@pytest.mark.parametrize("m,n", [(500, 500), (700, 500), (300, 450)])
def test_scaled_identity_and_zero_gpu(P, m, n):
    """T = c [I; 0] (only a_0 = c nonzero): x = conj(c) b[:n] / (|c|^2 + lambda^2) (with
    zeros past row m when m < n); T = 0: x = 0 from the least-squares entry and
    x = y / lambda^2 from the normal form.  Generators with all but one entry zero, or
    none, give residual columns that are exactly zero."""
    rng = np.random.default_rng(m + 7 * n)
    c = 1.5 - 0.5j
    col = np.zeros(m, complex); col[0] = c
    row = np.zeros(n, complex); row[0] = c
    b = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    lam = 0.8
    xe = np.zeros(n, complex)
    k = min(m, n)
    xe[:k] = np.conj(c) * b[:k] / (abs(c) ** 2 + lam ** 2)
    x = P.solve(dev(col), dev(row), dev(b), lam).cpu().numpy()
    assert relerr(x, xe) <= TOL, relerr(x, xe)
    z = np.zeros(m)
    x0 = P.solve(dev(z), dev(np.zeros(n)), dev(b.real), lam).cpu().numpy()
    assert np.abs(x0).max() == 0.0
    y = rng.standard_normal(n)
    xn = P.solve_normal(dev(z), dev(np.zeros(n)), dev(y), lam).cpu().numpy()
    assert relerr(xn, y / lam ** 2) <= TOL


def test_scaling_law_gpu(P):
    """x(alpha T, alpha lambda, b) = x(T, lambda, b) / alpha, for a ragged tall problem
    over three leaf levels, alpha a power of two and not."""
    rng = np.random.default_rng(404)
    col, row, b = W.random_problem(rng, 700, 611, cplx=True, L=15.0)
    lam = 0.05
    x1 = P.solve(dev(col), dev(row), dev(b), lam).cpu().numpy()
    assert relerr(x1, oracle.solve(col, row, b, lam)) <= TOL
    for alpha in (0.0625, 3.7, 1e3):
        xa = P.solve(dev(alpha * col), dev(alpha * row), dev(b), alpha * lam).cpu().numpy()
        assert relerr(alpha * xa, x1) <= TOL, (alpha, relerr(alpha * xa, x1))


def test_invalid_lambda_and_sizes(P):
    c = dev(np.ones(4)); r = dev(np.ones(4)); b = dev(np.ones(4))
    for lam in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(P.TikhError):
            P.solve(c, r, b, lam)


def test_nonfinite_input_reports_info(P):
    col = np.ones(20); col[3] = np.nan
    with pytest.raises(P.TikhError) as e:
        P.solve(dev(col), dev(np.ones(10)), dev(np.ones(20)), 0.5)
    assert e.value.code == -4
    # a non-finite right-hand side leaves the pivots (columns 1..4) intact: only the
    # non-finite bit (8) is set, for that solve alone
    rng = np.random.default_rng(8)
    col, row, _ = W.random_problem(rng, 40, 30, L=6.0)
    b = rng.standard_normal((2, 40))
    b[1, 5] = np.inf
    x, info = P.solve_batched([40], [30], dev(col), dev(row), [0.3], 2, dev(b.ravel()))
    torch.cuda.synchronize()
    assert info.cpu().numpy().tolist() == [0, 8]
    assert relerr(x[:30].cpu().numpy(), oracle.solve(col, row, b[0], 0.3)) <= TOL


@pytest.mark.parametrize("nrhs,cplx", [(3, False), (4, True), (5, False)])
def test_batched_rhs_groups(P, nrhs, cplx):
    """Right-hand sides of one (problem, lambda) share the pivot sequence and
    ride along in one recursion (groups of 1, 2 or 4; the last group padded):
    every solve must still match the oracle."""
    rng = np.random.default_rng(700 + nrhs)
    shapes = [(90, 64), (41, 77)]
    lams = []
    cols, rows, bs, probs = [], [], [], []
    for (m, n) in shapes:
        col, row, _ = W.random_problem(rng, m, n, cplx=cplx, L=9.0)
        B = [rng.standard_normal(m) + (1j * rng.standard_normal(m) if cplx else 0) for _ in range(nrhs)]
        L = [0.15, 0.6]
        probs.append((col, row, B, L)); cols.append(col); rows.append(row); bs.extend(B); lams.extend(L)
    x, info = P.solve_batched([s[0] for s in shapes], [s[1] for s in shapes], dev(np.concatenate(cols)),
                              dev(np.concatenate(rows)), lams, nrhs, dev(np.concatenate(bs)), complex_data=cplx)
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all()
    x = x.cpu().numpy()
    off = 0
    for (col, row, B, L) in probs:
        n = len(row)
        for lam in L:
            for b in B:
                assert relerr(x[off:off + n], oracle.solve(col, row, b, lam)) <= TOL
                off += n
    assert off == len(x)


def test_autotune_nlim(P):
    """The leaf-cutoff autotuner times the candidates on synthetic data, keeps the
    fastest in the options, and solves stay correct under the chosen cutoff."""
    try:
        best, ms = P.autotune_nlim(384, 256, groups=8, nrhs=2)
        assert best in (64, 128, 192, 256)
        assert best in ms and all(v > 0 for v in ms.values())
        assert ms[best] == min(ms.values())
        assert P.get_options()["n_lim"] == best
        pr = W.config0()
        x = P.solve(dev(pr.col), dev(pr.row), dev(pr.b[0]), pr.lams[0]).cpu().numpy()
        assert relerr(x, oracle.solve(pr.col, pr.row, pr.b[0], pr.lams[0])) <= TOL
    finally:
        P.set_options(n_lim=256)
    with pytest.raises(P.TikhError):
        P.autotune_nlim(384, 256, groups=0)


def _banded_normal_ld(h, n, v, lam):
    """(T^H T + lam^2 I) v in long double for T = full convolution with taps h (m = n + len(h) - 1)."""
    hl = np.asarray(h, np.longdouble); vl = np.asarray(v, np.longdouble)
    tv = np.convolve(hl, vl)                                  # T v, length n + len(h) - 1
    thtv = np.convolve(tv, hl[::-1])[len(h) - 1:len(h) - 1 + n]
    return thtv + np.longdouble(lam) ** 2 * vl


def test_deblurring_full_size_known_solution(P):
    """The plain method at scale (1-D deblurring, n = 2^16, m = n + 192, Gaussian PSF
    with 193 taps, lambda = 1e-2, kappa <= 1 + 1/lambda^2 = 1e4): normal form with a
    right-hand side formed in long double from the known piecewise-constant x."""
    pr = W.config1()
    h = pr.col[:193]
    assert np.all(pr.col[193:] == 0) and np.all(pr.row[1:] == 0)
    lam = pr.lams[0]
    y = _banded_normal_ld(h, pr.n, pr.x_true, lam).astype(np.float64)
    x = P.solve_normal(dev(pr.col), dev(pr.row), dev(y), lam).cpu().numpy()
    assert relerr(x, pr.x_true) <= TOL, relerr(x, pr.x_true)


def _band_oracle(col, row, rhs_by_lam, lams, normal=False):
    """Banded-QR oracle solutions for several lambdas at once (one thread per lambda; the
    C oracle releases the interpreter lock): returns [len(lams)][nrhs][n]."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(16, len(lams))) as ex:
        futs = [ex.submit(oracle.band_solve, col, row, rhs, lam, normal) for rhs, lam in zip(rhs_by_lam, lams)]
        return [f.result() for f in futs]


def test_headline_batch_full_config_sampled(P):
    """The benchmark's launch configuration: 256 problems of the headline shape
    (n = 2^14, m = n + U{0..n/4}) x 8 lambdas x 4 right-hand sides in one
    batched call, i.e. 2048 groups in one chunk, which takes the one-wavefront-
    per-group leaf steps.  32 generated problems are used 8 times each, every
    copy with its lambda path scaled by its own factor so that no two groups
    hold the same data.  Every solve of two copies of the generated problem
    with the narrowest generator support (all 8 lambdas, kappa up to 1 + 1e6,
    and all 4 right-hand sides) is compared element by element with the banded
    QR oracle; sampled solves elsewhere in the batch with the single-problem path."""
    base = [W.headline(i, n=2 ** 14, nrhs=4, nlam=8) for i in range(32)]
    probs = []
    for c in range(8):
        for p in base:
            probs.append((p, [lam * (1.0 + 0.01 * c) for lam in p.lams]))
    ms = [p.m for p, _ in probs]
    ns = [p.n for p, _ in probs]
    lams = [l for _, ls in probs for l in ls]
    col = dev(np.concatenate([p.col for p, _ in probs]))
    row = dev(np.concatenate([p.row for p, _ in probs]))
    bb = dev(np.concatenate([np.concatenate(p.b) for p, _ in probs]))
    P.set_options(n_lim=256, refine=1, leaf_wave_groups=1536)
    try:
        x, info = P.solve_batched(ms, ns, col, row, lams, 4, bb)
        torch.cuda.synchronize()
    finally:
        P.set_options(leaf_wave_groups=LEAF_WAVE_GROUPS)
    assert (info.cpu().numpy() == 0).all()
    x = x.cpu().numpy()
    n = 2 ** 14
    inarrow = min(range(32), key=lambda i: base[i].meta["L"])
    for ip in (inarrow, inarrow + 7 * 32):
        p, ls = probs[ip]
        ref = _band_oracle(p.col, p.row, [p.b] * 8, ls)
        for j in range(8):
            for r in range(4):
                off = ((ip * 8 + j) * 4 + r) * n
                e = relerr(x[off:off + n], ref[j][r])
                assert e <= TOL, (ip, j, r, e)
    for (ip, j, r) in [(0, 0, 0), (77, 7, 3), (150, 3, 1)]:
        p, ls = probs[ip]
        off = ((ip * 8 + j) * 4 + r) * n
        xs = P.solve(dev(p.col), dev(p.row), dev(p.b[r]), ls[j]).cpu().numpy()
        assert relerr(x[off:off + n], xs) <= TOL, (ip, j, r, relerr(x[off:off + n], xs))


def test_deblurring_full_size_vs_band_oracle(P):
    """The plain method at scale through the least-squares entry: 1-D deblurring at
    n = 2^16, m = n + 192 (193-tap Gaussian PSF, lambda = 1e-2, b with noise), against
    the banded QR oracle (exact for the PSF's finite support)."""
    pr = W.config1()
    lam = pr.lams[0]
    x = P.solve(dev(pr.col), dev(pr.row), dev(pr.b[0]), lam).cpu().numpy()
    xr = oracle.band_solve(pr.col, pr.row, [pr.b[0]], lam)[0]
    assert relerr(x, xr) <= TOL, relerr(x, xr)


def test_caller_workspace(P):
    """A caller-owned workspace (tikh_workspace_bytes / tikh_set_workspace): with
    the queried size the batch runs in one chunk, as with the library's own
    buffer, and gives its results bit for bit; with a third of it the batch runs
    in several chunks, whose product transforms are sized by each chunk's own
    degrees, so the results agree to rounding.  The backward too.  A buffer too
    small for one group is reported, and NULL returns to the library's own."""
    rng = np.random.default_rng(77)
    shapes = [(300, 211), (260, 230), (290, 199)]
    nlam, nrhs = 2, 4
    cols, rows, bs, lams = [], [], [], []
    for (m, n) in shapes:
        col, row, _ = W.random_problem(rng, m, n, L=12.0)
        cols.append(col); rows.append(row)
        bs.extend(rng.standard_normal(m) for _ in range(nrhs))
        lams.extend([0.3, 0.05])
    ms = [s[0] for s in shapes]; ns = [s[1] for s in shapes]
    args = (ms, ns, dev(np.concatenate(cols)), dev(np.concatenate(rows)), lams, nrhs, dev(np.concatenate(bs)))

    def run():
        x, info = P.solve_batched(*args)
        gx = x * 0.5
        gc, gr, gb, gl, binfo = P.backward_batched(*args, x, gx)
        torch.cuda.synchronize()
        assert (info.cpu().numpy() == 0).all() and (binfo.cpu().numpy() == 0).all()
        return [t.cpu().numpy() for t in (x, gc, gr, gb, gl)]

    ref = run()
    nbytes = P.workspace_bytes(ms, ns, nlam, nrhs)
    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    try:
        P.set_workspace(buf)
        for a, b in zip(run(), ref):
            assert np.array_equal(a, b)
        P.set_workspace(buf[:nbytes // 3])
        for a, b in zip(run(), ref):
            assert relerr(a, b) <= 1e-12
        P.set_workspace(buf[:1 << 16])
        with pytest.raises(P.TikhError):
            P.solve_batched(*args)
    finally:
        P.set_workspace(None)
    for a, b in zip(run(), ref):
        assert np.array_equal(a, b)
    x = ref[0]
    assert relerr(x[:211], oracle.solve(cols[0], rows[0], bs[0], lams[0])) <= TOL


def test_headline_problems_with_tight_extension(P):
    """Headline-shaped problems whose extension k = N - (m + n - 1) lies in 43..89 (4 of the
    256 benchmark problems).  With a zero threshold of 1e-11 their leaves pivoted the
    gamma_1 column on rounding noise (a residual entry that is zero in exact arithmetic)
    and the basis lost the solution; with 1e-9 they solve like the rest, with no fallback
    solve, and match known solutions (normal form, right-hand side formed in long double)
    at the ends of the lambda path."""
    picks = [35, 54, 94, 249]
    probs = [W.headline(i) for i in picks]
    for p in probs:
        assert 40 <= P.plan_info(p.m, p.n, 256)[3] <= 90
    args = ([p.m for p in probs], [p.n for p in probs], dev(np.concatenate([p.col for p in probs])),
            dev(np.concatenate([p.row for p in probs])), [l for p in probs for l in p.lams], 4,
            dev(np.concatenate([np.concatenate(p.b) for p in probs])))
    P.set_options(n_lim=256, refine=1)
    x, info = P.solve_batched(*args)
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all()
    assert P.get_stats()["fallback_groups"] == 0
    x = x.cpu().numpy()
    off = 0
    for p in probs:
        for j, lam in enumerate(p.lams):
            for r in range(4):
                res = oracle.normal_residual_fft(p.col, p.row, p.b[r], lam, x[off:off + p.n])
                assert res <= 1e-11, (j, r, res)
                off += p.n
    for p in probs[:2]:
        for j in (0, 7):
            lam = p.lams[j]
            y = (_ld_TH(p.col, p.row, _ld_T(p.col, p.row, p.x_true)) + np.longdouble(lam) ** 2 * p.x_true).astype(
                np.float64)
            xs = P.solve_normal(dev(p.col), dev(p.row), dev(y), lam).cpu().numpy()
            assert relerr(xs, p.x_true) <= TOL, (j, relerr(xs, p.x_true))


def test_fallback_leaf_cutoff(P):
    """A group whose solve failed is solved again with the fallback leaf cutoff.  Forced
    here with non-finite data (info bit 8 persists: the second solve fails too, and the
    outputs are those of the second solve) and, for a solvable problem, by counting: no
    group of a sound batch takes the fallback."""
    rng = np.random.default_rng(91)
    col, row, _ = W.random_problem(rng, 300, 250, L=8.0)
    b = rng.standard_normal((2, 300))
    b[0, 7] = np.nan
    x, info = P.solve_batched([300], [250], dev(col), dev(row), [0.2, 0.7], 2, dev(b.ravel()))
    torch.cuda.synchronize()
    st = P.get_stats()
    assert info.cpu().numpy().tolist() == [8, 0, 8, 0]
    assert st["fallback_groups"] == 2
    x = x.cpu().numpy()
    assert relerr(x[250:500], oracle.solve(col, row, b[1], 0.2)) <= TOL
    assert relerr(x[750:1000], oracle.solve(col, row, b[1], 0.7)) <= TOL
