"""GPU parity for the Toeplitz-Gramian problem (Sec. 2 third case, Sec. 3.4):
x = (G + L^H L)^{-1} y with G Hermitian Toeplitz and L a p x n Toeplitz
regularizer, through the C ABI, against the dense oracle, element by element.
Sizes span one leaf to several tree levels, p below, equal to and above n, real
and complex data, batched calls with several right-hand sides, and the
non-uniform Fourier reconstruction of Sec. 7.4 at its size (n = 4096)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle
import workloads as W

TOL = 1e-9


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1302_6945_amd as P
    P.set_options(n_lim=256, refine=1)
    return P


def dev(a):
    return torch.tensor(np.asarray(a), device="cuda:0")


def relerr(x, xr):
    return np.linalg.norm(np.asarray(x) - xr) / max(np.linalg.norm(xr), 1e-300)


@pytest.mark.parametrize("n,p", [(1, 1), (5, 3), (40, 40), (64, 90), (211, 150), (300, 300), (1000, 998)])
@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("nlim", [64, 256])
def test_gramian_parity(P, n, p, cplx, nlim):
    rng = np.random.default_rng(10 * n + p + 3 * cplx + nlim)
    pr = W.random_gramian(rng, n, p, cplx=cplx, L=6.0)
    P.set_options(n_lim=nlim)
    try:
        x = P.gramian_solve(dev(pr.gram), dev(pr.lcol), dev(pr.lrow), dev(pr.ys[0])).cpu().numpy()
    finally:
        P.set_options(n_lim=256)
    xr = oracle.gramian_solve(pr.gram, pr.lcol, pr.lrow, pr.ys[0])
    if not cplx:
        xr = xr.real
    assert relerr(x, xr) <= TOL, (n, p, cplx, nlim, relerr(x, xr))


def test_gramian_batched_rhs(P):
    """Ragged batch, 3 right-hand sides per problem (groups of 2 sharing the pivot sequence,
    the second padded), complex data."""
    rng = np.random.default_rng(5)
    probs = [W.random_gramian(rng, n, p, cplx=True, L=8.0) for (n, p) in [(120, 100), (77, 90), (256, 256)]]
    nrhs = 3
    ys = [[rng.standard_normal(pr.n) + 1j * rng.standard_normal(pr.n) for _ in range(nrhs)] for pr in probs]
    x, info = P.gramian_solve_batched([pr.p for pr in probs], [pr.n for pr in probs],
                                      dev(np.concatenate([pr.gram for pr in probs])),
                                      dev(np.concatenate([pr.lcol for pr in probs])),
                                      dev(np.concatenate([pr.lrow for pr in probs])), nrhs,
                                      dev(np.concatenate([np.concatenate(y) for y in ys])), complex_data=True)
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all()
    x = x.cpu().numpy()
    off = 0
    for pr, yy in zip(probs, ys):
        for y in yy:
            assert relerr(x[off:off + pr.n], oracle.gramian_solve(pr.gram, pr.lcol, pr.lrow, y)) <= TOL
            off += pr.n


def test_nufft_reconstruction(P):
    """The non-uniform Fourier reconstruction of Sec. 7.4 at its size (n = K = 4096, three
    low-frequency sinusoids, triangular sample density, Voronoi weights, second-difference
    regularizer).  Its regularized matrix has condition number about 1.3e7, beyond the 1e6 of
    the 1e-9 target, so the bound here is 1e-15 times that condition number times 10."""
    pr = W.nufft_problem()
    x = P.gramian_solve(dev(pr.gram), dev(pr.lcol), dev(pr.lrow), dev(pr.ys[0])).cpu().numpy()
    xr = oracle.gramian_solve(pr.gram, pr.lcol, pr.lrow, pr.ys[0])
    assert relerr(x, xr) <= 1.3e-7, relerr(x, xr)
    # the reconstruction itself is as good as the oracle's
    assert abs(relerr(x.real, pr.x_true) - relerr(xr.real, pr.x_true)) < 1e-6
