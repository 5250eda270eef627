"""Launch timing (tikh_profile_kernel / tikh_profile_read / tikh_profile_units), which the
benchmark's roofline figures rest on: the launch counts and the algorithmic units of the
timed launches against closed forms, for the batched FFT (one read and one write of every
transformed element per pass) and the leaf steps of one solve (Alg. 1, leaf case:
12 flops to score each remaining condition and 8 C to update it, C basis columns)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import workloads as W


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1302_6945_amd as P
    P.set_options(n_lim=256, refine=1, refine_max=3)
    yield P
    P.profile_kernel(None)


def test_fft_launches_and_bytes(P):
    rng = np.random.default_rng(5)
    P.profile_kernel("fft")
    try:
        # one pass: items x lines x len elements, 16 bytes read and 16 written each
        x = torch.tensor(rng.standard_normal((3, 5, 1024)) + 0j, device="cuda")
        P.fft_batched(x, -1)
        ms, count, units = P.profile_read()
        assert count == 1 and ms > 0.0
        assert units == 32.0 * 3 * 5 * 1024
        # 9216 points: two passes over every element (the reordering copy is not an FFT launch)
        P.profile_kernel("fft")
        y = torch.tensor(rng.standard_normal((2, 3, 9216)) + 0j, device="cuda")
        P.fft_batched(y, 1)
        ms, count, units = P.profile_read()
        assert count == 2 and ms > 0.0
        assert units == 2 * 32.0 * 2 * 3 * 9216
        # disabled: nothing is counted
        P.profile_kernel(None)
        P.fft_batched(x, 1)
        assert P.profile_read()[1] == 0
    finally:
        P.profile_kernel(None)


def test_leaf_launches_and_flops(P):
    rng = np.random.default_rng(6)
    m, n = 700, 600
    N, M, depth, k = P.plan_info(m, n, 256)
    K = 2 * M                          # two conditions per node, M nodes per leaf
    C = 5                              # four basis columns and one right-hand side
    per_leaf = 12.0 * K * (K + 1) / 2 + 8.0 * C * K * (K - 1) / 2
    col, row, b = W.random_problem(rng, m, n, L=12.0)
    dev = lambda a: torch.tensor(np.asarray(a), device="cuda")
    P.profile_kernel("leaf_loop")
    try:
        P.solve(dev(col), dev(row), dev(b), 0.3)
        ms, count, units = P.profile_read()
    finally:
        P.profile_kernel(None)
    # every recursion (the solve and each refinement step) runs one launch per leaf
    assert count >= 2 * 2 ** depth and count % 2 ** depth == 0, (count, depth)
    assert ms > 0.0
    assert units == count * per_leaf
