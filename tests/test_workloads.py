"""The seeded input generators follow their stated recipes (shapes, value laws, lambda paths,
right-hand-side construction); checked on the host against the definitions, with the
oracle's products with T as an independent matvec."""
import math

import numpy as np

import oracle
import workloads as W


def _tx(col, row, x):
    return oracle.T_apply(col, row, x).real


def test_config1_deblurring():
    p = W.config1(n=2 ** 10)
    h = p.col[:193]
    assert len(p.col) == 2 ** 10 + 192 and len(p.row) == 2 ** 10
    assert abs(h.sum() - 1.0) <= 1e-14 and np.argmax(h) == 96
    assert np.all(p.col[193:] == 0.0) and np.all(p.row[1:] == 0.0) and p.row[0] == p.col[0]
    assert p.lams == [1e-2] and p.x_true[0] == 0.0
    assert len(np.unique(np.diff(p.x_true) != 0)) == 2 and np.count_nonzero(np.diff(p.x_true)) <= 64
    noise = p.b[0] - _tx(p.col, p.row, p.x_true)
    assert 0.5e-3 < noise.std() < 2e-3


def test_config2_batching_law():
    for i in range(20):
        p = W.config2(i)
        assert 512 <= p.n <= 16384 and 0 <= p.m - p.n <= p.n // 4
        assert 8 <= p.meta["L"] <= 128
        assert np.allclose(p.lams, [10.0 ** (-4 + 4 * j / 7.0) for j in range(8)], rtol=1e-15)
        assert len(p.b) == 4 and all(len(b) == p.m for b in p.b)
        # the envelope is cut at 40 L on both sides of the main diagonal
        cut = int(40 * p.meta["L"])
        assert np.all(p.col[cut + 1:] == 0.0) and np.all(p.row[cut + 1:] == 0.0)


def test_headline_lambda_path_certifies_kappa():
    p = W.headline(3, n=1024)
    ratios = np.array(p.lams[1:]) / np.array(p.lams[:-1])
    assert np.allclose(ratios, 10.0 ** (3.0 / 7.0), rtol=1e-12)
    assert abs(p.lams[-1] - p.meta["smax"]) <= 1e-12 * p.meta["smax"]
    # lambda_0 = smax 1e-3 and smax >= ||T||_2 give kappa <= 1 + 1e6
    T = oracle.dense_T(p.col, p.row)
    s1 = np.linalg.norm(T, 2)
    assert s1 <= p.meta["smax"]
    assert 1.0 + (s1 / p.lams[0]) ** 2 <= 1.0 + 1e6 + 1e-6


def test_config4_bilevel_problems():
    for i in range(12):
        p = W.config4(i)
        sigma = p.meta["sigma"]
        taps = 2 * int(math.ceil(4 * sigma)) + 1
        assert 4.0 <= sigma <= 48.0
        assert 4096 <= p.n <= 65536 and p.m == p.n + taps - 1
        h = p.col[:taps]
        assert abs(h.sum() - 1.0) <= 1e-13 and np.all(p.col[taps:] == 0.0)
        assert p.row[0] == p.col[0] and np.all(p.row[1:] == 0.0)
        assert p.lams == [1e-2] and len(p.b) == 2
        tx = _tx(p.col, p.row, p.x_true)
        e1, e2 = p.b[0] - tx, p.b[1] - tx
        assert 0.5e-3 < e1.std() < 2e-3 and 0.5e-3 < e2.std() < 2e-3
        assert abs(np.corrcoef(e1, e2)[0, 1]) < 0.1           # independent noise draws


def test_nufft_workload_weights():
    g = W.nufft_problem()
    assert len(g.gram) == 4096 and len(g.lrow) == 4096
    assert abs(g.gram[0].imag) <= 1e-12 and g.gram[0].real > 0
