"""Bilevel lambda tuning at full size (256 deblurring problems, Gaussian PSF with sigma in
[4, 48], n log-uniform in [2^12, 2^16]; each problem's log lambda by Adam steps on a
validation loss with an independent noise draw), one captured graph per step: the
gradients and losses of the first step against the banded QR oracle on a sample, the first
replay against an eager step, every solve's info word, and the loss decrease over 5 steps
(the benchmark runs the workload's 20)."""
import sys
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle
import workloads as W

NPROB, STEPS = 256, 5


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1302_6945_amd as P
    P.set_options(n_lim=256, refine=1, refine_max=3, defer_tol=0.0)
    # the prepared batches hold workspaces of their own: return the library's shared one
    P.set_workspace(None)
    torch.cuda.empty_cache()
    yield P


def dev(a):
    return torch.tensor(np.asarray(a), device="cuda:0")


@pytest.fixture(scope="module")
def problems():
    return [W.config4(i) for i in range(NPROB)]


def _tuner(P, probs):
    ms = [p.m for p in probs]
    ns = [p.n for p in probs]
    col = dev(np.concatenate([p.col for p in probs]))
    row = dev(np.concatenate([p.row for p in probs]))
    b = dev(np.concatenate([p.b[0] for p in probs]))
    bval = dev(np.concatenate([p.b[1] for p in probs]))
    lam0 = dev(np.array([p.lams[0] for p in probs]))
    return P.BilevelTuner(ms, ns, col, row, b, bval, lam0)


def _oracle_step0(p):
    """Loss and dL/dlambda at the initial lambda by the banded QR oracle."""
    b, bval, lam = p.b[0], p.b[1], p.lams[0]
    x = oracle.band_solve(p.col, p.row, [b], lam)[0]
    r = oracle.T_apply(p.col, p.row, x) - bval
    gx = oracle.TH_apply(p.col, p.row, r).real
    g = oracle.band_gradients(p.col, p.row, b, lam, x, gx, with_lag_sums=False)
    return 0.5 * float(np.vdot(r, r).real), g["g_lam"]


def _say(msg, t0):
    print("config4: %s (%.1f s)" % (msg, time.perf_counter() - t0), file=sys.stderr, flush=True)


def test_config4_bilevel_captured(P, problems):
    t0 = time.perf_counter()
    tuner = _tuner(P, problems)
    _say("prepared", t0)
    try:
        tuner.capture()                 # (an eager step first, the state restored)
        eager = tuner.eager_step[:2]
        _say("captured", t0)
        losses, worst_info = [], 0
        for k in range(STEPS):
            tuner.step()
            torch.cuda.synchronize()
            fi, bi = tuner.info()
            worst_info = max(worst_info, int(fi.max().item()), int(bi.max().item()))
            # the loss at the lambdas this step started from (its forward solutions)
            losses.append(tuner.validation_loss().cpu().numpy())
            _say("step %d" % k, t0)
            est = tuner.loss.cpu().numpy()
            assert np.all(np.abs(est - losses[-1]) <= 1e-3 * losses[-1])
            if k == 0:
                for a, e in zip((tuner.loglam, tuner.grad), eager):
                    a, e = a.cpu().numpy(), e.cpu().numpy()
                    assert np.max(np.abs(a - e) / np.maximum(np.abs(e), 1e-300)) <= 1e-8
                grad0 = tuner.grad.cpu().numpy().copy()
        assert worst_info == 0
        # first step against the oracle: the smallest problems, and one of each PSF width extreme
        ns = np.array([p.n for p in problems])
        sig = np.array([p.meta["sigma"] for p in problems])
        sample = sorted(set(list(np.argsort(ns)[:3]) + [int(np.argmin(sig)), int(np.argmax(sig))]),
                        key=lambda i: ns[i])[:4]
        for i in sample:
            p = problems[i]
            L0, g_lam = _oracle_step0(p)
            assert abs(losses[0][i] - L0) <= 1e-9 * L0, (i, losses[0][i], L0)
            want = p.lams[0] * g_lam                 # dL/dlog(lambda)
            assert abs(grad0[i] - want) <= 1e-7 * max(abs(want), 1e-300), (i, grad0[i], want)
        # the validation loss goes down over the 20 steps
        assert losses[-1].sum() < losses[0].sum()
        assert np.mean(losses[-1] < losses[0]) >= 0.9
        lam = torch.exp(tuner.loglam).cpu().numpy()
        assert np.all(np.isfinite(lam)) and np.all(lam > 0)
    finally:
        tuner.free()
