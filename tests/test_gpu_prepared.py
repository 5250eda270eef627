"""GPU parity of prepared batches (tikh_prepare_batched / tikh_prepare_backward_batched /
tikh_prepared_run): a fixed launch schedule whose lambdas come from a device array, run
eagerly and captured into a graph, against the CPU oracle (dense Householder QR of
[T; lambda I] and its adjoint) and against the ordinary batched entry points."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle
import workloads as W

TOL = 1e-9
SHAPES = [(260, 200), (90, 70), (640, 500), (300, 420)]   # several plans: chunks side by side
NLAM, NRHS = 2, 2


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1302_6945_amd as P
    P.set_options(n_lim=256, refine=1, refine_max=3, defer_tol=0.0)
    yield P
    P.set_options(n_lim=256, refine=1, refine_max=3)


def dev(a):
    return torch.tensor(np.asarray(a), device="cuda:0")


def relerr(x, xr):
    return np.linalg.norm(np.asarray(x) - xr) / max(np.linalg.norm(xr), 1e-300)


@pytest.fixture(scope="module")
def batch():
    rng = np.random.default_rng(1302)
    probs = []
    for (m, n) in SHAPES:
        col, row, _ = W.random_problem(rng, m, n, L=12.0)
        B = [rng.standard_normal(m) for _ in range(NRHS)]
        xt = rng.standard_normal(n)
        lams = [0.08, 0.5]
        probs.append(dict(col=col, row=row, B=B, xt=xt, lams=lams, m=m, n=n))
    return probs


def _args(batch):
    ms = [p["m"] for p in batch]
    ns = [p["n"] for p in batch]
    col = dev(np.concatenate([p["col"] for p in batch]))
    row = dev(np.concatenate([p["row"] for p in batch]))
    b = dev(np.concatenate([np.concatenate(p["B"]) for p in batch]))
    return ms, ns, col, row, b


def _check_forward(batch, x, lams):
    x = x.cpu().numpy()
    off = 0
    for p, (l0, l1) in zip(batch, lams.reshape(-1, NLAM)):
        for lam in (l0, l1):
            for b in p["B"]:
                ref = oracle.solve(p["col"], p["row"], b, float(lam))
                assert relerr(x[off:off + p["n"]], ref) <= TOL, (p["m"], p["n"], lam)
                off += p["n"]
    assert off == len(x)


def test_prepared_forward_runs(P, batch):
    """The first (recording) run and later runs with other lambdas from the device array
    give the oracle's solutions; later runs synchronize nothing."""
    ms, ns, col, row, b = _args(batch)
    lam0 = np.array([l for p in batch for l in p["lams"]])
    lam = dev(lam0)
    pb = P.prepare_batched(ms, ns, col, row, lam, NRHS, b)
    try:
        torch.cuda.synchronize()
        assert (pb.info.cpu().numpy() == 0).all()
        _check_forward(batch, pb.x, lam0)
        assert pb.workspace_bytes() > 0
        for scale in (1.07, 0.93):
            lam.copy_(dev(lam0 * scale))
            pb.run()
            st = P.get_stats()
            torch.cuda.synchronize()
            assert st["host_syncs"] == 0 and st["launches"] > 0
            assert (pb.info.cpu().numpy() == 0).all()
            _check_forward(batch, pb.x, lam0 * scale)
    finally:
        pb.free()


def test_prepared_matches_batched_entry(P, batch):
    """Same solutions as tikh_toeplitz_solve_batched at the same lambdas (both within the
    oracle tolerance of each other)."""
    ms, ns, col, row, b = _args(batch)
    lam0 = [l for p in batch for l in p["lams"]]
    pb = P.prepare_batched(ms, ns, col, row, dev(np.array(lam0)), NRHS, b)
    try:
        x2, i2 = P.solve_batched(ms, ns, col, row, lam0, NRHS, b)
        pb.run()
        torch.cuda.synchronize()
        assert (i2.cpu().numpy() == 0).all() and (pb.info.cpu().numpy() == 0).all()
        assert relerr(pb.x.cpu().numpy(), x2.cpu().numpy()) <= TOL
    finally:
        pb.free()


def _check_backward(batch, g_lam, g_b, x, lams):
    """Gradients of L = 0.5 ||x - x_true||^2 per solve against the oracle's adjoint."""
    g_lam = g_lam.cpu().numpy()
    g_b = g_b.cpu().numpy()
    x = x.cpu().numpy()
    s = xo = bo = 0
    for p, ll in zip(batch, lams.reshape(-1, NLAM)):
        for lam in ll:
            for r in range(NRHS):
                xs = x[xo:xo + p["n"]]
                ref = oracle.gradients(p["col"], p["row"], p["B"][r], float(lam), xs - p["xt"])
                assert abs(g_lam[s] - ref["g_lam"]) <= 1e-9 * max(1.0, abs(ref["g_lam"])), (p["n"], lam, r)
                assert relerr(g_b[bo:bo + p["m"]], ref["g_b"].real) <= 1e-9
                s += 1
                xo += p["n"]
                bo += p["m"]


def test_prepared_graph_capture(P, batch):
    """Forward, the upstream gradient (torch ops) and backward captured into one graph
    and replayed with three lambda sets, with eager work and synchronizations between the
    replays: every replay matches an eager run of the same handles and the oracle."""
    ms, ns, col, row, b = _args(batch)
    lam0 = np.array([l for p in batch for l in p["lams"]])
    lam = dev(lam0)
    xt = dev(np.concatenate([np.tile(p["xt"], NLAM * NRHS) for p in batch]))
    fwd = P.prepare_batched(ms, ns, col, row, lam, NRHS, b)
    gx = torch.empty_like(fwd.x)
    torch.sub(fwd.x, xt, out=gx)
    bwd = P.prepare_backward_batched(ms, ns, col, row, lam, NRHS, b, fwd.x, gx)
    try:
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            fwd.run(); torch.sub(fwd.x, xt, out=gx); bwd.run()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph):
            fwd.run()
            torch.sub(fwd.x, xt, out=gx)
            bwd.run()
        torch.cuda.synchronize()
        for k, scale in enumerate((1.0, 1.15, 0.8)):
            lam.copy_(dev(lam0 * scale))
            graph.replay()
            torch.cuda.synchronize()
            xg, glg, gbg = fwd.x.clone(), bwd.g_lam.clone(), bwd.g_b.clone()
            assert (fwd.info.cpu().numpy() == 0).all() and (bwd.info.cpu().numpy() == 0).all()
            # eager runs of the same handles
            fwd.run(); torch.sub(fwd.x, xt, out=gx); bwd.run()
            torch.cuda.synchronize()
            assert relerr(xg.cpu().numpy(), fwd.x.cpu().numpy()) <= 1e-12
            assert relerr(glg.cpu().numpy(), bwd.g_lam.cpu().numpy()) <= 1e-12
            assert relerr(gbg.cpu().numpy(), bwd.g_b.cpu().numpy()) <= 1e-12
            if k != 1:
                _check_forward(batch, xg, lam0 * scale)
                _check_backward(batch, glg, gbg, xg, lam0 * scale)
    finally:
        bwd.free()
        fwd.free()


def test_prepared_info_bits(P, batch):
    """Recorded lengths too short for the degrees (a testing option records half of them)
    give info bit 32; a lambda that is not positive is replaced by 1 and gives bit 64 for
    its solves only."""
    ms, ns, col, row, b = _args(batch)
    lam0 = np.array([l for p in batch for l in p["lams"]])
    lam = dev(lam0)
    P.set_options(record_short=1)
    try:
        pb = P.prepare_batched(ms, ns, col, row, lam, NRHS, b)
    finally:
        P.set_options(record_short=0)
    try:
        pb.run()
        torch.cuda.synchronize()
        assert ((pb.info.cpu().numpy() & 32) != 0).any()
    finally:
        pb.free()
    pb = P.prepare_batched(ms, ns, col, row, lam, NRHS, b)
    try:
        bad = lam0.copy()
        bad[1] = -1.0                    # problem 0, second lambda
        lam.copy_(dev(bad))
        pb.run()
        torch.cuda.synchronize()
        info = pb.info.cpu().numpy()
        assert (info[NRHS:2 * NRHS] & 64 != 0).all()
        assert (info[:NRHS] & 64 == 0).all() and (info[2 * NRHS:] == 0).all()
        # the other lambda of that problem is solved as before
        x = pb.x.cpu().numpy()
        p = batch[0]
        for r in range(NRHS):
            ref = oracle.solve(p["col"], p["row"], p["B"][r], float(lam0[0]))
            assert relerr(x[r * p["n"]:(r + 1) * p["n"]], ref) <= TOL
    finally:
        pb.free()


def test_prepared_invalid_arguments(P, batch):
    ms, ns, col, row, b = _args(batch)
    lam = dev(np.array([l for p in batch for l in p["lams"]]))
    with pytest.raises(P.TikhError):
        P.prepare_batched(ms, ns, col, row, dev(-lam.cpu().numpy()), NRHS, b)
    P.set_options(defer_tol=1e-3)
    try:
        with pytest.raises(P.TikhError):
            P.prepare_batched(ms, ns, col, row, lam, NRHS, b)
    finally:
        P.set_options(defer_tol=0.0)
    pb = P.prepare_batched(ms, ns, col, row, lam, NRHS, b)
    pb.free()
    with pytest.raises(P.TikhError):
        pb.run()


def test_prepared_complex_forward_and_backward(P):
    """Complex data (complex T, b and x_true): a prepared forward and backward pair, run
    eagerly at two lambda sets and once from a captured graph, against the oracle's
    solutions and gradients (every gradient block: generator column and row, b, lambda)."""
    rng = np.random.default_rng(4471)
    shapes = [(150, 120), (96, 130)]
    nlam, nrhs = 2, 2
    probs = []
    for (m, n) in shapes:
        col, row, _ = W.random_problem(rng, m, n, cplx=True, L=10.0)
        B = [rng.standard_normal(m) + 1j * rng.standard_normal(m) for _ in range(nrhs)]
        xt = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        probs.append(dict(col=col, row=row, B=B, xt=xt, m=m, n=n))
    ms = [p["m"] for p in probs]
    ns = [p["n"] for p in probs]
    col = dev(np.concatenate([p["col"] for p in probs]))
    row = dev(np.concatenate([p["row"] for p in probs]))
    b = dev(np.concatenate([np.concatenate(p["B"]) for p in probs]))
    xt = dev(np.concatenate([np.tile(p["xt"], nlam * nrhs) for p in probs]))
    lam0 = np.array([0.1, 0.6, 0.25, 1.3])
    lam = dev(lam0)
    fwd = P.prepare_batched(ms, ns, col, row, lam, nrhs, b, complex_data=True)
    gx = torch.empty_like(fwd.x)
    torch.sub(fwd.x, xt, out=gx)
    bwd = P.prepare_backward_batched(ms, ns, col, row, lam, nrhs, b, fwd.x, gx, complex_data=True)

    def check(lams):
        assert (fwd.info.cpu().numpy() == 0).all() and (bwd.info.cpu().numpy() == 0).all()
        x = fwd.x.cpu().numpy()
        gc, gr, gb, gl = (t.cpu().numpy() for t in (bwd.g_col, bwd.g_row, bwd.g_b, bwd.g_lam))
        xo = co = k = 0
        for p, ll in zip(probs, lams.reshape(-1, nlam)):
            m, n = p["m"], p["n"]
            for lv in ll:
                for r in range(nrhs):
                    xs = x[xo:xo + n]
                    assert relerr(xs, oracle.solve(p["col"], p["row"], p["B"][r], float(lv))) <= TOL
                    ref = oracle.gradients(p["col"], p["row"], p["B"][r], float(lv), xs - p["xt"])
                    ref_row = ref["g_row"].copy(); ref_row[0] = 0
                    assert relerr(gc[co:co + m], ref["g_col"]) <= TOL, (m, n, lv, r)
                    assert relerr(gr[xo:xo + n], ref_row) <= TOL, (m, n, lv, r)
                    assert relerr(gb[co:co + m], ref["g_b"]) <= TOL, (m, n, lv, r)
                    assert abs(gl[k] - ref["g_lam"]) <= TOL * max(1.0, abs(ref["g_lam"])), (m, n, lv, r)
                    xo += n; co += m; k += 1
        assert xo == len(x)

    try:
        bwd.run()
        torch.cuda.synchronize()
        check(lam0)
        lam.copy_(dev(lam0 * 0.9))
        fwd.run(); torch.sub(fwd.x, xt, out=gx); bwd.run()
        torch.cuda.synchronize()
        check(lam0 * 0.9)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            fwd.run(); torch.sub(fwd.x, xt, out=gx); bwd.run()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            fwd.run()
            torch.sub(fwd.x, xt, out=gx)
            bwd.run()
        torch.cuda.synchronize()
        lam.copy_(dev(lam0 * 1.2))
        graph.replay()
        torch.cuda.synchronize()
        check(lam0 * 1.2)
    finally:
        bwd.free()
        fwd.free()


def test_prepared_single_wave_leaves_padded_groups(P, batch):
    """Options in force at preparation apply to every run: with the one-wavefront-per-group
    leaf steps forced (leaf_wave_groups = 1) and 3 right-hand sides per (problem, lambda)
    (groups of 2, the second padded), eager runs at two lambda sets give the oracle's
    solutions and gradients."""
    nrhs = 3
    rng = np.random.default_rng(977)
    ms = [p["m"] for p in batch]
    ns = [p["n"] for p in batch]
    B = [[rng.standard_normal(p["m"]) for _ in range(nrhs)] for p in batch]
    col = dev(np.concatenate([p["col"] for p in batch]))
    row = dev(np.concatenate([p["row"] for p in batch]))
    b = dev(np.concatenate([np.concatenate(bb) for bb in B]))
    xt = dev(np.concatenate([np.tile(p["xt"], NLAM * nrhs) for p in batch]))
    lam0 = np.array([l for p in batch for l in p["lams"]])
    lam = dev(lam0)
    P.set_options(leaf_wave_groups=1)
    try:
        fwd = P.prepare_batched(ms, ns, col, row, lam, nrhs, b)
        gx = torch.empty_like(fwd.x)
        torch.sub(fwd.x, xt, out=gx)
        bwd = P.prepare_backward_batched(ms, ns, col, row, lam, nrhs, b, fwd.x, gx)
    finally:
        P.set_options(leaf_wave_groups=1536)
    try:
        for scale in (1.0, 1.1):
            lam.copy_(dev(lam0 * scale))
            fwd.run(); torch.sub(fwd.x, xt, out=gx); bwd.run()
            torch.cuda.synchronize()
            assert (fwd.info.cpu().numpy() == 0).all() and (bwd.info.cpu().numpy() == 0).all()
            x = fwd.x.cpu().numpy()
            gb, gl = bwd.g_b.cpu().numpy(), bwd.g_lam.cpu().numpy()
            xo = bo = k = 0
            for p, bb, ll in zip(batch, B, (lam0 * scale).reshape(-1, NLAM)):
                for lv in ll:
                    for r in range(nrhs):
                        xs = x[xo:xo + p["n"]]
                        assert relerr(xs, oracle.solve(p["col"], p["row"], bb[r], float(lv))) <= TOL, (p["n"], lv, r)
                        ref = oracle.gradients(p["col"], p["row"], bb[r], float(lv), xs - p["xt"])
                        assert relerr(gb[bo:bo + p["m"]], ref["g_b"].real) <= TOL, (p["n"], lv, r)
                        assert abs(gl[k] - ref["g_lam"]) <= TOL * max(1.0, abs(ref["g_lam"])), (p["n"], lv, r)
                        xo += p["n"]; bo += p["m"]; k += 1
            assert xo == len(x)
    finally:
        bwd.free()
        fwd.free()
