"""GPU adjoint (backward) through the C ABI, against the CPU oracle's
hand-derived gradients (dense FP64), against central finite differences of the
GPU forward solve, and through torch.autograd."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle
import workloads as W

LEAF_WAVE_GROUPS = int(os.environ.get("TIKH_TEST_LEAF_WAVE_GROUPS", "1536"))


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1302_6945_amd as P
    # the leaf-step variant can be forced for the whole module (1: one wavefront per group)
    P.set_options(n_lim=256, refine=1, leaf_wave_groups=LEAF_WAVE_GROUPS)
    return P


def dev(a):
    return torch.tensor(np.asarray(a), device="cuda:0")


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("m,n,cplx", [(20, 13, False), (13, 20, True), (150, 97, False), (120, 160, True),
                                      (576, 512, True)])
def test_backward_vs_oracle(P, m, n, cplx):
    rng = np.random.default_rng(m * 31 + n + cplx)
    col, row, b = W.random_problem(rng, m, n, cplx=cplx, L=16.0)
    lam = 0.3
    xt = rng.standard_normal(n) + (1j * rng.standard_normal(n) if cplx else 0)
    x = P.solve(dev(col), dev(row), dev(b), lam)
    gx = x - dev(xt)                       # L = 0.5 ||x - x_true||^2
    g_col, g_row, g_b, g_lam = P.backward(dev(col), dev(row), dev(b), lam, x, gx)
    ref = oracle.gradients(col, row, b, lam, x.cpu().numpy() - xt)
    ref_row = ref["g_row"].copy(); ref_row[0] = 0
    for got, want in ((g_col, ref["g_col"]), (g_row, ref_row), (g_b, ref["g_b"])):
        got = got.cpu().numpy()
        want = want if cplx else want.real
        assert rel(got, want) <= 1e-9
    assert abs(float(g_lam) - ref["g_lam"]) <= 1e-9 * max(1.0, abs(ref["g_lam"]))


@pytest.mark.parametrize("cplx", [False, True])
def test_backward_central_differences(P, cplx):
    """Central differences of the GPU forward solve, h = 1e-6, 16 random unit directions."""
    rng = np.random.default_rng(77 + cplx)
    m, n = 90, 64
    col, row, b = W.random_problem(rng, m, n, cplx=cplx, L=12.0)
    lam = 0.4
    xt = rng.standard_normal(n) + (1j * rng.standard_normal(n) if cplx else 0)

    def loss(c, r, bb, l):
        x = P.solve(dev(c), dev(r), dev(bb), l).cpu().numpy()
        return 0.5 * np.sum(np.abs(x - xt) ** 2)

    x = P.solve(dev(col), dev(row), dev(b), lam)
    g_col, g_row, g_b, g_lam = [t.cpu().numpy() if hasattr(t, "cpu") else t
                                for t in P.backward(dev(col), dev(row), dev(b), lam, x, x - dev(xt))]
    g_lam = float(g_lam)
    h = 1e-6
    for _ in range(16):
        dc = rng.standard_normal(m) + (1j * rng.standard_normal(m) if cplx else 0)
        dr = rng.standard_normal(n) + (1j * rng.standard_normal(n) if cplx else 0); dr[0] = 0
        db = rng.standard_normal(m) + (1j * rng.standard_normal(m) if cplx else 0)
        dl = rng.standard_normal()
        nrm = np.sqrt(np.sum(np.abs(dc) ** 2) + np.sum(np.abs(dr) ** 2) + np.sum(np.abs(db) ** 2) + dl ** 2)
        dc, dr, db, dl = dc / nrm, dr / nrm, db / nrm, dl / nrm
        fd = (loss(col + h * dc, row + h * dr, b + h * db, lam + h * dl)
              - loss(col - h * dc, row - h * dr, b - h * db, lam - h * dl)) / (2 * h)
        an = (np.sum((np.conj(g_col) * dc).real) + np.sum((np.conj(g_row) * dr).real)
              + np.sum((np.conj(g_b) * db).real) + g_lam * dl)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


def test_autograd_function(P):
    rng = np.random.default_rng(9)
    col, row, b = W.random_problem(rng, 70, 50, L=10.0)
    xt = dev(rng.standard_normal(50))
    c, r, bb = dev(col).requires_grad_(), dev(row).requires_grad_(), dev(b).requires_grad_()
    lam = torch.tensor(0.25, dtype=torch.float64, device="cuda:0", requires_grad=True)
    x = P.tikhonov_solve(c, r, bb, lam)
    L = 0.5 * ((x - xt) ** 2).sum()
    L.backward()
    ref = oracle.gradients(col, row, b, 0.25, x.detach().cpu().numpy() - xt.cpu().numpy())
    assert rel(c.grad.cpu().numpy(), ref["g_col"].real) <= 1e-9
    assert rel(bb.grad.cpu().numpy(), ref["g_b"].real) <= 1e-9
    assert abs(float(lam.grad) - ref["g_lam"]) <= 1e-9 * max(1, abs(ref["g_lam"]))


@pytest.mark.parametrize("cplx", [False, True])
def test_autograd_function_all_blocks(P, cplx):
    """torch.autograd through tikhonov_solve, real and complex data: every gradient block
    (generator column, generator row with its entry 0 folded into the column, b, lambda)
    against the oracle's adjoint, in torch's complex convention dL/dRe + i dL/dIm."""
    rng = np.random.default_rng(31 + cplx)
    m, n = 84, 61
    col, row, b = W.random_problem(rng, m, n, cplx=cplx, L=10.0)
    xt_np = rng.standard_normal(n) + (1j * rng.standard_normal(n) if cplx else 0)
    c, r, bb = dev(col).requires_grad_(), dev(row).requires_grad_(), dev(b).requires_grad_()
    lam = torch.tensor(0.35, dtype=torch.float64, device="cuda:0", requires_grad=True)
    x = P.tikhonov_solve(c, r, bb, lam)
    loss = 0.5 * ((x - dev(xt_np)).abs() ** 2).sum()
    loss.backward()
    ref = oracle.gradients(col, row, b, 0.35, x.detach().cpu().numpy() - xt_np)
    ref_row = ref["g_row"].copy(); ref_row[0] = 0
    for got, want in ((c.grad, ref["g_col"]), (r.grad, ref_row), (bb.grad, ref["g_b"])):
        assert got.dtype == (torch.complex128 if cplx else torch.float64)
        assert rel(got.cpu().numpy(), want if cplx else want.real) <= 1e-9
    assert abs(float(lam.grad) - ref["g_lam"]) <= 1e-9 * max(1, abs(ref["g_lam"]))


def test_backward_batched_matches_single(P):
    rng = np.random.default_rng(123)
    shapes = [(60, 40), (35, 70)]
    nlam, nrhs = 2, 2
    cols, rows, bs, lams, xs, gxs = [], [], [], [], [], []
    for (m, n) in shapes:
        col, row, _ = W.random_problem(rng, m, n, L=9.0)
        cols.append(col); rows.append(row)
        B = [rng.standard_normal(m) for _ in range(nrhs)]
        bs.extend(B)
        L = [0.2, 0.7]
        lams.extend(L)
    ms = [s[0] for s in shapes]; ns = [s[1] for s in shapes]
    x, info = P.solve_batched(ms, ns, dev(np.concatenate(cols)), dev(np.concatenate(rows)), lams, nrhs,
                              dev(np.concatenate(bs)))
    gx = dev(rng.standard_normal(x.numel()))
    g_col, g_row, g_b, g_lam, info = P.backward_batched(ms, ns, dev(np.concatenate(cols)), dev(np.concatenate(rows)),
                                                        lams, nrhs, dev(np.concatenate(bs)), x, gx)
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all()
    xo = co = ro = 0; k = 0
    for pi, (m, n) in enumerate(shapes):
        for li in range(nlam):
            for ri in range(nrhs):
                xs_ = x[xo:xo + n]; gx_ = gx[xo:xo + n]
                gc, gr, gb, gl = P.backward(dev(cols[pi]), dev(rows[pi]), dev(bs[pi * nrhs + ri]), lams[pi * nlam + li],
                                            xs_, gx_)
                assert rel(g_col[co:co + m].cpu().numpy(), gc.cpu().numpy()) <= 1e-12
                assert rel(g_row[ro:ro + n].cpu().numpy(), gr.cpu().numpy()) <= 1e-12
                assert rel(g_b[co:co + m].cpu().numpy(), gb.cpu().numpy()) <= 1e-12
                assert abs(float(g_lam[k]) - float(gl)) <= 1e-12 * max(1, abs(float(gl)))
                xo += n; co += m; ro += n; k += 1


def test_complex_full_size_gradient_central_differences(P):
    """Differentiation workload at full size (complex T, n = 2^15, m = n + n/8,
    lambda = 0.02, loss 0.5 ||x - x_true||^2): central differences of the GPU forward
    solve along each gradient block's own direction (generator column, generator
    row, b, lambda) and 16 random unit directions over all of them.
    - The plain central difference D(h) at h = 1e-6 is held to 1e-5: along the generator
      its O(h^2) truncation is 1e-6 relative (measured 1e-4 at h = 1e-5).
    - The Richardson combination R = (4 D(h/2) - D(h)) / 3 at h = 1e-5 removes the h^2
      term (remainder about 1e-7) and is held to 1e-6: relative to the directional
      derivative along the four block directions, and relative to the gradient's norm
      along the random directions, whose directional derivatives (about ||g|| / 400
      here) are otherwise dominated by the loss's rounding: the solves are accurate to
      about 1e-13, i.e. 1e-11 in the loss, or 1e-6 after division by h."""
    pr = W.config3()
    col, row, b, lam, xt = pr.col, pr.row, pr.b[0], pr.lams[0], pr.x_true
    m, n = len(col), len(row)

    def xs(c, r, bb, l):
        return P.solve(dev(c), dev(r), dev(bb), l).cpu().numpy()

    x = P.solve(dev(col), dev(row), dev(b), lam)
    g_col, g_row, g_b, g_lam = P.backward(dev(col), dev(row), dev(b), lam, x, x - dev(xt))
    g_col, g_row, g_b, g_lam = g_col.cpu().numpy(), g_row.cpu().numpy(), g_b.cpu().numpy(), float(g_lam)
    gnorm = np.sqrt(np.sum(np.abs(g_col) ** 2) + np.sum(np.abs(g_row[1:]) ** 2) + np.sum(np.abs(g_b) ** 2) + g_lam ** 2)
    zc, zr, zb = np.zeros_like(col), np.zeros_like(row), np.zeros_like(b)
    dirs = [(g_col / np.linalg.norm(g_col), zr, zb, 0.0), (zc, g_row / np.linalg.norm(g_row), zb, 0.0),
            (zc, zr, g_b / np.linalg.norm(g_b), 0.0), (zc, zr, zb, 1.0)]
    rng = np.random.default_rng(2024)
    cn = lambda k: rng.standard_normal(k) + 1j * rng.standard_normal(k)
    for _ in range(16):
        dc, dr, db, dl = cn(m), cn(n), cn(m), rng.standard_normal()
        dr[0] = 0
        nrm = np.sqrt(np.sum(np.abs(dc) ** 2) + np.sum(np.abs(dr) ** 2) + np.sum(np.abs(db) ** 2) + dl ** 2)
        dirs.append((dc / nrm, dr / nrm, db / nrm, dl / nrm))

    def central(h, dc, dr, db, dl):
        # 0.5 ||xp - xt||^2 - 0.5 ||xm - xt||^2 = 0.5 Re <xp + xm - 2 xt, xp - xm>, without cancellation
        xp = xs(col + h * dc, row + h * dr, b + h * db, lam + h * dl)
        xm = xs(col - h * dc, row - h * dr, b - h * db, lam - h * dl)
        return 0.5 * np.sum((np.conj(xp + xm - 2 * xt) * (xp - xm)).real) / (2 * h)

    for i, (dc, dr, db, dl) in enumerate(dirs):
        an = (np.sum((np.conj(g_col) * dc).real) + np.sum((np.conj(g_row) * dr).real)
              + np.sum((np.conj(g_b) * db).real) + g_lam * dl)
        fd = central(1e-6, dc, dr, db, dl)
        assert abs(fd - an) <= 1e-5 * max(abs(an), 1.0), (i, fd, an)
        rich = (4.0 * central(5e-6, dc, dr, db, dl) - central(1e-5, dc, dr, db, dl)) / 3.0
        scale = abs(an) if i < 4 else gnorm
        assert abs(rich - an) <= 1e-6 * scale, (i, rich, an, scale)


def test_backward_batch_full_config_sampled(P):
    """The benchmark's launch configuration for the adjoint: 256 headline-shaped
    problems (n = 2^14) x 8 lambdas x 4 right-hand sides, forward and backward
    in one batched call each (2048 groups in one chunk).  32 generated problems
    are used 8 times, each copy with its own scaled lambda path.  For sampled
    solves every gradient block (generator column and row, b, lambda) must
    agree with the single-problem backward fed the same x and upstream gradient,
    whose accuracy is pinned against the oracle and central differences above."""
    base = [W.headline(i, n=2 ** 14, nrhs=4, nlam=8) for i in range(32)]
    probs = []
    for c in range(8):
        for p in base:
            probs.append((p, [lam * (1.0 + 0.01 * c) for lam in p.lams]))
    n = 2 ** 14
    ms = [p.m for p, _ in probs]
    ns = [n] * len(probs)
    lams = [l for _, ls in probs for l in ls]
    col = dev(np.concatenate([p.col for p, _ in probs]))
    row = dev(np.concatenate([p.row for p, _ in probs]))
    bb = dev(np.concatenate([np.concatenate(p.b) for p, _ in probs]))
    xt = dev(np.concatenate([np.tile(p.x_true, 32) for p, _ in probs]))
    P.set_options(n_lim=256, refine=1, leaf_wave_groups=1536)
    try:
        x, info = P.solve_batched(ms, ns, col, row, lams, 4, bb)
        gx = x - xt
        g_col, g_row, g_b, g_lam, binfo = P.backward_batched(ms, ns, col, row, lams, 4, bb, x, gx)
        torch.cuda.synchronize()
    finally:
        P.set_options(leaf_wave_groups=LEAF_WAVE_GROUPS)
    assert (info.cpu().numpy() == 0).all() and (binfo.cpu().numpy() == 0).all()
    x, gx = x.cpu().numpy(), gx.cpu().numpy()
    g_col, g_row, g_b, g_lam = g_col.cpu().numpy(), g_row.cpu().numpy(), g_b.cpu().numpy(), g_lam.cpu().numpy()
    tol = 1e-9
    colsum = np.concatenate([[0], np.cumsum(ms)])
    for (ip, j, r) in [(0, 0, 0), (77, 7, 3), (150, 3, 1), (255, 5, 2)]:
        p, ls = probs[ip]
        m = p.m
        k = (ip * 8 + j) * 4 + r
        xs = x[k * n:(k + 1) * n]
        gs = gx[k * n:(k + 1) * n]
        oc = colsum[ip] * 32 + (j * 4 + r) * m
        sc, sr, sb, sl = P.backward(dev(p.col), dev(p.row), dev(p.b[r]), ls[j], dev(xs), dev(gs))
        sc, sr, sb = sc.cpu().numpy(), sr.cpu().numpy(), sb.cpu().numpy()
        assert np.linalg.norm(g_col[oc:oc + m] - sc) <= tol * np.linalg.norm(sc), (ip, j, r, "col")
        assert np.linalg.norm(g_row[k * n:(k + 1) * n] - sr) <= tol * np.linalg.norm(sr), (ip, j, r, "row")
        assert np.linalg.norm(g_b[oc:oc + m] - sb) <= tol * np.linalg.norm(sb), (ip, j, r, "b")
        assert abs(g_lam[k] - float(sl)) <= tol * max(1.0, abs(float(sl))), (ip, j, r, "lambda")
