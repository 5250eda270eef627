#!/usr/bin/env python
"""Benchmark: batched Tikhonov-regularized Toeplitz solves per second, forward
plus backward, at n = 2^14 on one MI355X, against the plain one-problem-per-call
method on the same GPU.

Workload (synthetic, seeded; shaped like the paper's l2 experiments, Sec. 7):
n = 2^14 unknowns, m = n + U{0..n/4} rows, real Toeplitz generator a_s = N(0,1)
exp(-|s|/L) with L ~ U[8,128]; every problem is solved at 8 regularization
parameters lambda_j = s_max 10^(-3+3j/7) (s_max ~ ||T||_2, so the regularized
normal matrix has condition number <= 1 + 1e6) and 4 right-hand sides; loss
L = 0.5 ||x - x_true||^2, whose gradient drives the adjoint.  One step = one
batched forward solve of every (problem, lambda, rhs) triple plus one batched
backward (adjoint solve + gradients w.r.t. generator, b and lambda).

Prints ONE JSON line (rank 0).  `value` is whole-job fwd+bwd solves/s with the
inputs resident in HBM.  `roofline` reports the dominant kernel against its
bound with the method's algorithmic work (a derived count for the recursion of
Alg. 1 on 5 x 5 bases: per merge of K conditions 280 K bytes and
31 K log2(K/8) + 94 K log2(K/4) + 350 K flops, per leaf of K conditions 180 K
bytes and 45 K^2 flops, setup 16 (m+n) + 160 N bytes and 20 N log2 N flops,
times 2.05 for forward plus backward), credited in full to that kernel's
launches, whose average duration is measured live with HIP events on the
library stream; `step_roofline` is the same work over the whole step.
`cpu_baseline` times the CPU oracle (banded QR of [T; lambda I], exact for the
generators' finite support) on a bounded sample of the timed workload: every
lambda and right-hand side of the problem with the narrowest generator, forward
and adjoint.  The same oracle results gate the run (`parity`): the timed
forward solves of that problem must match the oracle element by element to
1e-9 (relative 2-norm), the batched backward in the timed launch configuration
fed the oracle's solutions must match the oracle's gradients to 1e-9, and the
optimality residual of eq. (tiksol) is checked on a stratified sample of timed
solves across the batch.  If the gate fails, `value` is null and the exit
status is 1.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


_T_START = time.perf_counter()


def progress(msg):
    """A progress line on stderr (the JSON result is the only line on stdout)."""
    print("bench: %s (%.0f s)" % (msg, time.perf_counter() - _T_START), file=sys.stderr, flush=True)


def source_digest(root):
    """Digest of the kernel and driver sources: HBM counters taken on other sources do not apply."""
    import hashlib
    h = hashlib.sha256()
    for f in ("tikh_kernels.hip", "tikh_driver.hip", "tikh_internal.h"):
        with open(os.path.join(root, "paper_1302_6945_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pick_nlim(tune_ms, tol=0.02):
    """Leaf cutoff from the autotuner's timings: the largest one within `tol` of the fastest
    (the timings of 256 groups carry about 1% noise; a larger cutoff means fewer tree levels)."""
    best = min(tune_ms.values())
    return max(int(k) for k, v in tune_ms.items() if v <= (1.0 + tol) * best)


def method_work(m, n, N, p, M):
    """Algorithmic (flops, HBM bytes) of one forward solve of the recursion on an m x n
    problem with N nodes, 2^p leaves of 2M conditions (derived count, +-30%)."""
    K_leaf = 2 * M
    flops = (1 << p) * 45.0 * K_leaf ** 2 + 20.0 * N * math.log2(N)
    nbytes = (1 << p) * 180.0 * K_leaf + 16.0 * (m + n) + 160.0 * N
    for d in range(p):
        K = (2 * N) >> d
        flops += (1 << d) * (31.0 * K * math.log2(K / 8) + 94.0 * K * math.log2(K / 4) + 350.0 * K)
        nbytes += (1 << d) * 280.0 * K
    return flops, nbytes


FWD_BWD = 2.05   # forward plus backward: one more solve and about 10 transforms of length ~2N


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_leg(probs, ip, nlam, nrhs, x_gpu, run_backward, cores):
    """CPU oracle on the problem `ip` of the timed batch (all lambdas and right-hand sides):
    banded QR forward solves and adjoint solves (upstream gradient x - x_true), one thread per
    lambda; returns (cpu_baseline, parity).  x_gpu: the timed forward solutions (numpy).
    run_backward(x_in) runs the batched backward in the timed launch configuration with forward
    solutions x_in and upstream gradient x_in - x_true, and returns numpy (g_col, g_row, g_b, g_lam)."""
    import numpy as np
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    pr = probs[ip]
    m, n = pr.m, pr.n

    def fwd_bwd(j):
        t0 = time.perf_counter()
        xs = oracle.band_solve(pr.col, pr.row, pr.b, pr.lams[j])
        ws = oracle.band_solve(pr.col, pr.row, [xs[r] - pr.x_true for r in range(nrhs)], pr.lams[j], normal=True)
        return xs, ws, time.perf_counter() - t0

    threads = max(1, min(cores, nlam))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        res = list(ex.map(fwd_bwd, range(nlam)))
    wall = time.perf_counter() - t0
    xref = [r[0] for r in res]
    wref = [r[1] for r in res]
    per_thread = [r[2] for r in res]

    # cost model of the banded QR: (m + n) (bandwidth + 1)^2 per factorization
    def band_cost(p_):
        wl = int(np.max(np.nonzero(p_.col)[0])) if np.any(p_.col) else 0
        wu = int(np.max(np.nonzero(p_.row[1:])[0]) + 1) if np.any(p_.row[1:]) else 0
        return (p_.m + p_.n) * float(wl + wu + 1) ** 2
    c_sample = band_cost(pr)
    c_mean = float(np.mean([band_cost(q) for q in probs]))
    nsol = nlam * nrhs
    rate_sample = nsol / wall
    cpu = {"value": rate_sample * c_sample / c_mean, "unit": "solves/s (fwd+bwd)", "cores": threads,
           "kind": "oracle", "cpu_model": cpu_model(),
           "sample": "banded QR of [T; lambda I] (Givens rows, exact for the generator's support) for the "
                     "%d forward and %d adjoint solves of problem %d (m=%d, n=%d, envelope L=%.2f) of the timed "
                     "batch, one thread per lambda: %.1f s wall on %d threads (%.1f s per lambda single-threaded, "
                     "4 right-hand sides per factorization); value scaled to the batch's average problem by the "
                     "banded-QR cost (m+n)(bandwidth+1)^2 (x%.1f)" % (nsol, nsol, ip, m, n, pr.meta["L"], wall,
                                                                       threads, float(np.median(per_thread)),
                                                                       c_mean / c_sample),
           "sample_rate": round(rate_sample, 4), "single_thread_s_per_lambda": round(float(np.median(per_thread)), 2)}

    # forward parity: timed solves of problem ip against the oracle, element by element
    def rel(a, b):
        return float(np.linalg.norm(np.asarray(a) - b) / max(np.linalg.norm(b), 1e-300))
    base = sum(q.n * nlam * nrhs for q in probs[:ip])
    fwd_err = []
    for j in range(nlam):
        for r in range(nrhs):
            o = base + (j * nrhs + r) * n
            fwd_err.append(rel(x_gpu[o:o + n], xref[j][r].real))

    # backward parity: the batched backward (timed launch configuration) fed the oracle's
    # solutions for problem ip, against the oracle's adjoint
    x_in = x_gpu.copy()
    for j in range(nlam):
        for r in range(nrhs):
            o = base + (j * nrhs + r) * n
            x_in[o:o + n] = xref[j][r].real
    g_col, g_row, g_b, g_lam = run_backward(x_in)
    mbase = sum(q.m * nlam * nrhs for q in probs[:ip])
    bwd_err = []
    lag_checked = []
    for j in range(nlam):
        for r in range(nrhs):
            k = ip * nlam * nrhs + j * nrhs + r
            w = wref[j][r]
            gb_ref = oracle.T_apply(pr.col, pr.row, w)
            gl_ref = float(-2.0 * pr.lams[j] * np.vdot(w, xref[j][r]).real)
            o = mbase + (j * nrhs + r) * m
            bwd_err.append(rel(g_b[o:o + m], gb_ref.real))
            bwd_err.append(abs(float(g_lam[k]) - gl_ref) / max(1.0, abs(gl_ref)))
            if r == j % nrhs and j % 2 == 0:       # generator gradient for 4 of the solves (O(mn) each)
                gc_ref, gr_ref = oracle.lag_sums(pr.col, pr.row, pr.b[r], xref[j][r], w)
                ro = base + (j * nrhs + r) * n
                bwd_err.append(rel(g_col[o:o + m], gc_ref.real))
                bwd_err.append(rel(g_row[ro + 1:ro + n], gr_ref.real[1:]))
                lag_checked.append([j, r])
    parity = {"oracle": "banded QR", "problem": ip, "tol": 1e-9,
              "fwd_solves_checked": len(fwd_err), "fwd_max_rel_err": max(fwd_err),
              "bwd_checked": "g_b and g_lambda of all %d solves, generator gradient of (lambda, rhs) %s" %
                             (nsol, lag_checked),
              "bwd_max_rel_err": max(bwd_err)}
    parity["ok"] = parity["fwd_max_rel_err"] <= 1e-9 and parity["bwd_max_rel_err"] <= 1e-9
    return cpu, parity


def residual_sample(probs, nlam, nrhs, x_gpu, count=64):
    """Optimality residual ||T^H (b - T x) - lambda^2 x|| / (||T^H b|| + lambda^2 ||x||) of eq. (tiksol)
    for a stratified sample of timed solves (every lambda, every right-hand side, problems spread
    over the batch), with FFT products on the CPU."""
    import numpy as np
    import oracle
    offs = np.concatenate([[0], np.cumsum([q.n * nlam * nrhs for q in probs])])
    worst = 0.0
    for i in range(count):
        ip = (i * 37) % len(probs)
        j, r = i % nlam, (i // nlam) % nrhs
        pr = probs[ip]
        o = offs[ip] + (j * nrhs + r) * pr.n
        worst = max(worst, oracle.normal_residual_fft(pr.col, pr.row, pr.b[r], pr.lams[j], x_gpu[o:o + pr.n]))
    return count, worst


def config2_leg(P, torch, W, steps, with_oracle):
    """The batching workload at full size: 1024 problems with n log-uniform in [2^9, 2^14],
    m = n + U{0..n/4}, 8 absolute lambdas 1e-4..1, 4 right-hand sides (32768 solves), forward and
    backward batched (ragged: chunks of different extended sizes side by side on several streams),
    against the plain one-problem-per-call method measured on one problem per octave of n and
    scaled by the octave counts.  With the oracle: sampled solves of the narrowest-band problem of
    two octaves against the oracle at every lambda with kappa <= 1e6 (1e-9)."""
    import numpy as np
    dev = torch.device("cuda:0")
    probs = [W.config2(i) for i in range(1024)]
    ms = [p.m for p in probs]
    ns = [p.n for p in probs]
    lams = [l for p in probs for l in p.lams]
    col = torch.tensor(np.concatenate([p.col for p in probs]), device=dev)
    row = torch.tensor(np.concatenate([p.row for p in probs]), device=dev)
    bb = torch.tensor(np.concatenate([np.concatenate(p.b) for p in probs]), device=dev)
    xt = torch.tensor(np.concatenate([np.tile(p.x_true, 32) for p in probs]), device=dev)

    def step():
        x, info = P.solve_batched(ms, ns, col, row, lams, 4, bb)
        g = P.backward_batched(ms, ns, col, row, lams, 4, bb, x, x - xt)
        return x, info, g[4]

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        x, info, binfo = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    nsol = 1024 * 8 * 4
    info = info.cpu().numpy()
    binfo = binfo.cpu().numpy()
    # plain method: one problem per octave of n, one fwd+bwd per call, scaled by the octave counts
    octs = [min(13, max(9, int(np.floor(np.log2(n))))) for n in ns]
    plain_s = 0.0
    plain_detail = {}
    for o in range(9, 14):
        idx = [i for i in range(1024) if octs[i] == o]
        if not idx:
            continue
        p0 = probs[idx[0]]
        c0, r0, b0 = (torch.tensor(a, device=dev) for a in (p0.col, p0.row, p0.b[0]))
        x0t = torch.tensor(p0.x_true, device=dev)
        x0 = P.solve(c0, r0, b0, p0.lams[4])
        P.backward(c0, r0, b0, p0.lams[4], x0, x0 - x0t)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x0 = P.solve(c0, r0, b0, p0.lams[4])
        P.backward(c0, r0, b0, p0.lams[4], x0, x0 - x0t)
        torch.cuda.synchronize()
        per = time.perf_counter() - t1
        plain_detail[str(2 ** o)] = round(per, 4)
        plain_s += per * len(idx) * 32
    out = {"workload": "1024 problems, n log-uniform 2^9..2^14, m = n + U{0..n/4}, 8 lambdas 1e-4..1 x 4 rhs",
           "solves_per_step": nsol, "value": round(nsol / dt, 2), "unit": "solves/s (fwd+bwd)",
           "ms_per_step": round(dt * 1e3, 1), "steps": steps,
           "plain_solves_per_s": round(nsol / plain_s, 4), "batched_over_plain": round(plain_s / dt, 1),
           "plain_s_per_solve_by_octave": plain_detail,
           "flagged_fwd": int(((info & 16) != 0).sum()), "flagged_bwd": int(((binfo & 16) != 0).sum()),
           "other_info": int(((info | binfo) & ~16).max())}
    if with_oracle:
        import oracle
        xh = x.cpu().numpy()
        xoff = np.concatenate([[0], np.cumsum([p.n * 32 for p in probs])])
        worst, checked = 0.0, 0
        for lo in (9, 11):
            cand = [i for i in range(1024) if 2 ** lo <= probs[i].n < 2 ** (lo + 1)]
            ip = min(cand, key=lambda i: probs[i].meta["L"] * (probs[i].m + probs[i].n))
            p = probs[ip]
            smax = W.norm2_estimate(p.col, p.row, iters=60)
            for j, lam in enumerate(p.lams):
                if 1.0 + (smax / lam) ** 2 > 1e6:
                    continue
                xr = (oracle.band_solve(p.col, p.row, p.b, lam) if p.n > 1100 else
                      np.array([oracle.solve(p.col, p.row, b, lam) for b in p.b]))
                for r in range(4):
                    o = xoff[ip] + (j * 4 + r) * p.n
                    e = float(np.linalg.norm(xh[o:o + p.n] - xr[r].real) / np.linalg.norm(xr[r]))
                    worst = max(worst, e)
                    checked += 1
        out["parity"] = {"solves_checked": checked, "max_rel_err": worst, "tol": 1e-9, "ok": worst <= 1e-9}
    return out


def config4_leg(P, torch, W, steps, with_oracle):
    """Bilevel lambda tuning at full size: 256 deblurring problems (Gaussian PSF, sigma in
    [4, 48], n log-uniform in [2^12, 2^16], one right-hand side), each problem's log lambda by
    `steps` Adam steps on a validation loss with an independent noise draw; one step (batched
    forward, upstream gradient, batched backward, Adam update) captured into one graph and
    replayed.  With the oracle: the first step's dL/dlambda of the three smallest problems
    against the banded QR oracle (1e-7)."""
    import numpy as np
    dev = torch.device("cuda:0")
    # the prepared batches hold workspaces of their own: return the library's shared one
    P.set_workspace(None)
    torch.cuda.empty_cache()
    probs = [W.config4(i) for i in range(256)]
    t_setup = time.perf_counter()
    ms = [p.m for p in probs]
    ns = [p.n for p in probs]
    col = torch.tensor(np.concatenate([p.col for p in probs]), device=dev)
    row = torch.tensor(np.concatenate([p.row for p in probs]), device=dev)
    b = torch.tensor(np.concatenate([p.b[0] for p in probs]), device=dev)
    bval = torch.tensor(np.concatenate([p.b[1] for p in probs]), device=dev)
    lam0 = torch.tensor([p.lams[0] for p in probs], dtype=torch.float64, device=dev)
    tuner = P.BilevelTuner(ms, ns, col, row, b, bval, lam0)
    try:
        torch.cuda.synchronize()
        prepare_s = time.perf_counter() - t_setup
        progress("bilevel batches prepared")
        s0 = tuner.state()
        t0 = time.perf_counter()
        tuner.step()                                   # eager (the same launches, not captured)
        torch.cuda.synchronize()
        eager_s = time.perf_counter() - t0
        tuner.set_state(s0)
        t0 = time.perf_counter()
        tuner.capture()
        capture_s = time.perf_counter() - t0
        progress("bilevel step captured")
        loss0 = tuner.validation_loss()
        grads0 = None
        info_max = 0
        t0 = time.perf_counter()
        for k in range(steps):
            tuner.step()
            if k == 0:
                grads0 = tuner.grad.clone()
            if k % 5 == 4:
                torch.cuda.synchronize()
                progress("bilevel step %d" % (k + 1))
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / max(steps, 1)
        fi, bi = tuner.info()
        info_max = max(int(fi.max().item()), int(bi.max().item()))
        tuner.step()                                   # forward solutions at the final lambdas
        torch.cuda.synchronize()
        loss1 = tuner.validation_loss()
        lam = torch.exp(tuner.loglam).cpu().numpy()
        out = {"workload": "256 deblurring problems, sigma U[4,48], n log-uniform 2^12..2^16, 1 rhs; Adam on "
                           "log lambda (lr 0.1) on a validation loss; one captured graph per step",
               "steps": steps, "ms_per_step": round(dt * 1e3, 1), "eager_ms_per_step": round(eager_s * 1e3, 1),
               "solves_per_s": round(256 / dt, 1), "unit": "fwd+bwd solves/s", "prepare_s": round(prepare_s, 1),
               "capture_s": round(capture_s, 1), "info_max": info_max,
               "val_loss_initial": float(loss0.sum().item()), "val_loss_final": float(loss1.sum().item()),
               "improved_frac": float((loss1 < loss0).double().mean().item()),
               "lambda_range": [float(lam.min()), float(lam.max())]}
        if with_oracle and grads0 is not None:
            import oracle
            g = grads0.cpu().numpy()
            worst = 0.0
            for i in sorted(range(256), key=lambda i: probs[i].n)[:3]:
                p = probs[i]
                x = oracle.band_solve(p.col, p.row, [p.b[0]], p.lams[0])[0]
                gx = oracle.TH_apply(p.col, p.row, oracle.T_apply(p.col, p.row, x) - p.b[1]).real
                want = p.lams[0] * oracle.band_gradients(p.col, p.row, p.b[0], p.lams[0], x, gx,
                                                         with_lag_sums=False)["g_lam"]
                worst = max(worst, float(abs(g[i] - want) / max(abs(want), 1e-300)))
            out["parity"] = {"grads_checked": 3, "max_rel_err": worst, "tol": 1e-7, "ok": bool(worst <= 1e-7)}
        return out
    finally:
        tuner.free()


def measured_traffic(root, kernel, args, nlim):
    """HBM bytes per launch of `kernel` from the committed counter summary, when it was taken on
    the current sources, at this workload and leaf cutoff; None otherwise."""
    path = os.path.join(root, "profiles", "%s_hbm_traffic_headline_n16384.md" % kernel)
    if not os.path.exists(path):
        return None
    rec = None
    with open(path) as fh:
        for line in fh:
            if line.startswith("traffic_json:"):
                rec = json.loads(line.split(":", 1)[1])
    if not rec or rec.get("source_digest") != source_digest(root):
        return None
    if rec.get("nprob") != args.nprob or rec.get("n") != args.n or rec.get("n_lim") != nlim:
        return None
    return rec.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nprob", type=int, default=256, help="problems per step (each 8 lambdas x 4 RHS)")
    ap.add_argument("--nlam", type=int, default=8)
    ap.add_argument("--nrhs", type=int, default=4)
    ap.add_argument("--n", type=int, default=2 ** 14)
    ap.add_argument("--nlim", default="auto",
                    help="leaf cutoff N_lim (Alg. 2), or 'auto': picked by the library's autotuner on 256 groups "
                         "of the workload's shape before the timed steps")
    ap.add_argument("--plain-solves", type=int, default=2)
    ap.add_argument("--no-oracle", "--no-cpu-baseline", dest="no_oracle", action="store_true",
                    help="skip the CPU-oracle leg (cpu_baseline and the parity gate)")
    ap.add_argument("--residual-sample", type=int, default=64,
                    help="timed solves whose optimality residual is checked on the CPU")
    ap.add_argument("--kernel", default="auto", help="kernel for the roofline object: fft, leaf_loop or auto "
                                                     "(the one with the larger share of the step)")
    ap.add_argument("--kernel-times", type=int, default=1,
                    help="time the dominant kernels with HIP events over one extra step each (0 = skip, e.g. under "
                         "a profiler)")
    ap.add_argument("--streams", type=int, default=0,
                    help="streams the library runs chunks on side by side (0 = library default; 1 = one stream, "
                         "e.g. for counter collection, which serializes dispatches)")
    ap.add_argument("--chunk-groups", type=int, default=-1,
                    help="most groups per chunk (chunks of one call run side by side on the streams); "
                         "-1 = library default")
    ap.add_argument("--leaf-wave-groups", type=int, default=0,
                    help="groups per chunk from which leaf steps run one wavefront per group (0 = library default)")
    ap.add_argument("--config2-steps", type=int, default=2,
                    help="timed steps of the 1024-problem ragged batching workload reported beside the headline "
                         "(0 = skip)")
    ap.add_argument("--config4-steps", type=int, default=20,
                    help="Adam steps of the 256-problem bilevel lambda tuning workload reported beside the headline "
                         "(one captured graph per step; 0 = skip)")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="after the run, negate a float64 buffer of this many MiB into another three times "
                         "(a plain streaming kernel of known traffic that calibrates the HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: runs on one GPU only; batches shard trivially across GPUs "
              "(independent solves), no multi-GPU path is provided", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as W
    import paper_1302_6945_amd as P

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    probs = [W.headline(i, n=args.n, nrhs=args.nrhs, nlam=args.nlam) for i in range(args.nprob)]
    ms = [p.m for p in probs]
    tune = None
    if args.nlim == "auto":
        P.set_options(refine=1)
        _, tune_ms = P.autotune_nlim(int(round(float(np.mean(ms)))), args.n, groups=256, nrhs=args.nrhs)
        nlim = pick_nlim(tune_ms)
        progress("leaf cutoff autotuned: %d" % nlim)
        tune = {str(k): round(v, 1) for k, v in tune_ms.items()}
    else:
        nlim = int(args.nlim)
    P.set_options(n_lim=nlim, refine=1)
    if args.streams:
        P.set_options(streams=args.streams)
    if args.chunk_groups >= 0:
        P.set_options(chunk_groups=args.chunk_groups)
    if args.leaf_wave_groups > 0:
        P.set_options(leaf_wave_groups=args.leaf_wave_groups)
    ns = [p.n for p in probs]
    lams = [l for p in probs for l in p.lams]
    col = torch.tensor(np.concatenate([p.col for p in probs]), device=dev)
    row = torch.tensor(np.concatenate([p.row for p in probs]), device=dev)
    bb = torch.tensor(np.concatenate([np.concatenate(p.b) for p in probs]), device=dev)
    xt = torch.tensor(np.concatenate([np.tile(p.x_true, args.nlam * args.nrhs) for p in probs]), device=dev)
    nsolve = args.nprob * args.nlam * args.nrhs

    call_stats = {}

    def step():
        x, info = P.solve_batched(ms, ns, col, row, lams, args.nrhs, bb)
        call_stats["fwd"] = P.get_stats()
        gx = x - xt
        g_col, g_row, g_b, g_lam, binfo = P.backward_batched(ms, ns, col, row, lams, args.nrhs, bb, x, gx)
        call_stats["bwd"] = P.get_stats()
        return x, info, binfo

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    progress("warmup done")
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        x, info, binfo = step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    ms_per_step = ms_total / args.steps
    progress("timed steps done: %.0f ms per step" % ms_per_step)
    value = nsolve * args.steps / (ms_total / 1e3)
    info_max = int(max(info.max().item(), binfo.max().item()))
    x_timed = x.cpu().numpy()
    per_call = {k: {f: v[f] for f in ("launches", "host_syncs", "refine_extra", "refine_skipped", "fallback_groups")}
                for k, v in call_stats.items()}

    # dominant kernels: live launch timing over one more step each (HIP events on the library stream)
    st = P.get_stats()
    rl = {}
    for kern in ("fft", "leaf_loop", "leaf_build"):
        if not args.kernel_times:
            rl[kern] = (0.0, 0, 0.0)
            continue
        P.profile_kernel(kern)
        step()
        torch.cuda.synchronize()
        k_ms, k_count, units = P.profile_read()
        rl[kern] = (k_ms, k_count, units)
    P.profile_kernel(None)
    kernel_ms = {k: round(v[0], 1) for k, v in rl.items()}
    progress("kernel timing done")

    # the method's algorithmic work per step, from each problem's plan
    alg_flops = alg_bytes = 0.0
    for p in probs:
        N, M, depth, _ = P.plan_info(p.m, p.n, nlim)
        f, b_ = method_work(p.m, p.n, N, depth, M)
        alg_flops += f * FWD_BWD * args.nlam * args.nrhs
        alg_bytes += b_ * FWD_BWD * args.nlam * args.nrhs
    step_s = ms_per_step / 1e3
    step_roofline = {"alg_bytes_per_step": alg_bytes, "alg_flops_per_step": alg_flops,
                     "hbm_TBps": round(alg_bytes / step_s / 1e12, 3), "hbm_frac": round(alg_bytes / step_s / 8e12, 4),
                     "fp64_TFLOPs": round(alg_flops / step_s / 1e12, 3),
                     "fp64_frac": round(alg_flops / step_s / 78.6e12, 4),
                     "ceiling_solves_per_s": round(nsolve / max(alg_bytes / 8e12, alg_flops / 78.6e12), 1)}

    main_kernel = args.kernel if args.kernel in ("fft", "leaf_loop") else max(("fft", "leaf_loop"),
                                                                                key=lambda k: rl[k][0])
    k_ms, k_count, units = rl[main_kernel]
    avg_ms = k_ms / max(k_count, 1)
    if main_kernel == "fft":
        per_launch = alg_bytes / max(k_count, 1)
        achieved = per_launch / (avg_ms / 1e3) / 1e9 if k_ms > 0 else 0.0
        roofline = {"bound": "hbm", "kernel": "k_fft", "achieved": round(achieved, 1), "peak": 8000.0, "unit": "GB/s",
                    "frac": round(achieved / 8000.0, 4), "traffic": None, "avg_launch_ms": round(avg_ms, 4),
                    "launches_per_step": k_count, "alg_bytes_per_launch": round(per_launch),
                    "alg_bytes_note": "every algorithmic byte of the step credited to k_fft's launches",
                    "pass_bytes_per_launch": round(units / max(k_count, 1)),
                    "pass_bytes_note": "one read and one write of every transformed element per pass"}
    else:
        per_launch = alg_flops / max(k_count, 1)
        achieved = per_launch / (avg_ms / 1e3) / 1e12 if k_ms > 0 else 0.0
        roofline = {"bound": "alu", "kernel": "k_leaf_loop", "achieved": round(achieved, 3), "peak": 78.6,
                    "unit": "TFLOP/s", "frac": round(achieved / 78.6, 5), "traffic": None,
                    "avg_launch_ms": round(avg_ms, 4), "launches_per_step": k_count,
                    "alg_flops_per_launch": round(per_launch), "pass_flops_per_launch": round(units / max(k_count, 1))}

    # plain method: single-problem C-ABI calls, one solve + one backward per call
    plain = None
    if args.plain_solves > 0:
        p0 = probs[0]
        c0 = torch.tensor(p0.col, device=dev)
        r0 = torch.tensor(p0.row, device=dev)
        b0 = torch.tensor(p0.b[0], device=dev)
        xt0 = torch.tensor(p0.x_true, device=dev)
        x0 = P.solve(c0, r0, b0, p0.lams[0])
        P.backward(c0, r0, b0, p0.lams[0], x0, x0 - xt0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.plain_solves):
            lam = p0.lams[i % len(p0.lams)]
            x0 = P.solve(c0, r0, b0, lam)
            P.backward(c0, r0, b0, lam, x0, x0 - xt0)
        torch.cuda.synchronize()
        plain = args.plain_solves / (time.perf_counter() - t0)

    cpu = parity = None
    if not args.no_oracle:
        cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
        cores = max(1, min(cores, 16))
        ip = min(range(args.nprob), key=lambda i: probs[i].meta["L"])

        def run_backward(x_in):
            xi = torch.tensor(x_in, device=dev)
            g_col, g_row, g_b, g_lam, binf = P.backward_batched(ms, ns, col, row, lams, args.nrhs, bb, xi, xi - xt)
            torch.cuda.synchronize()
            bi = binf.cpu().numpy()
            if bi.max() != 0:
                bad = np.nonzero(bi)[0]
                raise RuntimeError("backward fed the oracle's solutions reported info %s at solves %s"
                                   % (np.unique(bi).tolist(), bad[:16].tolist()))
            return g_col.cpu().numpy(), g_row.cpu().numpy(), g_b.cpu().numpy(), g_lam.cpu().numpy()

        cpu, parity = oracle_leg(probs, ip, args.nlam, args.nrhs, x_timed, run_backward, cores)
        progress("oracle leg done")
        if args.residual_sample > 0:
            cnt, worst = residual_sample(probs, args.nlam, args.nrhs, x_timed, args.residual_sample)
            parity["residual_solves_checked"] = cnt
            parity["residual_max"] = worst
            parity["residual_tol"] = 1e-11
            parity["ok"] = parity["ok"] and worst <= 1e-11
        parity["info_max"] = info_max
        parity["ok"] = parity["ok"] and info_max == 0

    cfg2 = None
    if args.config2_steps > 0:
        cfg2 = config2_leg(P, torch, W, args.config2_steps, not args.no_oracle)
        progress("ragged batching workload done")
        P.set_options(n_lim=nlim, refine=1)
    cfg4 = None
    if args.config4_steps > 0:
        P.set_options(n_lim=256, refine=1)
        cfg4 = config4_leg(P, torch, W, args.config4_steps, not args.no_oracle)
        progress("bilevel workload done")
        P.set_options(n_lim=nlim, refine=1)

    if args.copy_calib_mib > 0:
        src = torch.ones(args.copy_calib_mib * 2 ** 20 // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    traffic = measured_traffic(ROOT, roofline["kernel"], args, nlim)
    if traffic is not None:
        roofline["traffic"] = traffic
        if main_kernel == "fft":
            roofline["traffic_over_alg"] = round(traffic / roofline["alg_bytes_per_launch"], 3)
            roofline["traffic_over_pass"] = round(traffic / max(roofline["pass_bytes_per_launch"], 1), 3)

    if parity is not None and cfg2 is not None and "parity" in cfg2:
        parity["config2_ok"] = cfg2["parity"]["ok"] and cfg2["other_info"] == 0
        parity["ok"] = parity["ok"] and parity["config2_ok"]
    if parity is not None and cfg4 is not None and "parity" in cfg4:
        parity["config4_ok"] = cfg4["parity"]["ok"] and cfg4["info_max"] == 0
        parity["ok"] = parity["ok"] and parity["config4_ok"]
    ok = parity is None or parity["ok"]
    out = {
        "metric": "batched regularized solves/s (fwd+bwd) at n=2^14 vs plain, rel err <= 1e-9",
        "value": round(value, 3) if ok else None,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": "headline n=2^14, m=n+U{0..n/4}, envelope generators, 8 lambdas x 4 rhs",
                   "problems": args.nprob, "solves_per_step": nsolve, "n": args.n, "m_range": [min(ms), max(ms)],
                   "N": st["N"], "depth": st["depth"], "leaf_nodes": st["leaf_nodes"], "n_lim": nlim,
                   "n_lim_autotune_ms": tune, "refine": 1},
        "n_log2n_sq_rate": round(value * args.n * math.log2(args.n) ** 2, 1),
        "plain_solves_per_s": round(plain, 4) if plain else None,
        "batched_over_plain": round(value / plain, 2) if plain else None,
        "info_max": info_max,
        "calls": per_call,
        "parity": parity,
        "roofline": roofline,
        "step_roofline": step_roofline,
        "kernel_ms_per_step": kernel_ms,
        "cpu_baseline": cpu,
        "config2": cfg2,
        "config4": cfg4,
    }
    if not ok:
        out["unmeasured_reason"] = "parity gate failed: no value is reported"
    print(json.dumps(out), flush=True)
    if not ok:
        sys.exit(1)


if __name__ == "__main__":
    main()
