"""Host-side logic of bench.py (no GPU): the leaf-cutoff choice from autotuner timings, the
method's algorithmic work, the oracle leg's parity gate, when committed counter traffic applies and
the refusal of more than one GPU."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_pick_nlim_prefers_larger_cutoff_on_near_ties():
    b = _bench()
    # the measured headline timings: 192 and 256 within 0.1%
    assert b.pick_nlim({64: 711.1, 128: 1259.9, 192: 590.7, 256: 590.3}) == 256
    assert b.pick_nlim({64: 711.1, 128: 1259.9, 192: 590.3, 256: 600.0}) == 256
    assert b.pick_nlim({64: 500.0, 128: 700.0, 192: 590.3, 256: 620.0}) == 64
    assert b.pick_nlim({128: 100.0}) == 128


def test_method_work_headline_plan():
    """Algorithmic bytes of one forward solve at the headline plan (N = 36864, 2^9 leaves of
    144 conditions): 9 merge levels of 280 x 2N bytes, 512 leaves of 180 x 144 bytes and the
    setup's 16 (m + n) + 160 N bytes."""
    b = _bench()
    m, n = 18432, 16384
    flops, nbytes = b.method_work(m, n, 36864, 9, 72)
    expect = 9 * 280 * 73728 + 512 * 180 * 144 + 16 * (m + n) + 160 * 36864
    assert abs(nbytes - expect) < 1.0
    assert 1.2e9 < flops < 1.8e9


def _layout(probs, nlam, nrhs, per_solve, key):
    import numpy as np
    out = []
    for p in probs:
        for j in range(nlam):
            for r in range(nrhs):
                out.append(np.asarray(per_solve[(id(p), j, r)][key]).real)
    return np.concatenate(out)


def test_oracle_leg_indexing_and_gate():
    """The bench's oracle leg on a small batch whose 'timed' outputs come from the oracle
    itself: the parity gate passes at rounding level; a wrong entry in the checked problem's
    solutions fails it."""
    import numpy as np
    import oracle
    import workloads as W
    b = _bench()
    nlam, nrhs = 2, 2
    probs = [W.headline(i, n=48, nrhs=nrhs, nlam=nlam) for i in range(3)]
    ref = {}
    for p in probs:
        for j in range(nlam):
            xs = oracle.band_solve(p.col, p.row, p.b, p.lams[j])
            for r in range(nrhs):
                ref[(id(p), j, r)] = {"x": xs[r]}
    x_gpu = _layout(probs, nlam, nrhs, ref, "x")

    def run_backward(x_in):
        xo = 0
        gc, gr, gb, gl = [], [], [], []
        for p in probs:
            for j in range(nlam):
                for r in range(nrhs):
                    xi = x_in[xo:xo + p.n]
                    g = oracle.band_gradients(p.col, p.row, p.b[r], p.lams[j], xi, xi - p.x_true)
                    gc.append(g["g_col"].real); gr.append(g["g_row"].real); gb.append(g["g_b"].real)
                    gl.append(g["g_lam"])
                    xo += p.n
        return np.concatenate(gc), np.concatenate(gr), np.concatenate(gb), np.array(gl)

    ip = min(range(3), key=lambda i: probs[i].meta["L"])
    cpu, parity = b.oracle_leg(probs, ip, nlam, nrhs, x_gpu, run_backward, cores=2)
    assert parity["ok"] and parity["fwd_max_rel_err"] < 1e-13 and parity["bwd_max_rel_err"] < 1e-12
    assert parity["fwd_solves_checked"] == nlam * nrhs and cpu["value"] > 0
    cnt, worst = b.residual_sample(probs, nlam, nrhs, x_gpu, count=12)
    assert cnt == 12 and worst < 1e-13
    bad = x_gpu.copy()
    off = sum(p.n * nlam * nrhs for p in probs[:ip]) + (1 * nrhs + 1) * probs[ip].n + 5
    bad[off] += 1e-6 * np.abs(x_gpu).max()
    _, parity2 = b.oracle_leg(probs, ip, nlam, nrhs, bad, run_backward, cores=2)
    assert not parity2["ok"]


def test_measured_traffic_applies_only_to_its_sources_and_workload(tmp_path):
    """The bench's `roofline.traffic` comes from a committed counter summary only while the
    kernel and driver sources digest to the summary's value and the workload (problems, n)
    and leaf cutoff are the summary's; otherwise it is null."""
    import json
    import shutil
    from types import SimpleNamespace
    b = _bench()
    csrc = tmp_path / "paper_1302_6945_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in ("tikh_kernels.hip", "tikh_driver.hip", "tikh_internal.h"):
        shutil.copy(os.path.join(ROOT, "paper_1302_6945_amd", "csrc", f), csrc / f)
    (tmp_path / "profiles").mkdir()
    rec = {"source_digest": b.source_digest(str(tmp_path)), "nprob": 256, "n": 16384, "n_lim": 256,
           "bytes_per_launch": 123456789}
    (tmp_path / "profiles" / "k_fft_hbm_traffic_headline_n16384.md").write_text(
        "# summary\n\ntraffic_json: %s\n" % json.dumps(rec))
    args = SimpleNamespace(nprob=256, n=16384)
    assert b.measured_traffic(str(tmp_path), "k_fft", args, 256) == 123456789
    assert b.measured_traffic(str(tmp_path), "k_fft", args, 192) is None
    assert b.measured_traffic(str(tmp_path), "k_fft", SimpleNamespace(nprob=64, n=16384), 256) is None
    assert b.measured_traffic(str(tmp_path), "k_prod_mul", args, 256) is None
    with open(csrc / "tikh_kernels.hip", "a") as fh:
        fh.write("\n// changed\n")
    assert b.measured_traffic(str(tmp_path), "k_fft", args, 256) is None


def test_more_than_one_gpu_is_refused():
    """`bench.py --gpus N` with N > 1 (or under a launcher with WORLD_SIZE > 1) exits with a
    message before touching any device."""
    import subprocess
    import sys
    for argv, env in ((["--gpus", "2"], {}), ([], {"WORLD_SIZE": "4"})):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv, capture_output=True, text=True,
                           timeout=120, env=dict(os.environ, **env))
        assert r.returncode == 2
        assert "one GPU only" in r.stderr and r.stdout == ""
