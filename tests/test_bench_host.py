"""Host-side logic of bench.py (no GPU): the leaf-cutoff choice from autotuner timings."""
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
