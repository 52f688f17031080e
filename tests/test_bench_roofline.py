"""Host-side checks of the benchmark's roofline arithmetic (no GPU): a stage table whose
measured times equal the stage bounds must report a fraction of one, and the differentiation
workload, which runs every stage twice per image (forward and backward), must not be charged
twice for the same work."""
import importlib.util
import os
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _plan():
    # the L = 128, R = 64, c = 1/2 shape in round figures; only the fields the arithmetic reads
    return types.SimpleNamespace(L=128, grid_n=256, kernel_w=7, n_theta=512, n_xi=128, k_max=100,
                                 p_half=5000, p=[60] + [50] * 100)


def _stages_at_bound(bench, plan, names, images, launches, precision, passes=1):
    """Stage totals whose per-image time is exactly each stage's bound."""
    bpi = bench.algorithmic_bytes_per_image(plan)
    fpi = bench.algorithmic_flops_per_image(plan)
    out, per_image = {}, 0.0
    for st in names:
        t = max(bpi[st] / (bench.HBM_PEAK_GBS * 1e9), fpi[st] / (bench.stage_peak_tflops(st, precision) * 1e12))
        total_ms = t * images * passes * 1e3
        out[st] = {"total_ms": total_ms, "launches": launches, "avg_ms": total_ms / launches}
        per_image += passes * t
    return out, per_image


FWD = ["fwd_rows", "fwd_cols", "fwd_gather", "fwd_angular", "radial_fwd"]
ADJ = ["radial_adj", "adj_angular", "adj_spread", "adj_cols", "adj_rows"]


def test_step_roofline_at_bound_is_one(bench):
    plan = _plan()
    n, steps = 10000, 3
    stages, per_image = _stages_at_bound(bench, plan, FWD + ["covariance"], n * steps, 15, "bf16x3")
    r = bench.step_roofline(plan, "bf16x3", stages, n * steps, per_image * n * 1e3, n)
    assert r["frac"] == pytest.approx(1.0, abs=1e-3)
    assert all(v == pytest.approx(1.0, abs=1e-3) for v in r["stage_frac"].values())


def test_step_roofline_counts_forward_and_backward_once_each(bench):
    plan = _plan()
    n, steps = 20000, 3
    stages, per_image = _stages_at_bound(bench, plan, FWD + ADJ, n * steps, 60, "fp32", passes=2)
    two = bench.step_roofline(plan, "fp32", stages, n * steps, per_image * n * 1e3, n, passes=2)
    assert two["frac"] == pytest.approx(1.0, abs=1e-3)
    assert all(v == pytest.approx(1.0, abs=1e-3) for v in two["stage_frac"].values())
    # the same stage table read as one pass per image would halve every fraction
    one = bench.step_roofline(plan, "fp32", stages, n * steps, per_image * n * 1e3, n)
    assert one["frac"] == pytest.approx(0.5, abs=1e-3)
    # both directions' image and coefficient bytes, twice
    irr = 4 * plan.L ** 2 + 8 * plan.p_half
    assert two["irreducible_MB_per_image"] == pytest.approx(4 * irr / 1e6, abs=1e-3)


def test_kernel_roofline_rate_per_launch(bench):
    plan = _plan()
    n, steps, launches = 20000, 3, 60
    stages, _ = _stages_at_bound(bench, plan, FWD + ADJ, n * steps, launches, "fp32", passes=2)
    stages["adj_spread"]["total_ms"] *= 10.0  # make the spread dominant, at a tenth of its bound
    stages["adj_spread"]["avg_ms"] *= 10.0
    r = bench.kernel_roofline(plan, stages, 2 * n * steps, "fp32")
    assert r["kernel"] == "adj_spread" and r["bound"] == "hbm"
    assert r["images_per_launch"] == pytest.approx(2 * n * steps / launches)
    bpi = bench.algorithmic_bytes_per_image(plan)["adj_spread"]
    assert r["bytes_per_launch"] == pytest.approx(bpi * 2 * n * steps / launches, rel=1e-6)
    assert r["frac"] == pytest.approx(0.1, abs=1e-3)
