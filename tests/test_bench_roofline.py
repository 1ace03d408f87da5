"""The benchmark's roofline arithmetic on recorded counters (no GPU): the backward raster's
algorithmic bytes and FLOPs per launch follow the per-unit figures (40 B per consumed list entry,
44 B per pixel, 172 B of statistics per kernel and view; 222 FLOP per contributing pair, 18 per
re-evaluated entry), against the published FP32 vector peak and HBM bandwidth."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_backward_roofline_from_recorded_counters():
    b = _bench()
    steps, views, n = 20, 4, 1_000_000
    pixels = 1920 * 1080 + 3 * 960 * 540
    per_step = {"fwd_evals": 200961700, "bwd_evals": 2700717, "bwd_active": 113370003, "pairs": 68655427,
                "partials": 1346959, "fwd_staged": 5361017, "bwd_staged": 5361017, "fp64_solves": 0}
    counts = {k: v * steps for k, v in per_step.items()}
    launches = views * steps
    stages = {"raster_bwd": (0.9249 * launches, launches), "sort": (1.0, 40)}
    rl = b.roofline(stages, counts, steps, pixels, n, views)
    assert rl["kernel"] == "raster_bwd" and rl["bound"] == "alu" and rl["peak"] == 157.3
    bytes_launch = (40 * 5361017 + 44 * pixels + 172 * n * views) / views
    assert abs(rl["algorithmic_bytes_per_launch"] - bytes_launch) <= 1
    assert abs(rl["hbm_fraction"] - bytes_launch / 0.9249e-3 / 8e12) < 1e-5
    assert 0.035 < rl["hbm_fraction"] < 0.037
    flops = (222 * 113370003 + 18 * 2700717) / views
    assert abs(rl["algorithmic_flops_per_launch"] - flops) <= 1
    assert 0.042 < rl["frac"] < 0.044
    assert abs(rl["frac_unpacked"] - 2 * rl["frac"]) < 1e-4


def test_solve_rule_rates():
    b = _bench()
    c = {"solved": 1000.0}
    for g in ("position", "rotation", "scaling", "opacity"):
        c[f"escalated_{g}"] = 10.0
        c[f"fallback_{g}"] = 1.0
    for g in ("position", "rotation", "scaling", "colour"):
        c[f"clamped_{g}"] = 5.0
    c["opacity_bound"] = 2.0
    r = b.solve_rules(c)
    assert r["escalated_rotation"] == 0.01 and r["fallback_opacity"] == 0.001
    assert r["trust_clamped_colour"] == 0.005 and r["opacity_bound"] == 0.002
