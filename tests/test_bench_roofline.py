"""The benchmark's roofline arithmetic on the host (no GPU): from a synthetic
per-kernel profile of 10 steps at 256^3, the dominant kernel's figures and
the step's, as they can be re-derived by hand."""
import pytest

import bench

N = 256
ZONES = N ** 3
STEPS = 10


def _prof():
    # {class: (total ms over STEPS steps, launches)}: three launches per step
    return {"update": (3 * STEPS * 1.5, 3 * STEPS), "sweep_x1": (3 * STEPS * 0.7, 3 * STEPS),
            "edge_x1": (3 * STEPS * 0.4, 3 * STEPS), "cons2prim": (3 * STEPS * 0.7, 3 * STEPS),
            "advance": (STEPS * 0.005, STEPS)}


def test_dominant_kernel_priced_at_the_stage_bytes():
    roof, step, kernels = bench.rooflines(_prof(), N, STEPS, 16.0, "fp64")
    assert roof["kernel"] == "update" and roof["bound"] == "hbm" and roof["unit"] == "GB/s"
    alg = (256.0 + 320.0 + 320.0) / 3 * ZONES                  # 298.7 B x 16.78 M zones
    assert roof["algorithmic_bytes_per_launch"] == pytest.approx(alg)
    assert roof["avg_ms"] == pytest.approx(1.5)
    assert roof["achieved"] == pytest.approx(alg / 1.5e-3 / 1e9)
    assert roof["peak"] == 8000.0
    assert roof["frac"] == pytest.approx(alg / 1.5e-3 / 8e12)   # 0.4176
    assert kernels["update"]["share"] == pytest.approx(1.5 / (1.5 + 0.7 + 0.4 + 0.7 + 0.005 / 3))


def test_step_priced_at_896_bytes_per_zone():
    _, step, _ = bench.rooflines(_prof(), N, STEPS, 16.0, "fp64")
    assert step["algorithmic_bytes"] == pytest.approx(896.0 * ZONES)
    assert step["achieved"] == pytest.approx(896.0 * ZONES / 16e-3 / 1e9)
    assert step["frac"] == pytest.approx(896.0 * ZONES / 16e-3 / 8e12)


def test_measured_bytes_follow_the_counter_table():
    """With counters for the current sources, the measured step bytes are the
    sum over classes of bytes per launch times launches per step; without
    them (another precision or size) they are null."""
    t = bench._traffic_table()
    _, step, _ = bench.rooflines(_prof(), N, STEPS, 16.0, "fp64")
    if t is None or not all(k in t["kernels"] for k in ("update", "sweep_x1", "edge_x1", "cons2prim")):
        assert step["measured_bytes"] is None
    else:
        want = sum(t["kernels"][k]["bytes"] * 3 for k in ("update", "sweep_x1", "edge_x1", "cons2prim"))
        assert step["measured_bytes"] == pytest.approx(want)
        assert step["traffic_over_algorithmic"] == pytest.approx(want / (896.0 * ZONES))
    roof, step32, _ = bench.rooflines(_prof(), N, STEPS, 16.0, "fp32")
    assert roof["traffic"] is None and step32["measured_bytes"] is None


def test_launch_units():
    assert bench.launch_units("sweep_x2", N) == 261 * 266 * 266
    assert bench.launch_units("edge_x3", N) == 261 * 261 * 256
    assert bench.launch_units("cons2prim", N) == ZONES
