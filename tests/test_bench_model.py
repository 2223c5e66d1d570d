"""CPU: the byte model behind bench.py's roofline line (host logic only)."""

import types

import numpy as np

import bench


def _win(n, W, H, R, F=1):
    rho = np.zeros((F, H, W) if F > 1 else (H, W), np.float32)
    return types.SimpleNamespace(n=n, width=W, height=H, refs=[0.0] * R, rho=rho)


def test_splat_bytes_follow_the_plan_at_active_pixels():
    # tiled splat: 16 B of state (C, S of both polarities at FP32) per active
    # pixel and reference; the library's FP64 images are twice that
    assert bench.algorithmic_bytes("splat", 1000, 100, 2, True, 1, 37.0) == 16.0 * 37
    assert bench.algorithmic_bytes("splat", 1000, 100, 2, True, 1, 37.0,
                                   bench.STATE_BYTES_FP64) == 32.0 * 37
    # direct splat writes the whole images
    assert bench.algorithmic_bytes("splat", 1000, 100, 2, False, 1) == 13e3 + 400 + 16 * 2 * 100


def test_sweep_and_count_bytes():
    # events 13 B, inverse depth 4 B per pixel and flow set, state at active pixels
    assert bench.algorithmic_bytes("adjoint", 10, 50, 3, True, 2, 5.0) == 130 + 400 + 80
    assert bench.algorithmic_bytes("count", 10, 50, 3, True, 2, 5.0) == 130 + 400
    assert bench.algorithmic_bytes("scan", 10, 50, 3, True, 2, 5.0) == 0.0


def test_roofline_of_picks_the_dominant_phase_and_divides_per_launch():
    wins = [_win(1000, 10, 10, 2), _win(3000, 10, 10, 2)]
    act = [20.0, 40.0]
    # phase -> (total ms over 4 steps, launches): splat dominates (8 ms total)
    phases = {"splat": (8.0, 4), "count": (2.0, 4), "scan": (0.0, 0)}
    roof, per_launch = bench.roofline_of(phases, 4, wins, act, True, "none")
    assert roof["kernel"] == "splat"
    assert roof["avg_launch_ms"] == 2.0
    assert roof["algorithmic_bytes_per_launch"] == 16.0 * 60
    assert abs(roof["achieved"] - 16.0 * 60 / 2e-3 / 1e9) < 1e-12
    assert abs(roof["frac"] - roof["achieved"] / bench.HBM_PEAK_GBS) < 1e-15
    assert roof["fp64_state"]["algorithmic_bytes_per_launch"] == 32.0 * 60
    assert set(per_launch) == {"splat", "count"}
