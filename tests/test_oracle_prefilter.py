"""Pins for the oracle's hole-filling joint bilateral pre-filter (Section VI
pre-processing of live depth): exact cases (constant and linear depth),
colour guidance across an edge, the support threshold, untouched measured
and background pixels, and the fixed-point weights against the continuous
Gaussian definition within the bound their rounding allows."""
import math

import numpy as np
import pytest

import oracle

KW = dict(radius=2, sigma_s=1.5, sigma_c=24.0, min_valid=5)


def test_constant_depth_hole_is_filled_with_the_constant():
    rgb = np.full((9, 11, 3), 90, np.uint8)
    d = np.full((9, 11), 2345, np.uint16)
    d[4, 5] = 0
    d[4, 6] = 0
    out = oracle.prefilter(rgb, d, **KW)
    assert out[4, 5] == 2345 and out[4, 6] == 2345


def test_linear_ramp_is_reproduced_by_the_symmetric_window():
    rgb = np.full((12, 14, 3), 40, np.uint8)
    x = np.arange(14)
    d = np.tile(1000 + 7 * x, (12, 1)).astype(np.uint16)
    d[6, 7] = 0
    out = oracle.prefilter(rgb, d, **KW)
    assert out[6, 7] == 1000 + 7 * 7


def test_colour_guides_the_fill_across_an_edge():
    rgb = np.zeros((10, 12, 3), np.uint8)
    rgb[:, :6] = (200, 30, 30)
    rgb[:, 6:] = (20, 120, 220)
    d = np.zeros((10, 12), np.uint16)
    d[:, :6] = 1500
    d[:, 6:] = 4200
    d[5, 5] = 0          # a hole on the left side of the edge, right neighbours nearby
    d[3, 6] = 0          # and one on the right side
    out = oracle.prefilter(rgb, d, **KW)
    assert out[5, 5] == 1500 and out[3, 6] == 4200
    # without colour guidance (huge sigma_c) the edge bleeds in
    bleed = oracle.prefilter(rgb, d, radius=2, sigma_s=1.5, sigma_c=1e6, min_valid=5)
    assert 1500 < bleed[5, 5] < 4200


def test_support_threshold_and_untouched_pixels():
    rgb = np.full((7, 7, 3), 128, np.uint8)
    d = np.full((7, 7), oracle.BG_MM, np.uint16)     # background everywhere ...
    d[3, 3] = 0                                       # ... around one hole
    ys, xs = [2, 2, 2, 3], [2, 3, 4, 2]
    d[ys, xs] = 3000                                  # four supporting neighbours
    out = oracle.prefilter(rgb, d, **KW)
    assert out[3, 3] == 0                             # 4 < min_valid
    assert np.array_equal(out[d != 0], d[d != 0])     # measured and background untouched
    d[3, 4] = 3100                                    # a fifth one
    out = oracle.prefilter(rgb, d, **KW)
    assert 3000 <= out[3, 3] <= 3100
    assert np.array_equal(out[d != 0], d[d != 0])
    d2 = d.copy()
    d2[d2 == 3000] = 0
    d2[3, 4] = 0
    out = oracle.prefilter(rgb, d2, **KW)             # a hole among background only
    assert out[3, 3] == 0


@pytest.mark.parametrize("seed", range(3))
def test_fixed_point_weights_against_the_continuous_filter(seed):
    rng = np.random.default_rng(seed)
    H, W = 24, 30
    rgb = (100 + 24 * rng.integers(0, 2, (H, W, 3))).astype(np.uint8)   # L1 distances 0..72
    d = rng.integers(800, 6000, (H, W)).astype(np.uint16)
    d[rng.random((H, W)) < 0.3] = 0
    d[rng.random((H, W)) < 0.05] = oracle.BG_MM
    ss, sc, r = KW["sigma_s"], KW["sigma_c"], KW["radius"]
    out = oracle.prefilter(rgb, d, **KW)
    checked = 0
    for y in range(H):
        for x in range(W):
            if d[y, x] != 0:
                continue
            ws, vals, dw = [], [], []
            for dy in range(-r, r + 1):
                for dx in range(-r, r + 1):
                    yy, xx = y + dy, x + dx
                    if (dx, dy) == (0, 0) or not (0 <= yy < H and 0 <= xx < W):
                        continue
                    q = int(d[yy, xx])
                    if q in (0, oracle.BG_MM):
                        continue
                    dist = int(np.abs(rgb[y, x].astype(int) - rgb[yy, xx].astype(int)).sum())
                    a = 4096 * math.exp(-(dx * dx + dy * dy) / (2 * ss * ss))
                    b = 4096 * math.exp(-dist * dist / (2 * sc * sc))
                    if round(a) * round(b) == 0:
                        continue
                    ws.append(a * b)
                    vals.append(q)
                    dw.append(0.5 * (a + b) + 0.25)      # bound on the rounding error of a*b
            if len(vals) < KW["min_valid"]:
                assert out[y, x] == 0
                continue
            ws, vals, dw = np.array(ws), np.array(vals, float), np.array(dw)
            mean = (ws * vals).sum() / ws.sum()
            bound = (dw * np.abs(vals - mean)).sum() / (ws.sum() - dw.sum()) + 0.5 + 1e-9
            assert abs(int(out[y, x]) - mean) <= bound, (y, x, out[y, x], mean, bound)
            checked += 1
    assert checked > 20
