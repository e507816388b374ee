"""Pins for the CPU oracle (no GPU).

Each test ties one oracle step to something other than the oracle itself:
a closed form (pinhole homography, integer shift, 1.5x magnification),
an identity (virtual camera == source camera), brute force on tiny inputs,
hand-derived fixtures under ``tests/golden/`` or an independent scan-based
re-derivation.  Steps are named O1..O7 as in the oracle's header.
"""
import math
import os

import numpy as np
import pytest

import scenegen as sg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)


def f32bits(z):
    return int(np.float32(z).view(np.uint32))


def mkkey(z, cam, pix):
    return np.uint64((f32bits(z) << 32) | (cam << 27) | pix)


def plain_cam(w, h, fx, fy=None, cx=None, cy=None, R=None, t=(0, 0, 0), alpha=0.0, beta=1.0):
    fy = fx if fy is None else fy
    cx = (w - 1) / 2.0 if cx is None else cx
    cy = (h - 1) / 2.0 if cy is None else cy
    R = np.eye(3) if R is None else R
    return sg.Camera(w, h, fx, fy, cx, cy, R, np.asarray(t, float), alpha, beta)


def plane_frame(cam, depth_m, rgb_fn=None):
    """Fronto-parallel plane at constant depth; texture from pixel coords."""
    H, W = cam.height, cam.width
    jj, ii = np.mgrid[0:H, 0:W]
    if rgb_fn is None:
        rgb = np.stack([(ii * 37 + jj * 11) % 256, (ii * 5 + jj * 71) % 256,
                        (ii * 13 ^ jj * 29) % 256], -1).astype(np.uint8)
    else:
        rgb = rgb_fn(ii, jj)
    d = np.full((H, W), int(round(depth_m * 1000)), np.uint16)
    return sg.Frame(rgb, d)


# ------------------------------------------------------------------ O3 (Eq. 1)
def test_decode_identity_is_exact_for_every_code(oracle_lib):
    o = oracle_lib
    codes = np.arange(1, 65536, dtype=np.uint32)
    expect = codes.astype(np.float32) / np.float32(1000.0)   # IEEE float32 division
    got = np.array([o.decode_depth(int(c)) for c in codes[::7]], np.float32)
    assert np.array_equal(got.view(np.uint32), expect[::7].view(np.uint32))
    assert o.decode_depth(1000) == np.float32(1.0)


@pytest.mark.parametrize("alpha,beta", [(0.01, 0.98), (-0.02, 1.03), (0.0, 1.1)])
def test_decode_matches_quadratic_correction(oracle_lib, alpha, beta):
    o = oracle_lib
    a, b = float(np.float32(alpha)), float(np.float32(beta))
    for d in (1, 500, 999, 1234, 2500, 4000, 8191, 65535):
        z = float(np.float32(d) / np.float32(1000.0))
        exact = (a * z + b) * z                      # Eq. 1 in double
        got = float(o.decode_depth(d, alpha, beta))
        assert abs(got - exact) <= 3 * abs(np.spacing(np.float32(exact))), (d, got, exact)


# ------------------------------------------------------------------ O1
def test_selection_hand_rig(oracle_lib):
    o = oracle_lib
    # centres at x = -2,-1,0,1,2 (t = -R C with R = I), virtual at x = 0.4
    rig = [plain_cam(8, 8, 10.0, t=(-x, 0, 0)) for x in (-2.0, -1.0, 0.0, 1.0, 2.0)]
    v = plain_cam(8, 8, 10.0, t=(-0.4, 0, 0))
    idx, w = o.select(rig, v, 3)
    assert list(idx) == [2, 3, 1]            # distances 0.4, 0.6, 1.4
    np.testing.assert_allclose(w, [1 / 0.4, 1 / 0.6, 1 / 1.4], rtol=1e-6)
    # K larger than the rig
    idx, _ = o.select(rig, v, 8)
    assert list(idx) == [2, 3, 1, 4, 0]
    # absent cameras are skipped
    idx, _ = o.select(rig, v, 3, present=[1, 1, 0, 1, 1])
    assert list(idx) == [3, 1, 4]
    # exact tie -> lower rig index first
    v0 = plain_cam(8, 8, 10.0, t=(-0.5, 0, 0))
    idx, w = o.select(rig, v0, 2)
    assert list(idx) == [2, 3] and w[0] == w[1]
    # coincident virtual camera -> that camera alone, weight 1
    v1 = plain_cam(8, 8, 10.0, t=(-1.0, 0, 0))
    idx, w = o.select(rig, v1, 3)
    assert list(idx) == [3] and list(w) == [1.0]


# ------------------------------------------------------------------ O2
def _world_space_projection(src, virt, i, j, z):
    """Independent double-precision path through world space."""
    K = np.array([[src.fx, 0, src.cx], [0, src.fy, src.cy], [0, 0, 1.0]])
    Kv = np.array([[virt.fx, 0, virt.cx], [0, virt.fy, virt.cy], [0, 0, 1.0]])
    rays = np.linalg.solve(K, np.stack([i, j, np.ones_like(i)]))
    Xc = rays * z
    Xw = src.R.T @ (Xc - src.t[:, None])
    Xv = virt.R @ Xw + virt.t[:, None]
    p = Kv @ Xv
    return p[0] / p[2], p[1] / p[2], p[2]


@pytest.mark.parametrize("cfg", ["c1", "c2", "small"])
def test_pair_matrices_match_world_space(oracle_lib, cfg):
    o = oracle_lib
    w = {"c1": sg.config1, "c2": sg.config2, "small": sg.config_small}[cfg](0)
    rng = np.random.default_rng(1)
    for src in w.rig:
        for virt in w.virtual:
            P = o.pair_arrays(src, virt)
            i = rng.uniform(0, src.width - 1, 500)
            j = rng.uniform(0, src.height - 1, 500)
            z = rng.uniform(0.8, 6.0, 500)
            ue, ve, ze = _world_space_projection(src, virt, i, j, z)
            p = (P["A"].astype(np.float64) @ np.stack([i, j, np.ones_like(i)])) * z \
                + P["a"].astype(np.float64)[:, None]
            assert np.max(np.abs(p[0] / p[2] - ue)) < 1e-3
            assert np.max(np.abs(p[1] / p[2] - ve)) < 1e-3
            assert np.max(np.abs(p[2] / ze - 1)) < 1e-6
            # backward pair inverts the forward one
            x, y = p[0] / p[2], p[1] / p[2]
            q = (P["B"].astype(np.float64) @ np.stack([x, y, np.ones_like(x)])) * p[2] \
                + P["b"].astype(np.float64)[:, None]
            assert np.max(np.abs(q[0] / q[2] - i)) < 1e-3
            assert np.max(np.abs(q[2] / z - 1)) < 1e-6
            assert P["sx"] == np.float32(virt.fx / src.fx)


# ------------------------------------------------------------------ O4
def test_splat_identity_camera_maps_every_pixel_to_itself(oracle_lib):
    o = oracle_lib
    w = sg.config1(0)
    src, fr = w.rig[0], w.frames[0]
    Z = o.splat(w.rig, [fr.depth_mm], src, [0])
    valid = fr.depth_mm > 0
    H, W = fr.depth_mm.shape
    own = np.arange(H * W).reshape(H, W)
    assert np.array_equal(Z == EMPTY, ~valid)
    assert np.array_equal(o.key_pixel(Z)[valid], own[valid])
    assert np.all(o.key_cam(Z)[valid] == 0)
    dec = fr.depth_mm.astype(np.float32) / np.float32(1000.0)
    assert np.array_equal(o.key_depth(Z)[valid].view(np.uint32), dec[valid].view(np.uint32))


def test_splat_integer_shift_closed_form(oracle_lib):
    """Fronto-parallel plane at depth D, virtual camera translated along x by
    delta: the homography reduces to u = i - fx*delta/D, here exactly 7 px."""
    o = oracle_lib
    fx, D = 300.0, 2.0
    src = plain_cam(48, 20, fx)
    delta = 7.0 * D / fx
    virt = plain_cam(48, 20, fx, t=(-delta, 0, 0))
    fr = plane_frame(src, D)
    Z = o.splat([src], [fr.depth_mm], virt, [0])
    pix = o.key_pixel(Z)
    for y in range(20):
        for x in range(48):
            if x + 7 < 48:
                assert Z[y, x] != EMPTY and pix[y, x] == y * 48 + x + 7, (x, y)
            else:
                assert Z[y, x] == EMPTY


def test_splat_magnification_tiles_exactly_once(oracle_lib):
    """Pure 1.5x zoom of a fronto-parallel plane: source column i lands at
    u = 1.5 i; even i cover x = 3k, odd i cover x = 3k+1 and 3k+2, so every
    covered output pixel has exactly one possible source."""
    o = oracle_lib
    src = plain_cam(20, 14, 200.0, cx=0.0, cy=0.0)
    virt = plain_cam(30, 21, 300.0, cx=0.0, cy=0.0)
    fr = plane_frame(src, 1.7)
    Z = o.splat([src], [fr.depth_mm], virt, [0])
    pix = o.key_pixel(Z)

    def src_of(x):
        k, r = divmod(x, 3)
        return 2 * k if r == 0 else 2 * k + 1

    for y in range(21):
        for x in range(30):
            i, j = src_of(x), src_of(y)
            assert i < 20 and j < 14
            assert Z[y, x] != EMPTY and pix[y, x] == j * 20 + i, (x, y)


def test_splat_minification_ties_go_to_lowest_pixel(oracle_lib):
    """0.5x zoom of a fronto-parallel plane at one depth: every output pixel
    is covered by several source pixels with equal depth keys; the lowest
    source index wins."""
    o = oracle_lib
    src = plain_cam(16, 12, 200.0, cx=0.0, cy=0.0)
    virt = plain_cam(8, 6, 100.0, cx=0.0, cy=0.0)
    fr = plane_frame(src, 2.5)
    Z = o.splat([src], [fr.depth_mm], virt, [0])
    # u = i/2 covers x iff u - 0.5 <= x < u + 0.5  <=>  i in {2x, 2x+1}
    for y in range(6):
        for x in range(8):
            i, j = 2 * x, 2 * y
            assert o.key_pixel(Z)[y, x] == j * 16 + i
            assert o.key_depth(Z)[y, x] == np.float32(2.5)


def _f32_project(M, m, i, j, z):
    M = M.astype(np.float32)
    out = []
    for r in range(3):
        s = np.float32(M[r, 0] * np.float32(i)) + np.float32(M[r, 1] * np.float32(j))
        s = np.float32(s + M[r, 2])
        s = np.float32(s * z)
        out.append(np.float32(s + m[r]))
    return out


def _brute_force_splat(o, rig, depths, virt, sel, max_fp):
    """Gather formulation: for every output pixel enumerate every (camera,
    source pixel) whose footprint covers it and keep the smallest key."""
    H, W = virt.height, virt.width
    cands = []
    for c in sel:
        P = o.pair_arrays(rig[c], virt)
        d = depths[c]
        for j in range(d.shape[0]):
            for i in range(d.shape[1]):
                if d[j, i] == 0:
                    continue
                z = o.decode_depth(int(d[j, i]), rig[c].depth_alpha, rig[c].depth_beta)
                p0, p1, p2 = _f32_project(P["A"], P["a"], i, j, z)
                if not p2 > np.float32(0.01):
                    continue
                u, v = np.float32(p0 / p2), np.float32(p1 / p2)
                mx = min(max(np.float32(np.float32(P["sx"] * z) / p2), np.float32(1)), np.float32(max_fp))
                my = min(max(np.float32(np.float32(P["sy"] * z) / p2), np.float32(1)), np.float32(max_fp))
                lo_u, hi_u = np.float32(u - np.float32(0.5) * mx), np.float32(u + np.float32(0.5) * mx)
                lo_v, hi_v = np.float32(v - np.float32(0.5) * my), np.float32(v + np.float32(0.5) * my)
                key = (f32bits(p2) << 32) | (c << 27) | (j * d.shape[1] + i)
                cands.append((lo_u, hi_u, lo_v, hi_v, key))
    Z = np.full((H, W), EMPTY)
    for y in range(H):
        for x in range(W):
            best = None
            for lo_u, hi_u, lo_v, hi_v, key in cands:
                if lo_u <= x < hi_u and lo_v <= y < hi_v and (best is None or key < best):
                    best = key
            if best is not None:
                Z[y, x] = np.uint64(best)
    return Z


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_splat_brute_force_tiny(oracle_lib, seed):
    o = oracle_lib
    rng = np.random.default_rng(seed)
    rig = [sg.arc_camera(a, 2.0, 14, 10, hfov_deg=50) for a in (-10.0, 0.0, 12.0)]
    rig[1].depth_alpha, rig[1].depth_beta = float(np.float32(0.01)), float(np.float32(0.99))
    depths = []
    for c in rig:
        d = rng.integers(1200, 3200, size=(10, 14)).astype(np.uint16)
        d[rng.random((10, 14)) < 0.15] = 0
        depths.append(d)
    # duplicate depths across cameras to exercise the camera tie-break
    depths[2][:3, :] = depths[0][:3, :]
    virt = sg.arc_camera(4.0, 1.8, 16, 12, hfov_deg=50)
    sel = [2, 0, 1]
    Z = o.splat(rig, depths, virt, sel, max_fp=3.0)
    Zb = _brute_force_splat(o, rig, depths, virt, sel, 3.0)
    assert np.array_equal(Z, Zb)
    assert (Z != EMPTY).mean() > 0.5


# ------------------------------------------------------------------ O5
def _parse_cases(path):
    cases, cur, section = [], None, None
    for raw in open(path):
        line = raw.split("#", 1)[0].strip() if not raw.lstrip().startswith("#") else ""
        if raw.strip().startswith("case "):
            cur = {"name": raw.split()[1], "in": [], "out": []}
            section = "hdr"
            continue
        if cur is None:
            continue
        tokens = raw.strip().split()
        if not tokens:
            continue
        if tokens[0] in ("in", "out"):
            section = tokens[0]
            continue
        if tokens[0] == "end":
            cases.append(cur)
            cur = None
            continue
        if section == "hdr":
            cur["hdr"] = tokens
        else:
            cur[section] += tokens
    return cases


def _key_cell(tok):
    if tok == ".":
        return EMPTY
    z, p = tok.split(":")
    return mkkey(float(z), 0, int(p))


FILTER_CASES = _parse_cases(os.path.join(GOLDEN, "filter_cases.txt"))


@pytest.mark.parametrize("case", FILTER_CASES, ids=[c["name"] for c in FILTER_CASES])
def test_filter_golden(oracle_lib, case):
    W, H, tau = int(case["hdr"][0]), int(case["hdr"][1]), float(case["hdr"][2])
    Zin = np.array([_key_cell(t) for t in case["in"]], np.uint64).reshape(H, W)
    Zexp = np.array([_key_cell(t) for t in case["out"]], np.uint64).reshape(H, W)
    Zf = oracle_lib.depth_filter(Zin, tau)
    assert np.array_equal(Zf, Zexp)


# ------------------------------------------------------------------ O7
def _fill_cell(tok):
    if tok == "#":
        return (0, 0, 0), 1, 0.0
    col, z = tok.split("@")
    return tuple(int(v) for v in col.split(",")), 0, float(z)


FILL_CASES = _parse_cases(os.path.join(GOLDEN, "fill_cases.txt"))


@pytest.mark.parametrize("case", FILL_CASES, ids=[c["name"] for c in FILL_CASES])
def test_fill_golden(oracle_lib, case):
    W, H, mode = (int(v) for v in case["hdr"])
    cells = [_fill_cell(t) for t in case["in"]]
    rgb = np.array([c[0] for c in cells], np.uint8).reshape(H, W, 3)
    hole = np.array([c[1] for c in cells], np.uint8).reshape(H, W)
    dep = np.array([c[2] for c in cells], np.float32).reshape(H, W)
    exp = np.array([[int(v) for v in t.split(",")] for t in case["out"]], np.uint8).reshape(H, W, 3)
    assert np.array_equal(oracle_lib.fill(rgb, hole, dep, mode), exp)


def _scan_fill(rgb, hole, depth):
    """Independent formulation with prefix scans (nearest non-hole index via
    running max / min of indices), then a lexicographic choice."""
    H, W = hole.shape
    nh = hole == 0
    idx_x = np.broadcast_to(np.arange(W), (H, W))
    idx_y = np.broadcast_to(np.arange(H)[:, None], (H, W))
    left = np.maximum.accumulate(np.where(nh, idx_x, -1), axis=1)
    left = np.concatenate([np.full((H, 1), -1), left[:, :-1]], 1)
    right = np.minimum.accumulate(np.where(nh, idx_x, W)[:, ::-1], axis=1)[:, ::-1]
    right = np.concatenate([right[:, 1:], np.full((H, 1), W)], 1)
    up = np.maximum.accumulate(np.where(nh, idx_y, -1), axis=0)
    up = np.concatenate([np.full((1, W), -1), up[:-1]], 0)
    down = np.minimum.accumulate(np.where(nh, idx_y, H)[::-1], axis=0)[::-1]
    down = np.concatenate([down[1:], np.full((1, W), H)], 0)
    out = rgb.copy()
    for y, x in zip(*np.nonzero(hole)):
        cands = []
        if left[y, x] >= 0:
            cands.append((-depth[y, left[y, x]], x - left[y, x], 0, (y, left[y, x])))
        if right[y, x] < W:
            cands.append((-depth[y, right[y, x]], right[y, x] - x, 1, (y, right[y, x])))
        if up[y, x] >= 0:
            cands.append((-depth[up[y, x], x], y - up[y, x], 2, (up[y, x], x)))
        if down[y, x] < H:
            cands.append((-depth[down[y, x], x], down[y, x] - y, 3, (down[y, x], x)))
        out[y, x] = rgb[min(cands)[3]] if cands else 0
    return out


@pytest.mark.parametrize("seed", range(4))
def test_fill_matches_scan_formulation(oracle_lib, seed):
    rng = np.random.default_rng(seed)
    H, W = 23, 31
    rgb = rng.integers(0, 256, (H, W, 3)).astype(np.uint8)
    hole = (rng.random((H, W)) < [0.2, 0.5, 0.8, 0.97][seed]).astype(np.uint8)
    dep = rng.choice(np.float32([1.0, 2.0, 2.5, 4.0]), (H, W)).astype(np.float32)
    out = oracle_lib.fill(rgb, hole, dep, 0)
    assert np.array_equal(out, _scan_fill(rgb, hole, dep))
    assert np.array_equal(out[hole == 0], rgb[hole == 0])


# ------------------------------------------------------------------ O6 / whole path
def test_identity_view_reproduces_source(oracle_lib):
    o = oracle_lib
    w = sg.config1(0)
    r = o.synthesize(w.rig, w.frames, w.rig[0], k_nearest=3, taps=True, fill_mode=1)
    valid = w.frames[0].depth_mm > 0
    kept = valid & (r["z"] == r["zf"])
    assert kept.sum() > 0.6 * valid.size
    assert np.array_equal(r["blend_rgb"][kept], w.frames[0].rgb[kept])
    assert np.all(r["hole"][kept] == 0)
    # no point lands where the source had no depth, and every such pixel is
    # a hole, also where the filter closed a crack: the backward fetch of the
    # identity view lands exactly on the pixel itself, whose tap has no depth
    assert np.all(r["z"][~valid] == EMPTY)
    assert (r["zf"][~valid] != EMPTY).any(), "the case should include filter-closed cracks"
    assert np.all(r["hole"][~valid] == 1)
    # with fill disabled the whole valid region is an exact copy
    assert np.array_equal(r["rgb"][kept], w.frames[0].rgb[kept])


@pytest.mark.parametrize("cam", [0, 1, 2])
def test_identity_view_reproduces_source_noisy_rig(oracle_lib, cam):
    """Virtual camera = one camera of the three-camera rig with depth noise
    and 5 % isolated invalid pixels: that camera alone is selected (weight
    1), and every pixel with depth is an exact copy of the source unless the
    speckle filter replaced its key.  The rig's float32 rotations are
    orthonormal only to rounding, so the pair matrices of a camera with
    itself differ from the identity by ~1e-5 px: a pixel without depth whose
    crack the filter closed lands next to its own centre, and neighbour taps
    with bilinear weights of that size can carry it.  Such a pixel then
    holds a mix of its neighbours' source colours (each channel within their
    range); every other pixel without depth is a hole."""
    o = oracle_lib
    w = sg.config2(0)
    src = w.frames[cam]
    r = o.synthesize(w.rig, w.frames, w.rig[cam], k_nearest=3, taps=True, fill_mode=1)
    valid = src.depth_mm > 0
    assert np.all(r["z"][~valid] == EMPTY)
    assert np.all(o.key_cam(r["z"][valid]) == cam)
    closed = ~valid & (r["zf"] != EMPTY)
    assert closed.sum() > 1000
    assert np.all(r["hole"][~valid & ~closed] == 1)
    H, W = valid.shape
    for y, x in zip(*np.nonzero(~valid & (r["hole"] == 0))):
        nb = np.array([src.rgb[yy, xx] for yy in range(max(0, y - 1), min(H, y + 2))
                       for xx in range(max(0, x - 1), min(W, x + 2)) if (yy, xx) != (y, x) and valid[yy, xx]])
        assert len(nb) and np.all(nb.min(0) <= r["rgb"][y, x]) and np.all(r["rgb"][y, x] <= nb.max(0)), (y, x)
    kept = valid & (r["z"] == r["zf"])
    assert kept.sum() > 0.9 * valid.sum()
    assert np.all(r["hole"][kept] == 0)
    assert np.array_equal(r["rgb"][kept], src.rgb[kept])


def test_integer_shift_view_is_shifted_source(oracle_lib):
    o = oracle_lib
    fx, D = 300.0, 2.0
    src = plain_cam(64, 24, fx)
    virt = plain_cam(64, 24, fx, t=(-7.0 * D / fx, 0, 0))
    fr = plane_frame(src, D)
    r = o.synthesize([src], [fr], virt, k_nearest=1, taps=True, fill_mode=1)
    assert np.array_equal(r["rgb"][:, :57], fr.rgb[:, 7:])
    assert np.all(r["hole"][:, 57:] == 1)


def test_general_plane_matches_bilinear_homography(oracle_lib):
    """Tilted textured plane, virtual camera rotated and translated: the
    output equals bilinear sampling of the source at H^-1(x, y), computed
    independently in double through world space."""
    o = oracle_lib
    W, H = 80, 60
    src = plain_cam(W, H, 90.0)
    jj, ii = np.mgrid[0:H, 0:W].astype(np.float64)
    # plane n.X = 1 in camera coords with n = (0.15, -0.1, 0.5): z = 1/(n . K^-1 [i,j,1])
    n = np.array([0.15, -0.1, 0.5])
    rx = (ii - src.cx) / src.fx
    ry = (jj - src.cy) / src.fy
    z = 1.0 / (n[0] * rx + n[1] * ry + n[2])
    assert z.min() > 1.0 and z.max() < 4.0
    rgb = np.stack([128 + 100 * np.sin(ii / 5.0), 128 + 100 * np.cos(jj / 4.0),
                    128 + 100 * np.sin((ii + jj) / 7.0)], -1)
    rgb = np.floor(rgb + 0.5).astype(np.uint8)
    dmm = np.floor(z * 1000 + 0.5).astype(np.uint16)
    fr = sg.Frame(rgb, dmm)
    a = math.radians(3.0)
    Ry = np.array([[math.cos(a), 0, math.sin(a)], [0, 1, 0], [-math.sin(a), 0, math.cos(a)]])
    virt = plain_cam(W, H, 95.0, R=Ry, t=(0.05, 0.02, 0.03))
    r = o.synthesize([src], [fr], virt, k_nearest=1, taps=True, fill_mode=1)
    # independent: intersect the virtual pixel ray with the plane in world
    # space (source camera frame == world), project into the source, bilinear
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    dv = np.stack([(xx - virt.cx) / virt.fx, (yy - virt.cy) / virt.fy, np.ones_like(xx)])
    dw = np.einsum("ij,jhw->ihw", virt.R.T, dv)
    cw = -virt.R.T @ virt.t
    s = (1.0 - n @ cw) / np.einsum("i,ihw->hw", n, dw)
    Xw = cw[:, None, None] + s * dw
    u = src.fx * Xw[0] / Xw[2] + src.cx
    v = src.fy * Xw[1] / Xw[2] + src.cy
    inside = (u > 1) & (u < W - 2) & (v > 1) & (v < H - 2)
    i0, j0 = np.floor(u).astype(int), np.floor(v).astype(int)
    fu, fv = u - i0, v - j0
    i0c, j0c = np.clip(i0, 0, W - 2), np.clip(j0, 0, H - 2)
    c = rgb.astype(np.float64)
    bil = ((1 - fu) * (1 - fv))[..., None] * c[j0c, i0c] + (fu * (1 - fv))[..., None] * c[j0c, i0c + 1] \
        + ((1 - fu) * fv)[..., None] * c[j0c + 1, i0c] + (fu * fv)[..., None] * c[j0c + 1, i0c + 1]
    expect = np.floor(bil + 0.5)
    ok = inside & (r["hole"] == 0)
    assert ok.sum() > 0.7 * inside.sum()
    err = np.abs(r["blend_rgb"].astype(np.float64) - expect)[ok]
    # depth quantisation (1 mm) moves the sample by < 0.05 px here: <= 1 LSB
    # for most pixels, a few LSB where the texture is steepest
    assert np.mean(err <= 1) > 0.97 and err.max() <= 6


def test_constant_colour_scene_gives_constant_output(oracle_lib):
    o = oracle_lib
    w = sg.config_small(3)
    frames = [sg.Frame(np.full_like(f.rgb, 0) + np.uint8([37, 140, 222]), f.depth_mm) for f in w.frames]
    for v in w.virtual:
        r = o.synthesize(w.rig, frames, v, taps=True)
        assert r["hole"].mean() < 0.5
        assert np.all(r["rgb"].reshape(-1, 3) == [37, 140, 222])


def test_two_equidistant_cameras_average(oracle_lib):
    o = oracle_lib
    W, H, fx, D = 40, 30, 60.0, 2.0
    left = plain_cam(W, H, fx, t=(0.1, 0, 0))     # centre x = -0.1
    right = plain_cam(W, H, fx, t=(-0.1, 0, 0))   # centre x = +0.1
    virt = plain_cam(W, H, fx)
    fa = plane_frame(left, D, lambda i, j: np.zeros(i.shape + (3,), np.uint8) + np.uint8([0, 100, 255]))
    fb = plane_frame(right, D, lambda i, j: np.zeros(i.shape + (3,), np.uint8) + np.uint8([50, 0, 255]))
    r = o.synthesize([left, right], [fa, fb], virt, k_nearest=2, taps=True, fill_mode=1)
    both = r["hole"] == 0
    # columns seen by both cameras (3 px shift each way at this depth)
    assert np.all(r["blend_rgb"][:, 4:W - 4][both[:, 4:W - 4]] == [25, 50, 255])


def test_absent_camera_is_not_used(oracle_lib):
    o = oracle_lib
    w = sg.config_small(1)
    frames = list(w.frames)
    frames[1] = None
    r = o.synthesize(w.rig, frames, w.virtual[1])
    assert 1 not in list(r["sel"])


# ------------------------------------------------------------------ O6' (network input)
def test_stack_identity_view_holds_source(oracle_lib):
    """Virtual camera == rig camera 0 (selected alone): wherever the identity
    fetch keeps the pixel, the first camera slot holds the source colour / 255,
    0.5 / source depth (float32) and a validity flag; other slots are zero."""
    o = oracle_lib
    w = sg.config1(0)
    r = o.synthesize(w.rig, w.frames, w.rig[0], k_nearest=3, taps=True, fill_mode=1)
    assert list(r["sel"]) == [0]
    st = o.stack(r["zf"], w.rig, w.frames, w.rig[0], r["sel"], r["weights"], pad_rows=5)
    H, W = r["zf"].shape
    assert st.shape == (H + 5, W, 16)
    assert np.all(st[H:] == 0) and np.all(st[..., 15] == 0) and np.all(st[..., 5:] == 0)
    st = st[:H]
    valid = w.frames[0].depth_mm > 0
    kept = valid & (r["z"] == r["zf"])
    assert kept.sum() > 0.6 * valid.size
    src = w.frames[0].rgb.astype(np.float64)
    # the float32 identity warp lands within ~1e-5 px of the integer pixel
    assert np.abs(st[..., 0:3][kept] * 255.0 - src[kept]).max() < 0.01
    z = np.array([o.decode_depth(int(d)) for d in w.frames[0].depth_mm[kept][:2000]], np.float32)
    inv = np.minimum(np.float32(0.5) / z, np.float32(1.0))
    assert np.array_equal(st[..., 3][kept][:2000].astype(np.float32), inv)
    assert np.all(st[..., 4][kept] == 1.0)


def test_stack_two_cameras_keep_their_own_colours(oracle_lib):
    """Two cameras at equal distance see a constant-colour plane each: the
    two slots hold the two colours unmixed, in selection order, and the
    inverse depth of the plane (0.5 / 2 m)."""
    o = oracle_lib
    W, H, fx, D = 40, 30, 60.0, 2.0
    left = plain_cam(W, H, fx, t=(0.1, 0, 0))
    right = plain_cam(W, H, fx, t=(-0.1, 0, 0))
    virt = plain_cam(W, H, fx)
    ca, cb = np.uint8([0, 100, 255]), np.uint8([50, 0, 255])
    fa = plane_frame(left, D, lambda i, j: np.zeros(i.shape + (3,), np.uint8) + ca)
    fb = plane_frame(right, D, lambda i, j: np.zeros(i.shape + (3,), np.uint8) + cb)
    rig, frames = [left, right], [fa, fb]
    r = o.synthesize(rig, frames, virt, k_nearest=2, taps=True, fill_mode=1)
    st = o.stack(r["zf"], rig, frames, virt, r["sel"], r["weights"])
    both = (st[..., 4] == 1) & (st[..., 9] == 1)
    assert both[:, 4:W - 4].all()
    cols = {0: ca, 1: cb}
    for slot, cam in enumerate(r["sel"]):
        got = st[..., 5 * slot:5 * slot + 3][both] * 255.0
        assert np.abs(got - cols[int(cam)]).max() < 1e-9
        assert np.all(st[..., 5 * slot + 3][both] == 0.25)


@pytest.mark.parametrize("seed", [0, 1])
def test_stack_recombines_to_the_blend(oracle_lib, seed):
    """Mixing the stack's valid camera colours with the selection weights
    reproduces the blend (O6) pixel for pixel, and a pixel is a hole of the
    blend exactly when no camera slot is valid."""
    o = oracle_lib
    w = sg.config_small(seed, n_cams=4)
    for v in w.virtual[:2]:
        r = o.synthesize(w.rig, w.frames, v, k_nearest=3, taps=True, fill_mode=1)
        st = o.stack(r["zf"], w.rig, w.frames, v, r["sel"], r["weights"])
        K = len(r["sel"])
        valid = np.stack([st[..., 5 * k + 4] for k in range(K)], -1)
        assert np.array_equal(valid.any(-1), r["hole"] == 0)
        wk = np.asarray(r["weights"])[None, None, :] * valid
        num = sum(wk[..., k, None] * st[..., 5 * k:5 * k + 3] * 255.0 for k in range(K))
        den = wk.sum(-1)[..., None]
        ok = r["hole"] == 0
        mix = np.clip(np.floor(num[ok] / den[ok] + 0.5), 0, 255)
        diff = np.abs(mix - r["blend_rgb"][ok].astype(np.float64))
        assert diff.max() <= 1 and np.mean(diff > 0) < 1e-3


def test_timing_mode_equals_parity_mode(oracle_lib):
    """The benchmark's multi-threaded timing mode (views spread over OpenMP
    threads) returns, view by view, exactly the single-threaded result."""
    o = oracle_lib
    w = sg.config_small(4, n_cams=4, w=96, h=64, out_w=120, out_h=72, n_virtual=6)
    many = o.synthesize_views(w.rig, w.frames, w.virtual, 4)
    for v, got in zip(w.virtual, many):
        assert np.array_equal(got, o.synthesize(w.rig, w.frames, v)["rgb"])

