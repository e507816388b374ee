"""CPU oracle for the DIBR view-synthesis path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps ``fvv_oracle.c`` (plain single-threaded C, built
with gcc, sharing no code with the HIP library) through ctypes and takes its
inputs from :mod:`scenegen` objects and numpy arrays.

Steps (see the header of ``fvv_oracle.c`` for the definitions and readings):
O1 selection, O2 pair matrices, O3 depth decode (Eq. 1), O4 forward splat,
O5 depth filter, O6 backward fetch + blend, O7 hole fill.  The learned-path
reference lives in :mod:`oracle.unet`.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fvv_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_fvv.so")
EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class RefCamera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32),
                ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("R", C.c_float * 9), ("t", C.c_float * 3),
                ("depth_alpha", C.c_float), ("depth_beta", C.c_float)]


class RefPair(C.Structure):
    _fields_ = [("A", C.c_float * 9), ("a", C.c_float * 3), ("B", C.c_float * 9),
                ("b", C.c_float * 3), ("sx", C.c_float), ("sy", C.c_float)]


class RefSrc(C.Structure):
    _fields_ = [("depth", C.c_void_p), ("depth_pitch", C.c_int64),
                ("W", C.c_int32), ("H", C.c_int32), ("rig_index", C.c_int32),
                ("alpha", C.c_float), ("beta", C.c_float), ("pair", C.POINTER(RefPair))]


class RefTex(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("rgb_pitch", C.c_int64),
                ("depth", C.c_void_p), ("depth_pitch", C.c_int64),
                ("W", C.c_int32), ("H", C.c_int32),
                ("alpha", C.c_float), ("beta", C.c_float),
                ("pair", C.POINTER(RefPair)), ("weight", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.fvv_ref_select.restype = C.c_int32
        L.fvv_ref_select.argtypes = [C.POINTER(RefCamera), P, C.c_int32, C.POINTER(RefCamera),
                                     C.c_int32, P, P]
        L.fvv_ref_pair.restype = None
        L.fvv_ref_pair.argtypes = [C.POINTER(RefCamera), C.POINTER(RefCamera), C.POINTER(RefPair)]
        L.fvv_ref_decode_depth.restype = C.c_float
        L.fvv_ref_decode_depth.argtypes = [C.c_uint16, C.c_float, C.c_float]
        L.fvv_ref_splat.restype = None
        L.fvv_ref_splat.argtypes = [C.POINTER(RefSrc), C.c_int32, C.c_int32, C.c_int32, C.c_float, P]
        L.fvv_ref_filter.restype = None
        L.fvv_ref_filter.argtypes = [P, C.c_int32, C.c_int32, C.c_float, P]
        L.fvv_ref_blend.restype = None
        L.fvv_ref_blend.argtypes = [P, C.c_int32, C.c_int32, C.POINTER(RefTex), C.c_int32, C.c_float,
                                    P, P, P]
        L.fvv_ref_stack.restype = None
        L.fvv_ref_stack.argtypes = [P, C.c_int32, C.c_int32, C.POINTER(RefTex), C.c_int32, C.c_float, P]
        L.fvv_ref_depth_code.restype = C.c_uint16
        L.fvv_ref_depth_code.argtypes = [C.c_uint16, C.c_float, C.c_float]
        L.fvv_ref_code_depth.restype = C.c_uint16
        L.fvv_ref_code_depth.argtypes = [C.c_uint16, C.c_float, C.c_float]
        L.fvv_ref_depth_codes.restype = None
        L.fvv_ref_depth_codes.argtypes = [P, C.c_int64, C.c_int32, C.c_int32, C.c_float, C.c_float, P]
        L.fvv_ref_codes_depth.restype = None
        L.fvv_ref_codes_depth.argtypes = [P, C.c_int32, C.c_int32, C.c_float, C.c_float, P]
        L.fvv_ref_tx_cameras.restype = C.c_int32
        L.fvv_ref_tx_cameras.argtypes = [P, C.c_int32, P, C.c_int32, C.c_int32, P]
        L.fvv_ref_decode_plane.restype = None
        L.fvv_ref_decode_plane.argtypes = [P, C.c_int64, C.c_float, C.c_float, P]
        L.fvv_ref_prefilter.restype = None
        L.fvv_ref_prefilter.argtypes = [P, C.c_int64, P, C.c_int64, C.c_int32, C.c_int32, C.c_int32,
                                        C.c_float, C.c_float, C.c_int32, P]
        L.fvv_ref_pack_y12.restype = None
        L.fvv_ref_pack_y12.argtypes = [P, C.c_int32, C.c_int32, P, P, P]
        L.fvv_ref_unpack_y12.restype = None
        L.fvv_ref_unpack_y12.argtypes = [P, P, P, C.c_int32, C.c_int32, P]
        L.fvv_ref_fill.restype = None
        L.fvv_ref_fill.argtypes = [P, P, P, C.c_int32, C.c_int32, C.c_int32, P]
        L.fvv_ref_synthesize.restype = C.c_int32
        L.fvv_ref_synthesize.argtypes = [C.POINTER(RefCamera), C.c_int32, P, P, P, P,
                                         C.POINTER(RefCamera), C.c_int32, C.c_float, C.c_float,
                                         C.c_int32, P, P, P, P, P, P, P, P]
        L.fvv_ref_synthesize_views.restype = C.c_int32
        L.fvv_ref_synthesize_views.argtypes = [C.POINTER(RefCamera), C.c_int32, P, P, P, P,
                                               C.POINTER(RefCamera), C.c_int32, C.c_int32, C.c_float,
                                               C.c_float, C.c_int32, P, C.c_int32]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def ref_camera(cam) -> RefCamera:
    w, h, fx, fy, cx, cy, R, t, al, be = cam.as_tuple()
    return RefCamera(w, h, fx, fy, cx, cy, (C.c_float * 9)(*R), (C.c_float * 3)(*t), al, be)


# ---------------------------------------------------------------- O1 / O2 / O3
def select(rig: Sequence, virt, k: int, present: Optional[Sequence[bool]] = None):
    """O1: (selected rig indices, double weights)."""
    n = len(rig)
    arr = (RefCamera * n)(*[ref_camera(c) for c in rig])
    pres = None if present is None else np.asarray(present, np.int32)
    idx = np.zeros(8, np.int32)
    w = np.zeros(8, np.float64)
    K = lib().fvv_ref_select(arr, _ptr(pres), n, C.byref(ref_camera(virt)), k, _ptr(idx), _ptr(w))
    return idx[:K].copy(), w[:K].copy()


def pair(src, virt) -> RefPair:
    """O2: float32 pair matrices for (source, virtual)."""
    p = RefPair()
    lib().fvv_ref_pair(C.byref(ref_camera(src)), C.byref(ref_camera(virt)), C.byref(p))
    return p


def pair_arrays(src, virt):
    p = pair(src, virt)
    return dict(A=np.array(p.A, np.float32).reshape(3, 3), a=np.array(p.a, np.float32),
                B=np.array(p.B, np.float32).reshape(3, 3), b=np.array(p.b, np.float32),
                sx=np.float32(p.sx), sy=np.float32(p.sy))


def decode_depth(d: int, alpha: float = 0.0, beta: float = 1.0) -> np.float32:
    """O3 for one code."""
    return np.float32(lib().fvv_ref_decode_depth(int(d), alpha, beta))


# ---------------------------------------------------------------- O4 .. O7
def splat(rig, depths, virt, sel, max_fp: float = 4.0) -> np.ndarray:
    """O4: raw key map (H, W) uint64 from the selected cameras ``sel``."""
    pairs = [pair(rig[c], virt) for c in sel]
    depths = [np.ascontiguousarray(d, np.uint16) for d in depths]
    srcs = (RefSrc * len(sel))()
    for k, c in enumerate(sel):
        d = depths[c]
        srcs[k] = RefSrc(_ptr(d), d.shape[1], d.shape[1], d.shape[0], int(c),
                         rig[c].depth_alpha, rig[c].depth_beta, C.pointer(pairs[k]))
    Z = np.empty((virt.height, virt.width), np.uint64)
    lib().fvv_ref_splat(srcs, len(sel), virt.width, virt.height, max_fp, _ptr(Z))
    return Z


def depth_filter(Z: np.ndarray, tau: float = 0.05) -> np.ndarray:
    """O5: filtered key map."""
    Z = np.ascontiguousarray(Z, np.uint64)
    Zf = np.empty_like(Z)
    lib().fvv_ref_filter(_ptr(Z), Z.shape[1], Z.shape[0], tau, _ptr(Zf))
    return Zf


def blend(Zf, rig, frames, virt, sel, weights, tau: float = 0.05):
    """O6: (rgb (H,W,3) uint8, hole (H,W) uint8, depth (H,W) float32)."""
    Zf = np.ascontiguousarray(Zf, np.uint64)
    pairs = [pair(rig[c], virt) for c in sel]
    keep = []
    texs = (RefTex * len(sel))()
    for k, c in enumerate(sel):
        rgb = np.ascontiguousarray(frames[c].rgb, np.uint8)
        dep = np.ascontiguousarray(frames[c].depth_mm, np.uint16)
        keep += [rgb, dep]
        texs[k] = RefTex(_ptr(rgb), rgb.shape[1] * 3, _ptr(dep), dep.shape[1],
                         dep.shape[1], dep.shape[0], rig[c].depth_alpha, rig[c].depth_beta,
                         C.pointer(pairs[k]), float(weights[k]))
    H, W = Zf.shape
    rgb = np.empty((H, W, 3), np.uint8)
    hole = np.empty((H, W), np.uint8)
    dep = np.empty((H, W), np.float32)
    lib().fvv_ref_blend(_ptr(Zf), W, H, texs, len(sel), tau, _ptr(rgb), _ptr(hole), _ptr(dep))
    return rgb, hole, dep


def _texs(rig, frames, virt, sel, weights):
    pairs = [pair(rig[c], virt) for c in sel]
    keep = [pairs]
    texs = (RefTex * max(1, len(sel)))()
    for k, c in enumerate(sel):
        rgb = np.ascontiguousarray(frames[c].rgb, np.uint8)
        dep = np.ascontiguousarray(frames[c].depth_mm, np.uint16)
        keep += [rgb, dep]
        texs[k] = RefTex(_ptr(rgb), rgb.shape[1] * 3, _ptr(dep), dep.shape[1],
                         dep.shape[1], dep.shape[0], rig[c].depth_alpha, rig[c].depth_beta,
                         C.pointer(pairs[k]), float(weights[k]))
    return texs, keep


def stack(Zf, rig, frames, virt, sel, weights, tau: float = 0.05, pad_rows: int = 0,
          pad_cols: int = 0) -> np.ndarray:
    """O6': network input, float64 (H + pad_rows, W + pad_cols, 16): 15
    per-camera channels (R, G, B, inverse depth, validity for up to three
    cameras in selection order) and a zero channel; padding is zero.  Values
    are not rounded; the network rounds them to bfloat16."""
    Zf = np.ascontiguousarray(Zf, np.uint64)
    H, W = Zf.shape
    texs, keep = _texs(rig, frames, virt, sel, weights)
    st = np.zeros((H, W, 15), np.float64)
    lib().fvv_ref_stack(_ptr(Zf), W, H, texs, len(sel), tau, _ptr(st))
    out = np.zeros((H + pad_rows, W + pad_cols, 16), np.float64)
    out[:H, :W, :15] = st
    return out


def synthesize_learned(rig, frames, virt, net_params, k_nearest: int = 3, tau: float = 0.05,
                       max_fp: float = 4.0, widths=None):
    """Learned path for one view: O1..O5, the O6' stack on the padded grid
    (multiples of 8), the network (oracle.unet, bfloat16 points as on the
    device), RGB8 of the image area.  Returns (rgb, s, stack)."""
    from . import unet
    r = synthesize(rig, frames, virt, k_nearest=k_nearest, tau=tau, max_fp=max_fp, taps=True)
    H, W = virt.height, virt.width
    Hp, Wp = -(-H // 8) * 8, -(-W // 8) * 8
    st = stack(r["zf"], rig, frames, virt, r["sel"], r["weights"], tau, Hp - H, Wp - W)
    s, _ = unet.forward(net_params, st, widths or unet.WIDTHS)
    return unet.to_rgb8(s)[:H, :W], s, st


def fill(rgb, hole, depth, mode: int = 0) -> np.ndarray:
    """O7: final RGB (H,W,3)."""
    rgb = np.ascontiguousarray(rgb, np.uint8)
    hole = np.ascontiguousarray(hole, np.uint8)
    depth = np.ascontiguousarray(depth, np.float32)
    out = np.empty_like(rgb)
    lib().fvv_ref_fill(_ptr(rgb), _ptr(hole), _ptr(depth), rgb.shape[1], rgb.shape[0], mode,
                       _ptr(out))
    return out


def synthesize(rig, frames, virt, k_nearest: int = 3, tau: float = 0.05, max_fp: float = 4.0,
               fill_mode: int = 0, taps: bool = False):
    """O1..O7 for one virtual camera.  ``frames[c]`` may be None (absent).
    Returns a dict with 'rgb' and, if ``taps``, the per-stage maps."""
    n = len(rig)
    cams = (RefCamera * n)(*[ref_camera(c) for c in rig])
    rgbs, deps = [], []
    for f in frames:
        rgbs.append(None if f is None else np.ascontiguousarray(f.rgb, np.uint8))
        deps.append(None if f is None else np.ascontiguousarray(f.depth_mm, np.uint16))
    prgb = (C.c_void_p * n)(*[None if a is None else a.ctypes.data for a in rgbs])
    pdep = (C.c_void_p * n)(*[None if a is None else a.ctypes.data for a in deps])
    rp = np.array([0 if a is None else a.shape[1] * 3 for a in rgbs], np.int64)
    dp = np.array([0 if a is None else a.shape[1] for a in deps], np.int64)
    H, W = virt.height, virt.width
    out = np.empty((H, W, 3), np.uint8)
    t = {}
    if taps:
        t = dict(z=np.empty((H, W), np.uint64), zf=np.empty((H, W), np.uint64),
                 blend_rgb=np.empty((H, W, 3), np.uint8), hole=np.empty((H, W), np.uint8),
                 depth=np.empty((H, W), np.float32))
    sel = np.zeros(8, np.int32)
    w = np.zeros(8, np.float64)
    K = lib().fvv_ref_synthesize(cams, n, C.cast(prgb, C.c_void_p), _ptr(rp),
                                 C.cast(pdep, C.c_void_p), _ptr(dp),
                                 C.byref(ref_camera(virt)), k_nearest, tau, max_fp, fill_mode,
                                 _ptr(out), _ptr(t.get("z")), _ptr(t.get("zf")),
                                 _ptr(t.get("blend_rgb")), _ptr(t.get("hole")),
                                 _ptr(t.get("depth")), _ptr(sel), _ptr(w))
    if K < 0:
        raise ValueError("oracle rejected the arguments")
    res = dict(rgb=out, sel=sel[:K].copy(), weights=w[:K].copy())
    res.update(t)
    return res


def synthesize_views(rig, frames, virts, threads: int, k_nearest: int = 3, tau: float = 0.05,
                     max_fp: float = 4.0, fill_mode: int = 0):
    """Timing mode: O1..O7 for many virtual cameras of one frame set on
    `threads` OpenMP threads (one view per thread at a time); each view's
    RGB8 equals :func:`synthesize` of that view alone."""
    n = len(rig)
    cams = (RefCamera * n)(*[ref_camera(c) for c in rig])
    rgbs = [None if f is None else np.ascontiguousarray(f.rgb, np.uint8) for f in frames]
    deps = [None if f is None else np.ascontiguousarray(f.depth_mm, np.uint16) for f in frames]
    prgb = (C.c_void_p * n)(*[None if a is None else a.ctypes.data for a in rgbs])
    pdep = (C.c_void_p * n)(*[None if a is None else a.ctypes.data for a in deps])
    rp = np.array([0 if a is None else a.shape[1] * 3 for a in rgbs], np.int64)
    dp = np.array([0 if a is None else a.shape[1] for a in deps], np.int64)
    nv = len(virts)
    va = (RefCamera * nv)(*[ref_camera(v) for v in virts])
    outs = [np.empty((v.height, v.width, 3), np.uint8) for v in virts]
    po = (C.c_void_p * nv)(*[o.ctypes.data for o in outs])
    bad = lib().fvv_ref_synthesize_views(cams, n, C.cast(prgb, C.c_void_p), _ptr(rp), C.cast(pdep, C.c_void_p),
                                         _ptr(dp), va, nv, k_nearest, tau, max_fp, fill_mode,
                                         C.cast(po, C.c_void_p), threads)
    if bad:
        raise ValueError("oracle rejected the arguments of some views")
    return outs


def tx_cameras(rig, viewpoints, n_tx: int = 5):
    """OT: bit mask of the cameras to transmit for these client viewpoints."""
    n = len(rig)
    arr = (RefCamera * n)(*[ref_camera(c) for c in rig])
    nv = len(viewpoints)
    va = (RefCamera * max(nv, 1))(*[ref_camera(v) for v in viewpoints])
    mask = C.c_uint32(0)
    cnt = lib().fvv_ref_tx_cameras(C.cast(arr, C.c_void_p), n, C.cast(va, C.c_void_p), nv, n_tx, C.byref(mask))
    if cnt < 0:
        raise ValueError("oracle rejected the arguments")
    return mask.value


def decode_plane_bits(depth_mm, alpha: float = 0.0, beta: float = 1.0) -> np.ndarray:
    """O3 over a millimetre map: uint32 float32 bits, 0xFFFFFFFF = no depth."""
    d = np.ascontiguousarray(depth_mm, np.uint16)
    out = np.empty(d.shape, np.uint32)
    lib().fvv_ref_decode_plane(_ptr(d), d.size, alpha, beta, _ptr(out))
    return out


class _LayerFrame:
    def __init__(self, rgb, depth_mm):
        self.rgb = rgb
        self.depth_mm = depth_mm


# ---------------------------------------------------------------- OJ: joint bilateral pre-filter
JBF_DEFAULTS = dict(radius=2, sigma_s=1.5, sigma_c=24.0, min_valid=5)


def prefilter(rgb, depth_mm, radius: int = 2, sigma_s: float = 1.5, sigma_c: float = 24.0,
              min_valid: int = 5) -> np.ndarray:
    """Hole-filling joint bilateral filter of one live depth map (readings in
    the C source)."""
    rgb = np.ascontiguousarray(rgb, np.uint8)
    d = np.ascontiguousarray(depth_mm, np.uint16)
    H, W = d.shape
    out = np.empty((H, W), np.uint16)
    lib().fvv_ref_prefilter(_ptr(rgb), W * 3, _ptr(d), W, W, H, radius, sigma_s, sigma_c, min_valid, _ptr(out))
    return out


def prefilter_frames(frames, **kw):
    return [None if f is None else _LayerFrame(f.rgb, prefilter(f.rgb, f.depth_mm, **kw)) for f in frames]


# ---------------------------------------------------------------- OL: layered synthesis
BG_MM = 0xFFFF      # background signal in live millimetre maps (O3)


class _IdentityDepthCamera:
    """A rig camera whose Eq. 1 correction is the identity (0, 1)."""
    def __init__(self, cam):
        self._t = cam.as_tuple()[:8] + (0.0, 1.0)

    def as_tuple(self):
        return self._t


def layer_frames(rig, frames, bg_models):
    """Per-camera contributions to the two layers (Section VI, the per-camera
    process): the foreground keeps the live colour and live depth where the
    depth is not the background signal; the background keeps the live colour
    with the background model's depth where the live depth is the background
    signal.  The background model is calibration geometry, so the Eq. 1
    correction of the live stereo depth is not applied to it (reading).
    Returns (fg_frames, bg_rig, bg_frames)."""
    fg, bg = [], []
    for f, m in zip(frames, bg_models):
        if f is None:
            fg.append(None)
            bg.append(None)
            continue
        d = np.asarray(f.depth_mm, np.uint16)
        is_bg = d == BG_MM
        fg.append(_LayerFrame(f.rgb, np.where(is_bg, 0, d).astype(np.uint16)))
        bgd = np.zeros_like(d) if m is None else np.where(is_bg, np.asarray(m, np.uint16), 0).astype(np.uint16)
        bg.append(_LayerFrame(f.rgb, bgd))
    return fg, [_IdentityDepthCamera(c) for c in rig], bg


def synthesize_layered(rig, frames, bg_models, virt, k_nearest: int = 3, tau: float = 0.05,
                       max_fp: float = 4.0, fill_mode: int = 0):
    """Layered FG/BG synthesis (Section VI): each layer is warped, filtered
    and mixed over the same selected cameras by their distance weights (O1-O6
    on that layer's frames), the foreground layer is stacked over the
    background layer wherever it has a blended colour, and the hole fill (O7)
    runs on the composite.  Returns a dict with 'rgb', the composite 'hole',
    'depth' and 'blend_rgb', and each layer's taps under 'fg' and 'bg'."""
    fg_frames, bg_rig, bg_frames = layer_frames(rig, frames, bg_models)
    rf = synthesize(rig, fg_frames, virt, k_nearest=k_nearest, tau=tau, max_fp=max_fp, fill_mode=1, taps=True)
    rb = synthesize(bg_rig, bg_frames, virt, k_nearest=k_nearest, tau=tau, max_fp=max_fp, fill_mode=1, taps=True)
    fg_on = rf["hole"] == 0
    comp = np.where(fg_on[..., None], rf["blend_rgb"], rb["blend_rgb"]).astype(np.uint8)
    hole = (~fg_on & (rb["hole"] != 0)).astype(np.uint8)
    depth = np.where(fg_on, rf["depth"], rb["depth"]).astype(np.float32)
    comp[hole == 1] = 0
    depth[hole == 1] = 0
    return dict(rgb=fill(comp, hole, depth, fill_mode), hole=hole, depth=depth, blend_rgb=comp, fg=rf, bg=rb,
                sel=rf["sel"], weights=rf["weights"])


def key_depth(Z: np.ndarray) -> np.ndarray:
    """float32 depth held in the upper half of each key (garbage for EMPTY)."""
    return (Z >> np.uint64(32)).astype(np.uint32).view(np.float32)


def key_cam(Z: np.ndarray) -> np.ndarray:
    return ((Z >> np.uint64(27)) & np.uint64(31)).astype(np.int32)


def key_pixel(Z: np.ndarray) -> np.ndarray:
    return (Z & np.uint64((1 << 27) - 1)).astype(np.int64)


# ---------------------------------------------------------------- OC: depth codec
# Section V-A: 12-bit quantisation (Eq. 2) and the bit re-arrangement onto an
# 8-bit I420 image (Eq. 3 plus the U/V interleave); the C functions carry the
# readings.
def depth_codes(depth_mm: np.ndarray, z_near: float, z_far: float) -> np.ndarray:
    """Eq. 2 quantisation of a millimetre depth map to 12-bit codes (1 = none)."""
    d = np.ascontiguousarray(depth_mm, np.uint16)
    H, W = d.shape
    out = np.empty((H, W), np.uint16)
    lib().fvv_ref_depth_codes(_ptr(d), W, W, H, z_near, z_far, _ptr(out))
    return out


def codes_depth(codes: np.ndarray, z_near: float, z_far: float) -> np.ndarray:
    """Inverse of Eq. 2 to whole millimetres (0 for codes 0 and 1)."""
    c = np.ascontiguousarray(codes, np.uint16)
    H, W = c.shape
    out = np.empty((H, W), np.uint16)
    lib().fvv_ref_codes_depth(_ptr(c), W, H, z_near, z_far, _ptr(out))
    return out


def pack_y12(codes: np.ndarray):
    """12-bit codes (H, W even) -> I420 planes (Y (H,W), U (H/2,W/2), V)."""
    c = np.ascontiguousarray(codes, np.uint16)
    H, W = c.shape
    assert H % 2 == 0 and W % 2 == 0
    Y = np.empty((H, W), np.uint8)
    U = np.empty((H // 2, W // 2), np.uint8)
    V = np.empty((H // 2, W // 2), np.uint8)
    lib().fvv_ref_pack_y12(_ptr(c), W, H, _ptr(Y), _ptr(U), _ptr(V))
    return Y, U, V


def unpack_y12(Y, U, V) -> np.ndarray:
    """I420 planes -> 12-bit codes."""
    Y = np.ascontiguousarray(Y, np.uint8)
    U = np.ascontiguousarray(U, np.uint8)
    V = np.ascontiguousarray(V, np.uint8)
    H, W = Y.shape
    assert U.shape == V.shape == (H // 2, W // 2)
    codes = np.empty((H, W), np.uint16)
    lib().fvv_ref_unpack_y12(_ptr(Y), _ptr(U), _ptr(V), W, H, _ptr(codes))
    return codes


def encode_depth_y12(depth_mm, z_near: float, z_far: float):
    """Capture side: millimetre depth -> I420 planes (Y, U, V)."""
    return pack_y12(depth_codes(depth_mm, z_near, z_far))


def decode_depth_y12(Y, U, V, z_near: float, z_far: float) -> np.ndarray:
    """Receiving side: I420 planes -> whole-millimetre depth (0 = none)."""
    return codes_depth(unpack_y12(Y, U, V), z_near, z_far)
