"""Python binding of libfvv.so, the MI355X DIBR view-synthesis library.

Argument marshalling only: every step of the path runs in the library's HIP
kernels (see ``include/fvv.h`` for the ABI).  Device buffers and streams come
from PyTorch (``tensor.data_ptr()``, ``torch.cuda.current_stream()``); host
buffers may be numpy arrays.  The library must have been built in-tree
(``python -m paper_2007_00558_amd.build``); importing the binding without it
raises, there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libfvv.so")

FVV_OK, FVV_E_ARG, FVV_E_STATE, FVV_E_NOMEM, FVV_E_DEVICE, FVV_E_AGAIN, FVV_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
MEM_HOST, MEM_DEVICE = 0, 1
FILL_BG, FILL_NONE = 0, 1
PATH_PLAIN, PATH_LEARNED, PATH_LAYERED = 0, 1, 2
TAP_Z_RAW, TAP_Z_FILT, TAP_BLEND, TAP_DEPTH, TAP_BG_Z_RAW, TAP_BG_Z_FILT, TAP_TILES = 0, 1, 2, 3, 4, 5, 6
BG_MM = 0xFFFF          # background signal in millimetre depth maps
KEY_EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)

ERROR_NAMES = {0: "FVV_OK", -1: "FVV_E_ARG", -2: "FVV_E_STATE", -3: "FVV_E_NOMEM",
               -4: "FVV_E_DEVICE", -5: "FVV_E_AGAIN", -6: "FVV_E_UNSUPPORTED"}


class FvvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class Camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32),
                ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("R", C.c_float * 9), ("t", C.c_float * 3),
                ("depth_alpha", C.c_float), ("depth_beta", C.c_float)]


class View(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("rgb_pitch", C.c_int64),
                ("depth_mm", C.c_void_p), ("depth_pitch", C.c_int64)]


class SynthParams(C.Structure):
    _fields_ = [("k_nearest", C.c_int32), ("tau_rel", C.c_float), ("max_footprint", C.c_float),
                ("fill_mode", C.c_int32), ("path", C.c_int32), ("exclude_mask", C.c_uint32),
                ("frame_version", C.c_uint64)]


_lib = None


def lib():
    """Load libfvv.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2007_00558_amd.build` (no fallback path exists)")
        # PyTorch ships its own HIP runtime; loading torch first makes the
        # library bind to that same runtime (one HIP runtime per process,
        # so torch's device buffers and streams are valid for the library)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        P, I32, I64, U64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
        sig = {
            "fvv_abi_version": (I32, []),
            "fvv_create": (I32, [I32, U64, C.POINTER(P)]),
            "fvv_destroy": (None, [P]),
            "fvv_last_error": (C.c_char_p, [P]),
            "fvv_set_rig": (I32, [P, C.POINTER(Camera), I32]),
            "fvv_upload_mvd": (I32, [P, C.POINTER(View), I32, I32, P, C.POINTER(U64)]),
            "fvv_synthesize": (I32, [P, C.POINTER(Camera), C.POINTER(SynthParams), P, I64, I32, P]),
            "fvv_synthesize_batch": (I32, [P, C.POINTER(Camera), I32, C.POINTER(SynthParams), P, P, I32, P]),
            "fvv_synthesize_noalloc": (I32, [P, C.POINTER(Camera), C.POINTER(SynthParams), P, I64, P]),
            "fvv_select_cameras": (I32, [C.POINTER(Camera), P, I32, C.POINTER(Camera), I32, P, P]),
            "fvv_pair_matrices": (I32, [C.POINTER(Camera), C.POINTER(Camera), P]),
            "fvv_set_debug": (I32, [P, I32]),
            "fvv_set_debug_view": (I32, [P, I32]),
            "fvv_measure_peaks": (I32, [I32, P, I32]),
            "fvv_check_reciprocal": (I32, [I32, I32, I32, P]),
            "fvv_check_bf16": (I32, [I32, P]),
            "fvv_debug_read": (I32, [P, I32, P, I64]),
            "fvv_set_profiling": (I32, [P, I32]),
            "fvv_stage_count": (I32, []),
            "fvv_stage_name": (C.c_char_p, [I32]),
            "fvv_profile_read": (I32, [P, P, P, I32, I32]),
            "fvv_server_start": (I32, [P, I32, U64]),
            "fvv_server_stop": (I32, [P]),
            "fvv_server_pause": (I32, [P, I32]),
            "fvv_submit": (I32, [P, C.POINTER(Camera), C.POINTER(SynthParams), P, I64, C.POINTER(U64)]),
            "fvv_poll": (I32, [P, U64, C.POINTER(C.c_double)]),
            "fvv_server_stats": (I32, [P, P]),
            "fvv_net_param_count": (U64, []),
            "fvv_net_layer_info": (I32, [I32, P]),
            "fvv_net_layer_name": (C.c_char_p, [I32]),
            "fvv_net_load": (I32, [P, P, U64]),
            "fvv_net_read": (I32, [P, I32, P, U64]),
            "fvv_make_stack": (I32, [P, C.POINTER(Camera), I32, C.POINTER(SynthParams), P, P]),
            "fvv_net_forward": (I32, [P, P, I32, I32, I32, P, P]),
            "fvv_net_train_step": (I32, [P, P, P, I32, I32, I32, I32, C.c_float, I32, P, P]),
            "fvv_net_read_act": (I32, [P, I32, P, I64]),
            "fvv_net_device_bytes": (U64, [P]),
            "fvv_depth_encode_y12": (I32, [P, I64, I32, I32, C.c_float, C.c_float, P, I64, P]),
            "fvv_depth_decode_y12": (I32, [P, I64, I32, I32, C.c_float, C.c_float, P, I64, P]),
            "fvv_depth_encode_y12_batch": (I32, [I32, P, P, I32, I32, C.c_float, C.c_float, P, P, P]),
            "fvv_depth_decode_y12_batch": (I32, [I32, P, P, I32, I32, C.c_float, C.c_float, P, P, P]),
            "fvv_set_depth_format": (I32, [P, I32, C.c_float, C.c_float]),
            "fvv_set_bg_model": (I32, [P, P, P, I32, I32, P]),
            "fvv_set_prefilter": (I32, [P, I32, I32, C.c_float, C.c_float, I32]),
            "fvv_read_frame_depth": (I32, [P, I32, I32, U64, P, I64]),
            "fvv_tx_cameras": (I32, [C.POINTER(Camera), I32, C.POINTER(Camera), I32, I32, C.POINTER(C.c_uint32)]),
            "fvv_server_tx_cameras": (I32, [P, I32, C.c_double, C.POINTER(C.c_uint32)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


EXPORTED = ("fvv_abi_version", "fvv_create", "fvv_destroy", "fvv_last_error", "fvv_set_rig",
            "fvv_upload_mvd", "fvv_synthesize", "fvv_synthesize_batch", "fvv_select_cameras",
            "fvv_pair_matrices", "fvv_set_debug", "fvv_debug_read", "fvv_set_profiling",
            "fvv_stage_count", "fvv_stage_name", "fvv_profile_read", "fvv_server_start",
            "fvv_server_stop", "fvv_server_pause", "fvv_submit", "fvv_poll", "fvv_server_stats",
            "fvv_net_param_count", "fvv_net_layer_info", "fvv_net_layer_name", "fvv_net_load",
            "fvv_net_read", "fvv_make_stack", "fvv_net_forward", "fvv_net_train_step",
            "fvv_net_read_act", "fvv_net_device_bytes", "fvv_depth_encode_y12",
            "fvv_depth_decode_y12", "fvv_set_depth_format", "fvv_set_bg_model", "fvv_set_prefilter",
            "fvv_read_frame_depth", "fvv_tx_cameras", "fvv_server_tx_cameras",
            "fvv_depth_encode_y12_batch", "fvv_depth_decode_y12_batch", "fvv_synthesize_noalloc",
            "fvv_set_debug_view", "fvv_measure_peaks", "fvv_check_reciprocal",
            "fvv_check_bf16")
DEPTH_MM16, DEPTH_Y12 = 0, 1
NET_PARAMS, NET_GRADS = 0, 1
NET_ALIGN = 8           # network inputs: multiples of 8 in both dimensions
NET_IN = 16             # stack channels on the device (15 used, one zero channel)


def camera(cam) -> Camera:
    """Marshal a camera (any object with ``as_tuple()`` in boundary order, or a Camera)."""
    if isinstance(cam, Camera):
        return cam
    w, h, fx, fy, cx, cy, R, t, al, be = cam.as_tuple()
    return Camera(w, h, fx, fy, cx, cy, (C.c_float * 9)(*R), (C.c_float * 3)(*t), al, be)


def params(k_nearest=3, tau_rel=0.05, max_footprint=4.0, fill_mode=FILL_BG, path=PATH_PLAIN,
           frame_version=0, exclude=()) -> SynthParams:
    """Synthesis parameters; ``exclude`` lists rig cameras that may not be selected."""
    mask = 0
    for c in exclude:
        mask |= 1 << int(c)
    return SynthParams(k_nearest, tau_rel, max_footprint, fill_mode, path, mask, frame_version)


def net_layers():
    """[(name, kind, C_in, C_out, kernel)] of the learned-path network."""
    L = lib()
    out = []
    i = 0
    while True:
        name = L.fvv_net_layer_name(i)
        if name is None:
            return out
        a = np.zeros(4, np.int32)
        L.fvv_net_layer_info(i, a.ctypes.data)
        out.append((name.decode(), int(a[0]), int(a[1]), int(a[2]), int(a[3])))
        i += 1


def net_param_count() -> int:
    return int(lib().fvv_net_param_count())


def pad8(n: int) -> int:
    return (n + NET_ALIGN - 1) // NET_ALIGN * NET_ALIGN


def _addr(a) -> int:
    """Address of a numpy array or torch tensor."""
    if a is None:
        return 0
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _pitch(a, row_elems_bytes: int) -> int:
    if isinstance(a, np.ndarray):
        return a.strides[0]
    return a.stride(0) * a.element_size()


def _stream_handle(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def measure_peaks(device: int = 0) -> dict:
    """Measured HBM copy bandwidth and 64-bit atomicMin rates of the device."""
    out = np.zeros(5, np.float64)
    rc = lib().fvv_measure_peaks(device, out.ctypes.data, out.size)
    if rc < 0:
        raise FvvError(rc, lib().fvv_last_error(None).decode())
    return {"copy_GBs": float(out[0]), "global_atomic_min_distinct_per_s": float(out[1]),
            "global_atomic_min_wave_contended_per_s": float(out[2]),
            "lds_atomic_min_distinct_per_s": float(out[3]), "lds_atomic_min_window_per_s": float(out[4])}


def check_reciprocal(device: int = 0, e_lo: int = -7, e_hi: int = 20) -> int:
    """Mismatches of the kernels' reciprocal (and two quotients per divisor)
    against correctly rounded division over every significand of the
    binades 2^e_lo .. 2^e_hi, on the device."""
    bad = np.zeros(1, np.uint64)
    rc = lib().fvv_check_reciprocal(device, e_lo, e_hi, bad.ctypes.data)
    if rc < 0:
        raise FvvError(rc, lib().fvv_last_error(None).decode())
    return int(bad[0])


def check_bf16(device: int = 0) -> int:
    """Mismatches of the network kernels' bfloat16 rounding (hardware
    conversion) against round-to-nearest-even on the bits, over every
    non-NaN float32, on the device."""
    bad = np.zeros(1, np.uint64)
    rc = lib().fvv_check_bf16(device, bad.ctypes.data)
    if rc < 0:
        raise FvvError(rc, lib().fvv_last_error(None).decode())
    return int(bad[0])


def select_cameras(rig: Sequence, virt, k: int, present=None):
    """Host-only selection: (rig indices, float32 weights)."""
    n = len(rig)
    arr = (Camera * n)(*[camera(c) for c in rig])
    pres = None if present is None else np.ascontiguousarray(present, np.int32)
    idx = np.zeros(8, np.int32)
    w = np.zeros(8, np.float32)
    K = lib().fvv_select_cameras(arr, _addr(pres) or None, n, C.byref(camera(virt)), k,
                                 idx.ctypes.data, w.ctypes.data)
    if K < 0:
        raise FvvError(K, "fvv_select_cameras rejected its arguments")
    return idx[:K].copy(), w[:K].copy()


def tx_cameras(rig: Sequence, viewpoints: Sequence, n_tx: int = 5) -> int:
    """Bit mask of the cameras to transmit for these client viewpoints."""
    n, nv = len(rig), len(viewpoints)
    arr = (Camera * n)(*[camera(c) for c in rig])
    va = (Camera * max(nv, 1))(*[camera(v) for v in viewpoints])
    m = C.c_uint32(0)
    rc = lib().fvv_tx_cameras(arr, n, va, nv, n_tx, C.byref(m))
    if rc < 0:
        raise FvvError(rc, "fvv_tx_cameras rejected its arguments")
    return m.value


def pair_matrices(src, virt):
    out = np.zeros(26, np.float32)
    rc = lib().fvv_pair_matrices(C.byref(camera(src)), C.byref(camera(virt)), out.ctypes.data)
    if rc:
        raise FvvError(rc, "fvv_pair_matrices rejected its arguments")
    return dict(A=out[0:9].reshape(3, 3), a=out[9:12], B=out[12:21].reshape(3, 3), b=out[21:24],
                sx=out[24], sy=out[25])


def _codec_check(rc: int, what: str):
    if rc != FVV_OK:
        raise FvvError(rc, f"{what}: " + lib().fvv_last_error(None).decode())


def depth_encode_y12(depth, z_near: float, z_far: float, out=None, stream=None):
    """12-bit depth coding (Section V-A) of a device depth map (H, W) of
    2-byte millimetres into an I420 image; out (H*3/2, W) uint8 device tensor
    (a new one if None), rows of out.stride(0) bytes."""
    import torch
    H, W = depth.shape
    if out is None:
        out = torch.empty((H * 3 // 2, W), dtype=torch.uint8, device=depth.device)
    _codec_check(lib().fvv_depth_encode_y12(depth.data_ptr(), _pitch(depth, 0), W, H, z_near, z_far,
                                            out.data_ptr(), _pitch(out, 0), _stream_handle(stream)),
                 "fvv_depth_encode_y12")
    return out


def depth_decode_y12(yuv, width: int, height: int, z_near: float, z_far: float, out=None, stream=None):
    """Inverse of depth_encode_y12: I420 device image -> (H, W) int16 tensor
    holding the uint16 millimetres (0 = no depth)."""
    import torch
    if out is None:
        out = torch.empty((height, width), dtype=torch.int16, device=yuv.device)
    _codec_check(lib().fvv_depth_decode_y12(yuv.data_ptr(), _pitch(yuv, 0), width, height, z_near, z_far,
                                            out.data_ptr(), _pitch(out, 0), _stream_handle(stream)),
                 "fvv_depth_decode_y12")
    return out


def _y12_batch(fn, what, srcs, dsts, width, height, z_near, z_far, stream):
    n = len(srcs)
    if n != len(dsts):
        raise ValueError(f"{what}: {n} sources but {len(dsts)} destinations")
    ptr = C.c_void_p * max(n, 1)
    pit = C.c_int64 * max(n, 1)
    sp, spp = ptr(*[t.data_ptr() for t in srcs]), pit(*[_pitch(t, 0) for t in srcs])
    dp, dpp = ptr(*[t.data_ptr() for t in dsts]), pit(*[_pitch(t, 0) for t in dsts])
    _codec_check(fn(n, sp, spp, width, height, z_near, z_far, dp, dpp, _stream_handle(stream)), what)


def depth_encode_y12_batch(depths, z_near: float, z_far: float, outs=None, stream=None):
    """depth_encode_y12 of several equal-sized device depth maps in one
    launch; returns the list of I420 images."""
    import torch
    H, W = depths[0].shape
    if outs is None:
        outs = [torch.empty((H * 3 // 2, W), dtype=torch.uint8, device=d.device) for d in depths]
    _y12_batch(lib().fvv_depth_encode_y12_batch, "fvv_depth_encode_y12_batch", depths, outs, W, H,
               z_near, z_far, stream)
    return outs


def depth_decode_y12_batch(yuvs, width: int, height: int, z_near: float, z_far: float, outs=None, stream=None):
    """depth_decode_y12 of several equal-sized I420 device images in one
    launch; returns the list of (H, W) int16 depth maps."""
    import torch
    if outs is None:
        outs = [torch.empty((height, width), dtype=torch.int16, device=y.device) for y in yuvs]
    _y12_batch(lib().fvv_depth_decode_y12_batch, "fvv_depth_decode_y12_batch", yuvs, outs, width, height,
               z_near, z_far, stream)
    return outs


class Context:
    """One library context on one HIP device."""

    def __init__(self, device: int = 0, mem_budget: int = 0):
        self._L = lib()
        h = C.c_void_p()
        rc = self._L.fvv_create(device, mem_budget, C.byref(h))
        if rc:
            raise FvvError(rc, self._L.fvv_last_error(None).decode())
        self._h = h
        self.device = device
        self.rig = []
        self.depth_format = DEPTH_MM16

    def close(self):
        if getattr(self, "_h", None):
            self._L.fvv_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, rc: int):
        if rc != FVV_OK:
            raise FvvError(rc, self._L.fvv_last_error(self._h).decode())
        return rc

    def last_error(self) -> str:
        return self._L.fvv_last_error(self._h).decode()

    def set_rig(self, cams: Sequence):
        arr = (Camera * len(cams))(*[camera(c) for c in cams])
        self._check(self._L.fvv_set_rig(self._h, arr, len(cams)))
        self.rig = list(cams)

    def set_depth_format(self, fmt: int, z_near: float = 0.0, z_far: float = 0.0):
        """DEPTH_MM16 (uint16 millimetres) or DEPTH_Y12 (12-bit coded I420
        images, (H*3/2, W) uint8) for the following uploads."""
        self._check(self._L.fvv_set_depth_format(self._h, fmt, z_near, z_far))
        self.depth_format = fmt

    def set_prefilter(self, enable: bool = True, radius: int = 2, sigma_s: float = 1.5, sigma_c: float = 24.0,
                      min_valid: int = 5):
        """Hole-filling joint bilateral pre-filter of the live depth at ingest."""
        self._check(self._L.fvv_set_prefilter(self._h, 1 if enable else 0, radius, sigma_s, sigma_c, min_valid))

    def read_frame_depth(self, cam: int, layer: int = 0, version: int = 0) -> np.ndarray:
        """Decoded depth plane (float32 metres; NaN-pattern bits 0xFFFFFFFF = none)."""
        c = self.rig[cam]
        out = np.empty((c.height, c.width), np.float32)
        self._check(self._L.fvv_read_frame_depth(self._h, cam, layer, version, out.ctypes.data, out.nbytes))
        return out

    def set_bg_model(self, models: Optional[Sequence], mem: int = MEM_HOST, stream=None):
        """Background depth models (layered synthesis): models[c] a (H,W)
        uint16 millimetre map (numpy for MEM_HOST, torch CUDA tensor for
        MEM_DEVICE) or None; models=None clears them.  Drops resident frame
        sets."""
        if models is None:
            self._check(self._L.fvv_set_bg_model(self._h, None, None, 0, mem, None))
            return
        n = len(models)
        keep = []
        ptrs = (C.c_void_p * n)()
        pitches = np.zeros(n, np.int64)
        for k, m in enumerate(models):
            if m is None:
                continue
            if mem == MEM_HOST:
                m = np.ascontiguousarray(m, np.uint16)
            keep.append(m)
            ptrs[k] = _addr(m)
            pitches[k] = _pitch(m, 0)
        s = None if mem == MEM_HOST and stream is None else _stream_handle(stream)
        self._check(self._L.fvv_set_bg_model(self._h, ptrs, pitches.ctypes.data, n, mem, s))

    def upload_mvd(self, frames: Sequence, mem: int = MEM_HOST, stream=None) -> int:
        """frames[c] = (rgb (H,W,3) uint8, depth) -- numpy for MEM_HOST, torch
        CUDA tensors for MEM_DEVICE -- or None if absent.  depth is (H,W)
        uint16 millimetres, or the (H*3/2, W) uint8 I420 image in the 12-bit
        depth format."""
        n = len(frames)
        views = (View * n)()
        keep = []
        for k, f in enumerate(frames):
            if f is None:
                views[k] = View(None, 0, None, 0)
                continue
            rgb, dep = (f.rgb, f.depth_mm) if hasattr(f, "rgb") else f
            if mem == MEM_HOST:
                rgb = np.ascontiguousarray(rgb, np.uint8)
                dep = np.ascontiguousarray(dep, np.uint8 if self.depth_format == DEPTH_Y12 else np.uint16)
            keep += [rgb, dep]
            views[k] = View(_addr(rgb), _pitch(rgb, 0), _addr(dep), _pitch(dep, 0))
        ver = C.c_uint64(0)
        s = None if mem == MEM_HOST and stream is None else _stream_handle(stream)
        self._check(self._L.fvv_upload_mvd(self._h, views, n, mem, s, C.byref(ver)))
        return ver.value

    def synthesize(self, virt, out=None, p: Optional[SynthParams] = None, stream=None):
        """Render one view.  out=None -> new numpy (H,W,3) uint8 via host mode;
        a torch CUDA tensor -> device mode on ``stream`` (default: current)."""
        p = p or params()
        vc = camera(virt)
        if out is None:
            out = np.empty((vc.height, vc.width, 3), np.uint8)
        if isinstance(out, np.ndarray):
            assert out.flags.c_contiguous and out.dtype == np.uint8
            self._check(self._L.fvv_synthesize(self._h, C.byref(vc), C.byref(p), out.ctypes.data,
                                               out.strides[0], MEM_HOST, None))
        else:
            self._check(self._L.fvv_synthesize(self._h, C.byref(vc), C.byref(p), out.data_ptr(),
                                               out.stride(0), MEM_DEVICE, _stream_handle(stream)))
        return out

    def synthesize_noalloc(self, virt, out, p: Optional[SynthParams] = None, stream=None):
        """Render one view into the torch CUDA tensor ``out`` (H, W, 3) uint8
        without any allocation (the library's fixed per-GPU scratch)."""
        p = p or params()
        vc = camera(virt)
        self._check(self._L.fvv_synthesize_noalloc(self._h, C.byref(vc), C.byref(p), out.data_ptr(),
                                                   out.stride(0), _stream_handle(stream)))
        return out

    def synthesize_batch(self, virts: Sequence, outs: Sequence, p: Optional[SynthParams] = None,
                         stream=None):
        p = p or params()
        n = len(virts)
        arr = virts if isinstance(virts, C.Array) else (Camera * n)(*[camera(v) for v in virts])
        ptrs = (C.c_void_p * n)(*[_addr(o) for o in outs])
        dev = not isinstance(outs[0], np.ndarray)
        pitches = np.array([o.stride(0) if dev else o.strides[0] for o in outs], np.int64)
        s = _stream_handle(stream) if dev else None
        self._check(self._L.fvv_synthesize_batch(self._h, arr, n, C.byref(p), C.cast(ptrs, C.c_void_p),
                                                 pitches.ctypes.data, MEM_DEVICE if dev else MEM_HOST, s))
        return outs

    def set_debug(self, on: bool = True, view: int = 0):
        """Stage taps of the following syntheses, for view ``view`` of each call."""
        self._check(self._L.fvv_set_debug_view(self._h, view))
        self._check(self._L.fvv_set_debug(self._h, 1 if on else 0))

    def set_profiling(self, on: bool = True):
        self._check(self._L.fvv_set_profiling(self._h, 1 if on else 0))

    def profile(self, reset: bool = True) -> dict:
        """{stage name: (total kernel ms, launches)} since the last reset."""
        n = self._L.fvv_stage_count()
        ms = np.zeros(n, np.float64)
        cnt = np.zeros(n, np.int64)
        self._check(self._L.fvv_profile_read(self._h, ms.ctypes.data, cnt.ctypes.data, n, 1 if reset else 0))
        return {self._L.fvv_stage_name(k).decode(): (float(ms[k]), int(cnt[k])) for k in range(n)}

    # ---- learned path
    def net_load(self, flat: np.ndarray):
        flat = np.ascontiguousarray(flat, np.float32)
        self._check(self._L.fvv_net_load(self._h, flat.ctypes.data, flat.size))

    def net_read(self, what: int = NET_PARAMS) -> np.ndarray:
        a = np.empty(net_param_count(), np.float32)
        self._check(self._L.fvv_net_read(self._h, what, a.ctypes.data, a.size))
        return a

    def make_stack(self, virts: Sequence, ps: Sequence[SynthParams], stack, stream=None):
        """Stacks of views of one size into ``stack`` (torch bf16/int16 CUDA
        tensor of n * pad8(H) * pad8(W) * 32 elements)."""
        n = len(virts)
        arr = (Camera * n)(*[camera(v) for v in virts])
        parr = (SynthParams * n)(*ps)
        self._check(self._L.fvv_make_stack(self._h, arr, n, parr, stack.data_ptr(), _stream_handle(stream)))
        return stack

    def net_forward(self, stack, n: int, height: int, width: int, out, stream=None):
        self._check(self._L.fvv_net_forward(self._h, stack.data_ptr(), n, height, width, out.data_ptr(),
                                            _stream_handle(stream)))
        return out

    def net_train_step(self, stack, target, n: int, height: int, width: int, valid_rows: int,
                       lr: float = 1e-3, apply: bool = True, want_loss: bool = True, stream=None):
        loss = C.c_float(0.0)
        self._check(self._L.fvv_net_train_step(self._h, stack.data_ptr(), target.data_ptr(), n, height, width,
                                               valid_rows, lr, 1 if apply else 0,
                                               C.byref(loss) if want_loss else None, _stream_handle(stream)))
        return loss.value if want_loss else None

    def net_read_act(self, layer: int, shape) -> np.ndarray:
        """Layer output of the last forward as float32 (bf16 values), ``shape`` = (P, C)."""
        raw = np.empty(shape, np.uint16)
        self._check(self._L.fvv_net_read_act(self._h, layer, raw.ctypes.data, raw.nbytes))
        return (raw.astype(np.uint32) << 16).view(np.float32)

    def net_device_bytes(self) -> int:
        return int(self._L.fvv_net_device_bytes(self._h))

    def debug_read(self, tap: int, shape):
        dtype = {TAP_Z_RAW: np.uint64, TAP_Z_FILT: np.uint64, TAP_BLEND: np.uint32,
                 TAP_DEPTH: np.float32, TAP_BG_Z_RAW: np.uint64, TAP_BG_Z_FILT: np.uint64,
                 TAP_TILES: np.int32}[tap]
        a = np.empty(shape, dtype)
        self._check(self._L.fvv_debug_read(self._h, tap, a.ctypes.data, a.nbytes))
        return a


class Server:
    """Continuous-batching server of one context (see ``fvv_server_start``)."""

    def __init__(self, ctx: Context, max_slots: int = 64, step_bytes: int = 0):
        self.ctx = ctx
        ctx._check(ctx._L.fvv_server_start(ctx._h, max_slots, step_bytes))
        self.running = True

    def submit(self, virt, out, p: Optional[SynthParams] = None) -> int:
        """Queue one view into device tensor ``out`` (H, W, 3) uint8; returns a ticket."""
        p = p or params()
        t = C.c_uint64(0)
        rc = self.ctx._L.fvv_submit(self.ctx._h, C.byref(camera(virt)), C.byref(p), out.data_ptr(),
                                    out.stride(0), C.byref(t))
        if rc:
            raise FvvError(rc, self.ctx.last_error())
        return t.value

    def poll(self, ticket: int):
        """None while pending, else the latency in seconds (raises on failure)."""
        lat = C.c_double(0.0)
        rc = self.ctx._L.fvv_poll(self.ctx._h, ticket, C.byref(lat))
        if rc == FVV_E_AGAIN:
            return None
        if rc:
            raise FvvError(rc, f"request {ticket} failed")
        return lat.value

    def stats(self) -> dict:
        a = np.zeros(6, np.uint64)
        self.ctx._check(self.ctx._L.fvv_server_stats(self.ctx._h, a.ctypes.data))
        return dict(steps=int(a[0]), completed=int(a[1]), failed=int(a[2]), pixels=int(a[3]),
                    batch_sum=int(a[4]), busy_s=float(a[5]) * 1e-6)

    def pause(self, on: bool = True):
        self.ctx._check(self.ctx._L.fvv_server_pause(self.ctx._h, 1 if on else 0))

    def tx_cameras(self, n_tx: int = 5, window_s: float = 1.0) -> int:
        """Bit mask of the cameras the recent clients need (adaptive transmission)."""
        m = C.c_uint32(0)
        rc = self.ctx._L.fvv_server_tx_cameras(self.ctx._h, n_tx, window_s, C.byref(m))
        if rc < 0:
            self.ctx._check(rc)
        return m.value

    def stop(self):
        if self.running:
            self.ctx._check(self.ctx._L.fvv_server_stop(self.ctx._h))
            self.running = False
