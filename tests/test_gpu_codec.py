"""GPU parity of the 12-bit depth coding (Section V-A) through the C ABI:
the encoder and decoder bit-exact against the oracle, and 12-bit coded
uploads rendering exactly what the oracle renders from the oracle's decoded
millimetres."""
import sys

import numpy as np
import pytest

import scenegen as sg

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fvv():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2007_00558_amd as m
    m.lib()
    return m


def i420(Y, U, V):
    H, W = Y.shape
    return np.concatenate([Y.reshape(-1), U.reshape(-1), V.reshape(-1)]).reshape(H * 3 // 2, W)


def noisy_depth(rng, H, W, lo=1, hi=12000, zero_frac=0.1):
    d = rng.integers(lo, hi, size=(H, W)).astype(np.uint16)
    d[rng.random((H, W)) < zero_frac] = 0
    return d


PLANES = [(1.5, 7.0), (0.5, 10.0), (0.3, 20.0)]


@pytest.mark.parametrize("zn,zf", PLANES)
@pytest.mark.parametrize("H,W", [(2, 2), (66, 130), (1080, 1920)])
def test_encode_bit_exact(fvv, oracle_lib, zn, zf, H, W):
    import torch
    say(f"[gpu] y12 encode {W}x{H} planes {zn}..{zf}")
    rng = np.random.default_rng(H * 7 + W)
    d = noisy_depth(rng, H, W)
    d[0, 0] = int(round(zn * 1000))
    d[-1, -1] = int(round(zf * 1000))
    dev = torch.from_numpy(d.view(np.int16)).cuda()
    out = fvv.depth_encode_y12(dev, zn, zf)
    torch.cuda.synchronize()
    want = i420(*oracle_lib.encode_depth_y12(d, zn, zf))
    got = out.cpu().numpy()
    assert np.array_equal(got, want), np.argwhere(got != want)[:5]


@pytest.mark.parametrize("zn,zf", PLANES)
@pytest.mark.parametrize("H,W", [(2, 2), (66, 130), (1080, 1920)])
def test_decode_bit_exact(fvv, oracle_lib, zn, zf, H, W):
    """Random I420 bytes reach every code, the reserved ones included."""
    import torch
    say(f"[gpu] y12 decode {W}x{H} planes {zn}..{zf}")
    rng = np.random.default_rng(H * 11 + W)
    img = rng.integers(0, 256, size=(H * 3 // 2, W), dtype=np.uint8)
    out = fvv.depth_decode_y12(torch.from_numpy(img).cuda(), W, H, zn, zf)
    torch.cuda.synchronize()
    Y = img[:H]
    uv = img[H:].reshape(-1)
    U = uv[:H * W // 4].reshape(H // 2, W // 2)
    V = uv[H * W // 4:].reshape(H // 2, W // 2)
    want = oracle_lib.decode_depth_y12(Y, U, V, zn, zf)
    got = out.cpu().numpy().view(np.uint16)
    assert np.array_equal(got, want), np.argwhere(got != want)[:5]


@pytest.mark.parametrize("n", [1, 3, 9])
def test_batch_bit_exact(fvv, oracle_lib, n):
    """Batched coding of n equal-sized maps, some of them views with padded
    rows, against the oracle image by image; the batched decoder returns
    what the oracle decodes."""
    import torch
    H, W = 66, 130
    zn, zf = 0.5, 10.0
    say(f"[gpu] y12 batch n={n} {W}x{H}")
    rng = np.random.default_rng(100 + n)
    maps = [noisy_depth(rng, H, W) for _ in range(n)]
    devs = []
    for i, d in enumerate(maps):
        if i % 2:
            big = torch.zeros((H, W + 6), dtype=torch.int16, device="cuda")
            big[:, :W] = torch.from_numpy(d.view(np.int16)).cuda()
            devs.append(big[:, :W])
        else:
            devs.append(torch.from_numpy(d.view(np.int16)).cuda())
    outs = [torch.full((H * 3 // 2, W + 2 * (i % 3)), 7, dtype=torch.uint8, device="cuda")[:, :W]
            for i in range(n)]
    fvv.depth_encode_y12_batch(devs, zn, zf, outs=outs)
    torch.cuda.synchronize()
    for i, d in enumerate(maps):
        Y, U, V = oracle_lib.encode_depth_y12(d, zn, zf)
        o = outs[i]
        p = o.stride(0)
        flat = o.contiguous().cpu().numpy()
        base = torch.as_strided(o, (H * 3 // 2 * p,), (1,)).cpu().numpy() if p != W else flat.reshape(-1)
        got_y = base[:H * p].reshape(H, p)[:, :W]
        got_u = base[H * p:H * p + (H // 2) * (p // 2)].reshape(H // 2, p // 2)[:, :W // 2]
        got_v = base[H * p + (H // 2) * (p // 2):H * p + H * (p // 2)].reshape(H // 2, p // 2)[:, :W // 2]
        assert np.array_equal(got_y, Y) and np.array_equal(got_u, U) and np.array_equal(got_v, V), i
    imgs = [torch.from_numpy(rng.integers(0, 256, size=(H * 3 // 2, W), dtype=np.uint8)).cuda() for _ in range(n)]
    back = fvv.depth_decode_y12_batch(imgs, W, H, zn, zf)
    torch.cuda.synchronize()
    for img, b in zip(imgs, back):
        a = img.cpu().numpy()
        uv = a[H:].reshape(-1)
        want = oracle_lib.decode_depth_y12(a[:H], uv[:H * W // 4].reshape(H // 2, W // 2),
                                           uv[H * W // 4:].reshape(H // 2, W // 2), zn, zf)
        assert np.array_equal(b.cpu().numpy().view(np.uint16), want)


def test_every_code_round_trips_on_device(fvv, oracle_lib):
    """All 4096 codes through the oracle's packing, the device decoder and
    the device encoder: the bit re-arrangement is lossless and the
    quantiser's inverse agrees with the oracle's."""
    import torch
    zn, zf = 0.3, 20.0
    codes = np.random.default_rng(5).permutation(4096).astype(np.uint16).reshape(64, 64)
    img = i420(*oracle_lib.pack_y12(codes))
    mm = fvv.depth_decode_y12(torch.from_numpy(img).cuda(), 64, 64, zn, zf)
    re = fvv.depth_encode_y12(mm, zn, zf)
    torch.cuda.synchronize()
    mm_h = mm.cpu().numpy().view(np.uint16)
    assert np.array_equal(mm_h, oracle_lib.codes_depth(codes, zn, zf))
    assert np.array_equal(re.cpu().numpy(), i420(*oracle_lib.encode_depth_y12(mm_h, zn, zf)))


def test_pitched_buffers(fvv, oracle_lib):
    import torch
    zn, zf = 0.5, 10.0
    H, W = 34, 70
    d = noisy_depth(np.random.default_rng(9), H, W)
    big = torch.zeros((H, W + 9), dtype=torch.int16, device="cuda")
    big[:, :W] = torch.from_numpy(d.view(np.int16))
    src = big[:, :W]                                   # depth rows of (W + 9) * 2 bytes
    yuv = torch.full((H * 3 // 2, W + 6), 77, dtype=torch.uint8, device="cuda")   # luma pitch W + 6
    fvv.depth_encode_y12(src, zn, zf, out=yuv)
    torch.cuda.synchronize()
    Y, U, V = oracle_lib.encode_depth_y12(d, zn, zf)
    flat = yuv.cpu().numpy().reshape(-1)
    P = W + 6
    assert np.array_equal(flat[:H * P].reshape(H, P)[:, :W], Y)
    uv = flat[H * P:]
    assert np.array_equal(uv[:(H // 2) * (P // 2)].reshape(H // 2, P // 2)[:, :W // 2], U)
    assert np.array_equal(uv[(H // 2) * (P // 2):2 * (H // 2) * (P // 2)].reshape(H // 2, P // 2)[:, :W // 2], V)
    back = torch.full((H, W + 3), -1, dtype=torch.int16, device="cuda")
    fvv.depth_decode_y12(yuv, W, H, zn, zf, out=back[:, :W])
    torch.cuda.synchronize()
    b = back.cpu().numpy()
    assert np.array_equal(b[:, :W].view(np.uint16), oracle_lib.decode_depth_y12(Y, U, V, zn, zf))
    assert np.all(b[:, W:] == -1)                      # nothing written past the row


def coded_frames(oracle_lib, w, zn, zf):
    coded, decoded = [], []
    for f in w.frames:
        Y, U, V = oracle_lib.encode_depth_y12(f.depth_mm, zn, zf)
        coded.append((f.rgb, i420(Y, U, V)))
        decoded.append(sg.Frame(f.rgb, oracle_lib.decode_depth_y12(Y, U, V, zn, zf)))
    return coded, decoded


@pytest.mark.parametrize("zn,zf", [(1.5, 7.0), (0.5, 10.0)])
def test_coded_upload_renders_like_decoded_millimetres(fvv, oracle_lib, zn, zf):
    """Host upload of coded frames == host upload of the oracle's decoded
    millimetres (every tap identical), and both match the oracle's
    rendering of those millimetres at the synthesis bar."""
    w = sg.config2(0)
    coded, decoded = coded_frames(oracle_lib, w, zn, zf)
    assert any(np.count_nonzero(f.depth_mm == 0) > np.count_nonzero(g.depth_mm == 0)
               for f, g in zip(decoded, w.frames)) == (zn > 1.0)
    v = w.virtual[0]
    H, W = v.height, v.width
    res = []
    for fmt, frames in ((fvv.DEPTH_Y12, coded), (fvv.DEPTH_MM16, decoded)):
        say(f"[gpu] c2 upload format {fmt} planes {zn}..{zf}")
        with fvv.Context(0) as c:
            c.set_rig(w.rig)
            c.set_depth_format(fmt, zn, zf)
            c.upload_mvd(frames)
            c.set_debug(True)
            out = c.synthesize(v)
            taps = [c.debug_read(t, (H, W)) for t in (fvv.TAP_Z_RAW, fvv.TAP_Z_FILT, fvv.TAP_BLEND, fvv.TAP_DEPTH)]
        res.append((out, taps))
    assert np.array_equal(res[0][0], res[1][0])
    for a, b in zip(res[0][1], res[1][1]):
        assert np.array_equal(a, b)
    r = oracle_lib.synthesize(w.rig, decoded, v, taps=True)
    assert np.array_equal(res[0][1][0], r["z"])
    assert np.array_equal(res[0][1][1], r["zf"])
    assert np.abs(res[0][0].astype(np.int16) - r["rgb"].astype(np.int16)).max() <= 1


def test_coded_device_upload_full_size(fvv, oracle_lib):
    """The full 9-camera 1280x720 rig: device encode of every camera, device
    upload of the I420 images, one 1920x1080 view against the oracle on the
    decoded millimetres."""
    import torch
    zn, zf = 1.5, 7.0
    say("[gpu] c3 coded upload")
    w = sg.config3(0, n_frames=2)
    frames, decoded = [], []
    for f in w.frames:
        rgb = torch.from_numpy(f.rgb).cuda()
        yuv = fvv.depth_encode_y12(torch.from_numpy(f.depth_mm.view(np.int16)).cuda(), zn, zf)
        frames.append((rgb, yuv))
    torch.cuda.synchronize()
    for (rgb, yuv), f in zip(frames, w.frames):
        H, W = f.depth_mm.shape
        img = yuv.cpu().numpy()
        Y, uv = img[:H], img[H:].reshape(-1)
        U, V = uv[:H * W // 4].reshape(H // 2, W // 2), uv[H * W // 4:].reshape(H // 2, W // 2)
        assert np.array_equal(img, i420(*oracle_lib.encode_depth_y12(f.depth_mm, zn, zf)))
        decoded.append(sg.Frame(f.rgb, oracle_lib.decode_depth_y12(Y, U, V, zn, zf)))
    with fvv.Context(0) as c:
        c.set_rig(w.rig)
        c.set_depth_format(fvv.DEPTH_Y12, zn, zf)
        c.upload_mvd(frames, mem=fvv.MEM_DEVICE)
        torch.cuda.synchronize()
        v = w.virtual[1]
        out = c.synthesize(v)
    r = oracle_lib.synthesize(w.rig, decoded, v)
    assert np.abs(out.astype(np.int16) - r["rgb"].astype(np.int16)).max() <= 1


def test_codec_errors(fvv):
    import torch
    d = torch.zeros((4, 6), dtype=torch.int16, device="cuda")
    y = torch.zeros((6, 6), dtype=torch.uint8, device="cuda")
    L = fvv.lib()
    s = fvv._stream_handle(None)
    p = y.data_ptr()
    assert L.fvv_depth_encode_y12(d.data_ptr(), 12, 5, 4, 0.5, 10.0, p, 6, s) == fvv.FVV_E_ARG    # odd width
    assert L.fvv_depth_encode_y12(d.data_ptr(), 12, 6, 3, 0.5, 10.0, p, 6, s) == fvv.FVV_E_ARG    # odd height
    assert L.fvv_depth_encode_y12(d.data_ptr(), 10, 6, 4, 0.5, 10.0, p, 6, s) == fvv.FVV_E_ARG    # short depth rows
    assert L.fvv_depth_encode_y12(d.data_ptr(), 12, 6, 4, 0.5, 10.0, p, 5, s) == fvv.FVV_E_ARG    # odd luma pitch
    assert L.fvv_depth_encode_y12(d.data_ptr(), 12, 6, 4, 10.0, 0.5, p, 6, s) == fvv.FVV_E_ARG    # planes swapped
    assert L.fvv_depth_encode_y12(d.data_ptr(), 12, 6, 4, 0.0, 1.0, p, 6, s) == fvv.FVV_E_ARG     # z_near 0
    assert L.fvv_depth_decode_y12(p, 6, 6, 4, 0.5, float("nan"), d.data_ptr(), 12, s) == fvv.FVV_E_ARG
    assert L.fvv_depth_decode_y12(None, 6, 6, 4, 0.5, 1.0, d.data_ptr(), 12, s) == fvv.FVV_E_ARG
    assert "even" in L.fvv_last_error(None).decode() or "null" in L.fvv_last_error(None).decode()
    with fvv.Context(0) as c:
        with pytest.raises(fvv.FvvError):
            c.set_depth_format(fvv.DEPTH_Y12, 2.0, 1.0)
        with pytest.raises(fvv.FvvError):
            c.set_depth_format(7, 0.5, 1.0)
        w = sg.config_small(0, w=95, h=64)                   # odd camera width
        c.set_rig(w.rig)
        c.set_depth_format(fvv.DEPTH_Y12, 0.5, 10.0)
        fr = [(f.rgb, np.zeros((96, 95), np.uint8)) for f in w.frames]
        with pytest.raises(fvv.FvvError, match="even"):
            c.upload_mvd(fr)
