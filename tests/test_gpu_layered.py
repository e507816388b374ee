"""GPU parity of the layered FG/BG synthesis (Section VI) through the C ABI
against the oracle: each layer's raw and filtered key maps bit-exact, the
composite's hole map and depth bit-exact, RGB within one level; batches,
parameters, coded uploads, serving and the full 9-camera rig."""
import sys

import numpy as np
import pytest

import scenegen as sg

pytestmark = pytest.mark.gpu
EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)


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


@pytest.fixture(scope="module")
def ctx(fvv):
    c = fvv.Context(0)
    yield c
    c.close()


def run_layered(fvv, ctx, w, v, frames=None, models=None, k=3, fill=0, max_fp=4.0, tau=0.05, upload=True):
    H, W = v.height, v.width
    if upload:
        ctx.set_rig(w.rig)
        ctx.set_bg_model(w.bg_models if models is None else models)
        ctx.upload_mvd(w.frames if frames is None else frames)
    ctx.set_debug(True)
    out = ctx.synthesize(v, p=fvv.params(k_nearest=k, fill_mode=fill, max_footprint=max_fp, tau_rel=tau,
                                         path=fvv.PATH_LAYERED))
    taps = {name: ctx.debug_read(t, (H, W)) for name, t in
            (("z", fvv.TAP_Z_RAW), ("zf", fvv.TAP_Z_FILT), ("bz", fvv.TAP_BG_Z_RAW), ("bzf", fvv.TAP_BG_Z_FILT),
             ("blend", fvv.TAP_BLEND), ("depth", fvv.TAP_DEPTH))}
    ctx.set_debug(False)
    return out, taps


def compare_layered(oracle, w, v, out, taps, frames=None, models=None, k=3, fill=0, max_fp=4.0, tau=0.05):
    r = oracle.synthesize_layered(w.rig, w.frames if frames is None else frames,
                                  w.bg_models if models is None else models, v, k_nearest=k, tau=tau,
                                  max_fp=max_fp, fill_mode=fill)
    assert np.array_equal(taps["z"], r["fg"]["z"]), "foreground raw key map differs"
    assert np.array_equal(taps["zf"], r["fg"]["zf"]), "foreground filtered key map differs"
    assert np.array_equal(taps["bz"], r["bg"]["z"]), "background raw key map differs"
    assert np.array_equal(taps["bzf"], r["bg"]["zf"]), "background filtered key map differs"
    hole = (taps["blend"] >> 24) == 0
    assert np.array_equal(hole, r["hole"] == 1), "composite hole map differs"
    assert np.array_equal(taps["depth"].view(np.uint32), r["depth"].view(np.uint32)), "composite depth differs"
    rgb = np.stack([(taps["blend"] >> s) & 0xFF for s in (0, 8, 16)], -1).astype(np.int16)
    d = np.abs(rgb - r["blend_rgb"].astype(np.int16))[~hole]
    assert d.size == 0 or d.max() <= 1, f"composite rgb max diff {d.max()}"
    dfin = np.abs(out.astype(np.int16) - r["rgb"].astype(np.int16))
    assert dfin.max() <= 1, f"final rgb max diff {dfin.max()}"
    return r


@pytest.mark.parametrize("seed", range(4))
def test_small_layered_parity(fvv, ctx, oracle_lib, seed):
    w = sg.config_small(seed, layered=True)
    for vi, v in enumerate(w.virtual):
        say(f"[gpu] layered small seed={seed} view={vi}")
        out, taps = run_layered(fvv, ctx, w, v, upload=vi == 0)
        r = compare_layered(oracle_lib, w, v, out, taps)
        assert (r["fg"]["hole"] == 0).sum() > 100 and (r["bg"]["hole"] == 0).sum() > 100


@pytest.mark.parametrize("k,fill,max_fp,tau", [(1, 0, 4.0, 0.05), (2, 1, 4.0, 0.05), (4, 0, 8.0, 0.05),
                                               (3, 0, 1.0, 0.01), (3, 1, 4.0, 0.3)])
def test_layered_parameter_variants(fvv, ctx, oracle_lib, k, fill, max_fp, tau):
    say(f"[gpu] layered variants k={k} fill={fill} fp={max_fp} tau={tau}")
    w = sg.config_small(5, n_cams=5, w=160, h=96, out_w=203, out_h=117, layered=True)
    v = w.virtual[1]
    out, taps = run_layered(fvv, ctx, w, v, k=k, fill=fill, max_fp=max_fp, tau=tau)
    compare_layered(oracle_lib, w, v, out, taps, k=k, fill=fill, max_fp=max_fp, tau=tau)


def test_missing_model_and_depth_correction(fvv, ctx, oracle_lib):
    """A camera without a model has an empty background layer; Eq. 1 bends
    the live foreground depth but not the models."""
    w = sg.config_small(6, layered=True)
    rig = [sg.Camera(c.width, c.height, c.fx, c.fy, c.cx, c.cy, c.R, c.t, 0.01, 0.98) for c in w.rig]
    w2 = sg.Workload(w.name, rig, w.frames, w.virtual, w.scene, bg_models=w.bg_models)
    models = [w.bg_models[0], None, w.bg_models[2]]
    for v in w.virtual:
        say("[gpu] layered, one camera without a model, Eq. 1 on")
        out, taps = run_layered(fvv, ctx, w2, v, models=models)
        compare_layered(oracle_lib, w2, v, out, taps, models=models)


def test_ragged_and_tiny_outputs(fvv, ctx, oracle_lib):
    w = sg.config_small(7, layered=True)
    ctx.set_rig(w.rig)
    ctx.set_bg_model(w.bg_models)
    ctx.upload_mvd(w.frames)
    for (H, W) in [(1, 1), (5, 77), (33, 33), (97, 130)]:
        v = w.virtual[1].with_size(W, H, W / w.virtual[1].width)
        say(f"[gpu] layered ragged {W}x{H}")
        out, taps = run_layered(fvv, ctx, w, v, upload=False)
        compare_layered(oracle_lib, w, v, out, taps)


def test_plain_path_on_layered_frames(fvv, ctx, oracle_lib):
    """The single-layer path reads the background signal as no depth."""
    w = sg.config_small(8, layered=True)
    ctx.set_rig(w.rig)
    ctx.set_bg_model(w.bg_models)
    ctx.upload_mvd(w.frames)
    v = w.virtual[0]
    out = ctx.synthesize(v)
    r = oracle_lib.synthesize(w.rig, w.frames, v)
    assert np.abs(out.astype(np.int16) - r["rgb"].astype(np.int16)).max() <= 1


def test_batch_device_and_device_models(fvv, ctx, oracle_lib):
    import torch
    w = sg.config_small(9, layered=True, n_virtual=5)
    ctx.set_rig(w.rig)
    ctx.set_bg_model([torch.from_numpy(m.view(np.int16)).cuda() for m in w.bg_models], mem=fvv.MEM_DEVICE)
    ctx.upload_mvd(w.frames)
    p = fvv.params(path=fvv.PATH_LAYERED)
    say("[gpu] layered batch of 5, device models")
    outs = [torch.empty((v.height, v.width, 3), dtype=torch.uint8, device="cuda") for v in w.virtual]
    ctx.synthesize_batch(w.virtual, outs, p=p)
    torch.cuda.synchronize()
    for v, o in zip(w.virtual, outs):
        single = ctx.synthesize(v, p=p)
        assert np.array_equal(o.cpu().numpy(), single)
        r = oracle_lib.synthesize_layered(w.rig, w.frames, w.bg_models, v)
        assert np.abs(single.astype(np.int16) - r["rgb"].astype(np.int16)).max() <= 1


def test_coded_upload_carries_the_background_signal(fvv, oracle_lib):
    """12-bit coded frames: code 0 is the background signal, so a coded
    upload renders the layered view of the decoded millimetres."""
    zn, zf = 1.0, 8.0
    w = sg.config_small(10, layered=True)
    coded, decoded = [], []
    for f in w.frames:
        Y, U, V = oracle_lib.encode_depth_y12(f.depth_mm, zn, zf)
        coded.append((f.rgb, np.concatenate([Y.reshape(-1), U.reshape(-1), V.reshape(-1)]).reshape(-1, Y.shape[1])))
        decoded.append(sg.Frame(f.rgb, oracle_lib.decode_depth_y12(Y, U, V, zn, zf)))
        assert np.array_equal(decoded[-1].depth_mm == sg.BG_MM, f.depth_mm == sg.BG_MM)
    p = fvv.params(path=fvv.PATH_LAYERED)
    with fvv.Context(0) as c:
        c.set_rig(w.rig)
        c.set_bg_model(w.bg_models)
        c.set_depth_format(fvv.DEPTH_Y12, zn, zf)
        c.upload_mvd(coded)
        for v in w.virtual:
            say("[gpu] layered from coded upload")
            out = c.synthesize(v, p=p)
            r = oracle_lib.synthesize_layered(w.rig, decoded, w.bg_models, v)
            assert np.abs(out.astype(np.int16) - r["rgb"].astype(np.int16)).max() <= 1


def test_layered_errors(fvv):
    w = sg.config_small(11, layered=True)
    with fvv.Context(0) as c:
        c.set_rig(w.rig)
        c.upload_mvd(w.frames)
        p = fvv.params(path=fvv.PATH_LAYERED)
        with pytest.raises(fvv.FvvError, match="background"):
            c.synthesize(w.virtual[0], p=p)                       # no models
        c.set_bg_model(w.bg_models)
        with pytest.raises(fvv.FvvError) as e:
            c.synthesize(w.virtual[0], p=p)                       # frames dropped by the models
        assert e.value.code == fvv.FVV_E_STATE
        c.upload_mvd(w.frames)
        c.synthesize(w.virtual[0], p=p)
        with pytest.raises(fvv.FvvError) as e:
            c.synthesize(w.virtual[0], p=fvv.params(path=fvv.PATH_LAYERED, k_nearest=5))
        assert e.value.code == fvv.FVV_E_ARG
        with pytest.raises(fvv.FvvError):
            c.set_bg_model(w.bg_models[:2])                       # one model per camera
        bad = [np.zeros((10, 10), np.uint16)] * 3                 # rows shorter than the width
        with pytest.raises(fvv.FvvError):
            c.set_bg_model(bad)
        c.set_bg_model(None)
        c.upload_mvd(w.frames)
        with pytest.raises(fvv.FvvError, match="background"):
            c.synthesize(w.virtual[0], p=p)
        c.synthesize(w.virtual[0])                                # the plain path still works


@pytest.fixture(scope="module")
def c3l():
    say("[gpu] generating the layered 9x1280x720 frame set")
    return sg.config3(0, n_frames=60, layered=True)


def test_full_rig_layered_batch_sampled(fvv, ctx, oracle_lib, c3l):
    import torch
    w = c3l
    ctx.set_rig(w.rig)
    ctx.set_bg_model(w.bg_models)
    ctx.upload_mvd(w.frames)
    p = fvv.params(path=fvv.PATH_LAYERED)
    outs = [torch.empty((v.height, v.width, 3), dtype=torch.uint8, device="cuda") for v in w.virtual]
    say("[gpu] layered c3 batch of 60")
    ctx.synthesize_batch(w.virtual, outs, p=p)
    torch.cuda.synchronize()
    for vi in (0, 22, 41, 59):
        r = oracle_lib.synthesize_layered(w.rig, w.frames, w.bg_models, w.virtual[vi])
        d = np.abs(outs[vi].cpu().numpy().astype(np.int16) - r["rgb"].astype(np.int16))
        assert d.max() <= 1, (vi, d.max())
    v = w.virtual[33]
    say("[gpu] layered c3 view 33 with taps")
    out, taps = run_layered(fvv, ctx, w, v, upload=False)
    compare_layered(oracle_lib, w, v, out, taps)
