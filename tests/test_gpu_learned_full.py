"""Learned-path parity at the network's production tiling (through the C ABI,
against oracle.unet in float64 with the kernels' bfloat16 points).

The kernels pick their tiling from the layer width and the pixel count: the
64-channel layers of the half-resolution level run 64-channel x 16-row
patches once a level holds 65,536 pixels or more (forward and data
gradient), the finest transposed convolution runs 128 x 128 blocks once it
has a thousand of them, and the weight-gradient chunking reaches its
1,024-workgroup regime.  These tests run those shapes: two 960x544 views of
the 9x1280x720 rig through the forward (every layer compared), one 960x540
learned synthesis, a training step on four 256x256 crops (level 1 holds
exactly 65,536 pixels) with every weight and bias gradient compared, and
three Adam steps against the oracle's Adam.  Bars as in the smaller tests.
The 32-channel full-resolution convolutions switch to a weights-resident
kernel once a batch has 2,048 patches of 8 x 16 pixels or more; its output
must be the bytes of the per-patch kernel (the same MFMA sequence per
output), checked by running two 512x256 stacks together (resident kernel)
and one at a time (per-patch kernel).
"""
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


@pytest.fixture(scope="module")
def ctx(fvv):
    c = fvv.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def rig9():
    say("[gpu] learned-full: generating the 9x1280x720 rig")
    return sg.config3(0, n_frames=3)


def rand_params(seed, scale=1.0):
    from oracle import unet
    rng = np.random.default_rng(seed)
    P = {}
    for name, kind, ci, co in unet.LAYERS:
        shp = unet.weight_shape(kind, ci, co)
        fan = int(np.prod(shp[1:]))
        P[name] = (rng.normal(0.0, scale * np.sqrt(2.0 / fan), shp).astype(np.float32),
                   rng.normal(0.0, 0.05, co).astype(np.float32))
    return P


def flat(P):
    from oracle import unet
    return np.concatenate([np.concatenate([P[n][0].ravel(), P[n][1].ravel()]) for n, *_ in unet.LAYERS])


def unflat(v):
    from oracle import unet
    P, o = {}, 0
    for n, kind, ci, co in unet.LAYERS:
        shp = unet.weight_shape(kind, ci, co)
        k = int(np.prod(shp))
        P[n] = (v[o:o + k].reshape(shp), v[o + k:o + k + co])
        o += k + co
    return P


def to_device_stack(st16):
    import torch
    N, H, W, _ = st16.shape
    full = torch.from_numpy(np.asarray(st16, np.float32)).to(torch.bfloat16).view(torch.int16).numpy().view(
        np.uint16)
    return torch.from_numpy(full.view(np.int16)).cuda()


def view_stack(oracle, w, angle):
    """Oracle stack (544, 960, 16) of a 960x540 view at `angle` on the arc."""
    v = sg.arc_camera(angle, 2.5, 960, 540)
    r = oracle.synthesize(w.rig, w.frames, v, taps=True)
    return v, oracle.stack(r["zf"], w.rig, w.frames, v, r["sel"], r["weights"], 0.05, 4, 0)


LEVEL = {"enc0a": 0, "enc0b": 0, "enc1a": 1, "enc1b": 1, "enc2a": 2, "enc2b": 2, "mid_a": 3, "mid_b": 3,
         "up2": 2, "dec2a": 2, "dec2b": 2, "up1": 1, "dec1a": 1, "dec1b": 1, "up0": 0, "dec0a": 0, "dec0b": 0}


def check_close(name, got, ref):
    scale = max(np.abs(ref).max(), 1e-6)
    d = np.abs(got - ref)
    far = d > 2.0 ** -6 * np.abs(ref) + 2.0 ** -8 * scale
    assert np.mean(far) < 2e-3 and d.max() <= 0.1 * scale, \
        f"{name}: {np.mean(far):.2e} outside, max {d.max():.3g} of scale {scale:.3g}"


def test_forward_two_960x544_views(fvv, ctx, oracle_lib, rig9):
    import torch
    from oracle import unet
    H, W, N = 544, 960, 2
    P = rand_params(80)
    ctx.net_load(flat(P))
    st = np.stack([view_stack(oracle_lib, rig9, a)[1] for a in (-22.0, 37.0)])
    out = torch.empty((N, H, W, 3), dtype=torch.float32, device="cuda")
    say("[gpu] learned-full: forward 2x960x544")
    ctx.set_debug(True)        # keep every layer's output for the comparison
    ctx.net_forward(to_device_stack(st), N, H, W, out)
    torch.cuda.synchronize()
    ctx.set_debug(False)
    s_gpu = out.cpu().numpy()
    for q in range(N):
        say(f"[gpu] learned-full: oracle forward of view {q}")
        s_ref, acts = unet.forward(P, st[q], keep=True)
        for li, (name, kind, ci, co) in enumerate(unet.LAYERS[:-1]):
            lv = LEVEL[name]
            px = (H >> lv) * (W >> lv)
            a = ctx.net_read_act(li, (N * px, co)).reshape(N, px, co)[q]
            check_close(f"{name}[{q}]", a, acts[name].reshape(-1, co))
        d = np.abs(s_gpu[q] - s_ref)
        assert d.max() < 2e-2 and np.mean(d > 4e-3) < 2e-3, (d.max(), np.mean(d > 4e-3))


def test_learned_synthesis_960x540(fvv, ctx, oracle_lib, rig9):
    P = rand_params(81)
    w = rig9
    ctx.set_rig(w.rig)
    ctx.upload_mvd(w.frames)
    ctx.net_load(flat(P))
    v = sg.arc_camera(8.0, 2.5, 960, 540)
    say("[gpu] learned-full: 960x540 learned synthesis")
    got = ctx.synthesize(v, p=fvv.params(path=fvv.PATH_LEARNED))
    ref, _, _ = oracle_lib.synthesize_learned(w.rig, w.frames, v, P)
    d = np.abs(got.astype(int) - ref.astype(int))
    assert np.mean(d <= 2) >= 0.999 and d.max() <= 8, (np.mean(d <= 2), d.max())


def test_gradients_four_256_crops(fvv, ctx, oracle_lib, rig9):
    """One training step on four 256x256 crops of 960x544 stacks; every
    weight and bias gradient within twice the spread of a float32
    evaluation of the oracle (+1 %), as in the small gradient test."""
    import torch
    from oracle import unet
    H = W = 256
    valid = 250
    P = rand_params(82)
    ctx.net_load(flat(P))
    full = [view_stack(oracle_lib, rig9, a)[1] for a in (-40.0, 12.0)]
    crops = np.stack([full[0][0:256, 100:356], full[0][288:544, 600:856],
                      full[1][100:356, 0:256], full[1][200:456, 704:960]])
    rng = np.random.default_rng(83)
    target = rng.uniform(0, 1, (4, H, W, 3)).astype(np.float32)
    say("[gpu] learned-full: training step 4x256x256")
    loss = ctx.net_train_step(to_device_stack(crops), torch.from_numpy(target).cuda(), 4, H, W, valid,
                              lr=0.0, apply=False)
    g = unflat(ctx.net_read(fvv.NET_GRADS))
    rl, rg, rg32 = 0.0, None, None
    for q in range(4):
        say(f"[gpu] learned-full: oracle gradients of crop {q}")
        lq, gq = unet.loss_and_grads(P, crops[q], target[q], valid)
        _, gq32 = unet.loss_and_grads(P, crops[q], target[q], valid, acc=np.float32)
        rl += lq / 4
        if rg is None:
            rg = {n: [np.asarray(x, np.float64) / 4 for x in gq[n]] for n in gq}
            rg32 = {n: [np.asarray(x, np.float64) / 4 for x in gq32[n]] for n in gq32}
        else:
            for n in gq:
                for k in range(2):
                    rg[n][k] = rg[n][k] + np.asarray(gq[n][k], np.float64) / 4
                    rg32[n][k] = rg32[n][k] + np.asarray(gq32[n][k], np.float64) / 4
    assert abs(loss - rl) <= 1e-3 * rl
    bad = []
    for name, *_ in unet.LAYERS:
        for k, what in ((0, "W"), (1, "b")):
            ref = rg[name][k].ravel()
            nrm = max(np.linalg.norm(ref), 1e-30)
            rel = np.linalg.norm(g[name][k].astype(np.float64).ravel() - ref) / nrm
            floor = np.linalg.norm(rg32[name][k].ravel() - ref) / nrm
            say(f"  {name}.{what}: gpu {rel:.2e}  float32 oracle {floor:.2e}")
            if rel > 2 * floor + 0.01:
                bad.append((f"{name}.{what}", rel, floor))
    assert not bad, bad


def test_adam_three_steps_vs_oracle(fvv, ctx, oracle_lib, rig9):
    """Three Adam steps with lr > 0: each step's gradient (read back from
    the device) is fed to the oracle's Adam, whose float32 master weights
    must match the device's after every step (moment decay and bias
    correction change from step to step)."""
    import torch
    from oracle import unet
    H, W = 64, 96
    P = rand_params(84)
    ctx.net_load(flat(P))
    st = view_stack(oracle_lib, rig9, -5.0)[1][200:264, 400:496]
    dst = to_device_stack(st[None])
    target = torch.rand((1, H, W, 3), generator=torch.Generator().manual_seed(85)).cuda()
    master = {n: [P[n][0].copy(), P[n][1].copy()] for n in P}
    m = {n: [np.zeros(P[n][0].shape), np.zeros(P[n][1].shape)] for n in P}
    v = {n: [np.zeros(P[n][0].shape), np.zeros(P[n][1].shape)] for n in P}
    lr = 2e-3
    for step in range(1, 4):
        ctx.net_train_step(dst, target, 1, H, W, H, lr=lr, apply=True)
        g = unflat(ctx.net_read(fvv.NET_GRADS))
        unet.adam_step(master, {n: [g[n][0], g[n][1]] for n in g}, m, v, step, lr=lr)
        got = unflat(ctx.net_read(fvv.NET_PARAMS))
        for n in master:
            for k in range(2):
                np.testing.assert_allclose(got[n][k], master[n][k], rtol=1e-5, atol=1e-6,
                                           err_msg=f"step {step} {n}[{k}]")
        # continue both from the device's weights (float32 rounding of the
        # two updates may differ in the last place)
        for n in master:
            master[n] = [got[n][0].copy(), got[n][1].copy()]


def test_weights_resident_conv_equals_per_patch_conv(fvv, ctx):
    import torch
    H, W = 256, 512       # 1,024 patches per image: one image per-patch, two resident
    ctx.net_load(flat(rand_params(86)))
    g = torch.Generator(device="cuda").manual_seed(87)
    st = torch.rand((2, H, W, fvv.NET_IN), device="cuda", generator=g)
    st[..., 15] = 0
    st = st.to(torch.bfloat16).view(torch.int16).contiguous()
    say("[gpu] learned-full: resident vs per-patch 3x3 convolutions")
    two = torch.empty((2, H, W, 3), dtype=torch.float32, device="cuda")
    ctx.set_debug(True)        # every layer kept (the finest transposed convolution on its own)
    ctx.net_forward(st, 2, H, W, two)
    torch.cuda.synchronize()
    layers = layer_list()[:-1]
    px = {li: (H >> LEVEL[name]) * (W >> LEVEL[name]) for li, (name, *_) in enumerate(layers)}
    acts_two = {li: ctx.net_read_act(li, (2 * px[li], co)) for li, (name, kind, ci, co) in enumerate(layers)}
    for q in range(2):
        one = torch.empty((1, H, W, 3), dtype=torch.float32, device="cuda")
        ctx.net_forward(st[q:q + 1].contiguous(), 1, H, W, one)
        torch.cuda.synchronize()
        assert torch.equal(one[0], two[q]), q
        for li, (name, kind, ci, co) in enumerate(layers):
            a = ctx.net_read_act(li, (px[li], co))
            assert np.array_equal(a, acts_two[li].reshape(2, px[li], co)[q]), (name, q)
    ctx.set_debug(False)


def test_fused_transposed_convolution_equals_stored(fvv, ctx):
    """Without debug taps a forward of 2,048 patches or more computes the
    finest transposed convolution inside the convolution that reads it and
    the head inside dec0b (neither's input is stored): the network's output
    must be the bytes of the forward that stores every layer, for the
    production batch of 16 960x544 stacks and for two 512x256 stacks, and
    reading those two layers must fail."""
    import torch
    ctx.net_load(flat(rand_params(88)))
    g = torch.Generator(device="cuda").manual_seed(89)
    for n, H, W in ((16, 544, 960), (2, 256, 512)):
        st = torch.rand((n, H, W, fvv.NET_IN), device="cuda", generator=g)
        st[..., 15] = 0
        st = st.to(torch.bfloat16).view(torch.int16).contiguous()
        say(f"[gpu] learned-full: fused vs stored finest transposed convolution, {n}x{W}x{H}")
        fused = torch.empty((n, H, W, 3), dtype=torch.float32, device="cuda")
        ctx.net_forward(st, n, H, W, fused)
        torch.cuda.synchronize()
        for lname in ("up0", "dec0b"):
            li = [li for li, (name, *_) in enumerate(layer_list()) if name == lname][0]
            with pytest.raises(fvv.FvvError):
                ctx.net_read_act(li, (n * H * W, 32))
        ctx.set_debug(True)
        kept = torch.empty((n, H, W, 3), dtype=torch.float32, device="cuda")
        ctx.net_forward(st, n, H, W, kept)
        torch.cuda.synchronize()
        ctx.set_debug(False)
        assert torch.equal(fused, kept), (n, H, W)


def layer_list():
    from oracle import unet
    return unet.LAYERS
