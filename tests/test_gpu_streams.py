"""Direct calls of one context on alternating streams: they share the
context's workspace and network activations, so each call on a stream other
than the previous call's waits on the device for that call's work.  Results
of back-to-back calls alternating between two streams (no host
synchronisation in between) must be byte-identical to the same calls run
one at a time."""
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


def test_synthesis_alternating_streams(fvv, ctx):
    import torch
    say("[gpu] streams: generating the 9x1280x720 rig")
    w = sg.config3(0, n_frames=40)
    ctx.set_rig(w.rig)
    ctx.upload_mvd(w.frames)
    A = w.virtual[:20]                                                   # 20 x 1920x1080
    B = [sg.arc_camera(a, 2.3, 1280, 720) for a in np.linspace(-50, 50, 20)]
    mk = lambda vs: [torch.empty((v.height, v.width, 3), dtype=torch.uint8, device="cuda") for v in vs]
    say("[gpu] streams: one call at a time")
    refA, refB = mk(A), mk(B)
    ctx.synthesize_batch(A, refA)
    torch.cuda.synchronize()
    ctx.synthesize_batch(B, refB)
    torch.cuda.synchronize()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    say("[gpu] streams: three rounds alternating two streams")
    for _ in range(3):
        oa, ob = mk(A), mk(B)
        ctx.synthesize_batch(A, oa, stream=sa)
        ctx.synthesize_batch(B, ob, stream=sb)
        outs.append((oa, ob))
    # single views too, alternating with the batches
    v1, v2 = A[7], B[3]
    s1, s2 = mk([v1])[0], mk([v2])[0]
    ctx.synthesize_batch(A, outs[0][0], stream=sa)
    ctx.synthesize(v2, s2, stream=sb)
    ctx.synthesize(v1, s1, stream=sa)
    torch.cuda.synchronize()
    for oa, ob in outs:
        assert all(torch.equal(x, y) for x, y in zip(oa, refA)), "batch A differs from the one-at-a-time run"
        assert all(torch.equal(x, y) for x, y in zip(ob, refB)), "batch B differs from the one-at-a-time run"
    assert torch.equal(s1, refA[7]) and torch.equal(s2, refB[3])


def test_network_alternating_streams(fvv, ctx):
    import torch
    from paper_2007_00558_amd import learned
    w = sg.config_small(2, n_cams=4, w=160, h=96, out_w=256, out_h=192, n_virtual=2)
    ctx.set_rig(w.rig)
    ctx.upload_mvd(w.frames)
    ctx.net_load(learned.init_params(1))
    H, W = 192, 256
    stacks = []
    for v in w.virtual:
        st = torch.zeros(H * W * fvv.NET_IN, dtype=torch.int16, device="cuda")
        ctx.make_stack([v], [fvv.params(path=fvv.PATH_LEARNED)], st)
        stacks.append(st)
    torch.cuda.synchronize()
    refs = []
    for st in stacks:
        o = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
        ctx.net_forward(st, 1, H, W, o)
        torch.cuda.synchronize()
        refs.append(o)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    say("[gpu] streams: network forwards alternating two streams")
    got = []
    for _ in range(3):
        oa = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
        ob = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
        ctx.net_forward(stacks[0], 1, H, W, oa, stream=sa)
        ctx.net_forward(stacks[1], 1, H, W, ob, stream=sb)
        got.append((oa, ob))
    # learned syntheses (stack, network, RGB) alternating too
    la = torch.empty((H, W, 3), dtype=torch.uint8, device="cuda")
    lb = torch.empty((H, W, 3), dtype=torch.uint8, device="cuda")
    p = fvv.params(path=fvv.PATH_LEARNED)
    ctx.synthesize(w.virtual[0], la, p, stream=sa)
    ctx.synthesize(w.virtual[1], lb, p, stream=sb)
    torch.cuda.synchronize()
    for oa, ob in got:
        assert torch.equal(oa, refs[0]) and torch.equal(ob, refs[1])
    ra = ctx.synthesize(w.virtual[0], p=p)
    rb = ctx.synthesize(w.virtual[1], p=p)
    assert np.array_equal(la.cpu().numpy(), ra) and np.array_equal(lb.cpu().numpy(), rb)


def test_training_refused_while_serving(fvv, ctx):
    import torch
    from paper_2007_00558_amd import learned
    w = sg.config_small(1, n_cams=3)
    ctx.set_rig(w.rig)
    ctx.upload_mvd(w.frames)
    ctx.net_load(learned.init_params(0))
    H, W = 64, 96
    st = torch.zeros(H * W * fvv.NET_IN, dtype=torch.int16, device="cuda")
    tgt = torch.zeros((H, W, 3), dtype=torch.float32, device="cuda")
    srv = fvv.Server(ctx, max_slots=4)
    try:
        with pytest.raises(fvv.FvvError) as e:
            ctx.net_train_step(st, tgt, 1, H, W, H)
        assert e.value.code == fvv.FVV_E_STATE
    finally:
        srv.stop()
    ctx.net_train_step(st, tgt, 1, H, W, H, lr=0.0)
