"""Adaptive view transmission (Section V-C) on the GPU path: uploading only
the transmission set of the active clients renders their viewpoints exactly
as uploading every camera, and the server reports the set of its recent
clients."""
import sys
import time

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


@pytest.mark.parametrize("layered", [False, True])
def test_subset_upload_renders_like_full_upload(fvv, oracle_lib, layered):
    w = sg.config3(0, n_frames=2, src_w=320, src_h=180, out_w=480, out_h=270, layered=layered)
    rng = np.random.default_rng(3)
    users = [sg.arc_camera(a, 2.5, 480, 270) for a in rng.uniform(-55, 55, 3)]
    p = fvv.params(path=fvv.PATH_LAYERED if layered else fvv.PATH_PLAIN)
    for n_users in (1, 2, 3):
        views = users[:n_users]
        mask = fvv.tx_cameras(w.rig, views, 5)
        assert mask == oracle_lib.tx_cameras(w.rig, views, 5)
        sent = [f if mask >> k & 1 else None for k, f in enumerate(w.frames)]
        say(f"[gpu] tx subset layered={layered} users={n_users} cameras={bin(mask)}")
        with fvv.Context(0) as full, fvv.Context(0) as part:
            for c, frames in ((full, w.frames), (part, sent)):
                c.set_rig(w.rig)
                if layered:
                    c.set_bg_model(w.bg_models)
                c.upload_mvd(frames)
            for v in views:
                a = full.synthesize(v, p=p)
                b = part.synthesize(v, p=p)
                assert np.array_equal(a, b)


def test_server_reports_the_clients_transmission_set(fvv, oracle_lib):
    import torch
    w = sg.config_small(4, n_cams=7, w=96, h=64)
    ctx = fvv.Context(0)
    ctx.set_rig(w.rig)
    ctx.upload_mvd(w.frames)
    srv = fvv.Server(ctx, max_slots=4)
    views = [sg.arc_camera(a, 2.2, 64, 48) for a in (-40.0, -38.0, 30.0)]
    outs = [torch.empty((v.height, v.width, 3), dtype=torch.uint8, device="cuda") for v in views]
    say("[gpu] server transmission set")
    tickets = [srv.submit(v, o) for v, o in zip(views, outs)]
    deadline = time.time() + 30
    while time.time() < deadline and not all(srv.poll(t) is not None for t in tickets):
        time.sleep(0.005)
    assert srv.tx_cameras(5, 60.0) == oracle_lib.tx_cameras(w.rig, views, 5)
    assert srv.tx_cameras(3, 60.0) == oracle_lib.tx_cameras(w.rig, views, 3)
    time.sleep(0.05)
    assert srv.tx_cameras(5, 0.0) == 0                    # nobody within the last instant
    srv.stop()
    with pytest.raises(fvv.FvvError):
        srv.tx_cameras(5, 1.0)                            # server stopped
    ctx.close()
