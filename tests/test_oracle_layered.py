"""Pins for the oracle's layered FG/BG synthesis (Section VI): the two
special cases that reduce it to the single-layer synthesis, the stacking of
the foreground over a nearer background, and the separation of the layers'
colour mixing."""
import numpy as np

import scenegen as sg
import oracle


def test_without_background_signal_it_is_the_plain_synthesis():
    w = sg.config_small(1)                     # live depth everywhere, no background signal
    bgm = [np.full_like(f.depth_mm, 1500) for f in w.frames]
    for v in w.virtual:
        for mode in (0, 1):
            a = oracle.synthesize_layered(w.rig, w.frames, bgm, v, fill_mode=mode)
            b = oracle.synthesize(w.rig, w.frames, v, fill_mode=mode, taps=True)
            assert np.array_equal(a["rgb"], b["rgb"])
            assert np.array_equal(a["hole"], b["hole"])
            assert np.array_equal(a["depth"].view(np.uint32), b["depth"].view(np.uint32))


def test_all_background_is_the_plain_synthesis_of_the_background_model():
    w = sg.config_small(2, layered=True)
    rig = [sg.Camera(c.width, c.height, c.fx, c.fy, c.cx, c.cy, c.R, c.t, 0.02, 0.97) for c in w.rig]
    live = [sg.Frame(f.rgb, np.full_like(f.depth_mm, sg.BG_MM)) for f in w.frames]
    model = [sg.Frame(f.rgb, m) for f, m in zip(w.frames, w.bg_models)]
    ident = [sg.Camera(c.width, c.height, c.fx, c.fy, c.cx, c.cy, c.R, c.t) for c in w.rig]
    for v in w.virtual:
        a = oracle.synthesize_layered(rig, live, w.bg_models, v)
        b = oracle.synthesize(ident, model, v, taps=True)
        assert np.array_equal(a["rgb"], b["rgb"])
        assert np.array_equal(a["bg"]["zf"], b["zf"])
        assert np.all(a["fg"]["zf"] == np.uint64(0xFFFFFFFFFFFFFFFF))
        # Eq. 1 applies to live depth only: with the correction on the model
        # the result changes
        c = oracle.synthesize(rig, model, v)
        assert not np.array_equal(a["rgb"], c["rgb"])


def test_foreground_is_stacked_over_a_nearer_background():
    w = sg.config_small(3, layered=True)
    near = [np.where(m > 0, 800, 0).astype(np.uint16) for m in w.bg_models]    # a wall 0.8 m away
    v = w.virtual[1]
    r = oracle.synthesize_layered(w.rig, w.frames, near, v)
    fg_on = r["fg"]["hole"] == 0
    bg_on = r["bg"]["hole"] == 0
    both = fg_on & bg_on
    assert both.sum() >= 10
    assert np.all(r["bg"]["depth"][both] < r["fg"]["depth"][both])   # a depth test would pick the wall
    assert np.array_equal(r["blend_rgb"][fg_on], r["fg"]["blend_rgb"][fg_on])
    assert np.array_equal(r["blend_rgb"][~fg_on & bg_on], r["bg"]["blend_rgb"][~fg_on & bg_on])


def test_layers_mix_their_own_pixels_only():
    """Background pixels are painted pure red and foreground pixels carry no
    red: the foreground layer then never shows red and the background layer
    never shows anything else."""
    w = sg.config_small(4, layered=True)
    frames = []
    for f in w.frames:
        rgb = f.rgb.copy()
        is_bg = f.depth_mm == sg.BG_MM
        rgb[is_bg] = (255, 0, 0)
        rgb[~is_bg, 0] = 0
        frames.append(sg.Frame(rgb, f.depth_mm))
    for v in w.virtual:
        r = oracle.synthesize_layered(w.rig, frames, w.bg_models, v, fill_mode=1)
        fg_on = r["fg"]["hole"] == 0
        bg_on = r["bg"]["hole"] == 0
        assert fg_on.sum() > 100 and bg_on.sum() > 100
        assert np.all(r["fg"]["blend_rgb"][fg_on][:, 0] == 0)
        assert np.all(r["bg"]["blend_rgb"][bg_on] == (255, 0, 0))
