"""The torch ray caster (used to generate training sets on the device)
reproduces the numpy ray caster; run on the CPU here."""
import numpy as np
import torch

import scenegen as sg
from scenegen import gpu


def test_torch_render_matches_numpy():
    rng = np.random.default_rng(5)
    scene = sg.random_scene(rng, n_spheres=4, n_boxes=4, salt=5)
    for a in (-45.0, 0.0, 30.0):
        cam = sg.arc_camera(a, 2.5, 96, 54)
        rgb, z, _ = scene.render(cam)
        trgb, tz = gpu.render(scene, cam, device="cpu")
        same = np.all(trgb.numpy() == rgb, -1)
        assert same.mean() > 0.999
        np.testing.assert_allclose(tz.numpy(), z, rtol=1e-12)


def test_torch_capture_depth_recipe():
    rng = np.random.default_rng(6)
    scene = sg.random_scene(rng, salt=6)
    cam = sg.arc_camera(10.0, 2.5, 128, 72)
    g = torch.Generator().manual_seed(3)
    rgb, d = gpu.capture(scene, cam, g, noise_k=0.0, invalid_frac=0.1, device="cpu")
    _, z, _ = scene.render(cam)
    d = d.numpy()
    valid = d > 0
    assert 0.75 < valid.mean() < 0.95
    exp = np.clip(np.floor(z * 1000 + 0.5), 1, 65535)
    assert np.array_equal(d[valid], exp[valid])
