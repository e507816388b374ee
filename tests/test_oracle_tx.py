"""Pins for the oracle's adaptive view transmission set (Section V-C): the
N_Tx cameras nearest to each client viewpoint, united over the clients."""
import numpy as np
import pytest

import scenegen as sg
import oracle


def ranking(rig, v):
    cv = -(v.R.T @ v.t)
    d = [np.linalg.norm(-(c.R.T @ c.t) - cv) for c in rig]
    return list(np.argsort(np.array(d), kind="stable"))


def rig9():
    return [sg.arc_camera(-60.0 + 15.0 * k, 2.5, 64, 36) for k in range(9)]


def random_viewpoints(rng, n):
    """Viewpoints on the rig's arc (radius 2.5 m, 0.2 m up) at random angles."""
    return [sg.arc_camera(rng.uniform(-80, 80), 2.5, 64, 36) for _ in range(n)]


def test_brute_force_and_contiguity_on_the_arc():
    rig = rig9()
    rng = np.random.default_rng(0)
    for v in random_viewpoints(rng, 60):
        for n_tx in (1, 3, 5, 9):
            m = oracle.tx_cameras(rig, [v], n_tx)
            want = 0
            for c in ranking(rig, v)[:n_tx]:
                want |= 1 << int(c)
            assert m == want
            bits = [c for c in range(9) if m >> c & 1]
            assert bits == list(range(bits[0], bits[0] + n_tx))      # a run of neighbours on the arc


def test_everything_and_a_coincident_viewpoint():
    rig = rig9()
    assert oracle.tx_cameras(rig, [rig[4]], 9) == (1 << 9) - 1
    assert oracle.tx_cameras(rig, [rig[6]], 1) == 1 << 6
    m = oracle.tx_cameras(rig, [rig[6]], 3)
    assert m == (1 << 5) | (1 << 6) | (1 << 7)


def test_contains_the_rendering_selection_and_unites_clients():
    rig = rig9()
    rng = np.random.default_rng(1)
    views = random_viewpoints(rng, 12)
    union = 0
    for v in views:
        m = oracle.tx_cameras(rig, [v], 5)
        idx, _ = oracle.select(rig, v, 3)
        assert all(m >> int(c) & 1 for c in idx)
        union |= m
    assert oracle.tx_cameras(rig, views, 5) == union


def test_brute_force_anywhere():
    rig = rig9()
    rng = np.random.default_rng(2)
    for _ in range(80):
        eye = rng.uniform(-4, 4, 3)
        R, t = sg.look_at(eye, rng.uniform(-0.5, 0.5, 3))
        v = sg.Camera(64, 36, 50.0, 50.0, 31.5, 17.5, R, t)
        n_tx = int(rng.integers(1, 10))
        want = 0
        for c in ranking(rig, v)[:n_tx]:
            want |= 1 << int(c)
        assert oracle.tx_cameras(rig, [v], n_tx) == want
