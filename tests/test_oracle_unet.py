"""Pins for the learned-path oracle (CPU): its convolutions against direct
loops, its bfloat16 rounding against hand-worked bit patterns, its
hand-written backward against central finite differences, Adam against
hand-worked moments over three steps, and training against an overfit
check."""
import numpy as np
import pytest
import torch

from oracle import unet


def direct_conv(x, w, b):
    """x (H, W, Ci), w (Co, k, k, Ci): zero-padded same-size correlation."""
    H, W, Ci = x.shape
    Co, k, _, _ = w.shape
    p = k // 2
    xp = np.zeros((H + 2 * p, W + 2 * p, Ci))
    xp[p:p + H, p:p + W] = x
    out = np.zeros((H, W, Co))
    for y in range(H):
        for xx in range(W):
            for co in range(Co):
                out[y, xx, co] = np.sum(xp[y:y + k, xx:xx + k, :] * w[co]) + b[co]
    return out


def direct_convT(x, w, b):
    H, W, Ci = x.shape
    Co = w.shape[0]
    out = np.zeros((2 * H, 2 * W, Co))
    for y in range(H):
        for xx in range(W):
            for dy in range(2):
                for dx in range(2):
                    out[2 * y + dy, 2 * xx + dx] += w[:, dy, dx, :] @ x[y, xx]
    return out + b


def nchw(a):
    return torch.from_numpy(a).permute(2, 0, 1)[None]


def test_conv_matches_direct_loop():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(5, 6, 3))
    for k in (3, 1):
        w = rng.normal(size=(2, k, k, 3))
        b = rng.normal(size=2)
        got = unet._conv(nchw(x), torch.from_numpy(w), torch.from_numpy(b))[0].permute(1, 2, 0).numpy()
        np.testing.assert_allclose(got, direct_conv(x, w, b), rtol=1e-12, atol=1e-12)


def test_convT_matches_direct_loop():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(3, 4, 5))
    w = rng.normal(size=(2, 2, 2, 5))
    b = rng.normal(size=2)
    got = unet._convT(nchw(x), torch.from_numpy(w), torch.from_numpy(b))[0].permute(1, 2, 0).numpy()
    np.testing.assert_allclose(got, direct_convT(x, w, b), rtol=1e-12, atol=1e-12)


def test_bf16_rounding_is_nearest_even():
    # bfloat16 keeps 8 significand bits: ulp(1) = 2^-7
    vals = torch.tensor([1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, -(1 + 2 ** -8), 3.0, 1e-3],
                        dtype=torch.float64)
    want = [1.0, 1 + 2 ** -6, 1 + 2 ** -7, -1.0, 3.0]
    got = unet.bf16(vals).tolist()
    assert got[:5] == want
    # 1e-3 = 1.024 * 2^-10 -> nearest bfloat16 is 131/128 * 2^-10
    assert got[5] == 131 / 128 * 2 ** -10


def tiny_params(seed, widths=(2, 3, 3, 4), in_ch=4):
    rng = np.random.default_rng(seed)
    p = {}
    for name, kind, ci, co in unet.layer_shapes(widths, in_ch):
        shp = unet.weight_shape(kind, ci, co)
        fan = shp[1] * shp[2] * ci
        p[name] = [(rng.normal(size=shp) * np.sqrt(2.0 / fan)).astype(np.float32),
                   (rng.normal(size=co) * 0.1).astype(np.float32)]
    return p


def test_backward_matches_finite_differences():
    widths, in_ch = (2, 3, 3, 4), 4
    rng = np.random.default_rng(3)
    params = tiny_params(4, widths, in_ch)
    pd = {k: [v[0].astype(np.float64), v[1].astype(np.float64)] for k, v in params.items()}
    x = rng.uniform(0, 1, size=(16, 16, in_ch))
    t = rng.uniform(0, 1, size=(16, 16, 3))
    loss, grads = unet.loss_and_grads(pd, x, t, 14, widths, rounding=False)

    def L(p):
        s, _ = unet.forward(p, x, widths, rounding=False)
        return float(np.abs(s[:14] - t[:14]).mean())

    assert abs(L(pd) - loss) < 1e-12
    h = 1e-6
    checked = 0
    for name, (w, b) in pd.items():
        for k, arr in enumerate((w, b)):
            flat = arr.reshape(-1)
            for e in rng.choice(flat.size, size=min(3, flat.size), replace=False):
                old = flat[e]
                flat[e] = old + h
                lp = L(pd)
                flat[e] = old - h
                lm = L(pd)
                flat[e] = old
                fd = (lp - lm) / (2 * h)
                an = grads[name][k].reshape(-1)[e]
                assert abs(fd - an) <= 1e-6 + 1e-4 * abs(fd), (name, k, e, fd, an)
                checked += 1
    assert checked > 50


def test_rounded_forward_stays_close_to_exact():
    widths = (8, 8, 16, 16)
    params = tiny_params(5, widths, 16)
    x = np.random.default_rng(6).uniform(0, 1, size=(32, 24, 16))
    s1, _ = unet.forward(params, x, widths, rounding=True)
    s0, _ = unet.forward(params, x, widths, rounding=False)
    assert np.max(np.abs(s1 - s0)) < 0.02


def test_adam_overfits_one_sample():
    widths, in_ch = (8, 8, 8, 8), 4
    rng = np.random.default_rng(7)
    master = tiny_params(8, widths, in_ch)
    m = {k: [np.zeros_like(v[0], np.float64), np.zeros_like(v[1], np.float64)] for k, v in master.items()}
    v = {k: [np.zeros_like(a[0], np.float64), np.zeros_like(a[1], np.float64)] for k, a in master.items()}
    x = rng.uniform(0, 1, size=(16, 16, in_ch))
    t = 0.2 + 0.6 * x[..., :3]          # learnable from the input
    losses = []
    for step in range(1, 101):
        loss, g = unet.loss_and_grads(master, x, t, 16, widths, rounding=True)
        losses.append(loss)
        unet.adam_step(master, g, m, v, step, lr=1e-2)
    assert losses[-1] < 0.5 * losses[0]


def test_adam_three_steps_hand_worked():
    """Three Adam steps with gradients 1, -2, 0.5 (and their negatives, and a
    zero gradient) on a scalar weight and bias, beta = (0.9, 0.999), against
    moments worked out by hand:
      m1 = 0.1            v1 = 0.001             1 - b1^t = 0.1    1 - b2^t = 0.001
      m2 = 0.09 - 0.2     v2 = 0.000999 + 0.004            0.19             0.001999
         = -0.11             = 0.004999
      m3 = -0.099 + 0.05  v3 = 0.004994001 + 0.00025       0.271            0.002997001
         = -0.049            = 0.005244001
    A wrong decay, a missing square, a bias correction off by one step or a
    swapped beta changes the weights by far more than float32 rounding."""
    lr, eps = 1e-3, 1e-8
    gs = [1.0, -2.0, 0.5]
    hand_m = [0.1, -0.11, -0.049]
    hand_v = [0.001, 0.004999, 0.005244001]
    hand_c1 = [0.1, 0.19, 0.271]
    hand_c2 = [0.001, 0.001999, 0.002997001]
    master = {"L": [np.float32([[0.25]]), np.float32([-0.5, 0.75])]}
    m = {"L": [np.zeros((1, 1)), np.zeros(2)]}
    v = {"L": [np.zeros((1, 1)), np.zeros(2)]}
    w_want = np.float32(0.25)
    b_want = np.float32([-0.5, 0.75])
    for t in range(3):
        grads = {"L": [np.float32([[gs[t]]]), np.float32([-gs[t], 0.0])]}
        unet.adam_step(master, grads, m, v, t + 1, lr=lr)
        assert m["L"][0][0, 0] == pytest.approx(hand_m[t], rel=1e-12)
        assert v["L"][0][0, 0] == pytest.approx(hand_v[t], rel=1e-12)
        assert m["L"][1][0] == pytest.approx(-hand_m[t], rel=1e-12)
        assert v["L"][1][0] == pytest.approx(hand_v[t], rel=1e-12)
        assert m["L"][1][1] == 0.0 and v["L"][1][1] == 0.0
        step = lr * (hand_m[t] / hand_c1[t]) / (np.sqrt(hand_v[t] / hand_c2[t]) + eps)
        w_want = np.float32(np.float64(w_want) - step)
        b_want = np.float32(np.float64(b_want) - np.array([-step, 0.0]))
        assert master["L"][0].dtype == np.float32
        assert master["L"][0][0, 0] == w_want
        assert np.array_equal(master["L"][1], b_want)
    # net displacement: lr (1 - 0.5789474 / 1.5813761 - 0.1808118 / 1.3227810)
    # (step 1 moves by lr: its corrected moments are g and g^2); the bias with
    # zero gradient stays put (three float32 roundings near 0.25: 1e-7)
    assert float(np.float32(0.25) - w_want) == pytest.approx(lr * 0.4972058, abs=1e-7)
    assert b_want[1] == np.float32(0.75)
