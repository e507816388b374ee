"""CPU reference of the learned blend/inpaint network -- TEST INFRASTRUCTURE ONLY.

The paper mixes the warped reference cameras with fixed distance weights
(Section VI).  The learned path replaces that mix (and fills disocclusions)
with a small convolutional U-Net that reads, for each of the three selected
cameras, its depth-consistent backward-warped colour, the inverse depth of
the z-buffer winner and a validity flag (15 channels, one zero pad channel
makes 16), and predicts RGB.  This module is the definition the HIP kernels
are checked against.  It uses plain PyTorch CPU ops in float64; values the
kernels store in bfloat16 (the input stack, weights, activations and the
gradients fed to the matrix cores) are rounded to bfloat16 here at the same
points (round to nearest even), everything else stays float64.

Graph (H, W multiples of 8; NHWC tensors; 3x3 convs zero-padded):
  enc0a 16->32, enc0b 32->32            (conv3x3 + bias + ReLU)
  pool  enc1a 32->64,  enc1b 64->64
  pool  enc2a 64->128, enc2b 128->128
  pool  mid_a 128->256, mid_b 256->256
  up2  convT2x2 256->128 (+bias), concat [up2, enc2b] -> dec2a 256->128, dec2b 128->128
  up1  convT2x2 128->64,          concat [up1, enc1b] -> dec1a 128->64,  dec1b 64->64
  up0  convT2x2 64->32,           concat [up0, enc0b] -> dec0a 64->32,   dec0b 32->32
  head 1x1 32->3 + bias, sigmoid
Weights: conv (C_out, kh, kw, C_in) float32, bias (C_out,); convT (C_out,
2, 2, C_in) with out[2y+dy, 2x+dx, co] = sum_ci in[y, x, ci] W[co, dy, dx, ci].

Training: L1 loss mean |s - target| over the valid rows and 3 channels,
hand-written backward with the same bfloat16 points as the kernels, Adam
(beta1 0.9, beta2 0.999, eps 1e-8) on float32 master weights.
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np
import torch
import torch.nn.functional as F

IN_CH = 16          # 15 stack channels + 1 zero pad channel
WIDTHS = (32, 64, 128, 256)

# (name, kind, C_in, C_out)
LAYERS: List[Tuple[str, str, int, int]] = [
    ("enc0a", "conv", IN_CH, 32), ("enc0b", "conv", 32, 32),
    ("enc1a", "conv", 32, 64), ("enc1b", "conv", 64, 64),
    ("enc2a", "conv", 64, 128), ("enc2b", "conv", 128, 128),
    ("mid_a", "conv", 128, 256), ("mid_b", "conv", 256, 256),
    ("up2", "convT", 256, 128), ("dec2a", "conv", 256, 128), ("dec2b", "conv", 128, 128),
    ("up1", "convT", 128, 64), ("dec1a", "conv", 128, 64), ("dec1b", "conv", 64, 64),
    ("up0", "convT", 64, 32), ("dec0a", "conv", 64, 32), ("dec0b", "conv", 32, 32),
    ("head", "head", 32, 3),
]


def layer_shapes(widths=WIDTHS, in_ch=IN_CH):
    """Layer list for other widths (tests use tiny nets); same topology."""
    w0, w1, w2, w3 = widths
    return [
        ("enc0a", "conv", in_ch, w0), ("enc0b", "conv", w0, w0),
        ("enc1a", "conv", w0, w1), ("enc1b", "conv", w1, w1),
        ("enc2a", "conv", w1, w2), ("enc2b", "conv", w2, w2),
        ("mid_a", "conv", w2, w3), ("mid_b", "conv", w3, w3),
        ("up2", "convT", w3, w2), ("dec2a", "conv", 2 * w2, w2), ("dec2b", "conv", w2, w2),
        ("up1", "convT", w2, w1), ("dec1a", "conv", 2 * w1, w1), ("dec1b", "conv", w1, w1),
        ("up0", "convT", w1, w0), ("dec0a", "conv", 2 * w0, w0), ("dec0b", "conv", w0, w0),
        ("head", "head", w0, 3),
    ]


def weight_shape(kind, cin, cout):
    return {"conv": (cout, 3, 3, cin), "convT": (cout, 2, 2, cin), "head": (cout, 1, 1, cin)}[kind]


def bf16(x: torch.Tensor) -> torch.Tensor:
    """Round to bfloat16 (nearest even) and return in the input's dtype."""
    return x.to(torch.bfloat16).to(x.dtype)


class Rounding:
    """Where bfloat16 rounding is applied; off gives the exact float64 graph."""

    def __init__(self, on: bool = True):
        self.on = on

    def __call__(self, x):
        return bf16(x) if self.on else x


# ---------------------------------------------------------------- forward
def _conv(x, w, b):
    """x: (1, C, H, W); w: (C_out, kh, kw, C_in) -> same-size conv + bias."""
    wt = w.permute(0, 3, 1, 2)
    return F.conv2d(x, wt, b, padding=w.shape[1] // 2)


def _convT(x, w, b):
    wt = w.permute(3, 0, 1, 2)           # (C_in, C_out, 2, 2)
    return F.conv_transpose2d(x, wt, b, stride=2)


def forward(params: Dict[str, Tuple[np.ndarray, np.ndarray]], stack: np.ndarray, widths=WIDTHS,
            rounding: bool = True, keep: bool = False, acc=np.float64):
    """stack: (H, W, C_in) float values (bfloat16-representable).  Returns
    (s (H, W, 3) sigmoid output, dict of per-layer outputs as NHWC).  ``acc``
    is the arithmetic type (float64 for the reference; float32 gives a second,
    independently rounded evaluation used to size tolerances)."""
    R = Rounding(rounding)
    layers = layer_shapes(widths, stack.shape[2])
    P = {n: (R(torch.from_numpy(np.asarray(w, acc))), torch.from_numpy(np.asarray(b, acc)))
         for n, (w, b) in params.items()}
    x = R(torch.from_numpy(np.asarray(stack, acc)).permute(2, 0, 1)[None])
    acts = {"input": x}
    relu = lambda t: R(torch.clamp_min(t, 0.0))
    a = x
    skips = {}
    for lvl, (na, nb) in enumerate((("enc0a", "enc0b"), ("enc1a", "enc1b"), ("enc2a", "enc2b"))):
        if lvl > 0:
            a = F.max_pool2d(a, 2)
        a = relu(_conv(a, *P[na]))
        acts[na] = a
        a = relu(_conv(a, *P[nb]))
        acts[nb] = a
        skips[lvl] = a
    a = F.max_pool2d(a, 2)
    a = relu(_conv(a, *P["mid_a"]))
    acts["mid_a"] = a
    a = relu(_conv(a, *P["mid_b"]))
    acts["mid_b"] = a
    for lvl, (nu, na, nb) in zip((2, 1, 0), (("up2", "dec2a", "dec2b"), ("up1", "dec1a", "dec1b"),
                                            ("up0", "dec0a", "dec0b"))):
        u = R(_convT(a, *P[nu]))
        acts[nu] = u
        a = torch.cat([u, skips[lvl]], 1)
        a = relu(_conv(a, *P[na]))
        acts[na] = a
        a = relu(_conv(a, *P[nb]))
        acts[nb] = a
    z = _conv(a, *P["head"])
    acts["head_z"] = z
    s = torch.sigmoid(z)
    nhwc = lambda t: t[0].permute(1, 2, 0).numpy()
    out = nhwc(s)
    if keep:
        return out, {k: nhwc(v) for k, v in acts.items()}
    return out, None


def to_rgb8(s: np.ndarray) -> np.ndarray:
    return np.minimum(np.floor(s * 255.0 + 0.5), 255).astype(np.uint8)


# ---------------------------------------------------------------- training
def loss_and_grads(params, stack, target, valid_rows: int, widths=WIDTHS, rounding: bool = True,
                   acc=np.float64):
    """L1 loss over rows [0, valid_rows) and its gradients, written out with
    the kernels' bfloat16 points: every tensor fed to a matrix product
    (activations, weights, incoming gradients) is bfloat16, accumulations and
    the gradients passed between layers are float64 here (float32 on the GPU).
    target: (H, W, 3) in [0, 1].  Returns (loss, {name: (gW, gb)})."""
    R = Rounding(rounding)
    layers = {n: (k, ci, co) for n, k, ci, co in layer_shapes(widths, stack.shape[2])}
    P = {n: (R(torch.from_numpy(np.asarray(w, acc))), torch.from_numpy(np.asarray(b, acc)))
         for n, (w, b) in params.items()}
    x = R(torch.from_numpy(np.asarray(stack, acc)).permute(2, 0, 1)[None])
    relu = lambda t: R(torch.clamp_min(t, 0.0))
    # forward, keeping what the backward needs
    ins, outs = {}, {}
    a = x
    skips, pool_in = {}, {}
    for lvl, (na, nb) in enumerate((("enc0a", "enc0b"), ("enc1a", "enc1b"), ("enc2a", "enc2b"))):
        if lvl > 0:
            pool_in[lvl] = a
            a = F.max_pool2d(a, 2)
        ins[na] = a
        a = relu(_conv(a, *P[na]))
        outs[na] = a
        ins[nb] = a
        a = relu(_conv(a, *P[nb]))
        outs[nb] = a
        skips[lvl] = a
    pool_in[3] = a
    a = F.max_pool2d(a, 2)
    ins["mid_a"] = a
    a = relu(_conv(a, *P["mid_a"]))
    outs["mid_a"] = a
    ins["mid_b"] = a
    a = relu(_conv(a, *P["mid_b"]))
    outs["mid_b"] = a
    ups = (("up2", "dec2a", "dec2b", 2), ("up1", "dec1a", "dec1b", 1), ("up0", "dec0a", "dec0b", 0))
    for nu, na, nb, lvl in ups:
        ins[nu] = a
        u = R(_convT(a, *P[nu]))
        outs[nu] = u
        a = torch.cat([u, skips[lvl]], 1)
        ins[na] = a
        a = relu(_conv(a, *P[na]))
        outs[na] = a
        ins[nb] = a
        a = relu(_conv(a, *P[nb]))
        outs[nb] = a
    ins["head"] = a
    z = _conv(a, *P["head"])
    s = torch.sigmoid(z)
    H = s.shape[2]
    t = torch.from_numpy(np.asarray(target, acc)).permute(2, 0, 1)[None]
    diff = (s - t)[:, :, :valid_rows]
    n = diff.numel()
    loss = float(diff.abs().sum() / n)
    # backward
    gs = torch.zeros_like(s)
    gs[:, :, :valid_rows] = torch.sign(diff) / n
    g = gs * s * (1.0 - s)                      # d loss / d z
    grads = {}

    def conv_back(name, g_out, pre_relu_out):
        """g_out: gradient w.r.t. the layer output (after ReLU if any)."""
        w, b = P[name]
        kind = layers[name][0]
        if pre_relu_out is not None:
            g_out = g_out * (pre_relu_out > 0)
        G = R(g_out)
        inp = ins[name]
        wt = w.permute(0, 3, 1, 2)
        if kind == "convT":
            # out[2y+dy, 2x+dx, co] = sum_ci in[y, x, ci] W[co, dy, dx, ci]
            C = G[0].reshape(G.shape[1], inp.shape[2], 2, inp.shape[3], 2)   # co, y, dy, x, dx
            gW = torch.einsum("cydxe,iyx->cdei", C, inp[0])                  # co, dy, dx, ci
            gin = torch.einsum("cydxe,cdei->iyx", C, w)[None]
        else:
            pad = w.shape[1] // 2
            gW = torch.nn.grad.conv2d_weight(inp, wt.shape, G, padding=pad).permute(0, 2, 3, 1)
            gin = torch.nn.grad.conv2d_input(inp.shape, wt, G, padding=pad)
        gb = g_out.sum(dim=(0, 2, 3))
        grads[name] = (gW.numpy().copy(), gb.numpy().copy())
        return gin

    g = conv_back("head", g, None)
    skip_g = {}
    for nu, na, nb, lvl in ups[::-1]:
        g = conv_back(nb, g, outs[nb])
        g = conv_back(na, g, outs[na])
        cu = outs[nu].shape[1]
        g_up, skip_g[lvl] = g[:, :cu], g[:, cu:]
        g = conv_back(nu, g_up, None)
    g = conv_back("mid_b", g, outs["mid_b"])
    g = conv_back("mid_a", g, outs["mid_a"])
    for lvl, (na, nb) in zip((2, 1, 0), (("enc2a", "enc2b"), ("enc1a", "enc1b"), ("enc0a", "enc0b"))):
        g = _pool_back(pool_in[lvl + 1], g)
        g = g + skip_g[lvl]
        g = conv_back(nb, g, outs[nb])
        g = conv_back(na, g, outs[na])
    return loss, grads


def _pool_back(x, g):
    """Route each 2x2 window's gradient to its first maximum (raster order)."""
    N, C, H, W = x.shape
    win = x.reshape(N, C, H // 2, 2, W // 2, 2).permute(0, 1, 2, 4, 3, 5).reshape(N, C, H // 2, W // 2, 4)
    idx = win.argmax(-1)                       # first maximum
    out = torch.zeros_like(win)
    out.scatter_(-1, idx[..., None], g[..., None])
    return out.reshape(N, C, H // 2, W // 2, 2, 2).permute(0, 1, 2, 4, 3, 5).reshape(N, C, H, W)


def adam_step(master, grads, m, v, step: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step on float32 master weights (in place), bias-corrected."""
    for n in master:
        for k in range(2):
            g = np.asarray(grads[n][k], np.float64)
            m[n][k] = b1 * m[n][k] + (1 - b1) * g
            v[n][k] = b2 * v[n][k] + (1 - b2) * g * g
            mh = m[n][k] / (1 - b1 ** step)
            vh = v[n][k] / (1 - b2 ** step)
            master[n][k] = (master[n][k] - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32)
