"""Training and evaluation driver of the learned path.

Leave-one-camera-out on seeded procedural scenes: for every scene, nine
1280x720 cameras on a 2.5 m arc (-60..+60 degrees every 15) are captured
(depth noise 0.003 z^2, 10 % invalid as discs); each camera j in turn is the
held-out view: the library warps the three nearest *other* cameras to j's
pose at 960x540 (focal lengths x 0.75) and the network learns to predict the
ray-cast image of that pose.  Every step trains on the nine held-out views of
one scene.  Scenes, stacks and targets are made on the GPU (scenegen.gpu +
fvv_make_stack); all network arithmetic runs in the library's kernels.

    python -m paper_2007_00558_amd.learned --train-scenes 500 --test-scenes 50 --steps 2000
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

import scenegen as sg

from . import (MEM_DEVICE, NET_ALIGN, NET_IN, PATH_LEARNED, PATH_PLAIN, Context, net_layers, net_param_count,
               pad8, params)

ANGLES = [-60.0 + 15.0 * k for k in range(9)]
SRC_W, SRC_H = 1280, 720
OUT_W, OUT_H = 960, 540
FOCAL = 0.75
TEST_SEED0 = 1_000_000      # test scenes never overlap training scenes


def init_params(seed: int) -> np.ndarray:
    """He-normal weights, zero biases, flattened in the library's order."""
    rng = np.random.default_rng(seed)
    out = []
    for name, kind, ci, co, k in net_layers():
        fan = k * k * ci
        std = math.sqrt(2.0 / fan) if kind != 2 else math.sqrt(1.0 / fan)
        out.append(rng.normal(0.0, std, co * k * k * ci).astype(np.float32))
        out.append(np.zeros(co, np.float32))
    flat = np.concatenate(out)
    assert flat.size == net_param_count()
    return flat


def rig():
    return [sg.arc_camera(a, 2.5, SRC_W, SRC_H) for a in ANGLES]


def held_out_views(cams):
    return [c.with_size(OUT_W, OUT_H, FOCAL) for c in cams]


class SceneSet:
    """One scene on the device: its frame set uploaded to the context, the
    nine leave-one-out stacks and the ray-cast targets (RGB8, padded rows
    zero)."""

    def __init__(self, ctx: Context, seed: int, device="cuda"):
        import torch
        from scenegen import gpu as sgg
        rng = np.random.default_rng(5000 + seed)
        self.scene = sg.random_scene(rng, n_spheres=4, n_boxes=4, salt=seed % 100000)
        self.cams = rig()
        gen = torch.Generator().manual_seed(7919 * seed + 1)
        frames = []
        for c in self.cams:
            rgb, d = sgg.capture(self.scene, c, gen, noise_k=0.003, invalid_frac=0.10, device=device)
            frames.append((rgb.contiguous(), d.to(torch.int16).contiguous()))
        ctx.upload_mvd(frames, mem=MEM_DEVICE)
        self.views = held_out_views(self.cams)
        self.ps = [params(exclude=(j,)) for j in range(len(self.cams))]
        self.Hp, self.Wp = pad8(OUT_H), pad8(OUT_W)
        n = len(self.views)
        self.stack = torch.empty((n, self.Hp, self.Wp, NET_IN), dtype=torch.int16, device=device)
        ctx.make_stack(self.views, self.ps, self.stack)
        self.target8 = torch.zeros((n, self.Hp, self.Wp, 3), dtype=torch.uint8, device=device)
        for j, v in enumerate(self.views):
            rgb, _ = sgg.render(self.scene, v, device)
            self.target8[j, :OUT_H, :OUT_W] = rgb
        torch.cuda.synchronize()


def psnr(a, b) -> float:
    import torch
    mse = torch.mean((a.to(torch.float64) - b.to(torch.float64)) ** 2).item()
    return 10.0 * math.log10(255.0 ** 2 / max(mse, 1e-12))


def evaluate(ctx: Context, seeds, device="cuda"):
    """Mean PSNR (dB) of the plain and learned paths over every held-out view."""
    import torch
    res = {"plain": [], "learned": []}
    for s in seeds:
        S = SceneSet(ctx, s, device)
        for j, v in enumerate(S.views):
            for name, path in (("plain", PATH_PLAIN), ("learned", PATH_LEARNED)):
                out = torch.empty((OUT_H, OUT_W, 3), dtype=torch.uint8, device=device)
                ctx.synthesize(v, out, params(exclude=(j,), path=path))
                res[name].append(psnr(out, S.target8[j, :OUT_H, :OUT_W]))
        torch.cuda.synchronize()
    return {k: float(np.mean(v)) for k, v in res.items()}, res


def train(ctx: Context, train_seeds, steps: int, lr: float = 1e-3, log_every: int = 50, cache: int = 0,
          log=print):
    """Adam with a cosine learning-rate decay; one scene (nine held-out
    views) per step.  Up to ``cache`` scenes stay on the device after their
    first use (stacks + RGB8 targets, about 0.3 GB each)."""
    import torch
    losses = []
    store = {}
    tgt = None
    t0 = time.time()
    for it in range(steps):
        seed = train_seeds[it % len(train_seeds)]
        S = store.get(seed)
        if S is None:
            S = SceneSet(ctx, seed)
            if len(store) < cache:
                store[seed] = S
        if tgt is None:
            tgt = torch.empty(S.target8.shape, dtype=torch.float32, device=S.target8.device)
        tgt.copy_(S.target8)
        tgt.mul_(1.0 / 255.0)
        lr_t = lr * 0.5 * (1.0 + math.cos(math.pi * it / max(1, steps)))
        loss = ctx.net_train_step(S.stack, tgt, len(S.views), S.Hp, S.Wp, OUT_H, lr=lr_t, apply=True,
                                  want_loss=(it % log_every == 0 or it == steps - 1))
        if loss is not None:
            losses.append((it, loss))
            log(f"step {it} loss {loss:.5f} lr {lr_t:.2e} cached {len(store)} {time.time() - t0:.1f}s", flush=True)
    torch.cuda.synchronize()
    return losses


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--train-scenes", type=int, default=500)
    ap.add_argument("--test-scenes", type=int, default=50)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cache", type=int, default=0, help="training scenes kept on the device")
    ap.add_argument("--init", default="", help="float32 .npy parameters to start from")
    ap.add_argument("--save", default="", help="write the trained parameters here (.npy)")
    ap.add_argument("--json", default="", help="write the summary here")
    a = ap.parse_args(argv)
    import torch
    torch.cuda.init()
    ctx = Context(0)
    ctx.set_rig(rig())
    p0 = np.load(a.init) if a.init else init_params(a.seed)
    ctx.net_load(p0)
    test = list(range(TEST_SEED0, TEST_SEED0 + a.test_scenes))
    t0 = time.time()
    losses = train(ctx, list(range(a.train_scenes)), a.steps, a.lr, cache=a.cache)
    t_train = time.time() - t0
    if a.save:
        np.save(a.save, ctx.net_read())
    t1 = time.time()
    mean, _ = evaluate(ctx, test)
    out = {"train_scenes": a.train_scenes, "test_scenes": a.test_scenes, "steps": a.steps,
           "samples": a.steps * len(ANGLES), "train_s": t_train, "eval_s": time.time() - t1,
           "psnr_plain_db": mean["plain"], "psnr_learned_db": mean["learned"],
           "psnr_gain_db": mean["learned"] - mean["plain"], "losses": losses}
    print(json.dumps({k: v for k, v in out.items() if k != "losses"}), flush=True)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(out, f, indent=1)
    ctx.close()


if __name__ == "__main__":
    main()
