"""Torch (GPU) ray caster for the procedural scenes of ``scenegen``.

The same world, shading and camera model as ``Scene.render`` in float64, but
run with torch on any device, so that training sets of hundreds of scenes
can be generated next to the network instead of on the host.  Like the rest
of the package it only makes inputs.  ``capture`` draws its depth noise and
invalid discs from a torch generator (same distributions as the numpy
``capture``; not the same random numbers).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import Camera, Scene

__all__ = ["render", "capture"]


def _hash3(ix, iy, iz, salt: int):
    h = (ix.to(torch.int64) * 73856093) ^ (iy.to(torch.int64) * 19349663) \
        ^ (iz.to(torch.int64) * 83492791) ^ (int(salt) * 2654435761)
    h = h & 0xFFFFFFFF
    h = ((h ^ (h >> 13)) * 1274126177) & 0xFFFFFFFF
    h = h ^ (h >> 16)
    return (h & 0xFFFF).to(torch.float64) / 65535.0


def _value_noise(p, scale: float, salt: int):
    q = p / scale
    i = torch.floor(q)
    f = q - i
    f = f * f * (3.0 - 2.0 * f)
    ix, iy, iz = i[:, 0], i[:, 1], i[:, 2]
    out = torch.zeros_like(f[:, 0])
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                wx = f[:, 0] if dx else 1.0 - f[:, 0]
                wy = f[:, 1] if dy else 1.0 - f[:, 1]
                wz = f[:, 2] if dz else 1.0 - f[:, 2]
                out = out + wx * wy * wz * _hash3(ix + dx, iy + dy, iz + dz, salt)
    return out


def _intersect(scene: Scene, o, d):
    dev = d.device
    n = d.shape[0]
    inf = torch.tensor(math.inf, dtype=torch.float64, device=dev)
    tbest = torch.full((n,), math.inf, dtype=torch.float64, device=dev)
    nrm = torch.zeros((n, 3), dtype=torch.float64, device=dev)
    pid = torch.full((n,), -1, dtype=torch.int32, device=dev)

    def take(t, normal, ident):
        m = (t > 1e-6) & (t < tbest)
        tbest[m] = t[m]
        nrm[m] = normal[m] if normal.dim() == 2 else normal
        pid[m] = ident

    o_t = torch.tensor(o, dtype=torch.float64, device=dev)
    if scene.ground_y is not None:
        t = (scene.ground_y - o[1]) / d[:, 1]
        t = torch.where(torch.isfinite(t), t, inf)
        take(t, torch.tensor([0.0, 1.0, 0.0], dtype=torch.float64, device=dev), 0)
    if scene.backdrop_radius is not None:
        a = d[:, 0] ** 2 + d[:, 2] ** 2
        b = 2.0 * (o[0] * d[:, 0] + o[2] * d[:, 2])
        c = o[0] ** 2 + o[2] ** 2 - scene.backdrop_radius ** 2
        disc = b * b - 4 * a * c
        t = (-b + torch.sqrt(torch.clamp_min(disc, 0.0))) / (2 * a)
        t = torch.where((disc >= 0) & (a > 0), t, inf)
        p = o_t + t[:, None] * d
        normal = torch.stack([-p[:, 0], torch.zeros_like(p[:, 0]), -p[:, 2]], 1)
        normal = normal / torch.clamp_min(torch.linalg.norm(normal, dim=1, keepdim=True), 1e-12)
        take(t, normal, 1)
    for k, (c0, r, _col) in enumerate(scene.spheres):
        c0t = torch.tensor(c0, dtype=torch.float64, device=dev)
        oc = o_t - c0t
        a = (d * d).sum(1)
        b = 2.0 * (d @ oc)
        c = float(oc @ oc) - r * r
        disc = b * b - 4 * a * c
        sq = torch.sqrt(torch.clamp_min(disc, 0.0))
        t1 = (-b - sq) / (2 * a)
        t2 = (-b + sq) / (2 * a)
        t = torch.where(t1 > 1e-6, t1, t2)
        t = torch.where(disc >= 0, t, inf)
        p = o_t + t[:, None] * d
        take(t, (p - c0t) / r, 2 + k)
    base = 2 + len(scene.spheres)
    ar = torch.arange(n, device=dev)
    for k, (c0, half, yaw, _col) in enumerate(scene.boxes):
        cy, sy = math.cos(yaw), math.sin(yaw)
        Ry = torch.tensor([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]], dtype=torch.float64, device=dev)
        halft = torch.tensor(half, dtype=torch.float64, device=dev)
        ol = Ry.T @ (o_t - torch.tensor(c0, dtype=torch.float64, device=dev))
        dl = d @ Ry
        inv = 1.0 / dl
        t0 = (-halft - ol) * inv
        t1 = (halft - ol) * inv
        tmin = torch.minimum(t0, t1)
        tmax = torch.maximum(t0, t1)
        tmin = torch.where(torch.isnan(tmin), -inf, tmin)
        tmax = torch.where(torch.isnan(tmax), inf, tmax)
        tn = tmin.max(1).values
        tf = tmax.min(1).values
        hit = (tn <= tf) & (tf > 1e-6)
        t = torch.where(hit, torch.where(tn > 1e-6, tn, tf), inf)
        axis = torch.argmax(tmin, 1)
        nl = torch.zeros((n, 3), dtype=torch.float64, device=dev)
        nl[ar, axis] = -torch.sign(dl[ar, axis])
        take(t, nl @ Ry.T, base + k)
    return tbest, nrm, pid


def _shade(scene: Scene, p, nrm, pid):
    dev = p.device
    n = p.shape[0]
    base = torch.zeros((n, 3), dtype=torch.float64, device=dev)
    cols = {0: (0.55, 0.5, 0.42), 1: (0.45, 0.55, 0.65)}
    for k, (_c, _r, col) in enumerate(scene.spheres):
        cols[2 + k] = tuple(col)
    b0 = 2 + len(scene.spheres)
    for k, (_c, _h, _y, col) in enumerate(scene.boxes):
        cols[b0 + k] = tuple(col)
    for ident, col in cols.items():
        base[pid == ident] = torch.tensor(col, dtype=torch.float64, device=dev)
    chk = torch.remainder(torch.floor(p[:, 0] / 0.25) + torch.floor(p[:, 1] / 0.25) + torch.floor(p[:, 2] / 0.25), 2)
    tex = (0.75 + 0.25 * chk) * (0.55 + 0.45 * _value_noise(p, 0.07, scene.salt))
    tex = tex * (0.8 + 0.2 * _value_noise(p, 0.013, scene.salt + 1))
    light = np.array([0.3, 1.0, -0.5])
    light /= np.linalg.norm(light)
    lam = 0.35 + 0.65 * torch.clamp(nrm @ torch.tensor(light, dtype=torch.float64, device=dev), 0.0, 1.0)
    rgb = base * (tex * lam)[:, None]
    sky = torch.tensor(np.array(scene.sky_rgb) / 255.0, dtype=torch.float64, device=dev)
    rgb = torch.where((pid >= 0)[:, None], rgb, sky)
    return torch.clamp(torch.floor(rgb * 255.0 + 0.5), 0, 255).to(torch.uint8)


def render(scene: Scene, cam: Camera, device="cuda", chunk_rows: int = 0):
    """Ray-cast ``cam`` on ``device``: (rgb uint8 (H,W,3), zdepth float64
    (H,W), inf where nothing is hit)."""
    H, W = cam.height, cam.width
    Rt = torch.tensor(cam.R.T, dtype=torch.float64, device=device)
    o = cam.center
    rows = chunk_rows or max(1, (1 << 21) // W)
    rgb = torch.empty((H, W, 3), dtype=torch.uint8, device=device)
    z = torch.empty((H, W), dtype=torch.float64, device=device)
    for y0 in range(0, H, rows):
        y1 = min(H, y0 + rows)
        jj, ii = torch.meshgrid(torch.arange(y0, y1, dtype=torch.float64, device=device),
                                torch.arange(W, dtype=torch.float64, device=device), indexing="ij")
        dc = torch.stack([(ii - cam.cx) / cam.fx, (jj - cam.cy) / cam.fy, torch.ones_like(ii)], -1).reshape(-1, 3)
        dw = dc @ Rt.T
        t, nrm, pid = _intersect(scene, o, dw)
        p = torch.as_tensor(o, dtype=torch.float64, device=device) + torch.where(torch.isfinite(t), t, 0.0)[:, None] * dw
        rgb[y0:y1] = _shade(scene, p, nrm, pid).reshape(y1 - y0, W, 3)
        z[y0:y1] = t.reshape(y1 - y0, W)
    return rgb, z


def capture(scene: Scene, cam: Camera, gen: torch.Generator, noise_k=0.0, invalid_frac=0.0,
            disc_radius=(4.0, 24.0), device="cuda"):
    """Colour + millimetre depth (uint16 as int32 -> torch.int16 view) of one
    source camera on ``device``; invalid pixels as discs of random radius
    covering about ``invalid_frac`` of the image."""
    rgb, z = render(scene, cam, device)
    H, W = z.shape
    valid = torch.isfinite(z)
    zn = torch.where(valid, z, torch.zeros_like(z))
    if noise_k > 0:
        zn = zn + noise_k * zn * zn * torch.randn(z.shape, generator=gen, dtype=torch.float64).to(device)
    if invalid_frac > 0:
        r_mean = (disc_radius[0] + disc_radius[1]) / 2.0
        n_disc = max(1, int(round(invalid_frac * H * W / (math.pi * r_mean * r_mean))))
        cx = torch.rand(n_disc, generator=gen, dtype=torch.float64) * W
        cy = torch.rand(n_disc, generator=gen, dtype=torch.float64) * H
        rr = disc_radius[0] + torch.rand(n_disc, generator=gen, dtype=torch.float64) * (disc_radius[1] - disc_radius[0])
        yy = torch.arange(H, dtype=torch.float64, device=device)[:, None]
        xx = torch.arange(W, dtype=torch.float64, device=device)[None, :]
        hole = torch.zeros((H, W), dtype=torch.bool, device=device)
        for q in range(n_disc):
            hole |= (xx - float(cx[q])) ** 2 + (yy - float(cy[q])) ** 2 <= float(rr[q]) ** 2
        valid &= ~hole
    mm = torch.clamp(torch.floor(zn * 1000.0 + 0.5), 1, 65535)
    depth = torch.where(valid, mm, torch.zeros_like(mm)).to(torch.int32)
    return rgb, depth
