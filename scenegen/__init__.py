"""Seeded synthetic multiview-plus-depth (MVD) scenes.

This module only *makes inputs*: camera rigs, procedural scenes, ray-cast
colour and depth frames, virtual-camera trajectories and ground-truth renders.
It holds none of the view-synthesis arithmetic, and both the CPU oracle and the
HIP path consume what it produces.

The paper's recordings (nine stereo cameras on a 60 degree arc, Section IX) are
not available, so every workload is a procedural world ray-cast in float64:

* a ground plane, an optional cylindrical backdrop (so rays always hit
  something), spheres and yaw-rotated boxes;
* colour = per-primitive base colour x checker x value noise x Lambertian
  shading, quantised to RGB8;
* depth = exact Z-depth (along the optical axis, the quantity the paper's
  depth maps and its disparity mapping work on, Section V-A) plus Gaussian
  noise sigma = k * z**2 drawn from a counter-based Philox stream keyed by
  (seed, camera), then round(1000 * z) millimetres clamped to [1, 65535];
  invalid pixels hold 0.

Camera convention (pinhole, no distortion): OpenCV axes (x right, y down,
z forward), world->camera X_c = R X_w + t, pixel centres at integer
coordinates.  World axes: y up.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Camera", "look_at", "arc_camera", "Scene", "Frame", "Workload",
    "random_scene", "config1", "config2", "config3", "config_small",
    "swing_trajectory", "moving_scenes", "BG_MM", "capture_layered", "background_model", "background_scene",
]


# --------------------------------------------------------------------------
# cameras
# --------------------------------------------------------------------------
@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray            # (3,3) world->camera rotation
    t: np.ndarray            # (3,) world->camera translation, metres
    depth_alpha: float = 0.0  # quadratic depth-correction coefficients (Eq. 1);
    depth_beta: float = 1.0   # (0, 1) is the identity

    def __post_init__(self):
        # the boundary carries float32; keep the generator's copy identical
        self.R = np.asarray(self.R, np.float32).astype(np.float64)
        self.t = np.asarray(self.t, np.float32).astype(np.float64)
        for k in ("fx", "fy", "cx", "cy", "depth_alpha", "depth_beta"):
            setattr(self, k, float(np.float32(getattr(self, k))))

    @property
    def center(self) -> np.ndarray:
        return -self.R.T @ self.t

    def with_size(self, width: int, height: int, focal_scale: float) -> "Camera":
        """Same pose, new image size; focal lengths scaled, principal point centred."""
        return replace(self, width=width, height=height,
                       fx=self.fx * focal_scale, fy=self.fy * focal_scale,
                       cx=(width - 1) / 2.0, cy=(height - 1) / 2.0)

    def as_tuple(self):
        """Flat field tuple in boundary order: w, h, fx, fy, cx, cy, R[9], t[3], alpha, beta."""
        return (self.width, self.height, self.fx, self.fy, self.cx, self.cy,
                tuple(float(v) for v in self.R.reshape(-1)),
                tuple(float(v) for v in self.t.reshape(-1)),
                self.depth_alpha, self.depth_beta)


def look_at(eye, target, up=(0.0, 1.0, 0.0)) -> Tuple[np.ndarray, np.ndarray]:
    """World->camera (R, t) for a camera at ``eye`` looking at ``target``
    (OpenCV axes: image y points along world -up)."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    x = np.cross(f, np.asarray(up, np.float64))
    x /= np.linalg.norm(x)
    y = np.cross(f, x)
    R = np.stack([x, y, f])
    return R, -R @ eye


def _fx_for_hfov(width: int, hfov_deg: float) -> float:
    return (width / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)


def arc_camera(angle_deg: float, radius: float, width: int, height: int,
               hfov_deg: float = 60.0, height_m: float = 0.2,
               center=(0.0, 0.0, 0.0)) -> Camera:
    """Camera on a horizontal arc about ``center`` looking at it.
    Angle 0 sits on the -z side; positive angles move towards +x."""
    a = math.radians(angle_deg)
    c = np.asarray(center, np.float64)
    eye = c + np.array([radius * math.sin(a), height_m, -radius * math.cos(a)])
    R, t = look_at(eye, c)
    f = _fx_for_hfov(width, hfov_deg)
    return Camera(width, height, f, f, (width - 1) / 2.0, (height - 1) / 2.0, R, t)


def swing_trajectory(n_frames: int, a0: float, a1: float, radius: float,
                     width: int, height: int, hfov_deg: float = 60.0,
                     height_m: float = 0.2) -> List[Camera]:
    """Virtual cameras sweeping the arc from a0 to a1 degrees (the 'swing'
    navigation of the subjective tests, Section IX)."""
    if n_frames == 1:
        angles = [0.5 * (a0 + a1)]
    else:
        angles = [a0 + (a1 - a0) * k / (n_frames - 1) for k in range(n_frames)]
    return [arc_camera(a, radius, width, height, hfov_deg, height_m) for a in angles]


# --------------------------------------------------------------------------
# procedural texture
# --------------------------------------------------------------------------
def _hash3(ix, iy, iz, salt):
    h = (ix.astype(np.int64) * 73856093) ^ (iy.astype(np.int64) * 19349663) \
        ^ (iz.astype(np.int64) * 83492791) ^ (np.int64(salt) * 2654435761)
    h = h & 0xFFFFFFFF
    h = (h ^ (h >> 13)) * 1274126177 & 0xFFFFFFFF
    h = h ^ (h >> 16)
    return (h & 0xFFFF).astype(np.float64) / 65535.0


def _value_noise(p, scale, salt):
    q = p / scale
    i = np.floor(q)
    f = q - i
    f = f * f * (3.0 - 2.0 * f)
    ix, iy, iz = i[..., 0], i[..., 1], i[..., 2]
    out = 0.0
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                wx = f[..., 0] if dx else 1.0 - f[..., 0]
                wy = f[..., 1] if dy else 1.0 - f[..., 1]
                wz = f[..., 2] if dz else 1.0 - f[..., 2]
                out = out + wx * wy * wz * _hash3(ix + dx, iy + dy, iz + dz, salt)
    return out


# --------------------------------------------------------------------------
# scene
# --------------------------------------------------------------------------
@dataclass
class Scene:
    ground_y: Optional[float] = -0.8
    backdrop_radius: Optional[float] = 5.0      # vertical cylinder about the origin
    spheres: List[Tuple[np.ndarray, float, np.ndarray]] = field(default_factory=list)
    boxes: List[Tuple[np.ndarray, np.ndarray, float, np.ndarray]] = field(default_factory=list)
    sky_rgb: Tuple[int, int, int] = (40, 60, 90)
    salt: int = 0

    # ---- ray casting --------------------------------------------------------
    def _intersect(self, o, d):
        """o: (3,), d: (N,3) unnormalised (camera z component = 1).  Returns
        t (N,) ray parameter of the nearest hit (inf if none), normal (N,3),
        primitive id (N,) (-1 none, 0 ground, 1 backdrop, 2.. objects)."""
        n = d.shape[0]
        tbest = np.full(n, np.inf)
        nrm = np.zeros((n, 3))
        pid = np.full(n, -1, np.int32)

        def take(t, normal, ident):
            m = (t > 1e-6) & (t < tbest)
            tbest[m] = t[m]
            nrm[m] = normal[m] if normal.ndim == 2 else normal
            pid[m] = ident

        if self.ground_y is not None:
            with np.errstate(divide="ignore", invalid="ignore"):
                t = (self.ground_y - o[1]) / d[:, 1]
            t = np.where(np.isfinite(t), t, np.inf)
            take(t, np.array([0.0, 1.0, 0.0]), 0)
        if self.backdrop_radius is not None:
            a = d[:, 0] ** 2 + d[:, 2] ** 2
            b = 2.0 * (o[0] * d[:, 0] + o[2] * d[:, 2])
            c = o[0] ** 2 + o[2] ** 2 - self.backdrop_radius ** 2
            disc = b * b - 4 * a * c
            with np.errstate(invalid="ignore", divide="ignore"):
                t = (-b + np.sqrt(np.maximum(disc, 0.0))) / (2 * a)   # far root: inside surface
            t = np.where((disc >= 0) & (a > 0), t, np.inf)
            p = o + t[:, None] * d
            normal = np.stack([-p[:, 0], np.zeros(n), -p[:, 2]], 1)
            normal /= np.maximum(np.linalg.norm(normal, axis=1, keepdims=True), 1e-12)
            take(t, normal, 1)
        for k, (c0, r, _col) in enumerate(self.spheres):
            oc = o - c0
            a = np.einsum("ij,ij->i", d, d)
            b = 2.0 * (d @ oc)
            c = oc @ oc - r * r
            disc = b * b - 4 * a * c
            sq = np.sqrt(np.maximum(disc, 0.0))
            t1 = (-b - sq) / (2 * a)
            t2 = (-b + sq) / (2 * a)
            t = np.where(t1 > 1e-6, t1, t2)
            t = np.where(disc >= 0, t, np.inf)
            p = o + t[:, None] * d
            normal = (p - c0) / r
            take(t, normal, 2 + k)
        base = 2 + len(self.spheres)
        for k, (c0, half, yaw, _col) in enumerate(self.boxes):
            cy, sy = math.cos(yaw), math.sin(yaw)
            Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])   # box->world
            ol = Ry.T @ (o - c0)
            dl = d @ Ry            # = (Ry.T @ d.T).T
            with np.errstate(divide="ignore", invalid="ignore"):
                inv = 1.0 / dl
                t0 = (-half - ol) * inv
                t1 = (half - ol) * inv
            tmin = np.minimum(t0, t1)
            tmax = np.maximum(t0, t1)
            tmin = np.where(np.isnan(tmin), -np.inf, tmin)
            tmax = np.where(np.isnan(tmax), np.inf, tmax)
            tn = tmin.max(1)
            tf = tmax.min(1)
            hit = (tn <= tf) & (tf > 1e-6)
            t = np.where(hit, np.where(tn > 1e-6, tn, tf), np.inf)
            axis = np.argmax(tmin, 1)
            nl = np.zeros((n, 3))
            nl[np.arange(n), axis] = -np.sign(dl[np.arange(n), axis])
            take(t, nl @ Ry.T, base + k)
        return tbest, nrm, pid

    def _shade(self, p, nrm, pid):
        n = p.shape[0]
        base = np.zeros((n, 3))
        base[pid == 0] = (0.55, 0.5, 0.42)
        base[pid == 1] = (0.45, 0.55, 0.65)
        for k, (_c, _r, col) in enumerate(self.spheres):
            base[pid == 2 + k] = col
        b0 = 2 + len(self.spheres)
        for k, (_c, _h, _y, col) in enumerate(self.boxes):
            base[pid == b0 + k] = col
        chk = (np.floor(p[:, 0] / 0.25) + np.floor(p[:, 1] / 0.25) + np.floor(p[:, 2] / 0.25)) % 2
        tex = (0.75 + 0.25 * chk) * (0.55 + 0.45 * _value_noise(p, 0.07, self.salt))
        tex = tex * (0.8 + 0.2 * _value_noise(p, 0.013, self.salt + 1))
        light = np.array([0.3, 1.0, -0.5])
        light /= np.linalg.norm(light)
        lam = 0.35 + 0.65 * np.clip(nrm @ light, 0.0, 1.0)
        rgb = base * (tex * lam)[:, None]
        rgb = np.where((pid >= 0)[:, None], rgb, np.array(self.sky_rgb) / 255.0)
        return np.clip(np.floor(rgb * 255.0 + 0.5), 0, 255).astype(np.uint8)

    def render(self, cam: Camera, rows: Optional[slice] = None):
        """Ray-cast ``cam``.  Returns (rgb uint8 (H,W,3), zdepth float64 (H,W),
        primitive id int32 (H,W)); zdepth is inf where nothing is hit."""
        H, W = cam.height, cam.width
        out_rgb = np.empty((H, W, 3), np.uint8)
        out_z = np.empty((H, W))
        out_id = np.empty((H, W), np.int32)
        Rt = cam.R.T
        o = cam.center
        step = max(1, 262144 // W)
        for y0 in range(0, H, step):
            y1 = min(H, y0 + step)
            jj, ii = np.mgrid[y0:y1, 0:W]
            dc = np.stack([(ii - cam.cx) / cam.fx, (jj - cam.cy) / cam.fy,
                           np.ones(ii.shape)], -1).reshape(-1, 3)
            dw = dc @ Rt.T
            t, nrm, pid = self._intersect(o, dw)
            p = o + np.where(np.isfinite(t), t, 0.0)[:, None] * dw
            out_rgb[y0:y1] = self._shade(p, nrm, pid).reshape(y1 - y0, W, 3)
            out_z[y0:y1] = t.reshape(y1 - y0, W)   # camera z of d is 1, so t is Z-depth
            out_id[y0:y1] = pid.reshape(y1 - y0, W)
        return out_rgb, out_z, out_id


def random_scene(rng: np.random.Generator, n_spheres=3, n_boxes=3, radius=0.8,
                 ground_y=-0.8, backdrop=5.0, salt=0) -> Scene:
    """Boxes and spheres placed within ``radius`` metres of the origin."""
    sph, box = [], []
    for _ in range(n_spheres):
        r = rng.uniform(0.15, 0.35)
        ang = rng.uniform(0, 2 * math.pi)
        rad = rng.uniform(0, radius - r)
        c = np.array([rad * math.cos(ang), rng.uniform(ground_y + r, 0.5), rad * math.sin(ang)])
        sph.append((c, r, rng.uniform(0.3, 1.0, 3)))
    for _ in range(n_boxes):
        half = rng.uniform(0.1, 0.3, 3)
        ang = rng.uniform(0, 2 * math.pi)
        rad = rng.uniform(0, radius - half.max())
        c = np.array([rad * math.cos(ang), ground_y + half[1], rad * math.sin(ang)])
        box.append((c, half, rng.uniform(0, math.pi), rng.uniform(0.3, 1.0, 3)))
    return Scene(ground_y=ground_y, backdrop_radius=backdrop, spheres=sph, boxes=box, salt=salt)


def moving_scenes(scene: Scene, n_frames: int, amplitude: float = 0.15, period_frames: int = 30) -> List[Scene]:
    """A dynamic sequence of ``scene``: every sphere moves on a horizontal
    circle of radius ``amplitude`` metres through its starting point, with a
    small vertical bob (kept above the ground), one revolution every
    ``period_frames`` frames, so a sequence of that many frames loops without
    a jump; boxes and the background stay put.  Frame 0 is ``scene``."""
    out = []
    n = max(1, len(scene.spheres))
    for f in range(n_frames):
        a = 2.0 * math.pi * f / period_frames
        sph = []
        for k, (c0, r, col) in enumerate(scene.spheres):
            ph = 2.0 * math.pi * k / n
            d = amplitude * np.array([math.cos(a + ph) - math.cos(ph), 0.3 * math.sin(2.0 * a),
                                      math.sin(a + ph) - math.sin(ph)])
            c = np.asarray(c0, np.float64) + d
            if scene.ground_y is not None:
                c[1] = max(c[1], scene.ground_y + r)
            sph.append((c, r, col))
        out.append(replace(scene, spheres=sph))
    return out


# --------------------------------------------------------------------------
# frames
# --------------------------------------------------------------------------
@dataclass
class Frame:
    rgb: np.ndarray        # (H,W,3) uint8
    depth_mm: np.ndarray   # (H,W) uint16, 0 = invalid


def _disc_mask(rng, H, W, frac, rmin, rmax):
    m = np.zeros((H, W), bool)
    target = frac * H * W
    covered = 0
    while covered < target:
        r = rng.uniform(rmin, rmax)
        cx, cy = rng.uniform(0, W), rng.uniform(0, H)
        x0, x1 = int(max(0, cx - r - 1)), int(min(W, cx + r + 2))
        y0, y1 = int(max(0, cy - r - 1)), int(min(H, cy + r + 2))
        yy, xx = np.mgrid[y0:y1, x0:x1]
        sub = (xx - cx) ** 2 + (yy - cy) ** 2 <= r * r
        blk = m[y0:y1, x0:x1]
        covered += int((sub & ~blk).sum())
        blk |= sub
    return m


# background signal in millimetre depth maps: the capture side of the layered
# system removes background depth from the live stream (Section IV-B)
BG_MM = 0xFFFF


def capture(scene: Scene, cam: Camera, seed: int, cam_index: int, noise_k=0.0,
            invalid_frac=0.0, invalid_blobs=False, zrange=None) -> Frame:
    """Colour + millimetre depth of one source camera."""
    return _capture(scene, cam, seed, cam_index, noise_k, invalid_frac, invalid_blobs, zrange)[0]


def background_scene(scene: Scene) -> Scene:
    """The static part of a scene (ground and backdrop): the world the
    background model of each camera is computed from."""
    return replace(scene, spheres=[], boxes=[])


def background_model(scene: Scene, cam: Camera) -> np.ndarray:
    """Exact millimetre depth of the static background seen by ``cam``
    (0 where nothing is hit), as a calibration-time model would give it."""
    _, z, _ = background_scene(scene).render(cam)
    mm = np.clip(np.floor(np.where(np.isfinite(z), z, 0.0) * 1000.0 + 0.5), 1, BG_MM - 1)
    return np.where(np.isfinite(z), mm, 0).astype(np.uint16)


def capture_layered(scene: Scene, cam: Camera, seed: int, cam_index: int, noise_k=0.0,
                    invalid_frac=0.0, invalid_blobs=False) -> Frame:
    """Live frame of the layered system: colour everywhere; depth only on
    foreground pixels (objects), with the same noise and dropouts as
    ``capture``; pixels whose colour shows the background (ground, backdrop,
    sky) carry BG_MM.  The foreground/background classification is exact."""
    f, pid = _capture(scene, cam, seed, cam_index, noise_k, invalid_frac, invalid_blobs, None)
    depth = np.where(pid >= 2, f.depth_mm, BG_MM).astype(np.uint16)
    return Frame(f.rgb, depth)


def _capture(scene, cam, seed, cam_index, noise_k, invalid_frac, invalid_blobs, zrange):
    rgb, z, pid = scene.render(cam)
    rng = np.random.Generator(np.random.Philox(key=[seed & 0xFFFFFFFF, 0x5EED0000 + cam_index]))
    valid = np.isfinite(z)
    zn = np.where(valid, z, 0.0)
    if noise_k > 0:
        zn = zn + noise_k * zn * zn * rng.standard_normal(z.shape)
    if zrange is not None:
        valid &= (z >= zrange[0]) & (z <= zrange[1])
    if invalid_frac > 0:
        if invalid_blobs:
            valid &= ~_disc_mask(rng, cam.height, cam.width, invalid_frac, 4.0, 24.0)
        else:
            valid &= rng.random(z.shape) >= invalid_frac
    mm = np.clip(np.floor(zn * 1000.0 + 0.5), 1, 65535)
    depth = np.where(valid, mm, 0).astype(np.uint16)
    return Frame(rgb, depth), pid


@dataclass
class Workload:
    """A rig, one MVD frame per camera, and the virtual cameras to render."""
    name: str
    rig: List[Camera]
    frames: List[Frame]
    virtual: List[Camera]
    scene: Scene
    k_nearest: int = 3
    bg_models: Optional[List[np.ndarray]] = None   # layered workloads: per-camera background depth (mm)


def config1(seed: int = 0) -> Workload:
    """1 source camera 320x240 (fx=fy=300), ground plane 1.2 m below the
    camera which is pitched 15 deg down, 3 spheres at camera depth 1.5-3.5 m,
    depth outside [1, 4] m invalid, no noise.  Virtual camera: translated
    +0.10 m along the source x axis, then yawed +5 deg about its y axis."""
    rng = np.random.default_rng(seed)
    pitch = math.radians(15.0)
    # camera at world origin, forward tilted down by 15 deg
    fwd = np.array([0.0, -math.sin(pitch), math.cos(pitch)])
    R, t = look_at(np.zeros(3), fwd)
    src = Camera(320, 240, 300.0, 300.0, 159.5, 119.5, R, t)
    sph = []
    for _ in range(3):
        r = rng.uniform(0.3, 0.6)
        zc = rng.uniform(1.5, 3.5)
        xc = rng.uniform(-0.6, 0.6) * zc / 2.0
        yc = rng.uniform(-0.2, 0.3)
        pc = np.array([xc, yc, zc])            # camera frame
        sph.append((R.T @ (pc - t), r, rng.uniform(0.3, 1.0, 3)))
    scene = Scene(ground_y=-1.2, backdrop_radius=None, spheres=sph, salt=seed)
    frame = capture(scene, src, seed, 0, zrange=(1.0, 4.0))
    # virtual: translate +0.10 m along camera x, then yaw +5 deg about camera y
    yaw = math.radians(5.0)
    Ry = np.array([[math.cos(yaw), 0, math.sin(yaw)], [0, 1, 0], [-math.sin(yaw), 0, math.cos(yaw)]])
    c_src = src.center
    c_v = c_src + R.T @ np.array([0.10, 0.0, 0.0])
    Rv = Ry.T @ R          # camera axes rotated by +5 deg about the camera's own y
    tv = -Rv @ c_v
    virt = Camera(320, 240, 300.0, 300.0, 159.5, 119.5, Rv, tv)
    return Workload("c1_1cam_320x240", [src], [frame], [virt], scene, k_nearest=1)


def config2(seed: int = 0) -> Workload:
    """3 cameras 640x480 (hFOV 60 deg) on a 2 m arc at -15/0/+15 deg, boxes and
    spheres within 0.8 m of the centre, sigma = 0.002 z^2, 5% i.i.d. invalid;
    virtual cameras at arc angles 7.5 and 5 deg, output 640x480."""
    rng = np.random.default_rng(1000 + seed)
    scene = random_scene(rng, salt=seed)
    rig = [arc_camera(a, 2.0, 640, 480) for a in (-15.0, 0.0, 15.0)]
    frames = [capture(scene, c, seed, k, noise_k=0.002, invalid_frac=0.05) for k, c in enumerate(rig)]
    virt = [arc_camera(a, 2.0, 640, 480) for a in (7.5, 5.0)]
    return Workload("c2_3cam_640x480", rig, frames, virt, scene)


def config3(seed: int = 0, n_frames: int = 60, out_w: int = 1920, out_h: int = 1080,
            src_w: int = 1280, src_h: int = 720, layered: bool = False) -> Workload:
    """9 cameras 1280x720 (hFOV 60 deg) on a 2.5 m arc, -60..+60 deg every
    15 deg, sigma = 0.003 z^2, 10% invalid as discs of radius 4-24 px; a
    60-frame swing trajectory from -60 to +60 deg rendered at 1920x1080 with
    the same field of view (1.5x magnification).  layered: live depth on the
    objects only (background signalled) plus exact background models."""
    rng = np.random.default_rng(3000 + seed)
    scene = random_scene(rng, n_spheres=4, n_boxes=4, salt=seed)
    angles = [-60.0 + 15.0 * k for k in range(9)]
    rig = [arc_camera(a, 2.5, src_w, src_h) for a in angles]
    cap = capture_layered if layered else capture
    frames = [cap(scene, c, seed, k, noise_k=0.003, invalid_frac=0.10, invalid_blobs=True)
              for k, c in enumerate(rig)]
    virt = swing_trajectory(n_frames, -60.0, 60.0, 2.5, out_w, out_h)
    bgm = [background_model(scene, c) for c in rig] if layered else None
    return Workload("c3_9cam_1280x720_to_1920x1080" + ("_layered" if layered else ""), rig, frames, virt,
                    scene, bg_models=bgm)


def config_small(seed: int = 0, n_cams: int = 3, w: int = 96, h: int = 64,
                 out_w: int = 128, out_h: int = 80, n_virtual: int = 3,
                 noise_k: float = 0.002, invalid_frac: float = 0.05, layered: bool = False) -> Workload:
    """A scaled-down config-3-like rig for fast tests (several tiles and a
    ragged tail at small sizes)."""
    rng = np.random.default_rng(5000 + seed)
    scene = random_scene(rng, salt=seed)
    angles = [(-15.0 * (n_cams - 1) / 2.0) + 15.0 * k for k in range(n_cams)]
    rig = [arc_camera(a, 2.2, w, h) for a in angles]
    cap = capture_layered if layered else capture
    frames = [cap(scene, c, seed, k, noise_k=noise_k, invalid_frac=invalid_frac)
              for k, c in enumerate(rig)]
    virt = [arc_camera(a, 2.2, out_w, out_h) for a in
            np.linspace(angles[0] - 3.0, angles[-1] + 3.0, n_virtual)]
    bgm = [background_model(scene, c) for c in rig] if layered else None
    return Workload(f"small_{n_cams}cam_{w}x{h}" + ("_layered" if layered else ""), rig, frames, virt, scene,
                    bg_models=bgm)
