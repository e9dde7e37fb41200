"""Seeded synthetic workloads for the Gaussian-splatting mapping step.

The paper evaluates on Replica, TUM-RGBD and EuRoC (Sec. IV-A); none of them is
available here, so every input is drawn from a seeded generator with the
shapes, resolutions and value distributions of the five benchmark workloads
(one small render check, one 100k-Gaussian forward/backward, one 300k-Gaussian
mapping iteration on a structured point cloud, one 8-keyframe batch and one
16-keyframe stress case).  Point clouds imitate the output of the SLAM module
(Sec. III-A): points on planar surfaces with depth noise along the viewing ray.

This module holds input recipes only (distributions, shapes, camera poses).
Both the HIP path and the CPU oracle consume its output; it contains none of
the rasteriser's arithmetic.  The single constant below converts a drawn
display colour into the coefficient of the constant spherical harmonic so that
the degree-0 mode renders exactly that colour (RGB colour, Sec. III-B).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# Value of the l=0 real spherical harmonic, 1/(2*sqrt(pi)).
SH_C0 = 0.5 / math.sqrt(math.pi)


@dataclasses.dataclass
class Camera:
    """Pinhole camera.  R, t map world to camera (x right, y down, z forward)."""
    R: np.ndarray
    t: np.ndarray
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    @property
    def centre(self) -> np.ndarray:
        return -self.R.T @ self.t


@dataclasses.dataclass
class Scene:
    means: np.ndarray           # [N,3] f32
    log_scales: np.ndarray      # [N,3] f32
    quats: np.ndarray           # [N,4] f32, (w,x,y,z), not necessarily unit
    opacity_logits: np.ndarray  # [N]   f32
    sh_dc: np.ndarray           # [N,3] f32
    sh_rest: np.ndarray         # [N,K-1,3] f32 (K=(D+1)^2; shape [N,0,3] at D=0)
    sh_degree: int
    cameras: List[Camera]
    targets: Optional[List[np.ndarray]]  # per view [3,H,W] f32, or None
    name: str = ""
    work: str = "fwd"           # "fwd", "fwd+bwd", "fwd+bwd+adam"
    checkpoint: bool = False
    tile_size: int = 16
    lrs: Optional[dict] = None

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def n_views(self) -> int:
        return len(self.cameras)

    @property
    def total_pixels(self) -> int:
        return int(sum(c.width * c.height for c in self.cameras))

    def sh_full(self) -> np.ndarray:
        """[N,K,3] with the DC coefficient first."""
        return np.concatenate([self.sh_dc[:, None, :], self.sh_rest], axis=1)


# Per-group Adam learning rates: position and scale rates are the ones stated
# for the 300k-Gaussian mapping iteration; the others are the 3DGS defaults the
# paper adopts (Sec. IV-A, "default optimization configuration of 3DGS").
DEFAULT_LRS = {
    "means": 1.6e-4,
    "log_scales": 5e-3,
    "quats": 1e-3,
    "opacity_logits": 5e-2,
    "sh_dc": 2.5e-3,
    "sh_rest": 2.5e-3 / 20.0,
}


def _rngs(seed: int, k: int = 8):
    ss = np.random.SeedSequence(seed)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(k)]


def random_unit_quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def sh_coeffs(rng, rgb, degree, sigma_rest=0.2):
    """DC chosen so the degree-0 colour is `rgb`; higher bands N(0, sigma_rest)."""
    dc = (rgb - 0.5) / SH_C0
    k = (degree + 1) ** 2
    rest = rng.normal(0.0, sigma_rest, size=(rgb.shape[0], k - 1, 3))
    return dc, rest


def look_at(centre, target=(0.0, 0.0, 0.0), down=(0.0, 1.0, 0.0)):
    """World->camera rotation/translation for a camera at `centre` facing `target`."""
    c = np.asarray(centre, np.float64)
    z = np.asarray(target, np.float64) - c
    z /= np.linalg.norm(z)
    x = np.cross(np.asarray(down, np.float64), z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z])
    return R, -R @ c


def pinhole(width, height, f, R=None, t=None):
    R = np.eye(3) if R is None else R
    t = np.zeros(3) if t is None else t
    return Camera(np.asarray(R, np.float64), np.asarray(t, np.float64), float(f), float(f),
                  width / 2.0, height / 2.0, int(width), int(height))


def plane_point_cloud(rng, n, n_planes, ray_origin, room=2.0, noise=0.01):
    """Points on `n_planes` random planes clipped to the cube [-room, room]^3.

    Each plane has a normal uniform on the sphere and passes through a point
    uniform in [-1.5,1.5]^3; points are uniform on plane-within-room (rejection
    sampling).  Colour: a per-plane base colour plus 0.2*sin stripes of period
    0.3 m, clipped to [0,1].  Depth noise N(0, noise) is applied along the ray
    from `ray_origin`.
    """
    per = [n // n_planes + (1 if p < n % n_planes else 0) for p in range(n_planes)]
    pts, cols = [], []
    half = room * math.sqrt(3.0)
    for p in range(n_planes):
        nrm = rng.standard_normal(3)
        nrm /= np.linalg.norm(nrm)
        p0 = rng.uniform(-1.5, 1.5, size=3)
        u = np.cross(nrm, [1.0, 0.0, 0.0] if abs(nrm[0]) < 0.9 else [0.0, 1.0, 0.0])
        u /= np.linalg.norm(u)
        w = np.cross(nrm, u)
        base = rng.uniform(0.0, 1.0, size=3)
        got_p, got_a = [], []
        need = per[p]
        while need > 0:
            m = max(4 * need, 1024)
            ab = rng.uniform(-half, half, size=(m, 2))
            x = p0 + ab[:, :1] * u + ab[:, 1:] * w
            ok = np.all(np.abs(x) <= room, axis=1)
            x, a = x[ok][:need], ab[ok, 0][:need]
            got_p.append(x)
            got_a.append(a)
            need -= x.shape[0]
        x = np.concatenate(got_p)
        a = np.concatenate(got_a)
        stripe = 0.2 * np.sin(2.0 * math.pi * a / 0.3)
        cols.append(np.clip(base[None, :] + stripe[:, None], 0.0, 1.0))
        pts.append(x)
    pts = np.concatenate(pts)
    cols = np.concatenate(cols)
    d = pts - np.asarray(ray_origin, np.float64)[None, :]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    pts = pts + rng.normal(0.0, noise, size=(pts.shape[0], 1)) * d
    return pts, cols


def arc_cameras(rng, sizes):
    """Cameras on a 1 m arc (sin th, 0, -cos th), th ~ U(-45deg, 45deg), facing the origin.

    `sizes` is a list of (width, height, f); the principal point is the image centre.
    """
    cams = []
    for (w, h, f) in sizes:
        th = math.radians(rng.uniform(-45.0, 45.0))
        R, t = look_at((math.sin(th), 0.0, -math.cos(th)))
        cams.append(pinhole(w, h, f, R, t))
    return cams


def tracked_keyframe(seed, W, H, n):
    """A keyframe's tracked pixels and image for point-cloud densification: n distinct pixels at
    uniform random positions (integer xy) with the depths of a tilted plane plus N(0, 0.01) noise,
    and an image that is smooth (a product of sines) except for six vertical steps of +0.2, so both
    outcomes of a gradient test occur.  Returns xy int32 [n, 2], depth f32 [n], image f32 [3, H, W]."""
    rng = np.random.default_rng(seed)
    flat = rng.choice(W * H, n, replace=False)
    xy = np.stack([flat % W, flat // W], 1).astype(np.int32)
    depth = (2.0 + 0.002 * xy[:, 0] - 0.001 * xy[:, 1] + 0.01 * rng.standard_normal(n)).astype(np.float32)
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float32)
    base = 0.5 + 0.1 * np.sin(xx / 37.0) * np.cos(yy / 29.0)
    img = np.stack([base, base * 0.9, base * 1.1]).astype(np.float32)
    for x0 in rng.choice(W - 2, 6, replace=False):
        img[:, :, x0 + 1:] += 0.2
    return xy, depth, np.clip(img, 0.0, 1.0).astype(np.float32)


def _f32(*arrs):
    return [np.ascontiguousarray(a, dtype=np.float32) for a in arrs]


def make_scene(seed, n, sh_degree, cameras, means_kind="box", n_planes=6, ray_origin=None,
               log_scale_mu=-4.0, log_scale_sigma=0.7, logit_sigma=1.5,
               transparent_frac=0.0, targets=True, **meta):
    """Generic seeded scene.  `means_kind`: "box" (x,y in [-1,1], z in [2,5]) or "planes"."""
    r = _rngs(seed, 8)
    if means_kind == "box":
        means = np.stack([r[0].uniform(-1, 1, n), r[0].uniform(-1, 1, n), r[0].uniform(2, 5, n)], 1)
        rgb = r[4].uniform(0.0, 1.0, size=(n, 3))
    elif means_kind == "planes":
        origin = cameras[0].centre if ray_origin is None else ray_origin
        means, rgb = plane_point_cloud(r[0], n, n_planes, origin)
    else:
        raise ValueError(means_kind)
    log_scales = r[1].normal(log_scale_mu, log_scale_sigma, size=(n, 3))
    quats = random_unit_quats(r[2], n)
    logits = r[3].normal(0.0, logit_sigma, size=n)
    if transparent_frac > 0:
        k = int(round(transparent_frac * n))
        idx = r[3].choice(n, size=k, replace=False)
        o = r[3].uniform(0.001, 0.02, size=k)
        logits[idx] = np.log(o / (1.0 - o))
    dc, rest = sh_coeffs(r[5], rgb, sh_degree)
    tg = None
    if targets:
        tg = [r[6].uniform(0.0, 1.0, size=(3, c.height, c.width)).astype(np.float32) for c in cameras]
    means, log_scales, quats, logits, dc, rest = _f32(means, log_scales, quats, logits, dc, rest)
    return Scene(means, log_scales, quats, logits, dc, rest, sh_degree, cameras, tg, **meta)


WORKLOADS = {
    1: "render-1k-128x96",
    2: "fwdbwd-100k-640x480-sh3",
    3: "iter-300k-1200x680-planes6",
    4: "batch8-500k-mixed-planes10",
    5: "stress16-2m-1200x680-ckpt",
}


def make_config(idx: int, seed: Optional[int] = None, n: Optional[int] = None,
                res_div: int = 1, n_views: Optional[int] = None) -> Scene:
    """The five benchmark workloads (1..5).  `n`, `res_div` and `n_views`
    shrink a workload for quick parity runs while keeping its recipe."""
    seed = idx if seed is None else seed

    def cam(w, h, f, R=None, t=None):
        return pinhole(w // res_div, h // res_div, f / res_div, R, t)

    if idx == 1:
        cams = [cam(128, 96, 100.0)]
        return make_scene(seed, n or 1000, 0, cams, "box", log_scale_mu=-3.0, log_scale_sigma=0.5,
                          logit_sigma=1.0, targets=False, name=WORKLOADS[1], work="fwd")
    if idx == 2:
        cams = [cam(640, 480, 525.0)]
        return make_scene(seed, n or 100_000, 3, cams, "box", log_scale_mu=-4.0, log_scale_sigma=0.7,
                          logit_sigma=1.5, name=WORKLOADS[2], work="fwd+bwd")
    if idx == 3:
        cams = [cam(1200, 680, 600.0, np.eye(3), np.array([0.0, 0.0, 1.9]))]
        return make_scene(seed, n or 300_000, 3, cams, "planes", n_planes=6, name=WORKLOADS[3],
                          work="fwd+bwd+adam", lrs=dict(DEFAULT_LRS))
    if idx == 4:
        rc = _rngs(seed + 1000, 1)[0]
        sizes = [(640, 480, 525.0)] * 4 + [(752, 480, 460.0)] * 2 + [(1200, 680, 600.0)] * 2
        sizes = [(w // res_div, h // res_div, f / res_div) for (w, h, f) in sizes]
        cams = arc_cameras(rc, sizes)
        if n_views is not None:
            cams = cams[:n_views]
        return make_scene(seed, n or 500_000, 3, cams, "planes", n_planes=10, name=WORKLOADS[4],
                          work="fwd+bwd")
    if idx == 5:
        rc = _rngs(seed + 1000, 1)[0]
        nv = 16 if n_views is None else n_views
        cams = arc_cameras(rc, [(1200 // res_div, 680 // res_div, 600.0 / res_div)] * nv)
        return make_scene(seed, n or 2_000_000, 3, cams, "planes", n_planes=10, log_scale_sigma=1.0,
                          transparent_frac=0.2, name=WORKLOADS[5], work="fwd+bwd+adam",
                          checkpoint=True, lrs=dict(DEFAULT_LRS))
    raise ValueError(f"unknown workload {idx}")
