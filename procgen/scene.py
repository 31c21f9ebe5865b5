"""Procedural HDR scenes, camera clips and noisy sample pools (inputs only).

Scene: 64 additive Gaussian blobs and 16 opaque star-shaped polygons drawn in
painter's order, every intensity lognormal(0, 1).  The world box is 1.25x the frame,
so a moving camera reveals new content at the frame edges (screen-edge
disocclusions).  The camera of frame t is a global rotation by omega*t about the frame
centre followed by a translation v*t.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# E[lognormal(0, 0.8)] = exp(0.8^2 / 2)
_LN_MEAN = math.exp(0.32)


@dataclasses.dataclass
class FrameData:
    truth: np.ndarray    # [H, W, 3] float64 HDR radiance (noise-free)
    albedo: np.ndarray   # [H, W, 3] float32
    normal: np.ndarray   # [H, W, 3] float32
    depth: np.ndarray    # [H, W]    float32
    mv: np.ndarray       # [H, W, 2] float32 backward motion (dx, dy) in pixels, to frame t-1
    valid: np.ndarray    # [H, W]    bool, the back-projected position lies in frame t-1

    @property
    def aux(self) -> np.ndarray:
        """[H, W, 8] float32 GBuffer features: albedo 3, normal 3, log-depth 1, zero pad 1."""
        H, W = self.depth.shape
        a = np.zeros((H, W, 8), np.float32)
        a[..., 0:3] = self.albedo
        a[..., 3:6] = self.normal
        a[..., 6] = np.log(self.depth) / math.log(20.0)
        return a


def make_scene(seed: int, H: int, W: int, n_blobs: int = 64, n_polys: int = 16) -> dict:
    rng = np.random.default_rng([int(seed), 0x5CE7E])
    cx, cy = W / 2.0, H / 2.0
    ex, ey = 0.625 * W, 0.625 * H
    blobs = dict(
        centre=np.stack([rng.uniform(cx - ex, cx + ex, n_blobs),
                         rng.uniform(cy - ey, cy + ey, n_blobs)], 1),
        sigma=rng.uniform(0.015, 0.12, n_blobs) * H,
        rgb=rng.lognormal(0.0, 1.0, (n_blobs, 1)) * rng.uniform(0.2, 1.0, (n_blobs, 3)),
    )
    polys = []
    for _ in range(n_polys):
        nv = int(rng.integers(3, 8))
        R = rng.uniform(0.03, 0.2) * H
        ang = np.sort(rng.uniform(0, 2 * math.pi, nv))
        rad = rng.uniform(0.5, 1.0, nv) * R
        centre = np.array([rng.uniform(cx - ex, cx + ex), rng.uniform(cy - ey, cy + ey)])
        verts = centre[None, :] + np.stack([rad * np.cos(ang), rad * np.sin(ang)], 1)
        nrm = rng.normal(size=3)
        nrm[2] = abs(nrm[2]) + 0.3
        nrm /= np.linalg.norm(nrm)
        polys.append(dict(verts=verts, depth=rng.uniform(1.0, 10.0),
                          albedo=rng.uniform(0.05, 0.95, 3),
                          intensity=rng.lognormal(0.0, 1.0), normal=nrm))
    polys.sort(key=lambda p: -p["depth"])  # painter's order: far to near
    return dict(H=H, W=W, blobs=blobs, polys=polys)


def _rot(theta):
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[c, -s], [s, c]])


def _to_screen(P, H, W, theta, t):
    c = np.array([W / 2.0, H / 2.0])
    return (P - c) @ _rot(theta).T + c + np.asarray(t)


def _inside(px, py, verts):
    """Even-odd crossing test of points (px, py) against a closed polygon."""
    inside = np.zeros(px.shape, bool)
    n = len(verts)
    for k in range(n):
        x0, y0 = verts[k]
        x1, y1 = verts[(k + 1) % n]
        cond = (y0 > py) != (y1 > py)
        with np.errstate(divide="ignore", invalid="ignore"):
            xint = x0 + (py - y0) * (x1 - x0) / (y1 - y0)
        inside ^= cond & (px < xint)
    return inside


def render_view(scene: dict, theta: float = 0.0, t=(0.0, 0.0)):
    """Noise-free radiance and GBuffer of the scene under camera (theta, t)."""
    H, W = scene["H"], scene["W"]
    truth = np.full((H, W, 3), 0.05)
    field = np.zeros((H, W, 3))
    b = scene["blobs"]
    cs = _to_screen(b["centre"], H, W, theta, t)
    for k in range(len(b["sigma"])):
        sg = b["sigma"][k]
        x0 = max(int(cs[k, 0] - 4 * sg), 0)
        x1 = min(int(cs[k, 0] + 4 * sg) + 1, W)
        y0 = max(int(cs[k, 1] - 4 * sg), 0)
        y1 = min(int(cs[k, 1] + 4 * sg) + 1, H)
        if x0 >= x1 or y0 >= y1:
            continue
        xs = np.arange(x0, x1) + 0.5 - cs[k, 0]
        ys = np.arange(y0, y1) + 0.5 - cs[k, 1]
        g = np.exp(-(ys[:, None] ** 2 + xs[None, :] ** 2) / (2 * sg * sg))
        field[y0:y1, x0:x1] += g[..., None] * b["rgb"][k]
    albedo = np.full((H, W, 3), 0.5)
    normal = np.zeros((H, W, 3))
    normal[..., 2] = 1.0
    depth = np.full((H, W), 20.0)
    truth = (truth + field) * albedo
    for p in scene["polys"]:
        vs = _to_screen(p["verts"], H, W, theta, t)
        x0 = max(int(np.floor(vs[:, 0].min())), 0)
        x1 = min(int(np.ceil(vs[:, 0].max())) + 1, W)
        y0 = max(int(np.floor(vs[:, 1].min())), 0)
        y1 = min(int(np.ceil(vs[:, 1].max())) + 1, H)
        if x0 >= x1 or y0 >= y1:
            continue
        py, px = np.meshgrid(np.arange(y0, y1) + 0.5, np.arange(x0, x1) + 0.5, indexing="ij")
        m = _inside(px, py, vs)
        if not m.any():
            continue
        sub = (slice(y0, y1), slice(x0, x1))
        truth[sub][m] = p["albedo"] * (p["intensity"] + 0.5 * field[sub][m])
        albedo[sub][m] = p["albedo"]
        normal[sub][m] = p["normal"]
        depth[sub][m] = p["depth"]
    return truth, albedo.astype(np.float32), normal.astype(np.float32), depth.astype(np.float32)


def camera_motion(seed: int):
    """Per-clip rotation rate (radians/frame) and translation (px/frame)."""
    rng = np.random.default_rng([int(seed), 0xCA3E7A])
    omega = math.radians(rng.uniform(-2.0, 2.0))
    v = rng.uniform(-12.0, 12.0, 2)
    return omega, v


def make_frame(scene: dict, t: int, motion=(0.0, (0.0, 0.0))) -> FrameData:
    """Frame t of a clip: camera angle omega*t, translation v*t; backward mv to frame t-1."""
    H, W = scene["H"], scene["W"]
    omega, v = motion
    v = np.asarray(v, float)
    truth, albedo, normal, depth = render_view(scene, omega * t, v * t)
    if t == 0:
        mv = np.zeros((H, W, 2), np.float32)
        valid = np.zeros((H, W), bool)
    else:
        c = np.array([W / 2.0, H / 2.0])
        qy, qx = np.meshgrid(np.arange(H) + 0.5, np.arange(W) + 0.5, indexing="ij")
        q = np.stack([qx, qy], -1)
        # world point of q in frame t, seen from camera t-1:  R(-omega)(q - c - v t) + c + v (t-1)
        prev = (q - c - v * t) @ _rot(-omega).T + c + v * (t - 1)
        mv = (prev - q).astype(np.float32)
        valid = (prev[..., 0] >= 0) & (prev[..., 0] <= W) & (prev[..., 1] >= 0) & (prev[..., 1] <= H)
    return FrameData(truth, albedo, normal, depth, mv, valid)


def make_clip(seed: int, H: int, W: int, T: int = 8):
    scene = make_scene(seed, H, W)
    motion = camera_motion(seed)
    return [make_frame(scene, t, motion) for t in range(T)]


def sample_pool(truth: np.ndarray, seed: int, frame: int, J: int = 8) -> np.ndarray:
    """[H*W, J, 4] float32 pool of noisy samples truth * (1 + n), n = LN(0, 0.8) - E[LN].

    Sample j of pixel i is pool[i, j]; channel 3 is zero (16-byte RGBA records).
    A renderer stand-in hands these out in request order; a pixel asking for more than
    J samples reuses them cyclically.
    """
    H, W, _ = truth.shape
    rng = np.random.default_rng([int(seed), int(frame), 0x5A3B1E])
    g = rng.standard_normal((H * W, J))
    one_n = np.exp(0.8 * g) - _LN_MEAN + 1.0
    out = np.zeros((H * W, J, 4), np.float32)
    out[..., :3] = truth.reshape(H * W, 1, 3) * one_n[..., None]
    return out
