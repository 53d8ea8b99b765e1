"""Seeded synthetic inputs for the HashPoint hot path (arXiv 2404.14044).

This module only *generates inputs*: point clouds, neural features, pinhole
cameras, MLP weights and the run parameters of each workload.  It holds none of
the method's arithmetic (no projection, search, sampling or rendering), so both
the HIP path and the CPU oracle can be fed from it without sharing code.

The paper evaluates on Synthetic-NeRF (object scale) and Replica / Waymo
(scene scale, Sec. 4).  Those datasets are not used; the scenes below are
synthetic stand-ins with the same structure: a dense object-scale cloud of about
a million surface points, and a room-scale cloud of five million points whose
rays cross several surfaces, with outliers.

Conventions
-----------
* Scene representation P = {(x_i, f_i)} (Sec. 3.1): positions float32 (n, 3),
  features float32 (n, C) with C = 32.
* Cameras are pinhole, OpenCV axes (+x right, +y down, +z forward).  The
  world-to-camera rotation R has rows (x_c, y_c, z_c); camera-space position is
  R (p - C).  Pixel (u, v) has its centre at (u + 0.5, v + 0.5);
  fx = fy = (W / 2) / tan(hfov / 2), cx = W / 2, cy = H / 2.
* Every random draw uses numpy's PCG64 (`default_rng(seed)`), positions first,
  then features, in the order written below.
* MLP 32 -> 64 -> 64 -> 4, weights stored W[out][in]; W and b drawn from
  U(-1/sqrt(fan_in), +1/sqrt(fan_in)) in the order W1, b1, W2, b2, W3, b3.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

FEAT_DIM = 32
MLP_SHAPE = (32, 64, 64, 4)


# --------------------------------------------------------------------------
# cameras
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Camera:
    W: int
    H: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray  # (3, 3) float32, world -> camera, row-major
    C: np.ndarray  # (3,) float32, camera centre in world coordinates

    def as_tuple(self):
        return (self.W, self.H, self.fx, self.fy, self.cx, self.cy,
                tuple(float(v) for v in self.R.reshape(-1)),
                tuple(float(v) for v in self.C.reshape(-1)))


def look_at(C, target, up=(0.0, 1.0, 0.0)) -> np.ndarray:
    """Rows (x_c, y_c, z_c) of a world->camera rotation looking from C to target."""
    C = np.asarray(C, np.float64)
    target = np.asarray(target, np.float64)
    up = np.asarray(up, np.float64)
    z = target - C
    z /= np.linalg.norm(z)
    if abs(float(z @ up)) > 0.99:
        up = np.array([1.0, 0.0, 0.0])
    x = np.cross(z, up)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    return np.stack([x, y, z])


def pinhole(W: int, H: int, hfov_deg: float, R, C) -> Camera:
    f = (W / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)
    return Camera(W=int(W), H=int(H), fx=float(np.float32(f)), fy=float(np.float32(f)),
                  cx=float(np.float32(W / 2.0)), cy=float(np.float32(H / 2.0)),
                  R=np.asarray(R, np.float32).reshape(3, 3).copy(),
                  C=np.asarray(C, np.float32).reshape(3).copy())


# --------------------------------------------------------------------------
# run parameters
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Params:
    """Hyper-parameters of search, sampling and rendering.

    radius, inv_tref: search radius rho(t) = radius * max(1, t * inv_tref)
        (radius_mode 0); inv_tref = 0 is a fixed radius, 1 / t_near a linear
        cone equal to radius at t_near.
    radius_mode, rddot: radius_mode 1 is the per-pixel cone of Eq. 3 with
        kernel disc radius rddot (image plane at unit focal length), 2 and 3
        its two small-angle variants (AB replaced by AF, by AE); rho = t kappa
        with kappa per pixel.  `eq3_rddot` picks rddot so that the principal
        pixel's radius at t_near is `radius`.
    layout, search_chunk, search_blocks, search_band, window_shape,
        render_rays, render_blocks: bucket order and launch shapes; none of
        them changes a result (the autotuner picks them).
    sampler, ms_steps: sampler 0 is the adaptive primary-surface walk
        (Sec. 3.3); sampler 1 the uniform multi-surface baseline (Sec. 3.5):
        ms_steps uniform positions along [t_near, t_far], each kept when a
        point of the ray's neighbour list lies within rho of it.
    t_near, t_far: sampling range along the ray (Sec. 3.2).
    K: neighbours per sample (Eq. 4).  n_samples: cap on samples per ray.
    m_cap: cap on the per-ray neighbour list.
    gamma, inv_beta2: confidence alpha = gamma * exp(-d^2 / beta^2) (Sec. 3.3).
    eps_w: a candidate is kept when its weight (Eq. 5) exceeds eps_w.
    eps_idw: distance floor of the inverse-distance feature weights.
    delta_last: interval length given to the last sample of a ray (Eq. 2).
    bg: background colour.
    """
    radius: float
    inv_tref: float
    t_near: float
    t_far: float
    K: int
    n_samples: int
    m_cap: int = 64
    gamma: float = 0.9
    inv_beta2: float = 0.0
    eps_w: float = 1e-4
    eps_idw: float = 1e-6
    delta_last: float = 1e10
    bg: tuple = (0.0, 0.0, 0.0)
    layout: int = 0
    flags: int = 0
    search_chunk: int = 0
    search_blocks: int = 0
    radius_mode: int = 0
    rddot: float = 0.0
    sampler: int = 0
    ms_steps: int = 0
    search_band: int = 0
    window_shape: int = 0
    render_rays: int = 0
    render_blocks: int = 0

    def replace(self, **kw) -> "Params":
        return dataclasses.replace(self, **kw)


def eq3_rddot(mode: int, radius: float, t_near: float) -> float:
    """Kernel disc radius (unit focal length) for which the principal pixel's
    cone has radius `radius` at t_near: kappa(axis) = rddot / sqrt(1 + rddot^2)
    for the derived form, rddot for the small-angle forms (Sec. 3.2: the
    minimum radius sits at t_near and equals the radius hyper-parameter)."""
    r, tn = float(radius), float(t_near)
    if mode == 1:
        return float(np.float32(r / np.sqrt(tn * tn - r * r)))
    return float(np.float32(r / tn))


def point_colors(n: int, seed: int) -> np.ndarray:
    """Per-point RGB in [0, 1] for image-based blending (Eq. 1), seeded."""
    return np.random.default_rng(seed).random((n, 3)).astype(np.float32)


def default_params(radius, t_near, t_far, K, S, inv_tref=0.0) -> Params:
    r = float(np.float32(radius))
    return Params(radius=r, inv_tref=float(np.float32(inv_tref)),
                  t_near=float(np.float32(t_near)), t_far=float(np.float32(t_far)),
                  K=int(K), n_samples=int(S), m_cap=64, gamma=float(np.float32(0.9)),
                  inv_beta2=float(np.float32(1.0 / (r * r))),
                  eps_w=float(np.float32(1e-4)), eps_idw=float(np.float32(1e-6)),
                  delta_last=float(np.float32(1e10)), bg=(0.0, 0.0, 0.0))


# --------------------------------------------------------------------------
# MLP weights
# --------------------------------------------------------------------------
def make_mlp(seed: int, shape=MLP_SHAPE) -> Dict[str, np.ndarray]:
    rng = np.random.default_rng(seed)
    out = {}
    for li in range(len(shape) - 1):
        fi, fo = shape[li], shape[li + 1]
        bound = 1.0 / math.sqrt(fi)
        out[f"W{li + 1}"] = rng.uniform(-bound, bound, size=(fo, fi)).astype(np.float32)
        out[f"b{li + 1}"] = rng.uniform(-bound, bound, size=(fo,)).astype(np.float32)
    return out


# --------------------------------------------------------------------------
# surface samplers
# --------------------------------------------------------------------------
def _unit_vectors(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _random_rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


class _Sphere:
    def __init__(self, c, rad):
        self.c, self.rad = np.asarray(c), float(rad)

    def area(self):
        return 4.0 * math.pi * self.rad ** 2

    def sample(self, rng, n):
        return self.c + self.rad * _unit_vectors(rng, n)

    def inside(self, p):
        return np.linalg.norm(p - self.c, axis=1) < self.rad


class _Box:
    """Oriented box: centre c, rotation Q (columns = box axes), half extents e."""

    def __init__(self, c, Q, e, faces=(0, 1, 2, 3, 4, 5)):
        self.c, self.Q, self.e = np.asarray(c), np.asarray(Q), np.asarray(e)
        self.faces = tuple(faces)

    def _face_areas(self):
        e = self.e
        a = {0: 4 * e[1] * e[2], 1: 4 * e[1] * e[2], 2: 4 * e[0] * e[2],
             3: 4 * e[0] * e[2], 4: 4 * e[0] * e[1], 5: 4 * e[0] * e[1]}
        return np.array([a[f] for f in self.faces])

    def area(self):
        return float(self._face_areas().sum())

    def sample(self, rng, n):
        fa = self._face_areas()
        face = np.asarray(self.faces)[rng.choice(len(fa), size=n, p=fa / fa.sum())]
        loc = rng.uniform(-1.0, 1.0, size=(n, 3)) * self.e
        axis = face // 2
        sign = np.where(face % 2 == 0, 1.0, -1.0)
        loc[np.arange(n), axis] = sign * self.e[axis]
        return self.c + loc @ self.Q.T

    def inside(self, p):
        loc = (p - self.c) @ self.Q
        return np.all(np.abs(loc) < self.e, axis=1)


class _Torus:
    """Torus with major radius Rm, tube radius rt, axis = third column of Q."""

    def __init__(self, c, Q, Rm, rt):
        self.c, self.Q, self.Rm, self.rt = np.asarray(c), np.asarray(Q), float(Rm), float(rt)

    def area(self):
        return 4.0 * math.pi ** 2 * self.Rm * self.rt

    def sample(self, rng, n):
        out = np.empty((0, 3))
        while out.shape[0] < n:
            m = 2 * (n - out.shape[0]) + 16
            u = rng.uniform(0, 2 * math.pi, m)
            v = rng.uniform(0, 2 * math.pi, m)
            keep = rng.uniform(0, 1, m) < (self.Rm + self.rt * np.cos(v)) / (self.Rm + self.rt)
            u, v = u[keep], v[keep]
            loc = np.stack([(self.Rm + self.rt * np.cos(v)) * np.cos(u),
                            (self.Rm + self.rt * np.cos(v)) * np.sin(u),
                            self.rt * np.sin(v)], axis=1)
            out = np.concatenate([out, self.c + loc @ self.Q.T])
        return out[:n]

    def inside(self, p):
        loc = (p - self.c) @ self.Q
        q = np.sqrt(loc[:, 0] ** 2 + loc[:, 1] ** 2) - self.Rm
        return q * q + loc[:, 2] ** 2 < self.rt ** 2


def _sample_union(rng, prims, n, reject_inside=True):
    areas = np.array([p.area() for p in prims])
    out, have = [], 0
    while have < n:
        m = int((n - have) * 1.3) + 1024
        which = rng.choice(len(prims), size=m, p=areas / areas.sum())
        pts = np.empty((m, 3))
        for k, p in enumerate(prims):
            sel = which == k
            if sel.any():
                pts[sel] = p.sample(rng, int(sel.sum()))
        if reject_inside:
            bad = np.zeros(m, bool)
            for k, p in enumerate(prims):
                bad |= p.inside(pts) & (which != k)
            pts = pts[~bad]
        out.append(pts)
        have += pts.shape[0]
    return np.concatenate(out)[:n]


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Scene:
    name: str
    xyz: np.ndarray            # (n, 3) float32
    feat: np.ndarray           # (n, 32) float32
    cams: List[Camera]
    params: Params
    mlp: Dict[str, np.ndarray]
    extra: dict = dataclasses.field(default_factory=dict)


def sphere_plane(n_sphere=10_000, n_plane=10_000, res=64, seed=1, mlp_seed=101) -> Scene:
    """Plain FP32 case: unit sphere centred at z=3 plus a 4x4 square at z=4.5."""
    rng = np.random.default_rng(seed)
    sph = np.array([0.0, 0.0, 3.0]) + _unit_vectors(rng, n_sphere)
    pl = np.concatenate([rng.uniform(-2.0, 2.0, size=(n_plane, 2)),
                         np.full((n_plane, 1), 4.5)], axis=1)
    xyz = np.concatenate([sph, pl]).astype(np.float32)
    feat = rng.normal(size=(xyz.shape[0], FEAT_DIM)).astype(np.float32)
    cam = pinhole(res, res, 60.0, np.eye(3), np.zeros(3))
    return Scene("sphere_plane", xyz, feat, [cam],
                 default_params(0.02, 1.5, 10.0, K=8, S=8), make_mlp(mlp_seed))


def _object_points(rng, n, n_prims=12):
    prims = []
    for _ in range(n_prims):
        kind = rng.integers(0, 3)
        Q = _random_rotation(rng)
        if kind == 0:
            rad = rng.uniform(0.15, 0.4)
            ext = rad
            c = rng.uniform(-1 + ext, 1 - ext, size=3)
            prims.append(_Sphere(c, rad))
        elif kind == 1:
            e = rng.uniform(0.1, 0.4, size=3)
            ext = float(np.linalg.norm(e))
            c = rng.uniform(-1 + min(ext, 0.95), 1 - min(ext, 0.95), size=3)
            prims.append(_Box(c, Q, e))
        else:
            Rm, rt = rng.uniform(0.2, 0.4), rng.uniform(0.05, 0.12)
            ext = Rm + rt
            c = rng.uniform(-1 + ext, 1 - ext, size=3)
            prims.append(_Torus(c, Q, Rm, rt))
    pts = _sample_union(rng, prims, n)
    pts = pts + rng.normal(0.0, 0.002, size=pts.shape)
    return np.clip(pts, -1.0, 1.0)


def objects_1m(n=1_000_000, res=800, seed=2, mlp_seed=102) -> Scene:
    """Object scale: 12 random spheres, boxes and tori inside [-1, 1]^3."""
    rng = np.random.default_rng(seed)
    xyz = _object_points(rng, n).astype(np.float32)
    feat = rng.normal(size=(n, FEAT_DIM)).astype(np.float32)
    C = np.array([0.0, 0.0, -4.0])
    cam = pinhole(res, res, 40.0, look_at(C, np.zeros(3)), C)
    return Scene("objects_1m", xyz, feat, [cam],
                 default_params(0.01, 2.0, 6.0, K=8, S=16), make_mlp(mlp_seed))


def _room_points(rng, n_surface, n_box=40):
    lo, hi = np.array([-8.0, 0.0, -6.0]), np.array([8.0, 4.0, 6.0])
    prims = []
    thick = 0.05  # half thickness of a 0.1 m wall slab
    I = np.eye(3)
    size = hi - lo
    mid = (hi + lo) / 2
    for axis in range(3):
        for side in (0, 1):
            c = mid.copy()
            c[axis] = (lo if side == 0 else hi)[axis]
            e = size / 2
            e = e.copy()
            e[axis] = thick
            prims.append(_Box(c, I, e, faces=(2 * axis, 2 * axis + 1)))
    for _ in range(n_box):
        s = rng.uniform(0.3, 1.5, size=3)
        yaw = rng.uniform(0, 2 * math.pi)
        Q = np.array([[math.cos(yaw), 0, math.sin(yaw)], [0, 1, 0], [-math.sin(yaw), 0, math.cos(yaw)]])
        c = np.array([rng.uniform(-7.0, 7.0), s[1] / 2, rng.uniform(-5.0, 5.0)])
        prims.append(_Box(c, Q, s / 2, faces=(0, 1, 2, 4, 5)))  # no bottom face
    pts = _sample_union(rng, prims, n_surface, reject_inside=False)
    return pts + rng.normal(0.0, 0.005, size=pts.shape), lo, hi


def room_5m(n=5_000_000, W=1008, H=756, seed=3, mlp_seed=103, outlier_frac=0.05) -> Scene:
    """Scene scale: a walled room with 40 boxes, 5% uniform outliers."""
    rng = np.random.default_rng(seed)
    n_out = int(round(n * outlier_frac))
    surf, lo, hi = _room_points(rng, n - n_out)
    outl = rng.uniform(lo, hi, size=(n_out, 3))
    xyz = np.concatenate([surf, outl]).astype(np.float32)
    feat = rng.normal(size=(n, FEAT_DIM)).astype(np.float32)
    C = np.array([-7.0, 1.6, -5.0])
    cam = pinhole(W, H, 60.0, look_at(C, np.array([8.0, 1.0, 6.0])), C)
    return Scene("room_5m", xyz, feat, [cam],
                 default_params(0.02, 0.5, 21.0, K=16, S=16), make_mlp(mlp_seed))


def sphere_poses(rng, n_views, radius, sides, hfov=40.0) -> List[Camera]:
    cams = []
    for k in range(n_views):
        d = _unit_vectors(rng, 1)[0]
        C = radius * d
        cams.append(pinhole(int(sides[k]), int(sides[k]), hfov, look_at(C, np.zeros(3)), C))
    return cams


def batched_16(base: Optional[Scene] = None, seed=4, n_views=16, lo=256, hi=1024) -> Scene:
    """16 views of the object scene, sides uniform in {lo..hi}, on a radius-4 sphere."""
    base = base or objects_1m()
    rng = np.random.default_rng(seed)
    sides = rng.integers(lo, hi + 1, size=n_views)
    cams = sphere_poses(rng, n_views, 4.0, sides)
    return Scene("batched_16", base.xyz, base.feat, cams, base.params, base.mlp)


def diff_4x400(base: Optional[Scene] = None, seed=5, n_views=4, res=400) -> Scene:
    """Differentiable case: 4 views of 400x400 and a random target image."""
    base = base or objects_1m()
    rng = np.random.default_rng(seed)
    cams = sphere_poses(rng, n_views, 4.0, [res] * n_views)
    target = rng.uniform(0.0, 1.0, size=(n_views * res * res, 3)).astype(np.float32)
    return Scene("diff_4x400", base.xyz, base.feat, cams, base.params, base.mlp,
                 extra={"target": target})


def crop_camera(cam: Camera, u0: int, v0: int, w: int, h: int) -> Camera:
    """The same camera restricted to the pixel window [u0, u0+w) x [v0, v0+h)."""
    return Camera(W=w, H=h, fx=cam.fx, fy=cam.fy, cx=float(np.float32(cam.cx - u0)),
                  cy=float(np.float32(cam.cy - v0)), R=cam.R.copy(), C=cam.C.copy())


def tiny_scene(seed=0, n=600, res=8, hfov=60.0, radius=0.12) -> Scene:
    """A few hundred points in a thin slab filling the view of an 8x8 camera."""
    rng = np.random.default_rng(seed)
    xyz = np.concatenate([rng.uniform(-1.2, 1.2, size=(n, 2)),
                          rng.uniform(2.0, 2.3, size=(n, 1))], axis=1).astype(np.float32)
    feat = rng.normal(size=(n, FEAT_DIM)).astype(np.float32)
    cam = pinhole(res, res, hfov, np.eye(3), np.zeros(3))
    return Scene("tiny", xyz, feat, [cam], default_params(radius, 1.0, 5.0, K=4, S=8),
                 make_mlp(seed + 1000))


WORKLOADS = {
    "sphere_plane": sphere_plane,
    "objects_1m": objects_1m,
    "room_5m": room_5m,
}
