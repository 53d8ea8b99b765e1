"""Pins of the oracle's geometry: camera transform, rays, guard band and the pixel table.

Each check compares the oracle with an independent binary64 computation or a
closed form, chosen so that a transposed rotation, a wrong sign or a swapped
axis fails.
"""
import numpy as np

from paper_2404_14044_amd import scenes


def _rot(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


def test_camera_transform_matches_binary64(orc, rng):
    R = _rot(rng).astype(np.float32)
    C = rng.normal(size=3).astype(np.float32)
    cam = scenes.pinhole(64, 48, 50.0, R, C)
    xyz = rng.normal(size=(5000, 3)).astype(np.float32) * 3
    pc = orc.to_camera(xyz, cam)
    ref = (xyz.astype(np.float64) - C.astype(np.float64)) @ R.astype(np.float64).T
    assert np.abs(pc - ref).max() < 1e-5 * (1 + np.abs(ref).max())


def test_look_at_target_projects_to_principal_point(orc):
    Cw = np.array([1.0, 2.0, -3.0])
    tgt = np.array([-0.5, 0.25, 1.0])
    cam = scenes.pinhole(100, 80, 40.0, scenes.look_at(Cw, tgt), Cw)
    pc = orc.to_camera(tgt[None].astype(np.float32), cam)[0]
    assert abs(pc[0]) < 1e-6 and abs(pc[1]) < 1e-6
    assert abs(pc[2] - np.linalg.norm(tgt - Cw)) < 1e-5
    # a point above the target (world +y) appears above the centre: smaller v
    up = orc.to_camera((tgt + [0, 0.1, 0])[None].astype(np.float32), cam)[0]
    assert up[1] < 0


def test_ray_through_pixel_centre(orc):
    cam = scenes.pinhole(37, 23, 70.0, np.eye(3), np.zeros(3))
    for u, v in [(0, 0), (36, 22), (18, 11), (5, 20)]:
        d = orc.ray_dir(cam, u, v).astype(np.float64)
        assert abs(np.linalg.norm(d) - 1.0) < 1e-6
        uf = cam.fx * d[0] / d[2] + cam.cx
        vf = cam.fy * d[1] / d[2] + cam.cy
        assert abs(uf - (u + 0.5)) < 1e-4 and abs(vf - (v + 0.5)) < 1e-4


def test_single_pixel_axis_ray_is_exact(orc):
    cam = scenes.Camera(W=1, H=1, fx=1.0, fy=1.0, cx=0.5, cy=0.5,
                        R=np.eye(3, dtype=np.float32), C=np.zeros(3, np.float32))
    d = orc.ray_dir(cam, 0, 0)
    assert d.tolist() == [0.0, 0.0, 1.0]


def test_guard_band_bounds_sampled_neighbours(orc, rng):
    """Points within rho(t) of a ray at t in [t_near, t_far] project within the guard band."""
    for inv_tref in (0.0, 1.0 / 1.5):
        cam = scenes.pinhole(96, 64, 60.0, np.eye(3), np.zeros(3))
        p = scenes.default_params(0.05, 1.5, 8.0, K=4, S=4, inv_tref=inv_tref)
        g = orc.guard(cam, p)
        worst = 0.0
        for _ in range(20000):
            u, v = rng.integers(0, cam.W), rng.integers(0, cam.H)
            a = (u + 0.5 - cam.cx) / cam.fx
            b = (v + 0.5 - cam.cy) / cam.fy
            d = np.array([a, b, 1.0]) / np.sqrt(1 + a * a + b * b)
            t = p.t_near if rng.random() < 0.5 else rng.uniform(p.t_near, p.t_far)
            rho = p.radius * max(1.0, t * inv_tref)
            e = rng.normal(size=3)
            e -= (e @ d) * d
            e *= rho / np.linalg.norm(e)
            x = t * d + e
            off = np.hypot(cam.fx * x[0] / x[2] + cam.cx - (u + 0.5),
                           cam.fy * x[1] / x[2] + cam.cy - (v + 0.5))
            worst = max(worst, off)
        assert worst + 0.5 < g, (worst, g)
        assert g <= worst + 3.0, (worst, g)   # the bound is not vacuous


def test_table_lists_every_visible_point_once(orc, rng):
    cam = scenes.pinhole(32, 24, 60.0, np.eye(3), np.zeros(3))
    p = scenes.default_params(0.05, 1.0, 5.0, K=4, S=4)
    g = orc.guard(cam, p)
    xyz = np.concatenate([rng.uniform(-2, 2, size=(3000, 2)), rng.uniform(-1, 4, size=(3000, 1))],
                         axis=1).astype(np.float32)
    xyz[:50, 2] = 0.0                         # on the camera plane: dropped
    xyz[50:60] = np.nan                       # non-finite: dropped
    pc = orc.to_camera(xyz, cam)
    key, order = orc.table(pc, cam, g)
    # independent binary64 projection
    x64 = pc.astype(np.float64)
    with np.errstate(all="ignore"):
        uf = cam.fx * x64[:, 0] / x64[:, 2] + cam.cx
        vf = cam.fy * x64[:, 1] / x64[:, 2] + cam.cy
        inside = (x64[:, 2] > 0) & (uf >= -g) & (uf < cam.W + g) & (vf >= -g) & (vf < cam.H + g)
        near_edge = (np.abs(uf - np.round(uf)) < 1e-3) | (np.abs(vf - np.round(vf)) < 1e-3)
    listed = key >= 0
    assert (listed[~near_edge] == inside[~near_edge]).all()
    Wg = cam.W + 2 * g
    ok = inside & ~near_edge
    exp_key = (np.floor(vf[ok]).astype(np.int64) + g) * Wg + np.floor(uf[ok]).astype(np.int64) + g
    assert (key[ok] == exp_key).all()
    assert not listed[:60].any()
    # every listed point once, sorted by (key, z, idx)
    assert np.array_equal(np.sort(order), np.flatnonzero(listed))
    k, z = key[order], pc[order, 2]
    assert (np.diff(k) >= 0).all()
    same = np.diff(k) == 0
    dz = np.diff(z)
    assert (dz[same] >= 0).all()
    tie = same & (dz == 0)
    assert (np.diff(order)[tie] > 0).all()


def test_table_axis_point_lands_on_principal_pixel(orc):
    cam = scenes.pinhole(20, 10, 60.0, np.eye(3), np.zeros(3))
    p = scenes.default_params(0.05, 1.0, 5.0, K=4, S=4)
    g = orc.guard(cam, p)
    pc = orc.to_camera(np.array([[0.0, 0.0, 2.0], [0.0, 0.0, -2.0]], np.float32), cam)
    key, order = orc.table(pc, cam, g)
    assert key[1] == -1
    assert key[0] == (int(cam.cy) + g) * (cam.W + 2 * g) + int(cam.cx) + g
    assert order.tolist() == [0]
