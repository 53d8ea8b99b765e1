"""Pins of the oracle's per-pixel cone radius (Sec. 3.2, Eq. 3, and the
appendix's derivation and small-angle variants) and of the paper's kernel
size rule.

The radius of Eq. 3 at a point D at distance t along a pixel's ray is, by the
appendix's similar triangles, the distance from D to the cone's generator
line through the optical centre A and the kernel disc's edge point B (the
point of the disc around the pixel centre E on the side of the principal
point G).  Here that distance is computed in binary64 from cross products
of the actual 3-D points, and the small-angle variants from the foot F of the
perpendicular from B onto the ray: none of it retypes the oracle's formula.
"""
import numpy as np
import pytest

from paper_2404_14044_amd import scenes

EXACT, AF, AE = 1, 2, 3


def _cam(W=64, H=48, fov=60.0):
    return scenes.pinhole(W, H, fov, np.eye(3), np.zeros(3))


def _geometry(cam, u, v, rdd):
    """Binary64 points of the construction for pixel (u, v): unit focal plane."""
    a = (u + 0.5 - cam.cx) / cam.fx
    b = (v + 0.5 - cam.cy) / cam.fy
    E = np.array([a, b, 1.0])
    w = np.array([a, b, 0.0])
    wn = np.linalg.norm(w)
    B = E - rdd * w / wn if wn > 0 else E + np.array([rdd, 0.0, 0.0])
    return E, B


def _kappa_ref(cam, u, v, rdd, mode):
    E, B = _geometry(cam, u, v, rdd)
    e = E / np.linalg.norm(E)
    if mode == EXACT:
        # distance from D = t e to the line A B, divided by t
        return np.linalg.norm(np.cross(e, B)) / np.linalg.norm(B)
    BF = np.linalg.norm(np.cross(B, e))          # distance from B to the ray
    if mode == AF:
        AF_len = B @ e                           # A to the foot F of that perpendicular
        return BF / AF_len
    return BF / np.linalg.norm(E)


@pytest.mark.parametrize("mode", [EXACT, AF, AE])
def test_kappa_matches_cone_geometry(orc, rng, mode):
    cam = _cam()
    worst = 0.0
    for _ in range(3000):
        u, v = int(rng.integers(0, cam.W)), int(rng.integers(0, cam.H))
        rdd = float(np.float32(10 ** rng.uniform(-4, -1.3)))
        p = scenes.default_params(0.01, 1.0, 4.0, K=4, S=4).replace(radius_mode=mode, rddot=rdd)
        k = orc.ray_kappa(cam, p, u, v)
        ref = _kappa_ref(cam, u, v, rdd, mode)
        worst = max(worst, abs(k - ref) / ref)
    assert worst < 2e-6, worst


def test_axis_pixel_closed_forms(orc):
    cam = scenes.Camera(W=1, H=1, fx=1.0, fy=1.0, cx=0.5, cy=0.5,
                        R=np.eye(3, dtype=np.float32), C=np.zeros(3, np.float32))
    for rdd in (1e-3, 0.02, 0.3):
        rdd = float(np.float32(rdd))
        base = scenes.default_params(0.01, 1.0, 4.0, K=4, S=4)
        kx = orc.ray_kappa(cam, base.replace(radius_mode=EXACT, rddot=rdd), 0, 0)
        assert abs(kx - rdd / np.sqrt(1 + rdd * rdd)) <= 2e-7 * kx
        for mode in (AF, AE):
            assert orc.ray_kappa(cam, base.replace(radius_mode=mode, rddot=rdd), 0, 0) == np.float32(rdd)
        assert orc.ray_kappa(cam, base, 0, 0) == 0.0   # linear mode carries no slope


def test_variant_ordering_and_agreement(orc, rng):
    """AB >= AF and AE >= AF (AB^2 - AF^2 = rddot^2 / L^2; AF = AE - BF |w| / L),
    so the derived slope and the AE slope never exceed the AF slope, and the
    three agree to second order in rddot."""
    cam = _cam()
    for _ in range(2000):
        u, v = int(rng.integers(0, cam.W)), int(rng.integers(0, cam.H))
        rdd = float(np.float32(10 ** rng.uniform(-4, -1.5)))
        ks = {}
        for mode in (EXACT, AF, AE):
            p = scenes.default_params(0.01, 1.0, 4.0, K=4, S=4).replace(radius_mode=mode, rddot=rdd)
            ks[mode] = orc.ray_kappa(cam, p, u, v)
        assert ks[EXACT] <= ks[AF] * (1 + 1e-6) and ks[AE] <= ks[AF] * (1 + 1e-6)
        assert abs(ks[EXACT] / ks[AF] - 1) <= 2 * rdd + 1e-6
        assert abs(ks[AE] / ks[AF] - 1) <= 2 * rdd + 1e-6


@pytest.mark.parametrize("mode", [EXACT, AF, AE])
def test_rddot_pins_axis_radius_at_t_near(orc, mode):
    cam = scenes.Camera(W=1, H=1, fx=1.0, fy=1.0, cx=0.5, cy=0.5,
                        R=np.eye(3, dtype=np.float32), C=np.zeros(3, np.float32))
    for r, tn in ((0.01, 2.0), (0.02, 0.5), (0.05, 1.5)):
        p = scenes.default_params(r, tn, 10.0, K=4, S=4)
        p = p.replace(radius_mode=mode, rddot=scenes.eq3_rddot(mode, p.radius, p.t_near))
        k = orc.ray_kappa(cam, p, 0, 0)
        assert abs(k * p.t_near - p.radius) <= 1e-6 * p.radius


@pytest.mark.parametrize("mode", [EXACT, AF, AE])
def test_guard_band_bounds_cone_neighbours(orc, rng, mode):
    """Points within rho(t) = kappa t of a ray project within the guard band."""
    cam = scenes.pinhole(96, 64, 60.0, np.eye(3), np.zeros(3))
    p = scenes.default_params(0.05, 1.5, 8.0, K=4, S=4)
    p = p.replace(radius_mode=mode, rddot=scenes.eq3_rddot(mode, p.radius, p.t_near))
    g = orc.guard(cam, p)
    worst = 0.0
    for _ in range(20000):
        u, v = int(rng.integers(0, cam.W)), int(rng.integers(0, cam.H))
        a = (u + 0.5 - cam.cx) / cam.fx
        b = (v + 0.5 - cam.cy) / cam.fy
        d = np.array([a, b, 1.0]) / np.sqrt(1 + a * a + b * b)
        t = p.t_near if rng.random() < 0.5 else rng.uniform(p.t_near, p.t_far)
        rho = _kappa_ref(cam, u, v, p.rddot, mode) * t
        e = rng.normal(size=3)
        e -= (e @ d) * d
        e *= rho / np.linalg.norm(e)
        x = t * d + e
        off = np.hypot(cam.fx * x[0] / x[2] + cam.cx - (u + 0.5),
                       cam.fy * x[1] / x[2] + cam.cy - (v + 0.5))
        worst = max(worst, off)
    assert worst + 0.5 < g, (worst, g)
    assert g <= 1.7 * worst + 3.0, (worst, g)   # not vacuous


@pytest.mark.parametrize("mode", [EXACT, AF, AE])
def test_cone_search_matches_binary64_distance(orc, rng, mode):
    cam = scenes.pinhole(12, 10, 50.0, np.eye(3), np.zeros(3))
    xyz = np.concatenate([rng.uniform(-1, 1, size=(4000, 2)), rng.uniform(1.4, 3.2, size=(4000, 1))],
                         axis=1).astype(np.float32)
    p = scenes.default_params(0.06, 1.5, 3.0, K=4, S=8).replace(m_cap=4096)
    p = p.replace(radius_mode=mode, rddot=scenes.eq3_rddot(mode, p.radius, p.t_near))
    pc = orc.to_camera(xyz, cam)
    ex = orc.exact(pc, cam, p)
    x = pc.astype(np.float64)
    hits = 0
    for r in range(cam.W * cam.H):
        u, v = r % cam.W, r // cam.W
        a, b = (u + 0.5 - cam.cx) / cam.fx, (v + 0.5 - cam.cy) / cam.fy
        d = np.array([a, b, 1.0]) / np.sqrt(1 + a * a + b * b)
        t = x @ d
        e = np.linalg.norm(x - t[:, None] * d, axis=1)
        rho = _kappa_ref(cam, u, v, p.rddot, mode) * t
        tol = 1e-5
        sure_in = (e <= rho * (1 - tol)) & (t >= p.t_near * (1 + tol)) & (t <= p.t_far * (1 - tol))
        sure_out = (e > rho * (1 + tol)) | (t < p.t_near * (1 - tol)) | (t > p.t_far * (1 + tol))
        got = set(ex["nbr_idx"][r, :ex["n_nbr"][r]].tolist())
        assert set(np.flatnonzero(sure_in).tolist()) <= got
        assert not (set(np.flatnonzero(sure_out).tolist()) & got)
        hits += len(got)
    assert hits > 1000


def test_paper_kernel_size_rule(orc, rng):
    """s = 2 ceil(rddot / rdot) + 1 puts rddot in the range the appendix
    states: ((s-1)/2 - 1) rdot < rddot <= ((s-1)/2) rdot, rdot = sqrt(dx dy / pi)."""
    for _ in range(500):
        fx, fy = rng.uniform(50, 2000), rng.uniform(50, 2000)
        cam = scenes.Camera(W=64, H=64, fx=np.float32(fx), fy=np.float32(fy), cx=32.0, cy=32.0,
                            R=np.eye(3, dtype=np.float32), C=np.zeros(3, np.float32))
        rdd = float(np.float32(10 ** rng.uniform(-4, -1)))
        p = scenes.default_params(0.01, 1.0, 4.0, K=4, S=4).replace(radius_mode=EXACT, rddot=rdd)
        s = orc.paper_s(cam, p)
        rdot = np.sqrt((1.0 / float(cam.fx)) * (1.0 / float(cam.fy)) / np.pi)
        assert s % 2 == 1 and s >= 3
        assert ((s - 1) / 2 - 1) * rdot < rdd * (1 + 1e-12) and rdd <= (s - 1) / 2 * rdot * (1 + 1e-12)
