"""Pins of the oracle's uniform multi-surface sampler (the volume-rendering
baseline of Sec. 3.5 that primary-surface sampling is compared with).

Checks: the closed form of one point on the axis ray (a position is kept iff
it is within R of the point), two surfaces both sampled where the primary-
surface walk stops at the first, a second surface sampled although the
ray's first 64 neighbours (the list cut) all lie on the first, the uniform
grid of sample positions, agreement with an independent binary64 test of
every position against all of the ray's neighbours, invariants.
"""
import numpy as np

from paper_2404_14044_amd import scenes


def _axis_cam():
    return scenes.Camera(W=1, H=1, fx=1.0, fy=1.0, cx=0.5, cy=0.5,
                         R=np.eye(3, dtype=np.float32), C=np.zeros(3, np.float32))


def _ms(**kw):
    p = scenes.default_params(0.25, 1.0, 9.0, K=4, S=64).replace(sampler=1, ms_steps=64)
    return p.replace(**kw)


def _grid(p):
    step = np.float32(np.float32(p.t_far - p.t_near) / np.float32(p.ms_steps))
    k = np.arange(p.ms_steps, dtype=np.float32)
    # fma((k + 0.5), step, t_near) in binary64 then rounded once: exact for these sizes
    return (((k + np.float32(0.5)).astype(np.float64) * np.float64(step) + np.float64(p.t_near))
            .astype(np.float32))


def test_single_axis_point_closed_form(orc):
    cam = _axis_cam()
    p = _ms()
    tk = _grid(p)
    for z0 in (2.03, 4.61, 8.9):
        pc = np.array([[0.0, 0.0, z0]], np.float32)
        ex = orc.exact(pc, cam, p, [0])
        dist = np.abs(tk.astype(np.float64) - np.float64(np.float32(z0)))
        keep = dist <= p.radius
        assert not np.any(np.abs(dist - p.radius) < 1e-4)  # no position near the boundary
        assert ex["n_sel"][0] == keep.sum() > 0
        got = ex["t"][0, :ex["n_sel"][0]]
        assert np.array_equal(got, tk[keep])
        assert np.all(ex["knn_idx"][0, :ex["n_sel"][0], 0] == 0)
        assert np.allclose(ex["knn_dist"][0, :ex["n_sel"][0], 0], dist[keep], rtol=1e-6, atol=1e-6)
        assert ex["primary"][0] == 0


def test_two_surfaces_both_sampled(orc):
    """A near and a far surface on the axis ray: the walk with gamma = 1 stops
    at the first, the multi-surface sampler keeps positions at both."""
    cam = _axis_cam()
    near = np.stack([np.zeros(6), np.linspace(-0.1, 0.1, 6), np.full(6, 3.0)], 1)
    far = np.stack([np.zeros(6), np.linspace(-0.1, 0.1, 6), np.full(6, 7.0)], 1)
    pc = np.concatenate([near, far]).astype(np.float32)
    ms = orc.exact(pc, cam, _ms(), [0])
    t = ms["t"][0, :ms["n_sel"][0]]
    assert np.any(np.abs(t - 3.0) <= 0.25) and np.any(np.abs(t - 7.0) <= 0.25)
    assert not np.any((t > 3.3) & (t < 6.7))
    ps = orc.exact(pc, cam, _ms(sampler=0, gamma=1.0, inv_beta2=0.0), [0])
    assert ps["n_sel"][0] == 1 and abs(ps["t"][0, 0] - 3.0) < 0.2


def test_positions_match_binary64(orc, rng):
    """Every position against an independent binary64 computation of the
    ray's neighbours (all of them: the list cut m_cap = 8 is far below the
    neighbour counts here, and must not limit the positions' searches)."""
    cam = scenes.pinhole(10, 8, 50.0, np.eye(3), np.zeros(3))
    xyz = np.concatenate([rng.uniform(-1, 1, size=(3000, 2)), rng.uniform(1.2, 3.2, size=(3000, 1))],
                         axis=1).astype(np.float32)
    p = scenes.default_params(0.06, 1.0, 3.5, K=4, S=64).replace(sampler=1, ms_steps=200, m_cap=8)
    pc = orc.to_camera(xyz, cam)
    ex = orc.exact(pc, cam, p)
    assert ex["flags"].sum() > 20          # most rays have more neighbours than the cut
    tk = _grid(p).astype(np.float64)
    x = pc.astype(np.float64)
    r0, tn, tf = float(p.radius), float(p.t_near), float(p.t_far)
    checked = 0
    for r in range(cam.W * cam.H):
        u, v = r % cam.W, r // cam.W
        a, b = (u + 0.5 - cam.cx) / cam.fx, (v + 0.5 - cam.cy) / cam.fy
        d = np.array([a, b, 1.0]) / np.sqrt(1 + a * a + b * b)
        t = x @ d
        e = np.linalg.norm(x - t[:, None] * d[None, :], axis=1)
        sure_nb = (x[:, 2] > 0) & (t >= tn * (1 + 1e-6)) & (t <= tf * (1 - 1e-6)) & (e <= r0 * (1 - 1e-5))
        maybe_nb = (x[:, 2] > 0) & (t >= tn * (1 - 1e-6)) & (t <= tf * (1 + 1e-6)) & (e <= r0 * (1 + 1e-5))
        if not maybe_nb.any():
            assert ex["n_sel"][r] == 0
            continue
        # binary64 distance from every position to every (possible) neighbour
        dist = np.linalg.norm(x[maybe_nb][None, :, :] - tk[:, None, None] * d[None, None, :], axis=2)
        sure_pt = sure_nb[maybe_nb]
        sure = ((dist <= r0 * (1 - 1e-5)) & sure_pt[None, :]).any(axis=1)
        maybe = (dist <= r0 * (1 + 1e-5)).any(axis=1)
        kept = set(np.round((ex["t"][r, :ex["n_sel"][r]] - p.t_near) / (tk[1] - tk[0]) - 0.5)
                   .astype(int).tolist())
        want = np.flatnonzero(sure)
        if ex["n_sel"][r] < p.n_samples:
            assert set(want.tolist()) <= kept
            assert kept <= set(np.flatnonzero(maybe).tolist())
        checked += ex["n_sel"][r]
    assert checked > 200


def test_second_surface_beyond_the_list_cut(orc, rng):
    """A ray whose first surface alone holds 200 neighbours (m_cap = 64): the
    list N(ray) ends inside that surface, yet the positions at the second
    surface, 4 units further, are still samples, with their own points as
    nearest neighbours (the paper's multi-surface baseline samples every
    surface the ray crosses)."""
    cam = _axis_cam()
    ang = rng.uniform(0, 2 * np.pi, 200)
    rad = 0.2 * np.sqrt(rng.uniform(0, 1, 200))
    first = np.stack([rad * np.cos(ang), rad * np.sin(ang), rng.uniform(2.95, 3.05, 200)], 1)
    second = np.stack([np.zeros(5), np.linspace(-0.1, 0.1, 5), np.full(5, 7.0)], 1)
    pc = np.concatenate([first, second]).astype(np.float32)
    ex = orc.exact(pc, cam, _ms(), [0])
    assert ex["flags"][0] == 1 and ex["n_nbr"][0] == 64
    assert set(ex["nbr_idx"][0].tolist()) <= set(range(200))   # the cut list: first surface only
    ns = ex["n_sel"][0]
    t = ex["t"][0, :ns]
    far = np.abs(t - 7.0) <= 0.25
    assert far.sum() >= 2 and np.any(np.abs(t - 3.0) <= 0.3)
    idx = ex["knn_idx"][0, :ns][far]
    assert np.all((idx[:, 0] >= 200) & (idx[:, 0] < 205))
    # and exactly the positions within R of some far point, as in the closed form
    tk = _grid(_ms())
    d_far = np.abs(tk.astype(np.float64)[:, None] - 7.0)
    e_far = np.abs(np.linspace(-0.1, 0.1, 5))[None, :]
    want = np.flatnonzero((np.sqrt(d_far ** 2 + e_far ** 2) <= 0.25).any(axis=1))
    assert np.array_equal(t[far], tk[want])


def test_invariants(orc, rng):
    sc = scenes.sphere_plane(n_sphere=4000, n_plane=4000)
    p = sc.params.replace(sampler=1, ms_steps=300, n_samples=32)
    cam = sc.cams[0]
    pc = orc.to_camera(sc.xyz, cam)
    ex = orc.exact(pc, cam, p)
    grid = set(_grid(p).tolist())
    assert (ex["n_sel"] > 0).sum() > 200
    for r in np.flatnonzero(ex["n_sel"]):
        ns = ex["n_sel"][r]
        t = ex["t"][r, :ns]
        assert ns <= p.n_samples and np.all(np.diff(t) > 0)
        assert set(t.tolist()) <= grid
        kd = ex["knn_dist"][r, :ns]
        kc = ex["knn_cnt"][r, :ns]
        assert np.all(kc >= 1) and np.all(kc <= p.K)
        for s in range(ns):
            assert np.all(np.diff(kd[s, :kc[s]]) >= 0)
            assert kd[s, kc[s] - 1] <= p.radius * (1 + 1e-6)
        assert ex["primary"][r] == ex["knn_idx"][r, 0, 0]
