"""Pins of the oracle's neighbour search (Sec. 3.2) and candidate walk (Sec. 3.3, Eq. 4, Eq. 5).

Checks: hand cases with exactly representable answers, agreement with an
independent binary64 point-to-line distance away from the decision boundary,
closed forms of the weight recursion, the z-buffer special case, and the
invariants that Eq. 5 implies.
"""
import numpy as np

from paper_2404_14044_amd import scenes


def _axis_cam():
    # 1x1 image with the principal point at the pixel centre: the ray is +z exactly
    return scenes.Camera(W=1, H=1, fx=1.0, fy=1.0, cx=0.5, cy=0.5,
                         R=np.eye(3, dtype=np.float32), C=np.zeros(3, np.float32))


def _params(**kw):
    p = scenes.default_params(0.25, 1.0, 8.0, K=4, S=16)
    return p.replace(**kw)


def test_axis_hand_cases(orc):
    cam = _axis_cam()
    r = 0.25
    p = _params(radius=r)
    pts = np.array([
        [0.0, 0.0, 2.0],                     # on the axis: t = 2, e^2 = 0
        [r, 0.0, 3.0],                       # exactly at the radius: included (<=)
        [r * (1 + 2 ** -18), 0.0, 3.5],      # just outside
        [0.0, 0.0, 1.0],                     # t = t_near: included
        [0.0, 0.0, 8.0],                     # t = t_far: included
        [0.0, 0.0, 8.0 * (1 + 2 ** -20)],    # beyond t_far
        [0.0, 0.0, 0.99],                    # before t_near
        [0.0, 0.0, -2.0],                    # behind the camera
    ], np.float32)
    ex = orc.exact(pts, cam, p, pix=[0])
    m = ex["n_nbr"][0]
    assert m == 4
    assert ex["nbr_idx"][0, :m].tolist() == [3, 0, 1, 4]
    assert ex["nbr_t"][0, :m].tolist() == [1.0, 2.0, 3.0, 8.0]
    assert ex["flags"][0] == 0


def test_cap_and_tie_order(orc):
    cam = _axis_cam()
    p = _params(radius=0.1, m_cap=64)
    z = np.repeat(np.linspace(2.0, 6.0, 50, dtype=np.float32), 2)  # 100 points, pairs share t
    pts = np.stack([np.zeros(100), np.zeros(100), z], 1).astype(np.float32)
    perm = np.random.default_rng(3).permutation(100)
    pts = pts[perm]
    ex = orc.exact(pts, cam, p, pix=[0])
    assert ex["n_nbr"][0] == 64 and ex["flags"][0] == 1
    order = np.lexsort((np.arange(100), pts[:, 2]))[:64]
    assert ex["nbr_idx"][0].tolist() == order.tolist()


def _random_scene(rng, n=3000, res=12):
    cam = scenes.pinhole(res, res, 50.0, np.eye(3), np.zeros(3))
    xyz = np.concatenate([rng.uniform(-0.9, 0.9, size=(n, 2)),
                          rng.uniform(1.8, 2.4, size=(n, 1))], axis=1).astype(np.float32)
    return cam, xyz


def test_search_matches_binary64_distance(orc, rng):
    for inv_tref in (0.0, 1.0 / 1.5):
        cam, xyz = _random_scene(rng)
        p = scenes.default_params(0.06, 1.5, 3.0, K=4, S=8, inv_tref=inv_tref).replace(m_cap=4096)
        pc = orc.to_camera(xyz, cam)
        ex = orc.exact(pc, cam, p)
        x = pc.astype(np.float64)
        for r in range(cam.W * cam.H):
            u, v = r % cam.W, r // cam.W
            a, b = (u + 0.5 - cam.cx) / cam.fx, (v + 0.5 - cam.cy) / cam.fy
            d = np.array([a, b, 1.0]) / np.sqrt(1 + a * a + b * b)
            t = x @ d
            e = np.linalg.norm(x - t[:, None] * d, axis=1)
            rho = p.radius * np.maximum(1.0, t * inv_tref)
            tol = 1e-5
            sure_in = (e <= rho * (1 - tol)) & (t >= p.t_near * (1 + tol)) & (t <= p.t_far * (1 - tol))
            sure_out = (e > rho * (1 + tol)) | (t < p.t_near * (1 - tol)) | (t > p.t_far * (1 + tol))
            got = set(ex["nbr_idx"][r, :ex["n_nbr"][r]].tolist())
            assert set(np.flatnonzero(sure_in).tolist()) <= got
            assert not (set(np.flatnonzero(sure_out).tolist()) & got)
            # list order is (t, idx)
            lst = ex["nbr_idx"][r, :ex["n_nbr"][r]]
            tt = ex["nbr_t"][r, :ex["n_nbr"][r]]
            assert np.all((np.diff(tt) > 0) | ((np.diff(tt) == 0) & (np.diff(lst) > 0)))
            assert np.allclose(tt, t[lst], rtol=1e-6, atol=1e-6)


def test_weights_halve_when_alpha_is_half(orc):
    """gamma = 0.5, beta -> inf: alpha = 1/2, so w_j = 2^-(j+1) (Eq. 5) and the
    samples are the first 13 candidates at eps_w = 1e-4."""
    cam = _axis_cam()
    z = np.linspace(2.0, 4.0, 20, dtype=np.float32)
    pts = np.stack([np.zeros(20), np.zeros(20), z], 1).astype(np.float32)
    p = _params(gamma=0.5, inv_beta2=0.0, n_samples=16, K=4)
    ex = orc.exact(pts, cam, p, pix=[0], diagnostics=True)
    w = ex["cand_w"][0, :20].astype(np.float64)
    assert np.array_equal(w, 2.0 ** -(np.arange(20) + 1))
    assert ex["n_sel"][0] == 13
    assert ex["t"][0, :13].tolist() == z[:13].tolist()
    assert ex["primary"][0] == 0
    p2 = p.replace(n_samples=5)
    ex2 = orc.exact(pts, cam, p2, pix=[0])
    assert ex2["n_sel"][0] == 5


def test_zbuffer_special_case(orc, rng):
    """gamma = 1, beta -> inf: alpha = 1, so exactly one sample, at the nearest
    neighbour along the ray, like a z-buffer."""
    cam, xyz = _random_scene(rng, n=2000, res=8)
    p = scenes.default_params(0.06, 1.5, 3.0, K=4, S=8).replace(gamma=1.0, inv_beta2=0.0)
    pc = orc.to_camera(xyz, cam)
    ex = orc.exact(pc, cam, p)
    hit = ex["n_nbr"] > 0
    assert (ex["n_sel"][hit] == 1).all() and (ex["n_sel"][~hit] == 0).all()
    assert (ex["primary"][hit] == ex["nbr_idx"][hit, 0]).all()
    assert (ex["primary"][~hit] == -1).all()


def test_copies_of_one_axis_point_give_zero_udf(orc):
    cam = _axis_cam()
    K = 4
    pts = np.tile(np.array([[0.0, 0.0, 2.0]], np.float32), (K, 1))
    p = _params(K=K)
    ex = orc.exact(pts, cam, p, pix=[0], diagnostics=True)
    assert (ex["cand_d"][0, :K] == 0.0).all()
    assert np.allclose(ex["cand_alpha"][0, :K], p.gamma)
    assert ex["knn_idx"][0, 0].tolist() == [0, 1, 2, 3]
    # with one copy fewer than K, the missing neighbour counts as distance R_j
    ex3 = orc.exact(pts[:K - 1], cam, p, pix=[0], diagnostics=True)
    assert np.isclose(ex3["cand_d"][0, 0], p.radius / K, rtol=1e-6)


def test_walk_matches_binary64_knn(orc, rng):
    """d_j (Eq. 4 with padding) against a binary64 K-nearest search over N(ray)."""
    obj = scenes.objects_1m(n=60_000, res=48)
    cam, p = obj.cams[0], obj.params.replace(radius=0.03, inv_beta2=1.0 / 0.03 ** 2)
    pc = orc.to_camera(obj.xyz, cam)
    ex = orc.exact(pc, cam, p, diagnostics=True)
    x = pc.astype(np.float64)
    checked = 0
    for r in np.flatnonzero(ex["n_nbr"] > 0)[:300]:
        u, v = r % cam.W, r // cam.W
        a, b = (u + 0.5 - cam.cx) / cam.fx, (v + 0.5 - cam.cy) / cam.fy
        d = np.array([a, b, 1.0]) / np.sqrt(1 + a * a + b * b)
        m = ex["n_nbr"][r]
        nb = ex["nbr_idx"][r, :m]
        for j in range(m):
            tj = float(ex["nbr_t"][r, j])
            Rj = p.radius
            dist = np.linalg.norm(x[nb] - tj * d, axis=1)
            inr = dist[dist <= Rj]
            # skip decisions that rounding could flip
            if np.any(np.abs(dist - Rj) < 1e-5 * Rj):
                continue
            ds = np.sort(inr)
            if len(ds) > p.K and ds[p.K] - ds[p.K - 1] < 1e-7:
                continue
            kk = min(len(ds), p.K)
            dj = (ds[:kk].sum() + (p.K - kk) * Rj) / p.K
            assert abs(dj - ex["cand_d"][r, j]) < 1e-5 * Rj, (r, j)
            alpha = p.gamma * np.exp(-dj * dj * p.inv_beta2)
            assert abs(alpha - ex["cand_alpha"][r, j]) < 1e-5
            checked += 1
    assert checked > 1000


def test_walk_invariants(orc):
    obj = scenes.objects_1m(n=60_000, res=48)
    cam, p = obj.cams[0], obj.params.replace(radius=0.03, inv_beta2=1.0 / 0.03 ** 2)
    pc = orc.to_camera(obj.xyz, cam)
    ex = orc.exact(pc, cam, p, diagnostics=True)
    S, K = p.n_samples, p.K
    for r in range(cam.W * cam.H):
        m, ns = ex["n_nbr"][r], ex["n_sel"][r]
        assert 0 <= ns <= min(S, m)
        w = ex["cand_w"][r, :m].astype(np.float64)
        T = ex["cand_T"][r, :m].astype(np.float64)
        al = ex["cand_alpha"][r, :m].astype(np.float64)
        assert (w >= 0).all() and (w <= p.gamma).all()
        assert (al >= 0).all() and (al <= p.gamma).all()
        assert (np.diff(T) <= 0).all() and (T <= 1).all()
        assert w.sum() <= 1.0 + 1e-6
        sel = np.flatnonzero(w > p.eps_w)[:S]
        assert ns == len(sel)
        if ns:
            assert ex["primary"][r] == ex["nbr_idx"][r, sel[0]]
            assert (ex["t"][r, :ns] == ex["nbr_t"][r, sel]).all()
            assert (np.diff(ex["t"][r, :ns]) >= 0).all()
        else:
            assert ex["primary"][r] == -1
        for s in range(ns):
            kc = ex["knn_cnt"][r, s]
            assert 1 <= kc <= K
            dd = ex["knn_dist"][r, s, :kc]
            assert (np.diff(dd) >= 0).all() and (dd <= p.radius).all()
            assert set(ex["knn_idx"][r, s, :kc].tolist()) <= set(ex["nbr_idx"][r, :m].tolist())
            assert (ex["knn_idx"][r, s, kc:] == -1).all()
