"""Pins of the oracle's K-NP extraction and Eq. 1 blending (Sec. 3.1, the
image-based consumers of the neighbour search).

Checks: hand cases on the axis ray (order by distance to the ray, ties by
index, the closed-form blend), agreement with an independent binary64
selection away from ties and the radius boundary, and the blend's special
cases (one point, one colour, a point on the ray, no neighbour).
"""
import numpy as np

from paper_2404_14044_amd import scenes


def _axis_cam():
    return scenes.Camera(W=1, H=1, fx=1.0, fy=1.0, cx=0.5, cy=0.5,
                         R=np.eye(3, dtype=np.float32), C=np.zeros(3, np.float32))


def _params(**kw):
    return scenes.default_params(0.25, 1.0, 8.0, K=4, S=4).replace(**kw)


def test_axis_hand_case(orc):
    cam = _axis_cam()
    # perpendicular offsets 0.125, 0.0625, 0.25 (on the radius: kept), 0.5 (out),
    # and a duplicate of the 0.0625 point with a larger index
    pc = np.array([[0.125, 0, 3], [0, 0.0625, 5], [0.25, 0, 2], [0.5, 0, 4], [0, 0.0625, 6]],
                  np.float32)
    colors = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1], [0.5, 0.5, 0]], np.float32)
    out = orc.knp(pc, cam, _params(), 3, colors, [0])
    assert out["cnt"][0] == 3
    assert out["idx"][0].tolist() == [1, 4, 0]
    assert np.array_equal(out["dist"][0], np.float32([0.0625, 0.0625, 0.125]))
    w = np.array([16.0, 16.0, 8.0])
    want = (w[:, None] * colors[[1, 4, 0]].astype(np.float64)).sum(0) / w.sum()
    assert np.allclose(out["rgb"][0], want, rtol=0, atol=1e-15)
    out4 = orc.knp(pc, cam, _params(), 5, colors, [0])
    assert out4["cnt"][0] == 4 and out4["idx"][0].tolist() == [1, 4, 0, 2, -1]


def test_blend_special_cases(orc):
    cam = _axis_cam()
    one = np.array([[0.1, 0, 3]], np.float32)
    col = np.array([[0.2, 0.4, 0.8]], np.float32)
    out = orc.knp(one, cam, _params(), 4, col, [0])
    assert np.allclose(out["rgb"][0], col[0], rtol=0, atol=1e-15)
    many = np.array([[0.01 * i, 0.02, 3 + 0.1 * i] for i in range(6)], np.float32)
    same = np.tile(np.float32([[0.3, 0.6, 0.9]]), (6, 1))
    out = orc.knp(many, cam, _params(), 4, same, [0])
    assert np.allclose(out["rgb"][0], same[0], rtol=0, atol=1e-12)
    on_ray = np.array([[0, 0, 3], [0.2, 0, 3]], np.float32)
    cols = np.array([[1, 0, 0], [0, 0, 1]], np.float32)
    out = orc.knp(on_ray, cam, _params(eps_idw=1e-6), 2, cols, [0])
    assert out["rgb"][0, 0] > 1 - 1e-5 and out["rgb"][0, 2] < 1e-5
    none = np.array([[1.0, 1.0, 3]], np.float32)
    out = orc.knp(none, cam, _params(bg=(0.1, 0.2, 0.3)), 4, col, [0])
    assert out["cnt"][0] == 0 and np.allclose(out["rgb"][0], [0.1, 0.2, 0.3])


def test_matches_binary64_selection(orc, rng):
    cam = scenes.pinhole(12, 10, 50.0, np.eye(3), np.zeros(3))
    xyz = np.concatenate([rng.uniform(-1, 1, size=(5000, 2)), rng.uniform(1.4, 3.2, size=(5000, 1))],
                         axis=1).astype(np.float32)
    colors = scenes.point_colors(xyz.shape[0], 7)
    K = 8
    for inv_tref in (0.0, 1.0 / 1.5):
        p = scenes.default_params(0.08, 1.5, 3.0, K=4, S=8, inv_tref=inv_tref)
        pc = orc.to_camera(xyz, cam)
        out = orc.knp(pc, cam, p, K, colors)
        x = pc.astype(np.float64)
        checked = 0
        for r in range(cam.W * cam.H):
            u, v = r % cam.W, r // cam.W
            a, b = (u + 0.5 - cam.cx) / cam.fx, (v + 0.5 - cam.cy) / cam.fy
            d = np.array([a, b, 1.0]) / np.sqrt(1 + a * a + b * b)
            t = x @ d
            e = np.linalg.norm(x - t[:, None] * d, axis=1)
            rho = p.radius * np.maximum(1.0, t * inv_tref)
            inside = (e <= rho * (1 - 1e-5)) & (t >= p.t_near * (1 + 1e-5)) & (t <= p.t_far * (1 - 1e-5))
            edge = (np.abs(e - rho) <= rho * 1e-5) | (np.abs(t - p.t_near) <= 1e-5) | \
                   (np.abs(t - p.t_far) <= 1e-5)
            cand = np.flatnonzero(inside | edge)
            order = cand[np.argsort(e[cand], kind="stable")]
            cnt = out["cnt"][r]
            got = out["idx"][r, :cnt]
            if edge[order[:K + 1]].any() if order.size else False:
                continue  # a boundary point could enter or leave the K nearest
            want = order[:K]
            es = np.sort(e[want])
            if want.size > 1 and np.min(np.diff(es)) < 1e-6:
                continue  # near-tie in distance
            if order.size > K and e[order[K]] - e[order[K - 1]] < 1e-6:
                continue  # near-tie at the cut
            assert cnt == want.size
            assert np.array_equal(got, want)
            # blend vs binary64 geometry; the selection's binary32 e^2 carries
            # a cancellation error of about |x| 2^-23, so rays with a point
            # almost on them are left to the hand cases
            if cnt and e[want].min() > 2e-2:
                w = 1.0 / np.maximum(e[want], p.eps_idw)
                ref = (w[:, None] * colors[want].astype(np.float64)).sum(0) / w.sum()
                assert np.allclose(out["rgb"][r], ref, rtol=0, atol=2e-5)
            checked += 1
        assert checked > 60
