"""Pins of the oracle's binary64 render (Eq. 2 with an MLP decoder) and its gradient.

Closed forms: a single opaque sample returns the decoded colour; two samples
composite as a0 c0 + (1 - a0) a1 c1; with one neighbour the aggregated feature
is that neighbour's feature, so the decoder reduces to matrix products
(numpy); two neighbours give the inverse-distance mean.  The analytic gradient
is pinned by central finite differences of the render.
"""
import numpy as np

from paper_2404_14044_amd import scenes


def _axis_cam():
    return scenes.Camera(W=1, H=1, fx=1.0, fy=1.0, cx=0.5, cy=0.5,
                         R=np.eye(3, dtype=np.float32), C=np.zeros(3, np.float32))


def _mlp_np(mlp, f):
    h1 = np.maximum(mlp["W1"].astype(np.float64) @ f + mlp["b1"], 0)
    h2 = np.maximum(mlp["W2"].astype(np.float64) @ h1 + mlp["b2"], 0)
    return mlp["W3"].astype(np.float64) @ h2 + mlp["b3"]


def _sig(x):
    return 1.0 / (1.0 + np.exp(-x))


def _softplus(x):
    return np.log1p(np.exp(x))


def _samples(ts, idx, K):
    S = len(ts)
    ex = {"pix": np.array([0], np.int32), "n_sel": np.array([S], np.int32),
          "t": np.array([ts], np.float32),
          "knn_idx": np.full((1, S, K), -1, np.int32)}
    for s, row in enumerate(idx):
        ex["knn_idx"][0, s, :len(row)] = row
    return ex


def test_single_opaque_sample_returns_decoded_colour(orc, rng):
    mlp = scenes.make_mlp(7)
    feat = rng.normal(size=(3, 32)).astype(np.float32)
    pts = np.array([[0.01, 0.0, 2.0], [0.0, 0.02, 2.5], [0.0, 0.0, 3.0]], np.float32)
    p = scenes.default_params(0.05, 1.0, 5.0, K=1, S=4)
    out = orc.render64(pts, feat, mlp, _axis_cam(), p, _samples([2.0], [[0]], 1))
    o = _mlp_np(mlp, feat[0].astype(np.float64))
    assert np.allclose(out["rgb"][0], _sig(o[:3]), rtol=0, atol=1e-12)
    assert abs(out["acc"][0] - 1.0) < 1e-12
    assert abs(out["depth"][0] - 2.0) < 1e-12


def test_two_samples_closed_form(orc, rng):
    mlp = scenes.make_mlp(8)
    feat = rng.normal(size=(2, 32)).astype(np.float32)
    pts = np.array([[0.01, 0.0, 2.0], [0.0, 0.02, 2.3]], np.float32)
    p = scenes.default_params(0.05, 1.0, 5.0, K=1, S=4).replace(delta_last=0.7, bg=(0.2, 0.4, 0.6))
    ts = [2.0, 2.3]
    out = orc.render64(pts, feat, mlp, _axis_cam(), p, _samples(ts, [[0], [1]], 1))
    o0, o1 = _mlp_np(mlp, feat[0].astype(np.float64)), _mlp_np(mlp, feat[1].astype(np.float64))
    d0 = float(np.float32(2.3)) - 2.0
    a0 = 1 - np.exp(-_softplus(o0[3]) * d0)
    a1 = 1 - np.exp(-_softplus(o1[3]) * float(np.float32(0.7)))
    w0, w1 = a0, (1 - a0) * a1
    bg = np.array([np.float32(0.2), np.float32(0.4), np.float32(0.6)], np.float64)
    rgb = w0 * _sig(o0[:3]) + w1 * _sig(o1[:3]) + (1 - w0 - w1) * bg
    assert np.allclose(out["rgb"][0], rgb, atol=1e-12)
    assert abs(out["acc"][0] - (w0 + w1)) < 1e-12
    assert abs(out["depth"][0] - (w0 * 2.0 + w1 * float(np.float32(2.3)))) < 1e-12


def test_inverse_distance_mean_of_two(orc, rng):
    mlp = scenes.make_mlp(9)
    feat = rng.normal(size=(2, 32)).astype(np.float32)
    pts = np.array([[0.01, 0.0, 2.0], [0.0, 0.03, 2.0]], np.float32)
    p = scenes.default_params(0.05, 1.0, 5.0, K=2, S=4)
    out = orc.render64(pts, feat, mlp, _axis_cam(), p, _samples([2.0], [[0, 1]], 2))
    d1 = np.linalg.norm(pts[0].astype(np.float64) - [0, 0, 2.0])
    d2 = np.linalg.norm(pts[1].astype(np.float64) - [0, 0, 2.0])
    f = (feat[0] / d1 + feat[1] / d2) / (1 / d1 + 1 / d2)
    o = _mlp_np(mlp, f)
    assert np.allclose(out["rgb"][0], _sig(o[:3]), atol=1e-12)


def test_empty_ray_is_background(orc):
    mlp = scenes.make_mlp(1)
    p = scenes.default_params(0.05, 1.0, 5.0, K=2, S=4).replace(bg=(0.25, 0.5, 1.0))
    ex = {"pix": np.array([0], np.int32), "n_sel": np.array([0], np.int32),
          "t": np.zeros((1, 4), np.float32), "knn_idx": np.full((1, 4, 2), -1, np.int32)}
    out = orc.render64(np.zeros((1, 3), np.float32), np.zeros((1, 32), np.float32), mlp,
                       _axis_cam(), p, ex)
    assert out["rgb"][0].tolist() == [0.25, 0.5, 1.0]
    assert out["acc"][0] == 0.0 and out["depth"][0] == 0.0


def _tiny_pipeline(orc, seed=0):
    sc = scenes.tiny_scene(seed=seed)
    cam, p = sc.cams[0], sc.params
    pc = orc.to_camera(sc.xyz, cam)
    ex = orc.exact(pc, cam, p)
    return sc, cam, p, pc, ex


def test_render_invariants(orc):
    sc, cam, p, pc, ex = _tiny_pipeline(orc)
    out = orc.render64(pc, sc.feat, sc.mlp, cam, p, ex)
    assert (ex["n_sel"] > 0).sum() > 20
    assert (out["acc"] >= 0).all() and (out["acc"] <= 1 + 1e-12).all()
    assert (out["rgb"] >= 0).all() and (out["rgb"] <= 1 + 1e-12).all()
    ns = ex["n_sel"]
    for r in np.flatnonzero(ns > 0):
        t = ex["t"][r, :ns[r]]
        assert t[0] * out["acc"][r] - 1e-9 <= out["depth"][r] <= t[-1] * out["acc"][r] + 1e-9


def test_gradient_matches_central_differences(orc):
    sc, cam, p, pc, ex = _tiny_pipeline(orc, seed=1)
    rng = np.random.default_rng(4)
    R = ex["pix"].size
    gr = rng.normal(size=(R, 3))

    def loss(feat, mlp):
        return float((orc.render64(pc, feat, mlp, cam, p, ex)["rgb"] * gr).sum())

    g = orc.grad64(pc, sc.feat, sc.mlp, cam, p, ex, gr)
    used = np.unique(ex["knn_idx"][ex["knn_idx"] >= 0])
    checks = [("feat", (int(i), int(c))) for i, c in
              zip(rng.choice(used, 12), rng.integers(0, 32, 12))]
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        shp = sc.mlp[name].shape
        for _ in range(4):
            checks.append((name, tuple(int(rng.integers(0, s)) for s in shp)))
    for name, ij in checks:
        base = sc.feat if name == "feat" else sc.mlp[name]
        h = 1e-5
        vals = []
        for sgn in (+1, -1):
            pert = base.astype(np.float64).copy()
            pert[ij] += sgn * h
            # the render reads binary32 inputs; the step is the exact binary32 difference
            arr = pert.astype(np.float32)
            if name == "feat":
                vals.append(loss(arr, sc.mlp))
            else:
                m2 = dict(sc.mlp)
                m2[name] = arr
                vals.append(loss(sc.feat, m2))
        step = float(np.float32(base[ij] + h)) - float(np.float32(base[ij] - h))
        fd = (vals[0] - vals[1]) / step
        an = g[name][ij]
        assert abs(fd - an) <= 1e-4 * max(1.0, abs(an)), (name, ij, fd, an)
