"""Shared helpers for the GPU parity tests: run the HIP path and the oracle on
the same seeded inputs and compare their outputs."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2404_14044_amd import scenes


def gpu_forward(sc, params=None, debug=True, precision=None):
    import torch
    from paper_2404_14044_amd import hashpoint as hp
    p = params or sc.params
    dev = torch.device("cuda:0")
    xyz = torch.from_numpy(np.ascontiguousarray(sc.xyz)).to(dev)
    tab = hp.build_table(xyz, sc.cams, p)
    smp = hp.search_sample(tab, p, debug=debug)
    out = {"table": tab, "samples": smp}
    if precision is not None:
        feat = torch.from_numpy(np.ascontiguousarray(sc.feat)).to(dev)
        mlp = hp.to_device_mlp(sc.mlp, dev)
        out["render"] = hp.render(smp, tab.n_rays, feat, mlp, p, precision)
    torch.cuda.synchronize()
    return out


def host(t):
    return t.detach().cpu().numpy()


def gpu_table_lists(tab, view=0):
    """Per-pixel point lists of one view: dict (bx, by) -> list of indices."""
    info = tab.view(view)
    offs = host(tab.offsets())
    n_in = int(offs[-1])
    perm = host(tab.perm(n_in)) if n_in else np.zeros(0, np.int32)
    return info, offs, perm


def compare_table_rowmajor(sc, tab, view=0, params=None):
    cam, p = sc.cams[view], params or sc.params
    g = oracle.guard(cam, p)
    info, offs, perm = gpu_table_lists(tab, view)
    assert info.g == g
    pc = oracle.to_camera(sc.xyz, cam)
    key, order = oracle.table(pc, cam, g)
    b0 = info.bucket_base
    nb = info.Wg * info.Hg
    lo, hi = int(offs[b0]), int(offs[b0 + nb])
    assert hi - lo == order.size, (hi - lo, order.size)
    assert np.array_equal(perm[lo:hi], order)
    cnt = np.bincount(key[key >= 0], minlength=nb)
    assert np.array_equal(np.diff(offs[b0:b0 + nb + 1]), cnt)


def check_depth_summaries(sc, tab, view=0, params=None):
    """The table's depth summaries of a row-major view against the oracle's
    table: each bucket's first depth and each 8x8-bucket cell's minimum
    (+inf where empty), bit for bit.  Returns the expected cell minima as a
    (cells down, cells across) array."""
    cam, p = sc.cams[view], params or sc.params
    info = tab.view(view)
    Wg, Hg, b0 = info.Wg, info.Hg, info.bucket_base
    nb = Wg * Hg
    offs = host(tab.offsets())
    pc = oracle.to_camera(sc.xyz, cam)
    key, order = oracle.table(pc, cam, oracle.guard(cam, p))
    lo = int(offs[b0])
    first = offs[b0:b0 + nb] - lo
    hit = np.diff(offs[b0:b0 + nb + 1]) > 0
    want_bz = np.full(nb, np.inf, np.float32)
    want_bz[hit] = pc[order[first[hit]], 2]
    got_bz = host(tab.bucket_z())[b0:b0 + nb]
    assert np.array_equal(got_bz.view(np.uint32), want_bz.view(np.uint32))
    ncx, ncy = (Wg + 7) // 8, (Hg + 7) // 8
    cbase = sum(((tab.view(v).Wg + 7) // 8) * ((tab.view(v).Hg + 7) // 8) for v in range(view))
    grid = np.full((ncy * 8, ncx * 8), np.inf, np.float32)
    grid[:Hg, :Wg] = want_bz.reshape(Hg, Wg)
    want_cz = grid.reshape(ncy, 8, ncx, 8).min(axis=(1, 3))
    got_cz = host(tab.cell_zmin())[cbase:cbase + ncx * ncy]
    assert np.array_equal(got_cz.view(np.uint32), want_cz.reshape(-1).view(np.uint32))
    return want_cz


def compare_exact(sc, smp, pix, params=None, view=0, ray_base=0, check_lists=True):
    """Bit-exact comparison of the search and sampling outputs on rays `pix`."""
    cam = sc.cams[view]
    p = params or sc.params
    pc = oracle.to_camera(sc.xyz, cam)
    ex = oracle.exact(pc, cam, p, pix)
    rays = ray_base + np.asarray(pix, np.int64)
    S, K, M = p.n_samples, p.K, p.m_cap
    n_sel = host(smp["n_sel"])[rays]
    assert np.array_equal(host(smp["n_nbr"])[rays], ex["n_nbr"]), "neighbour counts"
    assert np.array_equal(host(smp["flags"])[rays].astype(np.uint32), ex["flags"]), "overflow flags"
    if check_lists and "nbr_idx" in smp:
        ni = host(smp["nbr_idx"]).reshape(-1, M)[rays]
        nt = host(smp["nbr_t"]).reshape(-1, M)[rays]
        assert np.array_equal(ni, ex["nbr_idx"]), "neighbour lists"
        assert np.array_equal(nt.view(np.int32), ex["nbr_t"].view(np.int32)), "neighbour t bits"
    assert np.array_equal(n_sel, ex["n_sel"]), "sample counts"
    assert np.array_equal(host(smp["primary"])[rays], ex["primary"]), "primary surface"
    t = host(smp["t"]).reshape(-1, S)[rays]
    ki = host(smp["knn_idx"]).reshape(-1, S, K)[rays]
    kd = host(smp["knn_dist"]).reshape(-1, S, K)[rays]
    mask = np.arange(S)[None, :] < n_sel[:, None]
    assert np.array_equal(t[mask].view(np.int32), ex["t"][mask].view(np.int32)), "sample t bits"
    assert np.array_equal(ki[mask], ex["knn_idx"][mask]), "nearest-neighbour indices"
    assert np.array_equal(kd[mask].view(np.int32), ex["knn_dist"][mask].view(np.int32)), \
        "nearest-neighbour distance bits"
    return ex


# Render tolerances (max abs vs the oracle's binary64 render).  RGB and
# acc = sum of the compositing weights are in [0, 1]; depth = sum of weight x t
# moves by at most t_far times the weights' error, so its bound is the RGB
# bound scaled by t_far.
FP32_TOL = 1e-5
BF16_TOL = 2e-3


def assert_render_error(err, precision, params):
    """rgb, acc within the precision's bound; depth within bound * t_far."""
    tol = FP32_TOL if precision == 0 else BF16_TOL
    assert err["rgb"] <= tol, ("rgb", err)
    assert err["acc"] <= tol, ("acc", err)
    assert err["depth"] <= tol * float(params.t_far), ("depth", err)


def render_error(sc, out, ex, pix, params=None, view=0, ray_base=0):
    cam = sc.cams[view]
    p = params or sc.params
    pc = oracle.to_camera(sc.xyz, cam)
    ref = oracle.render64(pc, sc.feat, sc.mlp, cam, p, ex)
    rays = ray_base + np.asarray(pix, np.int64)
    rgb = host(out["rgb"]).reshape(-1, 3)[rays].astype(np.float64)
    dep = host(out["depth"])[rays].astype(np.float64)
    acc = host(out["acc"])[rays].astype(np.float64)
    return {"rgb": np.abs(rgb - ref["rgb"]).max(initial=0.0),
            "depth": np.abs(dep - ref["depth"]).max(initial=0.0),
            "acc": np.abs(acc - ref["acc"]).max(initial=0.0)}


def sample_pixels(cam, k, seed):
    rng = np.random.default_rng(seed)
    n = cam.W * cam.H
    return np.sort(rng.choice(n, size=min(k, n), replace=False)).astype(np.int32)


def adversarial_scene(seed=0):
    """Points placed on the decision boundaries and in degenerate layouts."""
    rng = np.random.default_rng(seed)
    res = 24
    cam = scenes.pinhole(res, res, 60.0, np.eye(3), np.zeros(3))
    p = scenes.default_params(0.03, 1.0, 4.0, K=8, S=16)
    pts = []
    # ordinary surface
    pts.append(np.concatenate([rng.uniform(-0.9, 0.9, size=(3000, 2)),
                               rng.uniform(2.0, 2.05, size=(3000, 1))], 1))
    # points exactly on pixel-centre rays at the search radius, and just beyond
    for k in range(200):
        u, v = rng.integers(0, res, 2)
        a = (u + 0.5 - cam.cx) / cam.fx
        b = (v + 0.5 - cam.cy) / cam.fy
        d = np.array([a, b, 1.0]) / np.sqrt(1 + a * a + b * b)
        e = np.cross(d, rng.normal(size=3))
        e /= np.linalg.norm(e)
        t = rng.uniform(1.5, 3.0)
        for f in (1.0, 1.0 + 1e-7, 1.0 - 1e-7):
            pts.append((t * d + f * p.radius * e)[None])
    # duplicates and equal depths
    dup = np.array([[0.1, -0.05, 2.5]])
    pts.append(np.repeat(dup, 40, 0))
    eq = np.stack([rng.uniform(-0.2, 0.2, 300), rng.uniform(-0.2, 0.2, 300), np.full(300, 2.25)], 1)
    pts.append(eq)
    # a skewed bucket: many points along one pixel's ray (grazing surface)
    a = (10 + 0.5 - cam.cx) / cam.fx
    b = (7 + 0.5 - cam.cy) / cam.fy
    ts = rng.uniform(1.0, 4.0, 5000)
    pts.append(np.stack([a * ts, b * ts, ts], 1) + rng.normal(0, 1e-4, (5000, 3)))
    # behind the camera, on the camera plane, far outside the view, non-finite
    pts.append(np.array([[0.0, 0.0, -1.0], [0.3, 0.1, 0.0], [50.0, 0.0, 1.0],
                         [np.nan, 0.0, 2.0], [0.0, np.inf, 2.0], [1e30, 1e30, 1e-30]]))
    xyz = np.concatenate(pts).astype(np.float32)
    feat = rng.normal(size=(xyz.shape[0], 32)).astype(np.float32)
    return scenes.Scene("adversarial", xyz, feat, [cam], p, scenes.make_mlp(seed + 7))
