"""Batched views, graph replay and the autotuner (GPU).

* One table / search / render over many views gives, view by view, exactly
  what separate per-view launches give.
* A captured graph replayed several times, with other GPU work and
  synchronisations in between, reproduces the eager result bit for bit.
* Bucket layouts and launch shapes change no result, nor does the
  autotuner's choice among them (cached and reloaded).
"""
import numpy as np
import pytest

from paper_2404_14044_amd import scenes

from hp_cases import compare_exact, host, sample_pixels

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def views():
    base = scenes.objects_1m(n=200_000, res=64)
    return scenes.batched_16(base=base, lo=64, hi=256)


def _setup(sc):
    import torch
    from paper_2404_14044_amd import hashpoint as hp
    dev = torch.device("cuda:0")
    return (torch.from_numpy(sc.xyz).to(dev), torch.from_numpy(sc.feat).to(dev),
            hp.to_device_mlp(sc.mlp, dev))


def _snapshot(smp, out, S):
    ns = host(smp["n_sel"]).copy()
    mask = np.arange(S)[None, :] < ns[:, None]
    return {"n_sel": ns, "primary": host(smp["primary"]).copy(),
            "t": host(smp["t"]).reshape(-1, S)[mask].view(np.int32).copy(),
            "rgb": host(out["rgb"]).view(np.int32).copy()}


def test_batched_equals_separate_launches(views):
    import torch
    from paper_2404_14044_amd import hashpoint as hp
    from paper_2404_14044_amd.batched import BatchedRenderer, render_views_separately
    sc = views
    xyz, feat, mlp = _setup(sc)
    br = BatchedRenderer(xyz, feat, mlp, sc.cams, sc.params, hp.HP_BF16)
    br.run_eager()
    sep = render_views_separately(xyz, feat, mlp, sc.cams, sc.params, hp.HP_BF16)
    torch.cuda.synchronize()
    S, K = sc.params.n_samples, sc.params.K
    for sl, st in zip(br.ray_slices(), sep):
        for k in ("n_sel", "primary", "n_nbr", "flags"):
            assert np.array_equal(host(br.samples[k])[sl], host(st["smp"][k])), k
        ns = host(st["smp"]["n_sel"])
        mask = np.arange(S)[None, :] < ns[:, None]
        tb = host(br.samples["t"]).reshape(-1, S)[sl][mask]
        ts = host(st["smp"]["t"]).reshape(-1, S)[mask]
        assert np.array_equal(tb.view(np.int32), ts.view(np.int32))
        kb = host(br.samples["knn_idx"]).reshape(-1, S, K)[sl][mask]
        ks = host(st["smp"]["knn_idx"]).reshape(-1, S, K)[mask]
        assert np.array_equal(kb, ks)
        rb = host(br.out["rgb"]).reshape(-1, 3)[sl]
        rs = host(st["out"]["rgb"]).reshape(-1, 3)
        assert np.array_equal(rb.view(np.int32), rs.view(np.int32))


def test_batched_views_match_oracle(views):
    from paper_2404_14044_amd import hashpoint as hp
    from paper_2404_14044_amd.batched import BatchedRenderer
    sc = views
    xyz, feat, mlp = _setup(sc)
    br = BatchedRenderer(xyz, feat, mlp, sc.cams, sc.params, hp.HP_FP32)
    br.run_eager()
    for v in (0, 7, 15):
        info = br.table.view(v)
        pix = sample_pixels(sc.cams[v], 512, seed=40 + v)
        compare_exact(sc, br.samples, pix, view=v, ray_base=info.ray_base, check_lists=False)


def test_graph_replay_reproduces_eager(views):
    import torch
    from paper_2404_14044_amd import hashpoint as hp
    from paper_2404_14044_amd.batched import BatchedRenderer
    sc = views
    xyz, feat, mlp = _setup(sc)
    br = BatchedRenderer(xyz, feat, mlp, sc.cams, sc.params, hp.HP_BF16)
    br.run_eager()
    torch.cuda.synchronize()
    ref = _snapshot(br.samples, br.out, sc.params.n_samples)
    br.capture()
    for rep in range(3):
        # unrelated eager work and a synchronisation between replays
        junk = torch.randn(1 << 20, device=xyz.device).sum()
        br.out["rgb"].fill_(-1.0)
        br.samples["n_sel"].fill_(-7)
        torch.cuda.synchronize()
        br.replay()
        torch.cuda.synchronize()
        got = _snapshot(br.samples, br.out, sc.params.n_samples)
        for k in ref:
            assert np.array_equal(ref[k], got[k]), (rep, k)
        del junk


def _frame(xyz, feat, mlp, cams, p, precision):
    from paper_2404_14044_amd import hashpoint as hp
    tab = hp.build_table(xyz, cams, p)
    smp = hp.search_sample(tab, p, debug=True)
    out = hp.render(smp, tab.n_rays, feat, mlp, p, precision)
    return smp, out


def _assert_same_frame(a, b, S, K):
    sa, oa = a
    sb, ob = b
    for k in ("n_sel", "primary", "n_nbr", "flags", "nbr_idx"):
        assert np.array_equal(host(sa[k]), host(sb[k])), k
    assert np.array_equal(host(sa["nbr_t"]).view(np.int32), host(sb["nbr_t"]).view(np.int32))
    ns = host(sa["n_sel"])
    mask = np.arange(S)[None, :] < ns[:, None]
    for k, w in (("t", 1), ("knn_idx", K), ("knn_dist", K)):
        x = host(sa[k]).reshape(-1, S, w)[mask]
        y = host(sb[k]).reshape(-1, S, w)[mask]
        assert np.array_equal(x.view(np.int32), y.view(np.int32)), k
    for k in ("rgb", "depth", "acc"):
        assert np.array_equal(host(oa[k]).view(np.int32), host(ob[k]).view(np.int32)), k


@pytest.mark.parametrize("shape", [
    dict(layout=2),
    dict(layout=1, window_shape=1, search_chunk=8, search_blocks=1024, search_band=640),
    dict(window_shape=1, search_band=64, render_rays=16, render_blocks=64),
    dict(layout=2, search_chunk=1, render_rays=64, render_blocks=8),
])
def test_launch_shapes_change_no_result(views, shape):
    """Bucket layouts (row-major, tiles, Z-order tiles), window shapes, XCD
    bands and the persistent search and render grids: every output of the
    sixteen views, neighbour lists included, is bit-identical to the
    defaults'."""
    import torch
    from paper_2404_14044_amd import hashpoint as hp
    sc = views
    xyz, feat, mlp = _setup(sc)
    ref = _frame(xyz, feat, mlp, sc.cams, sc.params, hp.HP_BF16)
    got = _frame(xyz, feat, mlp, sc.cams, sc.params.replace(**shape), hp.HP_BF16)
    torch.cuda.synchronize()
    _assert_same_frame(ref, got, sc.params.n_samples, sc.params.K)


def test_autotuner_choice_changes_no_result(tmp_path, views):
    """The tuner's choice (a reduced space here) is cached and reloaded, and
    the frame it renders equals the default frame bit for bit."""
    import torch
    from paper_2404_14044_amd import hashpoint as hp
    from paper_2404_14044_amd.autotune import Autotuner
    from paper_2404_14044_amd.batched import BatchedRenderer
    sc = views
    xyz, feat, mlp = _setup(sc)
    space = {"layout": (0, 2), "search_chunk": (1, 4), "window_shape": (0, 1),
             "render_rays": (16, 32), "render_blocks": (0, 64)}
    tuner = Autotuner(str(tmp_path / "tune.json"))
    p = tuner.tune(xyz, feat, mlp, sc.cams, sc.params, hp.HP_BF16, reps=1, space=space)
    ent = tuner.entry(xyz, sc.cams, sc.params, hp.HP_BF16)
    assert ent["ms"] > 0 and ent["default_ms"] > 0 and len(ent["trials"]) >= 6
    again = Autotuner(str(tmp_path / "tune.json")).tune(xyz, feat, mlp, sc.cams, sc.params,
                                                        hp.HP_BF16)
    assert again == p
    br = BatchedRenderer(xyz, feat, mlp, sc.cams, sc.params, hp.HP_BF16,
                         tuner=Autotuner(str(tmp_path / "tune.json")))
    assert br.params == p
    ref = _frame(xyz, feat, mlp, sc.cams, sc.params, hp.HP_BF16)
    got = _frame(xyz, feat, mlp, sc.cams, p, hp.HP_BF16)
    torch.cuda.synchronize()
    _assert_same_frame(ref, got, sc.params.n_samples, sc.params.K)


def test_batched_16_full_size_matches_oracle():
    """The batched workload as stated: 16 views of the 1M-point object scene,
    sides uniform in {256..1024}, one table / search / render over all of them
    (BF16 decoder).  256 random rays of every view against the oracle: exact
    outputs bit for bit, rgb / depth / acc within the BF16 bounds."""
    from paper_2404_14044_amd import hashpoint as hp
    from paper_2404_14044_amd.batched import BatchedRenderer
    from hp_cases import assert_render_error, render_error
    sc = scenes.batched_16()
    assert min(c.W for c in sc.cams) >= 256 and max(c.W for c in sc.cams) <= 1024
    xyz, feat, mlp = _setup(sc)
    br = BatchedRenderer(xyz, feat, mlp, sc.cams, sc.params, hp.HP_BF16)
    br.run_eager()
    hit = 0
    for v in range(len(sc.cams)):
        info = br.table.view(v)
        pix = sample_pixels(sc.cams[v], 256, seed=90 + v)
        ex = compare_exact(sc, br.samples, pix, view=v, ray_base=info.ray_base, check_lists=False)
        err = render_error(sc, br.out, ex, pix, view=v, ray_base=info.ray_base)
        assert_render_error(err, 1, sc.params)
        hit += int((ex["n_sel"] > 0).sum())
    assert hit > 500
