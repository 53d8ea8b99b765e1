"""The allocation-free backward (hp_render_backward_noalloc) against the
recomputing backward with a caller workspace (hp_render_backward), through
the C ABI: two calls in a row on the library's per-GPU scratch array, the
second on a smaller input, each equal to the workspace call up to the order of
float atomics (the same bar as the chunked recompute: the chunk boundaries
differ, the arithmetic per sample does not)."""
import numpy as np
import pytest

from paper_2404_14044_amd import scenes

pytestmark = pytest.mark.gpu

KEYS = ("W1", "b1", "W2", "b2", "W3", "b3")


def _inputs(sc, dev, seed):
    import torch
    from paper_2404_14044_amd import hashpoint as hp
    xyz = torch.from_numpy(sc.xyz).to(dev)
    feat = torch.from_numpy(sc.feat).to(dev)
    mlp = hp.to_device_mlp(sc.mlp, dev)
    tab = hp.build_table(xyz, sc.cams, sc.params)
    g = torch.randn(tab.n_rays, 3, device=dev, generator=torch.Generator(device=dev).manual_seed(seed))
    return tab, feat, mlp, g


def _compare(sc, prec, seed):
    import torch
    from paper_2404_14044_amd import hashpoint as hp
    dev = torch.device("cuda:0")
    tab, feat, mlp, g = _inputs(sc, dev, seed)
    gf_a, gm_a = hp.render_backward(tab, feat, mlp, sc.params, prec, g)
    # outputs allocated before the call: the call itself allocates nothing
    gf_b = torch.zeros_like(feat)
    gm_b = {k: torch.zeros_like(v) for k, v in mlp.items()}
    print(f"noalloc backward: {tab.n_rays} rays, precision {prec}", flush=True)
    hp.render_backward_noalloc(tab, feat, mlp, sc.params, prec, g, gf_b, gm_b)
    torch.cuda.synchronize()
    assert float(gf_a.abs().max()) > 0
    assert float((gf_a - gf_b).norm() / gf_a.norm()) < 1e-6
    for k in KEYS:
        den = gm_a[k].abs().max().clamp_min(1e-30)
        assert float((gm_a[k] - gm_b[k]).abs().max() / den) < 1e-5, k
    return tab.n_rays


@pytest.mark.parametrize("prec_name", ["fp32", "bf16"])
def test_noalloc_backward_equals_workspace_backward_twice(prec_name):
    """First call: four 96x96 views of a 100k-point object scene (36,864 rays,
    more than one recompute chunk of the scratch ring at K = 8, S = 16).
    Second call: one 48x48 view of the sphere-and-plane scene (2,304 rays,
    K = 8, S = 8), which must not see the first call's slices or samples."""
    from paper_2404_14044_amd import hashpoint as hp
    prec = hp.HP_FP32 if prec_name == "fp32" else hp.HP_BF16
    big = scenes.diff_4x400(base=scenes.objects_1m(n=100_000, res=64), res=96)
    small = scenes.sphere_plane(n_sphere=3000, n_plane=3000, res=48)
    r1 = _compare(big, prec, seed=7)
    r2 = _compare(small, prec, seed=8)
    assert r2 < r1
