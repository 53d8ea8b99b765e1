"""Pins of the oracle's BF16-decoder render and gradient (reading R22: the
decoder's operands -- aggregated feature, hidden activations, weights -- are
rounded to bfloat16; biases, sums and everything outside the decoder are not).

* or_bf16 rounds like the textbook float32 -> bfloat16 round-to-nearest-even
  on the float32 bit pattern, and keeps ties even;
* with weights, features and every activation exactly representable in
  bfloat16 (small dyadic values), the BF16 render and gradient equal the
  unrounded ones bit for bit;
* the BF16 gradient treats each rounding as x -> x + (fixed offset): central
  differences of the render with the recorded offsets held fixed (a smooth
  function that equals the BF16 render at the recording point) agree with it.
"""
import numpy as np
import pytest

from paper_2404_14044_amd import scenes


def _bf16_bits_reference(x32):
    u = np.asarray(x32, np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def test_bf16_rounding_matches_float32_bit_rounding(orc, rng):
    x = np.concatenate([rng.normal(size=2000) * 10.0 ** rng.integers(-30, 30, 2000),
                        rng.uniform(-1, 1, 2000)]).astype(np.float32)
    # exact ties: 1 + (2k + 1) 2^-8 sits halfway between two bfloat16 values
    ties = (1.0 + (2 * np.arange(64) + 1) * 2.0 ** -8).astype(np.float32)
    x = np.concatenate([x, ties, -ties])
    got = orc.bf16(x.astype(np.float64))
    assert np.array_equal(got, _bf16_bits_reference(x).astype(np.float64))
    # ties go to the even neighbour: 1 + 2^-8 -> 1, 1 + 3 2^-8 -> 1 + 2^-6
    assert orc.bf16([1.0 + 2.0 ** -8])[0] == 1.0
    assert orc.bf16([1.0 + 3 * 2.0 ** -8])[0] == 1.0 + 2.0 ** -6


def _dyadic_case(rng):
    """One view, K = 1 and eps_idw = 1 (so every aggregated feature is one
    point's feature), small-integer features and sparse weights of +-1/8:
    every decoder operand and activation has at most 8 significant bits."""
    sc = scenes.tiny_scene(seed=3)
    n = sc.xyz.shape[0]
    feat = rng.integers(-4, 5, size=(n, 32)).astype(np.float32)
    mlp = {}
    for name, (o, i) in (("W1", (64, 32)), ("W2", (64, 64)), ("W3", (4, 64))):
        W = np.zeros((o, i), np.float32)
        for r in range(o):
            cols = rng.choice(i, 4, replace=False)
            W[r, cols] = rng.choice([-0.125, 0.125], 4)
        mlp[name] = W
    for name, o in (("b1", 64), ("b2", 64), ("b3", 4)):
        mlp[name] = (rng.integers(-8, 9, o) / 64.0).astype(np.float32)
    p = sc.params.replace(K=1, eps_idw=1.0)
    return sc, feat, mlp, p


def test_bf16_exact_operands_equal_unrounded(orc, rng):
    sc, feat, mlp, p = _dyadic_case(rng)
    cam = sc.cams[0]
    pc = orc.to_camera(sc.xyz, cam)
    ex = orc.exact(pc, cam, p)
    assert (ex["n_sel"] > 0).sum() > 20
    a = orc.render64(pc, feat, mlp, cam, p, ex)
    b = orc.render64(pc, feat, mlp, cam, p, ex, quant=orc.QUANT_BF16)
    for k in ("rgb", "depth", "acc"):
        assert np.array_equal(a[k], b[k]), k
    gr = rng.normal(size=(ex["pix"].size, 3))
    ga = orc.grad64(pc, feat, mlp, cam, p, ex, gr)
    gb = orc.grad64(pc, feat, mlp, cam, p, ex, gr, quant=orc.QUANT_BF16)
    assert np.abs(ga["feat"]).max() > 0
    for k in ga:
        assert np.array_equal(ga[k], gb[k]), k


def _generic(orc, seed):
    sc = scenes.tiny_scene(seed=seed)
    cam, p = sc.cams[0], sc.params
    pc = orc.to_camera(sc.xyz, cam)
    ex = orc.exact(pc, cam, p)
    return sc, cam, p, pc, ex


def test_bf16_render_rounds_and_stays_close(orc):
    sc, cam, p, pc, ex = _generic(orc, 1)
    a = orc.render64(pc, sc.feat, sc.mlp, cam, p, ex)
    b = orc.render64(pc, sc.feat, sc.mlp, cam, p, ex, quant=orc.QUANT_BF16)
    d = np.abs(a["rgb"] - b["rgb"]).max()
    assert 1e-6 < d < 2e-2, d
    assert np.array_equal(a["depth"] == 0, b["depth"] == 0)


def test_frozen_offsets_reproduce_bf16_render(orc):
    sc, cam, p, pc, ex = _generic(orc, 2)
    off = orc.QuantOffsets(ex["pix"].size, p)
    b = orc.render64(pc, sc.feat, sc.mlp, cam, p, ex, quant=orc.QUANT_BF16, offsets=off)
    f = orc.render64(pc, sc.feat, sc.mlp, cam, p, ex, quant=orc.QUANT_FROZEN, offsets=off)
    assert np.abs(off.act).max() > 0 and np.abs(off.w).max() > 0
    for k in ("rgb", "depth", "acc"):
        assert np.array_equal(b[k], f[k]), k
    with pytest.raises(ValueError):
        orc.render64(pc, sc.feat, sc.mlp, cam, p, ex, quant=orc.QUANT_FROZEN)


def test_bf16_gradient_matches_central_differences_of_frozen_render(orc):
    sc, cam, p, pc, ex = _generic(orc, 1)
    rng = np.random.default_rng(6)
    R = ex["pix"].size
    gr = rng.normal(size=(R, 3))
    off = orc.QuantOffsets(R, p)
    orc.render64(pc, sc.feat, sc.mlp, cam, p, ex, quant=orc.QUANT_BF16, offsets=off)
    g = orc.grad64(pc, sc.feat, sc.mlp, cam, p, ex, gr, quant=orc.QUANT_BF16)
    g_frozen = orc.grad64(pc, sc.feat, sc.mlp, cam, p, ex, gr, quant=orc.QUANT_FROZEN, offsets=off)
    for k in g:
        assert np.array_equal(g[k], g_frozen[k]), k
    g0 = orc.grad64(pc, sc.feat, sc.mlp, cam, p, ex, gr)
    # the roundings move the gradient, by far less than its size
    rel = np.linalg.norm(g["feat"] - g0["feat"]) / np.linalg.norm(g0["feat"])
    assert 1e-6 < rel < 0.2, rel

    def loss(feat, mlp):
        out = orc.render64(pc, feat, mlp, cam, p, ex, quant=orc.QUANT_FROZEN, offsets=off)
        return float((out["rgb"] * gr).sum())

    used = np.unique(ex["knn_idx"][ex["knn_idx"] >= 0])
    checks = [("feat", (int(i), int(c))) for i, c in
              zip(rng.choice(used, 12), rng.integers(0, 32, 12))]
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        for _ in range(4):
            checks.append((name, tuple(int(rng.integers(0, s)) for s in sc.mlp[name].shape)))
    for name, ij in checks:
        base = sc.feat if name == "feat" else sc.mlp[name]
        h = 1e-5
        vals = []
        for sgn in (+1, -1):
            pert = base.astype(np.float64).copy()
            pert[ij] += sgn * h
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
