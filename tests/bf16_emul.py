"""Reference for the BF16-forward gradient: the render's gradient when the
decoder's operands (aggregated feature, hidden activations, weights) are
rounded to bfloat16 (round to nearest even) and everything else is binary64.
The binary64 oracle differentiates the unrounded decoder, so the two differ by
the effect of those roundings (mostly ReLU units whose sign flips); this
reference isolates that effect.  Geometry comes from the oracle's exact stage."""
import numpy as np

import oracle


def bf16(x):
    x = np.asarray(x, np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def _sig(x):
    return 1.0 / (1.0 + np.exp(-x))


def _softplus(x):
    return np.maximum(x, 0) + np.log1p(np.exp(-np.abs(x)))


def grad_bf16(pc, feat, mlp, cam, p, ex, grad_rgb):
    W1, b1, W2, b2, W3, b3 = [np.asarray(mlp[k], np.float32) for k in ("W1", "b1", "W2", "b2", "W3", "b3")]
    q1, q2, q3 = (bf16(w).astype(np.float64) for w in (W1, W2, W3))
    out = {"feat": np.zeros(feat.shape), "W1": np.zeros(W1.shape), "b1": np.zeros(b1.shape),
           "W2": np.zeros(W2.shape), "b2": np.zeros(b2.shape), "W3": np.zeros(W3.shape),
           "b3": np.zeros(b3.shape)}
    bg = np.asarray(p.bg, np.float64)
    for r, pix in enumerate(ex["pix"]):
        n = int(ex["n_sel"][r])
        g = np.asarray(grad_rgb[r], np.float64)
        if n == 0 or not g.any():
            continue
        d = oracle.ray_dir(cam, int(pix) % cam.W, int(pix) // cam.W).astype(np.float64)
        t = ex["t"][r, :n].astype(np.float64)
        st = []
        for s in range(n):
            idx = ex["knn_idx"][r, s]
            idx = idx[idx >= 0]
            dist = np.linalg.norm(pc[idx].astype(np.float64) - t[s] * d, axis=1)
            w = 1.0 / np.maximum(dist, p.eps_idw)
            wn = w / w.sum()
            f = (wn[:, None] * feat[idx]).sum(0)
            h1 = np.maximum(q1 @ bf16(f) + b1, 0)
            h2 = np.maximum(q2 @ bf16(h1) + b2, 0)
            o = q3 @ bf16(h2) + b3
            st.append((idx, wn, f, h1, h2, o))
        T, Ts = 1.0, []
        for j in range(n):
            Ts.append(T)
            dl = t[j + 1] - t[j] if j + 1 < n else p.delta_last
            T *= np.exp(-_softplus(st[j][5][3]) * dl)
        U, P = np.zeros(3), 1.0
        for j in range(n - 1, -1, -1):
            idx, wn, f, h1, h2, o = st[j]
            c = _sig(o[:3])
            dl = t[j + 1] - t[j] if j + 1 < n else p.delta_last
            e = np.exp(-_softplus(o[3]) * dl)
            a = 1.0 - e
            dlda = float((g * (Ts[j] * (c - U) - bg * Ts[j] * P)).sum())
            do = np.concatenate([g * Ts[j] * a * c * (1 - c), [dlda * dl * e * _sig(o[3])]])
            U, P = a * c + e * U, e * P
            dh2 = (W3.T.astype(np.float64) @ do) * (h2 > 0)
            dh1 = (W2.T.astype(np.float64) @ dh2) * (h1 > 0)
            df = W1.T.astype(np.float64) @ dh1
            out["W3"] += np.outer(do, h2)
            out["b3"] += do
            out["W2"] += np.outer(dh2, h1)
            out["b2"] += dh2
            out["W1"] += np.outer(dh1, f)
            out["b1"] += dh1
            np.add.at(out["feat"], idx, wn[:, None] * df[None, :])
    return out
