"""Many views in one pass, replayed from a captured HIP graph.

All views share one table (one build launch per phase for every view), one
persistent search + sampling launch over the rays of every view, and one
persistent render launch over chunks of those rays.  Buffers are sized once for the views, so the whole frame can
be captured into a graph and each later frame is a single graph launch.
`render_views_separately` is the per-view baseline: one build, one search and
one render per view.
"""
from __future__ import annotations

from typing import Dict, List, Sequence

import torch

from . import hashpoint as hp


class BatchedRenderer:
    """All views in one build / search / render (capturable as one graph).
    With `tuner` (an autotune.Autotuner) the bucket layout and launch shapes
    are the tuner's choice for these views (tuned on first use, then cached);
    no result depends on them."""

    def __init__(self, xyz: torch.Tensor, feat: torch.Tensor, mlp: Dict[str, torch.Tensor],
                 cams: Sequence, params, precision: int = hp.HP_BF16, tuner=None):
        self.xyz, self.feat, self.mlp = xyz, feat, mlp
        self.cams, self.precision = list(cams), precision
        if tuner is not None:
            params = tuner.tune(xyz, feat, mlp, self.cams, params, precision)
        self.params = params
        dev = xyz.device
        self.ws = torch.empty(hp.table_workspace(xyz.shape[0], self.cams, params),
                              dtype=torch.uint8, device=dev)
        self.n_rays = sum(int(c.W) * int(c.H) for c in self.cams)
        self.samples = hp.alloc_samples(self.n_rays, params, dev)
        self.out = {"rgb": torch.empty(self.n_rays * 3, device=dev),
                    "depth": torch.empty(self.n_rays, device=dev),
                    "acc": torch.empty(self.n_rays, device=dev)}
        self.graph = None
        self.table = None

    def run_eager(self):
        self.table = hp.build_table(self.xyz, self.cams, self.params, ws=self.ws)
        hp.search_sample(self.table, self.params, out=self.samples)
        hp.render(self.samples, self.n_rays, self.feat, self.mlp, self.params, self.precision,
                  out=self.out)
        return self.out

    def capture(self):
        """Record build + search + render into one graph (after an eager run)."""
        self.run_eager()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run_eager()
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            self.capture()
        self.graph.replay()
        return self.out

    def ray_slices(self) -> List[slice]:
        out, base = [], 0
        for c in self.cams:
            n = int(c.W) * int(c.H)
            out.append(slice(base, base + n))
            base += n
        return out


def render_views_separately(xyz, feat, mlp, cams, params, precision=hp.HP_BF16, state=None):
    """Baseline: a full build / search / render sequence per view."""
    dev = xyz.device
    if state is None:
        state = []
        for c in cams:
            R = int(c.W) * int(c.H)
            state.append({
                "ws": torch.empty(hp.table_workspace(xyz.shape[0], [c], params), dtype=torch.uint8,
                                  device=dev),
                "smp": hp.alloc_samples(R, params, dev),
                "out": {"rgb": torch.empty(R * 3, device=dev), "depth": torch.empty(R, device=dev),
                        "acc": torch.empty(R, device=dev)},
            })
    for c, st in zip(cams, state):
        tab = hp.build_table(xyz, [c], params, ws=st["ws"])
        hp.search_sample(tab, params, out=st["smp"])
        hp.render(st["smp"], tab.n_rays, feat, mlp, params, precision, out=st["out"])
    return state
