"""Autotuner for the launch shape of the search kernel and the bucket layout.

None of the tuned values changes a result (the search is exact for any of
them); they trade work distribution against locality:
  layout         row-major buckets, or 8x8-pixel tiles stored contiguously;
  search_chunk   consecutive rays one workgroup takes at a time;
  search_blocks  size of the persistent search grid.
Results are cached by workload shape in an explicit cache object that can be
saved to and loaded from JSON.
"""
from __future__ import annotations

import itertools
import json
import os
from typing import Dict, Optional, Sequence

import torch

from . import hashpoint as hp

LAYOUTS = (hp.HP_LAYOUT_ROWMAJOR, hp.HP_LAYOUT_TILED)
CHUNKS = (1, 2, 4, 8, 16)
BLOCKS = (2048, 4096, 8192, 16384)


def shape_key(cams: Sequence, params, n_points: int) -> str:
    return json.dumps({"views": [[int(c.W), int(c.H)] for c in cams], "n": int(n_points),
                       "K": int(params.K), "S": int(params.n_samples),
                       "r": float(params.radius), "inv_tref": float(params.inv_tref)},
                      sort_keys=True)


class Autotuner:
    def __init__(self, cache_path: Optional[str] = None):
        self.cache_path = cache_path
        self.cache: Dict[str, dict] = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.cache = json.load(f)

    def save(self):
        if self.cache_path:
            with open(self.cache_path, "w") as f:
                json.dump(self.cache, f, indent=1, sort_keys=True)

    @staticmethod
    def _time(fn, reps: int) -> float:
        fn()
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
        times.sort()
        return times[len(times) // 2]

    def tune(self, xyz: torch.Tensor, cams: Sequence, params, reps: int = 3,
             layouts=LAYOUTS, chunks=CHUNKS, blocks=BLOCKS):
        """Return params with the fastest (layout, search_chunk, search_blocks)."""
        key = shape_key(cams, params, xyz.shape[0])
        if key in self.cache:
            return params.replace(**self.cache[key]["best"])
        trials = []
        for layout in layouts:
            p = params.replace(layout=layout)
            ws = torch.empty(hp.table_workspace(xyz.shape[0], cams, p), dtype=torch.uint8,
                             device=xyz.device)
            holder = {}

            def build():
                holder["tab"] = hp.build_table(xyz, cams, p, ws=ws)

            t_build = self._time(build, reps)
            tab = holder["tab"]
            out = hp.alloc_samples(tab.n_rays, p, xyz.device)
            for ch, bl in itertools.product(chunks, blocks):
                q = p.replace(search_chunk=ch, search_blocks=bl)
                t_search = self._time(lambda: hp.search_sample(tab, q, out=out), reps)
                trials.append({"layout": layout, "search_chunk": ch, "search_blocks": bl,
                               "build_ms": t_build, "search_ms": t_search,
                               "ms": t_build + t_search})
            del ws, out, tab, holder
        best = min(trials, key=lambda t: t["ms"])
        self.cache[key] = {"best": {k: best[k] for k in ("layout", "search_chunk", "search_blocks")},
                           "ms": best["ms"], "trials": trials}
        self.save()
        return params.replace(**self.cache[key]["best"])
