"""Autotuner for the bucket layout and the launch shapes of a frame.

None of the tuned values changes a result (the search is exact and the
render composites every ray from its own samples for any of them); they
trade work distribution against locality:
  layout          buckets row-major, in 8x8 tiles, or in 8x8 tiles in Z-order
                  (the Morton arrangement the paper mentions, Sec. 3.2);
  search_chunk    consecutive rays a search workgroup takes at a time;
  search_blocks   size of the search grid (workgroups dealt chunks of rays);
  search_band     consecutive rays dealt to one XCD (its own L2) at a time;
  window_shape    disc of buckets within the proven radius, or its square
                  (more buckets, fewer instructions per bucket);
  render_rays     rays a render wave composites at a time (its sample tile);
  render_blocks   size of the persistent render grid.
The objective is the time of one frame: table build + search + render of the
given views.  The search is coordinate descent from the defaults (each value
of one dimension tried with the others at their best so far, dimensions in
turn, twice over), so a workload costs a few dozen timed frames, not the
product of the ranges.  Results are cached by workload shape in an explicit
cache object that can be saved to and loaded from JSON; each entry keeps the
default and the tuned frame time and every trial.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Optional, Sequence

import torch

from . import hashpoint as hp

SPACE = {
    "layout": (hp.HP_LAYOUT_ROWMAJOR, hp.HP_LAYOUT_TILED, hp.HP_LAYOUT_MORTON),
    "search_chunk": (1, 2, 4, 8, 16),
    "search_blocks": (8192, 16384, 32768, 65536, 131072),
    "search_band": (800, 1600, 3200, 12800),
    "window_shape": (hp.HP_WINDOW_DISC, hp.HP_WINDOW_SQUARE),
    "render_rays": (16, 32, 64),
    "render_blocks": (0, 3072, 6144, 12288),
}
# the values the library takes for 0 (its defaults), the descent's start
DEFAULTS = {"layout": hp.HP_LAYOUT_ROWMAJOR, "search_chunk": 4, "search_blocks": 65536,
            "search_band": 1600, "window_shape": hp.HP_WINDOW_DISC, "render_rays": 16,
            "render_blocks": 0}


def shape_key(cams: Sequence, params, n_points: int, precision: int) -> str:
    return json.dumps({"views": [[int(c.W), int(c.H)] for c in cams], "n": int(n_points),
                       "K": int(params.K), "S": int(params.n_samples),
                       "r": float(params.radius), "inv_tref": float(params.inv_tref),
                       "radius_mode": int(params.radius_mode), "sampler": int(params.sampler),
                       "precision": int(precision)}, sort_keys=True)


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
        """Median of `reps` timed calls (ms, HIP events on the current stream)."""
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

    def _frame(self, xyz, feat, mlp, cams, params, precision, reps: int) -> float:
        """Time of build + search + render with these parameters (buffers
        allocated outside the timed calls)."""
        dev = xyz.device
        ws = torch.empty(hp.table_workspace(xyz.shape[0], cams, params), dtype=torch.uint8,
                         device=dev)
        R = sum(int(c.W) * int(c.H) for c in cams)
        smp = hp.alloc_samples(R, params, dev)
        out = {"rgb": torch.empty(R * 3, device=dev), "depth": torch.empty(R, device=dev),
               "acc": torch.empty(R, device=dev)}

        def frame():
            tab = hp.build_table(xyz, cams, params, ws=ws)
            hp.search_sample(tab, params, out=smp)
            hp.render(smp, R, feat, mlp, params, precision, out=out)

        return self._time(frame, reps)

    def tune(self, xyz: torch.Tensor, feat: torch.Tensor, mlp: Dict[str, torch.Tensor],
             cams: Sequence, params, precision: int = hp.HP_BF16, reps: int = 3,
             space: Optional[Dict[str, Sequence[int]]] = None, rounds: int = 2):
        """Return params with the fastest layout and launch shapes found."""
        key = shape_key(cams, params, xyz.shape[0], precision)
        if key in self.cache:
            return params.replace(**self.cache[key]["best"])
        space = dict(space or SPACE)
        best = {k: DEFAULTS[k] for k in space}
        trials = []

        def run(cfg):
            ms = self._frame(xyz, feat, mlp, cams, params.replace(**cfg), precision, reps)
            trials.append(dict(cfg, ms=ms))
            return ms

        default_ms = run(dict(best))
        best_ms = default_ms
        for _ in range(rounds):
            changed = False
            for dim, values in space.items():
                for v in values:
                    if v == best[dim]:
                        continue
                    cfg = dict(best, **{dim: v})
                    ms = run(cfg)
                    if ms < best_ms:
                        best_ms, best, changed = ms, cfg, True
            if not changed:
                break
        # the winner timed again beside the defaults, so that the two figures
        # kept in the cache come from the same moment (the defaults stay if
        # the winner's lead does not survive)
        default_cfg = {k: DEFAULTS[k] for k in space}
        default_ms = run(default_cfg)
        best_ms = run(dict(best))
        if default_ms <= best_ms:
            best, best_ms = default_cfg, default_ms
        self.cache[key] = {"best": best, "ms": best_ms, "default_ms": default_ms,
                           "trials": trials}
        self.save()
        return params.replace(**best)

    def entry(self, xyz, cams, params, precision: int = hp.HP_BF16) -> Optional[dict]:
        """The cached result for this workload, if it was tuned."""
        return self.cache.get(shape_key(cams, params, xyz.shape[0], precision))
