"""Autotuner of the batched iteration: tile shape, LDS batch, work-chunk
size of the persistent render kernels, the backward variant (pixel-wise
or splat-wise) and the tile binning (per-tile slot claims and sorts, or
the two radix sorts).  Each candidate is planned, captured
as a whole-iteration HIP graph and timed by the library's gs_graph_time (HIP
events on the replay stream); the fastest is returned and optionally cached
as JSON keyed by the workload signature.  Tuning runs on a copy of the
parameters, so the caller's model is not stepped.

Tile shape never changes the rendered image (the tile box is the exact
alpha >= 1/255 box), so the choice is purely a performance one.
"""
from __future__ import annotations

import itertools
import json
import os
from typing import Dict, List, Optional, Sequence, Tuple

import torch

from . import _lib as L
from .raster import Gaussians, Iteration, Plan, required_pairs

TILES = [(16, 16), (16, 8), (8, 8)]
LDS_BATCHES = [64, 128, 256]
CHUNKS = [1, 2, 4, 8]
BACKWARDS = ["pixel", "splat"]
BINNINGS = ["tiles", "radix"]


def signature(g: Gaussians, view_wh, flags) -> str:
    return json.dumps({"n": g.n, "deg": g.sh_degree, "views": [list(v) for v in view_wh],
                       "flags": int(flags)}, sort_keys=True)


def autotune(g: Gaussians, cams: torch.Tensor, view_wh: Sequence[Tuple[int, int]],
             target_rgb=None, target_depth=None, dL_dcolor=None, dL_ddepth=None,
             adam_lrs: Optional[dict] = None, persistent: bool = True,
             tiles=TILES, lds_batches=LDS_BATCHES, chunks=CHUNKS, backwards=BACKWARDS,
             binnings=("tiles",), reps: int = 10,
             cache_path: Optional[str] = None, log=None) -> Tuple[dict, List[dict]]:
    base_flags = (L.GS_FUSED_L1 if target_rgb is not None else 0) | (L.GS_PERSISTENT if persistent else 0)
    key = signature(g, view_wh, base_flags) + json.dumps(list(backwards)) + json.dumps(
        list(binnings))
    if cache_path and os.path.exists(cache_path):
        cache = json.load(open(cache_path))
        if key in cache:
            return cache[key]["best"], cache[key]["table"]
    work = Gaussians(*[t.clone() for t in g.tensors()], g.sh_degree)
    stream = torch.cuda.Stream()
    table = []
    for tile in tiles:
        cap = int(required_pairs(*work.tensors(), cams, view_wh, work.sh_degree, tile) * 1.3) + 4096
        for lds, chunk, bwd, binning in itertools.product(
                lds_batches, chunks if persistent else [1], backwards, binnings):
            flags = (base_flags | (L.GS_SPLAT_BWD if bwd == "splat" else 0) |
                     (L.GS_RADIX_BIN if binning == "radix" else 0))
            plan = Plan(work.n, work.sh_degree, view_wh, tile=tile, lds_batch=lds, chunk=chunk,
                        flags=flags, pair_capacity=cap)
            it = Iteration(plan, work, cams, target_rgb=target_rgb, target_depth=target_depth,
                           dL_dcolor=dL_dcolor, dL_ddepth=dL_ddepth, adam_lrs=adam_lrs)
            with torch.cuda.stream(stream):
                it.capture(stream)
                ms = it.time_graph(stream, warmup=2, reps=reps)
            over = int(plan.flags_of(it.ws)[L.F_OVERFLOW])
            it.close()
            row = {"tile": f"{tile[0]}x{tile[1]}", "lds_batch": lds, "chunk": chunk,
                   "backward": bwd, "binning": binning, "ms": round(ms, 4), "overflow": over}
            table.append(row)
            if log:
                log(row)
            del it
    ok = [r for r in table if not r["overflow"]]
    best = min(ok, key=lambda r: r["ms"])
    if cache_path:
        cache = json.load(open(cache_path)) if os.path.exists(cache_path) else {}
        cache[key] = {"best": best, "table": table}
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return best, table
