"""Schedule tuner for gbsub.

The loop's schedule has two knobs that do not change what is computed:
the tile size (bins per median block, binning bucket and dirty-flag unit)
and the split budget (how many dirty tiles the median still runs as one
block per 512-bin part).  `tune` times gbsub_run over a grid of both on the
caller's catalog and keeps the fastest setting whose resolved set and loop
count equal those of the default schedule (a different association of the
fp64 sums of 1/S can only move decisions within ~1e-15 of the threshold).

    best = tune(device_catalog, run_config)        # {"tile_bins": .., "split_blocks": ..}
    ctx = Context(config_from_run(run, **best))
"""
from __future__ import annotations

import time

import numpy as np

from . import gbsub as G

TILES = (2048, 1024, 512)
SPLITS = (1, 128, 256, 512, 1024, 2048)


def feasible_tiles(window_bins: int, tiles=TILES):
    room = 3072 - (window_bins - 1)
    return [t for t in tiles if t <= room]


def _time_run(cfg, dc, reps, stream=None):
    import torch
    ctx = G.Context(cfg)
    try:
        ctx.ensure_workspace(dc.n)
        s = ctx.run(dc)                                   # warm: tables, allocation
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            s = ctx.run(dc)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        ids, _ = ctx.resolved()
        return float(np.median(ts)) * 1e3, s, ids
    finally:
        ctx.close()


def tune(dc, run, tiles=TILES, splits=SPLITS, reps: int = 3, log=None):
    """Returns (best setting dict, table of (tile, split, ms)).  `dc` is a
    DeviceCatalog, `run` an inputs.RunConfig (or dict)."""
    d = run.as_dict() if hasattr(run, "as_dict") else dict(run)
    base_ms, base_s, base_ids = _time_run(G.config_from_run(d), dc, reps)
    table = [(0, 0, base_ms)]
    best, best_ms = {"tile_bins": 0, "split_blocks": 0}, base_ms
    for tile in feasible_tiles(d["window_bins"], tiles):
        for split in splits:
            cfg = G.config_from_run(d, tile_bins=tile, split_blocks=split)
            ms, s, ids = _time_run(cfg, dc, reps)
            same = s.n_iter == base_s.n_iter and np.array_equal(ids, base_ids)
            table.append((tile, split, ms if same else float("nan")))
            if log:
                log(f"[tune] tile {tile} split {split}: {ms:.3f} ms{'' if same else ' (different result)'}")
            if same and ms < best_ms:
                best, best_ms = {"tile_bins": tile, "split_blocks": split}, ms
    return best, table
