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


BATCH_TILES = (2048, 1024)
BATCH_SPLITS = (512, 2048, 8192, 32768)


def grid_class(run) -> tuple:
    """The key of a run's grid class: catalogs of one class share the grid
    and window, hence one schedule."""
    d = run.as_dict() if hasattr(run, "as_dict") else dict(run)
    return (float(d["t_obs_s"]), float(d["f_min_hz"]), float(d["f_max_hz"]), int(d["window_bins"]))


def run_batch(dcs, runs, schedule=None, chunk: int = 4, stream=None, workspaces=None):
    """Runs the catalogs `dcs` (with their RunConfigs) together as one batch
    to completion; returns (seconds, [Summary]) in catalog order."""
    import torch
    stream = stream or torch.cuda.Stream()
    sch = schedule or {}
    ctxs = [G.Context(G.config_from_run(r, **sch)) for r in runs]
    batch = G.Batch(len(dcs))
    try:
        wss = workspaces or [None] * len(dcs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for c, d, w in zip(ctxs, dcs, wss):
            batch.admit(c, d, ws=w, stream=stream)
        while True:
            _, running = batch.poll(stream)
            if running == 0:
                break
            batch.step(chunk, stream)
        out = []
        for k in range(len(dcs)):
            st, s = batch.retire(k, stream)
            if st != G.OK:
                raise G.GbsubError(st, "batched run")
            out.append(s)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, out
    finally:
        batch.close()
        for c in ctxs:
            c.close()


def tune_batch(dcs, runs, tiles=BATCH_TILES, splits=BATCH_SPLITS, chunk: int = 4, reps: int = 1, log=None):
    """Schedule for catalogs of one grid class run together as a batch: each
    setting runs the whole set through one batch, timed end to end, and the
    fastest whose loop and resolved counts equal those of the default
    schedule wins.  The split budget is shared by the running catalogs, so
    its best value for a batch is larger than for one catalog.  Returns
    (best setting dict, table of (tile, split, seconds))."""
    import torch
    d0 = runs[0].as_dict() if hasattr(runs[0], "as_dict") else dict(runs[0])
    # one workspace per catalog, large enough for every tile size tried (the
    # layout depends on the tile both ways: more tiles, larger partial sums)
    cand_tiles = [0] + feasible_tiles(d0["window_bins"], tiles)
    wss = []
    for r, dc in zip(runs, dcs):
        need = 0
        for t in cand_tiles:
            c = G.Context(G.config_from_run(r, tile_bins=t))
            need = max(need, c.workspace_size(dc.n))
            c.close()
        wss.append(torch.empty(need + 256, dtype=torch.uint8, device="cuda"))
    stream = torch.cuda.Stream()

    def timed(sch):
        best_t, summ = None, None
        for _ in range(reps):
            t, summ = run_batch(dcs, runs, sch, chunk, stream, wss)
            best_t = t if best_t is None else min(best_t, t)
        return best_t, [(s.n_iter, s.n_resolved) for s in summ]

    run_batch(dcs, runs, None, chunk, stream, wss)                   # warm
    base_t, base = timed({"tile_bins": 0, "split_blocks": 0})
    table = [(0, 0, base_t)]
    best, best_t = {"tile_bins": 0, "split_blocks": 0}, base_t
    for tile in feasible_tiles(d0["window_bins"], tiles):
        for split in splits:
            sch = {"tile_bins": tile, "split_blocks": split}
            t, res = timed(sch)
            same = res == base
            table.append((tile, split, t if same else float("nan")))
            if log:
                log(f"[tune-batch] tile {tile} split {split}: {t * 1e3:.1f} ms"
                    f"{'' if same else ' (different result)'}")
            if same and t < best_t:
                best, best_t = sch, t
    return best, table
