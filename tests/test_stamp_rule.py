"""The dirty-tile rule of the loop (host logic, checked on the CPU).

After a loop body subtracts a source with clipped track [glo, ghi], the next
body refilters only the tiles holding an output whose window contains a bin
of the track; every other output keeps its S.  Stated in Python here, the
rule must cover every bin where the oracle's S^{t+1} differs from S^t, on
catalogs built so that the clamped edge windows matter (Eq. "running
median": the window is shifted inward at the grid edges, and the whole grid
when B < W).  The naive rule [glo - h, ghi + h] must miss some of them, so
that these catalogs really exercise the edges (the GPU parity tests run the
same catalogs).
"""
import numpy as np
import pytest

from oracle import oracle as O
from tests.edge_catalogs import CASES


def tile_of_run(run, tile_bins=0):
    """The default tile: the largest power of two <= 2048 with
    tile + W - 1 <= 3072."""
    if tile_bins:
        return tile_bins
    t = 2048
    while t > 3072 - (run.window_bins - 1):
        t >>= 1
    return t


def reach_edge_aware(glo, ghi, B, W):
    h = (W - 1) // 2
    whole = B < W
    a = 0 if (whole or glo <= W - 1) else glo - h
    b = B - 1 if (whole or ghi >= B - W) else ghi + h
    return a, b


def reach_naive(glo, ghi, B, W):
    h = (W - 1) // 2
    return max(glo - h, 0), min(ghi + h, B - 1)


def emulate(cat, run, tile, reach):
    """S as a loop that refilters only the stamped tiles would hold it,
    given the oracle's decisions; returns (final S, oracle final S, number of
    (t, bin) where S changed on an unstamped tile)."""
    cfg = O.make_config(run)
    r = O.run(cat, cfg, trace=True, trace_fields=("S",))
    B, W = r.n_bins, run.window_bins
    tracks = [O.track(cfg, float(a), float(f), float(fd)) for a, f, fd in zip(cat.A, cat.f, cat.fdot)]
    S = r.trace[0]["S"].copy()
    missed = 0
    for t in range(len(r.trace) - 1):
        stamped = np.zeros((B + tile - 1) // tile, bool)
        for i in np.flatnonzero(r.iter_of == t):
            tr = tracks[i]
            if tr["glo"] > tr["ghi"]:
                continue
            a, b = reach(tr["glo"], tr["ghi"], B, W)
            stamped[a // tile: b // tile + 1] = True
        nxt = r.trace[t + 1]["S"]
        changed = np.flatnonzero(nxt != r.trace[t]["S"])
        missed += int(np.count_nonzero(~stamped[changed // tile]))
        for tl in np.flatnonzero(stamped):
            S[tl * tile:(tl + 1) * tile] = nxt[tl * tile:(tl + 1) * tile]
    return S, r.S_final, missed, r


@pytest.mark.parametrize("estimator", [O.MEDIAN, O.MEAN])
@pytest.mark.parametrize("case", sorted(CASES))
def test_edge_aware_rule_covers_every_change(case, estimator):
    cat, run, kw = CASES[case](estimator)
    tile = tile_of_run(run, kw.get("tile_bins", 0))
    S, S_ref, missed, r = emulate(cat, run, tile, reach_edge_aware)
    assert r.n_iter >= 2 and r.n_resolved > 0
    assert missed == 0
    np.testing.assert_array_equal(S, S_ref)


@pytest.mark.parametrize("estimator", [O.MEDIAN, O.MEAN])
@pytest.mark.parametrize("case", sorted(CASES))
def test_naive_rule_leaves_stale_edges(case, estimator):
    cat, run, kw = CASES[case](estimator)
    tile = tile_of_run(run, kw.get("tile_bins", 0))
    S, S_ref, missed, _ = emulate(cat, run, tile, reach_naive)
    assert missed > 0
    assert np.max(np.abs(S - S_ref) / S_ref) > 1e-4
