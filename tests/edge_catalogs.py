"""Catalogs whose subtractions change running-median windows at the grid
edges, where the window is shifted inward (Eq. "running median", window of W
bins clamped to the grid) and one bin can move outputs up to 2h = W - 1 away.

Each catalog has a dense block of moderate sources (candidates that never
resolve: 4 q / S stays far below 49) that gives the windows a nonzero median,
plus loud sources (rho_0^2 of several hundred) that resolve in the first loop
body inside the edge window but more than h bins away from the outputs at the
edge.  The next body must then refilter the edge outputs too.
"""
import numpy as np

from oracle import oracle as O
from tests.helpers import amp_for_power, bin_freq, catalog, small_run


def _build(B, W, dense, loud, n_dense, n_loud, seed, estimator):
    run, k0 = small_run(n_bins=B, W=W, estimator=estimator)
    Sx = O.sinstr_table(O.make_config(run))
    T = run.t_obs_s
    rng = np.random.default_rng(seed)
    db = rng.integers(dense[0], dense[1] + 1, n_dense)
    lb = rng.integers(loud[0], loud[1] + 1, n_loud)
    P = np.concatenate([Sx[db] * 0.3 * rng.exponential(1.0, n_dense),
                        Sx[lb] * rng.uniform(100.0, 300.0, n_loud)])
    bins = np.concatenate([db, lb])
    perm = rng.permutation(bins.size)
    P, bins = P[perm], bins[perm]
    cat = catalog([amp_for_power(p, T) for p in P], [bin_freq(k0, int(b), T) for b in bins])
    return cat, run


def upper_edge(estimator=0):
    """W = 1001 (tile 2048), B = 3 * 2048 + 100: the last tile holds 100 <= h
    bins.  Loud sources in [B-1001, B-601] lie in the upper edge window
    [B-W, B-1] but more than h bins below the last tile."""
    B = 3 * 2048 + 100
    cat, run = _build(B, 1001, (B - 1400, B - 1), (B - 1001, B - 601), 1400, 100, seed=31, estimator=estimator)
    return cat, run, {}


def lower_edge(estimator=0):
    """W = 2817 (tile 256): loud sources in [1700, 2800] lie in the lower edge
    window [0, W-1] but more than h = 1408 bins above tile 0."""
    cat, run = _build(6000, 2817, (0, 3500), (1700, 2800), 3500, 120, seed=32, estimator=estimator)
    return cat, run, {}


def short_grid(estimator=0):
    """B = 900 < W = 1001 with 256-bin tiles: every output's window is the
    whole grid; loud sources in [0, 200] are more than h bins below tile 3."""
    cat, run = _build(900, 1001, (0, 899), (0, 200), 900, 40, seed=33, estimator=estimator)
    return cat, run, {"tile_bins": 256}


CASES = {"upper_edge": upper_edge, "lower_edge": lower_edge, "short_grid": short_grid}
