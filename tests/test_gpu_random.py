"""Randomized parity: seeded small catalogs on random grids, windows, tiles,
split budgets and estimators, for the power model (gbsub_run) and the
complex-template model (gbsub_cx_run), each against the FP64 oracle with
the bars of tests/oracle_bar.py and tests/test_gpu_cx.py.

Amplitudes are drawn from the SNR a source would have alone against the
instrument (log-uniform over [0.3, 60]), so every case resolves some sources,
leaves some candidates unresolved and has cascades; frequencies reach 60
bins past either grid edge; fdot gives one-bin, narrow and wide tracks.
"""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2602_18560_amd import gbsub as G
from paper_2602_18560_amd.inputs import Catalog, RunConfig, YEAR_S, template_phases
from tests import oracle_bar as OB
from tests.test_gpu_cx import assert_cx_parity

pytestmark = pytest.mark.gpu

N_CASES = 24


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def random_case(seed):
    rng = np.random.default_rng(7000 + seed)
    T = float(rng.choice([0.5, 1.0, 2.0])) * YEAR_S
    n_bins = int(rng.integers(40, 20000))
    k0 = math.floor(10 ** rng.uniform(-3.7, -2.3) * T + 0.5)
    W = int(rng.choice([1, 3, 5, 31, 101, 251, 501, 1001]))
    est = int(rng.random() < 0.2)
    run = RunConfig(t_obs_s=T, f_min_hz=k0 / T, f_max_hz=(k0 + n_bins - 1) / T, window_bins=W, estimator=est)
    kw = {}
    tile = int(rng.choice([0, 256, 512, 1024, 2048]))
    if tile:
        kw["tile_bins"] = tile
    split = int(rng.choice([0, 1, 1 << 20]))
    if split:
        kw["split_blocks"] = split
    n = int(rng.integers(0, 4000))
    pos = rng.uniform(-60, n_bins + 60, n)
    f = (k0 + pos) / T
    kind = rng.random(n)
    d = np.where(kind < 0.3, 0.0, np.where(kind < 0.9, rng.uniform(0, 5, n), rng.uniform(5, 500, n)))
    fd = d * rng.choice([-1.0, 1.0], n) / T ** 2
    rho = 10 ** rng.uniform(math.log10(0.3), math.log10(60.0), n)
    sx = np.array([O.sinstr(max(x, 1e-5)) for x in f])
    A = rho * np.sqrt(sx / (2.0 * T))
    cat = Catalog(A.astype(np.float32), f.astype(np.float32), fd.astype(np.float32),
                  rng.permutation(n).astype(np.uint32) * 3 + 1)
    return cat, run, kw


@pytest.mark.parametrize("seed", range(N_CASES))
def test_power_model_random_case(seed):
    cat, run, kw = random_case(seed)
    say(f"[random power {seed}] n={cat.n} B~{round((run.f_max_hz - run.f_min_hz) * run.t_obs_s) + 1} "
        f"W={run.window_bins} est={run.estimator} {kw}")
    ctx = G.Context(G.config_from_run(run, **kw))
    try:
        st, s = ctx.run_raw(G.DeviceCatalog.from_host(cat))
        assert st == G.OK, G.status_str(st)
        S, X = ctx.spectrum(G.SPEC_SN), ctx.spectrum(G.SPEC_X_RESIDUAL)
        ids, it = ctx.resolved()
    finally:
        ctx.close()
    OB.check(cat, O.make_config(run), s, S, X, ids, it)


@pytest.mark.parametrize("seed", range(N_CASES))
def test_template_model_random_case(seed):
    cat, run, kw = random_case(seed)
    pa, pe = template_phases(cat.n, 7000 + seed)
    assert_cx_parity(cat, pa, pe, run, f"random {seed}", **kw)
