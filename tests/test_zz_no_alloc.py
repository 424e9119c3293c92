"""gbsub_run_static (the run in the library's fixed per-GPU array, for
callers that cannot allocate) against gbsub_run on the same catalogs.

Both entry points share every kernel, so the results must agree bit for
bit: resolved ids, their loop bodies, every candidate's rho^2, S_n and X.
Two static runs in a row, the second on a smaller catalog and another grid
(the array keeps the first run's contents, and its grid tables must be
recomputed)."""
import ctypes as C

import numpy as np
import pytest

from paper_2602_18560_amd import gbsub as G
from paper_2602_18560_amd.inputs import Population, RunConfig, YEAR_S, draw_catalog

pytestmark = pytest.mark.gpu


def _results(ctx):
    ids, it = ctx.resolved()
    cids, cit, r2 = ctx.candidates()
    return dict(S=ctx.spectrum(G.SPEC_SN), X=ctx.spectrum(G.SPEC_X_RESIDUAL),
                Sgal=ctx.spectrum(G.SPEC_S_GAL), ids=ids, it=it, cids=cids, cit=cit, r2=r2)


def _same(a, b):
    for k in a:
        assert a[k].dtype == b[k].dtype, k
        assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), k


def _case(seed, n, f_lo, f_hi, W, t_obs):
    cat = draw_catalog(Population(n=n, seed=seed, f_lo=f_lo, f_hi=f_hi))
    cat.A *= np.float32(8.0)
    run = RunConfig(t_obs_s=t_obs, f_min_hz=f_lo, f_max_hz=f_hi, window_bins=W)
    return cat, run


def test_static_run_equals_workspace_run_twice():
    cases = [_case(11, 20000, 1e-3, 1.6e-3, 101, YEAR_S),          # ~1.9e4 bins, dozens of loop bodies
             _case(12, 3000, 2e-3, 2.3e-3, 51, 2 * YEAR_S)]         # smaller catalog, another grid
    static = []
    for cat, run in cases:
        print(f"[no-alloc] n={cat.n} W={run.window_bins} T={run.t_obs_s:.0f}", flush=True)
        ctx = G.Context(G.config_from_run(run))
        assert ctx.workspace_size(cat.n) <= G.STATIC_WORKSPACE_BYTES
        dc = G.DeviceCatalog.from_host(cat)
        s_st = ctx.run_static(dc)
        static.append((s_st, _results(ctx)))
        ctx.close()
    for (cat, run), (s_st, r_st) in zip(cases, static):
        ctx = G.Context(G.config_from_run(run))
        dc = G.DeviceCatalog.from_host(cat)
        s_ws = ctx.run(dc)
        r_ws = _results(ctx)
        assert s_ws == s_st
        assert s_ws.n_resolved > 0 and s_ws.n_iter > 2
        _same(r_ws, r_st)
        # the same context again through the array, after a workspace run
        s2 = ctx.run_static(dc)
        assert s2 == s_ws
        _same(r_ws, _results(ctx))
        ctx.close()


def test_static_run_results_last_until_the_next_static_run():
    """A context's results live in the shared array: a static run of another
    context replaces them; a workspace run keeps its own."""
    (cat_a, run_a), (cat_b, run_b) = _case(13, 4000, 1e-3, 1.2e-3, 101, YEAR_S), \
        _case(14, 2000, 3e-3, 3.2e-3, 31, YEAR_S)
    a = G.Context(G.config_from_run(run_a))
    b = G.Context(G.config_from_run(run_b))
    da, db = G.DeviceCatalog.from_host(cat_a), G.DeviceCatalog.from_host(cat_b)
    a.run_static(da)
    ra = _results(a)
    b.run_static(db)
    rb = _results(b)
    # b's run overwrote the array; a run of a into a workspace gives a's results back
    a.run(da)
    _same(ra, _results(a))
    assert rb["S"].shape != ra["S"].shape or not np.array_equal(rb["S"], ra["S"])
    a.close()
    b.close()


def test_static_run_rejects_what_does_not_fit():
    run = RunConfig(t_obs_s=4 * YEAR_S, f_min_hz=1e-4, f_max_hz=3e-2, window_bins=1001)
    ctx = G.Context(G.config_from_run(run))
    assert ctx.workspace_size(1) > G.STATIC_WORKSPACE_BYTES
    cat, _ = _case(15, 10, 1e-3, 1.1e-3, 101, YEAR_S)
    dc = G.DeviceCatalog.from_host(cat)
    st, _ = ctx.run_static_raw(dc)
    assert st == G.E_NOMEM
    # no results appeared, and the context stays usable
    n = C.c_uint64()
    assert ctx._L.gbsub_spectrum(ctx.h, G.SPEC_SN, None, 0, C.byref(n), 0) == G.E_STATE
    ctx.close()
