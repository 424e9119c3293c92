"""The continuous-batching server (paper_2602_18560_amd/serve.py): jobs of
different sizes and observation times arrive while others run, are admitted
as slots and memory free up, and each result equals the job run alone."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2602_18560_amd import gbsub as G
from paper_2602_18560_amd import serve as SV
from paper_2602_18560_amd.inputs import Population, RunConfig, YEAR_S, WINDOW_FOR_YEARS, draw_catalog
from tests import oracle_bar as OB

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def jobs():
    out = []
    for j, (n, years, seed, scale) in enumerate([(30000, 1, 1, 30), (80000, 2, 2, 10), (5000, 4, 3, 40),
                                                 (120000, 1, 4, 5), (20000, 2, 5, 20), (60000, 4, 6, 8)]):
        cat = draw_catalog(Population(n=n, seed=seed, f_lo=5e-4, f_hi=4e-3))
        cat.A *= np.float32(scale)
        run = RunConfig(t_obs_s=years * YEAR_S, f_min_hz=5e-4, f_max_hz=4e-3,
                        window_bins=WINDOW_FOR_YEARS[years])
        out.append((cat, run))
    return out


def alone(cat, run):
    ctx = G.Context(G.config_from_run(run))
    try:
        s = ctx.run(G.DeviceCatalog.from_host(cat))
        return s, ctx.spectrum(G.SPEC_SN), ctx.resolved()
    finally:
        ctx.close()


@pytest.mark.parametrize("slots,budget_mb", [(3, 100000), (6, 60)])
def test_server_results_equal_alone(slots, budget_mb):
    js = jobs()
    ref = [alone(c, r) for c, r in js]
    reqs = [SV.Request(j, 0.002 * j, *SV.pin_catalog(c), run=r) for j, (c, r) in enumerate(js)]
    say(f"[serve] {len(reqs)} jobs, {slots} slots, budget {budget_mb} MB")
    done, srv = SV.serve(reqs, max_slots=slots, budget_bytes=budget_mb * 1e6, chunk=2,
                         keep_contexts=True)
    assert sorted(c.index for c in done) == list(range(len(js)))
    for c in done:
        s_ref, S_ref, (ids_ref, it_ref) = ref[c.index]
        assert c.status == G.OK
        assert c.summary.n_iter == s_ref.n_iter
        np.testing.assert_array_equal(c.context.spectrum(G.SPEC_SN), S_ref)
        ids, it = c.context.resolved()
        np.testing.assert_array_equal(ids, ids_ref)
        np.testing.assert_array_equal(it, it_ref)
        assert c.done_s >= c.admit_s >= c.arrival_s - 1e-9
        # the served result against the oracle
        cat, run = js[c.index]
        OB.check(cat, O.make_config(run), c.summary, c.context.spectrum(G.SPEC_SN),
                 c.context.spectrum(G.SPEC_X_RESIDUAL), ids, it)
        c.context.close()
    srv.close()


def test_served_jobs_on_the_job_stream_grids_match_the_oracle():
    """Jobs on the [0.1, 10] mHz grids of the model job stream at 1, 2 and 4
    yr (W = 251 / 501 / 1001; the 2- and 4-yr grids end in tiles of 201 and
    402 bins, at most h), catalogs of 2e4 .. 2e5 sources drawn on the host,
    served two at a time: every result meets the oracle bar."""
    js = []
    for j, (n, years, seed, scale) in enumerate([(20000, 1, 51, 20), (200000, 2, 52, 3), (60000, 4, 53, 8),
                                                 (120000, 4, 54, 4), (40000, 2, 55, 12)]):
        cat = draw_catalog(Population(n=n, seed=seed, f_lo=1e-4, f_hi=1e-2))
        cat.A *= np.float32(scale)
        js.append((cat, RunConfig(t_obs_s=years * YEAR_S, f_min_hz=1e-4, f_max_hz=1e-2,
                                  window_bins=WINDOW_FOR_YEARS[years])))
    reqs = [SV.Request(j, 0.001 * j, *SV.pin_catalog(c), run=r) for j, (c, r) in enumerate(js)]
    say(f"[serve] {len(reqs)} jobs on the job-stream grids, 2 slots")
    done, srv = SV.serve(reqs, max_slots=2, budget_bytes=1e12, chunk=2, keep_contexts=True)
    assert sorted(c.index for c in done) == list(range(len(js)))
    for c in done:
        assert c.status == G.OK
        cat, run = js[c.index]
        ids, it = c.context.resolved()
        say(f"  job {c.index}: n={cat.n} bins={c.summary.n_bins} bodies={c.summary.n_iter}")
        OB.check(cat, O.make_config(run), c.summary, c.context.spectrum(G.SPEC_SN),
                 c.context.spectrum(G.SPEC_X_RESIDUAL), ids, it)
        c.context.close()
    srv.close()


def test_server_with_catalogs_drawn_on_the_gpu():
    """Jobs given as population-model hyperparameters and a seed: the server
    draws each catalog on the GPU at admission; every result equals the
    catalog drawn and run alone."""
    from paper_2602_18560_amd.inputs import model_job_stream
    jobs = model_job_stream(5, rate_hz=500.0, n_lo=2e4, n_hi=2e5)
    ref = []
    for j in jobs:
        dc = G.generate(G.population(**j.model), j.seed, j.n)
        ctx = G.Context(G.config_from_run(j.run))
        try:
            s = ctx.run(dc)
            ref.append((s, ctx.spectrum(G.SPEC_SN), ctx.resolved()))
        finally:
            ctx.close()
    say(f"[serve] {len(jobs)} model jobs, n = {[j.n for j in jobs]}")
    done, srv = SV.serve([SV.model_request(j) for j in jobs], max_slots=2, budget_bytes=1e12, chunk=2,
                         keep_contexts=True)
    assert sorted(c.index for c in done) == list(range(len(jobs)))
    for c in done:
        s_ref, S_ref, (ids_ref, it_ref) = ref[c.index]
        assert c.status == G.OK
        assert c.summary.n_iter == s_ref.n_iter
        np.testing.assert_array_equal(c.context.spectrum(G.SPEC_SN), S_ref)
        ids, it = c.context.resolved()
        np.testing.assert_array_equal(ids, ids_ref)
        np.testing.assert_array_equal(it, it_ref)
        c.context.close()
    srv.close()
