"""Batched and continuously batched runs (gbsub_batch_*) against plain runs.

Every kernel of the loop covers all slots of a batch at once; each result
must be bitwise identical to gbsub_run on the same catalog (the binned
spectrum is exact integer arithmetic and every other reduction has a fixed
order), whatever the mix of catalogs it ran with.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2602_18560_amd import gbsub as G
from paper_2602_18560_amd.inputs import Population, RunConfig, YEAR_S, draw_catalog
from tests import oracle_bar as OB
from tests.helpers import bin_freq, catalog, small_run
from tests.test_oracle_pins import cascade_catalog

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def mixed_jobs():
    """Catalogs on different grids, windows and sizes, several of them dense."""
    jobs = []
    specs = [(20000, 1e-3, 1.6e-3, 101, 1, 30, 1), (50000, 5e-4, 1.2e-3, 251, 1, 20, 2),
             (200000, 3e-4, 3e-3, 501, 2, 3, 4), (3000, 2e-3, 2.1e-3, 1, 1, 20, 5),
             (30000, 1e-3, 1.3e-3, 51, 1, 20, 12), (100000, 3e-4, 2e-3, 251, 1, 4, 21),
             (8000, 2e-3, 2.3e-3, 2001, 1, 20, 6)]
    for n, flo, fhi, W, yrs, scale, seed in specs:
        cat = draw_catalog(Population(n=n, seed=seed, f_lo=flo, f_hi=fhi))
        cat.A *= np.float32(scale)
        jobs.append((cat, RunConfig(t_obs_s=yrs * YEAR_S, f_min_hz=flo, f_max_hz=fhi,
                                    window_bins=W)))
    return jobs


def plain(cat, run):
    ctx = G.Context(G.config_from_run(run))
    try:
        s = ctx.run(G.DeviceCatalog.from_host(cat))
        return s, ctx.spectrum(G.SPEC_SN), ctx.spectrum(G.SPEC_X_RESIDUAL), ctx.resolved()
    finally:
        ctx.close()


def drain(batch, chunk=4, limit=100000, stream=None):
    """Steps until no slot is running; returns the final state array."""
    for _ in range(limit):
        state, running = batch.poll(stream)
        if running == 0:
            return state
        batch.step(chunk, stream)
    raise AssertionError("batch did not settle")


def side_stream(kind):
    """None: the null stream (direct launches); "graph": a stream of its own,
    on which gbsub_batch_step captures the loop bodies once and replays them."""
    if kind is None:
        return None
    import torch
    torch.cuda.synchronize()
    return torch.cuda.Stream()


def results_of(ctx):
    return ctx.spectrum(G.SPEC_SN), ctx.spectrum(G.SPEC_X_RESIDUAL), ctx.resolved()


def assert_same(a, b):
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[2][0], b[2][0])
    np.testing.assert_array_equal(a[2][1], b[2][1])


@pytest.mark.parametrize("kind", [None, "graph"])
def test_batched_equals_plain_mixed_grids(kind):
    jobs = mixed_jobs()
    say(f"[batch {kind}] {len(jobs)} catalogs, plain runs")
    ref = [plain(cat, run) for cat, run in jobs]
    batch = G.Batch(max_slots=len(jobs))
    ctxs, cats = [], []
    for cat, run in jobs:
        ctx = G.Context(G.config_from_run(run))
        dc = G.DeviceCatalog.from_host(cat)
        ctx.ensure_workspace(dc.n)
        ctxs.append(ctx)
        cats.append(dc)
    st_ = side_stream(kind)
    for ctx, dc in zip(ctxs, cats):
        batch.admit(ctx, dc, stream=st_)
    say(f"[batch {kind}] stepping")
    state = drain(batch, stream=st_)
    assert np.all(state[:len(jobs)] == G.SLOT_SETTLED)
    for k, (ctx, (s_ref, S_ref, X_ref, r_ref)) in enumerate(zip(ctxs, ref)):
        st, s = batch.retire(k, st_)
        assert st == G.OK
        assert (s.n_iter, s.n_candidates, s.n_resolved) == (s_ref.n_iter, s_ref.n_candidates,
                                                           s_ref.n_resolved)
        assert_same(results_of(ctx), (S_ref, X_ref, r_ref))
        # and the batched result against the oracle
        cat, run = jobs[k]
        S, X, (ids, it) = results_of(ctx)
        OB.check(cat, O.make_config(run), s, S, X, ids, it)
    for c in ctxs:
        c.close()
    batch.close()


@pytest.mark.parametrize("kind", [None, "graph"])
def test_batched_equals_plain_mixed_precision(kind):
    """FP64, compensated FP32 and naive FP32 slots in one batch: the naive
    slot brings the loop-body tail back as a kernel of its own for every
    slot, which must not change the other slots' results.  The naive slot
    itself sums with fp32 atomics in arbitrary order, so no two of its runs
    need agree bit for bit: it must settle on the same candidate set."""
    jobs = mixed_jobs()
    picks = [(0, G.FP64), (1, G.FP32_COMP), (4, G.FP32_NAIVE), (5, G.FP32_COMP)]
    say(f"[batch precision {kind}] plain runs")
    ref = []
    for j, prec in picks:
        cat, run = jobs[j]
        ctx = G.Context(G.config_from_run(run, precision=prec))
        try:
            s = ctx.run(G.DeviceCatalog.from_host(cat))
            ref.append((s, ) + results_of(ctx))
        finally:
            ctx.close()
    batch = G.Batch(max_slots=len(picks))
    ctxs = []
    st_ = side_stream(kind)
    for j, prec in picks:
        cat, run = jobs[j]
        ctx = G.Context(G.config_from_run(run, precision=prec))
        dc = G.DeviceCatalog.from_host(cat)
        ctx.ensure_workspace(dc.n)
        batch.admit(ctx, dc, stream=st_)
        ctxs.append((ctx, dc))
    say(f"[batch precision {kind}] stepping")
    state = drain(batch, stream=st_)
    assert np.all(state[:len(picks)] == G.SLOT_SETTLED)
    for k, ((ctx, _), (s_ref, S_ref, X_ref, r_ref)) in enumerate(zip(ctxs, ref)):
        st, s = batch.retire(k, st_)
        assert st == G.OK
        assert s.n_candidates == s_ref.n_candidates
        if picks[k][1] == G.FP32_NAIVE:
            continue
        assert (s.n_iter, s.n_resolved) == (s_ref.n_iter, s_ref.n_resolved)
        assert_same(results_of(ctx), (S_ref, X_ref, r_ref))
    for ctx, _ in ctxs:
        ctx.close()
    batch.close()


def test_continuous_batching_alone_equals_mixed():
    jobs = mixed_jobs()
    ref = [plain(cat, run) for cat, run in jobs]
    batch = G.Batch(max_slots=3)
    pending = list(range(len(jobs)))
    live = {}                    # slot -> (job index, ctx, device catalog)
    done = {}
    say("[continuous] 7 jobs through 3 slots")
    while pending or live:
        while pending and len(live) < 3:
            j = pending.pop(0)
            cat, run = jobs[j]
            ctx = G.Context(G.config_from_run(run))
            dc = G.DeviceCatalog.from_host(cat)
            live[batch.admit(ctx, dc)] = (j, ctx, dc)
        batch.step(2)
        state, _ = batch.poll()
        for k in [k for k in live if state[k] != G.SLOT_RUNNING]:
            j, ctx, dc = live.pop(k)
            st, s = batch.retire(k)
            assert st == G.OK
            done[j] = (s, results_of(ctx))
            ctx.close()
    for j, (s, res) in done.items():
        assert s.n_iter == ref[j][0].n_iter
        assert_same(res, ref[j][1:])
    batch.close()


def test_invalid_and_maxiter_slots_do_not_disturb_others():
    run, k0 = small_run(n_bins=2000, W=21)
    T = run.t_obs_s
    bad = catalog([1e-22, float("nan")], [bin_freq(k0, 9, T), bin_freq(k0, 10, T)])
    casc, crun, _, _ = cascade_catalog(n_periods=40)
    good_cat, good_run = mixed_jobs()[0]
    ref = plain(good_cat, good_run)
    batch = G.Batch(max_slots=4)
    c_bad = G.Context(G.config_from_run(run))
    c_max = G.Context(G.config_from_run(crun, max_iter=2))
    c_ok = G.Context(G.config_from_run(good_run))
    d1, d2, d3 = (G.DeviceCatalog.from_host(x) for x in (bad, casc, good_cat))
    k1, k2, k3 = batch.admit(c_bad, d1), batch.admit(c_max, d2), batch.admit(c_ok, d3)
    state = drain(batch)
    assert state[k1] == G.SLOT_INVALID and state[k2] == G.SLOT_MAXITER
    assert state[k3] == G.SLOT_SETTLED
    assert batch.retire(k1)[0] == G.E_INVALID
    assert batch.retire(k2)[0] == G.E_MAXITER
    assert batch.retire(k3)[0] == G.OK
    assert_same(results_of(c_ok), ref[1:])
    for c in (c_bad, c_max, c_ok):
        c.close()
    batch.close()
