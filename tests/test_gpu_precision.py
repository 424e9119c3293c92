"""FP32 precision modes of the loop (gbsub_config.precision) against the FP64
oracle.  FP64 itself is the parity bar (test_gpu_parity.py); these modes are
measured, not pinned: compensated FP32 (double-fp32 sums) must stay within the error that fp32
rounding explains, with resolve decisions that differ from the oracle's
only within that error of the threshold; naive FP32 must run to completion
on the same candidates.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2602_18560_amd import gbsub as G
from paper_2602_18560_amd.inputs import Population, RunConfig, YEAR_S, draw_catalog, catalog_1e4

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_run(cat, run, **kw):
    ctx = G.Context(G.config_from_run(run, **kw))
    try:
        s = ctx.run(G.DeviceCatalog.from_host(cat))
        return s, ctx.spectrum(G.SPEC_SN), ctx.resolved(), ctx.candidates()
    finally:
        ctx.close()


def dense():
    cat = draw_catalog(Population(n=200000, seed=4, f_lo=3e-4, f_hi=3e-3))
    cat.A *= np.float32(3)
    return cat, RunConfig(t_obs_s=2 * YEAR_S, f_min_hz=3e-4, f_max_hz=3e-3, window_bins=501)


def flips(ids, ro, cat):
    ref = set(cat.id[ro.iter_of >= 0].tolist())
    got = set(ids.tolist())
    return len(ref ^ got)


# Bars of the compensated FP32 mode (double-fp32 sums, fp32 S and 1/S):
# S = C med + S_instr takes about four fp32 roundings (the scaled inputs,
# the product, the sum: < 5 * 2^-24 = 3e-7); the double-fp32 bin sums and
# prefixes add errors of order 2^-44 of the sums they carry.  rho^2 = 4 q
# sum 1/S takes the same S errors plus the roundings of q, of 1/S and of the
# final product.  1e-6 covers both with a margin.  A resolve decision can
# then differ from the oracle's only for a source whose oracle rho lies
# within 1e-6 of the threshold (rho^2 within 2e-6).
S_MAX = 1e-6
RHO2_MAX = 1e-6


def _near_band_sources(cat, run):
    """Sources whose oracle rho^2 is within 2e-6 relative of rho_th^2 at some
    evaluation (the only ones the FP32 bar lets flip)."""
    ref = O.run(cat, O.make_config(run), spectra=False, trace=True, trace_fields=("cand", "rho2"))
    th2 = run.snr_threshold ** 2
    near = set()
    for rec in ref.trace:
        ev = rec["rho2"] >= 0
        close = ev & (np.abs(rec["rho2"] / th2 - 1.0) <= 2e-6)
        near.update(cat.id[rec["cand"][close]].tolist())
    return ref, near


@pytest.mark.parametrize("which", ["catalog_1e4", "dense"])
def test_fp32_compensated_within_fp32_rounding(which):
    cat, run = catalog_1e4() if which == "catalog_1e4" else dense()
    say(f"[precision] compensated fp32, {which}")
    ro = O.run(cat, O.make_config(run))
    s, S, (ids, it), (cids, cit, cr2) = gpu_run(cat, run, precision=G.FP32_COMP)
    assert s.n_candidates == ro.n_candidates
    rel = np.abs(S - ro.S_final) / ro.S_final
    ref, near = _near_band_sources(cat, run)
    flipped = set(cat.id[ro.iter_of >= 0].tolist()) ^ set(ids.tolist())
    say(f"  S rel err max {rel.max():.2e} median {np.median(rel):.2e}; "
        f"flips {len(flipped)} of {int((ro.iter_of >= 0).sum())} ({len(near)} in the near band)")
    assert rel.max() < S_MAX
    assert flipped <= near
    # rho^2 of every candidate at its last evaluation (the same bodies when
    # no decision flipped)
    last = np.full(ref.trace[0]["cand"].shape[0], np.nan)
    for rec in ref.trace:
        ev = rec["rho2"] >= 0
        last[ev] = rec["rho2"][ev]
    order = np.argsort(ref.trace[0]["cand"])
    np.testing.assert_array_equal(cids, cat.id[ref.trace[0]["cand"][order]])
    r = np.abs(cr2 - last[order]) / last[order]
    say(f"  rho^2 rel err max {r.max():.2e} median {np.median(r):.2e}")
    if not flipped:
        assert r.max() < RHO2_MAX


def test_fp32_naive_runs_on_the_same_candidates():
    cat, run = dense()
    say("[precision] naive fp32")
    ro = O.run(cat, O.make_config(run))
    s, S, (ids, it), _ = gpu_run(cat, run, precision=G.FP32_NAIVE)
    assert s.n_candidates == ro.n_candidates
    assert np.all(np.isfinite(S)) and np.all(S > 0)
    rel = np.abs(S - ro.S_final) / ro.S_final
    say(f"  S rel err max {rel.max():.2e} median {np.median(rel):.2e}; "
        f"flips {flips(ids, ro, cat)} of {int((ro.iter_of >= 0).sum())}")


def test_fp64_mode_unaffected():
    """The precision field at its default leaves the bit-exact path alone."""
    cat, run = dense()
    a = gpu_run(cat, run)
    b = gpu_run(cat, run, precision=G.FP64)
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[2][0], b[2][0])


def test_compensated_fp32_on_the_1e7_catalog_every_bin():
    """The precision sweep at full size: the 1e7-binary workload in compensated
    FP32 against the oracle's stored resolved set and loop bodies, its rho^2
    of every candidate, and S on every one of the 3,774,290 bins (recomputed
    by the oracle from its resolved set).  Its smallest relative margin to
    the threshold is 1.35e-5, far outside the FP32 band: no decision may
    differ."""
    import os
    from paper_2602_18560_amd.inputs import catalog_1e7
    here = os.path.dirname(__file__)
    gold = np.load(os.path.join(here, "golden", "catalog1e7_oracle.npz"))
    grho = np.load(os.path.join(here, "golden", "catalog1e7_rho2.npz"))
    say("[precision] compensated fp32, 1e7 catalog")
    cat, run = catalog_1e7()
    assert float(gold["min_rel_margin"]) > 1e-5
    s, S, (ids, it), (cids, cit, cr2) = gpu_run(cat, run, precision=G.FP32_COMP)
    assert s.n_iter == int(gold["n_iter"])
    np.testing.assert_array_equal(ids, gold["resolved_ids"])
    np.testing.assert_array_equal(it, gold["resolved_iter"])
    np.testing.assert_array_equal(cids.astype(np.int64), grho["cand"].astype(np.int64))
    r = np.abs(cr2 - grho["rho2"]) / grho["rho2"]
    O.set_threads(0)
    _, So = O.spectra_after(cat, O.make_config(run), np.isin(cat.id, gold["resolved_ids"]))
    rel = np.abs(S - So) / So
    say(f"  S rel err max {rel.max():.2e} median {np.median(rel):.2e} over {rel.size} bins; "
        f"rho^2 rel err max {r.max():.2e} median {np.median(r):.2e}")
    assert rel.max() < S_MAX
    assert r.max() < RHO2_MAX
