"""GPU parity of the complex-template data model (gbsub_cx_*) against the
FP64 oracle (oracle/template_oracle.c).

Bar: identical candidate set, resolved set, loop body of each resolved
source and loop count, rho^2 of every candidate at its last evaluation
within 1e-9 relative (a source whose oracle SNR lies within 1e-6 relative
of the threshold may differ and is reported); S_A and S_E within 1e-9
relative per bin; X and h within 1e-9 of the largest value of their channel
(the GPU holds h as exact 64-bit fixed point with a unit of ~2^-62 of the
catalog's total template magnitude; the oracle sums in fp64); templates
within 1e-12 of their largest value (a 128-point FFT against the oracle's
term-by-term DFT).
"""
import math
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2602_18560_amd import gbsub as G
from paper_2602_18560_amd.inputs import (RunConfig, YEAR_S, Catalog, catalog_cx_1e4, catalog_cx_2e5,
                                          catalog_cx_1e7, template_phases)

pytestmark = pytest.mark.gpu

S_RTOL = 1e-9
X_ATOL = 1e-9
U_ATOL = 1e-12
RHO2_RTOL = 1e-9
NEAR = 1e-6


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def cat_of(A, f, fd):
    A = np.asarray(A, np.float32)
    return Catalog(A, np.asarray(f, np.float32), np.asarray(fd, np.float32),
                   np.arange(A.shape[0], dtype=np.uint32))


class Out:
    pass


def gpu_cx(cat, pa, pe, run, **kw):
    ctx = G.Context(G.config_from_run(run, **kw))
    try:
        cx = G.CxRun(ctx)
        dc = G.DeviceCxCatalog.from_host(cat, pa, pe)
        st, s = cx.run_raw(dc)
        o = Out()
        o.st, o.s = st, s
        if st == G.OK:
            o.S = np.stack([cx.spectrum(c, G.SPEC_SN) for c in (0, 1)])
            o.X = np.stack([cx.spectrum(c, G.SPEC_X_RESIDUAL) for c in (0, 1)])
            o.h = np.stack([cx.spectrum(c, G.SPEC_H_RESIDUAL) for c in (0, 1)])
            o.Sx = cx.spectrum(0, G.SPEC_S_INSTR)
            o.Sgal = np.stack([cx.spectrum(c, G.SPEC_S_GAL) for c in (0, 1)])
            o.ids, o.it = cx.resolved()
            o.cids, o.cit, o.cr2 = cx.candidates()
        return o
    finally:
        ctx.close()


def assert_cx_parity(cat, pa, pe, run, name, **kw):
    say(f"[cx parity] {name}: n={cat.n} W={run.window_bins}")
    g = gpu_cx(cat, pa, pe, run, **kw)
    assert g.st == G.OK, G.status_str(g.st)
    ro = O.cx_run(cat, pa, pe, O.make_config(run, **kw))
    assert ro.status == O.OK
    s = g.s
    assert s.n_bins == ro.n_bins
    assert s.n_candidates == ro.n_candidates
    sel = ro.iter_of >= 0
    order = np.argsort(cat.id[sel], kind="stable")
    ids_o, it_o = cat.id[sel][order], ro.iter_of[sel][order]
    if ro.n_near == 0:
        assert s.n_iter == ro.n_iter and s.n_resolved == ro.n_resolved
        assert np.array_equal(g.ids, ids_o)
        assert np.array_equal(g.it, it_o)
    else:
        # decisions inside the near band may go either way; everything else agrees
        say(f"[cx parity] {name}: {ro.n_near} near-threshold evaluations")
        near = np.abs(np.sqrt(np.maximum(ro.rho2_last, 0)) / 7.0 - 1.0) <= NEAR
        diff = set(map(int, g.ids)) ^ set(map(int, ids_o))
        assert all(near[int(np.nonzero(cat.id == v)[0][0])] for v in diff)
        return ro, g
    assert s.n_near_threshold == ro.n_near
    # every candidate: the same set, body and rho^2 at its last evaluation
    cand = np.nonzero(ro.is_candidate)[0]
    corder = np.argsort(cat.id[cand], kind="stable")
    assert np.array_equal(g.cids, cat.id[cand][corder])
    assert np.array_equal(g.cit, ro.iter_of[cand][corder])
    np.testing.assert_allclose(g.cr2, ro.rho2_last[cand][corder], rtol=RHO2_RTOL, atol=0)
    np.testing.assert_allclose(g.S, ro.S_final, rtol=S_RTOL, atol=0)
    for ch in (0, 1):
        scale = max(ro.X_final[ch].max(), 1e-300)
        assert np.abs(g.X[ch] - ro.X_final[ch]).max() <= X_ATOL * scale
        hs = max(np.abs(ro.h_final[ch]).max(), 1e-300)
        assert np.abs(g.h[ch] - ro.h_final[ch]).max() <= X_ATOL * hs
        np.testing.assert_array_equal(g.Sgal[ch], g.S[ch] - g.Sx)
    return ro, g


# ----------------------------------------------------------------- templates

def test_templates_against_the_oracle():
    """q bit-exact, U within 1e-12 of its largest value: off-bin and
    bin-centred tones, chirps up to |fdot| T^2 = 2^19, negative fdot,
    and sources without a template."""
    rng = np.random.default_rng(21)
    T = YEAR_S
    run = RunConfig(t_obs_s=T, f_min_hz=1e-4, f_max_hz=2e-2, window_bins=101)
    n = 3000
    f = rng.uniform(1e-4, 2e-2, n)
    fd = rng.choice([-1, 1], n) * 10 ** rng.uniform(-22, -13, n)
    fd[:200] = 0.0
    f[200:300] = np.round(f[200:300] * T) / T
    fd[300:320] = 2.0 ** rng.uniform(10, 19.9, 20) / T ** 2
    fd[320:330] = 2.0 ** 21 / T ** 2                     # no template
    A = 10 ** rng.uniform(-24, -20, n)
    cat = cat_of(A, f, fd)
    ctx = G.Context(G.config_from_run(run))
    try:
        import torch
        dc = G.DeviceCatalog.from_host(cat)
        q, U = G.CxRun(ctx).templates(dc.A, dc.f, dc.fdot)
    finally:
        ctx.close()
    cfg = O.make_config(run)
    worst = 0.0
    for i in range(n):
        qo, Uo = O.cx_template(cfg, cat.A[i], cat.f[i], cat.fdot[i])
        assert q[i] == qo, i
        if qo == O.NO_TEMPLATE:
            continue
        err = np.abs(U[i] - Uo).max() / np.abs(Uo).max()
        worst = max(worst, err)
    say(f"[cx templates] largest relative deviation {worst:.2e}")
    assert worst <= U_ATOL
    assert (q[320:330] == O.NO_TEMPLATE).all()


# ----------------------------------------------------------------- whole runs

def test_oracle_scale_catalog():
    cat, pa, pe, run = catalog_cx_1e4()
    ro, g = assert_cx_parity(cat, pa, pe, run, "1e4 catalog")
    assert ro.n_resolved > 100 and ro.n_iter >= 2


def test_mid_size_catalog_with_dense_tiles():
    """2e5 sources on the 1-yr grid: binning tiles of thousands of sources
    (several injection blocks each)."""
    cat, pa, pe, run = catalog_cx_2e5()
    ro, g = assert_cx_parity(cat, pa, pe, run, "2e5 catalog")
    assert ro.n_resolved > 1000


def _small_grid(n_bins, W, t_obs=YEAR_S, f_min=2e-3):
    k0 = math.floor(f_min * t_obs + 0.5)
    return RunConfig(t_obs_s=t_obs, f_min_hz=k0 / t_obs, f_max_hz=(k0 + n_bins - 1) / t_obs,
                     window_bins=W), k0


def test_templates_across_the_grid_edges():
    """Sources centred within a template's reach of either edge, and just
    outside the grid: only their in-grid bins count, in h and in rho^2."""
    run, k0 = _small_grid(1500, 31)
    T = run.t_obs_s
    rng = np.random.default_rng(22)
    off = np.r_[rng.uniform(-70, 70, 40), 1499 + rng.uniform(-70, 70, 40), rng.uniform(0, 1499, 200)]
    f = (k0 + off) / T
    A = 10 ** rng.uniform(-22.5, -21, off.shape[0])
    cat = cat_of(A, f, rng.uniform(-1, 1, off.shape[0]) * 3 / T ** 2)
    pa, pe = template_phases(cat.n, 22)
    assert_cx_parity(cat, pa, pe, run, "grid edges")


def test_grid_shorter_than_the_window():
    run, k0 = _small_grid(180, 251)
    T = run.t_obs_s
    rng = np.random.default_rng(23)
    cat = cat_of(10 ** rng.uniform(-22.5, -21, 60), (k0 + rng.uniform(0, 179, 60)) / T, np.zeros(60))
    pa, pe = template_phases(cat.n, 23)
    assert_cx_parity(cat, pa, pe, run, "B < W")


@pytest.mark.parametrize("W", [201, 2001])
def test_running_mean_estimator(W):
    cat, pa, pe, run = catalog_cx_1e4()
    run = RunConfig(**{**run.as_dict(), "window_bins": W, "estimator": 1})
    assert_cx_parity(cat, pa, pe, run, f"mean W={W}")


@pytest.mark.parametrize("tile,split", [(256, 0), (512, 1 << 20), (2048, 1)])
def test_tiles_and_split_modes(tile, split):
    """Other tiles and split budgets (every body split, or never): the
    dirty-tile stamps and the split decision of the tail serve both channels."""
    cat, pa, pe, run = catalog_cx_1e4()
    assert_cx_parity(cat, pa, pe, run, f"tile {tile} split {split}", tile_bins=tile, split_blocks=split)


def test_max_iter_guard():
    cat, pa, pe, run = catalog_cx_1e4()
    ctx = G.Context(G.config_from_run(run, max_iter=1))
    try:
        st, s = G.CxRun(ctx).run_raw(G.DeviceCxCatalog.from_host(cat, pa, pe))
    finally:
        ctx.close()
    assert st == G.E_MAXITER and s.n_iter == 1


def test_results_before_a_run_and_truncation():
    cat, pa, pe, run = catalog_cx_1e4()
    ctx = G.Context(G.config_from_run(run))
    try:
        L = ctx._L
        n = G.C.c_uint64()
        assert L.gbsub_cx_spectrum(ctx.h, 0, G.SPEC_SN, None, 0, G.C.byref(n), 0) == G.E_STATE
        assert L.gbsub_cx_resolved(ctx.h, None, None, 0, G.C.byref(n), 0) == G.E_STATE
        cx = G.CxRun(ctx)
        cx.run(G.DeviceCxCatalog.from_host(cat, pa, pe))
        buf = np.empty(10)
        assert L.gbsub_cx_spectrum(ctx.h, 0, G.SPEC_SN, buf.ctypes.data, 10, G.C.byref(n), 0) == G.E_TRUNCATED
        assert n.value == cat_bins(run)
        assert L.gbsub_cx_spectrum(ctx.h, 2, G.SPEC_SN, buf.ctypes.data, 10, G.C.byref(n), 0) == G.E_INVALID
        # the power-model results of this context are untouched by a template-model run
        assert L.gbsub_spectrum(ctx.h, G.SPEC_SN, None, 0, G.C.byref(n), 0) == G.E_STATE
    finally:
        ctx.close()


def cat_bins(run):
    return O.grid(run.t_obs_s, run.f_min_hz, run.f_max_hz)[1]


def test_everything_resolved_leaves_the_instrument_exactly():
    """Bright, well separated sources all resolve in body 0: the exact
    fixed-point subtraction leaves h = 0 bit for bit, so X = 0 and
    S = S_instr exactly in both channels."""
    run, k0 = _small_grid(6000, 51)
    T = run.t_obs_s
    rng = np.random.default_rng(24)
    off = 300 + 400 * np.arange(12) + rng.uniform(-0.5, 0.5, 12)
    cat = cat_of(np.full(12, 1e-19), (k0 + off) / T, rng.uniform(-1, 1, 12) * 5 / T ** 2)
    pa, pe = template_phases(cat.n, 24)
    ro, g = assert_cx_parity(cat, pa, pe, run, "all resolved")
    assert g.s.n_resolved == 12 and g.s.n_iter == 2
    assert not g.h.any() and not g.X.any()
    assert np.array_equal(g.S[0], g.Sx) and np.array_equal(g.S[1], g.Sx)


def test_empty_and_faint_catalogs():
    run, k0 = _small_grid(3000, 31)
    T = run.t_obs_s
    empty = cat_of([], [], [])
    g = gpu_cx(empty, np.zeros(0, np.float32), np.zeros(0, np.float32), run)
    assert g.st == G.OK and g.s.n_iter == 1 and g.s.n_candidates == 0
    assert np.array_equal(g.S[0], g.Sx) and not g.h.any()
    rng = np.random.default_rng(25)
    faint = cat_of(np.full(400, 1e-27), (k0 + rng.uniform(0, 2999, 400)) / T, np.zeros(400))
    pa, pe = template_phases(400, 25)
    assert_cx_parity(faint, pa, pe, run, "faint")


def test_invalid_entries_are_refused():
    run, k0 = _small_grid(3000, 31)
    T = run.t_obs_s
    cat = cat_of([1e-21, 1e-21], [(k0 + 100) / T, (k0 + 200) / T], [0, 0])
    pa = np.float32([0.1, np.nan])
    g = gpu_cx(cat, pa, np.float32([0.2, 0.3]), run)
    assert g.st == G.E_INVALID
    g = gpu_cx(cat_of([-1e-21], [(k0 + 100) / T], [0]), np.float32([0]), np.float32([0]), run)
    assert g.st == G.E_INVALID


def test_fp32_precision_modes_are_refused():
    cat, pa, pe, run = catalog_cx_1e4()
    ctx = G.Context(G.config_from_run(run, precision=G.FP32_COMP))
    try:
        with pytest.raises(G.GbsubError):
            G.CxRun(ctx).workspace_size(10)
    finally:
        ctx.close()


def test_run_is_deterministic():
    cat, pa, pe, run = catalog_cx_1e4()
    a = gpu_cx(cat, pa, pe, run)
    b = gpu_cx(cat, pa, pe, run)
    assert np.array_equal(a.S, b.S) and np.array_equal(a.h, b.h)
    assert np.array_equal(a.ids, b.ids) and np.array_equal(a.it, b.it)


# ----------------------------------------------------------------- full size

@pytest.fixture(scope="module")
def full_size():
    cat, pa, pe, run = catalog_cx_1e7()
    say(f"[cx full size] 1e7 catalog: n={cat.n}")
    return cat, pa, pe, run, gpu_cx(cat, pa, pe, run)


def test_full_size_subtraction_is_perfect(full_size):
    """After the loop, h equals bit for bit the injection of exactly the
    sources left (Eq. "vectorized-subtraction" with exact arithmetic): a
    second run on the same catalog with every resolved source moved off the
    grid (same size and amplitudes, so the same fixed-point unit) and a
    threshold nothing reaches injects only the others."""
    cat, pa, pe, run, g = full_size
    assert g.st == G.OK
    say(f"[cx full size] n_iter={g.s.n_iter} candidates={g.s.n_candidates} resolved={g.s.n_resolved}")
    assert g.s.n_resolved > 1000
    idx = np.searchsorted(cat.id, g.ids)
    assert np.array_equal(cat.id[idx], g.ids)
    f2 = cat.f.copy()
    f2[idx] = np.float32(0.9)                       # far above the grid: no template bin on it
    cat2 = Catalog(cat.A, f2, cat.fdot, cat.id)
    ctx = G.Context(G.config_from_run(run, snr_threshold=1e30))
    try:
        cx = G.CxRun(ctx)
        st, s = cx.run_raw(G.DeviceCxCatalog.from_host(cat2, pa, pe))
        assert st == G.OK and s.n_iter == 1 and s.n_resolved == 0
        h2 = np.stack([cx.spectrum(c, G.SPEC_H_RESIDUAL) for c in (0, 1)])
    finally:
        ctx.close()
    assert np.array_equal(h2, g.h)


def test_full_size_sampled_bins_against_oracle_templates(full_size):
    """X on 300 sampled bins against the oracle's templates of the sources
    left (summed on the host), and the fixed point: sampled candidates left
    unresolved have rho^2 against the final S_A, S_E at most rho_th^2."""
    cat, pa, pe, run, g = full_size
    cfg = O.make_config(run)
    T = run.t_obs_s
    k0, B = O.grid(run.t_obs_s, run.f_min_hz, run.f_max_hz)
    resolved = np.zeros(cat.n, bool)
    resolved[np.searchsorted(cat.id, g.ids)] = True
    fc = cat.f.astype(np.float64) + cat.fdot.astype(np.float64) * T / 2
    q = np.floor(fc * T + 0.5).astype(np.int64) - k0
    order = np.argsort(q, kind="stable")
    qs = q[order]
    rng = np.random.default_rng(26)
    # bins with at most 20,000 sources within a template's reach (the
    # densest ~0.3 % of the grid, near 0.1 mHz, would cost minutes here)
    cand_bins = rng.choice(B, 2000, replace=False)
    reach = np.searchsorted(qs, cand_bins + 65) - np.searchsorted(qs, cand_bins - 63)
    bins = cand_bins[reach <= 20000][:300]
    assert bins.shape[0] == 300
    tmpl = {}

    def template(i):
        if i not in tmpl:
            tmpl[i] = O.cx_template(cfg, cat.A[i], cat.f[i], cat.fdot[i])
        return tmpl[i]

    worst = 0.0
    for k in bins:
        # centres q with k - q in [-64, 63]: q in [k - 63, k + 64]
        lo, hi = np.searchsorted(qs, [k - 63, k + 65], side="left")
        h = np.zeros(2, complex)
        for i in order[max(lo - 8, 0):min(hi + 8, cat.n)]:
            if resolved[i]:
                continue
            qi, U = template(int(i))
            if qi == O.NO_TEMPLATE:
                continue
            j = k - (qi - k0)
            if -64 <= j < 64:
                h += np.exp(1j * np.array([pa[i], pe[i]], np.float64)) * U[j + 64]
        X = (2 / T) * np.abs(h) ** 2
        for ch in (0, 1):
            scale = max(g.X[ch].max(), 1e-300)
            worst = max(worst, abs(X[ch] - g.X[ch, k]) / scale)
    say(f"[cx full size] sampled X: largest deviation {worst:.2e} of the channel maximum")
    assert worst <= X_ATOL
    # the fixed point on sampled unresolved candidates
    left = np.nonzero(~resolved)[0]
    Sx = g.Sx
    checked = 0
    for i in rng.choice(left, 4000, replace=False):
        qi, U = template(int(i))
        if qi == O.NO_TEMPLATE:
            continue
        k = qi - k0 + np.arange(-64, 64)
        ok = (k >= 0) & (k < B)
        p = np.abs(U[ok]) ** 2
        r0 = (8 / T) * np.sum(p / Sx[k[ok]])
        if r0 < (cfg.kappa * cfg.snr_threshold) ** 2:
            continue
        r2 = (4 / T) * np.sum(p * (1 / g.S[0, k[ok]] + 1 / g.S[1, k[ok]]))
        assert r2 <= cfg.snr_threshold ** 2 * (1 + 2 * NEAR), (i, r2)
        checked += 1
    say(f"[cx full size] {checked} sampled unresolved candidates below the threshold")
    assert checked > 20
