"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bar: identical resolved set, iteration of resolution and iteration count
(except sources whose oracle SNR is within 1e-6 relative of the threshold,
counted and replayed), final spectrum within 1e-5 relative per bin.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_2602_18560_amd import gbsub as G
from paper_2602_18560_amd.inputs import Population, RunConfig, YEAR_S, draw_catalog, catalog_1e4
from tests.helpers import amp_for_power, bin_freq, catalog, small_run
from tests import oracle_bar as OB
from tests.edge_catalogs import CASES as EDGE_CASES
from tests.near_catalogs import cascade_near, sparse_near
from tests.test_oracle_pins import cascade_catalog

pytestmark = pytest.mark.gpu

S_RTOL = OB.S_RTOL
X_RTOL = OB.X_RTOL


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_run(cat, run, **kw):
    ctx = G.Context(G.config_from_run(run, **kw))
    try:
        dc = G.DeviceCatalog.from_host(cat)
        st, s = ctx.run_raw(dc)
        if st != G.OK:
            return st, s, None, None, None, None
        S = ctx.spectrum(G.SPEC_SN)
        X = ctx.spectrum(G.SPEC_X_RESIDUAL)
        ids, it = ctx.resolved()
        return st, s, S, X, ids, it
    finally:
        ctx.close()


def assert_parity(cat, run, name, **kw):
    say(f"[parity] {name}: n={cat.n} W={run.window_bins}")
    cfg = O.make_config(run, **kw)
    st, s, S, X, ids, it = gpu_run(cat, run, **kw)
    assert st == G.OK, G.status_str(st)
    ro = OB.check(cat, cfg, s, S, X, ids, it)
    return ro, s, S


# ----------------------------------------------------------------- closed-form catalogs

def test_lone_binary_and_sparse_loud():
    run, k0 = small_run(n_bins=3000, W=5)
    T = run.t_obs_s
    Sx = O.sinstr_table(O.make_config(run))
    bins = np.arange(7, 3000, 3)
    P = Sx[bins] * np.where(np.arange(len(bins)) % 2 == 0, 50.0, 5.0)
    cat = catalog([amp_for_power(p, T) for p in P], [bin_freq(k0, b, T) for b in bins])
    ro, s, S = assert_parity(cat, run, "sparse loud")
    assert s.n_iter == 2
    np.testing.assert_allclose(S, Sx, rtol=1e-13)


@pytest.mark.parametrize("which", ["sparse", "cascade"])
def test_near_threshold_guided_replay(which):
    """Sources within 1e-6 of the threshold (the guided branch): the sparse
    catalog has six near evaluations at t = 0 and 1, the cascade one medium
    source near at t = 1."""
    if which == "sparse":
        cat, run, _, _ = sparse_near()
        n_near = 6
    else:
        cat, run, _, _, _, _ = cascade_near()
        n_near = 1
    ro, s, _ = assert_parity(cat, run, f"near threshold {which}")
    assert s.n_near_threshold == n_near and ro.n_near == n_near
    assert s.min_rel_margin < 1e-6


def test_three_iteration_cascade():
    cat, run, kinds, bins = cascade_catalog(n_periods=900)   # 4500 bins: 3 tiles
    ro, s, S = assert_parity(cat, run, "cascade")
    assert s.n_iter == 3


def test_1e4_catalog_full():
    cat, run = catalog_1e4()
    assert_parity(cat, run, "catalog_1e4")


@pytest.mark.parametrize("n,flo,fhi,W,T,scale,seed", [
    (20000, 1e-3, 1.6e-3, 101, YEAR_S, 30, 1),        # ~400 iterations, 10 tiles
    (50000, 5e-4, 1.2e-3, 251, YEAR_S, 20, 2),
    (200000, 3e-4, 3e-3, 501, 2 * YEAR_S, 3, 4),       # 84 tiles, 13 iterations
    (5000, 2e-3, 2.1e-3, 1, YEAR_S, 20, 5),            # W = 1: the median is the bin itself
    (8000, 2e-3, 2.3e-3, 2817, YEAR_S, 20, 6),         # largest window: 256-bin tiles
])
def test_dense_catalogs(n, flo, fhi, W, T, scale, seed):
    cat = draw_catalog(Population(n=n, seed=seed, f_lo=flo, f_hi=fhi))
    cat.A *= np.float32(scale)
    run = RunConfig(t_obs_s=T, f_min_hz=flo, f_max_hz=fhi, window_bins=W)
    assert_parity(cat, run, f"dense n={n} W={W}")


@pytest.mark.parametrize("estimator", [G.MEDIAN, G.MEAN])
@pytest.mark.parametrize("case", sorted(EDGE_CASES))
def test_edge_clamped_windows(case, estimator):
    """Subtractions inside an edge window but more than h bins from the edge
    outputs (a ragged last tile of 100 <= h bins at W = 1001, W = 2817 with
    256-bin tiles at the lower edge, B < W over four tiles): the next body
    must refilter the edge outputs."""
    cat, run, kw = EDGE_CASES[case](estimator)
    assert_parity(cat, run, f"edge {case} estimator={estimator}", **kw)


def test_grid_shorter_than_window():
    run, k0 = small_run(n_bins=700, W=1001)
    T = run.t_obs_s
    rng = np.random.default_rng(9)
    f = (k0 + rng.uniform(0, 700, 3000)) / T
    Sx = O.sinstr(float(f.mean()))
    cat = catalog(np.sqrt(2 * Sx * rng.exponential(3.0, 3000) / T), f)
    assert_parity(cat, run, "B < W")


def test_wide_tracks_and_clipping():
    run, k0 = small_run(n_bins=9000, f_min=3e-3, W=201)
    T = run.t_obs_s
    rng = np.random.default_rng(10)
    n = 4000
    f = (k0 + rng.uniform(-3000, 12000, n)) / T
    fdot = rng.choice([0.0, 1.0], n) * rng.exponential(200.0, n) / T ** 2
    Sx = O.sinstr(3e-3)
    A = np.sqrt(2 * Sx * rng.exponential(60.0, n) / T)
    cat = catalog(A, f, fdot)
    assert_parity(cat, run, "wide tracks")


def test_single_bin_track_model():
    cat, run = catalog_1e4()
    assert_parity(cat, run, "catalog_1e4 single-bin", track_model=G.TRACK_SINGLE)


def test_kappa_zero_evaluates_everyone():
    cat = draw_catalog(Population(n=30000, seed=12, f_lo=1e-3, f_hi=1.3e-3))
    cat.A *= np.float32(20)
    run = RunConfig(t_obs_s=YEAR_S, f_min_hz=1e-3, f_max_hz=1.3e-3, window_bins=51)
    ro, s, _ = assert_parity(cat, run, "kappa=0", kappa=0.0)
    assert s.n_candidates == cat.n


# ----------------------------------------------------------------- running mean estimator

@pytest.mark.parametrize("which,W", [("catalog_1e4", 251), ("dense", 2001), ("dense", 101), ("short", 1001)])
def test_running_mean_estimator(which, W):
    if which == "catalog_1e4":
        cat, run = catalog_1e4()
        run = RunConfig(**{**run.as_dict(), "window_bins": W})
    elif which == "dense":
        cat = draw_catalog(Population(n=200000, seed=4, f_lo=3e-4, f_hi=3e-3))
        cat.A *= np.float32(3)
        run = RunConfig(t_obs_s=2 * YEAR_S, f_min_hz=3e-4, f_max_hz=3e-3, window_bins=W)
    else:                                   # B < W: the whole grid is the window
        run, k0 = small_run(n_bins=700, W=W)
        rng = np.random.default_rng(9)
        f = (k0 + rng.uniform(0, 700, 3000)) / run.t_obs_s
        Sx = O.sinstr(float(f.mean()))
        cat = catalog(np.sqrt(2 * Sx * rng.exponential(30.0, 3000) / run.t_obs_s), f)
    assert_parity(cat, run, f"mean {which} W={W}", estimator=G.MEAN)


def test_mean_rejects_fp32_modes():
    run, _ = small_run(n_bins=2000, W=21)
    with pytest.raises(G.GbsubError):
        G.Context(G.config_from_run(run, estimator=G.MEAN, precision=G.FP32_COMP))


# ----------------------------------------------------------------- edge cases and errors

def test_empty_catalog():
    run, _ = small_run(n_bins=5000, W=21)
    cat = catalog([], [])
    say("[edge] empty catalog")
    st, s, S, X, ids, it = gpu_run(cat, run)
    assert st == G.OK and s.n_iter == 1 and s.n_candidates == 0 and len(ids) == 0
    np.testing.assert_allclose(S, O.sinstr_table(O.make_config(run)), rtol=1e-13)
    assert np.all(X == 0)


def test_sources_outside_grid_and_zero_amplitude():
    run, k0 = small_run(n_bins=2000, W=21)
    T = run.t_obs_s
    cat = catalog([1e-21, 0.0, 1e-21], [bin_freq(k0, -50, T), bin_freq(k0, 10, T),
                                          bin_freq(k0, 5000, T)])
    assert_parity(cat, run, "outside grid")


def test_invalid_entries_and_configs():
    run, k0 = small_run(n_bins=2000, W=21)
    T = run.t_obs_s
    say("[edge] invalid")
    for A, f in [(float("nan"), bin_freq(k0, 5, T)), (-1e-22, bin_freq(k0, 5, T)), (1e-22, 0.0)]:
        st, *_ = gpu_run(catalog([1e-22, A], [bin_freq(k0, 9, T), f]), run)
        assert st == G.E_INVALID
    with pytest.raises(G.GbsubError):
        G.Context(G.config_from_run(run, window_bins=4))
    with pytest.raises(G.GbsubError):
        G.Context(G.config_from_run(run, window_bins=2819))
    # the context stays usable after an invalid catalog
    ctx = G.Context(G.config_from_run(run))
    st, _ = ctx.run_raw(G.DeviceCatalog.from_host(catalog([float("nan")], [bin_freq(k0, 3, T)])))
    assert st == G.E_INVALID
    s = ctx.run(G.DeviceCatalog.from_host(catalog([1e-22], [bin_freq(k0, 3, T)])))
    assert s.n_iter >= 1
    ctx.close()


def test_max_iter_guard():
    cat, run, _, _ = cascade_catalog(n_periods=40)
    say("[edge] max_iter")
    st, s, *_ = gpu_run(cat, run, max_iter=2)
    assert st == G.E_MAXITER
    st, s, *_ = gpu_run(cat, run, max_iter=3)
    assert st == G.OK and s.n_iter == 3


def test_results_before_run_and_truncation():
    run, k0 = small_run(n_bins=2000, W=21)
    ctx = G.Context(G.config_from_run(run))
    import ctypes as C
    n = C.c_uint64()
    assert ctx._L.gbsub_spectrum(ctx.h, 0, None, 0, C.byref(n), 0) == G.E_STATE
    ctx.run(G.DeviceCatalog.from_host(catalog_1e4()[0].subset(np.arange(10))))
    assert ctx._L.gbsub_spectrum(ctx.h, 0, None, 0, C.byref(n), 0) == G.E_TRUNCATED
    assert n.value == 2000
    ctx.close()


def test_run_is_deterministic():
    cat = draw_catalog(Population(n=100000, seed=21, f_lo=3e-4, f_hi=2e-3))
    cat.A *= np.float32(4)
    run = RunConfig(t_obs_s=YEAR_S, f_min_hz=3e-4, f_max_hz=2e-3, window_bins=251)
    say("[determinism]")
    a = gpu_run(cat, run)
    b = gpu_run(cat, run)
    np.testing.assert_array_equal(a[2], b[2])
    np.testing.assert_array_equal(a[3], b[3])
    np.testing.assert_array_equal(a[4], b[4])


# ----------------------------------------------------------------- full size

def test_1e7_full_size_against_oracle_golden():
    """The 1e7-binary workload in the configuration bench.py times, against
    the oracle: the resolved set, loop bodies and counts stored by
    tests/golden/make_golden.py, and S and X on every one of the 3,774,290
    bins, recomputed by the oracle from that resolved set (the final loop
    body's own X^t and S^t; its stored samples must agree bit for bit)."""
    import os
    from paper_2602_18560_amd.inputs import catalog_1e7
    gold = np.load(os.path.join(os.path.dirname(__file__), "golden", "catalog1e7_oracle.npz"))
    say("[parity] catalog_1e7 full size: drawing the catalog")
    cat, run = catalog_1e7()
    st, s, S, X, ids, it = gpu_run(cat, run)
    assert st == G.OK
    assert int(gold["n_near"]) == 0
    assert s.n_iter == int(gold["n_iter"])
    assert s.n_candidates == int(gold["n_candidates"])
    np.testing.assert_array_equal(ids, gold["resolved_ids"])
    np.testing.assert_array_equal(it, gold["resolved_iter"])
    assert s.n_near_threshold == 0
    assert abs(s.min_rel_margin - float(gold["min_rel_margin"])) <= 1e-9
    say("[parity] catalog_1e7: the oracle's final X and S on every bin")
    cfg = O.make_config(run)
    O.set_threads(0)
    Xo, So = O.spectra_after(cat, cfg, np.isin(cat.id, gold["resolved_ids"]))
    bins = gold["S_bins"]
    np.testing.assert_array_equal(So[bins], gold["S_final"])
    np.testing.assert_array_equal(Xo[bins], gold["X_final"])
    rel = np.abs(S - So) / So
    assert rel.max() <= S_RTOL, rel.max()
    zx = Xo == 0
    assert np.all(X[zx] == 0)
    np.testing.assert_allclose(X[~zx], Xo[~zx], rtol=X_RTOL)
    say(f"  max rel S error {rel.max():.2e} over {rel.size} bins")


def test_hot_tiles_beyond_one_accumulation_block():
    """A 1e6-source catalog on a 3,157-bin grid (two tiles of ~5e5 binning
    events, against 65,536 per accumulation block): the partial sums of hot
    tiles and their reduction, compared bin by bin.  0.2 % of the sources are
    made 100 times louder in amplitude so that the loop subtracts some."""
    cat = draw_catalog(Population(n=1_000_000, seed=41, f_lo=3e-4, f_hi=4e-4))
    rng = np.random.default_rng(41)
    loud = rng.random(cat.n) < 0.002
    cat.A *= np.float32(30)
    cat.A[loud] *= np.float32(100)
    run = RunConfig(t_obs_s=YEAR_S, f_min_hz=3e-4, f_max_hz=4e-4, window_bins=251)
    ro, s, _ = assert_parity(cat, run, "hot tiles")
    assert s.n_resolved > 0


@pytest.mark.parametrize("tile", [2048, 512])
def test_two_year_grid_ragged_last_tile(tile):
    """The 2-yr [0.1, 10] mHz grid of the job stream (W = 501, 624,841 bins:
    the last 2048-bin tile holds 201 <= h bins)."""
    T = 2 * YEAR_S
    cat = draw_catalog(Population(n=200_000, seed=42, f_lo=1e-4, f_hi=1e-2))
    cat.A *= np.float32(3)
    run = RunConfig(t_obs_s=T, f_min_hz=1e-4, f_max_hz=1e-2, window_bins=501)
    assert_parity(cat, run, f"2-yr grid tile {tile}", tile_bins=tile)


# ----------------------------------------------------------------- coarse-graining

@pytest.mark.parametrize("which", ["1e4", "dense"])
def test_coarse_graining_against_oracle(which):
    if which == "1e4":
        cat, run = catalog_1e4()
    else:
        cat = draw_catalog(Population(n=200000, seed=4, f_lo=1e-4, f_hi=1.2e-2))
        run = RunConfig(t_obs_s=YEAR_S, f_min_hz=1e-4, f_max_hz=1.2e-2, window_bins=251)
    say(f"[coarse] {which}")
    ro = O.run(cat, O.make_config(run))
    cfg = O.make_config(run)
    k0, B = O.grid(cfg.t_obs_s, cfg.f_min_hz, cfg.f_max_hz)
    Sx = O.sinstr_table(cfg)
    ctx = G.Context(G.config_from_run(run))
    try:
        ctx.run(G.DeviceCatalog.from_host(cat))
        for kind, ref_spec in ((G.SPEC_SN, ro.S_final), (G.SPEC_S_GAL, ro.S_final - Sx)):
            fo, so, cnt = O.coarse(ref_spec, k0, run.t_obs_s)
            f, s, hc, n = ctx.coarse(kind)
            np.testing.assert_array_equal(n, cnt)
            np.testing.assert_allclose(f, fo, rtol=1e-13)
            nz = cnt > 0
            if kind == G.SPEC_SN:
                np.testing.assert_allclose(s[nz], so[nz], rtol=S_RTOL)
                np.testing.assert_allclose(hc[nz], np.sqrt(fo[nz] * so[nz]), rtol=S_RTOL)
            else:   # the foreground alone: absolute error relative to the total PSD
                assert np.all(np.abs(s[nz] - so[nz]) <= S_RTOL * O.coarse(ro.S_final, k0, run.t_obs_s)[1][nz])
            assert np.all(s[~nz] == 0) and np.all(f[~nz] == 0)
    finally:
        ctx.close()


def test_tracks_longer_than_two_to_the_31_bins():
    """Sources whose track n = 1 + floor(|fdot| T^2) exceeds 2^31 bins, some
    beyond 2^52 (no power on the grid), next to ordinary ones (the
    population model's Gamma tail of log fdot)."""
    run, k0 = small_run(n_bins=4000, W=21)
    T = run.t_obs_s
    rng = np.random.default_rng(8)
    n = 3000
    bins = rng.integers(0, 4000, n)
    fd = np.where(rng.random(n) < 0.05, 2.0 ** rng.uniform(31, 60, n) / (T * T), rng.uniform(0, 20, n) / (T * T))
    Sx = O.sinstr_table(O.make_config(run))
    P = Sx[bins] * 10 ** rng.uniform(-1, 3, n)
    cat = catalog([amp_for_power(p, T) for p in P], [bin_freq(k0, b, T) for b in bins], list(fd))
    assert_parity(cat, run, "tracks beyond 2^31 bins")


# ----------------------------------------------------------------- device-side outputs

def test_resolved_list_and_s_gal_built_on_the_device():
    """The resolved list is compacted and radix-sorted by id on the device:
    opaque ids spread over all 32 bits (high bits set, unsorted), more than
    one sort block of resolved sources; ids ascending and their loop bodies
    equal the oracle's, also when written to device memory.  S_gal = S_n -
    S_instr is computed on the device, bit for bit the host difference."""
    import ctypes as C
    import torch
    cat = draw_catalog(Population(n=20000, seed=11, f_lo=1e-3, f_hi=1.6e-3))
    cat.A *= np.float32(8.0)
    rng = np.random.default_rng(77)
    cat.id = rng.choice(np.iinfo(np.uint32).max, size=cat.n, replace=False).astype(np.uint32)
    cat.id[:50] |= np.uint32(0x80000000)
    run = RunConfig(t_obs_s=YEAR_S, f_min_hz=1e-3, f_max_hz=1.6e-3, window_bins=101)
    ro, s, S = assert_parity(cat, run, "random 32-bit ids")
    assert s.n_resolved > 2 * 4096
    ctx = G.Context(G.config_from_run(run))
    try:
        ctx.run(G.DeviceCatalog.from_host(cat))
        ids, it = ctx.resolved()
        assert np.all(np.diff(ids.astype(np.int64)) > 0)
        m = ids.shape[0]
        dids = torch.empty(m, dtype=torch.int32, device="cuda")
        dit = torch.empty(m, dtype=torch.int32, device="cuda")
        n = C.c_uint64()
        st = ctx._L.gbsub_resolved(ctx.h, C.c_void_p(dids.data_ptr()), C.c_void_p(dit.data_ptr()), m,
                                   C.byref(n), 1)
        assert st == G.OK and n.value == m
        np.testing.assert_array_equal(dids.cpu().numpy().view(np.uint32), ids)
        np.testing.assert_array_equal(dit.cpu().numpy(), it)
        Sn = ctx.spectrum(G.SPEC_SN)
        Sx = ctx.spectrum(G.SPEC_S_INSTR)
        Sg = ctx.spectrum(G.SPEC_S_GAL)
        np.testing.assert_array_equal(Sg, Sn - Sx)
        dS = torch.empty(Sn.shape[0], dtype=torch.float64, device="cuda")
        ctx.spectrum(G.SPEC_S_GAL, out=dS)
        np.testing.assert_array_equal(dS.cpu().numpy(), Sg)
    finally:
        ctx.close()
