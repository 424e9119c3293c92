"""The parity bar of a GPU result against the FP64 oracle, shared by the
plain, batched and served tests.

Resolved ids, their loop body and the loop count must be identical (after a
guided replay of any near-threshold evaluation: the oracle then takes the
GPU's decision for exactly the logged (t, i)), the near-threshold count and
the smallest relative margin must agree, S within 1e-5 relative per bin and
X within 1e-7 (the fixed-point unit's bound), zero where the oracle's is 0.
"""
import numpy as np

from oracle import oracle as O

S_RTOL = 1e-5
# X is accumulated exactly in fixed point with a unit of 2^(ilogb(P_max) - 61),
# P_max the largest one-bin power of the catalog; bins holding only powers
# ~1e-10 of P_max therefore carry ~1e-9..1e-8 relative quantisation error
# (irrelevant to S there, where S_instr dominates by orders of magnitude).
X_RTOL = 1e-7


def check(cat, cfg, s, S, X, ids, it, ro=None):
    """Asserts the bar for the GPU summary s, spectra S, X and resolved
    (ids, it) of catalog ``cat`` under oracle config ``cfg``; returns the
    (possibly replayed) oracle result."""
    if ro is None:
        ro = O.run(cat, cfg)
    assert ro.status == O.OK
    assert s.n_bins == ro.n_bins
    assert s.n_candidates == ro.n_candidates
    if ro.n_near:
        index_of = {int(v): i for i, v in enumerate(cat.id)}
        gpu_iter = np.full(cat.n, -1, np.int64)
        for v, t in zip(ids, it):
            gpu_iter[index_of[int(v)]] = t
        over = [(t, i, bool(gpu_iter[i] == t)) for (t, i) in ro.near]
        ro = O.run(cat, cfg, overrides=over)
        assert ro.status == O.OK
    sel = ro.iter_of >= 0
    ids_o = cat.id[sel]
    it_o = ro.iter_of[sel]
    order = np.argsort(ids_o, kind="stable")
    assert s.n_iter == ro.n_iter, (s.n_iter, ro.n_iter)
    np.testing.assert_array_equal(ids, ids_o[order])
    np.testing.assert_array_equal(it, it_o[order])
    assert s.n_resolved == int(sel.sum())
    # every unresolved candidate is judged at every body on both sides
    assert s.n_near_threshold == ro.n_near, (s.n_near_threshold, ro.n_near)
    if np.isfinite(ro.min_rel_margin):
        assert abs(s.min_rel_margin - ro.min_rel_margin) <= 1e-9 * max(1.0, ro.min_rel_margin), \
            (s.min_rel_margin, ro.min_rel_margin)
    else:
        assert not np.isfinite(s.min_rel_margin)
    rel = np.abs(S - ro.S_final) / ro.S_final
    assert rel.max() <= S_RTOL, rel.max()
    zx = ro.X_final == 0
    assert np.all(X[zx] == 0)
    np.testing.assert_allclose(X[~zx], ro.X_final[~zx], rtol=X_RTOL)
    return ro
