"""Pins of the oracle's near-threshold log and guided replay (CPU).

The resolve rule is strict, rho > rho_th (appendix "Subtraction algorithm",
the subtraction step), so a source whose SNR sits within rounding of rho_th
may be decided either way by two correct implementations.  The oracle logs
every evaluation (t, i) with |rho_i / rho_th - 1| <= 1e-6 and can replay a
run with given decisions at given (t, i).  Expected values below come from
the lone-binary closed form rho^2 = 2 A^2 T / S_x (every window of the sparse
catalog has median 0) and from the cascade's construction, never from the
oracle itself.
"""
import numpy as np
import pytest

from oracle import oracle as O
from tests.near_catalogs import amp_for_rho, cascade_near, rel_margin, sparse_near


def _run(cat, run, **kw):
    r = O.run(cat, O.make_config(run), **kw)
    assert r.status == O.OK
    return r


def test_sparse_near_catalog_is_what_it_claims():
    cat, run, bins, m = sparse_near()
    assert 4.3e-7 < m[2] < 5.7e-7 and 4.3e-7 < m[3] < 5.7e-7
    assert 7.3e-7 < m[4] < 8.7e-7 and 7.3e-7 < m[6] < 8.7e-7
    # outside the band on rho, and a band on rho^2 (twice as wide in
    # relative terms) would exclude the 8e-7 sources
    assert 1.4e-6 < m[5] < 1.6e-6
    assert (1 + m[4]) ** 2 - 1 > 1e-6


def test_near_log_holds_exactly_the_near_evaluations():
    cat, run, bins, m = sparse_near()
    r = _run(cat, run)
    # t = 0 resolves +5e-7, +8e-7, +1.5e-6 and the loud source; the two
    # sources below the threshold are evaluated again at t = 1, then nothing
    # resolves: n_iter = 2
    np.testing.assert_array_equal(r.iter_of, [-1, -1, 0, -1, 0, 0, -1, 0])
    assert r.n_iter == 2
    assert sorted(r.near) == [(0, 2), (0, 3), (0, 4), (0, 6), (1, 3), (1, 6)]
    assert r.n_near == 6
    assert abs(r.min_rel_margin - min(m[2:])) <= 1e-12


def test_replay_flips_only_the_overridden_decision():
    cat, run, bins, m = sparse_near()
    base = _run(cat, run)
    # (0, 2) not resolved: source 2 is evaluated again at t = 1 against the
    # same S and resolves there; nothing else changes; one more body
    r = _run(cat, run, overrides=[(0, 2, False)])
    exp = base.iter_of.copy()
    exp[2] = 1
    np.testing.assert_array_equal(r.iter_of, exp)
    assert r.n_iter == 3
    assert (1, 2) in r.near
    # both of its evaluations overridden: never resolved, and t = 1 then
    # resolves nothing, so the loop stops there
    r = _run(cat, run, overrides=[(0, 2, False), (1, 2, False)])
    exp[2] = -1
    np.testing.assert_array_equal(r.iter_of, exp)
    assert r.n_iter == 2 and (1, 2) in r.near and r.n_near == 7
    # (0, 3) resolved: it is no longer evaluated at t = 1
    r = _run(cat, run, overrides=[(0, 3, True)])
    exp = base.iter_of.copy()
    exp[3] = 0
    np.testing.assert_array_equal(r.iter_of, exp)
    assert r.n_iter == 2 and r.n_near == 5 and (1, 3) not in r.near


def test_override_is_keyed_on_the_source_index_and_iteration():
    cat, run, bins, m = sparse_near()
    base = _run(cat, run)
    # sources 0 and 1 are not candidates, so candidate slots differ from
    # source indices: an override of source 4 must not touch anyone else
    r = _run(cat, run, overrides=[(0, 4, False)])
    diff = np.flatnonzero(r.iter_of != base.iter_of)
    np.testing.assert_array_equal(diff, [4])
    # an override at an iteration where the source is not evaluated is inert
    r = _run(cat, run, overrides=[(5, 4, False), (1, 2, False)])
    np.testing.assert_array_equal(r.iter_of, base.iter_of)
    assert r.n_iter == base.n_iter


def test_cascade_near_source_logged_at_its_own_iteration():
    cat, run, kinds, bins, mid, lk = cascade_near()
    r = _run(cat, run)
    assert r.near == [(1, mid)]
    assert r.n_iter == 3 and r.iter_of[mid] == 1
    np.testing.assert_array_equal(r.iter_of[kinds == "L"], 0)
    np.testing.assert_array_equal(r.iter_of[kinds == "M"], 1)
    # flipped at t = 1 it resolves at t = 2 (S = S_x on its bin at both)
    f = _run(cat, run, overrides=[(1, mid, False)])
    exp = r.iter_of.copy()
    exp[mid] = 2
    np.testing.assert_array_equal(f.iter_of, exp)
    assert f.n_iter == 4 and f.near == [(1, mid), (2, mid)]


def test_cascade_follows_a_flipped_loud_source():
    """Keeping loud source lk (bin 5j) at t = 0 leaves three occupied bins in
    the windows of the medium sources at 5j - 1 and 5j + 1, whose median is
    then q_M: they cannot resolve at t = 1 (4 / C < 49); lk resolves at t = 1
    against C q_M + S_x, and those two at t = 2.  No other source moves."""
    cat, run, kinds, bins, mid, lk = cascade_near()
    base = _run(cat, run)
    r = _run(cat, run, overrides=[(0, lk, False)])
    exp = base.iter_of.copy()
    exp[lk] = 1
    blocked = np.flatnonzero(np.isin(bins, [bins[lk] - 1, bins[lk] + 1]))
    assert len(blocked) == 2 and np.all(kinds[blocked] == "M")
    exp[blocked] = 2
    np.testing.assert_array_equal(r.iter_of, exp)
    assert r.n_iter == 4


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_rho_band_not_rho_squared_band(sign):
    """A margin of 7e-7 on rho is 1.4e-6 on rho^2: logged, since the band is
    on rho."""
    cat, run, bins, _ = sparse_near()
    Sx = O.sinstr_table(O.make_config(run))
    T = run.t_obs_s
    b = int(bins[4])
    cat.A[4] = amp_for_rho(7.0 * (1.0 + sign * 7e-7), Sx[b], T)
    assert 6.3e-7 < rel_margin(cat.A[4], Sx[b], T) < 7.7e-7
    r = _run(cat, run)
    assert (0, 4) in r.near
