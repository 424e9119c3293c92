"""Catalogs with sources whose SNR lies near the threshold (the strict rule
rho > rho_th of the appendix "Subtraction algorithm"), for the oracle's
near-threshold log and guided replay and for the GPU's guided parity branch.

Amplitudes are fp32, so a source aimed at rho = rho_th (1 + delta) lands
within ~6e-8 of that delta; `rel_margin` gives the value it actually has,
from the lone-binary closed form rho^2 = 2 A^2 T / S_instr(f_c).
"""
import numpy as np

from oracle import oracle as O
from tests.helpers import C_MED, bin_freq, catalog, small_run
from tests.test_oracle_pins import cascade_catalog

RHO_TH = 7.0


def amp_for_rho(rho, sx, T):
    """fp32 amplitude of a one-bin source with rho^2 = 2 A^2 T / S_x = rho^2."""
    return np.float32(rho * np.sqrt(sx / (2.0 * T)))


def rel_margin(A, sx, T, S_over_sx=1.0):
    """|rho / rho_th - 1| of a one-bin source of fp32 amplitude A against
    S = S_over_sx * S_x (closed form, fp64)."""
    a = float(A)
    rho = np.sqrt(2.0 * a * a * T / (sx * S_over_sx))
    return abs(rho / RHO_TH - 1.0)


def sparse_near():
    """Sources 10 bins apart on a grid with W = 5: every window holds at most
    one occupied bin, so the median is 0 and S^t = S_x at every t.  Index
    (kind, delta): 0-1 quiet non-candidates (their indices differ from the
    candidate slots of the rest), then rho = rho_th (1 + delta) with delta =
    +5e-7, -5e-7, +8e-7 (inside the band on rho, outside a band on rho^2),
    +1.5e-6 (outside), -8e-7, and one loud source."""
    run, k0 = small_run(n_bins=200, W=5)
    T = run.t_obs_s
    Sx = O.sinstr_table(O.make_config(run))
    deltas = [None, None, 5e-7, -5e-7, 8e-7, 1.5e-6, -8e-7, 2.0]
    bins = [10 * (j + 1) for j in range(len(deltas))]
    A = []
    for b, dl in zip(bins, deltas):
        if dl is None:
            A.append(amp_for_rho(0.5, Sx[b], T))          # rho_0 = 0.5 < kappa rho_th = 1
        else:
            A.append(amp_for_rho(RHO_TH * (1.0 + dl), Sx[b], T))
    cat = catalog(A, [bin_freq(k0, b, T) for b in bins])
    margins = [rel_margin(a, Sx[b], T) for a, b in zip(cat.A, bins)]
    return cat, run, np.array(bins), margins


def cascade_near(n_periods=40, delta=5e-7):
    """The period-5 cascade [L, M, 0, L, M] (W = 5): loud sources resolve at
    t = 0, medium ones at t = 1 against S_x.  One medium source, `mid`, is
    re-aimed at rho = rho_th (1 + delta) against S_x, so its t = 1 evaluation
    is near the threshold (at t = 0 it sees S = C q_M + S_x and is far below).
    Returns the catalog, the run, kinds, bins, mid's index and a loud source
    `lk` two bins from medium sources on both sides."""
    cat, run, kinds, bins = cascade_catalog(n_periods)
    T = run.t_obs_s
    Sx = O.sinstr_table(O.make_config(run))
    mids = np.flatnonzero(kinds == "M")
    mid = int(mids[len(mids) // 2])
    cat.A[mid] = amp_for_rho(RHO_TH * (1.0 + delta), Sx[bins[mid]], T)
    louds = np.flatnonzero((kinds == "L") & (bins % 5 == 0))
    lk = int(louds[len(louds) // 4])
    return cat, run, kinds, bins, mid, lk


__all__ = ["sparse_near", "cascade_near", "rel_margin", "amp_for_rho", "C_MED"]
