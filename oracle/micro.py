"""Brute-force numpy micro-oracle for tiny inputs (TEST INFRASTRUCTURE ONLY).

An independent second statement of the same subtraction as ``gbsub_oracle.c``
(appendix "Subtraction algorithm", Eqs. "running median", "SNR inner
product", appendices on the instrumental noise and the TDI response), written
without looking at speed: every window is sorted in full, every source's
track is summed bin by bin.  It is used to cross-check the C oracle on random
tiny catalogs; it shares no code with it.
"""
from __future__ import annotations

import math

import numpy as np

C_LIGHT = 299792458.0


def grid(T, fmin, fmax):
    k0 = math.floor(fmin * T + 0.5)
    k1 = math.floor(fmax * T + 0.5)
    return k0, k1 - k0 + 1


def sinstr(f, oms_pm=15.0, tm_fm=3.0, L=2.5e9):
    """S_AA / R_AA, element-wise (appendices on LISA noise and TDI response)."""
    f = np.asarray(f, np.float64)
    fstar = C_LIGHT / (2 * math.pi * L)
    u = f / fstar
    p_oms = (oms_pm * 1e-12) ** 2 * (1 + (2e-3 / f) ** 4) * (2 * math.pi * f / C_LIGHT) ** 2
    p_tm = ((tm_fm * 1e-15) ** 2 * (1 + (4e-4 / f) ** 2) * (1 + (f / 8e-3) ** 4)
            * (2 * math.pi * f) ** -4 * (2 * math.pi * f / C_LIGHT) ** 2)
    s_aa = 8 * np.sin(u) ** 2 * (4 * (1 + np.cos(u) + np.cos(u) ** 2) * p_tm
                                 + (2 + np.cos(u)) * p_oms)
    r_aa = 16 * np.sin(u) ** 2 * u ** 2 * (9 / 20) / (1 + 0.7 * u ** 2)
    return s_aa / r_aa


def tracks(A, f, fdot, T, k0, B, single=False):
    """Per source: (first bin, last bin, per-bin power) on the grid, unclipped."""
    A = np.asarray(A, np.float64)
    f = np.asarray(f, np.float64)
    fdot = np.asarray(fdot, np.float64)
    P = A * A * T / 2
    c = np.floor((f + fdot * T / 2) * T + 0.5).astype(np.int64) - k0
    n = np.ones_like(c) if single else 1 + np.floor(np.abs(fdot) * T * T).astype(np.int64)
    lo = c - (n - 1) // 2
    return lo, lo + n - 1, P / n


def binned_power(lo, hi, q, B, active):
    X = np.zeros(B)
    for i in np.flatnonzero(active):
        a, b = max(lo[i], 0), min(hi[i], B - 1)
        if a <= b:
            X[a:b + 1] += q[i]
    return X


def running_median(X, W):
    B = len(X)
    out = np.empty(B)
    if B < W:
        out[:] = np.sort(X)[(B + 1) // 2 - 1]
        return out
    h = (W - 1) // 2
    for k in range(B):
        a = min(max(k - h, 0), B - W)
        out[k] = np.sort(X[a:a + W])[h]
    return out


def snr2(lo, hi, q, S):
    B = len(S)
    a, b = max(lo, 0), min(hi, B - 1)
    if a > b:
        return 0.0
    return 4 * q * np.sum(1.0 / S[a:b + 1])


def run(A, f, fdot, T, fmin, fmax, W, rho_th=7.0, kappa=1 / 7.0, Cmed=729 / 512,
        single=False, noise_scale=1.0):
    """Returns (iter_of per source, n_iter, S_final, X_final, candidate mask)."""
    k0, B = grid(T, fmin, fmax)
    fk = (k0 + np.arange(B)) / T
    Sx = sinstr(fk) * noise_scale
    lo, hi, q = tracks(A, f, fdot, T, k0, B, single)
    n = len(q)
    rho0 = np.array([snr2(lo[i], hi[i], q[i], Sx) for i in range(n)])
    cand = rho0 >= (kappa * rho_th) ** 2
    iter_of = np.full(n, -1)
    t = 0
    while True:
        X = binned_power(lo, hi, q, B, iter_of < 0)
        S = Cmed * running_median(X, W) + Sx
        new = [i for i in np.flatnonzero(cand & (iter_of < 0))
               if snr2(lo[i], hi[i], q[i], S) > rho_th ** 2]
        if not new:
            return iter_of, t + 1, S, X, cand
        iter_of[new] = t
        t += 1
