"""Small hand-built catalogs for the oracle pins and the GPU parity tests."""
import math

import numpy as np

from paper_2602_18560_amd.inputs import Catalog, RunConfig, YEAR_S

C_MED = 729.0 / 512.0


def small_run(n_bins=200, f_min=3e-3, t_obs=YEAR_S, W=5, **kw):
    """A grid of exactly ``n_bins`` bins starting at the bin nearest f_min."""
    k0 = math.floor(f_min * t_obs + 0.5)
    f_lo = k0 / t_obs
    f_hi = (k0 + n_bins - 1) / t_obs
    return RunConfig(t_obs_s=t_obs, f_min_hz=f_lo, f_max_hz=f_hi, window_bins=W, **kw), k0


def bin_freq(k0, k, t_obs):
    return (k0 + k) / t_obs


def amp_for_power(P, t_obs):
    """Amplitude whose one-bin power A^2 T / 2 equals P."""
    return math.sqrt(2.0 * P / t_obs)


def catalog(A, f, fdot=None):
    A = np.asarray(A, np.float32)
    f = np.asarray(f, np.float32)
    fd = np.zeros_like(f) if fdot is None else np.asarray(fdot, np.float32)
    return Catalog(A, f, fd, np.arange(len(A), dtype=np.uint32))
