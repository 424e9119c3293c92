"""Seeded synthetic galactic-binary catalogs (input generation only).

This module draws the catalogs that both the FP64 oracle and the HIP path
consume.  It holds none of the subtraction method's arithmetic: no grid, no
noise model, no power, track, SNR or median.  It only turns a seed and a set of
population hyperparameters into structure-of-arrays ``A`` (fp32 strain
amplitude), ``f`` (fp32 Hz), ``fdot`` (fp32 Hz/s) and ``id`` (uint32).

Population recipe (a stand-in for the paper's catalogs, which are not
available; the paper's own population model is its Table of priors):

* ``f`` follows a power law p(f) ~ f^-gamma on [f_lo, f_hi], drawn by inverting
  the CDF of one uniform number per source;
* a Gaussian copula with correlation ``rho`` couples the amplitude variable and
  the frequency-derivative scatter (the copula construction of the paper's
  appendix on copulas, applied here to (A~, g)): (z1, z2) are standard normals
  with correlation rho, A~ = F_Gamma^-1(Phi(z1); k, theta), A = 1e-23 A~;
* fdot = 1e-16 (f / 1 mHz)^(11/3) g with g = exp(0.5 z2), i.e. the GW-driven
  f^(11/3) scaling of the paper's fdot relation times a log-normal scatter.

Random numbers come from numpy's PCG64 (``numpy.random.default_rng``), so a
seed gives the same catalog on every machine with the same numpy.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np
from scipy.special import gammaincinv, ndtr

YEAR_S = 31557600.0  # Julian year in seconds

# The paper's constants that the workloads use (threshold, kappa = 1/rho_th).
SNR_THRESHOLD = 7.0


@dataclass(frozen=True)
class Population:
    """Hyperparameters of one synthetic catalog."""
    n: int
    seed: int
    f_lo: float = 3e-4
    f_hi: float = 1e-2
    gamma: float = 3.0      # power-law index: p(f) ~ f^-gamma
    k: float = 1.5          # Gamma shape of A~
    theta: float = 2.0      # Gamma scale of A~
    rho: float = 0.5        # copula correlation of (A~, g)


@dataclass(frozen=True)
class RunConfig:
    """The run parameters of one subtraction job (mirrors ``gbsub_config``)."""
    t_obs_s: float
    f_min_hz: float
    f_max_hz: float
    window_bins: int
    snr_threshold: float = SNR_THRESHOLD
    kappa: float = 1.0 / SNR_THRESHOLD
    median_scale: float = 729.0 / 512.0
    estimator: int = 0          # 0 = running median
    track_model: int = 0        # 0 = linear-drift sweep, 1 = single bin
    precision: int = 0          # 0 = FP64 totals
    max_iter: int = 0

    def as_dict(self):
        return asdict(self)


@dataclass
class Catalog:
    A: np.ndarray
    f: np.ndarray
    fdot: np.ndarray
    id: np.ndarray
    population: Population | None = field(default=None)

    @property
    def n(self) -> int:
        return int(self.A.shape[0])

    def subset(self, idx) -> "Catalog":
        return Catalog(self.A[idx].copy(), self.f[idx].copy(),
                       self.fdot[idx].copy(), self.id[idx].copy(), None)


def _chunks(n: int, size: int):
    for s in range(0, n, size):
        yield s, min(n, s + size)


def draw_catalog(pop: Population, chunk: int = 1 << 21) -> Catalog:
    """Draw one catalog.  Deterministic in ``pop``; O(n) memory in fp32."""
    n = int(pop.n)
    rng = np.random.default_rng(pop.seed)
    u = rng.random(n)
    Z = rng.standard_normal((n, 2))
    A = np.empty(n, np.float32)
    f = np.empty(n, np.float32)
    fd = np.empty(n, np.float32)
    g1 = 1.0 - pop.gamma
    rho = float(pop.rho)
    sr = math.sqrt(max(0.0, 1.0 - rho * rho))
    for s, e in _chunks(n, chunk):
        uu = u[s:e]
        if abs(g1) < 1e-12:
            ff = pop.f_lo * np.exp(uu * math.log(pop.f_hi / pop.f_lo))
        else:
            lo = pop.f_lo ** g1
            hi = pop.f_hi ** g1
            ff = (lo + uu * (hi - lo)) ** (1.0 / g1)
        z1 = Z[s:e, 0]
        z2 = rho * z1 + sr * Z[s:e, 1]
        At = pop.theta * gammaincinv(pop.k, ndtr(z1))
        g = np.exp(0.5 * z2)
        f[s:e] = ff
        A[s:e] = 1e-23 * At
        fd[s:e] = 1e-16 * (ff / 1e-3) ** (11.0 / 3.0) * g
    ids = np.arange(n, dtype=np.uint32)
    return Catalog(A, f, fd, ids, pop)


# --------------------------------------------------------------------------
# The workloads.  Sizes and hyperparameters follow the stated configurations;
# seeds are fixed so every run draws the same catalogs.
# --------------------------------------------------------------------------

def catalog_1e4():
    """N=1e4, f in [0.3, 10] mHz, T = 1 yr, median window 251 bins, seed 0."""
    pop = Population(n=10_000, seed=0, f_lo=3e-4, f_hi=1e-2)
    run = RunConfig(t_obs_s=1 * YEAR_S, f_min_hz=3e-4, f_max_hz=1e-2, window_bins=251)
    return draw_catalog(pop), run


def catalog_1e7(n: int = 10_000_000):
    """N=1e7, f in [0.1, 30] mHz, T = 4 yr, median window 1001 bins, seed 2."""
    pop = Population(n=n, seed=2, f_lo=1e-4, f_hi=3e-2)
    run = RunConfig(t_obs_s=4 * YEAR_S, f_min_hz=1e-4, f_max_hz=3e-2, window_bins=1001)
    return draw_catalog(pop), run


def template_phases(n: int, seed: int):
    """Per-source phases (phi_A, phi_E) of the complex-template data model:
    independent and uniform on [0, 2 pi), fp32.  Stream seed + 7919 of numpy
    PCG64, so the phases do not reuse the catalog's own draws."""
    rng = np.random.default_rng(seed + 7919)
    ph = rng.uniform(0.0, 2.0 * math.pi, size=(2, n)).astype(np.float32)
    return ph[0].copy(), ph[1].copy()


def catalog_cx_1e4():
    """The 1e4 catalog (seed 0; T = 1 yr, [0.3, 10] mHz, W = 251) with its
    template phases: the oracle-scale case of the complex-template model."""
    cat, run = catalog_1e4()
    pa, pe = template_phases(cat.n, 0)
    return cat, pa, pe, run


def catalog_cx_2e5():
    """2e5 sources by the same recipe (seed 11) on the 1e4 catalog's grid
    (T = 1 yr, [0.3, 10] mHz, W = 251): the mid-size parity case of the
    complex-template model."""
    pop = Population(n=200_000, seed=11, f_lo=3e-4, f_hi=1e-2)
    run = RunConfig(t_obs_s=1 * YEAR_S, f_min_hz=3e-4, f_max_hz=1e-2, window_bins=251)
    cat = draw_catalog(pop)
    pa, pe = template_phases(cat.n, 11)
    return cat, pa, pe, run


def catalog_cx_1e7():
    """The 1e7 catalog (seed 2; T = 4 yr, [0.1, 30] mHz, W = 1001) with its
    template phases: the measured workload of the complex-template model."""
    cat, run = catalog_1e7()
    pa, pe = template_phases(cat.n, 2)
    return cat, pa, pe, run


def _meta_population(rng, n: int, seed: int, f_lo=1e-4, f_hi=3e-2) -> Population:
    return Population(n=n, seed=seed, f_lo=f_lo, f_hi=f_hi,
                      gamma=float(rng.uniform(2.0, 4.0)), k=float(rng.uniform(1.0, 3.0)),
                      theta=float(rng.uniform(1.0, 4.0)), rho=float(rng.uniform(0.0, 0.8)))


def batch_populations(n_catalogs: int = 64, n_lo: float = 1e5, n_hi: float = 2e7):
    """64 catalogs, N log-uniform in [1e5, 2e7], per-catalog hyperparameters
    uniform (gamma in [2,4], Gamma shape in [1,3], scale in [1,4], rho in
    [0,0.8]); T = 4 yr, W = 1001 on the [0.1, 30] mHz grid.  Meta seed 3,
    catalog j seed 3000+j."""
    rng = np.random.default_rng(3)
    pops = []
    for j in range(n_catalogs):
        n = int(round(10 ** rng.uniform(math.log10(n_lo), math.log10(n_hi))))
        pops.append(_meta_population(rng, n, 3000 + j))
    run = RunConfig(t_obs_s=4 * YEAR_S, f_min_hz=1e-4, f_max_hz=3e-2, window_bins=1001)
    return pops, run


WINDOW_FOR_YEARS = {1: 251, 2: 501, 4: 1001}


@dataclass(frozen=True)
class Job:
    index: int
    arrival_s: float
    population: Population
    run: RunConfig


def job_stream(n_jobs: int = 2000, rate_hz: float = 1.0, n_lo: float = 1e5, n_hi: float = 3e7):
    """Poisson stream of subtraction jobs: N log-uniform in [1e5, 3e7], T in
    {1, 2, 4} yr uniform, W = 251/501/1001 for 1/2/4 yr (about 7.9 uHz),
    hyperparameters as for the batched catalogs.  Meta seed 5, job j seed
    5000+j.  ``rate_hz`` is the Poisson arrival rate."""
    rng = np.random.default_rng(5)
    t = 0.0
    jobs = []
    for j in range(n_jobs):
        t += float(rng.exponential(1.0 / rate_hz))
        n = int(round(10 ** rng.uniform(math.log10(n_lo), math.log10(n_hi))))
        years = int(rng.choice([1, 2, 4]))
        pop = _meta_population(rng, n, 5000 + j)
        run = RunConfig(t_obs_s=years * YEAR_S, f_min_hz=1e-4, f_max_hz=3e-2,
                        window_bins=WINDOW_FOR_YEARS[years])
        jobs.append(Job(j, t, pop, run))
    return jobs


def _draw_one(pop: Population):
    c = draw_catalog(pop)
    return c.A, c.f, c.fdot, c.id


def draw_catalogs(pops, workers: int | None = None):
    """Draws several catalogs in a pool of processes (same results as
    ``draw_catalog`` one by one; order follows ``pops``).  Start it before
    the calling process touches a GPU."""
    import multiprocessing as mp
    import os
    pops = list(pops)
    workers = max(1, min(workers or min(16, os.cpu_count() or 1), len(pops)))
    if workers == 1:
        return [draw_catalog(p) for p in pops]
    order = sorted(range(len(pops)), key=lambda j: -pops[j].n)     # largest first
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_draw_one, [pops[j] for j in order], chunksize=1)
    out = [None] * len(pops)
    for j, (A, f, fd, ids) in zip(order, res):
        out[j] = Catalog(A, f, fd, ids, pops[j])
    return out


# Uniform prior box of the population model's hyperparameters (Table
# "priors"): alpha_PL, alpha_Gamma, beta_Gamma, mu_Gamma, mu, sigma, rho.
MODEL_PRIOR_BOX = {"alpha_pl": (-4.0, -2.0), "alpha_g": (1.0, 3.0), "beta_g": (1.0, 3.0),
                   "mu_g": (-22.0, -20.0), "mu": (-23.0, -21.0), "sigma": (0.1, 0.3), "rho": (0.0, 1.0)}


@dataclass(frozen=True)
class ModelJob:
    """A subtraction job whose catalog is drawn on the GPU from the
    population model: hyperparameters, generator seed and size."""
    index: int
    arrival_s: float
    model: dict
    seed: int
    n: int
    run: RunConfig


def model_job_stream(n_jobs: int = 64, rate_hz: float = 1.0, n_lo: float = 1e5, n_hi: float = 3e7):
    """Poisson stream of jobs drawn from the model: hyperparameters uniform
    in the prior box (rho below 0.999), N log-uniform in [n_lo, n_hi], T in
    {1, 2, 4} yr with W = 251/501/1001, f in [0.1, 10] mHz (the model's
    support).  Meta seed 7, job j generator seed 7000+j."""
    rng = np.random.default_rng(7)
    t = 0.0
    jobs = []
    for j in range(n_jobs):
        t += float(rng.exponential(1.0 / rate_hz))
        n = int(round(10 ** rng.uniform(math.log10(n_lo), math.log10(n_hi))))
        years = int(rng.choice([1, 2, 4]))
        lam = {k: float(rng.uniform(lo, hi)) for k, (lo, hi) in MODEL_PRIOR_BOX.items()}
        lam["rho"] = min(lam["rho"], 0.999)
        run = RunConfig(t_obs_s=years * YEAR_S, f_min_hz=1e-4, f_max_hz=1e-2,
                        window_bins=WINDOW_FOR_YEARS[years])
        jobs.append(ModelJob(j, t, lam, 7000 + j, n, run))
    return jobs

