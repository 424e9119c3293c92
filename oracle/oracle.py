"""Python access to the FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).

Loads ``oracle/_build/libgbsub_oracle.so`` (built from ``gbsub_oracle.c`` by
:func:`build` with gcc, FMA contraction off, OpenMP on) and wraps it with
ctypes.  Only the tests, the smoke check and the benchmark's CPU-baseline leg
use this module; the product library never does.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gbsub_oracle.c")
POP_SRC = os.path.join(HERE, "population_oracle.c")
CX_SRC = os.path.join(HERE, "template_oracle.c")
HDR = os.path.join(HERE, "gbsub_oracle.h")
BUILD_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(BUILD_DIR, "libgbsub_oracle.so")

OK, E_INVALID, E_MAXITER = 0, -1, -6
MEDIAN, MEAN = 0, 1
TRACK_SWEEP, TRACK_SINGLE = 0, 1


def build(force: bool = False) -> str:
    """Compile the oracle (gcc, -O2, no FMA contraction, OpenMP, libquadmath)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= max(
            os.path.getmtime(SRC), os.path.getmtime(POP_SRC), os.path.getmtime(CX_SRC),
            os.path.getmtime(HDR)):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-o", tmp, SRC, POP_SRC, CX_SRC, "-lquadmath", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


class Config(C.Structure):
    _fields_ = [("t_obs_s", C.c_double), ("f_min_hz", C.c_double), ("f_max_hz", C.c_double),
                ("window_bins", C.c_int64), ("snr_threshold", C.c_double), ("kappa", C.c_double),
                ("median_scale", C.c_double), ("estimator", C.c_int32), ("track_model", C.c_int32),
                ("max_iter", C.c_int64), ("oms_pm", C.c_double), ("tm_fm", C.c_double),
                ("arm_m", C.c_double), ("noise_scale", C.c_double)]


class Summary(C.Structure):
    _fields_ = [("n_iter", C.c_int64), ("n_bins", C.c_int64), ("k0", C.c_int64),
                ("n_candidates", C.c_int64), ("n_resolved", C.c_int64), ("n_near", C.c_int64),
                ("min_rel_margin", C.c_double)]


TRACE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_int64, C.c_int64, C.POINTER(C.c_double),
                       C.POINTER(C.c_double), C.c_int64, C.POINTER(C.c_int64),
                       C.POINTER(C.c_double))


class IO(C.Structure):
    _fields_ = [("iter_of", C.POINTER(C.c_int32)), ("is_candidate", C.POINTER(C.c_uint8)),
                ("rho0_sq", C.POINTER(C.c_double)), ("S_final", C.POINTER(C.c_double)),
                ("X_final", C.POINTER(C.c_double)), ("near_band", C.c_double),
                ("near_cap", C.c_int64), ("near_t", C.POINTER(C.c_int64)),
                ("near_i", C.POINTER(C.c_int64)), ("n_over", C.c_int64),
                ("over_t", C.POINTER(C.c_int64)), ("over_i", C.POINTER(C.c_int64)),
                ("over_dec", C.POINTER(C.c_uint8)), ("trace", TRACE_FN),
                ("trace_user", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("GBSUB_ORACLE_LIB") or build()
        L = C.CDLL(path)
        L.orc_default_config.argtypes = [C.POINTER(Config)]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = C.c_int
        L.orc_grid.argtypes = [C.c_double, C.c_double, C.c_double, C.POINTER(C.c_int64),
                               C.POINTER(C.c_int64)]
        L.orc_grid.restype = C.c_int
        for name in ("orc_s_aa", "orc_sinstr"):
            getattr(L, name).argtypes = [C.c_double] * 4
            getattr(L, name).restype = C.c_double
        L.orc_r_aa.argtypes = [C.c_double, C.c_double]
        L.orc_r_aa.restype = C.c_double
        L.orc_sinstr_table.argtypes = [C.POINTER(Config), C.c_int64, C.c_int64, C.c_void_p]
        L.orc_track.argtypes = [C.POINTER(Config), C.c_int64, C.c_int64, C.c_float, C.c_float,
                                C.c_float] + [C.POINTER(C.c_int64)] * 2 + [
                                    C.POINTER(C.c_double)] + [C.POINTER(C.c_int64)] * 2
        L.orc_track.restype = C.c_int
        L.orc_snr2.argtypes = [C.c_double, C.c_int64, C.c_int64, C.c_void_p]
        L.orc_snr2.restype = C.c_double
        L.orc_running_median.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p]
        L.orc_running_mean_psd.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64,
                                           C.c_void_p]
        L.orc_coarse.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_double, C.c_double,
                                 C.c_double, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_coarse.restype = C.c_int
        L.orc_run.argtypes = [C.POINTER(Config), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                              C.POINTER(IO), C.POINTER(Summary)]
        L.orc_run.restype = C.c_int
        L.orc_spectra_after.argtypes = [C.POINTER(Config), C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_spectra_after.restype = C.c_int
        _lib = L
    return _lib


def set_threads(n: int = 0) -> int:
    return lib().orc_set_threads(int(n))


def make_config(run=None, **kw) -> Config:
    """Oracle config from a ``RunConfig``-like object (or keywords)."""
    c = Config()
    lib().orc_default_config(C.byref(c))
    src = {}
    if run is not None:
        src.update(run.as_dict() if hasattr(run, "as_dict") else dict(run))
    src.update(kw)
    for k, v in src.items():
        if k in ("precision",):
            continue
        if k == "max_iter" and v is None:
            v = 0
        setattr(c, k, v)
    return c


def grid(t_obs_s: float, f_min_hz: float, f_max_hz: float):
    k0, B = C.c_int64(), C.c_int64()
    rc = lib().orc_grid(t_obs_s, f_min_hz, f_max_hz, C.byref(k0), C.byref(B))
    if rc != OK:
        raise ValueError("invalid grid")
    return k0.value, B.value


def sinstr(f: float, oms_pm=15.0, tm_fm=3.0, arm_m=2.5e9) -> float:
    return lib().orc_sinstr(float(f), oms_pm, tm_fm, arm_m)


def s_aa(f: float, oms_pm=15.0, tm_fm=3.0, arm_m=2.5e9) -> float:
    return lib().orc_s_aa(float(f), oms_pm, tm_fm, arm_m)


def r_aa(f: float, arm_m=2.5e9) -> float:
    return lib().orc_r_aa(float(f), arm_m)


def sinstr_table(cfg: Config) -> np.ndarray:
    k0, B = grid(cfg.t_obs_s, cfg.f_min_hz, cfg.f_max_hz)
    out = np.empty(B, np.float64)
    lib().orc_sinstr_table(C.byref(cfg), k0, B, out.ctypes.data)
    return out


def track(cfg: Config, A: float, f: float, fdot: float):
    k0, B = grid(cfg.t_obs_s, cfg.f_min_hz, cfg.f_max_hz)
    lo, n, glo, ghi = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
    q = C.c_double()
    rc = lib().orc_track(C.byref(cfg), k0, B, A, f, fdot, C.byref(lo), C.byref(n), C.byref(q),
                         C.byref(glo), C.byref(ghi))
    if rc != OK:
        raise ValueError("invalid source")
    return dict(lo=lo.value, n=n.value, q=q.value, glo=glo.value, ghi=ghi.value)


def snr2(q: float, glo: int, ghi: int, S: np.ndarray) -> float:
    S = np.ascontiguousarray(S, np.float64)
    return lib().orc_snr2(q, glo, ghi, S.ctypes.data)


def running_median(X: np.ndarray, W: int) -> np.ndarray:
    X = np.ascontiguousarray(X, np.float64)
    out = np.empty_like(X)
    lib().orc_running_median(X.ctypes.data, X.shape[0], int(W), out.ctypes.data)
    return out


def coarse(S: np.ndarray, k0: int, T: float, f_lo: float = 1e-4, f_hi: float = 1e-2,
           n_out: int = 100):
    """(f_k, S_k, N_k) of the logarithmic coarse-graining of S on the grid
    f_i = (k0+i)/T."""
    S = np.ascontiguousarray(S, np.float64)
    fo = np.zeros(n_out)
    so = np.zeros(n_out)
    cnt = np.zeros(n_out, np.int64)
    rc = lib().orc_coarse(S.ctypes.data, int(k0), S.shape[0], float(T), float(f_lo), float(f_hi),
                          int(n_out), fo.ctypes.data, so.ctypes.data, cnt.ctypes.data)
    if rc != OK:
        raise ValueError("invalid coarse-graining arguments")
    return fo, so, cnt


def running_mean_psd(X: np.ndarray, Sx: np.ndarray, W: int) -> np.ndarray:
    X = np.ascontiguousarray(X, np.float64)
    Sx = np.ascontiguousarray(Sx, np.float64)
    out = np.empty_like(X)
    lib().orc_running_mean_psd(X.ctypes.data, Sx.ctypes.data, X.shape[0], int(W),
                               out.ctypes.data)
    return out


def spectra_after(catalog, cfg: Config, subtracted) -> tuple[np.ndarray, np.ndarray]:
    """(X, S) of a loop body once exactly the sources flagged in
    ``subtracted`` (bool [n]) are subtracted; with the final resolved set
    these are the run's X_final and S_final."""
    A = np.ascontiguousarray(catalog.A, np.float32)
    f = np.ascontiguousarray(catalog.f, np.float32)
    fd = np.ascontiguousarray(catalog.fdot, np.float32)
    m = np.ascontiguousarray(np.asarray(subtracted, bool).astype(np.uint8))
    assert m.shape == A.shape
    k0, B = grid(cfg.t_obs_s, cfg.f_min_hz, cfg.f_max_hz)
    X = np.empty(B, np.float64)
    S = np.empty(B, np.float64)
    rc = lib().orc_spectra_after(C.byref(cfg), A.shape[0], A.ctypes.data, f.ctypes.data, fd.ctypes.data,
                                 m.ctypes.data, X.ctypes.data, S.ctypes.data)
    if rc != OK:
        raise ValueError("invalid catalog or configuration")
    return X, S


@dataclass
class Result:
    status: int
    n_iter: int
    n_bins: int
    k0: int
    n_candidates: int
    n_resolved: int
    n_near: int
    min_rel_margin: float
    iter_of: np.ndarray          # int32 [n], -1 = not resolved
    is_candidate: np.ndarray     # bool [n]
    rho0_sq: np.ndarray          # float64 [n]
    S_final: np.ndarray | None
    X_final: np.ndarray | None
    near: list                   # [(t, i)]
    trace: list                  # per iteration dicts when requested

    def resolved_ids(self, ids: np.ndarray) -> np.ndarray:
        sel = self.iter_of >= 0
        order = np.argsort(ids[sel], kind="stable")
        return ids[sel][order]


def run(catalog, cfg: Config, *, spectra: bool = True, trace: bool = False,
        near_cap: int = 4096, overrides=None, trace_fields=("X", "S", "cand", "rho2")) -> Result:
    """Run the whole subtraction on ``catalog`` (arrays A, f, fdot).  With
    ``trace``, every loop body appends a dict of ``trace_fields`` (X^t, S^t,
    the candidate indices and their rho^2 at t, -1 once resolved)."""
    A = np.ascontiguousarray(catalog.A, np.float32)
    f = np.ascontiguousarray(catalog.f, np.float32)
    fd = np.ascontiguousarray(catalog.fdot, np.float32)
    n = A.shape[0]
    k0, B = grid(cfg.t_obs_s, cfg.f_min_hz, cfg.f_max_hz)
    iter_of = np.empty(max(n, 1), np.int32)
    is_c = np.zeros(max(n, 1), np.uint8)
    rho0 = np.zeros(max(n, 1), np.float64)
    S = np.empty(B, np.float64) if spectra else None
    X = np.empty(B, np.float64) if spectra else None
    near_t = np.zeros(near_cap, np.int64)
    near_i = np.zeros(near_cap, np.int64)
    io = IO()
    io.iter_of = iter_of.ctypes.data_as(C.POINTER(C.c_int32))
    io.is_candidate = is_c.ctypes.data_as(C.POINTER(C.c_uint8))
    io.rho0_sq = rho0.ctypes.data_as(C.POINTER(C.c_double))
    if spectra:
        io.S_final = S.ctypes.data_as(C.POINTER(C.c_double))
        io.X_final = X.ctypes.data_as(C.POINTER(C.c_double))
    io.near_band = 1e-6
    io.near_cap = near_cap
    io.near_t = near_t.ctypes.data_as(C.POINTER(C.c_int64))
    io.near_i = near_i.ctypes.data_as(C.POINTER(C.c_int64))
    keep = []
    if overrides:
        ot = np.array([o[0] for o in overrides], np.int64)
        oi = np.array([o[1] for o in overrides], np.int64)
        od = np.array([1 if o[2] else 0 for o in overrides], np.uint8)
        keep += [ot, oi, od]
        io.n_over = len(overrides)
        io.over_t = ot.ctypes.data_as(C.POINTER(C.c_int64))
        io.over_i = oi.ctypes.data_as(C.POINTER(C.c_int64))
        io.over_dec = od.ctypes.data_as(C.POINTER(C.c_uint8))
    traces = []
    if trace:
        def _cb(user, t, nb, Xp, Sp, nc, cp, rp):
            rec = dict(t=int(t))
            if "X" in trace_fields:
                rec["X"] = np.ctypeslib.as_array(Xp, (nb,)).copy()
            if "S" in trace_fields:
                rec["S"] = np.ctypeslib.as_array(Sp, (nb,)).copy()
            if "cand" in trace_fields:
                rec["cand"] = np.ctypeslib.as_array(cp, (nc,)).copy() if nc else np.zeros(0, np.int64)
            if "rho2" in trace_fields:
                rec["rho2"] = np.ctypeslib.as_array(rp, (nc,)).copy() if nc else np.zeros(0)
            traces.append(rec)
        cb = TRACE_FN(_cb)
        keep.append(cb)
        io.trace = cb
    summ = Summary()
    rc = lib().orc_run(C.byref(cfg), n, A.ctypes.data, f.ctypes.data, fd.ctypes.data,
                       C.byref(io), C.byref(summ))
    nn = min(summ.n_near, near_cap)
    return Result(status=rc, n_iter=summ.n_iter, n_bins=summ.n_bins, k0=summ.k0,
                  n_candidates=summ.n_candidates, n_resolved=summ.n_resolved,
                  n_near=summ.n_near, min_rel_margin=summ.min_rel_margin,
                  iter_of=iter_of[:n].copy(), is_candidate=is_c[:n].astype(bool),
                  rho0_sq=rho0[:n].copy(), S_final=S, X_final=X,
                  near=[(int(near_t[j]), int(near_i[j])) for j in range(nn)], trace=traces)


# ---------------------------------------------------------------- population model

class Population(C.Structure):
    """Hyperparameters of the population model (Sec. "Population model",
    Table "priors"); f_lo_hz / f_hi_hz bound the power law."""
    _fields_ = [("alpha_pl", C.c_double), ("alpha_g", C.c_double), ("beta_g", C.c_double),
                ("mu_g", C.c_double), ("mu", C.c_double), ("sigma", C.c_double), ("rho", C.c_double),
                ("f_lo_hz", C.c_double), ("f_hi_hz", C.c_double)]


def population(alpha_pl=-2.9, alpha_g=1.96, beta_g=1.8, mu_g=-21.0, mu=-22.0, sigma=0.18, rho=0.99,
               f_lo_hz=1e-4, f_hi_hz=1e-2) -> Population:
    return Population(alpha_pl, alpha_g, beta_g, mu_g, mu, sigma, rho, f_lo_hz, f_hi_hz)


def _pop_lib():
    L = lib()
    if not getattr(L, "_pop_ready", False):
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32 * 4), C.POINTER(C.c_uint32 * 2),
                                        C.POINTER(C.c_uint32 * 4)]
        L.orc_gamma_p.argtypes = [C.c_double, C.c_double]
        L.orc_gamma_p.restype = C.c_double
        L.orc_gamma_quantile.argtypes = [C.c_double, C.c_double, C.c_double]
        L.orc_gamma_quantile.restype = C.c_double
        L.orc_pop_transform.argtypes = [C.POINTER(Population), C.c_double, C.c_double, C.c_double,
                                        C.POINTER(C.c_double), C.POINTER(C.c_double),
                                        C.POINTER(C.c_double)]
        L.orc_pop_draw.argtypes = [C.POINTER(Population), C.c_uint64, C.c_uint64, C.c_int64,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.orc_pop_draw.restype = C.c_int
        L._pop_ready = True
    return L


def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    _pop_lib().orc_philox4x32_10(C.byref(c), C.byref(k), C.byref(o))
    return tuple(o)


def gamma_p(a: float, x: float) -> float:
    return _pop_lib().orc_gamma_p(a, x)


def gamma_quantile(shape: float, rate: float, p: float) -> float:
    return _pop_lib().orc_gamma_quantile(shape, rate, p)


def pop_transform(pop: Population, u: float, v: float, w: float):
    f, fd, A = C.c_double(), C.c_double(), C.c_double()
    _pop_lib().orc_pop_transform(C.byref(pop), u, v, w, C.byref(f), C.byref(fd), C.byref(A))
    return f.value, fd.value, A.value


def pop_draw(pop: Population, seed: int, n: int, first: int = 0):
    """(A, f, fdot, id) of sources first .. first+n-1, fp32 / uint32."""
    A = np.empty(n, np.float32)
    f = np.empty(n, np.float32)
    fd = np.empty(n, np.float32)
    ids = np.empty(n, np.uint32)
    rc = _pop_lib().orc_pop_draw(C.byref(pop), seed, first, n, A.ctypes.data, f.ctypes.data,
                                 fd.ctypes.data, ids.ctypes.data)
    if rc != OK:
        raise ValueError(f"orc_pop_draw: {rc}")
    return A, f, fd, ids


# ---------------------------------------------------------------- complex-template data model

CX_NF = 128


class CxIO(C.Structure):
    _fields_ = [("iter_of", C.c_void_p), ("is_candidate", C.c_void_p), ("rho0_sq", C.c_void_p),
                ("rho2_last", C.c_void_p), ("q", C.c_void_p), ("S_final", C.c_void_p),
                ("X_final", C.c_void_p), ("h_final", C.c_void_p), ("near_band", C.c_double)]


def _cx_lib():
    L = lib()
    if not getattr(L, "_cx_ready", False):
        L.orc_cx_template.argtypes = [C.POINTER(Config), C.c_float, C.c_float, C.c_float,
                                      C.POINTER(C.c_int64), C.c_void_p]
        L.orc_cx_template.restype = C.c_int
        L.orc_cx_run.argtypes = [C.POINTER(Config), C.c_int64] + [C.c_void_p] * 5 + [
            C.POINTER(CxIO), C.POINTER(Summary)]
        L.orc_cx_run.restype = C.c_int
        L._cx_ready = True
    return L


NO_TEMPLATE = -(1 << 63)


def cx_template(cfg: Config, A: float, f: float, fdot: float):
    """(q, U): the central DFT index and the CX_NF complex template values
    U_j, j = -CX_NF/2 .. CX_NF/2-1 (q = NO_TEMPLATE and U = 0 if the source
    has no template)."""
    q = C.c_int64()
    U = np.zeros(2 * CX_NF, np.float64)
    rc = _cx_lib().orc_cx_template(C.byref(cfg), float(A), float(f), float(fdot), C.byref(q),
                                   U.ctypes.data)
    if rc != OK:
        raise ValueError("invalid source")
    return q.value, U[0::2] + 1j * U[1::2]


@dataclass
class CxResult:
    status: int
    n_iter: int
    n_bins: int
    k0: int
    n_candidates: int
    n_resolved: int
    n_near: int
    min_rel_margin: float
    iter_of: np.ndarray          # int32 [n]
    is_candidate: np.ndarray     # bool [n]
    rho0_sq: np.ndarray          # [n]
    rho2_last: np.ndarray        # [n] (nan for non-candidates)
    q: np.ndarray                # int64 [n]
    S_final: np.ndarray | None   # [2, B]
    X_final: np.ndarray | None   # [2, B]
    h_final: np.ndarray | None   # complex [2, B]


def cx_run(catalog, phi_a, phi_e, cfg: Config, *, spectra: bool = True) -> CxResult:
    """The subtraction on the complex-template data model (template_oracle.c)."""
    A = np.ascontiguousarray(catalog.A, np.float32)
    f = np.ascontiguousarray(catalog.f, np.float32)
    fd = np.ascontiguousarray(catalog.fdot, np.float32)
    pa = np.ascontiguousarray(phi_a, np.float32)
    pe = np.ascontiguousarray(phi_e, np.float32)
    n = A.shape[0]
    assert pa.shape == (n,) and pe.shape == (n,)
    k0, B = grid(cfg.t_obs_s, cfg.f_min_hz, cfg.f_max_hz)
    m = max(n, 1)
    iter_of = np.empty(m, np.int32)
    is_c = np.zeros(m, np.uint8)
    rho0 = np.zeros(m)
    rho2 = np.full(m, np.nan)
    q = np.zeros(m, np.int64)
    io = CxIO()
    io.iter_of, io.is_candidate, io.rho0_sq = iter_of.ctypes.data, is_c.ctypes.data, rho0.ctypes.data
    io.rho2_last, io.q = rho2.ctypes.data, q.ctypes.data
    S = X = h = None
    if spectra:
        S = np.empty((2, B))
        X = np.empty((2, B))
        h = np.empty((2, B, 2))
        io.S_final, io.X_final, io.h_final = S.ctypes.data, X.ctypes.data, h.ctypes.data
    io.near_band = 1e-6
    summ = Summary()
    rc = _cx_lib().orc_cx_run(C.byref(cfg), n, A.ctypes.data, f.ctypes.data, fd.ctypes.data,
                              pa.ctypes.data, pe.ctypes.data, C.byref(io), C.byref(summ))
    return CxResult(status=rc, n_iter=summ.n_iter, n_bins=summ.n_bins, k0=summ.k0,
                    n_candidates=summ.n_candidates, n_resolved=summ.n_resolved, n_near=summ.n_near,
                    min_rel_margin=summ.min_rel_margin, iter_of=iter_of[:n].copy(),
                    is_candidate=is_c[:n].astype(bool), rho0_sq=rho0[:n].copy(),
                    rho2_last=rho2[:n].copy(), q=q[:n].copy(), S_final=S, X_final=X,
                    h_final=None if h is None else h[..., 0] + 1j * h[..., 1])
