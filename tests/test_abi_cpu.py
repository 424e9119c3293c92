"""Host-side checks of the C-ABI library (no GPU needed, no compute calls)."""
import ctypes as C
import os
import re

import pytest

from paper_2602_18560_amd import gbsub as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gbsub.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gbsub_[a-z_]+)\s*\(", text)))


def test_library_is_built():
    assert os.path.exists(G.LIB_PATH), "run python -m paper_2602_18560_amd.build"


def test_exports_every_declared_symbol():
    L = C.CDLL(G.LIB_PATH)
    declared = _declared_functions()
    assert set(G.EXPORTS) <= set(declared)
    for name in declared:
        assert hasattr(L, name), name


def test_struct_layouts_match_header():
    # sizes implied by the header's field order (no padding by construction)
    assert C.sizeof(G.Config) == 104
    assert C.sizeof(G.CatalogStruct) == 40
    assert C.sizeof(G.CxCatalogStruct) == 56
    assert C.sizeof(G.SummaryStruct) == 48
    assert C.sizeof(G.KernelStat) == 64


def test_default_config_is_the_papers():
    c = G.default_config()
    assert c.snr_threshold == 7.0 and c.kappa == 1.0 / 7.0
    assert c.median_scale == 729.0 / 512.0
    assert (c.oms_pm, c.tm_fm, c.arm_m) == (15.0, 3.0, 2.5e9)
    assert c.window_bins == 1001 and c.estimator == G.MEDIAN and c.precision == G.FP64
    assert G.status_str(G.E_MAXITER) == "iteration limit reached"


def test_binding_refuses_without_gpu(monkeypatch):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        G.Context(G.default_config())


def test_generate_validates_parameters_without_launching():
    """gbsub_generate checks its arguments before any device call; with
    n = 0 there is nothing to launch."""
    L = G.load()
    ok = G.population()
    assert C.sizeof(G.PopulationStruct) == 72
    assert L.gbsub_generate(C.byref(ok), 1, 0, 0, None, None, None, None, None) == G.OK
    for bad in (dict(rho=1.0), dict(rho=-1.0), dict(alpha_pl=-1.0), dict(alpha_g=0.0), dict(beta_g=-1.0),
                dict(sigma=-0.1), dict(f_lo_hz=0.0), dict(f_hi_hz=1e-5), dict(mu=float("nan"))):
        p = G.population(**bad)
        assert L.gbsub_generate(C.byref(p), 1, 0, 0, None, None, None, None, None) == G.E_INVALID, bad
    assert L.gbsub_generate(C.byref(ok), 1, 0, 10, None, None, None, None, None) == G.E_INVALID
