"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function include/subsmc.h declares, and its argument validation and
workspace sizing behave as documented."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1805_03317_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "subsmc.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:smc_status|size_t|void|int32_t|const char\*)\s+(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        from paper_1805_03317_amd import build
        build.build()
    return B.lib()


def test_header_declares_the_method_entry_points():
    names = declared_functions()
    for must in ("smc_init", "smc_temper", "smc_resample", "smc_move", "loglik_est", "loglik_grad", "smc_mass"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(B.EXPORTS) == names


def test_status_strings(lib):
    assert lib.smc_status_string(0) == b"ok"
    assert lib.smc_status_string(4) == b"matrix not positive definite"


def _problem(d=5, n=1000, M=64, m=100, G=4, ld=8, family=0, precision=0):
    pb = B._Problem()
    pb.family, pb.precision, pb.cv_order, pb.d = family, precision, 2, d
    pb.n, pb.ld, pb.xy_fp32, pb.Xy = n, ld, 0, 0x1000
    pb.gauss_s2, pb.M, pb.m, pb.G = 1.0, M, m, G
    pb.seed, pb.ess_frac = 1, 0.5
    pb.prior_mean = pb.prior_prec = 0x2000
    for f in ("theta", "u", "logw", "lhat", "sig2", "accept", "workspace"):
        setattr(pb, f, 0x3000)
    return pb


def test_workspace_size_and_validation(lib):
    pb = _problem()
    size = lib.smc_workspace_size(C.byref(pb))
    # packed rows (16 doubles of pitch for d = 5) dominate
    assert size >= 1000 * 16 * 8 + 64 * 100 * 4
    pb_mixed = _problem(precision=1)
    assert lib.smc_workspace_size(C.byref(pb_mixed)) < size
    for bad in (dict(d=0), dict(G=200), dict(M=0), dict(M=10_000), dict(ld=5), dict(n=0), dict(family=7)):
        p = _problem(**bad)
        assert lib.smc_workspace_size(C.byref(p)) == 0, bad
    p = _problem(d=40, ld=48)
    assert lib.smc_workspace_size(C.byref(p)) > 0   # lane-group rows for 32 < d <= 128
    p = _problem(d=130, ld=136)
    assert lib.smc_workspace_size(C.byref(p)) == 0  # d > 128 is not built
    p = _problem(d=40, ld=48, family=2)
    assert lib.smc_workspace_size(C.byref(p)) == 0  # Gaussian test family: d <= 32 only


def test_init_rejects_bad_problem_without_touching_the_device(lib):
    pb = _problem(G=500)
    h = C.c_void_p()
    st = lib.smc_init(C.byref(pb), None, C.byref(h))
    assert st == 1 and not h.value


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(B, "_lib", None)
    with pytest.raises(RuntimeError, match="no fallback"):
        B.lib()


def test_batch_workspace_size(lib):
    assert lib.smc_batch_workspace_size(0) == 0
    assert lib.smc_batch_workspace_size(-3) == 0
    assert lib.smc_batch_workspace_size(65537) == 0
    a, b = lib.smc_batch_workspace_size(1), lib.smc_batch_workspace_size(64)
    assert 0 < a < b
    assert b >= 64 * 8 * 8                            # a results slot per member
    assert lib.smc_batch_workspace_size(65536) > 0


def test_batch_calls_reject_null(lib):
    import ctypes as C
    h = C.c_void_p()
    assert lib.smc_batch_create(None, 1, None, 0, C.byref(h)) == 1
    assert lib.smc_batch_temper(None, None, None, None, None) == 1
    assert lib.smc_batch_mass(None) == 1
    assert lib.smc_batch_resample(None, 0) == 1
    assert lib.smc_batch_move(None, None, 1, 1) == 1
    assert lib.smc_batch_set_graph(None, 1) == 1
    assert lib.smc_batch_graph_captures(None) == 0
    assert lib.smc_batch_launches(None) == 0
    assert lib.smc_batch_last_error(None) == b"no batch"
    lib.smc_batch_destroy(None)
