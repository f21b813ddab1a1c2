"""The C-ABI library loads on the CPU host and exports every function that
the headers under include/ declare; host-only entry points validate their
arguments.  No device work is launched here."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


@pytest.fixture(scope="module")
def lib():
    from paper_2003_07968_amd import lbm
    if not os.path.exists(lbm.LIB_PATH):
        from paper_2003_07968_amd import build
        build.build()
    return lbm._load()


def declared_functions():
    names = set()
    for header in HEADERS:
        text = open(header).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names.update(re.findall(r"\b(lbm_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("lbm_init", "lbm_step", "lbm_moments", "lbm_sync", "lbm_diagnostics",
                     "lbm_get_populations", "lbm_set_populations", "lbm_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2003_07968_amd import lbm
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(lbm.EXPORTED)


def test_workspace_size_and_validation(lib):
    from paper_2003_07968_amd import lbm
    from paper_2003_07968_amd import workloads as W
    p = lbm.make_params(W.params(64, 48, tr=0.8))
    n = lib.lbm_workspace_bytes(ctypes.byref(p))
    # two population copies of 9 planes, one density snapshot, small scratch
    assert n >= (2 * 9 + 1) * 64 * 48 * 8
    assert n < (2 * 9 + 1) * 64 * 48 * 8 + 4 * 2**20
    for field, value in (("tau", 0.5), ("G", 0.0), ("nx", 2), ("storage", 5), ("force_on", 2)):
        q = lbm.make_params(W.params(64, 48, tr=0.8))
        setattr(q, field, value)
        assert lib.lbm_workspace_bytes(ctypes.byref(q)) == 0, field
    m = lbm.make_params(W.params(64, 48, tr=0.8, collision="mrt", mrt=(1.0, 0.9, 1.1, 1.0, 1.2)))
    assert lib.lbm_workspace_bytes(ctypes.byref(m)) == n
    for field, value in (("collision", 2), ("tau_e", 0.5), ("tau_q", float("nan")),
                         ("tau_rho", 0.4)):
        q = lbm.make_params(W.params(64, 48, tr=0.8, collision="mrt"))
        setattr(q, field, value)
        assert lib.lbm_workspace_bytes(ctypes.byref(q)) == 0, field
    # the MRT relaxation times are not read for BGK
    q = lbm.make_params(W.params(64, 48, tr=0.8))
    q.tau_e = 0.1
    assert lib.lbm_workspace_bytes(ctypes.byref(q)) == n
    h = ctypes.c_void_p()
    st = lib.lbm_init(ctypes.byref(p), None, 0, None, None, None, None, ctypes.byref(h))
    assert st == lbm.LBM_ERR_INVALID_ARG and not h.value


def test_status_strings(lib):
    from paper_2003_07968_amd import lbm
    for st in (lbm.LBM_OK, lbm.LBM_ERR_INVALID_ARG, lbm.LBM_ERR_DOMAIN, lbm.LBM_ERR_DEVICE,
               lbm.LBM_ERR_OOM, lbm.LBM_ERR_STATE):
        assert lib.lbm_status_string(st)
    assert lib.lbm_last_error(None) == b""
    assert lib.lbm_time(None) == -1


def test_null_handle_rejected_by_host_entry_points(lib):
    from paper_2003_07968_amd import lbm
    out = (ctypes.c_int32 * 3)()
    assert lib.lbm_set_fusion(None, 2, 0, 0) == lbm.LBM_ERR_INVALID_ARG
    assert lib.lbm_set_fusion(None, 1, 0, 0) == lbm.LBM_ERR_INVALID_ARG
    assert lib.lbm_get_fusion(None) == -1
    assert lib.lbm_set_launch(None, 256, 8) == lbm.LBM_ERR_INVALID_ARG
    assert lib.lbm_get_launch(None, out) == lbm.LBM_ERR_INVALID_ARG
    assert lib.lbm_step(None, 1) == lbm.LBM_ERR_INVALID_ARG


def test_probe_sizes_and_validation(lib):
    # the bandwidth probe's buffer size (nine planes of nx rounded up to 16
    # FP64 values, one per row) and its argument checks, before any launch
    from paper_2003_07968_amd import lbm
    assert lib.lbm_probe_stream_bytes(2048, 8192) == 9 * 2048 * 8192 * 8
    assert lib.lbm_probe_stream_bytes(37, 23) == 9 * 48 * 23 * 8
    assert lib.lbm_probe_stream_bytes(2, 10) == 0 and lib.lbm_probe_stream_bytes(10, 2) == 0
    a, b = ctypes.c_void_p(16), ctypes.c_void_p(32)   # never dereferenced: rejected first
    for args in ((None, b, 16, 16, 4), (a, None, 16, 16, 4), (a, a, 16, 16, 4),
                 (a, b, 2, 16, 4), (a, b, 16, 2, 4), (a, b, 16, 16, 0), (a, b, 16, 10**7, 1)):
        assert lib.lbm_probe_stream(*args, None) == lbm.LBM_ERR_INVALID_ARG, args
