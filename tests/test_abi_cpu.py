"""The C-ABI library loads and exports every function include/gwg.h declares;
argument errors are reported before anything touches a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gwg.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2601_04370_amd import build, gwg
    stale = not os.path.exists(gwg.LIB_PATH) or any(
        os.path.getmtime(s) > os.path.getmtime(gwg.LIB_PATH) for s in build.sources())
    if stale:
        build.build()
    return gwg.load_library()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gwg_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("gwg_tmm_rt", "gwg_trace_forward", "gwg_trace_backward", "gwg_loss"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2601_04370_amd import gwg
    names = declared_functions()
    assert set(names) == set(gwg.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_abi_version(lib):
    assert lib.gwg_abi_version() == 2


def test_null_context_is_rejected(lib):
    from paper_2601_04370_amd import gwg
    assert lib.gwg_trace_forward(None, None, None, None, None, None, 0, 0, 0, 0, None, None, 1, None, None) == gwg.GWG_E_INVAL
    assert lib.gwg_trace_backward(None, None, None, 1, None, None) == gwg.GWG_E_INVAL
    assert lib.gwg_loss(None, None, 1, 1, 1, 1, 0, 1.0, 1.0, None, None, None) == gwg.GWG_E_INVAL
    assert lib.gwg_tmm_rt(None, None, None, 0, None, None, 0, None, None) == gwg.GWG_E_INVAL
    assert lib.gwg_destroy(None) == gwg.GWG_E_INVAL
    assert lib.gwg_set_tuning(None, None) == gwg.GWG_E_INVAL
    assert lib.gwg_set_timing(None, 1) == gwg.GWG_E_INVAL
    assert lib.gwg_kernel_times(None, 0, 1, None) == gwg.GWG_E_INVAL
    assert lib.gwg_set_step_source(None, None) == gwg.GWG_E_INVAL
    assert lib.gwg_forward_kept_entries(None, None) == gwg.GWG_E_INVAL
    assert lib.gwg_omega_gradient(None, None, None, None, None) == gwg.GWG_E_INVAL
    assert lib.gwg_autotune(None, None, None, None, None, None, 0, 0, 0, None, None, None) == gwg.GWG_E_INVAL


def test_create_reports_missing_device(lib):
    """Without a gfx950 device visible, gwg_create fails loudly (no CPU fallback)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    from paper_2601_04370_amd import gwg
    h = C.c_void_p(1)
    rc = lib.gwg_create(C.byref(h), 0)
    assert rc == gwg.GWG_E_NODEVICE
    assert not h.value
    assert len(lib.gwg_last_error(None)) > 0
    with pytest.raises(Exception):
        gwg.Context(0)


def test_library_matches_its_sources(lib):
    """The loaded library carries the hash of the sources beside it."""
    from paper_2601_04370_amd import build, gwg
    h = lib.gwg_source_hash()
    assert h.decode() == build.source_hash() == gwg.source_hash()
    assert len(h) == 16
