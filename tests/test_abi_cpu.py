"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching a GPU."""

import ctypes
import os
import re

import pytest

import paper_1508_00115_amd as sph

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sph.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sph_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(sph.LIB_PATH):
        pytest.fail("libsph.so missing: run __graft_entry__.build() first")
    return sph.load_library()


def test_header_declares_the_binding_exports():
    assert _declared() == sorted(sph.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_status_strings_and_version(lib):
    assert sph.status_string(sph.SPH_OK) == "ok"
    for code in range(1, 7):
        assert sph.status_string(code) not in ("ok", "unknown status")
    assert sph.status_string(99) == "unknown status"
    assert "gfx950" in sph.sph_version()


def test_struct_layouts_match_header(lib):
    # the ctypes mirrors must have the sizes the C compiler gave the structs
    for which, mirror in enumerate((sph.sph_params, sph.sph_stats, sph.sph_timings, sph.sph_build_info)):
        assert lib.sph_struct_size(which) == ctypes.sizeof(mirror), mirror.__name__
    assert lib.sph_struct_size(4) == -1
    assert ctypes.sizeof(sph.sph_stats) == 96


def test_create_rejects_null_out_and_bad_params(lib):
    assert lib.sph_create(None, 0, None) == sph.SPH_E_ARG
    out = ctypes.c_void_p()
    bad = sph.sph_params()
    bad.h_margin = 0.5  # a margin must exceed 1
    assert lib.sph_create(ctypes.byref(bad), 0, ctypes.byref(out)) == sph.SPH_E_ARG
    assert "sph_params" in sph.sph_last_error(None)
    bad = sph.sph_params()
    bad.n_tol = float("nan")
    assert lib.sph_create(ctypes.byref(bad), 0, ctypes.byref(out)) == sph.SPH_E_ARG
    assert lib.sph_create(None, -1, ctypes.byref(out)) == sph.SPH_E_ARG
    assert out.value is None


def test_calls_on_null_context_are_argument_errors(lib):
    st = sph.sph_stats()
    assert lib.sph_build_cells(None, 1, None, None, 1, None, None, None) == sph.SPH_E_ARG
    assert lib.sph_density(None, None, None, None, None, None, ctypes.byref(st), None) == sph.SPH_E_ARG
    assert lib.sph_force(None, None, None, None, None, None, None, None) == sph.SPH_E_ARG
    assert lib.sph_density_f64(None, None, None, None, None, None, None, None) == sph.SPH_E_ARG
    assert lib.sph_force_f64(None, None, None, None, None, None, None, None) == sph.SPH_E_ARG
    lib.sph_destroy(None)  # no-op


def test_binding_refuses_missing_library(tmp_path):
    with pytest.raises(RuntimeError, match="not built"):
        sph._lib = None
        try:
            sph.load_library(str(tmp_path / "nope.so"))
        finally:
            sph._lib = None
