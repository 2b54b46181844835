"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects invalid arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "crsolve.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(\w+)\s*\(", txt, flags=re.M))
    return sorted(n for n in names if n not in {"if", "while"})


def _lib():
    from paper_1710_00621_amd import _lib
    return _lib


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("sht_synth", "sht_adjoint", "apply_A", "apply_pinv_precond", "pcg_solve",
              "constrained_realization", "build_rhs", "apply_diag_precond", "crs_model_create"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = _lib()
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libcrsolve.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(L.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    assert set(_declared()) == set(L.exported_symbols())


def test_invalid_arguments_rejected_on_host():
    L = _lib()
    lib = L.lib()
    h = ctypes.c_void_p()
    assert lib.crs_grid_healpix(0, ctypes.byref(h)) == L.CRS_EINVAL
    assert lib.crs_grid_healpix(4, None) == L.CRS_EINVAL
    assert lib.crs_grid_healpix(4096, ctypes.byref(h)) == L.CRS_EUNSUPPORTED
    assert lib.crs_grid_gauss_legendre(0, 5, ctypes.byref(h)) == L.CRS_EINVAL
    assert lib.crs_grid_gauss_legendre(5, 9000, ctypes.byref(h)) == L.CRS_EUNSUPPORTED
    assert lib.crs_grid_gauss_legendre(5, 4099, ctypes.byref(h)) == L.CRS_EUNSUPPORTED  # odd prime
    assert lib.crs_model_create(None, None, ctypes.byref(h)) == L.CRS_EINVAL
    assert lib.sht_synth(None, 4, 1, None, 25, None, 10, None) == L.CRS_EINVAL
    assert lib.apply_A(None, 1, None, None, None) == L.CRS_EINVAL
    assert lib.crs_autotune_legendre(None, 8, 1, None) == L.CRS_EINVAL
    out5 = (ctypes.c_int * 5)()
    assert lib.crs_legendre_choice(None, 8, 1, out5) == L.CRS_EINVAL
    assert lib.pcg_solve(None, 2, 1, None, None, 1e-8, 10, None, None, None, None) == L.CRS_EINVAL
    buf = ctypes.create_string_buffer(256)
    assert lib.crs_last_error(buf, 256) == L.CRS_EINVAL
    assert b"NULL" in buf.value or b"must" in buf.value
    assert lib.crs_strerror(L.CRS_EBREAKDOWN) == b"PCG breakdown"
    assert lib.crs_version().startswith(b"crsolve")


def test_model_desc_validation_on_host():
    """Descriptor errors (negative tau, negative C^-1, NULL pointers) are found
    before any device work: no grid handle is needed for the first ones."""
    L = _lib()
    lib = L.lib()
    lk = (ctypes.c_int * 1)(4)
    icl_arr = (ctypes.c_double * 5)(0, 0, 1, 1, -1.0)
    icl = (L.c_double_p * 1)(ctypes.cast(icl_arr, L.c_double_p))
    bands = (L.BandDesc * 1)()
    desc = L.ModelDesc(1, lk, icl, 1, bands, 0)
    h = ctypes.c_void_p()
    assert lib.crs_model_create(ctypes.byref(desc), None, ctypes.byref(h)) == L.CRS_EINVAL
    buf = ctypes.create_string_buffer(256)
    lib.crs_last_error(buf, 256)
    assert b"inv_cl" in buf.value
    desc = L.ModelDesc(0, lk, icl, 1, bands, 0)
    assert lib.crs_model_create(ctypes.byref(desc), None, ctypes.byref(h)) == L.CRS_EINVAL
