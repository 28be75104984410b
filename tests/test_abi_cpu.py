"""Host-side checks of the C-ABI library (no GPU needed).

The library must load, export every function declared in include/mpe.h, and
its host-only entry points (coefficients, version, argument validation that
fails before any device work) must behave as documented.
"""
import ctypes as C
import os
import re
from fractions import Fraction

import pytest

from oracle import mpe as oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpe.h")
LIBPATH = os.path.join(ROOT, "paper_0809_3739_amd", "libmpe.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:mpe|wsn)_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIBPATH):
        pytest.fail("libmpe.so is not built (run __graft_entry__.build())")
    from paper_0809_3739_amd import _lib
    return _lib.load(LIBPATH)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["mpe_plan_create", "mpe_plan_destroy", "mpe_set_potential", "mpe_step", "mpe_orthonormalize",
                     "mpe_rayleigh_ritz", "mpe_residuals", "mpe_iterate", "mpe_last_error"]:
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    raw = C.CDLL(LIBPATH)
    for name in declared_functions():
        assert hasattr(raw, name), name


def test_binding_covers_every_declared_symbol():
    from paper_0809_3739_amd import _lib
    assert sorted(_lib.SIGNATURES) == declared_functions()


def test_abi_version(lib):
    assert lib.mpe_abi_version() == 1


@pytest.mark.parametrize("order", [2, 4, 6, 8, 10, 12])
def test_library_coefficients_match_oracle(lib, order):
    K = order // 2
    buf = (C.c_double * K)()
    assert lib.mpe_coefficients(order, buf) == 0
    exact = oracle.mpe_coefficients_exact(K)
    for k in range(K):
        assert buf[k] == float(exact[k])          # one correct rounding of the exact rational
        assert Fraction(buf[k]) == Fraction(float(exact[k]))


@pytest.mark.parametrize("order", [0, 1, 3, 14, -2])
def test_bad_order_rejected(lib, order):
    buf = (C.c_double * 8)()
    assert lib.mpe_coefficients(order, buf) == 1
    h = C.c_void_p(123)
    g = (C.c_int32 * 3)(32, 32, 32)
    b = (C.c_double * 3)(16.0, 16.0, 16.0)
    assert lib.mpe_plan_create(C.byref(h), g, b, 10, order, 0, 0, None) == 1
    assert h.value is None


def test_plan_create_argument_validation(lib):
    h = C.c_void_p()
    b = (C.c_double * 3)(16.0, 16.0, 16.0)
    odd = (C.c_int32 * 3)(33, 32, 32)
    assert lib.mpe_plan_create(C.byref(h), odd, b, 4, 4, 0, 0, None) == 1          # odd size
    g = (C.c_int32 * 3)(40, 40, 40)
    assert lib.mpe_plan_create(C.byref(h), g, b, 4, 4, 0, 0, None) == 2            # 40 = 2^3*5: no kernel
    g = (C.c_int32 * 3)(32, 32, 32)
    assert lib.mpe_plan_create(C.byref(h), g, b, 120, 4, 0, 20, None) == 2         # 140 states > 128
    assert lib.mpe_plan_create(C.byref(h), g, b, 0, 4, 0, 0, None) == 1            # no states
    bad = (C.c_double * 3)(16.0, -1.0, 16.0)
    assert lib.mpe_plan_create(C.byref(h), g, bad, 4, 4, 0, 0, None) == 1          # box
    g384 = (C.c_int32 * 3)(384, 192, 192)
    assert lib.mpe_plan_create(C.byref(h), g384, b, 4, 4, 0, 0, None) == 2         # no 384-point row pass
    g36 = (C.c_int32 * 3)(32, 36, 32)
    assert lib.mpe_plan_create(C.byref(h), g36, b, 4, 4, 1, 0, None) == 2          # no 36-point column pass
    assert lib.mpe_plan_create(None, g, b, 4, 4, 0, 0, None) == 1


def test_status_strings(lib):
    for code in range(9):
        assert lib.mpe_status_string(code)


def test_warm_start_net_rejects_bad_shapes_before_device_work(lib):
    h = C.c_void_p()
    for grid, n_out, batch in [(6, 8, 1), (30, 8, 1), (32, 12, 1), (32, 136, 1), (32, 8, 0)]:
        assert lib.wsn_create(C.byref(h), grid, n_out, batch, 0, None) == 1, (grid, n_out, batch)
        assert not h.value
    assert lib.wsn_num_params(None) == -1
    assert lib.wsn_destroy(None) == 1
    assert lib.wsn_last_error(None) == b"null network"
    assert lib.wsn_upsample_periodic(None, 1, 4, 2, None, None) == 1


def test_null_plan_setters_fail_before_device_work(lib):
    """Setters on a null plan return MPE_ERR_INVALID_ARGUMENT without touching a device."""
    mask = (C.c_uint8 * 4)(0, 1, 0, 1)
    assert lib.mpe_set_locked(None, 1) == 1
    assert lib.mpe_set_locked_states(None, C.cast(mask, C.c_void_p)) == 1
    assert lib.mpe_set_locked_states(None, None) == 1
    assert lib.mpe_get_locked(None) == -1
    assert lib.mpe_set_graph(None, 1) == 1
    assert lib.mpe_set_variances(None, 1) == 1
