"""Plausible mistakes planted in the CPU oracle must fail at least one pin.

Each case monkeypatches one oracle routine with a wrong variant (a dropped
factor, transposed axes, a wrong sign or step) and runs the fast pins that
should catch it.  Nothing here touches a GPU.
"""
import numpy as np
import pytest
import scipy.fft as sfft

from tests import test_oracle_pins as pins  # noqa: E402
from oracle import mpe


def _fails(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


def _ks_no_half(grid, box, hbar2_over_m=1.0):
    return 2.0 * _REAL_KS(grid, box, hbar2_over_m)


def _ks_axes_swapped(grid, box, hbar2_over_m=1.0):
    nx, ny, nz = grid
    Lx, Ly, Lz = box
    qx = 2 * np.pi * sfft.rfftfreq(nx, d=Lz / nx)      # wrong box length on x
    qy = 2 * np.pi * sfft.fftfreq(ny, d=Ly / ny)
    qz = 2 * np.pi * sfft.fftfreq(nz, d=Lx / nz)
    return 0.5 * hbar2_over_m * (qz[:, None, None] ** 2 + qy[None, :, None] ** 2 + qx[None, None, :] ** 2)


_REAL_KS = mpe.kinetic_symbol
_REAL_COEF = mpe.mpe_coefficients_exact
_REAL_T2 = mpe.t2


def _coef_sign(K):
    c = _REAL_COEF(K)
    return [-x if i == 0 else x for i, x in enumerate(c)] if K > 1 else c


def _t2_full_v(psi, V, tau, grid, box, hbar2_over_m=1.0, _ksym=None):
    return _REAL_T2(psi, 2.0 * V, tau, grid, box, hbar2_over_m, _ksym)


def _mpe_wrong_substep(psi, V, dt, K, grid, box, hbar2_over_m=1.0):
    c = mpe.mpe_coefficients(K)
    acc = np.zeros_like(psi)
    for k in range(1, K + 1):
        u = psi
        for _ in range(k):
            u = _REAL_T2(u, V, dt / (k * k), grid, box, hbar2_over_m)    # dt/k^2 instead of dt/k
        acc += c[k - 1] * u
    return acc


_REAL_ITERATE = mpe.iterate


def _iterate_lock_off_by_one(psi, V, dt, K, grid, box, hbar2_over_m=1.0, keep_phi=False, locked=0, romberg6=False):
    return _REAL_ITERATE(psi, V, dt, K, grid, box, hbar2_over_m, keep_phi, locked + 1 if locked else 0, romberg6)


def _iterate_variances_swapped(psi, V, dt, K, grid, box, hbar2_over_m=1.0, keep_phi=False, locked=0,
                              romberg6=False):
    r = _REAL_ITERATE(psi, V, dt, K, grid, box, hbar2_over_m, True, locked, romberg6)
    re, re_perp, _ = mpe.residual_e(r.phi, psi)     # propagated block in place of the incoming one
    r.re, r.re_perp = re, re_perp
    return r


_REAL_MPE_APPLY = mpe.mpe_apply


def _romberg_half_step_once(psi, V, dt, grid, box, hbar2_over_m=1.0):
    full = _REAL_MPE_APPLY(psi, V, dt, 2, grid, box, hbar2_over_m)
    half = _REAL_MPE_APPLY(psi, V, 0.5 * dt, 2, grid, box, hbar2_over_m)   # T4(eps/2) once, not squared
    return (-1.0 / 15.0) * full + (16.0 / 15.0) * half


CASES = [
    ("kinetic symbol without the 1/2", "kinetic_symbol", _ks_no_half,
     [(pins.test_h_apply_matches_dense, ((8, 8, 8), (8.0, 8.0, 8.0)))]),
    ("kinetic symbol with box lengths of x and z exchanged", "kinetic_symbol", _ks_axes_swapped,
     [(pins.test_h_apply_matches_dense, ((8, 6, 4), (7.0, 5.0, 9.0)))]),
    ("first coefficient with the wrong sign", "mpe_coefficients_exact", _coef_sign,
     [(pins.test_coefficients_match_printed_fractions, ()), (pins.test_coefficients_are_richardson_weights, (3,))]),
    ("full potential on both sides of T2", "t2", _t2_full_v,
     [(pins.test_t2_matches_dense, ((8, 8, 8), (8.0, 8.0, 8.0), 0.4))]),
    ("sub-step dt/k^2 in the expansion", "mpe_apply", _mpe_wrong_substep,
     [(pins.test_mpe_apply_matches_dense_expansion, (2,))]),
    ("one state too many left unpropagated", "iterate", _iterate_lock_off_by_one,
     [(pins.test_locked_iteration_matches_dense_subspace, (2,))]),
    ("R^E formed with the propagated and incoming blocks exchanged", "iterate", _iterate_variances_swapped,
     [(pins.test_iterate_variances_on_unconverged_block, (2, 0))]),
    ("Romberg T6 with one half step instead of two", "romberg6_apply", _romberg_half_step_once,
     [(pins.test_romberg6_matches_dense, ((6, 8, 4), (6.0, 8.0, 5.0))), (pins.test_romberg6_local_error_order, ())]),
]


@pytest.mark.parametrize("name,attr,wrong,checks", CASES, ids=[c[0] for c in CASES])
def test_planted_mistake_is_caught(monkeypatch, name, attr, wrong, checks):
    monkeypatch.setattr(mpe, attr, wrong)
    assert any(_fails(fn, *args) for fn, args in checks), name
