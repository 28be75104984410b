"""Checks of the seeded inputs that stand for the paper's workloads (no GPU).

The sech cage of Section III prints V0 = 1 (hbar^2/2m units) and d = 0.05 bohr;
the study's "fitted" reading instead takes the well depth and width for which
one isolated well -V0/cosh(r/d) has its 1s and 1p levels at the centres of the
paper's two groups of levels, -5.245 and -2.992 hbar^2/2m.  The radial
equations -u'' + (l(l+1)/r^2 + V(r)) u = E u are solved here by second-order
finite differences on a fine radial grid (extrapolated in the spacing).
"""
import numpy as np
import scipy.linalg as sla

import workloads as W


def radial_level(V0, d, l, h, R=14.0):
    n = int(R / h) - 1
    r = h * np.arange(1, n + 1)
    main = 2.0 / h ** 2 + l * (l + 1) / r ** 2 - V0 / np.cosh(r / d)
    off = -np.ones(n - 1) / h ** 2
    return sla.eigvalsh_tridiagonal(main, off, select="i", select_range=(0, 0))[0]


def test_fitted_sech_well_levels():
    from paper_0809_3739_amd.sech_study import READINGS
    V0, d, _, _ = READINGS["fitted"]
    for l, want in ((0, -5.245), (1, -2.992)):
        e1, e2 = radial_level(V0, d, l, 0.004), radial_level(V0, d, l, 0.002)
        e = e2 + (e2 - e1) / 3.0          # second order in h: Richardson step
        assert abs(e - want) < 2e-3, (l, e)


def test_printed_sech_well_binds_nothing():
    # V0 d^2 = 0.0025 in -Lap units: one well has no bound level
    assert radial_level(1.0, 0.05, 0, 0.002) > 0


def test_disjoint_sign_states_exactly_orthonormal_in_float32():
    x = W.disjoint_sign_states(5, 125, (64, 64, 64)).reshape(125, -1)
    assert np.array_equal(x.astype(np.float32).astype(np.float64), x)
    assert np.array_equal(x @ x.T, np.eye(125))
