"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks ``oracle.mpe`` against something other than itself: the
fractions printed in the paper, an independent exact-rational Vandermonde
solve, dense operators built from explicit DFT matrices (``oracle.dense``, no
FFT routine), closed forms of the oscillator, LAPACK's generalised symmetric
eigensolver, and brute-force diagonalisation of tiny grids.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import dense, mpe

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def soft8(grid=(8, 8, 8), box=(16.0, 16.0, 16.0)):
    """Smooth, weak potential whose spectrum is narrow enough for dt-asymptotics at dt ~ 0.1."""
    Z, Y, X = W.mesh(grid, box)
    L = box[0]
    return (0.6 * np.cos(2 * np.pi * X / L) * np.cos(2 * np.pi * Y / L) + 0.4 * np.sin(2 * np.pi * Z / L)
            - 1.2 * np.exp(-((X - 0.7) ** 2 + (Y + 0.3) ** 2 + (Z - 0.4) ** 2) / 4))


def toy8(grid=(8, 8, 8), box=(8.0, 8.0, 8.0)):
    """Non-separable 8^3 toy: oscillator plus an off-centre Gaussian dip."""
    Z, Y, X = W.mesh(grid, box)
    return 0.5 * (X * X + Y * Y + Z * Z) - 1.5 * np.exp(-((X - 0.7) ** 2 + (Y + 0.3) ** 2 + (Z - 0.4) ** 2))


# ------------------------------------------------------------------ coefficients (Eq. coef)
def _golden_coefficients():
    out = {}
    with open(os.path.join(GOLDEN, "mpe_coefficients.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, rest = line.split(":")
            out[int(k)] = [Fraction(t) for t in rest.split()]
    return out


def test_coefficients_match_printed_fractions():
    gold = _golden_coefficients()
    assert sorted(gold) == [2, 3, 4, 5]
    for K, printed in gold.items():
        assert mpe.mpe_coefficients_exact(K) == printed
        np.testing.assert_array_equal(mpe.mpe_coefficients(K), [float(c) for c in printed])


@pytest.mark.parametrize("K", range(1, 7))
def test_coefficients_are_richardson_weights(K):
    c = mpe.mpe_coefficients_exact(K)
    assert c == dense.mpe_weights_vandermonde(K)
    assert sum(c) == 1
    for m in range(1, K):
        assert sum(ck / Fraction(k) ** (2 * m) for k, ck in zip(range(1, K + 1), c)) == 0
    lead = sum(ck / Fraction(k) ** (2 * K) for k, ck in zip(range(1, K + 1), c))
    assert lead == Fraction((-1) ** (K - 1), math.factorial(K) ** 2)


def test_order12_coefficients_and_cost():
    c = mpe.mpe_coefficients_exact(6)
    assert c == [Fraction(-1, 302400), Fraction(8, 945), Fraction(-2187, 4480), Fraction(65536, 14175),
                 Fraction(-9765625, 798336), Fraction(17496, 1925)]
    # Section II: orders 4, 6, 8, 10 need 3, 6, 10, 15 complete FFTs; the same count gives 21 at order 12
    assert [mpe.t2_count(K) for K in range(1, 7)] == [1, 3, 6, 10, 15, 21]
    assert abs(float(sum(abs(x) for x in c)) - 26.4413) < 1e-4


# ------------------------------------------------------------------ operators (Eq. Ham, Eq. so)
@pytest.mark.parametrize("grid,box", [((8, 8, 8), (8.0, 8.0, 8.0)), ((8, 6, 4), (7.0, 5.0, 9.0))])
def test_h_apply_matches_dense(grid, box):
    V = toy8(grid, box)
    H = dense.hamiltonian_dense(V, grid, box, hbar2_over_m=0.7)
    psi = W.random_states(3, 4, grid)
    got = mpe.h_apply(psi, V, grid, box, hbar2_over_m=0.7)
    want = (H @ psi.reshape(4, -1).T).T.reshape(psi.shape)
    np.testing.assert_allclose(got, want, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("grid,box", [((8, 8, 8), (8.0, 8.0, 8.0)), ((6, 8, 4), (9.0, 6.0, 5.0))])
@pytest.mark.parametrize("tau", [0.05, 0.4])
def test_t2_matches_dense(grid, box, tau):
    V = toy8(grid, box)
    psi = W.random_states(5, 3, grid)
    got = mpe.t2(psi, V, tau, grid, box)
    T2 = dense.t2_dense(V, grid, box, tau)
    want = (T2 @ psi.reshape(3, -1).T).T.reshape(psi.shape)
    np.testing.assert_allclose(got, want, atol=1e-13 * np.abs(want).max())


def test_t2_free_plane_wave_and_constant_potential():
    grid, box = (16, 12, 10), (10.0, 6.0, 5.0)
    Z, Y, X = W.mesh(grid, box)
    q = (2 * np.pi * 3 / 10.0, 2 * np.pi * 2 / 6.0, 2 * np.pi * 1 / 5.0)
    psi = np.cos(q[0] * X + q[1] * Y + q[2] * Z)[None]
    tau, v0 = 0.3, -0.7
    q2 = sum(t * t for t in q)
    got = mpe.t2(psi, np.zeros(X.shape), tau, grid, box)
    np.testing.assert_allclose(got, np.exp(-0.5 * tau * q2) * psi, atol=1e-14)
    got = mpe.t2(psi, np.full(X.shape, v0), tau, grid, box)
    np.testing.assert_allclose(got, np.exp(-tau * v0) * np.exp(-0.5 * tau * q2) * psi, atol=1e-13)


def test_t2_free_gaussian_spreads_like_heat_kernel():
    # exp(tau Lap/2) maps a Gaussian of variance s^2 to variance s^2 + tau (amplitude (s^2/(s^2+tau))^{3/2})
    grid, box = (48, 48, 48), (24.0, 24.0, 24.0)
    Z, Y, X = W.mesh(grid, box)
    r2 = X * X + Y * Y + Z * Z
    s2, tau = 1.3, 0.6
    psi = np.exp(-r2 / (2 * s2))[None]
    got = mpe.t2(psi, np.zeros(X.shape), tau, grid, box)
    want = (s2 / (s2 + tau)) ** 1.5 * np.exp(-r2 / (2 * (s2 + tau)))
    np.testing.assert_allclose(got[0], want, atol=1e-12)


# ------------------------------------------------------------------ the expansion (Eq. mcomp)
@pytest.mark.parametrize("K", [1, 2, 3, 4])
def test_mpe_apply_matches_dense_expansion(K):
    grid, box = (6, 8, 4), (6.0, 8.0, 5.0)
    V = toy8(grid, box)
    psi = W.random_states(7, 2, grid)
    dt = 0.3
    got = mpe.mpe_apply(psi, V, dt, K, grid, box)
    M = dense.mpe_dense(V, grid, box, dt, K)
    want = (M @ psi.reshape(2, -1).T).T.reshape(psi.shape)
    np.testing.assert_allclose(got, want, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("K,dts", [(1, (0.1, 0.05)), (2, (0.1, 0.05)), (3, (0.2, 0.1))])
def test_mpe_local_error_order(K, dts):
    """One step of T_2K differs from exp(-dt H) by O(dt^(2K+1)) (Eq. mcomp)."""
    grid, box = (8, 8, 8), (16.0, 16.0, 16.0)   # h = 2 keeps dt*||T|| small
    V = soft8(grid, box)
    H = dense.hamiltonian_dense(V, grid, box)
    psi = W.random_states(9, 1, grid)
    err = []
    for dt in dts:
        E = dense.exact_propagator_dense(H, dt)
        got = mpe.mpe_apply(psi, V, dt, K, grid, box).ravel()
        err.append(np.linalg.norm(got - E @ psi.ravel()))
    slope = math.log2(err[0] / err[1])
    assert abs(slope - (2 * K + 1)) < 0.35, (err, slope)


def _dense_fixed_point(V, grid, box, dt, K, m):
    """Dominant m-dimensional invariant subspace of the dense T_2K, with its Ritz pairs in H."""
    H = dense.hamiltonian_dense(V, grid, box)
    M = dense.mpe_dense(V, grid, box, dt, K)
    M = 0.5 * (M + M.T)              # symmetric up to roundoff: T2 is symmetric
    w, U = np.linalg.eigh(M)
    Q = U[:, ::-1][:, :m]            # largest propagator eigenvalues = lowest states
    th, R = np.linalg.eigh(Q.T @ H @ Q)
    X = Q @ R
    resid = np.linalg.norm(H @ X - X * th, axis=0) ** 2
    return th, resid, H


def test_oracle_iteration_reaches_dense_fixed_point():
    grid, box = (8, 8, 8), (8.0, 8.0, 8.0)
    V = toy8(grid, box)
    m, K, dt = 4, 2, 0.3
    th_ref, rh_ref, _ = _dense_fixed_point(V, grid, box, dt, K, m)
    psi = W.random_states(11, m, grid)
    for _ in range(120):
        r = mpe.iterate(psi, V, dt, K, grid, box)
        psi = r.psi
    np.testing.assert_allclose(r.theta, th_ref, rtol=1e-12)
    np.testing.assert_allclose(r.rh, rh_ref, rtol=1e-6, atol=1e-20)


@pytest.mark.parametrize("K,dts,check_e", [(1, (0.2, 0.1), True), (2, (0.8, 0.4), True), (3, (0.4, 0.2), False)])
def test_fixed_point_error_slopes(K, dts, check_e):
    """At the fixed point of T_2K(dt), the residual norm of the Ritz vector goes as dt^(2K) and
    its Ritz value error as dt^(4K) (the power laws of the paper's convergence figures)."""
    grid, box = (8, 8, 8), (16.0, 16.0, 16.0)
    V = soft8(grid, box)
    H = dense.hamiltonian_dense(V, grid, box)
    e_exact = np.linalg.eigvalsh(H)[0]
    eerr, rnorm = [], []
    for dt in dts:
        th, rh, _ = _dense_fixed_point(V, grid, box, dt, K, 1)
        eerr.append(abs(th[0] - e_exact))
        rnorm.append(math.sqrt(rh[0]))
    assert abs(math.log2(rnorm[0] / rnorm[1]) - 2 * K) < 0.25
    if check_e:   # for K = 3 the Ritz value error is already at roundoff
        assert abs(math.log2(eerr[0] / eerr[1]) - 4 * K) < 0.5


# ------------------------------------------------------------------ orthonormalisation and Rayleigh-Ritz
def test_cholesky_rr_equals_generalised_eigenproblem():
    grid, box = (8, 8, 8), (8.0, 8.0, 8.0)
    V = toy8(grid, box)
    Phi = W.random_states(13, 6, grid)
    Psi, S, L = mpe.cholesky_orthonormalize(Phi)
    G = Psi.reshape(6, -1) @ Psi.reshape(6, -1).T
    assert np.abs(G - np.eye(6)).max() < 1e-13
    HPhi = mpe.h_apply(Phi, V, grid, box)
    Hs = Phi.reshape(6, -1) @ HPhi.reshape(6, -1).T
    want = sla.eigh(0.5 * (Hs + Hs.T), S, eigvals_only=True)
    theta, P, HP, U = mpe.rayleigh_ritz(Psi, mpe.h_apply(Psi, V, grid, box))
    np.testing.assert_allclose(theta, want, rtol=1e-12)
    # rotated vectors stay orthonormal and H-orthogonal
    Pf, HPf = P.reshape(6, -1), HP.reshape(6, -1)
    assert np.abs(Pf @ Pf.T - np.eye(6)).max() < 1e-13
    np.testing.assert_allclose(Pf @ HPf.T, np.diag(theta), atol=1e-12)


def test_residual_e_zero_on_exact_eigenvectors():
    grid, box = (8, 8, 8), (8.0, 8.0, 8.0)
    V = toy8(grid, box)
    H = dense.hamiltonian_dense(V, grid, box)
    w, U = np.linalg.eigh(H)
    psi = U[:, :3].T.reshape(3, 8, 8, 8)
    phi = mpe.mpe_apply(psi, V, 0.2, 3, grid, box)
    re, re_perp, mu = mpe.residual_e(psi, phi)
    # the propagator is not exactly exp(-dt H): its own eigenvectors differ at O(dt^7) only
    assert re.max() < 1e-12 and re_perp.max() < 1e-12
    np.testing.assert_allclose(mu, np.exp(-0.2 * w[:3]), rtol=1e-5)
    rh = mpe.residual_h(psi, mpe.h_apply(psi, V, grid, box), w[:3])
    assert rh.max() < 1e-24


@pytest.mark.parametrize("locked", [0, 2, 5, (1, 3), (0, 2, 4)])
def test_locked_iteration_matches_dense_subspace(locked):
    """Selective propagation (Section III): with the locked states left
    unpropagated, the iteration's Ritz pairs are those of H on the span of the
    locked psi_j and of T psi_j for the others, built here from the dense
    propagator matrix and a QR factorisation; R^E vanishes for the locked
    states and equals the unlocked iteration's value for the others.  An
    integer locks a leading run, a tuple any set of states."""
    grid, box = (8, 8, 8), (8.0, 8.0, 8.0)
    V = toy8(grid, box)
    m, K, dt = 5, 2, 0.3
    Q0, _ = np.linalg.qr(W.random_states(21, m, grid).reshape(m, -1).T)
    psi = Q0.T.reshape(m, *grid)
    H = dense.hamiltonian_dense(V, grid, box)
    M = dense.mpe_dense(V, grid, box, dt, K)
    lk = np.zeros(m, dtype=bool)
    if isinstance(locked, int):
        lk[:locked] = True
    else:
        lk[list(locked)] = True
    B = Q0.copy()
    B[:, ~lk] = M @ Q0[:, ~lk]
    Qb, _ = np.linalg.qr(B)
    want = np.linalg.eigvalsh(Qb.T @ H @ Qb)
    r = mpe.iterate(psi, V, dt, K, grid, box, locked=locked)
    np.testing.assert_allclose(r.theta, want, rtol=1e-11, atol=1e-12)
    # the output block spans the same subspace
    P = r.psi.reshape(m, -1).T
    assert np.abs(P @ (P.T @ Qb) - Qb).max() < 1e-10
    full = mpe.iterate(psi, V, dt, K, grid, box)
    assert np.abs(r.re[lk]).max(initial=0.0) < 1e-14 and np.abs(r.re_perp[lk]).max(initial=0.0) < 1e-14
    np.testing.assert_allclose(r.re[~lk], full.re[~lk], rtol=1e-12, atol=1e-20)
    np.testing.assert_allclose(r.re_perp[~lk], full.re_perp[~lk], rtol=1e-10, atol=1e-20)
    if not lk.any():
        return
    # a different locked set gives a different subspace (the set is honoured, not just its size)
    other = np.roll(lk, 1)
    if (other != lk).any():
        ro = mpe.iterate(psi, V, dt, K, grid, box, locked=tuple(np.flatnonzero(other)))
        assert np.abs(ro.theta - r.theta).max() > 1e-8


# ------------------------------------------------------------------ harmonic oscillator
def test_separable_oscillator_levels():
    e = dense.separable_oscillator_levels(32, 16.0, 10)
    want = np.array([1.5, 2.5, 2.5, 2.5] + [3.5] * 6)
    assert np.abs(e - want).max() < 2e-13
    # 1-D spectral oscillator levels against n + 1/2
    x = -8.0 + 0.5 * np.arange(32)
    e1 = np.linalg.eigvalsh(dense.kinetic_1d(32, 16.0) + np.diag(0.5 * x * x))[:5]
    assert np.abs(e1 - (np.arange(5) + 0.5)).max() < 1e-10


def test_oscillator_t2_fixed_point_closed_form():
    """For V = r^2/2 the T2(dt) fixed point is the Gaussian exp(-a r^2/2), a = sqrt(1 + dt^2/4):
    its Ritz value is 3(a + 1/a)/4 and its R^H is 3(a^2-1)^2/(8a^2)."""
    s = W.harmonic_system(32, 16.0, 1)
    dt = 0.1
    psi = W.random_states(0, 1, s.grid)
    for _ in range(360):
        r = mpe.iterate(psi, s.V, dt, 1, s.grid, s.box)
        psi = r.psi
    a = math.sqrt(1 + dt * dt / 4)
    assert abs(r.theta[0] - 0.75 * (a + 1 / a)) < 1e-13
    assert abs(r.rh[0] / (3 * (a * a - 1) ** 2 / (8 * a * a)) - 1) < 1e-9


@pytest.mark.slow
def test_oracle_solves_oscillator_to_exact_levels():
    s = W.harmonic_system(32, 16.0, 10)
    psi0 = W.random_states(0, 10, s.grid)
    r = mpe.solve(psi0, s.V, 2, s.grid, s.box, dt0=0.1, gamma=1e-10)
    assert r.converged and r.rh.max() < 1e-10
    exact = dense.separable_oscillator_levels(32, 16.0, 10)
    np.testing.assert_allclose(r.theta, exact, rtol=1e-10)
    # degeneracies 1, 3, 6
    assert np.ptp(r.theta[1:4]) < 1e-10 and np.ptp(r.theta[4:10]) < 1e-10


def test_oracle_solves_dense_toy():
    grid, box = (8, 8, 8), (8.0, 8.0, 8.0)
    V = toy8(grid, box)
    exact = np.linalg.eigvalsh(dense.hamiltonian_dense(V, grid, box))[:5]
    psi0 = W.random_states(2, 6, grid)
    r = mpe.solve(psi0, V, 3, grid, box, n_check=5, dt0=0.3, gamma=1e-12)
    assert r.converged
    np.testing.assert_allclose(r.theta[:5], exact, rtol=1e-11)


# ------------------------------------------------------------------ inputs
def test_truncated_icosahedron_geometry():
    P = W.truncated_icosahedron(6.7)
    assert P.shape == (60, 3)
    np.testing.assert_allclose(np.linalg.norm(P, axis=1), 6.7, rtol=1e-13)
    D = np.linalg.norm(P[:, None] - P[None], axis=-1) + np.eye(60) * 1e9
    dmin = D.min()
    assert abs(dmin - 2 * 6.7 / math.sqrt(9 * W.GOLDEN + 10)) < 1e-12
    nb = (D < dmin * 1.0001).sum(axis=1)
    assert (nb == 3).all()          # every carbon has three nearest neighbours; 90 edges
    assert nb.sum() // 2 == 90


# ------------------------------------------------------------------ variances on an unconverged block
@pytest.mark.parametrize("K,locked", [(2, 0), (3, 2)])
def test_iterate_variances_on_unconverged_block(K, locked):
    """R^E_j and R^E_perp_j of one iteration (Section III) on a random orthonormal
    block, far from convergence, against least-squares distances built from the
    dense propagator matrix: R^E_j is the squared distance of T psi_j from the
    line through psi_j, R^E_perp_j its squared distance from span(Psi).  A mix-up
    of the incoming and the propagated block changes both."""
    grid, box = (8, 8, 8), (8.0, 8.0, 8.0)
    V = toy8(grid, box)
    m, dt = 5, 0.3
    Q0, _ = np.linalg.qr(W.random_states(33, m, grid).reshape(m, -1).T)
    psi = Q0.T.reshape(m, *grid)
    F = dense.mpe_dense(V, grid, box, dt, K) @ Q0
    F[:, :locked] = Q0[:, :locked]
    re_ref = np.array([np.sum((F[:, j] - Q0[:, [j]] @ np.linalg.lstsq(Q0[:, [j]], F[:, j], rcond=None)[0]) ** 2)
                       for j in range(m)])
    coef = np.linalg.lstsq(Q0, F, rcond=None)[0]
    perp_ref = np.sum((F - Q0 @ coef) ** 2, axis=0)
    r = mpe.iterate(psi, V, dt, K, grid, box, locked=locked)
    assert re_ref[locked:].min() > 1e-6          # the block is far from an invariant subspace
    np.testing.assert_allclose(r.re, re_ref, rtol=1e-10, atol=1e-14)
    np.testing.assert_allclose(r.re_perp, perp_ref, rtol=1e-10, atol=1e-14)
    assert np.all(r.re_perp <= r.re * (1 + 1e-12) + 1e-15)


# ------------------------------------------------------------------ Romberg-type T6 (Eq. sixp)
def test_romberg6_weights_match_printed():
    # Eq. sixp prints -1/15 and 16/15; the weights follow from cancelling T4's leading error
    assert dense.romberg_weights(4) == [Fraction(-1, 15), Fraction(16, 15)]


@pytest.mark.parametrize("grid,box", [((6, 8, 4), (6.0, 8.0, 5.0)), ((8, 8, 8), (8.0, 8.0, 8.0))])
def test_romberg6_matches_dense(grid, box):
    V = toy8(grid, box)
    psi = W.random_states(7, 2, grid)
    dt = 0.3
    got = mpe.romberg6_apply(psi, V, dt, grid, box)
    R = dense.romberg6_dense(V, grid, box, dt)
    want = (R @ psi.reshape(2, -1).T).T.reshape(psi.shape)
    np.testing.assert_allclose(got, want, atol=1e-12 * np.abs(want).max())
    # a different operator from the multi-product T6 of the same order
    assert np.abs(got - mpe.mpe_apply(psi, V, dt, 3, grid, box)).max() > 1e-8 * np.abs(want).max()


def test_romberg6_local_error_order():
    """Local error of one Romberg step (Eq. sixp) built on the order-4 expansion
    (Eq. four) against exp(-dt H).  The expansion's error is not a pure odd-power
    exponent: with T2(e) = exp(eH + e^3 A + ...), T4 = -T2(e)/3 + 4 T2(e/2)^2/3
    keeps a term -e^6 A^2/8 from the second order of each exponential, which
    halving the step does not cancel (-1/15 and 16/15 of it leave e^6 A^2/240).
    So the Romberg combination has local error O(dt^6) -- fifth order -- while the
    multi-product T6 of the same cost class has O(dt^7)."""
    grid, box = (8, 8, 8), (16.0, 16.0, 16.0)
    V = soft8(grid, box)
    H = dense.hamiltonian_dense(V, grid, box)
    psi = W.random_states(9, 1, grid)
    err, err_mpe = [], []
    for dt in (0.2, 0.1):
        E = dense.exact_propagator_dense(H, dt) @ psi.ravel()
        err.append(np.linalg.norm(mpe.romberg6_apply(psi, V, dt, grid, box).ravel() - E))
        err_mpe.append(np.linalg.norm(mpe.mpe_apply(psi, V, dt, 3, grid, box).ravel() - E))
    slope = math.log2(err[0] / err[1])
    assert abs(slope - 6) < 0.3, (err, slope)
    assert math.log2(err_mpe[0] / err_mpe[1]) > 6.4
    assert err[1] > 3 * err_mpe[1]


def test_romberg6_cost():
    """Section II: going from order 4 to 6 the Romberg form triples the T2 count (3 -> 9)
    while the expansion adds K + 1 = 3 (3 -> 6)."""
    assert mpe.romberg6_t2_count() == 3 * mpe.t2_count(2) == 9
    assert mpe.t2_count(3) - mpe.t2_count(2) == 3


def test_iterate_with_romberg6_matches_dense_subspace():
    grid, box = (8, 8, 8), (8.0, 8.0, 8.0)
    V = toy8(grid, box)
    m, dt = 4, 0.3
    Q0, _ = np.linalg.qr(W.random_states(35, m, grid).reshape(m, -1).T)
    psi = Q0.T.reshape(m, *grid)
    B = dense.romberg6_dense(V, grid, box, dt) @ Q0
    Qb, _ = np.linalg.qr(B)
    want = np.linalg.eigvalsh(Qb.T @ dense.hamiltonian_dense(V, grid, box) @ Qb)
    r = mpe.iterate(psi, V, dt, 3, grid, box, romberg6=True)
    np.testing.assert_allclose(r.theta, want, rtol=1e-11, atol=1e-12)


# ------------------------------------------------------------------ the paper's model inputs
def test_plane_wave_states_are_orthonormal_kinetic_eigenstates():
    """The plane-wave start (Section III, convergence figures): discretely orthonormal,
    each an eigenvector of the dense spectral kinetic operator, and together the
    lowest eigenvalues of that operator in order."""
    grid, box = (8, 6, 10), (7.0, 5.0, 9.0)
    n = 20
    P = W.plane_wave_states(n, grid, box).reshape(n, -1)
    assert np.abs(P @ P.T - np.eye(n)).max() < 1e-13
    T = dense.hamiltonian_dense(np.zeros((10, 6, 8)), grid, box, hbar2_over_m=2.0)
    TP = (T @ P.T).T
    e = np.einsum("ij,ij->i", P, TP)
    assert np.abs(TP - e[:, None] * P).max() < 1e-10
    assert np.all(np.diff(e) >= -1e-12) and abs(e[0]) < 1e-12
    np.testing.assert_allclose(e, np.linalg.eigvalsh(T)[:n], atol=1e-10)


def test_sech_cage_potential():
    grid, box = (32, 32, 32), (16.0, 16.0, 16.0)
    c = W.truncated_icosahedron(3.0)
    V = W.sech_wells(grid, box, c[:1], 2.0, 0.7)
    Z, Y, X = W.mesh(grid, box)
    r = np.sqrt((X - c[0, 0]) ** 2 + (Y - c[0, 1]) ** 2 + (Z - c[0, 2]) ** 2)
    i = np.unravel_index(np.argmin(r), r.shape)
    assert abs(V[i] + 2.0 / math.cosh(r[i] / 0.7)) < 1e-14
    assert V.max() < 0 and V.min() >= -2.0
    full = W.sech_cage_potential(grid, box, V0=1.0, d=0.5, radius=3.0)
    assert full.shape == (32, 32, 32) and full.min() < -1.0    # neighbouring wells overlap at d = 0.5
