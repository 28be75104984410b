"""Dense exact references on small grids (test infrastructure only).

Independent of ``oracle.mpe``: no FFT routine is used.  Every operator is an
explicit matrix built from the DFT matrix ``F_jk = exp(-2 pi i j k / n)`` written
out element by element, so a mistake in the oracle's FFT-based operators (axis
order, half-spectrum handling, Nyquist, normalisation) shows up as a mismatch.

* ``kinetic_1d`` -- the spectral kinetic matrix -(hbar^2/2m) d^2/dx^2 on a periodic
  axis (Eq. Ham restricted to one axis).
* ``hamiltonian_dense`` -- the full N x N spectral H = T + V for N <= ~1000.
* ``separable_oscillator_levels`` -- exact grid eigenvalues of the 3-D oscillator
  as sums of 1-D dense eigenvalues (the discrete H is a Kronecker sum).
* ``t2_dense`` / ``mpe_dense`` -- the split operator (Eq. so) and the
  multi-product expansion (Eq. mcomp) as explicit matrices, with exp(-tau T)
  from the eigen-decomposition of the 1-D kinetic matrices.
* ``romberg6_dense`` -- the Romberg-type sixth-order operator of Eq. sixp as an
  explicit matrix, its weights from an exact 2 x 2 solve.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def dft_matrix(n: int) -> np.ndarray:
    j = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(j, j) / n)


def wavenumbers(n: int, L: float) -> np.ndarray:
    """q_m = 2 pi m / L for m = 0..n/2, -(n/2-1)..-1 (Nyquist taken positive)."""
    m = np.arange(n)
    m = np.where(m <= n // 2, m, m - n)
    return 2.0 * np.pi * m / L


def kinetic_1d(n: int, L: float, hbar2_over_m: float = 1.0) -> np.ndarray:
    """Real symmetric matrix of -(hbar^2/2m) d^2/dx^2 in the periodic spectral basis."""
    F = dft_matrix(n)
    q = wavenumbers(n, L)
    T = (F.conj().T @ np.diag(0.5 * hbar2_over_m * q * q) @ F) / n
    assert np.max(np.abs(T.imag)) < 1e-9 * max(1.0, np.max(np.abs(T.real)))
    return T.real.copy()


def _kron_sum(Tx, Ty, Tz):
    """T acting on vectors flattened in [z][y][x] order (x fastest)."""
    Ix, Iy, Iz = (np.eye(len(T)) for T in (Tx, Ty, Tz))
    return (np.kron(np.kron(Tz, Iy), Ix) + np.kron(np.kron(Iz, Ty), Ix)
            + np.kron(np.kron(Iz, Iy), Tx))


def hamiltonian_dense(V: np.ndarray, grid, box, hbar2_over_m: float = 1.0) -> np.ndarray:
    nx, ny, nz = grid
    Lx, Ly, Lz = box
    T = _kron_sum(kinetic_1d(nx, Lx, hbar2_over_m), kinetic_1d(ny, Ly, hbar2_over_m),
                  kinetic_1d(nz, Lz, hbar2_over_m))
    return T + np.diag(np.asarray(V, dtype=np.float64).ravel())


def separable_oscillator_levels(n: int, L: float, count: int, omega: float = 1.0) -> np.ndarray:
    """Lowest ``count`` eigenvalues of the 3-D oscillator on an n^3 grid of side L.

    H = H1(x) + H1(y) + H1(z) with H1 = T1 + omega^2 x^2 / 2 (dense n x n), so the
    3-D levels are all sums e_a + e_b + e_c of the 1-D levels.
    """
    x = -0.5 * L + (L / n) * np.arange(n)
    e = np.linalg.eigvalsh(kinetic_1d(n, L) + np.diag(0.5 * omega * omega * x * x))
    k = min(n, count + 2)
    e = e[:k]
    sums = (e[:, None, None] + e[None, :, None] + e[None, None, :]).ravel()
    return np.sort(sums)[:count]


def _expm_sym(A: np.ndarray, t: float) -> np.ndarray:
    w, U = np.linalg.eigh(A)
    return (U * np.exp(t * w)) @ U.T


def kinetic_propagator_dense(grid, box, tau: float, hbar2_over_m: float = 1.0) -> np.ndarray:
    """exp(-tau T) as a dense matrix; the 1-D kinetic parts commute, so it is a Kronecker product."""
    nx, ny, nz = grid
    Lx, Ly, Lz = box
    Ex = _expm_sym(kinetic_1d(nx, Lx, hbar2_over_m), -tau)
    Ey = _expm_sym(kinetic_1d(ny, Ly, hbar2_over_m), -tau)
    Ez = _expm_sym(kinetic_1d(nz, Lz, hbar2_over_m), -tau)
    return np.kron(np.kron(Ez, Ey), Ex)


def t2_dense(V: np.ndarray, grid, box, tau: float, hbar2_over_m: float = 1.0) -> np.ndarray:
    """Dense split operator exp(-tau V/2) exp(-tau T) exp(-tau V/2) (Eq. so, eps = -tau)."""
    d = np.exp(-0.5 * tau * np.asarray(V, dtype=np.float64).ravel())
    return d[:, None] * kinetic_propagator_dense(grid, box, tau, hbar2_over_m) * d[None, :]


def mpe_weights_vandermonde(K: int) -> np.ndarray:
    """Richardson weights: the w_k with sum_k w_k k^(-2m) = delta_m0 for m = 0..K-1.

    An independent route to the MPE coefficients: T2(eps/k)^k carries only even
    powers eps^2m / k^2m of error in its exponent (Eq. secerr), so eliminating
    m = 1..K-1 is a Vandermonde solve at nodes 1/k^2.  Solved exactly in rationals.
    """
    A = [[Fraction(1, k ** (2 * m)) for k in range(1, K + 1)] for m in range(K)]
    b = [Fraction(1 if m == 0 else 0) for m in range(K)]
    n = K
    M = [row[:] + [b[i]] for i, row in enumerate(A)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col] / M[col][col]
                M[r] = [a - f * c for a, c in zip(M[r], M[col])]
    return [M[i][n] / M[i][i] for i in range(n)]


def mpe_dense(V: np.ndarray, grid, box, dt: float, K: int, hbar2_over_m: float = 1.0) -> np.ndarray:
    """Dense order-2K MPE operator sum_k w_k T2(dt/k)^k with Vandermonde weights."""
    w = [float(x) for x in mpe_weights_vandermonde(K)]
    N = int(np.prod(grid))
    out = np.zeros((N, N))
    for k in range(1, K + 1):
        out += w[k - 1] * np.linalg.matrix_power(t2_dense(V, grid, box, dt / k, hbar2_over_m), k)
    return out


def romberg_weights(order: int) -> list:
    """Weights (w_1, w_2) with w_1 + w_2 = 1 and w_1 + w_2 / 2^order = 0.

    An integrator of order ``order`` has a one-step error C eps^(order+1); two
    steps at eps/2 carry 2 C (eps/2)^(order+1) = C eps^(order+1) / 2^order, so
    these weights cancel it (an exact rational 2 x 2 solve, independent of the
    printed fractions of Eq. sixp)."""
    r = Fraction(1, 2 ** order)
    w2 = Fraction(1) / (1 - r)
    return [1 - w2, w2]


def romberg6_dense(V: np.ndarray, grid, box, dt: float, hbar2_over_m: float = 1.0) -> np.ndarray:
    """Dense Romberg T6 = w_1 T4(dt) + w_2 T4(dt/2)^2 (Eq. sixp) with T4 the dense order-4 MPE matrix."""
    w = [float(x) for x in romberg_weights(4)]
    A = mpe_dense(V, grid, box, dt, 2, hbar2_over_m)
    B = mpe_dense(V, grid, box, 0.5 * dt, 2, hbar2_over_m)
    return w[0] * A + w[1] * (B @ B)


def exact_propagator_dense(H: np.ndarray, dt: float) -> np.ndarray:
    return _expm_sym(H, -dt)
