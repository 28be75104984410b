"""Plain FP64 CPU oracle of the MPE imaginary-time eigensolver.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.  It shares no code with
the GPU library (no kernels, headers, tables or helpers); it depends on NumPy /
SciPy and on the seeded input generators in ``workloads`` only.

Every function follows one passage of Chin, Janecek and Krotscheck, "Any order
imaginary time propagation method for solving the Schroedinger equation"
(arXiv:0809.3739), cited by section and equation label.  Conventions:

* states are real arrays ``[m][nz][ny][nx]`` (x fastest), normalised discretely
  (sum over grid points of psi^2 = 1, no volume element);
* ``dt`` is the positive imaginary time step, the paper's epsilon = -dt
  (Introduction, Eq. evol);
* ``hbar2_over_m`` is hbar^2/m, so the kinetic operator is T = -(hbar2_over_m/2) Lap
  (Eq. Ham), applied spectrally on the periodic grid;
* grid and box are given as (nx, ny, nz) and (Lx, Ly, Lz).

Readings of silent or garbled passages are listed in the module constants and
the docstrings below (sign of epsilon, the index E_i in the variances, the
orthogonalisation method, the step schedule).
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field
from fractions import Fraction

import numpy as np
import scipy.fft as sfft
import scipy.linalg as sla

WORKERS = int(os.environ.get("ORACLE_WORKERS", os.cpu_count() or 1))


# ------------------------------------------------------------------ Eq. coef
def mpe_coefficients_exact(K: int) -> list:
    """Exact c_k of the K-term multi-product expansion (Section II, Eq. coef).

    c_i = prod_{j != i} k_i^2 / (k_i^2 - k_j^2) with {k_1..k_K} = {1..K}.
    Returned as ``fractions.Fraction``.
    """
    if K < 1:
        raise ValueError("K >= 1")
    out = []
    for i in range(1, K + 1):
        c = Fraction(1)
        for j in range(1, K + 1):
            if j != i:
                c *= Fraction(i * i, i * i - j * j)
        out.append(c)
    return out


def mpe_coefficients(K: int) -> np.ndarray:
    """c_k rounded to float64 (Eq. coef)."""
    return np.array([float(c) for c in mpe_coefficients_exact(K)], dtype=np.float64)


def t2_count(K: int) -> int:
    """T2 applications per state per MPE step: K(K+1)/2 (Section II, after Eq. ten)."""
    return K * (K + 1) // 2


# ------------------------------------------------------------------ grid and k-space
def _shape(grid):
    nx, ny, nz = (int(g) for g in grid)
    return nz, ny, nx


def kinetic_symbol(grid, box, hbar2_over_m: float = 1.0) -> np.ndarray:
    """(hbar^2/2m)|q|^2 on the real-to-complex half spectrum [nz][ny][nx//2+1].

    q_a = 2 pi m / L_a with m in FFT frequency order; the x axis keeps
    m = 0..nx/2 (Eq. Ham, T is diagonal in Fourier space on a periodic grid).
    """
    nx, ny, nz = (int(g) for g in grid)
    Lx, Ly, Lz = (float(b) for b in box)
    qx = 2.0 * np.pi * sfft.rfftfreq(nx, d=Lx / nx)
    qy = 2.0 * np.pi * sfft.fftfreq(ny, d=Ly / ny)
    qz = 2.0 * np.pi * sfft.fftfreq(nz, d=Lz / nz)
    q2 = qz[:, None, None] ** 2 + qy[None, :, None] ** 2 + qx[None, None, :] ** 2
    return 0.5 * hbar2_over_m * q2


def _rfft3(a):
    return sfft.rfftn(a, axes=(-3, -2, -1), workers=WORKERS)


def _irfft3(a, shape):
    return sfft.irfftn(a, s=shape, axes=(-3, -2, -1), workers=WORKERS)


# ------------------------------------------------------------------ Eq. so
def t2(psi: np.ndarray, V: np.ndarray, tau: float, grid, box, hbar2_over_m: float = 1.0,
       _ksym=None) -> np.ndarray:
    """Second-order split operator T2(epsilon) with epsilon = -tau (Section I, Eq. so).

    T2 = exp(eps V/2) exp(eps T) exp(eps V/2): a pointwise multiply, one complete
    FFT pair with the kinetic factor in between, and a second pointwise multiply.
    """
    shape = _shape(grid)
    ks = kinetic_symbol(grid, box, hbar2_over_m) if _ksym is None else _ksym
    half = np.exp(-0.5 * tau * V)
    u = half * psi
    u = _irfft3(np.exp(-tau * ks) * _rfft3(u), shape)
    return half * u


def mpe_apply(psi: np.ndarray, V: np.ndarray, dt: float, K: int, grid, box,
              hbar2_over_m: float = 1.0) -> np.ndarray:
    """Order-2K multi-product expansion sum_k c_k T2(eps/k)^k psi (Section II, Eq. mcomp).

    Each term is k successive T2 applications at step dt/k; the terms are summed
    with the (partly negative) c_k of Eq. coef pointwise on the grid, in float64.
    """
    psi = np.asarray(psi, dtype=np.float64)
    ks = kinetic_symbol(grid, box, hbar2_over_m)
    c = mpe_coefficients(K)
    acc = np.zeros_like(psi)
    for k in range(1, K + 1):
        u = psi
        for _ in range(k):
            u = t2(u, V, dt / k, grid, box, hbar2_over_m, _ksym=ks)
        acc += c[k - 1] * u
    return acc


def romberg6_apply(psi: np.ndarray, V: np.ndarray, dt: float, grid, box,
                   hbar2_over_m: float = 1.0) -> np.ndarray:
    """Romberg-type sixth-order operator built from the fourth-order one (Section II, Eq. sixp).

    T6(eps) = -T4(eps)/15 + 16 T4(eps/2)^2 / 15 with T4 the order-4 expansion
    (Eq. four): one T4 step at dt and two successive T4 steps at dt/2, i.e.
    nine T2 applications against six for the multi-product T6 (Eq. six).
    """
    psi = np.asarray(psi, dtype=np.float64)
    full = mpe_apply(psi, V, dt, 2, grid, box, hbar2_over_m)
    half = mpe_apply(psi, V, 0.5 * dt, 2, grid, box, hbar2_over_m)
    half = mpe_apply(half, V, 0.5 * dt, 2, grid, box, hbar2_over_m)
    return (-1.0 / 15.0) * full + (16.0 / 15.0) * half


def romberg6_t2_count() -> int:
    """T2 applications per state of one Romberg T6 step: three T4 steps of three each."""
    return 3 * t2_count(2)


def h_apply(psi: np.ndarray, V: np.ndarray, grid, box, hbar2_over_m: float = 1.0) -> np.ndarray:
    """H psi = -(hbar^2/2m) Lap psi + V psi with the Laplacian applied spectrally (Eq. Ham)."""
    psi = np.asarray(psi, dtype=np.float64)
    ks = kinetic_symbol(grid, box, hbar2_over_m)
    return _irfft3(ks * _rfft3(psi), _shape(grid)) + V * psi


# ------------------------------------------------------------------ Eq. ortho
def _flat(a):
    return a.reshape(a.shape[0], -1)


def overlap(Phi: np.ndarray, Psi: np.ndarray | None = None) -> np.ndarray:
    """S_ij = (Phi_i | Psi_j) = sum over grid points (discrete inner product)."""
    A = _flat(Phi)
    B = A if Psi is None else _flat(Psi)
    return A @ B.T


def cholesky_orthonormalize(Phi: np.ndarray):
    """Orthonormalise the propagated states (Section I, Eq. ortho).

    psi_j = sum_i c_ji phi_i with (psi_j|psi_i) = delta_ij, realised as a
    Cholesky QR: S = Phi^T Phi = L L^T, Psi = Phi L^{-T} (the paper names the
    subspace method only by reference; this reading is the Cholesky form).
    Returns (Psi, S, L).
    """
    S = overlap(Phi)
    L = np.linalg.cholesky(S)
    A = _flat(Phi)
    # Psi^T = L^{-1} Phi^T  (rows are states)
    Psi = sla.solve_triangular(L, A, lower=True)
    return Psi.reshape(Phi.shape), S, L


def rayleigh_ritz(Psi: np.ndarray, HPsi: np.ndarray):
    """Subspace rotation that diagonalises H in span(Psi) (Section III, subspace orthogonalisation).

    Hs = Psi^T (H Psi), symmetrised; theta, U = eigh(Hs) ascending;
    Psi <- Psi U, HPsi <- HPsi U.  Returns (theta, Psi_rot, HPsi_rot, U).
    """
    Hs = overlap(Psi, HPsi)
    Hs = 0.5 * (Hs + Hs.T)
    theta, U = np.linalg.eigh(Hs)
    P = (U.T @ _flat(Psi)).reshape(Psi.shape)
    HP = (U.T @ _flat(HPsi)).reshape(HPsi.shape)
    return theta, P, HP, U


def residual_h(Psi: np.ndarray, HPsi: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """R^H_j = sum_k |H psi_j(r_k) - E_j psi_j(r_k)|^2 (Section III; E_i read as E_j)."""
    r = _flat(HPsi) - theta[:, None] * _flat(Psi)
    return np.einsum("ij,ij->i", r, r)


def residual_e(psi_old: np.ndarray, phi: np.ndarray):
    """Variance with respect to the evolution operator (Section III, R^E).

    The paper writes exp(eps E_i); it is read as the best scalar for state j,
    mu_j = (psi_j|phi_j) with phi_j = T psi_j and psi_j normalised, so
    R^E_j = ||phi_j - mu_j psi_j||^2.  Also returned is the basis-invariant
    form R^E_perp_j = ||phi_j - Psi Psi^T phi_j||^2, which stays meaningful
    inside (near-)degenerate groups.
    """
    P = _flat(psi_old)
    F = _flat(phi)
    M = P @ F.T  # M_ij = (psi_i | phi_j)
    mu = np.diag(M)
    re = np.einsum("ij,ij->i", F - mu[:, None] * P, F - mu[:, None] * P)
    perp = F - (P.T @ M).T
    re_perp = np.einsum("ij,ij->i", perp, perp)
    return re, re_perp, mu


# ------------------------------------------------------------------ one iteration
@dataclass
class IterResult:
    psi: np.ndarray          # rotated, orthonormal Ritz vectors
    hpsi: np.ndarray         # H applied to them
    theta: np.ndarray        # Ritz values, ascending
    rh: np.ndarray           # R^H per state
    re: np.ndarray           # R^E per state (vs the incoming psi)
    re_perp: np.ndarray      # basis-invariant R^E
    phi: np.ndarray = None   # propagated states before orthonormalisation


def iterate(psi: np.ndarray, V: np.ndarray, dt: float, K: int, grid, box,
            hbar2_over_m: float = 1.0, keep_phi: bool = False, locked: int = 0,
            romberg6: bool = False) -> IterResult:
    """One iteration: propagate (Eq. propstep with Eq. mcomp), orthonormalise (Eq. ortho),
    Rayleigh-Ritz, and the variances R^E and R^H (Section III).

    ``locked``: selective propagation (Section III, only states whose variance is
    still above the bound are propagated): the locked states are taken over
    unpropagated, phi_j = psi_j, before the orthonormalisation.  An integer
    locks the first ``locked`` states, a sequence of indices locks those states.
    ``romberg6``: propagate with the Romberg-type T6 of Eq. sixp instead of the
    order-2K expansion (K is then ignored)."""
    phi = np.array(psi, dtype=np.float64, copy=True)
    act = np.ones(len(psi), dtype=bool)
    if np.ndim(locked) == 0:
        act[:int(locked)] = False
    else:
        act[np.asarray(locked, dtype=np.int64)] = False
    if act.any():
        if romberg6:
            phi[act] = romberg6_apply(psi[act], V, dt, grid, box, hbar2_over_m)
        else:
            phi[act] = mpe_apply(psi[act], V, dt, K, grid, box, hbar2_over_m)
    re, re_perp, _ = residual_e(psi, phi)
    Psi, _, _ = cholesky_orthonormalize(phi)
    HPsi = h_apply(Psi, V, grid, box, hbar2_over_m)
    theta, Psi, HPsi, _ = rayleigh_ritz(Psi, HPsi)
    rh = residual_h(Psi, HPsi, theta)
    return IterResult(Psi, HPsi, theta, rh, re, re_perp, phi if keep_phi else None)


# ------------------------------------------------------------------ driver
@dataclass
class SolveResult:
    theta: np.ndarray
    psi: np.ndarray
    rh: np.ndarray
    dt: float
    iterations: int
    levels: int
    converged: bool
    history: list = field(default_factory=list)


def solve(psi0: np.ndarray, V: np.ndarray, K: int, grid, box, n_check: int | None = None,
          dt0: float = 0.5, gamma: float = 1e-8, reduce: float = 0.5, gamma_e: float | None = None,
          max_iter_per_level: int = 2000, max_levels: int = 30, hbar2_over_m: float = 1.0,
          margin: float = 0.01) -> SolveResult:
    """Step-size protocol of Section III.

    At fixed dt, iterate until every checked state's variance with respect to the
    evolution operator is small; then evaluate R^H; stop if R^H_j < gamma for all
    checked states, otherwise multiply dt by ``reduce`` (0.5 in a realistic run,
    0.9 for the convergence figures) and restart from the current states.

    Readings: the fixed-dt test uses the basis-invariant R^E_perp against
    ``gamma_e``, default ``margin * gamma * dt^2``.  Since phi - mu psi ~
    -dt (H psi - E psi), R^E_perp / dt^2 is on the scale of the part of R^H that
    further iterations at this dt would still remove; the margin keeps that part
    well below gamma so that the R^H test afterwards measures the dt bias.  Only
    the first ``n_check`` states (default all) are tested; extra states are guard
    states.
    """
    m = psi0.shape[0]
    n_check = m if n_check is None else n_check
    psi = np.asarray(psi0, dtype=np.float64)
    dt = dt0
    hist = []
    total = 0
    for level in range(max_levels):
        ge = margin * gamma * dt * dt if gamma_e is None else gamma_e
        res = None
        for it in range(max_iter_per_level):
            res = iterate(psi, V, dt, K, grid, box, hbar2_over_m)
            psi = res.psi
            total += 1
            rep = float(np.max(res.re_perp[:n_check]))
            hist.append({"dt": dt, "it": total, "re_perp": rep,
                         "rh": float(np.max(res.rh[:n_check])), "theta0": float(res.theta[0])})
            if it > 0 and rep <= ge:
                break
        if float(np.max(res.rh[:n_check])) < gamma:
            return SolveResult(res.theta, psi, res.rh, dt, total, level + 1, True, hist)
        dt *= reduce
    return SolveResult(res.theta, psi, res.rh, dt, total, max_levels, False, hist)
