"""Seeded synthetic inputs for the MPE eigensolver.

This module is shared by the plain CPU oracle and by the GPU library's tests and
benchmarks.  It holds only the *inputs* of the method -- grid coordinates,
model potentials, molecule geometries and random starting states -- and none of
the method's arithmetic (no propagator, no transform, no orthogonalisation).

Grid convention (used by every caller): a periodic cube of side ``L`` sampled at
``n`` points per axis, ``x_j = -L/2 + j*h`` with ``h = L/n``; arrays are C-ordered
``[z][y][x]`` with x fastest.

Workloads (restated as seeded recipes, no external data):

* harmonic oscillator ``V = |r|^2/2`` (hbar = m = omega = 1);
* the "C60-like" Gaussian-well cage: 60 wells of depth ``V0`` and width ``sigma``
  centred on the vertices of a truncated icosahedron of radius ``R``;
* random molecules of Gaussian wells for the batched uneven workload;
* jittered C60-like cages for the warm-start data set;
* the paper's own cage model (Section "Quantum well model of C60"): sech wells
  -V0/cosh(|r - R_i|/d) on the same truncated-icosahedron vertices;
* plane-wave starting states (the start of the paper's convergence figures).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GOLDEN = (1.0 + math.sqrt(5.0)) / 2.0


# ----------------------------------------------------------------------------- grid
def axis(n: int, L: float) -> np.ndarray:
    """Sample points of one periodic axis: x_j = -L/2 + j*L/n, j = 0..n-1."""
    return -0.5 * L + (L / n) * np.arange(n, dtype=np.float64)


def mesh(grid, box):
    """Return (Z, Y, X) coordinate arrays of shape (nz, ny, nx); ``grid``/``box`` are (nx, ny, nz)."""
    nx, ny, nz = (int(g) for g in grid)
    Lx, Ly, Lz = (float(b) for b in box)
    z = axis(nz, Lz)[:, None, None]
    y = axis(ny, Ly)[None, :, None]
    x = axis(nx, Lx)[None, None, :]
    return np.broadcast_arrays(z, y, x)


# ----------------------------------------------------------------------------- potentials
def harmonic_potential(grid, box, omega: float = 1.0) -> np.ndarray:
    """V = omega^2 |r|^2 / 2 on the grid (hbar = m = 1), float64 [z][y][x]."""
    Z, Y, X = mesh(grid, box)
    return 0.5 * omega * omega * (X * X + Y * Y + Z * Z)


def truncated_icosahedron(radius: float = 6.7) -> np.ndarray:
    """The 60 vertices of a truncated icosahedron scaled to circumradius ``radius``.

    With edge length 2 the vertices are the even (cyclic) permutations of
    (0, +-1, +-3g), (+-1, +-(2+g), +-2g) and (+-g, +-2, +-(2g+1)) with g the golden
    ratio; the circumradius is then sqrt(9g+10).  The 2-fold axes lie along x, y, z.
    """
    g = GOLDEN
    bases = [(0.0, 1.0, 3 * g), (1.0, 2 + g, 2 * g), (g, 2.0, 2 * g + 1)]
    pts = set()
    for a, b, c in bases:
        for sa in (-1, 1):
            for sb in (-1, 1):
                for sc in (-1, 1):
                    v = (sa * a, sb * b, sc * c)
                    for p in (v, (v[1], v[2], v[0]), (v[2], v[0], v[1])):
                        pts.add(tuple(round(t, 12) for t in p))
    P = np.array(sorted(pts), dtype=np.float64)
    assert P.shape == (60, 3), P.shape
    return P * (radius / math.sqrt(9 * g + 10))


def gaussian_wells(grid, box, centers, depths, sigmas) -> np.ndarray:
    """V(r) = -sum_a V0_a exp(-|r - R_a|^2 / (2 sigma_a^2)), float64 [z][y][x].

    Wells are summed directly (no periodic images); for every workload here the
    nearest image lies > 9 sigma away, below double-precision resolution.
    """
    Z, Y, X = mesh(grid, box)
    V = np.zeros(X.shape, dtype=np.float64)
    centers = np.asarray(centers, dtype=np.float64).reshape(-1, 3)
    depths = np.broadcast_to(np.asarray(depths, dtype=np.float64), (len(centers),))
    sigmas = np.broadcast_to(np.asarray(sigmas, dtype=np.float64), (len(centers),))
    for (cx, cy, cz), v0, s in zip(centers, depths, sigmas):
        r2 = (X - cx) ** 2 + (Y - cy) ** 2 + (Z - cz) ** 2
        V -= v0 * np.exp(-r2 / (2.0 * s * s))
    return V


def sech_wells(grid, box, centers, V0: float, d: float) -> np.ndarray:
    """V(r) = -sum_i V0 / cosh(|r - R_i| / d), float64 [z][y][x] (the paper's cage model).

    Wells are summed directly (no periodic images)."""
    Z, Y, X = mesh(grid, box)
    V = np.zeros(X.shape, dtype=np.float64)
    for cx, cy, cz in np.asarray(centers, dtype=np.float64).reshape(-1, 3):
        r = np.sqrt((X - cx) ** 2 + (Y - cy) ** 2 + (Z - cz) ** 2)
        V -= V0 / np.cosh(r / d)
    return V


def sech_cage_potential(grid, box=(32.0, 32.0, 32.0), V0: float = 1.0, d: float = 0.05,
                        radius: float = 6.7) -> np.ndarray:
    """The paper's cage model: sech wells on the 60 truncated-icosahedron vertices.

    The paper prints V0 = 1 (in units of hbar^2/2m) and d = 0.05 a.u. but no cage
    radius, box or grid; the defaults here take the 6.7-bohr radius of the
    Gaussian cage and its 32-bohr box.  In these units the Hamiltonian is
    -Lap + V, i.e. hbar^2/m = 2 for the solver."""
    return sech_wells(grid, box, truncated_icosahedron(radius), V0, d)


def c60_like_potential(grid, box=(32.0, 32.0, 32.0), V0: float = 1.2, sigma: float = 0.9,
                       radius: float = 6.7, centers=None) -> np.ndarray:
    """Gaussian-well C60-like cage (60 wells on a truncated icosahedron), float64."""
    if centers is None:
        centers = truncated_icosahedron(radius)
    return gaussian_wells(grid, box, centers, V0, sigma)


# ----------------------------------------------------------------------------- states
def random_states(seed: int, count: int, grid) -> np.ndarray:
    """i.i.d. N(0,1) starting states, float64 [count][nz][ny][nx] (numpy default_rng)."""
    nx, ny, nz = (int(g) for g in grid)
    return np.random.default_rng(seed).standard_normal((count, nz, ny, nx))


def disjoint_sign_states(seed: int, count: int, grid) -> np.ndarray:
    """``count`` states, exactly orthonormal and exactly representable in float32.

    The grid points are shuffled (seeded) and dealt out in disjoint sets of 4^k
    points, 4^k the largest power of four with count * 4^k <= N; state j is
    +-2^-k (random signs) on its set and 0 elsewhere, so every inner product is
    exactly 0 or 1 in any precision.  float64 [count][nz][ny][nx].
    """
    nx, ny, nz = (int(g) for g in grid)
    N = nx * ny * nz
    k = 0
    while count * 4 ** (k + 1) <= N:
        k += 1
    if count * 4 ** k > N:
        raise ValueError("more states than grid points")
    rng = np.random.default_rng(seed)
    perm = rng.permutation(N)
    signs = rng.integers(0, 2, (count, 4 ** k)) * 2.0 - 1.0
    out = np.zeros((count, N), dtype=np.float64)
    for j in range(count):
        out[j, perm[j * 4 ** k:(j + 1) * 4 ** k]] = signs[j] * 2.0 ** (-k)
    return out.reshape(count, nz, ny, nx)


def plane_wave_states(count: int, grid, box) -> np.ndarray:
    """The ``count`` lowest real plane waves of the periodic box, float64 [count][nz][ny][nx].

    Wave vectors q = 2 pi (mx/Lx, my/Ly, mz/Lz) are taken in order of increasing
    |q|^2 (ties broken by the integer vector), one of each pair +-m, giving the
    constant state and then cos(q.r) and sin(q.r) per pair; Nyquist components
    are skipped (their sine vanishes on the grid).  Each state is normalised
    discretely: sum over grid points of psi^2 = 1."""
    nx, ny, nz = (int(g) for g in grid)
    Lx, Ly, Lz = (float(b) for b in box)
    Z, Y, X = mesh(grid, box)
    N = nx * ny * nz
    lim = [n // 2 - 1 for n in (nx, ny, nz)]
    reps = []
    for mx in range(-lim[0], lim[0] + 1):
        for my in range(-lim[1], lim[1] + 1):
            for mz in range(-lim[2], lim[2] + 1):
                m = (mx, my, mz)
                first = next((t for t in m if t != 0), 0)
                if first < 0:
                    continue            # keep one of each pair +-m
                q2 = (mx / Lx) ** 2 + (my / Ly) ** 2 + (mz / Lz) ** 2
                reps.append((q2, m))
    reps.sort()
    out = []
    for q2, (mx, my, mz) in reps:
        if len(out) >= count:
            break
        if (mx, my, mz) == (0, 0, 0):
            out.append(np.full(X.shape, 1.0 / math.sqrt(N)))
            continue
        ph = 2.0 * math.pi * (mx * (X + 0.5 * Lx) / Lx + my * (Y + 0.5 * Ly) / Ly + mz * (Z + 0.5 * Lz) / Lz)
        out.append(math.sqrt(2.0 / N) * np.cos(ph))
        if len(out) < count:
            out.append(math.sqrt(2.0 / N) * np.sin(ph))
    if len(out) < count:
        raise ValueError("grid too small for that many plane waves")
    return np.stack(out)


# ----------------------------------------------------------------------------- workloads
@dataclass
class System:
    """One independent eigenproblem: grid, box, potential and state count."""
    grid: tuple
    box: tuple
    V: np.ndarray
    n_states: int
    seed: int = 0
    meta: dict = field(default_factory=dict)


def harmonic_system(n: int = 32, L: float = 16.0, n_states: int = 10) -> System:
    """3-D isotropic oscillator on [-L/2, L/2)^3 (default 32^3 on [-8, 8)^3, 10 states)."""
    grid, box = (n, n, n), (L, L, L)
    return System(grid, box, harmonic_potential(grid, box), n_states)


def c60_system(n: int = 128, L: float = 32.0, n_states: int = 120) -> System:
    """C60-like Gaussian cage (V0 = 1.2 Ha, sigma = 0.9 bohr, radius 6.7 bohr) in a 32-bohr box."""
    grid, box = (n, n, n), (L, L, L)
    return System(grid, box, c60_like_potential(grid, box), n_states)


def random_molecule(seed: int, grids=(32, 48, 64, 96), L: float = 24.0, ball_radius: float = 5.0,
                    min_sep: float = 2.0, n_wells=(4, 40), n_states=(4, 60),
                    v0_range=(0.8, 1.5), sigma_range=(0.7, 1.1)) -> System:
    """A random Gaussian-well molecule for the batched uneven workload.

    Well count ~ U{4..40}, centres uniform in a ball of radius 5 bohr with a
    2-bohr minimum separation (rejection sampling), V0 ~ U[0.8, 1.5] Ha,
    sigma ~ U[0.7, 1.1] bohr, grid drawn from {32, 48, 64, 96} in a fixed
    24-bohr box, state count ~ U{4..60}.
    """
    rng = np.random.default_rng(seed)
    nw = int(rng.integers(n_wells[0], n_wells[1] + 1))
    centers = []
    tries = 0
    while len(centers) < nw and tries < 100000:
        tries += 1
        p = rng.uniform(-ball_radius, ball_radius, 3)
        if np.dot(p, p) > ball_radius ** 2:
            continue
        if all(np.linalg.norm(p - c) >= min_sep for c in centers):
            centers.append(p)
    centers = np.array(centers)
    v0 = rng.uniform(*v0_range, len(centers))
    sig = rng.uniform(*sigma_range, len(centers))
    n = int(rng.choice(np.asarray(grids)))
    ns = int(rng.integers(n_states[0], n_states[1] + 1))
    grid, box = (n, n, n), (L, L, L)
    V = gaussian_wells(grid, box, centers, v0, sig)
    return System(grid, box, V, ns, seed, {"centers": centers, "V0": v0, "sigma": sig})


def molecule_batch(seed: int = 0, count: int = 64, **kw):
    """``count`` independent random molecules; molecule i uses SeedSequence(seed).spawn(count)[i]."""
    children = np.random.SeedSequence(seed).spawn(count)
    return [random_molecule(int(c.generate_state(1)[0]), **kw) for c in children]


def jittered_c60_centers(seed: int, radius: float = 6.7, jitter: float = 0.2) -> tuple:
    """Cage centres with per-atom N(0, jitter^2 I) displacements and one V0 ~ U[1.0, 1.4]."""
    rng = np.random.default_rng(seed)
    c = truncated_icosahedron(radius) + rng.normal(0.0, jitter, (60, 3))
    v0 = float(rng.uniform(1.0, 1.4))
    return c, v0


def jittered_c60_potential(seed: int, grid: int, box: float = 32.0, sigma: float = 0.9) -> np.ndarray:
    """C60-like cage of jittered_c60_centers(seed) on a grid^3 mesh of the cubic box, float64."""
    centers, v0 = jittered_c60_centers(seed)
    return gaussian_wells((grid,) * 3, (box,) * 3, centers, v0, sigma)
