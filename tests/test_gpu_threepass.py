"""GPU parity of the three-pass transforms (x rows, y columns, z pencils as
separate passes) against the oracle, through the C ABI: grids with nx != ny,
float64 planes of 192 points, and the forced three-pass form of grids the
two-pass form also runs.

Bars as for the two-pass steps (the same transforms, one more rounding per
pass): float64 1e-12 * sum|c_k|, float32 1e-6 * sum|c_k| per step (measured
at most 2.3e-7 per unit of sum|c_k|); H 1e-12 / 5e-7 (measured 1.5e-7 in
float32); iterations 1e-10 (Ritz values) and 1e-9 (subspace) in float64; the
three-pass float32 iteration against the two-pass one 1e-6 / 1e-5 (measured
2.6e-7 / 3.1e-6).
"""
import math
import sys

import numpy as np
import pytest

import workloads as W
from oracle import dense
from oracle import mpe as oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_0809_3739_amd as P
    P.lib()
    return P


def toy_potential(grid, box):
    Z, Y, X = W.mesh(grid, box)
    L = min(box)
    return (0.5 * (X * X + Y * Y + Z * Z) * (8.0 / L) ** 2
            - 1.5 * np.exp(-((X - 0.7) ** 2 + (Y + 0.3) ** 2 + (Z - 0.4) ** 2)))


def rounded(a, prec):
    return a.astype(np.float32).astype(np.float64) if prec == "fp32" else a


def rel_err(got, ref):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def sum_abs_c(order):
    return float(sum(abs(c) for c in oracle.mpe_coefficients_exact(order // 2)))


STEP_CASES = [((48, 32, 16), (12.0, 10.0, 8.0), 3, 6, "fp64", False),
              ((32, 64, 8), (10.0, 14.0, 6.0), 2, 12, "fp32", False),
              ((16, 8, 32), (8.0, 6.0, 10.0), 3, 4, "fp64", False),
              ((8, 192, 16), (6.0, 24.0, 8.0), 2, 4, "fp32", False),
              ((192, 96, 8), (24.0, 12.0, 6.0), 2, 8, "fp64", False),
              ((192, 192, 8), (24.0, 24.0, 6.0), 2, 4, "fp64", False),     # float64 planes of 192 points
              ((64, 64, 32), (12.0, 12.0, 9.0), 3, 8, "fp64", True),        # forced on a two-pass grid
              ((128, 128, 16), (16.0, 16.0, 8.0), 2, 12, "fp32", True)]


@pytest.mark.parametrize("grid,box,m,order,prec,force", STEP_CASES,
                         ids=[f"{c[0]}-o{c[3]}-{c[4]}{'-forced' if c[5] else ''}" for c in STEP_CASES])
def test_three_pass_step_matches_oracle(P, grid, box, m, order, prec, force):
    say("three-pass step", grid, prec, "m", m, "order", order, "forced", force)
    V = toy_potential(grid, box)
    psi0 = rounded(W.random_states(27, m, grid), prec)
    plan = P.Plan(grid, box, m, order, prec)
    plan.set_potential(V)
    if force:
        assert not plan.three_pass
        plan.set_three_pass(True)
    assert plan.three_pass
    psi = plan.new_states(psi0)
    plan.step(psi, 0.3)
    got = psi.cpu().numpy().astype(np.float64)
    ref = oracle.mpe_apply(psi0, V, 0.3, order // 2, grid, box)
    err = rel_err(got, ref)
    tol = (1e-12 if prec == "fp64" else 1e-6) * sum_abs_c(order)
    say(f"  rel err {err:.2e} tol {tol:.1e}")
    assert err < tol


@pytest.mark.parametrize("grid,prec", [((48, 32, 16), "fp64"), ((96, 64, 32), "fp32"), ((192, 192, 8), "fp64")])
def test_three_pass_apply_h_matches_oracle(P, grid, prec):
    box = tuple(0.25 * g + 2.0 for g in grid)
    say("three-pass apply_h", grid, prec)
    V = toy_potential(grid, box)
    psi0 = rounded(W.random_states(6, 3, grid), prec)
    plan = P.Plan(grid, box, 3, 2, prec)
    plan.set_potential(V, hbar2_over_m=0.8)
    assert plan.three_pass
    psi = plan.new_states(psi0)
    h = plan.apply_h(psi).cpu().numpy().astype(np.float64)
    ref = oracle.h_apply(psi0, V, grid, box, hbar2_over_m=0.8)
    err = rel_err(h, ref)
    say("  rel err", err)
    assert err < (1e-12 if prec == "fp64" else 5e-7)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_three_pass_agrees_with_two_pass(P, prec):
    grid, box = (64, 64, 64), (12.0, 12.0, 12.0)
    say("three-pass against two-pass", prec)
    V = toy_potential(grid, box)
    psi0 = W.random_states(28, 5, grid)
    outs = []
    for three in (False, True):
        plan = P.Plan(grid, box, 5, 12, prec)
        plan.set_potential(V)
        plan.set_three_pass(three)
        psi = plan.new_states(psi0)
        plan.orthonormalize(psi)
        r = plan.iterate(psi, 0.4)
        outs.append((psi.cpu().numpy().astype(np.float64), r["eig"], r["rh"]))
    e = rel_err(outs[1][1], outs[0][1])
    G, R = outs[1][0].reshape(5, -1), outs[0][0].reshape(5, -1)
    proj = float(np.linalg.norm(R - (R @ G.T) @ G) / math.sqrt(5))
    say(f"  eig rel {e:.2e} subspace {proj:.2e}")
    assert e < (1e-13 if prec == "fp64" else 1e-6)
    assert proj < (1e-11 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("locked,spl", [(0, 0), (3, 2)])
def test_three_pass_iterate_matches_oracle(P, locked, spl):
    """Iterations of a three-pass plan against the oracle, also with locked states
    and launches split into groups of states (every pass then starts at a state
    offset)."""
    grid, box = (48, 32, 16), (12.0, 10.0, 8.0)
    m = 8
    say("three-pass iterate", grid, "locked", locked, "states per launch", spl)
    V = toy_potential(grid, box)
    ref0, _, _ = oracle.cholesky_orthonormalize(W.random_states(29, m, grid))
    plan = P.Plan(grid, box, m, 8, "fp64")
    plan.set_potential(V)
    plan.set_states_per_launch(spl)
    plan.set_locked(locked)
    psi = plan.new_states(ref0)
    for it in range(3):
        out = plan.iterate(psi, 0.3)
        r = oracle.iterate(ref0, V, 0.3, 4, grid, box, locked=locked)
        ref0 = r.psi
        e = float(np.max(np.abs(out["eig"] - r.theta)) / np.max(np.abs(r.theta)))
        G = psi.cpu().numpy().reshape(m, -1)
        R = r.psi.reshape(m, -1)
        proj = float(np.linalg.norm(R - (R @ G.T) @ G) / math.sqrt(m))
        say(f"  it {it} eig rel {e:.2e} subspace {proj:.2e}")
        assert e < 1e-10 and proj < 1e-9
        assert np.max(np.abs(out["re_perp"][:locked]), initial=0.0) < 1e-13   # locked: phi_j = psi_j
        np.testing.assert_allclose(out["re_perp"][locked:], r.re_perp[locked:], rtol=1e-8, atol=1e-16)


def test_three_pass_solves_noncubic_oscillator(P):
    """The oscillator on a 48 x 32 x 32 grid (h = 0.5 on every axis; nx != ny, so three
    passes): exact levels are sums of the 1-D dense levels of each axis; 1.5, 2.5 x3,
    3.5 x6 to grid accuracy."""
    grid, box = (48, 32, 32), (24.0, 16.0, 16.0)
    say("three-pass oscillator", grid)
    V = W.harmonic_potential(grid, box)
    e1 = []
    for n, L in zip(grid, box):
        x = W.axis(n, L)
        e1.append(np.linalg.eigvalsh(dense.kinetic_1d(n, L) + np.diag(0.5 * x * x))[:6])
    exact = np.sort((e1[2][:, None, None] + e1[1][None, :, None] + e1[0][None, None, :]).ravel())[:10]
    plan = P.Plan(grid, box, 10, 4, "fp64")
    plan.set_potential(V)
    assert plan.three_pass
    psi = plan.new_states(W.random_states(1, 10, grid))
    res = P.solve(plan, psi, dt0=0.1, gamma=1e-10)
    err = float(np.max(np.abs(res.eig[:10] - exact) / exact))
    say("  iterations", res.iterations, "levels", res.levels, "eig rel err", err)
    assert res.converged and err < 1e-10
    assert abs(exact[0] - 1.5) < 1e-9


@pytest.mark.timeout(600)
def test_fp64_192_step_sampled(P):
    """The 192^3 cage in float64 (three passes per transform): one order-12 step of
    120 states in the precision-at-scale launch configuration, one sampled state
    against the oracle."""
    s = W.c60_system(192, 32.0, 120)
    m = 120
    say("192^3 float64 step", m)
    plan = P.Plan(s.grid, s.box, 120, 12, "fp64")
    plan.set_potential(s.V)
    assert plan.three_pass
    x0 = W.random_states(3, m, s.grid)
    psi = plan.new_states(x0)
    plan.step(psi, 0.5)
    j = 101
    got = psi[j:j + 1].cpu().numpy()
    ref = oracle.mpe_apply(x0[j:j + 1], s.V, 0.5, 6, s.grid, s.box)
    err = rel_err(got, ref)
    tol = 1e-12 * sum_abs_c(12)
    say(f"  state {j} rel err {err:.3e} tol {tol:.1e}")
    assert err < tol


def test_batch_refuses_three_pass_grids(P):
    sy = W.random_molecule(3, grids=(32,), n_states=(4, 4))
    sy.grid = (48, 32, 32)
    sy.V = np.zeros((32, 32, 48))
    say("batch with a three-pass grid")
    with pytest.raises(P.MpeError) as ei:
        P.Batch([sy], 4, "fp32")
    assert ei.value.name == "MPE_ERR_UNSUPPORTED"
