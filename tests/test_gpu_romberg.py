"""GPU parity of the Romberg-type T6 propagator (Section II, Eq. sixp) against the
oracle, through the C ABI (mpe_set_propagator on an order-4 plan).

Bars: one Romberg step is three order-4 steps and a float64 combination with
weights -1/15 and 16/15, so its rounding is that of three order-4 steps times
17/15: float64 3 * 1e-12 * sum|c_k| (sum|c_k| = 5/3 for order 4); float32
3 * 1e-6 * sum|c_k| (the intermediate T4(dt/2) block is stored in float32 once
more; measured 7.0e-7 against the bar 5e-6).  Iterations: as the expansion's
iterations (1e-10 / 1e-9 float64, 1e-6 / 1.5e-6 float32 Ritz values /
subspace; measured 1.1e-7 / 4.1e-7).
"""
import math
import sys

import numpy as np
import pytest

import workloads as W
from oracle import dense
from oracle import mpe as oracle

pytestmark = pytest.mark.gpu

SUM_C4 = 5.0 / 3.0


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


STEP_CASES = [((32, 32, 32), (16.0, 16.0, 16.0), 3, "fp64", 0.3),
              ((64, 64, 32), (12.0, 12.0, 9.0), 2, "fp32", 0.5),
              ((128, 128, 8), (16.0, 16.0, 8.0), 2, "fp64", 0.4),     # float64 split tail
              ((48, 48, 16), (12.0, 12.0, 8.0), 3, "fp32", 0.25)]


@pytest.mark.parametrize("grid,box,m,prec,dt", STEP_CASES, ids=[f"{c[0]}-{c[3]}" for c in STEP_CASES])
def test_romberg6_step_matches_oracle(P, grid, box, m, prec, dt):
    say("romberg6 step", grid, prec, "m", m, "dt", dt)
    V = toy_potential(grid, box)
    psi0 = rounded(W.random_states(19, m, grid), prec)
    plan = P.Plan(grid, box, m, 4, prec)
    plan.set_potential(V)
    plan.set_propagator("romberg6")
    assert plan.propagator == "romberg6"
    psi = plan.new_states(psi0)
    plan.step(psi, dt)
    got = psi.cpu().numpy().astype(np.float64)
    ref = oracle.romberg6_apply(psi0, V, dt, grid, box)
    err = rel_err(got, ref)
    tol = 3 * (1e-12 if prec == "fp64" else 1e-6) * SUM_C4
    # the expansion's T4 of the same plan is a different operator
    off = rel_err(oracle.mpe_apply(psi0, V, dt, 2, grid, box), ref)
    say(f"  rel err {err:.2e} tol {tol:.1e}; T4 differs by {off:.2e}")
    assert err < tol and off > 100 * err


@pytest.mark.parametrize("prec,locked", [("fp64", 0), ("fp64", 3), ("fp32", 0)])
def test_romberg6_iterate_matches_oracle(P, prec, locked):
    grid, box = (32, 32, 32), (12.0, 12.0, 12.0)
    m = 8
    say("romberg6 iterate", prec, "locked", locked)
    V = toy_potential(grid, box)
    ref0, _, _ = oracle.cholesky_orthonormalize(rounded(W.random_states(23, m, grid), prec))
    ref0 = rounded(ref0, prec)
    plan = P.Plan(grid, box, m, 4, prec)
    plan.set_potential(V)
    plan.set_propagator("romberg6")
    plan.set_locked(locked)
    psi = plan.new_states(ref0)
    out = plan.iterate(psi, 0.3)
    r = oracle.iterate(ref0, V, 0.3, 2, grid, box, locked=locked, romberg6=True)
    e = float(np.max(np.abs(out["eig"] - r.theta)) / np.max(np.abs(r.theta)))
    G = psi.cpu().numpy().astype(np.float64).reshape(m, -1)
    R = r.psi.reshape(m, -1)
    proj = float(np.linalg.norm(R - (R @ G.T) @ G) / math.sqrt(m))
    say(f"  eig rel {e:.2e} subspace {proj:.2e}")
    if prec == "fp64":
        assert e < 1e-10 and proj < 1e-9
        np.testing.assert_allclose(out["re_perp"][locked:], r.re_perp[locked:], rtol=1e-8, atol=1e-16)
    else:
        assert e < 1e-6 and proj < 1.5e-6


def test_romberg6_graph_replay_matches_eager(P):
    grid, box = (32, 32, 32), (12.0, 12.0, 12.0)
    say("romberg6 graph replay vs eager")
    V = toy_potential(grid, box)
    psi0 = W.random_states(4, 6, grid)
    runs = []
    for graph in (False, True):
        plan = P.Plan(grid, box, 6, 4, "fp64")
        plan.set_potential(V)
        plan.set_propagator("romberg6")
        plan.set_graph(graph)
        psi = plan.new_states(psi0)
        plan.orthonormalize(psi)
        outs = []
        for dt in (0.3, 0.3, 0.15, 0.3):
            r = plan.iterate(psi, dt)
            outs.append((psi.cpu().numpy().copy(), r["eig"].copy(), r["rh"].copy()))
        runs.append(outs)
    for a, b in zip(*runs):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def test_romberg6_needs_order4_and_switches_back(P):
    grid, box = (16, 16, 16), (8.0, 8.0, 8.0)
    say("romberg6 plan checks")
    V = toy_potential(grid, box)
    p6 = P.Plan(grid, box, 2, 6, "fp64")
    with pytest.raises(P.MpeError) as ei:
        p6.set_propagator("romberg6")
    assert ei.value.name == "MPE_ERR_UNSUPPORTED"
    plan = P.Plan(grid, box, 2, 4, "fp64")
    plan.set_potential(V)
    x0 = W.random_states(3, 2, grid)
    a = plan.new_states(x0)
    plan.step(a, 0.2)
    plan.set_propagator("romberg6")
    plan.set_propagator("expansion")
    b = plan.new_states(x0)
    plan.step(b, 0.2)
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())


def test_romberg6_solves_oscillator_to_exact_levels(P):
    s = W.harmonic_system(32, 16.0, 10)
    say("romberg6 solve oscillator")
    plan = P.Plan(s.grid, s.box, 10, 4, "fp64")
    plan.set_potential(s.V)
    plan.set_propagator("romberg6")
    psi = plan.new_states(W.random_states(1, 10, s.grid))
    res = P.solve(plan, psi, dt0=0.1, gamma=1e-10)
    exact = dense.separable_oscillator_levels(32, 16.0, 10)
    err = float(np.max(np.abs(res.eig[:10] - exact) / exact))
    say("  iterations", res.iterations, "levels", res.levels, "dt", res.dt, "eig rel err", err)
    assert res.converged and err < 1e-10
