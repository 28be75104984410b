"""Time to convergence against the order of the expansion (the single-processor
comparison of the Parallelization section, which found the 6th order fastest:
the T2 applications per step grow as K(K+1)/2 while the step size that
reaches a given error grows with the order).

For each order 2K the C60-like cage is solved from the same random start with
the step-size protocol of Section III (``solver.solve``: dt0, halving after
the per-step variance test) to max_{j < n} R^H_j <= gamma, and the seconds,
iterations, levels, final dt, state propagations and T2 applications per state
are reported, one JSON line per order.  The order "r6" is the Romberg-type
sixth-order operator of Eq. sixp built from the order-4 expansion
(-T4(dt)/15 + 16 T4(dt/2)^2/15, nine T2 applications per state and step),
which Section II contrasts with the expansion's six at order 6.

    python -m paper_0809_3739_amd.order_study [--grid 64] [--orders 2,4,6,8,10,12,r6]
        [--precision fp64] [--states 120] [--guards 5] [--gamma 1e-8] [--lock]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np
import torch

import workloads as W

from . import solver


def t2_per_step(order) -> int:
    if order == "r6":
        return 9
    K = int(order) // 2
    return K * (K + 1) // 2


def run(grid: int = 64, orders=(2, 4, 6, 8, 10, 12), precision: str = "fp64", n_states: int = 120,
        n_guard: int = 5, gamma: float = 1e-8, dt0: float = 0.5, lock: bool = False, seed: int = 3,
        max_levels: int = 12, log=print) -> list:
    s = W.c60_system(grid, 32.0, n_states)
    m = n_states + n_guard
    rows = []
    for order in orders:
        plan = solver.Plan(s.grid, s.box, n_states, 4 if order == "r6" else int(order), precision, n_guard=n_guard)
        plan.set_potential(s.V)
        if order == "r6":
            plan.set_propagator("romberg6")
        psi = plan.new_states(W.random_states(seed, m, s.grid))
        last = [time.perf_counter()]

        def progress(h):
            if time.perf_counter() - last[0] > 20:
                last[0] = time.perf_counter()
                log(f"  order {order}: it {h['it']} dt {h['dt']:.5f} max R^H {h['rh']:.3e}")

        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = solver.solve(plan, psi, dt0=dt0, gamma=gamma, n_check=n_states, max_levels=max_levels,
                         callback=progress, lock_tol=0.1 * gamma if lock else None)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        row = {"order": order, "grid": grid, "precision": precision, "states": m, "seconds": round(secs, 3),
               "iterations": r.iterations, "levels": r.levels, "final_dt": r.dt, "converged": bool(r.converged),
               "max_rh": float(np.max(r.rh[:n_states])), "state_propagations": r.propagations,
               "t2_per_state": int(r.propagations * t2_per_step(order) / m), "t2_per_step": t2_per_step(order),
               "lock": lock,
               "eig0": float(r.eig[0]), "eig_last": float(r.eig[n_states - 1])}
        log(json.dumps(row))
        rows.append(row)
        plan.close()
        del psi
        torch.cuda.empty_cache()
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--grid", type=int, default=64)
    ap.add_argument("--orders", default="2,4,6,8,10,12")
    ap.add_argument("--precision", default="fp64", choices=["fp32", "fp64"])
    ap.add_argument("--states", type=int, default=120)
    ap.add_argument("--guards", type=int, default=5)
    ap.add_argument("--gamma", type=float, default=1e-8)
    ap.add_argument("--dt0", type=float, default=0.5)
    ap.add_argument("--lock", action="store_true", help="selective propagation at gamma/10")
    ap.add_argument("--max-levels", type=int, default=12)
    a = ap.parse_args(argv)
    run(a.grid, tuple(x if x == "r6" else int(x) for x in a.orders.split(",")), a.precision, a.states, a.guards,
        a.gamma, a.dt0,
        a.lock, max_levels=a.max_levels, log=lambda msg: print(msg, flush=True))


if __name__ == "__main__":
    main()
