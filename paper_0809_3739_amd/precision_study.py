"""Ritz values and overlap time per overlap-GEMM precision (the precision split's
GEMM variants: float64, float32 and BF16-split MFMA).

For each grid the C60-like cage (120 + 5 states, order 12, float32 plan) is
iterated 40 times from a random start; the block is then Rayleigh-Ritz rotated
once with each overlap mode and the Ritz values are compared with the
float64-MFMA ones, and three further iterations per mode time the overlap
phase with HIP events.  One JSON line per (grid, mode).

    python -m paper_0809_3739_amd.precision_study [--grids 128,192]

``--converged``: the per-state eigenvalue error of the float32 path against
float64, both converged (the precision-at-scale comparison at 192^3).  The
cage is solved to max R^H <= 1e-8 (float32 iterations, float64 finish) and
polished in float64 to max R^H <= 1e-10; that float64 block and its Ritz values
are the reference.  For each overlap mode the float32 plan then iterates from
the rounded block until its max R^H stops falling (its own fixed point at
float32 resolution), and |theta_32 - theta_64| is reported per state.

    python -m paper_0809_3739_amd.precision_study --converged [--grids 192]
"""
from __future__ import annotations

import argparse
import json

import numpy as np
import torch

import workloads as W

from . import solver

MODES = ("fp64", "fp32", "bf16x6", "bf16x3")


def run(grids=(128, 192), n_states: int = 120, n_guard: int = 5, order: int = 12, warm: int = 40, log=print):
    rows = []
    for grid in grids:
        s = W.c60_system(grid, 32.0, n_states)
        plan = solver.Plan(s.grid, s.box, n_states, order, "fp32", n_guard=n_guard)
        plan.set_potential(s.V)
        psi = plan.new_states(W.random_states(0, n_states + n_guard, s.grid))
        plan.orthonormalize(psi)
        for _ in range(warm):
            out = plan.iterate(psi, 0.5)
        ref = None
        for mode in MODES:
            plan.set_gemm_precision(mode)
            q = psi.clone()
            eig = plan.rayleigh_ritz(q)
            if ref is None:
                ref = eig.copy()
            d = np.abs(eig[:n_states] - ref[:n_states])
            q2 = psi.clone()
            plan.kernel_times()
            plan.profile(True)
            for _ in range(3):
                plan.iterate(q2, 0.5)
            torch.cuda.synchronize()
            plan.profile(False)
            kt = plan.kernel_times()
            row = {"grid": grid, "gemm": mode, "start_max_rh": float(np.max(out["rh"])),
                   "max_abs_dtheta": float(d.max()), "mean_abs_dtheta": float(d.mean()),
                   "max_rel_dtheta": float(np.max(d / np.abs(ref[:n_states]))),
                   "overlap_ms": round(kt["gram"][0] / 3, 3)}
            log(json.dumps(row))
            rows.append(row)
            del q, q2
        plan.close()
        del psi
        torch.cuda.empty_cache()
    return rows


def converged(grid: int = 192, n_states: int = 120, n_guard: int = 5, order: int = 12, dt: float = 0.5,
              max_fp32_iters: int = 80, log=print) -> dict:
    import time
    s = W.c60_system(grid, 32.0, n_states)
    m = n_states + n_guard
    p32 = solver.Plan(s.grid, s.box, n_states, order, "fp32", n_guard=n_guard)
    p64 = solver.Plan(s.grid, s.box, n_states, order, "fp64", n_guard=n_guard)
    for p in (p32, p64):
        p.set_potential(s.V)
    p32.set_gemm_precision("fp32")
    psi = p32.new_states(W.random_states(0, m, s.grid))
    t0 = time.perf_counter()
    r = solver.solve_ladder(p32, p64, psi, dt0=dt, gamma=1e-8, n_check=n_states, lock32=3e-8, lock64=1e-9,
                            callback=lambda h: log(f"  it {h['it']} dt {h['dt']} max R^H {h['rh']:.3e}")
                            if h["it"] % 50 == 0 else None)
    t_solve = time.perf_counter() - t0
    x64 = r.psi
    t1 = time.perf_counter()
    r64 = solver.solve(p64, x64, dt0=r.dt, gamma=1e-10, n_check=n_states, orthonormalize_first=False,
                       lock_tol=1e-11, max_levels=2)
    torch.cuda.synchronize()
    t_polish = time.perf_counter() - t1
    ref = np.asarray(r64.eig[:n_states])
    p64.kernel_times()
    p64.profile(True)
    p64.iterate(x64, r64.dt)
    p64.profile(False)
    kt64 = p64.kernel_times()
    out = {"study": "converged", "grid": grid, "states": m, "order": order,
           "reference": {"solve_seconds": round(t_solve, 2), "polish_seconds": round(t_polish, 2),
                         "iterations": r.iterations + r64.iterations, "stages": r.stages,
                         "max_rh_float64": float(np.max(r64.rh[:n_states])), "dt": r64.dt,
                         "float64_iteration_ms": round(sum(v[0] for v in kt64.values()), 2),
                         "eig": [float(e) for e in ref]}, "modes": []}
    scale = np.maximum(np.abs(ref), np.abs(ref).max())
    for mode in MODES:
        p32.set_gemm_precision(mode)
        x = x64.to(torch.float32)
        p32.orthonormalize(x)
        best, best_eig, hist = None, None, []
        for it in range(max_fp32_iters):
            o = p32.iterate(x, r64.dt)
            rh = float(np.max(o["rh"][:n_states]))
            hist.append(rh)
            if best is None or rh < best:
                best, best_eig = rh, o["eig"][:n_states].copy()
            if it >= 20 and min(hist[-10:]) > 0.98 * min(hist[:-10]):
                break
        d = np.abs(best_eig - ref)
        row = {"gemm": mode, "iterations": len(hist), "float32_floor_max_rh": best,
               "max_abs_dtheta": float(d.max()), "mean_abs_dtheta": float(d.mean()),
               "max_rel_dtheta": float(np.max(d / scale)), "dtheta": [float(v) for v in d]}
        log(json.dumps({k: v for k, v in row.items() if k != "dtheta"}))
        out["modes"].append(row)
        del x
    p32.close()
    p64.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--grids", default="128,192")
    ap.add_argument("--converged", action="store_true")
    a = ap.parse_args(argv)
    if a.converged:
        for g in a.grids.split(","):
            print(json.dumps(converged(int(g), log=lambda m: print(m, flush=True))), flush=True)
        return
    run(tuple(int(x) for x in a.grids.split(",")), log=lambda m: print(m, flush=True))


if __name__ == "__main__":
    main()
