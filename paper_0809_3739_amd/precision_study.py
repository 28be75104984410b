"""Ritz values and overlap time per overlap-GEMM precision (the precision split's
GEMM variants: float64, float32 and BF16-split MFMA).

For each grid the C60-like cage (120 + 5 states, order 12, float32 plan) is
iterated 40 times from a random start; the block is then Rayleigh-Ritz rotated
once with each overlap mode and the Ritz values are compared with the
float64-MFMA ones, and three further iterations per mode time the overlap
phase with HIP events.  One JSON line per (grid, mode).

    python -m paper_0809_3739_amd.precision_study [--grids 128,192]
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


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--grids", default="128,192")
    a = ap.parse_args(argv)
    run(tuple(int(x) for x in a.grids.split(",")), log=lambda m: print(m, flush=True))


if __name__ == "__main__":
    main()
