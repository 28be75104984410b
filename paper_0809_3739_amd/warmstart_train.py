"""Training data, training and use of the learned warm start.

Workload (the jittered C60-like cage): 60 Gaussian wells of width 0.9 bohr on
a truncated icosahedron of radius 6.7 bohr, every atom displaced by
N(0, 0.2^2 I) bohr, one depth V0 ~ U[1.0, 1.4] Ha per molecule, periodic
box of 32 bohr.  The network sees the potential on the 32^3 grid divided by
1.2 Ha and predicts the solver's whole block on the same grid: 120 orbitals
and the guard states above them (128 in all by default).

* ``generate``: the solver itself produces the targets: each training
  geometry is solved on a finer grid (64^3, float32, 120 + guard states,
  order 12) starting from the previous geometry's converged states; the
  converged states are sampled at the 32^3 points (fine point 2i sits at
  coarse point i on both grids) and orthonormalised there.
* ``train``: Adam on the rotation-invariant subspace loss, all on the GPU
  through the ``wsn_*`` kernels.
* ``learned_start``: network output, periodic trilinear up-sampling to the
  solver's grid, seeded random guard states; the solver orthonormalises and
  then judges the start through its residual R^H.

Run ``python -m paper_0809_3739_amd.warmstart_train --help``.
"""
from __future__ import annotations

import argparse
import json
import re
import math
import os
import time

import numpy as np
import torch

import workloads as W

from . import solver
from .warmstart import WarmStartNet, upsample_periodic

BOX = 32.0
V_UNIT = 1.2          # input normalisation of the potential (Ha)
COARSE = 32
N_STATES = 120
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "wsn_c60_32.npz")


def coarse_input(seed: int, d: int = COARSE) -> torch.Tensor:
    """The network input of one geometry: V on the d^3 grid / 1.2, float32 on the GPU."""
    v = W.jittered_c60_potential(seed, d, BOX) / V_UNIT
    return torch.from_numpy(v.astype(np.float32)).cuda()


def generate(seeds, fine: int = 64, d: int = COARSE, n_guard: int = 8, order: int = 12, gamma: float = 1e-4,
             start_seed: int = 12345, log=print):
    """(inputs [N, d, d, d], targets [N, 120 + n_guard, d, d, d], per-run stats) on the GPU.

    The targets are the whole converged block: the 120 checked states and the
    guard states above them (less converged, but close to the next levels),
    so that a start built from them holds the states just above the gap too."""
    if fine % d:
        raise ValueError("the fine grid must be a multiple of the coarse one")
    step = fine // d
    plan = solver.Plan((fine,) * 3, (BOX,) * 3, N_STATES, order, "fp32", n_guard=n_guard)
    m = N_STATES + n_guard
    cplan = solver.Plan((d,) * 3, (BOX,) * 3, m, 2, "fp32")
    psi = plan.new_states(W.random_states(start_seed, N_STATES + n_guard, (fine,) * 3))
    N = len(seeds)
    X = torch.empty((N, d, d, d), dtype=torch.float32, device="cuda")
    T = torch.empty((N, m, d, d, d), dtype=torch.float32, device="cuda")
    stats = []
    t0 = time.perf_counter()
    for i, s in enumerate(seeds):
        plan.set_potential(W.jittered_c60_potential(s, fine, BOX))
        r = solver.solve(plan, psi, gamma=gamma, n_check=N_STATES, max_iter_per_level=1500, max_levels=4,
                         stall_window=60)
        t = psi[:, ::step, ::step, ::step].contiguous()
        cplan.orthonormalize(t)
        T[i].copy_(t)
        X[i].copy_(coarse_input(s, d))
        stats.append({"seed": int(s), "iterations": r.iterations, "seconds": round(r.seconds, 3),
                      "max_rh": float(np.max(r.rh[:N_STATES])), "converged": bool(r.converged),
                      "eig0": float(r.eig[0]), "eig119": float(r.eig[N_STATES - 1])})
        if i % 16 == 0 or i == N - 1:
            log(f"[data] {i + 1}/{N} seed {s}: {r.iterations} it, max R^H {stats[-1]['max_rh']:.2e}, "
                f"{time.perf_counter() - t0:.1f}s total")
    plan.close()
    cplan.close()
    return X, T, stats


def train(net: WarmStartNet, X: torch.Tensor, T: torch.Tensor, steps: int, batch: int = 4, lr: float = 1e-3,
          lr_final: float = 1e-4, seed: int = 0, log=print, log_every: int = 200, loss: str = "procrustes",
          checkpoint=None, checkpoint_every: int = 2000):
    """Adam on a rotation-invariant loss; the learning rate decays geometrically from lr to lr_final.

    ``procrustes`` (default): distance to the nearest rotation of the targets,
    whose gradient never vanishes away from the minimum; ``subspace``: the
    projection loss, which has a stationary point at y = 0 where training
    from a small random network tends to stall.
    """
    lossfn = net.procrustes_loss if loss == "procrustes" else net.subspace_loss
    N, d = int(X.shape[0]), int(X.shape[1])
    P = d ** 3
    yscale = 1.0 / math.sqrt(P)      # keeps the network's own outputs O(1) for unit-norm orbitals
    rng = np.random.default_rng(seed)
    y = torch.empty((batch, net.n_out, d, d, d), dtype=torch.float32, device="cuda")
    dy = torch.zeros_like(y)
    hist = []
    t0 = time.perf_counter()
    run = 0.0
    for it in range(steps):
        idx = rng.choice(N, size=batch, replace=False)
        v = X[torch.from_numpy(idx).cuda()].contiguous()
        net.forward(v, out=y, yscale=yscale)
        tot = 0.0
        for b in range(batch):
            L, _, _ = lossfn(y[b], T[int(idx[b])], dy=dy[b])
            tot += L
        net.backward(dy)
        rate = lr * (lr_final / lr) ** (it / max(steps - 1, 1))
        net.adam_step(lr=rate)
        run = tot / batch if it == 0 else 0.98 * run + 0.02 * tot / batch
        if it % log_every == 0 or it == steps - 1:
            hist.append({"step": it, "loss": tot / batch, "smoothed": run, "lr": rate,
                         "t": round(time.perf_counter() - t0, 2)})
            log(f"[train] step {it}: loss {tot / batch:.4f} (smoothed {run:.4f}) lr {rate:.2e}")
        if checkpoint is not None and it > 0 and it % checkpoint_every == 0:
            checkpoint(it)
    return hist


def evaluate_loss(net: WarmStartNet, X: torch.Tensor, T: torch.Tensor, loss: str = "procrustes") -> float:
    """Mean loss over a set (no gradient step)."""
    lossfn = net.procrustes_loss if loss == "procrustes" else net.subspace_loss
    d = int(X.shape[1])
    y = torch.empty((1, net.n_out, d, d, d), dtype=torch.float32, device="cuda")
    dy = torch.empty((net.n_out, d, d, d), dtype=torch.float32, device="cuda")
    tot = 0.0
    for i in range(int(X.shape[0])):
        net.forward(X[i:i + 1].contiguous(), out=y, yscale=1.0 / math.sqrt(d ** 3))
        tot += lossfn(y[0], T[i], dy=dy)[0]
    return tot / int(X.shape[0])


def learned_start(net: WarmStartNet, seed: int, grid: int, n_guard: int, dtype=torch.float32,
                  guard_seed: int = 777) -> torch.Tensor:
    """Starting block [120 + n_guard, grid^3] for the geometry of ``seed``: the
    network's orbitals (as many as it predicts, up to the block size), then
    seeded random states for the rest of the block."""
    if grid % COARSE:
        raise ValueError("the solver grid must be a multiple of 32")
    m = N_STATES + n_guard
    k = min(net.n_out, m)
    y = net.forward(coarse_input(seed)[None].contiguous())
    up = upsample_periodic(y[0, :k].contiguous(), grid // COARSE)
    psi = torch.empty((m, grid, grid, grid), dtype=dtype, device="cuda")
    psi[:k].copy_(up)
    if k < m:
        g = W.random_states(guard_seed, m - k, (grid,) * 3)
        psi[k:].copy_(torch.from_numpy(g))
    return psi


def start_quality(plan: solver.Plan, psi: torch.Tensor) -> dict:
    """Orthonormalise and Rayleigh-Ritz rotate a start in place; its max R^H and Ritz values."""
    plan.orthonormalize(psi)
    eig = plan.rayleigh_ritz(psi)
    rh = plan.residuals(psi, eig)
    return {"max_rh": float(np.max(rh[:N_STATES])), "eig": eig}


def compare_starts(net: WarmStartNet, seeds, grid: int = 128, n_guard: int = 5, order: int = 12,
                   gamma: float = 1e-8, variants=("learned_ladder_lock3_g32", "random_ladder_lock3_g32",
                                                  "random_fp64_lock", "random_fp64"), log=print, dt0: float = 0.5):
    """Iterations and seconds to max_{j<120} R^H_j < gamma from the learned and the random start.

    ``*_ladder``: float32 iterations until gamma or the float32 floor, then
    float64 (solver.solve_ladder); ``random_fp64``: float64 throughout.  The
    random start is i.i.d. N(0, 1) from the geometry's seed.  A ``_lock<f>``
    suffix adds selective propagation: states are locked once their R^H is
    below ``f * gamma`` (f = 1 when omitted) in float32 and below ``gamma / 10``
    in float64; ``_any`` after it locks every such state, not only a leading
    run of them; ``_c<x>`` after that sets the ladder's ``check_below`` (the
    float64 checks of the float32 stage start below x * gamma; 10 when omitted,
    0 leaves only the check once every state is locked).  ``_g32`` runs the float32 stage's overlaps on float32 MFMA, and
    a final ``_v<k>`` forms the float32 stage's variances only every k-th
    iteration (10 when omitted).  Every variant starts at the step ``dt0``.
    """
    box = (BOX,) * 3
    p32 = solver.Plan((grid,) * 3, box, N_STATES, order, "fp32", n_guard=n_guard)
    p64 = solver.Plan((grid,) * 3, box, N_STATES, order, "fp64", n_guard=n_guard)
    m = N_STATES + n_guard
    rows = []

    def progress(h):
        if h["it"] % 100 == 0:
            log(f"    it {h['it']} dt {h['dt']:.4f} max R^H {h['rh']:.3e}")

    tuned = False
    for s in seeds:
        V = W.jittered_c60_potential(s, grid, BOX)
        p32.set_potential(V)
        p64.set_potential(V)
        if not tuned:
            # both plans take their fastest plane-pass and pencil shapes (bitwise the same results) before
            # any timed solve; the block they are timed on is only read
            scratch = p32.new_states(W.random_states(0, m, (grid,) * 3))
            p32.autotune(scratch, dt0)
            p64.autotune(scratch.to(torch.float64), dt0)
            del scratch
            tuned = True
        row = {"seed": int(s)}
        for var in variants:
            name, ve = var, 10
            mv = re.search(r"_v(\d+)$", name)
            if mv:
                ve = int(mv.group(1))
                name = name[:mv.start()]
            g32 = name.endswith("_g32")
            name = name[:-4] if g32 else name
            cb = 10.0
            mc = re.search(r"_c(\d+(?:\.\d+)?)$", name)
            if mc:
                cb = float(mc.group(1))
                name = name[:mc.start()]
            anywhere = name.endswith("_any")
            name = name[:-4] if anywhere else name
            base, _, lf = name.partition("_lock")
            lock = "_lock" in name
            p32.set_gemm_precision("fp32" if g32 else "fp64")
            lock32, lock64 = ((float(lf) if lf else 1.0) * gamma, 0.1 * gamma) if lock else (None, None)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if base.startswith("learned"):
                psi = learned_start(net, s, grid, n_guard)
            else:
                psi = p32.new_states(W.random_states(s, m, (grid,) * 3))
            if base.endswith("fp64"):
                psi = psi.to(torch.float64)
                q = start_quality(p64, psi)
                r = solver.solve(p64, psi, dt0=dt0, gamma=gamma, n_check=N_STATES, callback=progress,
                                 lock_tol=lock64, lock_anywhere=anywhere)
            else:
                q = start_quality(p32, psi)
                r = solver.solve_ladder(p32, p64, psi, dt0=dt0, gamma=gamma, n_check=N_STATES, callback=progress,
                                        lock32=lock32, lock64=lock64, variance_every32=ve, lock_anywhere=anywhere,
                                        check_below=cb)
            torch.cuda.synchronize()
            secs = time.perf_counter() - t0
            # propagations of states that sat below the lock threshold but outside the leading run
            hs = r.history
            unlocked_below = sum(max(0, a.get("below_lock", 0) - b["locked"]) for a, b in zip(hs, hs[1:]))
            row[var] = {"start_max_rh": q["max_rh"], "first_iteration_max_rh": r.history[0]["rh"],
                        "iterations": r.iterations, "propagations": r.propagations, "seconds": round(secs, 3),
                        "propagations_below_lock_outside_leading_run": int(unlocked_below),
                        "converged": bool(r.converged), "max_rh": float(np.max(r.rh[:N_STATES])),
                        "stages": r.stages, "eig": [float(e) for e in r.eig[:N_STATES]]}
            log(f"[eval] seed {s} {var}: start R^H {q['max_rh']:.3e}, after one iteration "
                f"{r.history[0]['rh']:.3e} -> {r.iterations} it ({r.propagations} state propagations), {secs:.1f}s, "
                f"converged {r.converged}, stages {r.stages}")
            del psi
        refv = "random_fp64" if "random_fp64" in row else ("random_fp64_lock" if "random_fp64_lock" in row else None)
        if refv:
            ref = np.array(row[refv]["eig"])
            for var in variants:
                if var != refv:
                    row[var]["max_rel_eig_diff_vs_fp64"] = float(np.max(np.abs(np.array(row[var]["eig"]) - ref)
                                                                        / np.abs(ref)))
        rows.append(row)
    p32.close()
    p64.close()
    return rows


def save_weights(net: WarmStartNet, path: str = WEIGHTS, meta: dict | None = None) -> None:
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path, params=net.get_vector(0), meta=json.dumps(meta or {}))


def load_weights(net: WarmStartNet, path: str = WEIGHTS) -> dict:
    with np.load(path, allow_pickle=False) as z:
        net.set_vector(z["params"])
        return json.loads(str(z["meta"]))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--train-geometries", type=int, default=192)
    ap.add_argument("--val-geometries", type=int, default=8)
    ap.add_argument("--fine", type=int, default=64)
    ap.add_argument("--data-guards", type=int, default=8,
                    help="guard states of the training solves; the network predicts 120 + this many orbitals")
    ap.add_argument("--gamma", type=float, default=1e-4)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-final", type=float, default=1e-4)
    ap.add_argument("--loss", default="procrustes", choices=["procrustes", "subspace"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--log", default=None, help="JSON file for data and training statistics")
    ap.add_argument("--eval-seeds", type=str, default="",
                    help="comma-separated held-out seeds: compare learned and random starts (skips training "
                         "and loads --out)")
    ap.add_argument("--eval-grid", type=int, default=128)
    ap.add_argument("--guards", type=int, default=5)
    ap.add_argument("--eval-gamma", type=float, default=1e-8)
    ap.add_argument("--eval-dt0", type=float, default=0.5, help="initial step of every evaluated solve")
    ap.add_argument("--variants", default="learned_ladder_lock3_g32,random_ladder_lock3_g32,random_fp64_lock,random_fp64")
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    if a.eval_seeds:
        with np.load(a.out, allow_pickle=False) as z:
            n_out = int(json.loads(str(z["meta"])).get("n_out", N_STATES))
        net = WarmStartNet(grid=COARSE, n_out=n_out, max_batch=1)
        meta = load_weights(net, a.out)
        log(f"[eval] weights {a.out}: {meta}")
        rows = compare_starts(net, [int(x) for x in a.eval_seeds.split(",")], grid=a.eval_grid,
                              n_guard=a.guards, gamma=a.eval_gamma, variants=tuple(a.variants.split(",")), log=log,
                              dt0=a.eval_dt0)
        if a.log:
            with open(a.log, "w") as f:
                json.dump({"weights": meta, "rows": rows}, f, indent=1)
        return

    train_seeds = list(range(a.train_geometries))
    val_seeds = list(range(5000, 5000 + a.val_geometries))
    X, T, st = generate(train_seeds + val_seeds, fine=a.fine, n_guard=a.data_guards, gamma=a.gamma, log=log)
    nt = len(train_seeds)
    net = WarmStartNet(grid=COARSE, n_out=N_STATES + a.data_guards, max_batch=a.batch, seed=a.seed)
    val0 = evaluate_loss(net, X[nt:], T[nt:], a.loss)
    log(f"[train] validation loss before training {val0:.4f}")
    base_meta = {"loss": a.loss, "n_out": N_STATES + a.data_guards, "train_geometries": nt,
                 "val_geometries": a.val_geometries, "fine_grid": a.fine, "gamma": a.gamma, "batch": a.batch,
                 "lr": a.lr}

    def checkpoint(it):
        save_weights(net, a.out, {**base_meta, "steps": it, "checkpoint": True})
        log(f"[train] checkpoint at step {it}")

    hist = train(net, X[:nt], T[:nt], a.steps, batch=a.batch, lr=a.lr, lr_final=a.lr_final, seed=a.seed, log=log,
                 loss=a.loss, checkpoint=checkpoint)
    val1 = evaluate_loss(net, X[nt:], T[nt:], a.loss)
    log(f"[train] validation loss after training {val1:.4f}")
    meta = {**base_meta, "steps": a.steps, "val_loss_before": val0, "val_loss_after": val1}
    save_weights(net, a.out, meta)
    if a.log:
        with open(a.log, "w") as f:
            json.dump({"meta": meta, "data": st, "train": hist}, f, indent=1)
    log(f"[train] saved {a.out}")


if __name__ == "__main__":
    main()
