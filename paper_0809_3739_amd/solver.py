"""Python front end of libmpe: a Plan over torch device tensors and the
step-size protocol of Section III (host logic; every array operation runs in
the library's HIP kernels).
"""
from __future__ import annotations

import ctypes as C
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib

PRECISIONS = {"fp64": _lib.MPE_FP64, "fp32": _lib.MPE_FP32}
DTYPES = {"fp64": torch.float64, "fp32": torch.float32}


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Plan:
    """An MPE plan on the current HIP device.

    grid = (nx, ny, nz), box = (Lx, Ly, Lz); order = 2K; the state block has
    m = n_states + n_guard states, a torch tensor of shape (m, nz, ny, nx) and
    dtype float64 ("fp64") or float32 ("fp32") on the GPU.
    """

    def __init__(self, grid, box, n_states: int, order: int, precision: str = "fp64", n_guard: int = 0,
                 stream: torch.cuda.Stream | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("libmpe needs a HIP device (torch.cuda.is_available() is False)")
        self.lib = _lib.lib()
        self.grid = tuple(int(g) for g in grid)
        self.box = tuple(float(b) for b in box)
        self.n_states, self.n_guard = int(n_states), int(n_guard)
        self.m = self.n_states + self.n_guard
        self.order = int(order)
        self.precision = precision
        self.dtype = DTYPES[precision]
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        g = (C.c_int32 * 3)(*self.grid)
        b = (C.c_double * 3)(*self.box)
        h = C.c_void_p()
        code = self.lib.mpe_plan_create(C.byref(h), g, b, self.n_states, self.order, PRECISIONS[precision],
                                        self.n_guard, C.c_void_p(self.stream.cuda_stream))
        _lib.check(code)
        self.h = h
        self.shape = (self.m, self.grid[2], self.grid[1], self.grid[0])
        self._hkey = None   # (address, torch version) of the block whose H psi the library keeps

    # --------------------------------------------------------------- plumbing
    def close(self):
        if getattr(self, "h", None):
            self.lib.mpe_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, code):
        _lib.check(code, self.h)

    def _cached_h_valid_for(self, t: torch.Tensor):
        """The library keeps H psi of the last Rayleigh-Ritz / iteration block keyed by its
        address only; drop it unless ``t`` is that block, untouched by torch since."""
        if self._hkey is not None and self._hkey != (t.data_ptr(), t._version):
            self._check(self.lib.mpe_forget_cached_h(self.h))
            self._hkey = None

    def _remember_h(self, t: torch.Tensor):
        self._hkey = (t.data_ptr(), t._version)

    def _arr(self, t: torch.Tensor, shape=None):
        shape = self.shape if shape is None else shape
        if not (t.is_cuda and t.is_contiguous() and t.dtype == self.dtype and tuple(t.shape) == shape):
            raise ValueError(f"expected a contiguous {self.dtype} CUDA tensor of shape {shape}, got "
                             f"{t.dtype} {tuple(t.shape)} cuda={t.is_cuda} contiguous={t.is_contiguous()}")
        return C.c_void_p(t.data_ptr())

    def new_states(self, data=None) -> torch.Tensor:
        """A state block on the device (zeros, or a copy of ``data``)."""
        if data is None:
            return torch.zeros(self.shape, dtype=self.dtype, device="cuda")
        t = torch.as_tensor(np.ascontiguousarray(data)).to(device="cuda", dtype=self.dtype)
        return t.reshape(self.shape).contiguous()

    @property
    def workspace_bytes(self) -> int:
        return int(self.lib.mpe_workspace_bytes(self.h))

    # --------------------------------------------------------------- the C-ABI calls
    def set_potential(self, V, hbar2_over_m: float = 1.0):
        Vt = torch.as_tensor(np.ascontiguousarray(V) if isinstance(V, np.ndarray) else V)
        Vt = Vt.to(device="cuda", dtype=torch.float64).contiguous()
        if tuple(Vt.shape) != self.shape[1:]:
            raise ValueError(f"V must have shape {self.shape[1:]}")
        self._V = Vt   # keep alive until the copy has run
        self._check(self.lib.mpe_set_potential(self.h, C.c_void_p(Vt.data_ptr()), float(hbar2_over_m)))

    def step(self, psi: torch.Tensor, dt: float):
        self._hkey = None   # the library drops its H psi on every call but the three below
        self._check(self.lib.mpe_step(self.h, self._arr(psi), float(dt)))

    def apply_h(self, psi: torch.Tensor, hpsi: torch.Tensor | None = None) -> torch.Tensor:
        out = torch.empty_like(psi) if hpsi is None else hpsi
        self._hkey = None
        self._check(self.lib.mpe_apply_h(self.h, self._arr(psi), self._arr(out)))
        return out

    def orthonormalize(self, psi: torch.Tensor):
        self._hkey = None
        self._check(self.lib.mpe_orthonormalize(self.h, self._arr(psi)))

    def rayleigh_ritz(self, psi: torch.Tensor) -> np.ndarray:
        eig = np.zeros(self.m)
        self._hkey = None
        self._check(self.lib.mpe_rayleigh_ritz(self.h, self._arr(psi), _dptr(eig)))
        self._remember_h(psi)
        return eig

    def residuals(self, psi: torch.Tensor, eig, with_re: bool = False):
        eig = np.ascontiguousarray(eig, dtype=np.float64)
        rh = np.zeros(self.m)
        re = np.zeros(self.m) if with_re else None
        self._cached_h_valid_for(psi)
        self._check(self.lib.mpe_residuals(self.h, self._arr(psi), _dptr(eig), _dptr(rh),
                                           _dptr(re) if with_re else None))
        self._remember_h(psi)   # residuals leave the block and its H psi in place
        return (rh, re) if with_re else rh

    def iterate(self, psi: torch.Tensor, dt: float) -> dict:
        out = {k: np.zeros(self.m) for k in ("eig", "rh", "re", "re_perp")}
        self._cached_h_valid_for(psi)
        self._hkey = None
        self._check(self.lib.mpe_iterate(self.h, self._arr(psi), float(dt), _dptr(out["eig"]), _dptr(out["rh"]),
                                         _dptr(out["re"]), _dptr(out["re_perp"])))
        self._remember_h(psi)
        return out

    def small_dense_phases(self) -> dict:
        us = np.zeros(5)
        self._check(self.lib.mpe_small_dense_phases(self.h, _dptr(us)))
        return dict(zip(("cholesky", "reduction", "jacobi", "sort", "replay"), us.tolist()))

    @property
    def last_jacobi_sweeps(self) -> int:
        return int(self.lib.mpe_last_jacobi_sweeps(self.h))

    def set_graph(self, on: bool):
        self._check(self.lib.mpe_set_graph(self.h, 1 if on else 0))

    def set_locked(self, locked: int):
        """Leave the first ``locked`` states unpropagated in the following
        iterations (selective propagation; see mpe_set_locked)."""
        self._check(self.lib.mpe_set_locked(self.h, int(locked)))

    def set_locked_states(self, mask):
        """Leave the states where ``mask`` (m booleans) is true unpropagated in
        the following iterations, wherever they sit in the block (selective
        propagation; see mpe_set_locked_states).  None unlocks every state."""
        if mask is None:
            self._check(self.lib.mpe_set_locked_states(self.h, None))
            return
        mk = np.ascontiguousarray(np.asarray(mask, dtype=bool), dtype=np.uint8)
        if mk.shape != (self.m,):
            raise ValueError(f"mask must hold {self.m} entries")
        self._check(self.lib.mpe_set_locked_states(self.h, mk.ctypes.data_as(C.c_void_p)))

    def set_variances(self, on: bool):
        """Form R^E / R^E_perp in the following iterations (default) or skip them
        (NaN outputs, one overlap product fewer); see mpe_set_variances."""
        self._check(self.lib.mpe_set_variances(self.h, 1 if on else 0))

    def set_propagator(self, kind: str):
        """"expansion" (the plan's order-2K multi-product expansion, default) or
        "romberg6" (order-4 plans: -T4(dt)/15 + 16 T4(dt/2)^2/15, Eq. sixp)."""
        self._hkey = None
        self._check(self.lib.mpe_set_propagator(self.h, {"expansion": 0, "romberg6": 1}[kind]))

    def set_three_pass(self, on: bool):
        """Transforms as separate x, y and z passes (see mpe_set_three_pass)."""
        self._check(self.lib.mpe_set_three_pass(self.h, 1 if on else 0))

    @property
    def three_pass(self) -> bool:
        return bool(self.lib.mpe_get_three_pass(self.h) == 1)

    @property
    def propagator(self) -> str:
        return ["expansion", "romberg6"][int(self.lib.mpe_get_propagator(self.h))]

    @property
    def locked(self) -> int:
        return int(self.lib.mpe_get_locked(self.h))

    def set_states_per_launch(self, states: int):
        self._check(self.lib.mpe_set_states_per_launch(self.h, int(states)))

    def set_plane_shape(self, kernel_class: str, mode: int, blocks_per_cu: int = 0):
        """kernel_class "plane_fwd" or "plane_link"; see mpe_set_plane_shape."""
        kc = _lib.KERNEL_CLASSES.index(kernel_class)
        self._check(self.lib.mpe_set_plane_shape(self.h, kc, int(mode), int(blocks_per_cu)))

    def set_gemm_precision(self, mode: str):
        """Overlap GEMMs in "fp64" (default), "fp32", "bf16x3" or "bf16x6" MFMA
        (the last three for float32 plans; see mpe_set_gemm_precision)."""
        self._check(self.lib.mpe_set_gemm_precision(self.h, {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3}[mode]))

    def set_pencil_shape(self, tile: int):
        """Pencil work-group shape: 0 = 256 threads, 1 = 128, 2 = 512 (see mpe_set_pencil_shape)."""
        self._check(self.lib.mpe_set_pencil_shape(self.h, int(tile)))

    def plane_shape(self) -> dict:
        buf = (C.c_int32 * 4)()
        self._check(self.lib.mpe_get_plane_shape(self.h, buf))
        return {"plane_fwd": (buf[0], buf[1]), "plane_link": (buf[2], buf[3]),
                "pencil_tile": int(self.lib.mpe_get_pencil_shape(self.h))}

    def autotune(self, psi: torch.Tensor, dt: float, reps: int = 2, cache: str | None = None) -> dict:
        """Pick the fastest plane-pass shapes (mpe_autotune); ``cache`` defaults to $MPE_TUNE_CACHE."""
        import os
        cache = os.environ.get("MPE_TUNE_CACHE") if cache is None else cache
        ms = np.zeros(2)
        self._check(self.lib.mpe_autotune(self.h, self._arr(psi), float(dt), int(reps),
                                          cache.encode() if cache else None, _dptr(ms)))
        return {**self.plane_shape(), "ms_per_step": {"plane_fwd": ms[0], "plane_link": ms[1]}}

    def profile(self, on: bool = True):
        self._check(self.lib.mpe_profile_enable(self.h, 1 if on else 0))

    def kernel_times(self) -> dict:
        ms = (C.c_double * len(_lib.KERNEL_CLASSES))()
        cnt = (C.c_int64 * len(_lib.KERNEL_CLASSES))()
        self._check(self.lib.mpe_get_kernel_times(self.h, ms, cnt))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(_lib.KERNEL_CLASSES)}


class Batch:
    """Many independent systems advanced together (one order and precision).

    ``systems``: objects with ``grid``, ``box``, ``V`` (float64 [nz][ny][nx]) and
    ``n_states``; ``n_guard`` is added to every system.  State blocks are torch
    tensors, one per system, shaped (m_i, nz, ny, nx).
    """

    def __init__(self, systems, order: int, precision: str = "fp32", n_guard: int = 0,
                 hbar2_over_m: float = 1.0, stream: torch.cuda.Stream | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("libmpe needs a HIP device")
        self.lib = _lib.lib()
        self.order, self.precision, self.dtype = int(order), precision, DTYPES[precision]
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._V = [torch.as_tensor(np.ascontiguousarray(sy.V)).to("cuda", torch.float64).contiguous()
                   for sy in systems]
        descs = (_lib.SystemDesc * len(systems))()
        self.shapes = []
        for i, sy in enumerate(systems):
            d = descs[i]
            for a in range(3):
                d.grid[a] = int(sy.grid[a])
                d.box[a] = float(sy.box[a])
            d.n_states, d.n_guard = int(sy.n_states), int(n_guard)
            d.V = self._V[i].data_ptr()
            self.shapes.append((int(sy.n_states) + n_guard, int(sy.grid[2]), int(sy.grid[1]), int(sy.grid[0])))
        h = C.c_void_p()
        code = self.lib.mpe_batch_create(C.byref(h), len(systems), descs, self.order, PRECISIONS[precision],
                                         float(hbar2_over_m), C.c_void_p(self.stream.cuda_stream))
        _lib.check(code)
        self.h = h
        self.count = len(systems)
        self.m = [s[0] for s in self.shapes]

    def close(self):
        if getattr(self, "h", None):
            self.lib.mpe_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, code):
        if code != _lib.MPE_OK:
            raise _lib.MpeError(code, self.lib.mpe_batch_last_error(self.h).decode())

    def new_states(self, i: int, data=None) -> torch.Tensor:
        if data is None:
            return torch.zeros(self.shapes[i], dtype=self.dtype, device="cuda")
        return torch.as_tensor(np.ascontiguousarray(data)).to("cuda", self.dtype).reshape(self.shapes[i]).contiguous()

    def _ptrs(self, psis):
        if len(psis) != self.count:
            raise ValueError("one state block per system")
        for t, shp in zip(psis, self.shapes):
            if not (t.is_cuda and t.is_contiguous() and t.dtype == self.dtype and tuple(t.shape) == shp):
                raise ValueError(f"state block must be a contiguous {self.dtype} CUDA tensor of shape {shp}")
        return (C.c_void_p * self.count)(*[t.data_ptr() for t in psis])

    def step(self, psis, dt: float):
        self._check(self.lib.mpe_batch_step(self.h, self._ptrs(psis), float(dt)))

    def iterate(self, psis, dt: float):
        tot = sum(self.m)
        out = {k: np.zeros(tot) for k in ("eig", "rh", "re", "re_perp")}
        self._check(self.lib.mpe_batch_iterate(self.h, self._ptrs(psis), float(dt), _dptr(out["eig"]),
                                               _dptr(out["rh"]), _dptr(out["re"]), _dptr(out["re_perp"])))
        res, off = [], 0
        for mi in self.m:
            res.append({k: v[off:off + mi].copy() for k, v in out.items()})
            off += mi
        return res

    def set_batched_la(self, on: bool):
        """Per-system linear algebra as one launch per kernel for all systems (default) or per system."""
        self._check(self.lib.mpe_batch_set_batched_la(self.h, 1 if on else 0))

    @property
    def launches_per_step(self) -> int:
        return int(self.lib.mpe_batch_launches_per_step(self.h))


# ------------------------------------------------------------------ step-size protocol
@dataclass
class SolveResult:
    eig: np.ndarray
    rh: np.ndarray
    dt: float
    iterations: int
    levels: int
    converged: bool
    seconds: float
    history: list = field(default_factory=list)
    stalled: bool = False
    stages: list = field(default_factory=list)
    propagations: int = 0     # state propagations performed (fewer than iterations * m with locking)


def flat(hist: list, window: int, gain: float) -> bool:
    """True when the last ``window`` values lowered the best earlier one by less
    than the fraction ``gain`` (False while fewer than window + 1 values exist)."""
    return len(hist) > window and min(hist[-window:]) > (1.0 - gain) * min(hist[:-window])


def solve(plan: Plan, psi: torch.Tensor, dt0: float = 0.5, gamma: float = 1e-8, reduce: float = 0.5,
          n_check: int | None = None, margin: float = 0.01, max_iter_per_level: int = 2000,
          max_levels: int = 30, orthonormalize_first: bool = True, callback=None,
          stall_window: int | None = None, stall_gain: float = 0.02, accept=None,
          lock_tol: float | None = None, variance_every: int = 1, re_tol: float | None = None,
          level_stall: int | None = None, stall_below: float | None = None,
          lock_anywhere: bool = True) -> SolveResult:
    """Iterate with the protocol of Section III until R^H_j < gamma for the
    first ``n_check`` states.

    At each dt the fused iteration is repeated until the basis-invariant
    variance with respect to the evolution operator satisfies
    max_j R^E_perp_j <= margin * gamma * dt^2 (R^E_perp/dt^2 is on the scale
    of the part of R^H still removable at this dt); then R^H decides between
    stopping and dt <- reduce * dt with the current states as the new start.

    With ``stall_window`` the solve also ends (``stalled``, not converged, dt
    kept) when the last ``stall_window`` iterations of a level lowered the best
    max R^H by less than the fraction ``stall_gain``: the rounding floor of the
    plan's precision has been reached (in float32 it lies above the gamma
    that float64 reaches, and it rises as dt shrinks, so halving would not help).

    ``accept(out, iteration, final=False)``, if given, is called after every
    iteration; a non-None return {"eig", "rh"} ends the solve as converged with
    those values (an external, more accurate convergence check).

    With ``lock_tol`` the solve propagates selectively (Section III: only
    states whose variance is still above the bound need propagating): after
    each iteration the states (ascending Ritz values, among the first
    ``n_check``) with R^H_j <= lock_tol are left unpropagated in the next
    iteration; with ``lock_anywhere`` (the default) every one of those states
    is, wherever it sits (``Plan.set_locked_states``: a converged state behind
    an unconverged one is left alone too), else only the leading run of them
    (``Plan.set_locked``).  R^H is evaluated for every state in every
    iteration, so a locked state whose R^H rises again is released at once;
    locks are dropped when dt changes, and a level only ends on an iteration
    without locks, so its R^E test sees every state propagated.  When every
    one of the first ``n_check`` states is locked while max R^H is still above
    gamma (``lock_tol`` >= gamma, as in a float32 stage that hands its states
    to float64), nothing is left to propagate: ``accept`` is called once more
    with ``final=True`` and, if it declines, the solve ends as stalled.

    A level also ends when max R^H has not improved by the fraction
    ``stall_gain`` over the last ``level_stall`` iterations (default 20 for
    float32 plans, off for float64): in float32, R^E_perp carries a floor near
    1e-7 of the propagated norm (the block is orthonormal to float32 rounding
    only), above the variance bound, so the fixed point at this dt shows as R^H
    no longer falling; the R^H test then decides as after a variance-test exit.
    (With ``stall_window`` a stall ends the whole solve first.)

    With ``stall_below`` both stall tests apply only once the level's best max
    R^H is below ``stall_below``: a rounding floor lies a few gamma up, and far
    above it a slow fall is slow convergence (a small gap at the edge of the
    block), which a change of precision or dt would only make slower.  A level
    whose best max R^H has not fallen by ``stall_gain`` over ten windows counts
    as stalled at any height.

    With ``re_tol`` the fixed-dt test is max_j R^E_perp_j exp(2 dt theta_j)
    <= re_tol instead: R^E_perp relative to the propagated norm S_jj ~
    exp(-2 dt theta_j), e.g. to converge every level to its fixed point.

    With ``variance_every`` = k > 1 the variances are formed only in every k-th
    iteration of a level (and in the iteration that confirms a level's end);
    the others skip the overlap M = Psi^T Phi (``Plan.set_variances``) and
    cannot end a level.
    """
    n_check = plan.n_states if n_check is None else n_check
    if level_stall is None and getattr(plan, "precision", "fp64") == "fp32":
        level_stall = 20
    t0 = time.perf_counter()
    if orthonormalize_first:
        plan.orthonormalize(psi)
    dt = dt0
    hist = []
    total = 0
    props = 0
    out = None

    def result(eig, rh, lev, conv, stalled=False):
        r = SolveResult(eig, rh, dt, total, lev, conv, time.perf_counter() - t0, hist, stalled=stalled)
        r.propagations = props
        return r

    plan.set_locked(0)
    var_now = True
    plan.set_variances(True)
    try:
        for level in range(max_levels):
            ge = margin * gamma * dt * dt if re_tol is None else re_tol
            rh_level = []
            plan.set_locked(0)
            var_next = True
            for it in range(max_iter_per_level):
                locked = plan.locked
                if var_next != var_now:
                    plan.set_variances(var_next)
                    var_now = var_next
                out = plan.iterate(psi, dt)
                total += 1
                props += plan.m - locked
                rep = float(np.max(out["re_perp"][:n_check]))
                if re_tol is not None:
                    rep = float(np.max(out["re_perp"][:n_check] * np.exp(2.0 * dt * out["eig"][:n_check])))
                rhm = float(np.max(out["rh"][:n_check]))
                rh_level.append(rhm)
                # states this iteration leaves below the lock threshold anywhere among the
                # checked ones (without lock_anywhere only a leading run of them is locked next)
                below = 0 if lock_tol is None else int(np.count_nonzero(out["rh"][:n_check] <= lock_tol))
                hist.append({"dt": dt, "it": total, "re_perp": rep, "rh": rhm, "eig0": float(out["eig"][0]),
                             "locked": locked, "below_lock": below, "t": time.perf_counter() - t0})
                if callback:
                    callback(hist[-1])
                if accept is not None:
                    ok = accept(out, total)
                    if ok is not None:
                        return result(ok["eig"], ok["rh"], level + 1, True)
                if rhm < gamma:
                    break
                if it > 0 and rep <= ge and locked == 0:
                    break
                near_floor = stall_below is None or min(rh_level) < stall_below
                if stall_window and ((near_floor and flat(rh_level, stall_window, stall_gain))
                                     or flat(rh_level, 10 * stall_window, stall_gain)):
                    return result(out["eig"], out["rh"], level + 1, False, stalled=True)
                if level_stall and locked == 0 and ((near_floor and flat(rh_level, level_stall, stall_gain))
                                                    or flat(rh_level, 10 * level_stall, stall_gain)):
                    break
                confirm = False
                if lock_tol is not None:
                    nl = 0
                    rh = out["rh"]
                    mask = None
                    if lock_anywhere:
                        mask = np.zeros(plan.m, dtype=bool)
                        mask[:n_check] = rh[:n_check] <= lock_tol
                        nl = int(np.count_nonzero(mask))
                    else:
                        while nl < n_check and rh[nl] <= lock_tol:
                            nl += 1
                    if nl >= n_check:
                        # every checked state is locked, yet max R^H >= gamma (so lock_tol >= gamma):
                        # with nothing left to propagate among them, further iterations at this
                        # precision cannot lower it; a last external check, else the solve stalls
                        if accept is not None:
                            ok = accept(out, total, True)
                            if ok is not None:
                                return result(ok["eig"], ok["rh"], level + 1, True)
                        return result(out["eig"], out["rh"], level + 1, False, stalled=True)
                    if it > 0 and rep <= ge:
                        nl = 0   # the level may be done: confirm with every state propagated
                        confirm = True
                    if mask is not None and nl > 0:
                        plan.set_locked_states(mask)
                    else:
                        plan.set_locked(nl)
                var_next = variance_every <= 1 or confirm or (it + 1) % variance_every == 0
            if float(np.max(out["rh"][:n_check])) < gamma:
                return result(out["eig"], out["rh"], level + 1, True)
            dt *= reduce
        return result(out["eig"], out["rh"], max_levels, False)
    finally:
        plan.set_locked(0)
        plan.set_variances(True)


def solve_ladder(plan32: Plan, plan64: Plan, psi32: torch.Tensor, dt0: float = 0.5, gamma: float = 1e-8,
                 stall_window: int = 20, check_below: float = 10.0, check_every: int = 10, callback=None,
                 lock32: float | None = None, lock64: float | None = None, variance_every32: int = 10,
                 stall_below: float | None = None, **kw) -> SolveResult:
    """Float32 iterations until converged, then float64 only if needed.

    Float32 arithmetic puts a floor under the R^H it measures (the transforms'
    rounding, not the stored states: a float32 block evaluated in float64 shows
    a far smaller residual).  So once the float32 max R^H is below
    ``check_below * gamma``, every ``check_every`` iterations the block is
    converted to float64 and orthonormalised, Rayleigh-Ritz rotated and
    measured with the float64 plan; the solve ends there when that R^H is below
    gamma; once every checked state is locked in float32 (``lock32`` >= gamma)
    one such check decides at once.  If float32 stalls first, float64
    iterations continue from the converted states at the same dt until gamma.  The two plans must describe
    the same system; iterations and seconds of both stages are summed, and the
    result's ``psi`` is the float64 block.  ``lock32`` and ``lock64`` are the
    ``lock_tol`` of the two stages (selective propagation; None: every state
    is propagated); ``variance_every32`` is the float32 stage's
    ``variance_every`` (10: that stage ends by R^H, the float64 check or a
    stall, so its variances are only needed for the rare level change).
    ``stall_below`` (default 100 gamma) is the float32 stage's: its floor sits
    at a few gamma, so a slow fall far above it is slow convergence and stays
    in float32, three times cheaper per iteration than float64.
    """
    t0 = time.perf_counter()
    n_check = kw.get("n_check") or plan32.n_states
    box = {}

    def accept(out, it, final=False):
        if final and box.get("checked_at") == it:
            return None   # this iteration's block was checked already
        if not final and (it % check_every or float(np.max(out["rh"][:n_check])) >= check_below * gamma):
            return None
        box["checked_at"] = it
        psi64 = psi32.to(torch.float64)
        plan64.orthonormalize(psi64)
        eig = plan64.rayleigh_ritz(psi64)
        rh = plan64.residuals(psi64, eig)
        box["checks"] = box.get("checks", 0) + 1
        if float(np.max(rh[:n_check])) < gamma:
            box["psi"] = psi64
            return {"eig": eig, "rh": rh}
        return None

    r1 = solve(plan32, psi32, dt0=dt0, gamma=gamma, stall_window=stall_window, callback=callback, accept=accept,
               lock_tol=lock32, variance_every=variance_every32,
               stall_below=100.0 * gamma if stall_below is None else stall_below, **kw)
    stages = [{"precision": "fp32", "iterations": r1.iterations, "seconds": round(r1.seconds, 3), "dt": r1.dt,
               "float64_checks": box.get("checks", 0), "max_rh": float(np.max(r1.rh[:n_check]))}]
    if r1.converged:
        r1.stages = stages
        r1.psi = box.get("psi")
        return r1
    psi64 = psi32.to(torch.float64)
    r2 = solve(plan64, psi64, dt0=r1.dt, gamma=gamma, callback=callback, lock_tol=lock64, **kw)
    stages.append({"precision": "fp64", "iterations": r2.iterations, "seconds": round(r2.seconds, 3), "dt": r2.dt,
                   "max_rh": float(np.max(r2.rh[:n_check]))})
    r2.iterations += r1.iterations
    r2.propagations += r1.propagations
    r2.levels += r1.levels - 1
    r2.seconds = time.perf_counter() - t0
    r2.history = r1.history + r2.history
    r2.stages = stages
    r2.psi = psi64
    return r2
