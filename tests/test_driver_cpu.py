"""Host logic of the solve driver (no GPU): the step-size protocol and the
selective-propagation locks, exercised on a scripted stand-in for a plan.

The stand-in returns per-iteration R^H / R^E_perp arrays from a script and
records the lock count in force at each iteration, so the tests check what the
driver asks of the plan, not any arithmetic.
"""
import numpy as np
import pytest

from paper_0809_3739_amd import solver


class ScriptedPlan:
    def __init__(self, m, n_states, script):
        self.m, self.n_states = m, n_states
        self.script = list(script)      # per iteration: (rh array, re_perp array)
        self.locked_seen = []
        self.sets_seen = []
        self.var_seen = []
        self.dts = []
        self._locked = 0
        self._var = True

    @property
    def locked(self):
        return self._locked

    def set_locked(self, n):
        assert 0 <= n <= self.m
        self._locked = n
        self.mask_seen_next = None

    def set_locked_states(self, mask):
        mask = np.asarray(mask, dtype=bool)
        assert mask.shape == (self.m,)
        self._locked = int(mask.sum())
        self.mask_seen_next = tuple(np.flatnonzero(mask))

    def set_variances(self, on):
        self._var = bool(on)

    def orthonormalize(self, psi):
        pass

    def iterate(self, psi, dt):
        self.locked_seen.append(self._locked)
        self.sets_seen.append(getattr(self, "mask_seen_next", None))
        self.var_seen.append(self._var)
        self.dts.append(dt)
        rh, rep = self.script.pop(0)
        if not self._var:
            rep = [float("nan")] * self.m
        return {"rh": np.asarray(rh, float), "re_perp": np.asarray(rep, float), "eig": np.arange(self.m, dtype=float),
                "re": np.asarray(rep, float)}


def test_locks_follow_the_leading_converged_run_and_release_at_once():
    m = 5
    big, small = 1e-3, 1e-12
    script = [
        ([small, small, big, big, big], [1.0] * m),      # 2 leading states below lock_tol
        ([small, small, small, big, small], [1.0] * m),  # 3 (state 4 does not count: not leading)
        ([small, big, small, big, big], [1.0] * m),      # state 1 rose: lock drops to 1
        ([1e-20] * m, [1.0] * m),                         # all below gamma: converged
    ]
    plan = ScriptedPlan(m, 4, script)
    r = solver.solve(plan, None, dt0=0.5, gamma=1e-10, lock_tol=1e-11, n_check=4, lock_anywhere=False)
    assert r.converged
    assert plan.locked_seen == [0, 2, 3, 1]
    assert r.propagations == 5 + 3 + 2 + 4
    assert plan.locked == 0                               # restored at the end


def test_lock_anywhere_locks_every_converged_checked_state():
    m = 5
    big, small = 1e-3, 1e-12
    script = [
        ([small, big, small, big, small], [1.0] * m),    # states 0, 2 (4 is a guard: not checked)
        ([small, small, small, big, big], [1.0] * m),    # a leading run 0..2: plain count
        ([big, small, big, small, small], [1.0] * m),    # 1 and 3, behind an unconverged state 0
        ([1e-20] * m, [1.0] * m),                         # converged
    ]
    plan = ScriptedPlan(m, 4, script)
    r = solver.solve(plan, None, dt0=0.5, gamma=1e-10, lock_tol=1e-11, n_check=4, lock_anywhere=True)
    assert r.converged
    assert plan.locked_seen == [0, 2, 3, 2]
    assert plan.sets_seen[1] == (0, 2)
    assert plan.sets_seen[3] == (1, 3)
    assert r.propagations == 5 + 3 + 2 + 3
    assert [h["below_lock"] for h in r.history] == [2, 3, 2, 4]
    assert plan.locked == 0


def test_level_ends_only_on_an_unlocked_iteration_and_locks_reset_with_dt():
    m = 3
    lo = [1e-12] * m
    script = [
        ([1e-12, 1e-3, 1e-3], [1.0] * m),      # lock 1
        ([1e-12, 1e-3, 1e-3], [0.0] * m),      # R^E test met with a lock: confirm next iteration, unlocked
        ([1e-12, 1e-3, 1e-3], [0.0] * m),      # unlocked and met: the level ends, R^H > gamma -> dt halves
        ([1e-12, 1e-3, 1e-3], [1.0] * m),      # new level starts unlocked
        (lo, [1.0] * m),                       # converged
    ]
    plan = ScriptedPlan(m, 3, script)
    r = solver.solve(plan, None, dt0=0.4, gamma=1e-10, lock_tol=1e-11, lock_anywhere=False)
    assert r.converged
    assert plan.locked_seen == [0, 1, 0, 0, 1]
    assert plan.dts == [0.4, 0.4, 0.4, 0.2, 0.2]


def test_without_lock_tol_nothing_is_locked():
    m = 3
    script = [([1e-12, 1e-3, 1e-3], [1.0] * m)] * 3 + [([1e-20] * m, [1.0] * m)]
    plan = ScriptedPlan(m, 3, script)
    r = solver.solve(plan, None, gamma=1e-10)
    assert r.converged and plan.locked_seen == [0, 0, 0, 0]
    assert r.propagations == 4 * m


def test_stall_ends_the_solve_without_convergence():
    m = 2
    script = [([1e-3, 1e-3], [1.0, 1.0])] * 40
    plan = ScriptedPlan(m, 2, script)
    r = solver.solve(plan, None, gamma=1e-10, stall_window=5)
    assert r.stalled and not r.converged
    assert r.iterations == 6


def test_slow_fall_far_above_the_floor_is_not_a_stall():
    """A max R^H falling 1 % per 20 iterations at 1e-4: without stall_below the
    20-iteration window calls it a stall; with stall_below = 1e-6 the solve goes
    on (the floor is far below), until the fall flattens near the floor."""
    m = 2
    slow = [([1e-4 * 0.9995 ** i] * m, [1.0] * m) for i in range(60)]
    near = [([5e-7] * m, [1.0] * m)] * 30
    r = solver.solve(ScriptedPlan(m, 2, slow + near), None, gamma=1e-10, stall_window=20)
    assert r.stalled and r.iterations == 21
    r = solver.solve(ScriptedPlan(m, 2, slow + near), None, gamma=1e-10, stall_window=20, stall_below=1e-6)
    assert r.stalled and r.iterations == 60 + 21          # the plateau at 5e-7 is below 1e-6


def test_flat_at_any_height_over_ten_windows_is_a_stall():
    m = 2
    script = [([1e-3, 1e-3], [1.0, 1.0])] * 80
    r = solver.solve(ScriptedPlan(m, 2, script), None, gamma=1e-10, stall_window=5, stall_below=1e-6)
    assert r.stalled and r.iterations == 51


@pytest.mark.parametrize("lock", [None, 1e-11])
def test_accept_hook_ends_the_solve(lock):
    m = 2
    script = [([1e-3, 1e-3], [1.0, 1.0])] * 10
    plan = ScriptedPlan(m, 2, script)
    r = solver.solve(plan, None, gamma=1e-10, lock_tol=lock,
                     accept=lambda out, it: {"eig": out["eig"], "rh": out["rh"]} if it == 3 else None)
    assert r.converged and r.iterations == 3


def test_variances_every_k_iterations_and_for_the_confirming_one():
    m = 3
    far, part, done = ([1e-3] * m, [1.0] * m), ([1e-12, 1e-3, 1e-3], [1.0] * m), ([1e-12, 1e-3, 1e-3], [0.0] * m)
    script = [far, part, part, done, done, ([1e-20] * m, [1.0] * m)]
    plan = ScriptedPlan(m, 3, script)
    r = solver.solve(plan, None, dt0=0.4, gamma=1e-10, lock_tol=1e-11, variance_every=3, lock_anywhere=False)
    assert r.converged
    # variances in iterations 0 and 3 by the period; 3 meets the R^E test with a lock in force, so 4
    # confirms it unlocked and with variances; the level ends there and the next starts with them
    assert plan.var_seen == [True, False, False, True, True, True]
    assert plan.locked_seen == [0, 0, 1, 1, 0, 0]
    assert plan.dts == [0.4] * 5 + [0.2]
    assert plan._var is True        # restored at the end


# ------------------------------------------------------------------ the Plan wrapper's cached H psi
class _RecordingLib:
    """Stands in for libmpe: records the entry points called, returns MPE_OK."""

    def __init__(self):
        self.calls = []

    def __getattr__(self, name):
        def call(*args):
            self.calls.append(name)
            return 0
        return call


def _plan_on_recording_lib():
    import ctypes as C
    import torch
    p = object.__new__(solver.Plan)
    p.lib = _RecordingLib()
    p.h = None
    p.m = p.n_states = 2
    p.dtype = torch.float32
    p.shape = (2, 2, 2, 2)
    p._hkey = None
    p._arr = lambda t, shape=None: C.c_void_p(t.data_ptr())
    return p


def test_plan_drops_the_cached_h_psi_when_the_block_changes_outside_the_library():
    """The library keys its kept H psi by the block's address only; the wrapper
    asks it to forget H psi when torch has written the block (its version
    counter moved) or another block comes in, and not otherwise."""
    import torch
    p = _plan_on_recording_lib()
    forgets = lambda: p.lib.calls.count("mpe_forget_cached_h")   # noqa: E731
    x = torch.zeros(p.shape)
    p.iterate(x, 0.1)                     # the library now keeps H x
    p.residuals(x, np.zeros(2))
    p.iterate(x, 0.1)
    assert forgets() == 0
    x.mul_(2.0)                           # torch writes the block in place
    p.residuals(x, np.zeros(2))
    assert forgets() == 1
    y = torch.zeros(p.shape)              # a different block
    p.iterate(y, 0.1)
    assert forgets() == 2
    p.rayleigh_ritz(y)
    p.residuals(y, np.zeros(2))
    assert forgets() == 2
    p.step(y, 0.1)                        # the library drops its H psi itself on other calls
    y.add_(1.0)
    p.iterate(y, 0.1)
    assert forgets() == 2


def test_float32_level_ends_when_rh_stops_falling():
    """Float32 plans: R^E_perp sits on its float32 floor (never below the variance
    bound), so a level ends when max R^H stops improving; the R^H test then halves dt."""
    m = 2
    plateau = [([1e-6, 1e-6], [1e-7, 1e-7])] * 25
    script = plateau + [([1e-20] * m, [1e-7] * m)]
    plan = ScriptedPlan(m, 2, script)
    plan.precision = "fp32"
    r = solver.solve(plan, None, dt0=0.4, gamma=1e-10)
    assert r.converged
    assert plan.dts == [0.4] * 21 + [0.2] * 5      # 20-iteration stall window, then halving
    plan64 = ScriptedPlan(m, 2, [([1e-6, 1e-6], [1e-7, 1e-7])] * 30 + [([1e-20] * m, [1e-7] * m)])
    r64 = solver.solve(plan64, None, dt0=0.4, gamma=1e-10, max_iter_per_level=30)
    assert plan64.dts == [0.4] * 30 + [0.2]       # float64: no stall exit, the level runs to its cap


@pytest.mark.parametrize("passes", [False, True])
def test_every_checked_state_locked_above_gamma_ends_the_stage(passes):
    """lock_tol above gamma (a float32 stage): once the first n_check states are
    all locked while max R^H is still above gamma, the next iterations would
    propagate none of them; the solve asks accept once more (final=True) and
    ends there, converged if it accepts, else stalled."""
    m = 3
    script = [
        ([2e-10, 5e-4, 1e-3], [1.0] * m),      # one leading state below lock_tol
        ([2e-10, 2.5e-10, 1e-3], [1.0] * m),   # both checked states locked, max R^H 2.5e-10 > gamma
    ] + [([2e-10, 2.5e-10, 1e-3], [1.0] * m)] * 30
    calls = []

    def accept(out, it, final=False):
        calls.append((it, final))
        return {"eig": out["eig"], "rh": np.zeros(m)} if (final and passes) else None

    plan = ScriptedPlan(m, 2, script)
    r = solver.solve(plan, None, gamma=1e-10, lock_tol=3e-10, n_check=2, stall_window=20, accept=accept,
                     lock_anywhere=False)
    assert r.iterations == 2
    assert calls == [(1, False), (2, False), (2, True)]
    assert plan.locked_seen == [0, 1]
    assert (r.converged, r.stalled) == ((True, False) if passes else (False, True))
    assert plan.locked == 0


def test_every_checked_state_locked_anywhere_ends_the_stage():
    """With converged states locked wherever they sit, the stage also ends once
    every checked state is locked, reached through a non-leading set first."""
    m = 4
    script = [
        ([5e-4, 2e-10, 1e-3, 2e-10], [1.0] * m),       # checked states 1 (and 3, a guard) below lock_tol
        ([5e-4, 2e-10, 2.5e-10, 1e-3], [1.0] * m),     # states 1, 2: a non-leading set of two
        ([2e-10, 2e-10, 2.5e-10, 1e-3], [1.0] * m),    # all three checked states locked, max 2.5e-10 > gamma
    ] + [([2e-10, 2e-10, 2.5e-10, 1e-3], [1.0] * m)] * 30
    calls = []

    def accept(out, it, final=False):
        calls.append((it, final))
        return None

    plan = ScriptedPlan(m, 3, script)
    r = solver.solve(plan, None, gamma=1e-10, lock_tol=3e-10, n_check=3, stall_window=20, accept=accept)
    assert r.iterations == 3
    assert calls == [(1, False), (2, False), (3, False), (3, True)]
    assert plan.locked_seen == [0, 1, 2]
    assert plan.sets_seen[1] == (1,) and plan.sets_seen[2] == (1, 2)
    assert (r.converged, r.stalled) == (False, True)
    assert r.propagations == 4 + 3 + 2
    assert plan.locked == 0
