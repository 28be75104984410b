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

    def set_variances(self, on):
        self._var = bool(on)

    def orthonormalize(self, psi):
        pass

    def iterate(self, psi, dt):
        self.locked_seen.append(self._locked)
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
    r = solver.solve(plan, None, dt0=0.5, gamma=1e-10, lock_tol=1e-11, n_check=4)
    assert r.converged
    assert plan.locked_seen == [0, 2, 3, 1]
    assert r.propagations == 5 + 3 + 2 + 4
    assert plan.locked == 0                               # restored at the end


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
    r = solver.solve(plan, None, dt0=0.4, gamma=1e-10, lock_tol=1e-11)
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
    r = solver.solve(plan, None, dt0=0.4, gamma=1e-10, lock_tol=1e-11, variance_every=3)
    assert r.converged
    # variances in iterations 0 and 3 by the period; 3 meets the R^E test with a lock in force, so 4
    # confirms it unlocked and with variances; the level ends there and the next starts with them
    assert plan.var_seen == [True, False, False, True, True, True]
    assert plan.locked_seen == [0, 0, 1, 1, 0, 0]
    assert plan.dts == [0.4] * 5 + [0.2]
    assert plan._var is True        # restored at the end
