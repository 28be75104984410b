"""The allocation-free orthonormalisation (mpe_orthonormalize_noalloc, through
the C ABI) against the plan's mpe_orthonormalize on the same inputs, on two
calls in a row with the second one smaller, and against the oracle's Cholesky
orthonormalisation.  mpe_noalloc_prepare() resolves the scratch array first
(the runtime may materialise its storage then, once per GPU).

Bars: bitwise equality with the plan where both chunk the overlap alike (up to
64 * 4096 points); beyond, the float64 overlap sums are grouped differently, so
1e-12 relative (float64) and 2e-6 (float32, the float32 orthonormalisation bar);
against the oracle the same 1e-12 / 2e-6.  Device free memory is read before and
after each call: the entry point must not allocate.
"""
import ctypes as C
import sys

import numpy as np
import pytest

import workloads as W
from oracle import mpe as oracle

pytestmark = pytest.mark.gpu

PREC = {"fp64": 0, "fp32": 1}


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


def rel_err(got, ref):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


CASES = [
    ("fp64", [(40, (48, 48, 48), 1), (7, (16, 16, 32), 2)]),
    ("fp32", [(33, (64, 64, 64), 3), (5, (32, 32, 32), 4)]),
    ("fp64", [(100, (96, 96, 96), 5), (12, (32, 32, 32), 6)]),     # 884736 points: 64 chunks, not 216
    ("fp32", [(128, (64, 64, 96), 7), (1, (8, 8, 8), 8)]),
]


@pytest.mark.parametrize("prec,calls", CASES, ids=[f"{c[0]}-{c[1][0][0]}x{c[1][0][1][0]}" for c in CASES])
def test_noalloc_orthonormalize_matches_plan(P, prec, calls):
    import torch
    lib = P.lib()
    stream = torch.cuda.current_stream().cuda_stream
    assert lib.mpe_noalloc_prepare() == 0, lib.mpe_noalloc_last_error().decode()
    for m, grid, seed in calls:
        N = int(np.prod(grid))
        say("noalloc orthonormalize", prec, "m", m, "grid", grid, "points", N)
        x0 = W.random_states(seed, m, grid)
        if prec == "fp32":
            x0 = x0.astype(np.float32).astype(np.float64)
        plan = P.Plan(grid, (10.0, 10.0, 10.0), m, 2, prec)
        a = plan.new_states(x0)
        b = a.clone()
        plan.orthonormalize(a)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        code = lib.mpe_orthonormalize_noalloc(C.c_void_p(b.data_ptr()), m, N, PREC[prec], C.c_void_p(stream))
        free1 = torch.cuda.mem_get_info()[0]
        assert code == 0, lib.mpe_noalloc_last_error().decode()
        assert lib.mpe_noalloc_last_error().decode() == ""
        assert free1 == free0, (free0, free1)
        ga, gb = a.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64)
        ref, _, _ = oracle.cholesky_orthonormalize(x0)
        e_plan, e_ref = rel_err(gb, ga), rel_err(gb, ref)
        say(f"  vs plan {e_plan:.2e}  vs oracle {e_ref:.2e}")
        if N <= 64 * 4096:
            assert np.array_equal(ga, gb)
        bar = 1e-12 if prec == "fp64" else 2e-6
        assert e_plan < bar and e_ref < bar
        plan.close()


def test_noalloc_orthonormalize_errors(P):
    import torch
    lib = P.lib()
    stream = torch.cuda.current_stream().cuda_stream
    grid = (16, 16, 16)
    say("noalloc orthonormalize: limits and a rank-deficient block")
    x = torch.zeros((129, 16, 16, 16), dtype=torch.float64, device="cuda")
    code = lib.mpe_orthonormalize_noalloc(C.c_void_p(x.data_ptr()), 129, 4096, 0, C.c_void_p(stream))
    assert code == 2 and b"128" in lib.mpe_noalloc_last_error()
    code = lib.mpe_orthonormalize_noalloc(C.c_void_p(x.data_ptr()), 0, 4096, 0, C.c_void_p(stream))
    assert code == 1
    code = lib.mpe_orthonormalize_noalloc(None, 4, 4096, 0, C.c_void_p(stream))
    assert code == 1
    x0 = W.random_states(9, 5, grid)
    x0[3] = x0[1]
    t = torch.from_numpy(x0).cuda()
    before = t.cpu().numpy().copy()
    code = lib.mpe_orthonormalize_noalloc(C.c_void_p(t.data_ptr()), 5, 4096, 0, C.c_void_p(stream))
    assert code == 4, lib.mpe_noalloc_last_error().decode()
    assert b"pivot" in lib.mpe_noalloc_last_error()
    assert np.array_equal(t.cpu().numpy(), before)
