"""Achievable peaks of the GPU, as context for the roofline fractions: HBM
bandwidth of a plain copy kernel and the dense GEMM rate of the vendor BLAS in
float64, float32 and bfloat16 (square products, operands resident in HBM,
timed with HIP events after a warm-up).  One JSON line.

    python -m paper_0809_3739_amd.peaks
"""
from __future__ import annotations

import json

import torch


def _time(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps * 1e-3


def run() -> dict:
    out = {}
    n = (2 << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    t = _time(lambda: dst.copy_(src), 10)
    out["copy_GBps"] = round(2 * n * 4 / t / 1e9, 1)
    t = _time(lambda: torch.neg(src, out=dst), 10)   # an elementwise kernel: one read and one write
    out["neg_GBps"] = round(2 * n * 4 / t / 1e9, 1)
    del src, dst
    torch.backends.cuda.matmul.allow_tf32 = False
    for name, dt, size in (("fp64", torch.float64, 8192), ("fp32", torch.float32, 8192), ("bf16", torch.bfloat16, 16384)):
        x = torch.randn(size, size, device="cuda").to(dt)
        y = torch.randn(size, size, device="cuda").to(dt)
        t = _time(lambda: torch.matmul(x, y), 5)
        out[f"gemm_{name}_TFLOPs"] = round(2 * size ** 3 / t / 1e12, 1)
        del x, y
    torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    print(json.dumps(run()))
