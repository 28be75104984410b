"""Each convolution of the warm-start network alone, at its training shape
(batch 4, the real channel counts, 32^3 / 16^3 / 8^3), through wsn_layer: the
forward output, the pre-activation gradient, the data gradient and the weight
and bias gradients against the float64 reference of oracle/unet.py.

Checked one layer at a time, there is no cascade of rounding differences
through the network, so the bars are those of one layer:

* against the reference fed the kernels' bfloat16 operand roundings (inputs,
  weights and output gradients rounded to nearest-even bfloat16; the bias
  gradient sums the float32 output gradient): the two differ only in the order
  and width of their accumulations (float32 on the GPU, float64 here):
  measured <= 4.1e-7 relative by norm on MI355X; bar 2e-6 per tensor;
* against the exact float64 layer: bfloat16 keeps 8 significant bits (unit
  roundoff 2^-9); each product rounds both operands and independent roundings
  add in quadrature, so the relative error by norm is ~sqrt(2/3) 2^-9 = 2.3e-3
  (measured 2.3e-3 to 2.4e-3); bar 5e-3 per tensor (the bias gradient, a plain
  float32 sum, 2e-6).

The backward uses the GPU forward's own ReLU mask (the pre-activation gradient
is the output gradient times [y > 0], compared exactly), so each gradient is
checked on its own inputs.
"""
import sys

import numpy as np
import pytest

from oracle import unet

pytestmark = pytest.mark.gpu

# layer index, input grid of its training shape
LAYERS = [(0, 32), (1, 32), (2, 32), (3, 16), (4, 16), (5, 8), (6, 16), (7, 32), (8, 32)]
NAMES = ["c1a", "c1b", "c2a", "c2b", "c3a", "c3b", "d2", "d1", "head"]


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def rnorm(got, ref):
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


def bf16(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.fixture(scope="module")
def net():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_0809_3739_amd import warmstart
    n = warmstart.WarmStartNet(grid=32, n_out=128, max_batch=4, seed=5)
    p64 = unet.init_params(5, n_out=128)
    rng = np.random.default_rng(55)
    for k in p64:
        if k.endswith(".b"):
            p64[k] = 0.1 * rng.standard_normal(p64[k].shape)
    n.set_params(p64)
    return n


@pytest.mark.timeout(600)
@pytest.mark.parametrize("li,d", LAYERS, ids=NAMES)
def test_layer_matches_reference(net, li, d):
    import torch
    info = net.layer_info(li)
    ci, co, cp, s, act = info["ci"], info["co"], info["ci_pad"], info["stride"], info["relu"]
    B, do = 4, d // info["stride"]
    name = NAMES[li]
    say("wsn layer", name, "input", (B, d, d, d, ci), "output", (B, do, do, do, co), "stride", s)
    p = {k: v.astype(np.float64) for k, v in net.params().items()}
    W, b = p[name + ".w"], p[name + ".b"]
    rng = np.random.default_rng(100 + li)
    x = np.zeros((B, d, d, d, cp), np.float32)
    x[..., :ci] = rng.standard_normal((B, d, d, d, ci))
    g = rng.standard_normal((B, do, do, do, co)).astype(np.float32)
    net.zero_grads()
    dz_t = torch.from_numpy(g.copy()).cuda()
    y_t, dx_t = net.layer(li, torch.from_numpy(x).cuda(), dz_t, want_dx=True)
    y, dz, dx = y_t.cpu().numpy(), dz_t.cpu().numpy(), dx_t.cpu().numpy()
    gr = net.grads()
    dW, db = gr[name + ".w"], gr[name + ".b"]

    x64 = x[..., :ci].astype(np.float64)
    z_emu = unet.conv(bf16(x64), bf16(W), b, s)
    z_ref = unet.conv(x64, W, b, s)
    y_emu = unet.relu(z_emu) if act else z_emu
    y_ref = unet.relu(z_ref) if act else z_ref
    dz_ref = g.astype(np.float64) * (y > 0) if act else g.astype(np.float64)
    assert np.array_equal(dz.astype(np.float64), dz_ref.astype(np.float32).astype(np.float64))
    dx_emu, dW_emu, _ = unet.conv_backward(bf16(x64), bf16(W), bf16(dz_ref), s)
    dx_ex, dW_ex, db_ex = unet.conv_backward(x64, W, dz_ref, s)
    errs = {"y": (rnorm(y, y_emu), rnorm(y, y_ref)), "dx": (rnorm(dx, dx_emu), rnorm(dx, dx_ex)),
            "dW": (rnorm(dW, dW_emu), rnorm(dW, dW_ex)), "db": (rnorm(db, db_ex), rnorm(db, db_ex))}
    for k, (e1, e2) in errs.items():
        say(f"  {k}: vs bf16 emulation {e1:.2e}  vs float64 {e2:.2e}")
    for k, (e1, e2) in errs.items():
        assert e1 < 2e-6, (k, e1)
        assert e2 < 5e-3, (k, e2)
