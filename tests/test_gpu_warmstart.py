"""GPU parity of the warm-start network kernels (through the C ABI) against the
float64 reference network of oracle/unet.py.

Two references for the bfloat16-MFMA convolutions:

* an emulation that feeds the float64 reference the same bfloat16 roundings
  the kernels apply (every convolution operand rounded to nearest even
  bfloat16, float32 or wider accumulation).  Where the kernels round a float32
  activation and the emulation a float64 one, the two disagree by one bfloat16
  ulp for a small fraction of elements (~1e-6 relative accumulation
  difference over the 2^-8 spacing), and each disagreement perturbs the next
  layer's sums by ~2^-8 / sqrt(K), enough to tip further roundings: the
  disagreements multiply layer by layer.  With at most 512 voxels per call
  (one 8^3 sample) there are few enough elements that the results agree to
  ~1e-5 (bar 1e-3, far below any indexing mistake, which is O(1)); with more
  the cascade reaches the size of the bfloat16 error itself and the emulation
  bars become 1e-2 (output) and 0.1 (gradients).
* the exact float64 network: bfloat16 keeps 8 significant bits (unit
  roundoff u = 2^-9); each of the 9 layers rounds both operands (2u per
  product) and independent roundings add in quadrature over the sums, so the
  output's relative error by norm stays near 2u * sqrt(9) ~ 1.2e-2 (bar
  3e-2).  Parameter gradients are sums over voxels of random-sign terms gated
  by ReLU masks; where the bfloat16 and float64 forward passes disagree on a
  mask (a fraction f of the voxels) a whole term changes and the sums differ
  by about sqrt(f): a sanity bar of 0.35 for these random networks.

The losses and the up-sampling run in float64 / float32 arithmetic on float32
inputs and are held to 1e-10 (subspace loss), 1e-9 of ||y||^2 (Procrustes
loss, a difference of O(n) terms) and 2e-6 (gradients, up-sampling).
"""
import sys

import numpy as np
import pytest

from oracle import unet

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def WS():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_0809_3739_amd import warmstart
    return warmstart


def rnorm(got, ref):
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


def bf16(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def emulated_forward(p, v):
    """Reference network with every convolution operand rounded to bfloat16."""
    acts = {}

    def layer(name, x, stride, act):
        z = unet.conv(bf16(x), bf16(p[name + ".w"]), p[name + ".b"], stride)
        out = unet.relu(z) if act else z
        acts[name] = (x, out, stride, act)
        return out

    h = layer("c1a", v, 1, True)
    e1 = layer("c1b", h, 1, True)
    h = layer("c2a", e1, 2, True)
    e2 = layer("c2b", h, 1, True)
    h = layer("c3a", e2, 2, True)
    e3 = layer("c3b", h, 1, True)
    d2 = layer("d2", np.concatenate([unet.up2(e3), e2], axis=-1), 1, True)
    d1 = layer("d1", np.concatenate([unet.up2(d2), e1], axis=-1), 1, True)
    y = layer("head", d1, 1, False)
    return y, acts


def emulated_backward(p, acts, dy):
    """Reference chain rule with the kernels' bfloat16 operand roundings."""
    g = {}

    def back(name, dout):
        x, out, stride, act = acts[name]
        dz = dout * (out > 0) if act else dout
        dx, dw, _ = unet.conv_backward(bf16(x), bf16(p[name + ".w"]), bf16(dz), stride)
        g[name + ".w"], g[name + ".b"] = dw, dz.sum(axis=(0, 1, 2, 3))
        return dx

    dd1 = back("head", dy)
    dcat1 = back("d1", dd1)
    dd2 = unet.up2_backward(dcat1[..., :32])
    de1 = dcat1[..., 32:]
    dcat2 = back("d2", dd2)
    de3 = unet.up2_backward(dcat2[..., :64])
    de2 = dcat2[..., 64:]
    dh = back("c3b", de3)
    de2 = de2 + back("c3a", dh)
    dh = back("c2b", de2)
    de1 = de1 + back("c2a", dh)
    dh = back("c1b", de1)
    back("c1a", dh)
    return g


def make_case(WS, grid, n_out, batch, seed):
    import torch
    net = WS.WarmStartNet(grid=grid, n_out=n_out, max_batch=max(batch, 2), seed=seed)
    p64 = unet.init_params(seed, n_out=n_out)
    rng = np.random.default_rng(seed + 100)
    for k in p64:
        if k.endswith(".b"):
            p64[k] = 0.1 * rng.standard_normal(p64[k].shape)
    net.set_params(p64)
    p = {k: v.astype(np.float64) for k, v in net.params().items()}   # the float32 values the GPU holds
    v = rng.standard_normal((batch, grid, grid, grid)).astype(np.float32)
    return net, p, v, torch.from_numpy(v).cuda()


def emu_bar(grid, batch, kind):
    if batch * grid ** 3 <= 512:
        return 1e-3
    return 1e-2 if kind == "forward" else 0.1


@pytest.mark.parametrize("grid,n_out,batch", [(8, 24, 1), (8, 120, 1), (8, 40, 1), (8, 72, 1), (8, 104, 1),
                                              (8, 56, 1), (8, 120, 2), (8, 40, 3), (16, 8, 2), (16, 120, 1)])
def test_forward_matches_reference(WS, grid, n_out, batch):
    say("wsn forward", grid, n_out, batch)
    net, p, v, vd = make_case(WS, grid, n_out, batch, seed=grid + n_out)
    y = net.forward(vd).cpu().numpy()
    x = v.astype(np.float64)[..., None]
    ye, _ = emulated_forward(p, x)
    yx = unet.forward(p, x)
    e_emu = rnorm(y, unet.orbitals_from_output(ye))
    e_ref = rnorm(y, unet.orbitals_from_output(yx))
    say("rel err vs emulation", e_emu, "vs float64", e_ref)
    assert e_emu < emu_bar(grid, batch, "forward")
    assert e_ref < 3e-2


def test_forward_full_size_sampled(WS):
    """The training configuration (32^3, 120 orbitals, batch 4): whole output
    of the first sample against the emulation, and the batch's samples are
    independent (sample 2 alone gives the same result)."""
    import torch
    say("wsn forward 32^3 x 120, batch 4")
    net, p, v, vd = make_case(WS, 32, 120, 4, seed=7)
    y = net.forward(vd).cpu().numpy()
    ye, _ = emulated_forward(p, v[:1].astype(np.float64)[..., None])
    e = rnorm(y[:1], unet.orbitals_from_output(ye))
    say("rel err vs emulation", e)
    assert e < emu_bar(32, 1, "forward")
    y2 = net.forward(vd[2:3].contiguous()).cpu().numpy()
    assert np.array_equal(y2[0], y[2])
    y3 = net.forward(vd[2:3].contiguous(), yscale=0.125).cpu().numpy()   # a power of two: exact
    assert np.array_equal(y3[0], 0.125 * y[2])


@pytest.mark.parametrize("grid,n_out,batch", [(8, 24, 1), (8, 120, 1), (8, 8, 1), (8, 120, 2), (8, 8, 3),
                                              (16, 8, 2)])
def test_backward_matches_reference(WS, grid, n_out, batch):
    import torch
    say("wsn backward", grid, n_out, batch)
    net, p, v, vd = make_case(WS, grid, n_out, batch, seed=3 * grid + n_out)
    x = v.astype(np.float64)[..., None]
    rng = np.random.default_rng(11)
    dy = rng.standard_normal((batch, n_out, grid, grid, grid)).astype(np.float32)
    net.zero_grads()
    net.forward(vd)
    net.backward(torch.from_numpy(dy).cuda())
    g = net.grads()
    ye, acts = emulated_forward(p, x)
    dy_cl = np.moveaxis(dy.astype(np.float64), 1, -1)
    ge = emulated_backward(p, acts, dy_cl)
    _, acts_x = unet.forward(p, x, cache=True)
    gx = unet.backward(p, acts_x, dy_cl)
    worst_e, worst_x = 0.0, 0.0
    for k in ge:
        e1, e2 = rnorm(g[k], ge[k]), rnorm(g[k], gx[k])
        say(k, "vs emulation", e1, "vs float64", e2)
        worst_e, worst_x = max(worst_e, e1), max(worst_x, e2)
    assert worst_e < emu_bar(grid, batch, "gradient")
    assert worst_x < 0.35


def test_output_scale_scales_gradients(WS):
    import torch
    say("wsn output scale")
    net, p, v, vd = make_case(WS, 8, 8, 1, seed=9)
    dy = torch.from_numpy(np.random.default_rng(4).standard_normal((1, 8, 8, 8, 8)).astype(np.float32)).cuda()
    net.zero_grads()
    net.forward(vd)
    net.backward(dy)
    g1 = net.get_vector(1)
    net.zero_grads()
    net.forward(vd, yscale=0.25)
    net.backward(dy)
    g2 = net.get_vector(1)
    assert rnorm(g2.astype(np.float64), 0.25 * g1.astype(np.float64)) < 1e-6


def test_gradients_accumulate_and_adam_clears_them(WS):
    import torch
    say("wsn accumulate + adam")
    net, p, v, vd = make_case(WS, 8, 8, 1, seed=5)
    dy = torch.from_numpy(np.random.default_rng(2).standard_normal((1, 8, 8, 8, 8)).astype(np.float32)).cuda()
    net.zero_grads()
    net.forward(vd)
    net.backward(dy)
    g1 = net.get_vector(1).astype(np.float64)
    net.backward(dy)
    g2 = net.get_vector(1).astype(np.float64)
    assert rnorm(g2, 2 * g1) < 1e-5
    p0 = net.get_vector(0).astype(np.float64)
    lr, eps = 1e-3, 1e-8
    net.adam_step(lr=lr, eps=eps)
    p1 = net.get_vector(0).astype(np.float64)
    # t = 1 with zero moments: the bias-corrected step is lr * g / (|g| + eps)
    want = p0 - lr * g2 / (np.abs(g2) + eps)
    assert np.max(np.abs(p1 - want)) < 1e-6 * lr + 1e-7
    assert not net.get_vector(1).any()


@pytest.mark.parametrize("n,grid", [(24, 16), (120, 32), (5, 8)])
def test_subspace_loss_matches_reference(WS, n, grid):
    import torch
    say("wsn subspace loss", n, grid)
    P = grid ** 3
    net = WS.WarmStartNet(grid=8, n_out=8, max_batch=1, seed=0)
    rng = np.random.default_rng(n)
    T = np.ascontiguousarray(np.linalg.qr(rng.standard_normal((P, n)))[0].T, dtype=np.float32)
    Y = (rng.standard_normal((n, P)) / np.sqrt(P)).astype(np.float32)
    L, Lo, dy = net.subspace_loss(torch.from_numpy(Y).cuda(), torch.from_numpy(T).cuda())
    Lr, dyr = unet.subspace_loss(Y.astype(np.float64), T.astype(np.float64))
    M = Y.astype(np.float64) @ T.astype(np.float64).T
    G = M @ M.T - np.eye(n)
    say("loss", L, Lr)
    assert abs(L - Lr) <= 1e-10 * abs(Lr)
    assert abs(Lo - np.sum(G * G)) <= 1e-10 * abs(Lr)
    d = dy.cpu().numpy()
    assert np.max(np.abs(d - dyr)) <= 2e-6 * np.max(np.abs(dyr))
    # the exact minimum: a rotated target
    R = np.linalg.qr(rng.standard_normal((n, n)))[0]
    Yr = np.ascontiguousarray(R @ T.astype(np.float64), dtype=np.float32)
    L0, _, _ = net.subspace_loss(torch.from_numpy(Yr).cuda(), torch.from_numpy(T).cuda())
    Lr0, _ = unet.subspace_loss(Yr.astype(np.float64), T.astype(np.float64))
    assert abs(L0 - Lr0) <= 1e-9 * n


@pytest.mark.parametrize("n,grid", [(24, 16), (120, 32), (5, 8), (1, 8)])
def test_procrustes_loss_matches_reference(WS, n, grid):
    import torch
    say("wsn procrustes loss", n, grid)
    P = grid ** 3
    net = WS.WarmStartNet(grid=8, n_out=8, max_batch=1, seed=0)
    rng = np.random.default_rng(n + 1)
    T = np.ascontiguousarray(np.linalg.qr(rng.standard_normal((P, n)))[0].T, dtype=np.float32)
    Y = (rng.standard_normal((n, P)) / np.sqrt(P)).astype(np.float32)
    for case in ("random", "close"):
        if case == "close":   # near the minimum: a rotated target plus a little noise
            R = np.linalg.qr(rng.standard_normal((n, n)))[0]
            Y = np.ascontiguousarray(R @ T.astype(np.float64) + 1e-3 * rng.standard_normal((n, P)) / np.sqrt(P),
                                     dtype=np.float32)
        L, nuc, dy = net.procrustes_loss(torch.from_numpy(Y).cuda(), torch.from_numpy(T).cuda())
        Lr, dyr, nucr = unet.procrustes_loss(Y.astype(np.float64), T.astype(np.float64))
        say(case, "loss", L, Lr, "nuclear", nuc, nucr)
        # float64 throughout on float32 inputs: the loss to 1e-9 of ||y||^2 (a difference of O(n) terms)
        assert abs(L - Lr) <= 1e-9 * max(float(np.sum(Y.astype(np.float64) ** 2)), 1.0)
        assert abs(nuc - nucr) <= 1e-10 * nucr
        d = dy.cpu().numpy()
        # the float32 rotation sums n terms of size ~|y| (C rounded to float32): ~sqrt(n) eps32 |y|
        assert np.max(np.abs(d - dyr)) <= 2e-6 * np.max(np.abs(dyr)) + 2e-6 * np.max(np.abs(Y))


@pytest.mark.parametrize("C,d,f", [(3, 8, 2), (2, 6, 3), (120, 32, 4)])
def test_upsample_matches_reference(WS, C, d, f):
    import torch
    say("wsn upsample", C, d, f)
    u = np.random.default_rng(C + d).standard_normal((C, d, d, d)).astype(np.float32)
    got = WS.upsample_periodic(torch.from_numpy(u).cuda(), f).cpu().numpy()
    want = unet.trilinear_upsample_periodic(u.astype(np.float64), f)
    assert np.max(np.abs(got - want)) <= 2e-6 * np.max(np.abs(want))


def test_errors(WS):
    import torch
    say("wsn errors")
    from paper_0809_3739_amd import MpeError
    net = WS.WarmStartNet(grid=8, n_out=8, max_batch=1, seed=0)
    with pytest.raises(MpeError):
        net.backward(torch.zeros((0, 8, 8, 8, 8), device="cuda"))
    with pytest.raises(MpeError):
        net.forward(torch.zeros((2, 8, 8, 8), device="cuda"))
    y = torch.zeros((8, 512), device="cuda")
    with pytest.raises(MpeError):
        net.subspace_loss(y, y, dy=y)


def test_trained_network_gains_over_the_random_start(WS):
    """The committed network (trained on solver-converged jittered cages) against
    the plain random start on a held-out geometry: the start's residual and the
    iterations to max R^H < 1e-5 on a 64^3 grid (120 states + 8 guards, order 12,
    float32; both starts orthonormalised by the solver, same protocol)."""
    import torch
    import workloads as W
    from paper_0809_3739_amd import solver, warmstart_train as WT
    say("trained network vs random start, 64^3, seed 10003")
    grid, guards, seed = 64, 8, 10003
    net = WS.WarmStartNet(grid=32, n_out=WT.N_STATES + guards, max_batch=1)
    meta = WT.load_weights(net)
    assert meta["n_out"] == WT.N_STATES + guards
    plan = solver.Plan((grid,) * 3, (WT.BOX,) * 3, WT.N_STATES, 12, "fp32", n_guard=guards)
    plan.set_potential(W.jittered_c60_potential(seed, grid, WT.BOX))
    res = {}
    for kind in ("learned", "random"):
        if kind == "learned":
            psi = WT.learned_start(net, seed, grid, guards)
        else:
            psi = plan.new_states(W.random_states(seed, WT.N_STATES + guards, (grid,) * 3))
        q = WT.start_quality(plan, psi)
        r = solver.solve(plan, psi, gamma=1e-5, n_check=WT.N_STATES, max_iter_per_level=1500, max_levels=3)
        res[kind] = (q["max_rh"], r.iterations, r.converged, r.eig[:WT.N_STATES])
        say(kind, "start max R^H", q["max_rh"], "iterations", r.iterations, "converged", r.converged)
    assert res["learned"][2] and res["random"][2]
    assert res["learned"][0] < 1e-2 * res["random"][0]
    assert res["learned"][1] < res["random"][1]
    # both reach the same states: Ritz values err by at most R^H / gap (Kato-Temple),
    # here 1e-5 over gaps of 1e-2 Ha or more
    assert np.max(np.abs(res["learned"][3] - res["random"][3])) < 2e-3
