"""Float64 reference of the warm-start network -- TEST INFRASTRUCTURE ONLY.

Only ``tests/`` (and the CPU-baseline leg of the benchmark) use this module.
It defines, by plain gathers and sums, the small 3-D U-Net that maps a coarse
potential to starting orbitals, its hand-written backward pass, and the
rotation-invariant subspace loss.  The learned start is not part of the paper
(which starts from plane waves, Section III); it is an addition whose error the
solver itself judges through R^H.

Conventions (shared with the GPU implementation by specification only):
* tensors are channels-last, x[b, z, y, x, c], periodic in z, y, x;
* a convolution has 3x3x3 taps, weights W[co, tz, ty, tx, ci], bias b[co];
  y[b, o, co] = b[co] + sum_{t, ci} W[co, t, ci] x[b, s*o + t - 1, ci]  (mod D);
* architecture (channels 16/32/64, ReLU after every convolution but the head):
    e1 = relu(conv(relu(conv(v, 1->16)), 16->16))                 32^3
    e2 = relu(conv(relu(conv_s2(e1, 16->32)), 32->32))            16^3
    e3 = relu(conv(relu(conv_s2(e2, 32->64)), 64->64))             8^3
    d2 = relu(conv(concat(up(e3), e2), 96->32))                   16^3
    d1 = relu(conv(concat(up(d2), e1), 48->16))                   32^3
    y  = conv(d1, 16->n_out)                                      32^3
  with up = nearest-neighbour doubling.
* subspace loss of the prediction Y (n x P, rows = orbitals) against target
  states T (n x P, orthonormal rows): with M = Y T^T,
    L = ||Y - M T||^2 + ||M M^T - I||^2,
  zero exactly when Y = R T with R orthogonal; dL/dY = 2(Y - M T) + 4 (M M^T - I) M T.
  This loss has a stationary point at Y = 0 (its gradient vanishes with M).
* Procrustes loss (used for training): with the polar factor Q = U V^T of
  M = U Sigma V^T,  L_P = ||Y - Q T||^2, the distance from Y to the nearest
  rotation of the targets (the orthogonal Procrustes problem, for orthonormal
  T); dL_P/dY = 2 (Y - Q T) wherever M has full rank (the derivative of the
  nuclear norm of M is Q).  Its gradient never vanishes away from the minimum.
"""
from __future__ import annotations

import numpy as np

LAYERS = [  # name, ci, co, stride, relu
    ("c1a", 1, 16, 1, True), ("c1b", 16, 16, 1, True),
    ("c2a", 16, 32, 2, True), ("c2b", 32, 32, 1, True),
    ("c3a", 32, 64, 2, True), ("c3b", 64, 64, 1, True),
    ("d2", 96, 32, 1, True), ("d1", 48, 16, 1, True),
    ("head", 16, None, 1, False),
]


def init_params(seed: int, n_out: int = 120, scale: float = 1.0) -> dict:
    """He-style random weights (float64), zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, ci, co, _, _ in LAYERS:
        co = n_out if co is None else co
        std = scale * np.sqrt(2.0 / (27 * ci))
        p[name + ".w"] = rng.normal(0.0, std, (co, 3, 3, 3, ci))
        p[name + ".b"] = np.zeros(co)
    return p


def _gather_index(D_in: int, D_out: int, stride: int, t: int) -> np.ndarray:
    return (stride * np.arange(D_out) + t - 1) % D_in


def conv(x: np.ndarray, w: np.ndarray, b: np.ndarray, stride: int = 1) -> np.ndarray:
    B, D, _, _, ci = x.shape
    Do = D // stride
    co = w.shape[0]
    y = np.broadcast_to(b, (B, Do, Do, Do, co)).copy()
    for tz in range(3):
        iz = _gather_index(D, Do, stride, tz)
        for ty in range(3):
            iy = _gather_index(D, Do, stride, ty)
            for tx in range(3):
                ix = _gather_index(D, Do, stride, tx)
                g = x[:, iz][:, :, iy][:, :, :, ix]                  # B, Do, Do, Do, ci
                y += np.einsum("bzyxc,oc->bzyxo", g, w[:, tz, ty, tx, :])
    return y


def conv_backward(x, w, dy, stride=1):
    """Gradients (dx, dw, db) of conv(x, w, b, stride) for the upstream gradient dy."""
    B, D, _, _, ci = x.shape
    Do = dy.shape[1]
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    db = dy.sum(axis=(0, 1, 2, 3))
    for tz in range(3):
        iz = _gather_index(D, Do, stride, tz)
        for ty in range(3):
            iy = _gather_index(D, Do, stride, ty)
            for tx in range(3):
                ix = _gather_index(D, Do, stride, tx)
                g = x[:, iz][:, :, iy][:, :, :, ix]
                dw[:, tz, ty, tx, :] = np.einsum("bzyxo,bzyxc->oc", dy, g)
                contrib = np.einsum("bzyxo,oc->bzyxc", dy, w[:, tz, ty, tx, :])
                Z, Y, X = np.meshgrid(iz, iy, ix, indexing="ij")
                for bb in range(B):
                    np.add.at(dx[bb], (Z, Y, X), contrib[bb])
    return dx, dw, db


def up2(x):
    return x.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)


def up2_backward(dy):
    B, D, _, _, c = dy.shape
    return dy.reshape(B, D // 2, 2, D // 2, 2, D // 2, 2, c).sum(axis=(2, 4, 6))


def relu(x):
    return np.maximum(x, 0.0)


def forward(params: dict, v: np.ndarray, cache: bool = False):
    """v: [B, 32, 32, 32, 1] -> y: [B, 32, 32, 32, n_out]."""
    acts = {}

    def layer(name, x, stride, act):
        z = conv(x, params[name + ".w"], params[name + ".b"], stride)
        out = relu(z) if act else z
        acts[name] = (x, out, stride, act)
        return out

    h = layer("c1a", v, 1, True)
    e1 = layer("c1b", h, 1, True)
    h = layer("c2a", e1, 2, True)
    e2 = layer("c2b", h, 1, True)
    h = layer("c3a", e2, 2, True)
    e3 = layer("c3b", h, 1, True)
    d2 = layer("d2", np.concatenate([up2(e3), e2], axis=-1), 1, True)
    d1 = layer("d1", np.concatenate([up2(d2), e1], axis=-1), 1, True)
    y = layer("head", d1, 1, False)
    return (y, acts) if cache else y


def backward(params: dict, acts: dict, dy: np.ndarray) -> dict:
    """Gradients of every parameter given dL/dy (hand-written chain rule)."""
    g = {}

    def back(name, dout):
        x, out, stride, act = acts[name]
        dz = dout * (out > 0) if act else dout
        dx, dw, db = conv_backward(x, params[name + ".w"], dz, stride)
        g[name + ".w"], g[name + ".b"] = dw, db
        return dx

    dd1 = back("head", dy)
    dcat1 = back("d1", dd1)
    c2 = acts["d2"][1].shape[-1]
    dd2 = up2_backward(dcat1[..., :c2])
    de1 = dcat1[..., c2:]
    dcat2 = back("d2", dd2)
    c3 = acts["c3b"][1].shape[-1]
    de3 = up2_backward(dcat2[..., :c3])
    de2 = dcat2[..., c3:]
    dh = back("c3b", de3)
    de2 = de2 + back("c3a", dh)
    dh = back("c2b", de2)
    de1 = de1 + back("c2a", dh)
    dh = back("c1b", de1)
    back("c1a", dh)
    return g


def subspace_loss(Y: np.ndarray, T: np.ndarray):
    """L = ||Y - M T||^2 + ||M M^T - I||^2 with M = Y T^T; returns (L, dL/dY)."""
    M = Y @ T.T
    R1 = Y - M @ T
    G = M @ M.T - np.eye(M.shape[0])
    L = float(np.sum(R1 * R1) + np.sum(G * G))
    dY = 2.0 * R1 + 4.0 * (G @ M) @ T
    return L, dY


def procrustes_loss(Y: np.ndarray, T: np.ndarray):
    """L = ||Y - Q T||^2 with Q the polar factor of M = Y T^T; returns (L, dL/dY, sum of singular values)."""
    M = Y @ T.T
    U, sig, Vt = np.linalg.svd(M)
    Q = U @ Vt
    R = Y - Q @ T
    return float(np.sum(R * R)), 2.0 * R, float(np.sum(sig))


def orbitals_from_output(y: np.ndarray) -> np.ndarray:
    """[B, D, D, D, n] channels-last -> [B, n, D, D, D] states."""
    return np.moveaxis(y, -1, 1)


def trilinear_upsample_periodic(u: np.ndarray, factor: int) -> np.ndarray:
    """Periodic trilinear interpolation of u[..., D, D, D] onto the grid with D*factor points.

    Fine point j of an axis sits at coarse coordinate j / factor (same origin);
    the value interpolates the two neighbouring coarse samples, wrapping around.
    """
    out = u
    for ax in (-3, -2, -1):
        D = out.shape[ax]
        j = np.arange(D * factor)
        c = j / factor
        i0 = np.floor(c).astype(int)
        w = c - i0
        a = np.take(out, i0 % D, axis=ax)
        b = np.take(out, (i0 + 1) % D, axis=ax)
        shape = [1] * out.ndim
        shape[ax] = D * factor
        w = w.reshape(shape)
        out = (1.0 - w) * a + w * b
    return out


def block_average(u: np.ndarray, factor: int) -> np.ndarray:
    """Mean over factor^3 blocks of u[..., D, D, D] (coarsening of target states)."""
    *lead, D, _, _ = u.shape
    d = D // factor
    return u.reshape(*lead, d, factor, d, factor, d, factor).mean(axis=(-5, -3, -1))
