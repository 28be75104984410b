"""Pins of the float64 warm-start network reference (oracle/unet.py).

Convolutions against brute-force loops, every backward against central finite
differences, the loss against its closed-form minimum, the trilinear
up-sampling against SciPy's map_coordinates (order 1, periodic).
"""
import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import unet


def brute_conv(x, w, b, stride):
    B, D, _, _, ci = x.shape
    Do = D // stride
    co = w.shape[0]
    y = np.zeros((B, Do, Do, Do, co))
    for bb in range(B):
        for oz in range(Do):
            for oy in range(Do):
                for ox in range(Do):
                    for o in range(co):
                        s = b[o]
                        for tz in range(3):
                            for ty in range(3):
                                for tx in range(3):
                                    iz = (stride * oz + tz - 1) % D
                                    iy = (stride * oy + ty - 1) % D
                                    ix = (stride * ox + tx - 1) % D
                                    s += np.dot(w[o, tz, ty, tx], x[bb, iz, iy, ix])
                        y[bb, oz, oy, ox, o] = s
    return y


@pytest.mark.parametrize("stride", [1, 2])
def test_conv_matches_brute_force(stride):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 4, 4, 4, 3))
    w = rng.standard_normal((5, 3, 3, 3, 3))
    b = rng.standard_normal(5)
    np.testing.assert_allclose(unet.conv(x, w, b, stride), brute_conv(x, w, b, stride), atol=1e-12)


@pytest.mark.parametrize("stride", [1, 2])
def test_conv_backward_finite_differences(stride):
    rng = np.random.default_rng(2)
    x = rng.standard_normal((1, 4, 4, 4, 2))
    w = rng.standard_normal((3, 3, 3, 3, 2))
    b = rng.standard_normal(3)
    dy = rng.standard_normal(unet.conv(x, w, b, stride).shape)
    dx, dw, db = unet.conv_backward(x, w, dy, stride)
    f = lambda xx, ww, bb: float(np.sum(unet.conv(xx, ww, bb, stride) * dy))
    h = 1e-6
    for _ in range(6):
        i = tuple(rng.integers(0, s) for s in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[i] += h
        xm[i] -= h
        assert abs((f(xp, w, b) - f(xm, w, b)) / (2 * h) - dx[i]) < 1e-7
        j = tuple(rng.integers(0, s) for s in w.shape)
        wp, wm = w.copy(), w.copy()
        wp[j] += h
        wm[j] -= h
        assert abs((f(x, wp, b) - f(x, wm, b)) / (2 * h) - dw[j]) < 1e-7
    np.testing.assert_allclose(db, dy.sum(axis=(0, 1, 2, 3)))


def test_up2_adjoint():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 3, 3, 3, 4))
    y = rng.standard_normal((2, 6, 6, 6, 4))
    assert abs(np.sum(unet.up2(x) * y) - np.sum(x * unet.up2_backward(y))) < 1e-10


def test_network_backward_finite_differences():
    rng = np.random.default_rng(4)
    params = unet.init_params(5, n_out=3)
    v = rng.standard_normal((1, 8, 8, 8, 1))
    y, acts = unet.forward(params, v, cache=True)
    dy = rng.standard_normal(y.shape)
    grads = unet.backward(params, acts, dy)
    f = lambda p: float(np.sum(unet.forward(p, v) * dy))
    h = 1e-6
    checked = 0
    for name in ["c1a.w", "c2a.w", "c3b.w", "d2.w", "d1.w", "head.w", "c2b.b", "head.b"]:
        for _ in range(2):
            idx = tuple(rng.integers(0, s) for s in params[name].shape)
            pp = {k: v_.copy() for k, v_ in params.items()}
            pm = {k: v_.copy() for k, v_ in params.items()}
            pp[name][idx] += h
            pm[name][idx] -= h
            fd = (f(pp) - f(pm)) / (2 * h)
            g = grads[name][idx]
            assert abs(fd - g) <= 1e-6 * max(1.0, abs(g)), (name, idx, fd, g)
            checked += 1
    assert checked == 16


def test_subspace_loss_minimum_and_gradient():
    rng = np.random.default_rng(6)
    n, P = 5, 40
    T = np.linalg.qr(rng.standard_normal((P, n)))[0].T            # orthonormal rows
    R = np.linalg.qr(rng.standard_normal((n, n)))[0]
    L0, g0 = unet.subspace_loss(R @ T, T)
    assert L0 < 1e-24 and np.abs(g0).max() < 1e-11                 # rotated target: exact minimum
    Y = rng.standard_normal((n, P))
    L, dY = unet.subspace_loss(Y, T)
    h = 1e-6
    for _ in range(8):
        i = (rng.integers(0, n), rng.integers(0, P))
        Yp, Ym = Y.copy(), Y.copy()
        Yp[i] += h
        Ym[i] -= h
        fd = (unet.subspace_loss(Yp, T)[0] - unet.subspace_loss(Ym, T)[0]) / (2 * h)
        assert abs(fd - dY[i]) < 1e-5 * max(1.0, abs(fd))
    # invariance under rotations of the target basis
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    assert abs(unet.subspace_loss(Y, Q @ T)[0] - L) < 1e-9 * L


def test_procrustes_loss_is_the_distance_to_the_nearest_rotation():
    import scipy.linalg as sla
    rng = np.random.default_rng(9)
    n, P = 6, 50
    T = np.linalg.qr(rng.standard_normal((P, n)))[0].T
    Y = rng.standard_normal((n, P))
    L, dY, nuc = unet.procrustes_loss(Y, T)
    # SciPy solves min_R ||R A - B|| over orthogonal R (as A^T R^T = B^T): A = T, B = Y
    R, _ = sla.orthogonal_procrustes(T.T, Y.T)
    assert abs(L - np.sum((Y - R.T @ T) ** 2)) < 1e-10 * L
    for _ in range(20):                                   # no rotation does better
        Qr = np.linalg.qr(rng.standard_normal((n, n)))[0]
        assert np.sum((Y - Qr @ T) ** 2) >= L - 1e-10
    # closed form through the nuclear norm, and the special cases
    assert abs(L - (np.sum(Y * Y) + n - 2 * nuc)) < 1e-10 * L
    R0 = np.linalg.qr(rng.standard_normal((n, n)))[0]
    L0, g0, _ = unet.procrustes_loss(R0 @ T, T)
    assert L0 < 1e-24 and np.abs(g0).max() < 1e-11
    Qrot = np.linalg.qr(rng.standard_normal((n, n)))[0]
    assert abs(unet.procrustes_loss(Y, Qrot @ T)[0] - L) < 1e-10 * L
    h = 1e-6
    for _ in range(8):
        i = (rng.integers(0, n), rng.integers(0, P))
        Yp, Ym = Y.copy(), Y.copy()
        Yp[i] += h
        Ym[i] -= h
        fd = (unet.procrustes_loss(Yp, T)[0] - unet.procrustes_loss(Ym, T)[0]) / (2 * h)
        assert abs(fd - dY[i]) < 1e-5 * max(1.0, abs(fd))


def test_trilinear_upsample_matches_map_coordinates():
    rng = np.random.default_rng(7)
    u = rng.standard_normal((2, 6, 6, 6))
    f = 3
    got = unet.trilinear_upsample_periodic(u, f)
    j = np.arange(18) / f
    Z, Y, X = np.meshgrid(j, j, j, indexing="ij")
    for k in range(2):
        want = ndi.map_coordinates(u[k], [Z, Y, X], order=1, mode="grid-wrap")
        np.testing.assert_allclose(got[k], want, atol=1e-12)


def test_block_average_is_adjoint_of_repeat():
    rng = np.random.default_rng(8)
    u = rng.standard_normal((3, 8, 8, 8))
    c = rng.standard_normal((3, 4, 4, 4))
    rep = c.repeat(2, 1).repeat(2, 2).repeat(2, 3)
    assert abs(np.sum(unet.block_average(u, 2) * c) * 8 - np.sum(u * rep)) < 1e-10
