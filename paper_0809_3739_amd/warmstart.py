"""Learned warm start: a 3-D U-Net from a coarse potential to starting orbitals.

Thin wrappers over the ``wsn_*`` calls of ``include/mpe.h`` (every array
operation runs in the library's HIP kernels; torch supplies device memory).
The paper starts its iterations from random or plane-wave states (Section
III); this network is an addition whose output the solver judges through its
own residual R^H, so a poor prediction costs iterations, never correctness.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib

# name, ci, co (None = n_out), stride -- the layer order of the parameter vector
LAYERS = [
    ("c1a", 1, 16, 1), ("c1b", 16, 16, 1), ("c2a", 16, 32, 2), ("c2b", 32, 32, 1),
    ("c3a", 32, 64, 2), ("c3b", 64, 64, 1), ("d2", 96, 32, 1), ("d1", 48, 16, 1),
    ("head", 16, None, 1),
]


def _ptr(t: torch.Tensor) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


def _need(t: torch.Tensor, shape, what: str) -> None:
    if not (t.is_cuda and t.is_contiguous() and t.dtype == torch.float32 and tuple(t.shape) == tuple(shape)):
        raise ValueError(f"{what}: expected a contiguous float32 CUDA tensor of shape {tuple(shape)}, got "
                         f"{t.dtype} {tuple(t.shape)} cuda={t.is_cuda} contiguous={t.is_contiguous()}")


class WarmStartNet:
    """The network on the current HIP device (grid d, n_out orbitals)."""

    def __init__(self, grid: int = 32, n_out: int = 120, max_batch: int = 4, seed: int = 0,
                 stream: torch.cuda.Stream | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("the warm-start network needs a HIP device")
        self.lib = _lib.lib()
        self.grid, self.n_out, self.max_batch = int(grid), int(n_out), int(max_batch)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        _lib.check(self.lib.wsn_create(C.byref(h), self.grid, self.n_out, self.max_batch, int(seed),
                                       C.c_void_p(self.stream.cuda_stream)))
        self.h = h
        self.num_params = int(self.lib.wsn_num_params(self.h))
        self.t = 0

    def close(self):
        if getattr(self, "h", None):
            self.lib.wsn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, code):
        if code != _lib.MPE_OK:
            raise _lib.MpeError(code, self.lib.wsn_last_error(self.h).decode())

    # ------------------------------------------------------------ parameters
    def layer_shapes(self):
        """[(name, weight shape (co, 3, 3, 3, ci), bias length)] in vector order."""
        out = []
        for name, ci, co, _ in LAYERS:
            co = self.n_out if co is None else co
            out.append((name, (co, 3, 3, 3, ci), co))
        return out

    def get_vector(self, which: int = 0) -> np.ndarray:
        buf = np.empty(self.num_params, dtype=np.float32)
        self._check(self.lib.wsn_get_params(self.h, C.c_void_p(buf.ctypes.data), which))
        return buf

    def set_vector(self, vec: np.ndarray) -> None:
        vec = np.ascontiguousarray(vec, dtype=np.float32)
        if vec.shape != (self.num_params,):
            raise ValueError(f"parameter vector must have {self.num_params} entries")
        self._check(self.lib.wsn_set_params(self.h, C.c_void_p(vec.ctypes.data)))

    def to_dict(self, vec: np.ndarray) -> dict:
        d, off = {}, 0
        for name, wshape, nb in self.layer_shapes():
            nw = int(np.prod(wshape))
            d[name + ".w"] = vec[off:off + nw].reshape(wshape)
            off += nw
            d[name + ".b"] = vec[off:off + nb]
            off += nb
        return d

    def from_dict(self, d: dict) -> np.ndarray:
        parts = []
        for name, wshape, nb in self.layer_shapes():
            parts.append(np.asarray(d[name + ".w"], dtype=np.float32).reshape(-1))
            parts.append(np.asarray(d[name + ".b"], dtype=np.float32).reshape(nb))
        return np.concatenate(parts)

    def params(self) -> dict:
        return self.to_dict(self.get_vector(0))

    def grads(self) -> dict:
        return self.to_dict(self.get_vector(1))

    def set_params(self, d: dict) -> None:
        self.set_vector(self.from_dict(d))

    def zero_grads(self) -> None:
        self._check(self.lib.wsn_zero_grads(self.h))

    # ------------------------------------------------------------- passes
    def forward(self, v: torch.Tensor, vscale: float = 1.0, out: torch.Tensor | None = None,
                yscale: float = 1.0) -> torch.Tensor:
        """v [B, d, d, d] float32 (device) -> yscale * orbitals [B, n_out, d, d, d]."""
        B, d = int(v.shape[0]), self.grid
        _need(v, (B, d, d, d), "potential")
        if out is None:
            out = torch.empty((B, self.n_out, d, d, d), dtype=torch.float32, device=v.device)
        _need(out, (B, self.n_out, d, d, d), "output")
        self._check(self.lib.wsn_forward(self.h, _ptr(v), float(vscale), float(yscale), B, _ptr(out)))
        self._batch = B
        return out

    def backward(self, dy: torch.Tensor) -> None:
        d = self.grid
        _need(dy, (getattr(self, "_batch", 0), self.n_out, d, d, d), "output gradient")
        self._check(self.lib.wsn_backward(self.h, _ptr(dy)))

    def layer_info(self, layer: int) -> dict:
        buf = (C.c_int32 * 5)()
        self._check(self.lib.wsn_layer_info(self.h, int(layer), buf))
        return dict(zip(("ci", "co", "ci_pad", "stride", "relu"), list(buf)))

    def layer(self, layer: int, x: torch.Tensor, dz: torch.Tensor | None = None, want_dx: bool = False):
        """One convolution layer alone (see wsn_layer): x [B, d, d, d, ci_pad] float32 on the
        device -> y [B, d/s, d/s, d/s, co]; with dz (dL/dy, overwritten by the
        pre-activation gradient) the backward too, returning (y, dx or None)."""
        info = self.layer_info(layer)
        B, d = int(x.shape[0]), int(x.shape[1])
        _need(x, (B, d, d, d, info["ci_pad"]), "layer input")
        do = d // info["stride"]
        y = torch.empty((B, do, do, do, info["co"]), dtype=torch.float32, device=x.device)
        dx = None
        if dz is not None:
            _need(dz, (B, do, do, do, info["co"]), "layer output gradient")
            if want_dx:
                dx = torch.empty((B, d, d, d, info["ci"]), dtype=torch.float32, device=x.device)
        self._check(self.lib.wsn_layer(self.h, int(layer), B, d, _ptr(x), _ptr(y),
                                       _ptr(dz) if dz is not None else None, _ptr(dx) if dx is not None else None))
        return y, dx

    def adam_step(self, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
        self.t += 1
        self._check(self.lib.wsn_adam_step(self.h, lr, beta1, beta2, eps, self.t))

    def subspace_loss(self, y: torch.Tensor, target: torch.Tensor, dy: torch.Tensor | None = None):
        """(L, ||M M^T - I||^2, dL/dy) for y, target [n, ...] float32 on the device."""
        return self._loss(self.lib.wsn_subspace_loss, y, target, dy)

    def procrustes_loss(self, y: torch.Tensor, target: torch.Tensor, dy: torch.Tensor | None = None):
        """(L, sum of singular values of M, dL/dy): distance to the nearest rotation of the targets."""
        return self._loss(self.lib.wsn_procrustes_loss, y, target, dy)

    def _loss(self, fn, y, target, dy):
        n, P = int(y.shape[0]), int(np.prod(y.shape[1:]))
        _need(y, y.shape, "prediction")
        _need(target, y.shape, "target")
        if dy is None:
            dy = torch.empty_like(y)
        _need(dy, y.shape, "gradient")
        loss = (C.c_double * 2)()
        self._check(fn(self.h, _ptr(y), _ptr(target), n, P, loss, _ptr(dy)))
        return loss[0], loss[1], dy


def upsample_periodic(u: torch.Tensor, factor: int, stream: torch.cuda.Stream | None = None) -> torch.Tensor:
    """Periodic trilinear interpolation of u [C, d, d, d] onto (d*factor)^3 points."""
    Cn, d = int(u.shape[0]), int(u.shape[1])
    _need(u, (Cn, d, d, d), "coarse field")
    D = d * int(factor)
    out = torch.empty((Cn, D, D, D), dtype=torch.float32, device=u.device)
    st = stream if stream is not None else torch.cuda.current_stream()
    code = _lib.lib().wsn_upsample_periodic(_ptr(u), Cn, d, int(factor), _ptr(out), C.c_void_p(st.cuda_stream))
    _lib.check(code)
    return out
