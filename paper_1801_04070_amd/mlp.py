"""Binding of the order-prediction network (``include/gigaqbx_mlp.h``): argument marshalling only.

Forward pass, gradients and Adam steps all run in the library's HIP kernels; inputs and outputs
are FP32 torch tensors on the network's device.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import GQError, library, _ptr


class MLP:
    """Three-layer ReLU network with BF16 matrix-core products and FP32 accumulation."""

    def __init__(self, n_in: int, n_hidden: int, n_out: int, seed: int = 0, device: int = 0,
                 stream=None):
        import torch
        self._L = library()
        self.device = device
        self.n_in, self.n_hidden, self.n_out = n_in, n_hidden, n_out
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._stream = stream
        h = C.c_void_p()
        st = self._L.gq_mlp_create(C.byref(h), device, C.c_void_p(stream.cuda_stream), n_in,
                                   n_hidden, n_out, seed)
        if st != 0:
            raise GQError(st, "gq_mlp_create failed (sizes or device)")
        self._h = h

    def _check(self, st):
        if st != 0:
            raise GQError(st, self._L.gq_mlp_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.gq_mlp_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def param_count(self) -> int:
        return int(self._L.gq_mlp_param_count(self._h))

    def get_params(self) -> np.ndarray:
        p = np.empty(self.param_count, np.float32)
        self._check(self._L.gq_mlp_get_params(self._h, p.ctypes.data))
        return p

    def set_params(self, p) -> None:
        p = np.ascontiguousarray(p, dtype=np.float32)
        if p.size != self.param_count:
            raise ValueError(f"expected {self.param_count} parameters, got {p.size}")
        self._check(self._L.gq_mlp_set_params(self._h, p.ctypes.data))

    def _dev(self, a, cols):
        import torch
        a = torch.as_tensor(a, dtype=torch.float32, device=f"cuda:{self.device}").contiguous()
        if a.dim() != 2 or a.shape[1] != cols:
            raise ValueError(f"expected (n, {cols}) array, got {tuple(a.shape)}")
        return a

    def forward(self, x):
        import torch
        x = self._dev(x, self.n_in)
        y = torch.empty((x.shape[0], self.n_out), dtype=torch.float32, device=x.device)
        self._check(self._L.gq_mlp_forward(self._h, x.shape[0], _ptr(x), _ptr(y)))
        return y

    def gradients(self, x, t, w=None):
        x, t = self._dev(x, self.n_in), self._dev(t, self.n_out)
        w = None if w is None else self._dev(w, self.n_out)
        g = np.empty(self.param_count, np.float32)
        loss = C.c_float()
        self._check(self._L.gq_mlp_gradients(self._h, x.shape[0], _ptr(x), _ptr(t), _ptr(w),
                                             g.ctypes.data, C.byref(loss)))
        return float(loss.value), g

    def train_step(self, x, t, w=None, lr: float = 1e-3, want_loss: bool = False):
        x, t = self._dev(x, self.n_in), self._dev(t, self.n_out)
        w = None if w is None else self._dev(w, self.n_out)
        loss = C.c_float()
        self._check(self._L.gq_mlp_train_step(self._h, x.shape[0], _ptr(x), _ptr(t), _ptr(w), lr,
                                              C.byref(loss) if want_loss else None))
        return float(loss.value) if want_loss else None
