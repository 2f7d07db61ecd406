"""Control-variate network (dwos_mlp_* of include/dwos.h): argument marshalling.

The network N(x) -- Fourier features, four tanh layers of width 64, a scalar
output -- lives on the GPU with FP32 master parameters and Adam moments; every
evaluation, gradient and update runs in the HIP library's matrix-core kernels.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np
import torch

from . import capi
from .capi import check


def theta_size() -> int:
    return int(capi.lib().dwos_mlp_theta_size())


def _dev(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError("expected a contiguous float32 GPU tensor")
    return C.c_void_p(t.data_ptr())


class Network:
    """One dwos_mlp: frequencies B (F x dim), parameters theta."""

    def __init__(self, dim: int, B, theta=None, stream: Optional[torch.cuda.Stream] = None):
        self.dim = int(dim)
        Bh = np.ascontiguousarray(B, dtype=np.float32).reshape(-1, self.dim)
        self.F = Bh.shape[0]
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._m = C.c_void_p()
        check(capi.dwos_mlp_create(self.dim, self.F, Bh.ctypes.data_as(C.POINTER(C.c_float)),
                                   C.c_void_p(self.stream.cuda_stream), C.byref(self._m)))
        if theta is not None:
            self.set_params(theta)

    def __del__(self):
        m = getattr(self, "_m", None)
        if m is not None and m.value:
            try:
                capi.lib().dwos_mlp_destroy(m)
            except Exception:   # interpreter shutdown: module globals already gone
                pass
            self._m = None

    @property
    def handle(self):
        return self._m

    def set_params(self, theta):
        t = torch.as_tensor(np.asarray(theta, dtype=np.float32) if not torch.is_tensor(theta) else theta,
                            dtype=torch.float32).contiguous().cuda()
        if t.numel() != theta_size():
            raise ValueError(f"theta must have {theta_size()} entries")
        self._keep = t
        check(capi.dwos_mlp_set_params(self._m, _dev(t)))

    def params(self) -> torch.Tensor:
        t = torch.empty(theta_size(), dtype=torch.float32, device="cuda")
        check(capi.dwos_mlp_get_params(self._m, _dev(t)))
        return t

    def eval(self, X: torch.Tensor, derivatives: bool = False):
        """N (n), and with derivatives grad N (n x dim) and Lap N (n)."""
        X = X.to(torch.float32).contiguous()
        n = X.shape[0]
        N = torch.empty(n, dtype=torch.float32, device=X.device)
        G = torch.empty(n, self.dim, dtype=torch.float32, device=X.device) if derivatives else None
        L = torch.empty(n, dtype=torch.float32, device=X.device) if derivatives else None
        check(capi.dwos_mlp_eval(self._m, _dev(X), n, _dev(N), _dev(G), _dev(L)))
        return (N, G, L) if derivatives else N

    def loss_grad(self, X, T, w=None):
        """(loss, grad) of sum_i 1/2 w_i (N(x_i) - t_i)^2."""
        X = X.to(torch.float32).contiguous()
        T = T.to(torch.float32).contiguous()
        w = None if w is None else w.to(torch.float32).contiguous()
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
        g = torch.empty(theta_size(), dtype=torch.float32, device=X.device)
        check(capi.dwos_mlp_loss_grad(self._m, _dev(X), _dev(T), _dev(w), X.shape[0], _dev(loss), _dev(g)))
        return loss, g

    def vjp(self, X, Nbar, Lbar=None):
        """d/dtheta sum_i (Nbar_i N(x_i) + Lbar_i Lap N(x_i))."""
        X = X.to(torch.float32).contiguous()
        Nbar = Nbar.to(torch.float32).contiguous()
        Lbar = None if Lbar is None else Lbar.to(torch.float32).contiguous()
        g = torch.empty(theta_size(), dtype=torch.float32, device=X.device)
        check(capi.dwos_mlp_vjp(self._m, _dev(X), _dev(Nbar), _dev(Lbar), X.shape[0], _dev(g)))
        return g

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        check(capi.dwos_mlp_adam_step(self._m, float(lr), float(beta1), float(beta2), float(eps)))
