"""Shape-optimisation step for mesh vertices (dwos_opt_* of include/dwos.h):
argument marshalling only; the solves and updates run in the HIP library."""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np
import torch

from . import capi
from .capi import check


def _dev(t: torch.Tensor):
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 GPU tensor")
    return C.c_void_p(t.data_ptr())


class LargeSteps:
    """Vector Adam on u = (I + lam L) x with the max second moment."""

    def __init__(self, dim: int, nv: int, prims, lam: float, movable=None,
                 stream: Optional[torch.cuda.Stream] = None):
        self.dim, self.nv = int(dim), int(nv)
        P = np.ascontiguousarray(prims, dtype=np.int32).reshape(-1, self.dim)
        mv = None if movable is None else np.ascontiguousarray(movable, dtype=np.int32)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._o = C.c_void_p()
        check(capi.dwos_opt_create(self.dim, self.nv, P.ctypes.data_as(C.POINTER(C.c_int32)), P.shape[0],
                                   mv.ctypes.data_as(C.POINTER(C.c_int32)) if mv is not None else None,
                                   float(lam), C.c_void_p(self.stream.cuda_stream), C.byref(self._o)))

    def __del__(self):
        o = getattr(self, "_o", None)
        if o is not None and o.value:
            try:
                capi.lib().dwos_opt_destroy(o)
            except Exception:   # interpreter shutdown
                pass
            self._o = None

    def reset(self, x: torch.Tensor):
        check(capi.dwos_opt_reset(self._o, _dev(x)))

    def step(self, g: torch.Tensor, x: torch.Tensor, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
             max_iters=1000, tol=1e-10):
        it = (C.c_int32 * 2)()
        check(capi.dwos_opt_step(self._o, _dev(g), _dev(x), float(lr), float(beta1), float(beta2), float(eps),
                                 int(max_iters), float(tol), it))
        return it[0], it[1]

    def solve(self, b: torch.Tensor, x: torch.Tensor, max_iters=1000, tol=1e-12):
        it = C.c_int32()
        check(capi.dwos_opt_solve(self._o, _dev(b), _dev(x), int(max_iters), float(tol), C.byref(it)))
        return it.value
