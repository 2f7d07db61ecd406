"""Isotropic remeshing of a boundary (dwos_remesh): the periodic remeshing of
the paper's shape-optimisation loop (Sec. 7.2, "Gradient preconditioning").
Host code in the library; this module only marshals the arrays."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import capi
from .capi import check


def remesh(V, prims, target: float, iters: int = 5, fixed=None):
    """Remesh the polyline (2D) or triangle mesh (3D) toward edge length
    ``target``.  Returns (V, prims, src): the new vertices and primitives
    and, per new vertex, the index of the input vertex it continues (-1 for
    a vertex created by a split).  ``fixed`` (bool per input vertex) keeps
    vertices in place and in the mesh."""
    V = np.ascontiguousarray(V, dtype=np.float64)
    dim = V.shape[1]
    prims = np.ascontiguousarray(prims, dtype=np.int32).reshape(-1, dim)
    fx = None if fixed is None else np.ascontiguousarray(np.asarray(fixed, bool).astype(np.int32))
    h = C.c_void_p()
    L = capi.lib()
    check(L.dwos_remesh(dim, V.ctypes.data_as(C.POINTER(C.c_double)), V.shape[0],
                        prims.ctypes.data_as(C.POINTER(C.c_int32)), prims.shape[0],
                        fx.ctypes.data_as(C.POINTER(C.c_int32)) if fx is not None else None,
                        float(target), int(iters), C.byref(h)))
    try:
        nv, npr = C.c_int64(), C.c_int64()
        check(L.dwos_mesh_size(h, C.byref(nv), C.byref(npr)))
        V2 = np.zeros((nv.value, dim))
        P2 = np.zeros((npr.value, dim), np.int32)
        src = np.zeros(nv.value, np.int64)
        check(L.dwos_mesh_get(h, V2.ctypes.data_as(C.POINTER(C.c_double)),
                              P2.ctypes.data_as(C.POINTER(C.c_int32)), src.ctypes.data_as(C.POINTER(C.c_int64))))
    finally:
        L.dwos_mesh_destroy(h)
    return V2, P2, src
