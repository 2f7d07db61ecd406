"""ctypes binding of libdwos.so (include/dwos.h): argument marshalling only.

Every function here has the name and argument order of the C entry point it
wraps; all arithmetic happens in the HIP library.  Importing this module fails
loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdwos.so")

DWOS_OK, DWOS_EINVAL, DWOS_ENOMEM, DWOS_EDEVICE, DWOS_ESTATE = 0, 1, 2, 3, 4
DWOS_FP32, DWOS_FP64 = 0, 1
MAX_LABELS, MAX_GAUSS = 16, 8


class dwos_bc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pad_", C.c_int32), ("c", C.c_double),
                ("b", C.c_double * 3), ("A", C.c_double * 9)]


class dwos_problem(C.Structure):
    _fields_ = [("sigma", C.c_double), ("eps", C.c_double), ("delta", C.c_double),
                ("K", C.c_int32), ("kmax", C.c_int32), ("rr", C.c_int32), ("n_gauss", C.c_int32),
                ("src_c0", C.c_double), ("gauss", (C.c_double * 5) * MAX_GAUSS),
                ("n_labels", C.c_int32), ("dudn", C.c_int32), ("bc", dwos_bc * MAX_LABELS)]


class dwos_stats(C.Structure):
    _fields_ = [("walks", C.c_int64), ("nested_walks", C.c_int64), ("steps", C.c_int64),
                ("terminal", C.c_int64), ("truncated", C.c_int64), ("nodes", C.c_int64),
                ("prims", C.c_int64), ("stack_overflow", C.c_int64), ("invalid", C.c_int64),
                ("walk_ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class dwos_tuning(C.Structure):
    _fields_ = [("variant", C.c_int32), ("park", C.c_int32), ("tail", C.c_int32), ("chunk", C.c_int32),
                ("stage_nodes", C.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


DWOS_TUNE_CACHE = 1
DWOS_TUNE_GRAD = 2


class dwos_quad(C.Structure):
    _fields_ = [("c", C.c_double), ("b", C.c_double * 3), ("A", C.c_double * 9)]


class DwosError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dwos error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libdwos.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not built: run __graft_entry__.build() or "
                              "python -m paper_2405_12964_amd.build")
        L = C.CDLL(LIB_PATH)
        vp, dp, i32p, i64p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
        st = C.c_int32
        sig = {
            "dwos_create": [C.c_int32, C.c_int32, vp, C.POINTER(vp)],
            "dwos_destroy": [vp],
            "dwos_set_boundary": [vp, dp, C.c_int64, i32p, C.c_int64, i32p, dp],
            "dwos_update_vertices": [vp, vp],
            "dwos_apply_parameters": [vp, vp, vp],
            "dwos_set_problem": [vp, C.POINTER(dwos_problem)],
            "dwos_set_parameters": [vp, C.c_int64, i64p, i32p, dp, i32p],
            "dwos_solve": [vp, vp, C.c_int64, C.c_int32, C.c_uint64, vp, vp, C.POINTER(dwos_stats)],
            "dwos_grad": [vp, vp, C.c_int64, vp, C.c_int32, C.c_uint64, vp, vp, C.POINTER(dwos_stats)],
            "dwos_grad_sqloss": [vp, vp, C.c_int64, vp, C.c_int32, C.c_int32, C.c_uint64, vp, vp, vp,
                                 C.POINTER(dwos_stats)],
            "dwos_jvp": [vp, vp, C.c_int64, C.c_int32, C.c_uint64, vp, vp, vp, C.POINTER(dwos_stats)],
            "dwos_walk_records": [vp, vp, C.c_int64, C.c_int32, C.c_uint64, C.c_int32, vp, vp, vp, vp, vp],
            "dwos_closest": [vp, vp, C.c_int64, vp],
            "dwos_eval_ball_kernels": [vp, vp, vp, C.c_int64, C.c_double, vp, vp],
            "dwos_walk_timing": [vp, C.c_int32, C.c_int32, dp, i64p, C.POINTER(dwos_stats)],
            "dwos_set_seed_buffer": [vp, vp],
            "dwos_autotune": [vp, vp, i64p, C.c_int32, C.c_uint64, C.c_int32, C.POINTER(dwos_tuning), dp],
            "dwos_set_tuning": [vp, C.POINTER(dwos_tuning)],
            "dwos_get_tuning": [vp, C.POINTER(dwos_tuning)],
            "dwos_set_variant": [vp, C.c_int32],
            "dwos_batch_add_instance": [vp, dp, C.c_int64, i32p, C.c_int64, i32p, C.c_double,
                                        C.c_double, C.c_double, i32p],
            "dwos_batch_solve": [vp, vp, i64p, C.c_int32, C.c_uint64, vp, vp, C.POINTER(dwos_stats)],
            "dwos_batch_set_parameters": [vp, C.c_int32, C.c_int64, i64p, i32p, dp],
            "dwos_batch_grad": [vp, vp, i64p, vp, C.c_int32, C.c_uint64, vp, vp, C.POINTER(dwos_stats)],
            "dwos_adjoint_grad": [vp, vp, vp, vp, C.c_int64, C.POINTER(dwos_quad), C.c_int32, C.c_uint64, vp, vp,
                                  vp, C.POINTER(dwos_stats)],
            "dwos_mlp_create": [C.c_int32, C.c_int32, C.POINTER(C.c_float), vp, C.POINTER(vp)],
            "dwos_mlp_set_params": [vp, vp],
            "dwos_mlp_get_params": [vp, vp],
            "dwos_mlp_eval": [vp, vp, C.c_int64, vp, vp, vp],
            "dwos_mlp_loss_grad": [vp, vp, vp, vp, C.c_int64, vp, vp],
            "dwos_mlp_vjp": [vp, vp, vp, vp, C.c_int64, vp],
            "dwos_mlp_adam_step": [vp, C.c_float, C.c_float, C.c_float, C.c_float],
            "dwos_cv_attach": [vp, vp, C.c_double],
            "dwos_cv_beta": [vp, dp],
            "dwos_cv_train": [vp, C.c_int32, C.c_int32, C.c_float, C.c_uint64, vp],
            "dwos_cv_walk_records": [vp, vp, C.c_int64, C.c_int32, C.c_uint64, vp, vp],
            "dwos_set_reflecting": [vp, dp, C.c_int64, i32p, C.c_int64],
            "dwos_set_start_segments": [vp, i32p, C.c_int64],
            "dwos_reflect_query": [vp, vp, vp, vp, vp, vp, C.c_int64, vp],
            "dwos_eval_reflect_weight": [vp, vp, vp, C.c_int64, C.c_double, vp],
            "dwos_set_implicit": [vp, dp, C.c_int64, C.c_double],
            "dwos_implicit_band_grad": [vp, vp, C.c_int64, vp, C.c_double, vp, vp],
            "dwos_remesh": [C.c_int32, dp, C.c_int64, i32p, C.c_int64, i32p, C.c_double, C.c_int32,
                            C.POINTER(vp)],
            "dwos_mesh_size": [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)],
            "dwos_mesh_get": [vp, dp, i32p, i64p],
            "dwos_opt_create": [C.c_int32, C.c_int64, i32p, C.c_int64, i32p, C.c_double, vp, C.POINTER(vp)],
            "dwos_opt_reset": [vp, vp],
            "dwos_opt_step": [vp, vp, vp, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int32,
                              C.c_double, i32p],
            "dwos_opt_solve": [vp, vp, vp, C.c_int32, C.c_double, i32p],
            "dwos_probe_bandwidth": [C.c_int64, C.c_int32, C.c_int32, dp, dp],
            "dwos_scene_info": [vp, i64p],
            "dwos_solve_noalloc": [vp, vp, C.c_int64, C.c_int32, C.c_uint64, vp, vp],
            "dwos_set_robin": [vp, C.c_double, C.POINTER(dwos_bc)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = st
        L.dwos_last_error.argtypes = []
        L.dwos_last_error.restype = C.c_char_p
        L.dwos_mlp_theta_size.argtypes = []
        L.dwos_mlp_theta_size.restype = C.c_int32
        L.dwos_mlp_destroy.argtypes = [vp]
        L.dwos_mlp_destroy.restype = None
        L.dwos_opt_destroy.argtypes = [vp]
        L.dwos_opt_destroy.restype = None
        L.dwos_mesh_destroy.argtypes = [vp]
        L.dwos_mesh_destroy.restype = None
        _lib = L
    return _lib


EXPORTED = [
    "dwos_create", "dwos_destroy", "dwos_last_error", "dwos_set_boundary", "dwos_update_vertices",
    "dwos_apply_parameters",
    "dwos_set_problem", "dwos_set_parameters", "dwos_solve", "dwos_grad", "dwos_grad_sqloss",
    "dwos_jvp", "dwos_walk_records", "dwos_closest", "dwos_eval_ball_kernels", "dwos_walk_timing",
    "dwos_batch_add_instance", "dwos_batch_solve", "dwos_batch_set_parameters", "dwos_batch_grad", "dwos_set_seed_buffer", "dwos_autotune",
    "dwos_set_variant", "dwos_mlp_theta_size", "dwos_mlp_create", "dwos_mlp_destroy",
    "dwos_mlp_set_params", "dwos_mlp_get_params", "dwos_mlp_eval", "dwos_mlp_loss_grad",
    "dwos_mlp_vjp", "dwos_mlp_adam_step", "dwos_cv_attach", "dwos_cv_beta", "dwos_cv_train", "dwos_cv_walk_records",
    "dwos_set_reflecting", "dwos_set_start_segments", "dwos_reflect_query", "dwos_eval_reflect_weight",
    "dwos_set_implicit", "dwos_implicit_band_grad", "dwos_adjoint_grad",
    "dwos_remesh", "dwos_mesh_size", "dwos_mesh_get", "dwos_mesh_destroy",
    "dwos_opt_create", "dwos_opt_destroy", "dwos_opt_reset", "dwos_opt_step", "dwos_opt_solve",
    "dwos_probe_bandwidth", "dwos_scene_info", "dwos_solve_noalloc", "dwos_set_robin",
    "dwos_set_tuning", "dwos_get_tuning",
]


def check(code):
    if code != DWOS_OK:
        raise DwosError(code, lib().dwos_last_error().decode(errors="replace"))
    return code


def _wrap(name):
    def f(*args):
        return getattr(lib(), name)(*args)
    f.__name__ = name
    f.__doc__ = f"Call {name} of include/dwos.h (returns the dwos_status)."
    return f


for _n in EXPORTED:
    globals()[_n] = _wrap(_n)
