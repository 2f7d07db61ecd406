"""FP64 CPU oracle for differential walk on spheres -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never loads it and
shares no code with it.

The numerics live in ``dwos_oracle.cpp`` (plain C++17, FP64, brute-force
closest points, its own Philox4x32-10, Bessel functions from libstdc++'s
``std::cyl_bessel_i/k``).  This module compiles it with g++ and marshals
``scenes.Scene`` objects into its C struct with ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dwos_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle shared library with g++ (host only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        lp = C.POINTER(C.c_int64)
        up = C.POINTER(C.c_uint32)
        sp = C.POINTER(OracleScene)
        L.oracle_threads.restype = C.c_int
        L.oracle_philox.argtypes = [up, up, up]
        L.oracle_green.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double]
        L.oracle_green.restype = C.c_double
        L.oracle_poisson_scale.argtypes = [C.c_int, C.c_double, C.c_double]
        L.oracle_poisson_scale.restype = C.c_double
        L.oracle_green_mass.argtypes = [C.c_int, C.c_double, C.c_double]
        L.oracle_green_mass.restype = C.c_double
        L.oracle_closest.argtypes = [sp, dp, dp]
        L.oracle_neumann_weight.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double]
        L.oracle_neumann_weight.restype = C.c_double
        L.oracle_silhouette.argtypes = [sp, dp, C.c_int32, dp, C.c_double, dp]
        L.oracle_ray.argtypes = [sp, dp, dp, C.c_double, C.c_int32, dp]
        L.oracle_boundary_sample.argtypes = [sp, dp, C.c_double, C.c_uint64, C.c_uint32, C.c_int32, dp]
        L.oracle_safe_radius.argtypes = [sp, dp, dp]
        L.oracle_walk_records.argtypes = [sp, dp, C.c_int64, C.c_int32, C.c_uint64, C.c_int32,
                                          C.c_int32, dp, dp, lp, ip, dp, lp, dp, C.c_int]
        L.oracle_solve.argtypes = [sp, dp, C.c_int64, C.c_int32, C.c_uint64, C.c_int32, dp, dp,
                                   lp, C.c_int]
        cvp = C.POINTER(OracleCV)
        L.oracle_jvp.argtypes = [sp, dp, C.c_int64, C.c_int32, C.c_uint64, C.c_int32, dp, dp, dp,
                                 lp, C.c_int, cvp]
        L.oracle_grad.argtypes = [sp, dp, C.c_int64, dp, C.c_int32, C.c_uint64, C.c_int32, dp, dp,
                                  lp, C.c_int, cvp]
        L.oracle_grad_sqloss.argtypes = [sp, dp, C.c_int64, dp, C.c_int32, C.c_int32, C.c_uint64,
                                         C.c_int32, dp, dp, dp, lp, C.c_int, cvp]
        L.oracle_mlp_eval.argtypes = [C.c_int32, C.c_int32, dp, dp, dp, C.c_int64, dp, dp, dp]
        L.oracle_mlp_theta_size.restype = C.c_int32
        L.oracle_mlp_loss_grad.argtypes = [C.c_int32, C.c_int32, dp, dp, dp, dp, dp, C.c_int64,
                                           dp, dp]
        L.oracle_mlp_vjp.argtypes = [C.c_int32, C.c_int32, dp, dp, dp, dp, dp, C.c_int64, dp]
        L.oracle_adam.argtypes = [C.c_int64, dp, dp, dp, dp, C.c_double, C.c_double, C.c_double,
                                  C.c_double, C.c_int64]
        L.oracle_walk_records_cv.argtypes = [sp, cvp, dp, C.c_int64, C.c_int32, C.c_uint64,
                                             C.c_int32, dp, dp, C.c_int]
        L.oracle_adjoint_grad.argtypes = [sp, ip, dp, dp, C.c_int64, dp, C.c_int32, C.c_uint64, dp, dp, dp,
                                          lp, C.c_int]
        _lib = L
    return _lib


class OracleScene(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("nv", C.c_int32), ("V", C.POINTER(C.c_double)),
        ("np", C.c_int32), ("prims", C.POINTER(C.c_int32)), ("label", C.POINTER(C.c_int32)),
        ("sigma", C.c_double), ("eps", C.c_double), ("delta", C.c_double),
        ("K", C.c_int32), ("kmax", C.c_int32), ("rr", C.c_int32),
        ("src_c0", C.c_double), ("n_gauss", C.c_int32), ("gauss", C.POINTER(C.c_double)),
        ("n_labels", C.c_int32), ("bc_kind", C.POINTER(C.c_int32)),
        ("bc_quad", C.POINTER(C.c_double)), ("gvert", C.POINTER(C.c_double)),
        ("N", C.c_int32), ("rowptr", C.POINTER(C.c_int64)), ("pid", C.POINTER(C.c_int32)),
        ("vel", C.POINTER(C.c_double)), ("bc_pid", C.POINTER(C.c_int32)),
        ("n_nv", C.c_int32), ("NV", C.POINTER(C.c_double)), ("n_ns", C.c_int32),
        ("nsegs", C.POINTER(C.c_int32)), ("start_seg", C.POINTER(C.c_int32)),
        ("n_mono", C.c_int32), ("mono", C.POINTER(C.c_double)), ("mono_c", C.c_double),
        ("dudn", C.c_int32), ("robin_mu", C.c_double), ("robin_quad", C.POINTER(C.c_double)),
    ]


class OracleCV(C.Structure):
    _fields_ = [("F", C.c_int32), ("B", C.POINTER(C.c_double)), ("theta", C.POINTER(C.c_double)),
                ("q", C.c_double)]


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct)) if a is not None else None


class Oracle:
    """Oracle bound to one scene (keeps the marshalled arrays alive)."""

    def __init__(self, scene, V: Optional[np.ndarray] = None, threads: int = 0):
        self.scene = scene
        self.threads = int(threads)
        D = scene.dim
        self._V = np.ascontiguousarray(scene.V if V is None else V, dtype=np.float64)
        self._prims = np.ascontiguousarray(scene.prims, dtype=np.int32)
        self._label = np.ascontiguousarray(scene.label, dtype=np.int32)
        self._gauss = np.ascontiguousarray(np.asarray(scene.gauss, float).reshape(-1, D + 2))
        kinds, quads = [], []
        for b in scene.bc:
            if b["kind"] == "mapped":
                kinds.append(1)
                quads.append(np.zeros(1 + D + D * D))
            else:
                kinds.append(0)
                quads.append(np.concatenate([[b["c"]], np.asarray(b["b"], float).ravel(),
                                             np.asarray(b["A"], float).ravel()]))
        self._kind = np.ascontiguousarray(kinds, dtype=np.int32)
        self._quad = np.ascontiguousarray(np.concatenate(quads), dtype=np.float64)
        self._gvert = np.ascontiguousarray(scene.gvert, dtype=np.float64)
        nv = self._V.shape[0]
        if scene.rowptr is not None:
            self._rowptr = np.ascontiguousarray(scene.rowptr, dtype=np.int64)
            self._pid = np.ascontiguousarray(scene.pid, dtype=np.int32)
            self._vel = np.ascontiguousarray(scene.vel, dtype=np.float64).reshape(-1)
        else:
            self._rowptr = np.zeros(nv + 1, np.int64)
            self._pid = np.zeros(1, np.int32)
            self._vel = np.zeros(D, np.float64)
        self._bcpid = (np.ascontiguousarray(scene.bc_pid, dtype=np.int32)
                       if scene.bc_pid is not None else None)
        s = OracleScene()
        s.dim = D
        s.nv = nv
        s.V = _ptr(self._V, C.c_double)
        s.np = self._prims.shape[0]
        s.prims = _ptr(self._prims, C.c_int32)
        s.label = _ptr(self._label, C.c_int32)
        s.sigma, s.eps, s.delta = float(scene.sigma), float(scene.eps), float(scene.delta)
        s.K, s.kmax, s.rr = int(scene.K), int(scene.kmax), int(scene.rr)
        s.src_c0 = float(scene.src_c0)
        s.n_gauss = self._gauss.shape[0]
        s.gauss = _ptr(self._gauss, C.c_double)
        s.n_labels = len(kinds)
        s.bc_kind = _ptr(self._kind, C.c_int32)
        s.bc_quad = _ptr(self._quad, C.c_double)
        s.gvert = _ptr(self._gvert, C.c_double)
        s.N = int(scene.N)
        s.rowptr = _ptr(self._rowptr, C.c_int64)
        s.pid = _ptr(self._pid, C.c_int32)
        s.vel = _ptr(self._vel, C.c_double)
        s.bc_pid = _ptr(self._bcpid, C.c_int32)
        if getattr(scene, "nsegs", None) is not None and len(scene.nsegs) > 0:
            self._NV = np.ascontiguousarray(scene.NV, dtype=np.float64)
            self._nsegs = np.ascontiguousarray(scene.nsegs, dtype=np.int32)
            s.n_nv = self._NV.shape[0]
            s.NV = _ptr(self._NV, C.c_double)
            s.n_ns = self._nsegs.shape[0]
            s.nsegs = _ptr(self._nsegs, C.c_int32)
        if getattr(scene, "mono", None) is not None and len(scene.mono) > 0:
            self._mono = np.ascontiguousarray(scene.mono, dtype=np.float64).reshape(-1, 3)
            s.n_mono = self._mono.shape[0]
            s.mono = _ptr(self._mono, C.c_double)
            s.mono_c = float(scene.mono_c)
        s.dudn = int(getattr(scene, "dudn", 0))
        s.robin_mu = float(getattr(scene, "robin_mu", 0.0))
        rh = getattr(scene, "robin_h", None)
        self._robin = None
        if rh is not None:
            self._robin = np.ascontiguousarray(np.concatenate([[rh["c"]], np.asarray(rh["b"], float).ravel(),
                                                               np.asarray(rh["A"], float).ravel()]))
            s.robin_quad = _ptr(self._robin, C.c_double)
        self._start = None
        self._s = s

    def _starts(self, start_seg, P):
        """Per-point start segments (None: every point inside the domain)."""
        if start_seg is None:
            self._start = None
        else:
            self._start = np.ascontiguousarray(start_seg, dtype=np.int32)
            assert self._start.shape == (P,)
        self._s.start_seg = _ptr(self._start, C.c_int32)

    @staticmethod
    def _X(X):
        return np.ascontiguousarray(X, dtype=np.float64)

    def closest(self, x):
        out = np.zeros(8)
        x = np.ascontiguousarray(x, dtype=np.float64)
        rc = lib().oracle_closest(C.byref(self._s), _ptr(x, C.c_double), _ptr(out, C.c_double))
        assert rc == 0
        return dict(d=out[0], prim=int(out[1]), bary=out[2:5].copy(), xbar=out[5:8].copy())

    def walk_records(self, X, W, seed, mode=0, instance=0, want_udot=True, start_seg=None):
        X = self._X(X)
        P = X.shape[0]
        self._starts(start_seg, P)
        N = self.scene.N
        u = np.zeros(P * W)
        udot = np.zeros(P * W * N) if (mode == 1 and want_udot and N > 0) else None
        steps = np.zeros(P * W, np.int64)
        prim = np.zeros(P * W, np.int32)
        uoff = np.zeros(P * W)
        xbar = np.zeros(P * W * 3)
        tr = np.zeros(1, np.int64)
        rc = lib().oracle_walk_records(C.byref(self._s), _ptr(X, C.c_double), P, W, seed, mode,
                                       instance, _ptr(u, C.c_double), _ptr(udot, C.c_double),
                                       _ptr(steps, C.c_int64), _ptr(prim, C.c_int32),
                                       _ptr(uoff, C.c_double), _ptr(tr, C.c_int64),
                                       _ptr(xbar, C.c_double), self.threads)
        assert rc == 0
        out = dict(u=u.reshape(P, W), steps=steps.reshape(P, W), prim=prim.reshape(P, W),
                   uoff=uoff.reshape(P, W), truncated=int(tr[0]), xbar=xbar.reshape(P, W, 3))
        if udot is not None:
            out["udot"] = udot.reshape(P, W, N)
        return out

    def solve(self, X, W, seed, instance=0, start_seg=None):
        X = self._X(X)
        P = X.shape[0]
        self._starts(start_seg, P)
        m, v, st = np.zeros(P), np.zeros(P), np.zeros(1, np.int64)
        rc = lib().oracle_solve(C.byref(self._s), _ptr(X, C.c_double), P, W, seed, instance,
                                _ptr(m, C.c_double), _ptr(v, C.c_double), _ptr(st, C.c_int64),
                                self.threads)
        assert rc == 0
        return m, v, int(st[0])

    def jvp(self, X, W, seed, instance=0, cv=None, start_seg=None):
        X = self._X(X)
        P = X.shape[0]
        self._starts(start_seg, P)
        N = self.scene.N
        m, v, um, st = np.zeros(P * N), np.zeros(P * N), np.zeros(P), np.zeros(1, np.int64)
        rc = lib().oracle_jvp(C.byref(self._s), _ptr(X, C.c_double), P, W, seed, instance,
                              _ptr(m, C.c_double), _ptr(v, C.c_double), _ptr(um, C.c_double),
                              _ptr(st, C.c_int64), self.threads, _cvref(cv))
        assert rc == 0
        return m.reshape(P, N), v.reshape(P, N), um, int(st[0])

    def grad(self, X, w, W, seed, instance=0, cv=None, start_seg=None):
        X = self._X(X)
        P = X.shape[0]
        self._starts(start_seg, P)
        w = np.ascontiguousarray(w, dtype=np.float64)
        g, um, st = np.zeros(self.scene.N), np.zeros(P), np.zeros(1, np.int64)
        rc = lib().oracle_grad(C.byref(self._s), _ptr(X, C.c_double), P, _ptr(w, C.c_double), W,
                               seed, instance, _ptr(g, C.c_double), _ptr(um, C.c_double),
                               _ptr(st, C.c_int64), self.threads, _cvref(cv))
        assert rc == 0
        return g, um, int(st[0])

    def grad_sqloss(self, X, uref, W, B, seed, instance=0, cv=None, start_seg=None):
        X = self._X(X)
        P = X.shape[0]
        self._starts(start_seg, P)
        uref = np.ascontiguousarray(uref, dtype=np.float64)
        g, um, st, L = np.zeros(self.scene.N), np.zeros(P), np.zeros(1, np.int64), np.zeros(1)
        rc = lib().oracle_grad_sqloss(C.byref(self._s), _ptr(X, C.c_double), P,
                                      _ptr(uref, C.c_double), W, B, seed, instance,
                                      _ptr(L, C.c_double), _ptr(g, C.c_double),
                                      _ptr(um, C.c_double), _ptr(st, C.c_int64), self.threads,
                                      _cvref(cv))
        if rc != 0:
            raise ValueError("oracle_grad_sqloss: invalid arguments")
        return float(L[0]), g, um, int(st[0])

    def silhouette(self, x, on=-1, nin=None, cap=np.inf):
        """Distance from x to the closest silhouette point of the reflecting
        boundary (x on reflecting primitive ``on`` with domain side ``nin``,
        or inside)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        n = np.zeros(3)
        if nin is not None:
            n[:len(nin)] = nin
        out = np.zeros(1)
        rc = lib().oracle_silhouette(C.byref(self._s), _ptr(x, C.c_double), int(on),
                                     _ptr(n, C.c_double), float(cap), _ptr(out, C.c_double))
        assert rc == 0
        return float(out[0])

    def ray(self, x, d, tmax=np.inf, skip=-1):
        """First reflecting primitive hit by x + t d, 0 < t < tmax: (t, index)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        d = np.ascontiguousarray(d, dtype=np.float64)
        out = np.zeros(2)
        rc = lib().oracle_ray(C.byref(self._s), _ptr(x, C.c_double), _ptr(d, C.c_double),
                              float(tmax), int(skip), _ptr(out, C.c_double))
        assert rc == 0
        return float(out[0]), int(out[1])

    def boundary_sample(self, x, R, n, seed=1, k=0):
        """n draws of the Robin boundary sample around x with radius R: an
        (n, 5) array of (primitive or -1, L, z)."""
        x = np.zeros(3) if x is None else np.concatenate([np.asarray(x, float), np.zeros(3 - len(x))])
        out = np.zeros((n, 5))
        rc = lib().oracle_boundary_sample(C.byref(self._s), _ptr(x, C.c_double), float(R), int(seed), int(k),
                                          int(n), _ptr(out, C.c_double))
        assert rc == 0
        return out

    def safe_radius(self, x, harnack=False):
        """Radius of a disk around x on which the implicit h stays positive
        (harnack=True: the Harnack radius alone)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        out = np.zeros(2)
        rc = lib().oracle_safe_radius(C.byref(self._s), _ptr(x, C.c_double), _ptr(out, C.c_double))
        assert rc == 0
        return float(out[1 if harnack else 0])

    def adjoint_grad(self, code, bary, wq, ref, W, seed):
        """Adjoint formulation (Appendix B) of the squared-loss shape
        derivative over the domain, uref(x) = c + b.x + x^T A x with
        ref = (c, b, A): boundary samples (prim * 2 + flip, barycentrics
        b1 (, b2), quadrature weights), W walks each.  Returns (grad,
        per-walk adjoint estimates at the offset points, per-walk offset
        means, per-walk step counts), the records S x W."""
        D = self.scene.dim
        code = np.ascontiguousarray(code, dtype=np.int32)
        S = len(code)
        bary = np.ascontiguousarray(np.asarray(bary, float).reshape(S, D - 1))
        wq = np.ascontiguousarray(wq, dtype=np.float64)
        ref = np.ascontiguousarray(ref, dtype=np.float64)
        assert ref.size == 1 + D + D * D
        g = np.zeros(self.scene.N)
        lam, uoff, st = np.zeros((S, W)), np.zeros((S, W)), np.zeros((S, W), np.int64)
        rc = lib().oracle_adjoint_grad(C.byref(self._s), _ptr(code, C.c_int32), _ptr(bary, C.c_double),
                                       _ptr(wq, C.c_double), C.c_int64(S), _ptr(ref, C.c_double), W, seed,
                                       _ptr(g, C.c_double), _ptr(lam, C.c_double), _ptr(uoff, C.c_double),
                                       _ptr(st, C.c_int64), self.threads)
        if rc != 0:
            raise ValueError("oracle_adjoint_grad: invalid arguments")
        return g, lam, uoff, st

    def band_grad(self, X, coef, eps_band):
        """Band term on an implicit boundary: (sum over the points in the band
        of coef_p (dh/dpi)/|grad h|, region per point: 1 band, 2 rest of the
        domain, 0 outside)."""
        X = self._X(X)
        coef = np.ascontiguousarray(coef, dtype=np.float64)
        g = np.zeros(3 * len(self.scene.mono))
        m = np.zeros(len(X), np.int32)
        rc = lib().oracle_band_grad(C.byref(self._s), _ptr(X, C.c_double), C.c_int64(len(X)),
                                    _ptr(coef, C.c_double), C.c_double(eps_band), _ptr(g, C.c_double),
                                    _ptr(m, C.c_int32))
        assert rc == 0
        return g, m

    def walk_records_cv(self, X, W, seed, cv, instance=0):
        """Differential walks with the control variate: per-walk records
        (run, xoff, uoff plain, uoff_cv, target, u, prim) and per nested walk
        (S, alive, xstop, y, rho, d)."""
        X = self._X(X)
        P = X.shape[0]
        self._starts(None, P)
        K = int(self.scene.K)
        walk = np.zeros(P * W * 9)
        nested = np.zeros(P * W * K * 10)
        rc = lib().oracle_walk_records_cv(C.byref(self._s), _cvref(cv), _ptr(X, C.c_double), P, W,
                                          seed, instance, _ptr(walk, C.c_double),
                                          _ptr(nested, C.c_double), self.threads)
        assert rc == 0
        w = walk.reshape(P, W, 9)
        n = nested.reshape(P, W, K, 10)
        return dict(run=w[..., 0].astype(np.int32), xoff=w[..., 1:4], uoff=w[..., 4],
                    uoff_cv=w[..., 5], target=w[..., 6], u=w[..., 7], prim=w[..., 8].astype(np.int32),
                    S=n[..., 0], alive=n[..., 1].astype(np.int32),
                    xstop=n[..., 2:5], y=n[..., 5:8], rho=n[..., 8], d=n[..., 9])


class Net:
    """The control-variate network of the oracle: frequencies B (F x dim) and
    parameters theta (THETA_SIZE); q is the probability of running the nested
    walks.  Arrays are kept alive for the C structure."""

    def __init__(self, dim, B, theta, q=1.0):
        self.dim = int(dim)
        self.B = np.ascontiguousarray(B, dtype=np.float64).reshape(-1, self.dim)
        self.theta = np.ascontiguousarray(theta, dtype=np.float64)
        assert self.theta.size == theta_size()
        self.q = float(q)
        self._c = OracleCV()
        self._c.F = self.B.shape[0]
        self._c.B = _ptr(self.B, C.c_double)
        self._c.theta = _ptr(self.theta, C.c_double)
        self._c.q = self.q

    def eval(self, X):
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, self.dim)
        n = X.shape[0]
        N, G, Lp = np.zeros(n), np.zeros(n * self.dim), np.zeros(n)
        rc = lib().oracle_mlp_eval(self.dim, self.B.shape[0], _ptr(self.B, C.c_double),
                                   _ptr(self.theta, C.c_double), _ptr(X, C.c_double), n,
                                   _ptr(N, C.c_double), _ptr(G, C.c_double), _ptr(Lp, C.c_double))
        assert rc == 0
        return N, G.reshape(n, self.dim), Lp

    def loss_grad(self, X, T, w=None):
        X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, self.dim)
        T = np.ascontiguousarray(T, dtype=np.float64)
        w = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
        g = np.zeros(theta_size())
        L = np.zeros(1)
        rc = lib().oracle_mlp_loss_grad(self.dim, self.B.shape[0], _ptr(self.B, C.c_double),
                                        _ptr(self.theta, C.c_double), _ptr(X, C.c_double),
                                        _ptr(T, C.c_double), _ptr(w, C.c_double), X.shape[0],
                                        _ptr(L, C.c_double), _ptr(g, C.c_double))
        assert rc == 0
        return float(L[0]), g


def _vjp(self, X, Nbar, Lbar=None):
    """d/dtheta sum_i (Nbar_i N(x_i) + Lbar_i Lap N(x_i))."""
    X = np.ascontiguousarray(X, dtype=np.float64).reshape(-1, self.dim)
    Nb = np.ascontiguousarray(Nbar, dtype=np.float64)
    Lb = None if Lbar is None else np.ascontiguousarray(Lbar, dtype=np.float64)
    g = np.zeros(theta_size())
    rc = lib().oracle_mlp_vjp(self.dim, self.B.shape[0], _ptr(self.B, C.c_double),
                              _ptr(self.theta, C.c_double), _ptr(X, C.c_double), _ptr(Nb, C.c_double),
                              _ptr(Lb, C.c_double), X.shape[0], _ptr(g, C.c_double))
    assert rc == 0
    return g


Net.vjp = _vjp


def _cvref(cv):
    return C.byref(cv._c) if cv is not None else None


def theta_size():
    return int(lib().oracle_mlp_theta_size())


def adam(theta, m, v, g, lr, beta1, beta2, eps, step):
    """One Adam step in place on float64 arrays."""
    for a in (theta, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = np.ascontiguousarray(g, dtype=np.float64)
    lib().oracle_adam(theta.size, _ptr(theta, C.c_double), _ptr(m, C.c_double),
                      _ptr(v, C.c_double), _ptr(g, C.c_double), lr, beta1, beta2, eps, step)


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, np.uint32)
    lib().oracle_philox(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(o, C.c_uint32))
    return o


def green(dim, sigma, r, R):
    return lib().oracle_green(dim, sigma, r, R)


def poisson_scale(dim, sigma, R):
    return lib().oracle_poisson_scale(dim, sigma, R)


def green_mass(dim, sigma, R):
    return lib().oracle_green_mass(dim, sigma, R)


def neumann_weight(dim, sigma, r, R):
    return lib().oracle_neumann_weight(dim, sigma, r, R)
