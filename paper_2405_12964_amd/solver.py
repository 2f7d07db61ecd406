"""Object wrapper over the C ABI: a Solver owns one dwos_ctx.

Host-side setup arrays are numpy; hot-path arrays are torch tensors on the
GPU (float64), passed to the library as device pointers on torch's current
stream.  No estimator arithmetic happens here.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np
import torch

from . import capi
from .capi import check


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _lp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _dev(t: Optional[torch.Tensor], dtype=torch.float64):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a GPU tensor")
    if t.dtype != dtype:
        raise ValueError(f"expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def make_problem(sigma=0.0, eps=1e-3, delta=1e-2, K=1, kmax=65536, rr=1, src_c0=0.0,
                 gauss=None, bc=None, dim=3, dudn=0) -> capi.dwos_problem:
    """Fill a dwos_problem.  bc: list of dicts kind='restricted' (c, b, A) or
    kind='mapped'; gauss: rows (amplitude, centre[dim], width); dudn: 0 the
    backward-difference normal derivative, 1 the offset-point gradient
    estimator (Laplace only)."""
    p = capi.dwos_problem()
    p.dudn = int(dudn)
    p.sigma, p.eps, p.delta = float(sigma), float(eps), float(delta)
    p.K, p.kmax, p.rr = int(K), int(kmax), int(rr)
    p.src_c0 = float(src_c0)
    g = np.zeros((0, dim + 2)) if gauss is None else np.asarray(gauss, float).reshape(-1, dim + 2)
    if g.shape[0] > capi.MAX_GAUSS:
        raise ValueError("too many gaussians")
    p.n_gauss = g.shape[0]
    for i in range(g.shape[0]):
        p.gauss[i][0] = g[i, 0]
        for k in range(dim):
            p.gauss[i][1 + k] = g[i, 1 + k]
        p.gauss[i][4] = g[i, 1 + dim]
    bc = bc or [dict(kind="restricted", c=0.0)]
    if len(bc) > capi.MAX_LABELS:
        raise ValueError("too many labels")
    p.n_labels = len(bc)
    for l, b in enumerate(bc):
        if b["kind"] == "mapped":
            p.bc[l].kind = 1
        else:
            p.bc[l].kind = 0
            p.bc[l].c = float(b.get("c", 0.0))
            bb = np.zeros(3)
            bv = np.asarray(b.get("b", np.zeros(dim)), float).ravel()
            bb[:bv.size] = bv
            A = np.zeros((3, 3))
            Av = np.asarray(b.get("A", np.zeros((dim, dim))), float)
            A[:Av.shape[0], :Av.shape[1]] = Av
            for i in range(3):
                p.bc[l].b[i] = bb[i]
            for i in range(9):
                p.bc[l].A[i] = A.ravel()[i]
    return p


class Solver:
    """One library context: a boundary, problem constants and parameters."""

    def __init__(self, dim: int, precision: str = "fp32", stream: Optional[torch.cuda.Stream] = None):
        self.dim = int(dim)
        self.precision = precision
        prec = capi.DWOS_FP32 if precision == "fp32" else capi.DWOS_FP64
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._ctx = C.c_void_p()
        check(capi.dwos_create(self.dim, prec, C.c_void_p(self.stream.cuda_stream), C.byref(self._ctx)))
        self.N = 0
        self.nv = 0

    def __del__(self):
        ctx = getattr(self, "_ctx", None)
        if ctx is not None and ctx.value:
            try:
                capi.dwos_destroy(ctx)
            except Exception:   # interpreter shutdown: module globals already gone
                pass
            self._ctx = None

    # ---- setup (host arrays) ------------------------------------------------
    def set_boundary(self, V, prims, label=None, gvert=None):
        V = np.ascontiguousarray(V, dtype=np.float64)
        prims = np.ascontiguousarray(prims, dtype=np.int32)
        lab = None if label is None else np.ascontiguousarray(label, dtype=np.int32)
        gv = None if gvert is None else np.ascontiguousarray(gvert, dtype=np.float64)
        check(capi.dwos_set_boundary(self._ctx, _dp(V), V.shape[0], _ip(prims), prims.shape[0],
                                     _ip(lab) if lab is not None else None,
                                     _dp(gv) if gv is not None else None))
        self.nv = V.shape[0]

    def update_vertices(self, V: torch.Tensor):
        check(capi.dwos_update_vertices(self._ctx, _dev(V)))

    def apply_parameters(self, V_base: torch.Tensor, pi: torch.Tensor):
        check(capi.dwos_apply_parameters(self._ctx, _dev(V_base), _dev(pi)))

    def set_problem(self, prob: capi.dwos_problem):
        check(capi.dwos_set_problem(self._ctx, C.byref(prob)))
        self._K = int(prob.K)

    def set_parameters(self, N, rowptr, pid, vel, bc_pid=None):
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        pid = np.ascontiguousarray(pid, dtype=np.int32)
        vel = np.ascontiguousarray(vel, dtype=np.float64)
        bcp = None if bc_pid is None else np.ascontiguousarray(bc_pid, dtype=np.int32)
        check(capi.dwos_set_parameters(self._ctx, int(N), _lp(rowptr), _ip(pid), _dp(vel),
                                       _ip(bcp) if bcp is not None else None))
        self.N = int(N)

    def set_reflecting(self, V, segs):
        """Fixed reflecting boundary (2D segments or 3D triangles over vertices
        V, the domain on each primitive's left normal); walks on stars from
        then on.  An empty ``segs`` removes it."""
        V = np.ascontiguousarray(V, dtype=np.float64).reshape(-1, self.dim)
        segs = np.ascontiguousarray(segs, dtype=np.int32).reshape(-1, self.dim)
        check(capi.dwos_set_reflecting(self._ctx, _dp(V), V.shape[0], _ip(segs), segs.shape[0]))

    def set_robin(self, mu: float, h=None):
        """Robin condition du/dn - mu u = h on the reflecting boundary (n into
        the domain); h a restricted field dict(c=, b=, A=) or None."""
        hb = None
        if h is not None:
            hb = make_problem(bc=[h], dim=self.dim).bc[0]
        check(capi.dwos_set_robin(self._ctx, float(mu), C.byref(hb) if hb is not None else None))

    def set_start_segments(self, seg):
        """Per query point of the following calls: the reflecting primitive it
        lies on (domain on its left normal) or -1; None clears."""
        if seg is None:
            check(capi.dwos_set_start_segments(self._ctx, None, 0))
            return
        seg = np.ascontiguousarray(seg, dtype=np.int32)
        check(capi.dwos_set_start_segments(self._ctx, _ip(seg), seg.shape[0]))

    def reflect_query(self, X, dirs, cap, on, nin):
        """Per row: (silhouette distance capped at cap, first ray hit t (cap if
        none), hit primitive or -1) on the reflecting boundary; X, dirs and
        nin are rows of the context's dimension."""
        X = self._X(X)
        n = X.shape[0]
        out = torch.empty(n, 3, dtype=torch.float64, device=X.device)
        check(capi.dwos_reflect_query(self._ctx, _dev(X), _dev(dirs), _dev(cap), _dev(on, torch.int32),
                                      _dev(nin), n, _dev(out)))
        return out

    def eval_reflect_weight(self, r, R, sigma):
        w = torch.empty_like(r)
        check(capi.dwos_eval_reflect_weight(self._ctx, _dev(r), _dev(R), r.numel(), float(sigma), _dev(w)))
        return w

    def set_implicit(self, mono, c):
        """Implicit boundary: the zero set of c + sum_n a_n / |x - p_n| (rows
        (a_n, p_nx, p_ny) of ``mono``); the parameters become the 3n monopole
        coordinates.  An empty ``mono`` removes it."""
        mono = np.ascontiguousarray(mono, dtype=np.float64).reshape(-1, 3)
        check(capi.dwos_set_implicit(self._ctx, _dp(mono), mono.shape[0], float(c)))
        self.N = 3 * mono.shape[0]

    def implicit_band_grad(self, X, coef, eps_band, grad=None, want_mask=False):
        """Adds, over the points of X in the band next to the implicit
        boundary (first-order distance h/|grad h| below eps_band), coef_p
        times the normal velocity (dh/dpi)/|grad h| at the point to ``grad``
        (a new zero vector if None).  Returns grad, or (grad, region) with
        region 1 in the band, 2 elsewhere in the domain, 0 outside."""
        X = self._X(X)
        if grad is None:
            grad = torch.zeros(self.N, dtype=torch.float64, device=X.device)
        mask = torch.empty(X.shape[0], dtype=torch.int32, device=X.device) if want_mask else None
        check(capi.dwos_implicit_band_grad(self._ctx, _dev(X), X.shape[0], _dev(coef), float(eps_band), _dev(grad),
                                           _dev(mask, torch.int32) if mask is not None else None))
        return (grad, mask) if want_mask else grad

    @classmethod
    def from_scene(cls, scene, precision: str = "fp32", V=None, stream=None) -> "Solver":
        """Configure from a scene description (attributes as in ``scenes.Scene``)."""
        s = cls(scene.dim, precision, stream)
        mono = getattr(scene, "mono", None)
        if mono is not None and len(mono) > 0:
            s.set_implicit(mono, scene.mono_c)
        else:
            s.set_boundary(scene.V if V is None else V, scene.prims, scene.label, scene.gvert)
        if getattr(scene, "nsegs", None) is not None and len(scene.nsegs) > 0:
            s.set_reflecting(scene.NV, scene.nsegs)
            if getattr(scene, "robin_mu", 0.0) > 0 or getattr(scene, "robin_h", None) is not None:
                s.set_robin(scene.robin_mu, scene.robin_h)
        s.set_problem(make_problem(scene.sigma, scene.eps, scene.delta, scene.K, scene.kmax,
                                   scene.rr, scene.src_c0, scene.gauss, scene.bc, scene.dim,
                                   getattr(scene, "dudn", 0)))
        if scene.N > 0 and scene.rowptr is not None and (mono is None or len(mono) == 0):
            s.set_parameters(scene.N, scene.rowptr, scene.pid, scene.vel, scene.bc_pid)
        return s

    # ---- hot path (device tensors) -----------------------------------------
    def _X(self, X: torch.Tensor):
        if X.dim() != 2 or X.shape[1] != self.dim:
            raise ValueError(f"points must be (P, {self.dim})")
        return X

    def solve(self, X, W, seed, var=True, stats=False):
        X = self._X(X)
        P = X.shape[0]
        m = torch.empty(P, dtype=torch.float64, device=X.device)
        v = torch.empty(P, dtype=torch.float64, device=X.device) if var else None
        st = capi.dwos_stats() if stats else None
        check(capi.dwos_solve(self._ctx, _dev(X), P, int(W), int(seed), _dev(m), _dev(v),
                              C.byref(st) if st is not None else None))
        return (m, v, st.as_dict()) if stats else (m, v)

    def solve_noalloc(self, X, W, seed, u_mean: torch.Tensor, u_var: Optional[torch.Tensor] = None):
        """dwos_solve_noalloc into caller-provided outputs (no device
        allocation inside the call)."""
        X = self._X(X)
        check(capi.dwos_solve_noalloc(self._ctx, _dev(X), X.shape[0], int(W), int(seed), _dev(u_mean),
                                      _dev(u_var)))
        return u_mean, u_var

    def grad(self, X, w, W, seed, u_mean=True, stats=False):
        X = self._X(X)
        P = X.shape[0]
        g = torch.empty(self.N, dtype=torch.float64, device=X.device)
        um = torch.empty(P, dtype=torch.float64, device=X.device) if u_mean else None
        st = capi.dwos_stats() if stats else None
        check(capi.dwos_grad(self._ctx, _dev(X), P, _dev(w), int(W), int(seed), _dev(g), _dev(um),
                             C.byref(st) if st is not None else None))
        return (g, um, st.as_dict()) if stats else (g, um)

    def grad_sqloss(self, X, uref, W, B, seed, stats=False):
        X = self._X(X)
        P = X.shape[0]
        g = torch.empty(self.N, dtype=torch.float64, device=X.device)
        L = torch.empty(1, dtype=torch.float64, device=X.device)
        um = torch.empty(P, dtype=torch.float64, device=X.device)
        st = capi.dwos_stats() if stats else None
        check(capi.dwos_grad_sqloss(self._ctx, _dev(X), P, _dev(uref), int(W), int(B), int(seed),
                                    _dev(L), _dev(g), _dev(um), C.byref(st) if st is not None else None))
        return (L, g, um, st.as_dict()) if stats else (L, g, um)

    def jvp(self, X, W, seed, var=True, stats=False):
        X = self._X(X)
        P = X.shape[0]
        ud = torch.empty(P, self.N, dtype=torch.float64, device=X.device)
        uv = torch.empty(P, self.N, dtype=torch.float64, device=X.device) if var else None
        um = torch.empty(P, dtype=torch.float64, device=X.device)
        st = capi.dwos_stats() if stats else None
        check(capi.dwos_jvp(self._ctx, _dev(X), P, int(W), int(seed), _dev(ud), _dev(uv), _dev(um),
                            C.byref(st) if st is not None else None))
        return (ud, uv, um, st.as_dict()) if stats else (ud, uv, um)

    def walk_records(self, X, W, seed, mode=0, udot=False):
        X = self._X(X)
        P = X.shape[0]
        dev = X.device
        u = torch.empty(P * W, dtype=torch.float64, device=dev)
        steps = torch.empty(P * W, dtype=torch.int64, device=dev)
        prim = torch.empty(P * W, dtype=torch.int32, device=dev)
        uoff = torch.empty(P * W, dtype=torch.float64, device=dev)
        ud = torch.empty(P * W * self.N, dtype=torch.float64, device=dev) if (udot and mode == 1) else None
        check(capi.dwos_walk_records(self._ctx, _dev(X), P, int(W), int(seed), int(mode), _dev(u),
                                     _dev(steps, torch.int64), _dev(prim, torch.int32), _dev(uoff),
                                     _dev(ud)))
        out = dict(u=u.view(P, W), steps=steps.view(P, W), prim=prim.view(P, W), uoff=uoff.view(P, W))
        if ud is not None:
            out["udot"] = ud.view(P, W, self.N)
        return out

    def closest(self, X):
        X = self._X(X)
        out = torch.empty(X.shape[0], 8, dtype=torch.float64, device=X.device)
        check(capi.dwos_closest(self._ctx, _dev(X), X.shape[0], _dev(out)))
        return out

    def eval_ball_kernels(self, r, R, sigma):
        GB = torch.empty_like(r)
        al = torch.empty_like(r)
        check(capi.dwos_eval_ball_kernels(self._ctx, _dev(r), _dev(R), r.numel(), float(sigma),
                                          _dev(GB), _dev(al)))
        return GB, al

    # ---- batched instances ------------------------------------------------
    def batch_add_instance(self, V, prims, label, sigma, eps, delta) -> int:
        V = np.ascontiguousarray(V, dtype=np.float64)
        prims = np.ascontiguousarray(prims, dtype=np.int32)
        lab = None if label is None else np.ascontiguousarray(label, dtype=np.int32)
        idx = C.c_int32()
        check(capi.dwos_batch_add_instance(self._ctx, _dp(V), V.shape[0], _ip(prims), prims.shape[0],
                                           _ip(lab) if lab is not None else None, float(sigma),
                                           float(eps), float(delta), C.byref(idx)))
        return idx.value

    def batch_solve(self, X_all, P, W, seed, var=True, stats=False):
        X_all = self._X(X_all)
        Pn = np.ascontiguousarray(P, dtype=np.int64)
        tot = int(Pn.sum())
        if tot != X_all.shape[0]:
            raise ValueError("sum of P must equal the number of points")
        m = torch.empty(tot, dtype=torch.float64, device=X_all.device)
        v = torch.empty(tot, dtype=torch.float64, device=X_all.device) if var else None
        st = capi.dwos_stats() if stats else None
        check(capi.dwos_batch_solve(self._ctx, _dev(X_all), _lp(Pn), int(W), int(seed), _dev(m), _dev(v),
                                    C.byref(st) if st is not None else None))
        return (m, v, st.as_dict()) if stats else (m, v)

    def batch_set_parameters(self, index, N, rowptr=None, pid=None, vel=None):
        """Parameter Jacobian of instance ``index`` over its own vertices
        (CSR by vertex, as set_parameters); its parameters follow those of
        the instances before it in batch_grad's output."""
        rp = None if rowptr is None else np.ascontiguousarray(rowptr, dtype=np.int64)
        pd = None if pid is None else np.ascontiguousarray(pid, dtype=np.int32)
        vl = None if vel is None else np.ascontiguousarray(vel, dtype=np.float64)
        check(capi.dwos_batch_set_parameters(self._ctx, int(index), int(N), _lp(rp) if rp is not None else None,
                                             _ip(pd) if pd is not None else None,
                                             _dp(vl) if vl is not None else None))
        self._batch_N = getattr(self, "_batch_N", {})
        self._batch_N[int(index)] = int(N)

    def batch_grad(self, X_all, P, w, W, seed, u_mean=True, stats=False):
        """Reverse mode over every instance in one launch: the gradient with
        respect to all instances' parameters, instance by instance."""
        X_all = self._X(X_all)
        Pn = np.ascontiguousarray(P, dtype=np.int64)
        tot = int(Pn.sum())
        if tot != X_all.shape[0]:
            raise ValueError("sum of P must equal the number of points")
        N = sum(getattr(self, "_batch_N", {}).values())
        g = torch.empty(max(1, N), dtype=torch.float64, device=X_all.device)
        um = torch.empty(tot, dtype=torch.float64, device=X_all.device) if u_mean else None
        st = capi.dwos_stats() if stats else None
        check(capi.dwos_batch_grad(self._ctx, _dev(X_all), _lp(Pn), _dev(w), int(W), int(seed), _dev(g), _dev(um),
                                   C.byref(st) if st is not None else None))
        g = g[:N]
        return (g, um, st.as_dict()) if stats else (g, um)

    def adjoint_grad(self, code, bary, wq, uref, W, seed, records=False, stats=False):
        """Adjoint formulation (Appendix B) of the derivative of
        J = int_Omega 1/2 (u - uref)^2, uref = (c, b, A) the quadratic
        c + b.x + x^T A x, from boundary samples (GPU tensors: code int32
        prim * 2 + flip, bary S x (dim - 1), wq quadrature weights) with W
        walks each.  Returns grad, plus (lambda, uoff) S x W records if
        ``records``, plus the stats dict if ``stats``."""
        c0, b, A = uref
        q = capi.dwos_quad()
        q.c = float(c0)
        bb = np.zeros(3)
        bb[:self.dim] = np.asarray(b if b is not None else np.zeros(self.dim), float).ravel()[:self.dim]
        AA = np.zeros((3, 3))
        if A is not None:
            AA[:self.dim, :self.dim] = np.asarray(A, float).reshape(self.dim, self.dim)
        for i in range(3):
            q.b[i] = bb[i]
        for i in range(9):
            q.A[i] = AA.ravel()[i]
        S = int(code.shape[0])
        dev = code.device
        g = torch.empty(max(1, self.N), dtype=torch.float64, device=dev)
        lam = torch.empty((S, W), dtype=torch.float64, device=dev) if records else None
        uo = torch.empty((S, W), dtype=torch.float64, device=dev) if records else None
        st = capi.dwos_stats() if stats else None
        check(capi.dwos_adjoint_grad(self._ctx, _dev(code, torch.int32), _dev(bary), _dev(wq), S, C.byref(q), int(W),
                                     int(seed), _dev(g), _dev(lam), _dev(uo), C.byref(st) if st is not None else None))
        g = g[:self.N]
        out = (g,) + ((lam, uo) if records else ()) + ((st.as_dict(),) if stats else ())
        return out if len(out) > 1 else g

    def autotune(self, X, W, seed=0, P=None, cache=True, grad=False):
        """Autotune the walk kernels' scheduling knobs (dwos_autotune) on forward
        solves of X: a prefix of the points on a single-scene context, the
        whole batch (P: points per instance) on a batch context; grad=True
        also times a reverse-mode call with unit weights on the same points
        (DWOS_TUNE_GRAD, needs parameters).  Returns (tuning dict, [ms under
        the setting at the call, ms under the chosen one]); both are -1 when
        the process-wide table already held a setting for this scene-size
        bucket (cache=True)."""
        X = self._X(X)
        counts = [X.shape[0]] if P is None else [int(p) for p in P]
        Pa = (C.c_int64 * len(counts))(*counts)
        t = capi.dwos_tuning()
        ms = (C.c_double * 2)()
        check(capi.dwos_autotune(self._ctx, _dev(X), Pa, int(W), int(seed),
                                 (capi.DWOS_TUNE_CACHE if cache else 0) | (capi.DWOS_TUNE_GRAD if grad else 0),
                                 C.byref(t), ms))
        return t.as_dict(), [ms[0], ms[1]]

    def get_tuning(self) -> dict:
        t = capi.dwos_tuning()
        check(capi.dwos_get_tuning(self._ctx, C.byref(t)))
        return t.as_dict()

    def set_tuning(self, **kw):
        """Change some of the knobs (variant, park, tail, chunk, stage_nodes)."""
        t = capi.dwos_tuning(**{**self.get_tuning(), **kw})
        check(capi.dwos_set_tuning(self._ctx, C.byref(t)))

    def scene_info(self) -> dict:
        """Sizes of the BVH and primitive arrays and the LDS staging plan."""
        info = (C.c_int64 * 8)()
        check(capi.dwos_scene_info(self._ctx, info))
        keys = ["nodes", "node_bytes", "prim_bytes", "staged_nodes", "staged_prims", "prims", "vertices",
                "lds_bytes"]
        return {k: int(info[i]) for i, k in enumerate(keys)}

    def set_variant(self, v: int):
        check(capi.dwos_set_variant(self._ctx, int(v)))

    def set_seed_buffer(self, seed_dev: Optional[torch.Tensor]):
        """Use seed + seed_dev[0] (a 1-element int64 GPU tensor) in every later
        call, so that a captured graph replays with fresh streams."""
        self._seed_buf = seed_dev
        check(capi.dwos_set_seed_buffer(self._ctx, _dev(seed_dev, torch.int64) if seed_dev is not None else None))

    # ---- learned control variate of the nested walks ----------------------
    def attach_cv(self, net, q: float = 1.0):
        """Use net (a cv.Network, or None to detach) as the control variate of
        every later differential call; nested walks run with probability q."""
        self._cv = net
        check(capi.dwos_cv_attach(self._ctx, net.handle if net is not None else None, float(q)))

    def cv_beta(self) -> float:
        """Coefficient of the control variate in the next differential call."""
        b = C.c_double()
        check(capi.dwos_cv_beta(self._ctx, C.byref(b)))
        return b.value

    def cv_train(self, steps: int, batch: int, lr: float, seed: int):
        """Adam steps of the attached network on the last differential walks'
        records; returns the last step's loss (device float32 tensor)."""
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        check(capi.dwos_cv_train(self._ctx, int(steps), int(batch), float(lr), int(seed),
                                 C.c_void_p(loss.data_ptr())))
        return loss

    def cv_walk_records(self, X, W, seed):
        X = self._X(X)
        P = X.shape[0]
        K = self._K
        walk = torch.empty(P * W * 9, dtype=torch.float64, device=X.device)
        nested = torch.empty(P * W * K * 10, dtype=torch.float64, device=X.device)
        check(capi.dwos_cv_walk_records(self._ctx, _dev(X), P, int(W), int(seed), _dev(walk), _dev(nested)))
        w = walk.view(P, W, 9)
        n = nested.view(P, W, K, 10)
        return dict(run=w[..., 0].to(torch.int32), xoff=w[..., 1:4], uoff=w[..., 4], uoff_cv=w[..., 5],
                    target=w[..., 6], u=w[..., 7], prim=w[..., 8].to(torch.int32),
                    S=n[..., 0], alive=n[..., 1].to(torch.int32), xstop=n[..., 2:5],
                    y=n[..., 5:8], rho=n[..., 8], d=n[..., 9])

    def walk_timing(self, kind: int, reset=False):
        """(ms, launches, totals dict) of the walk kernels of one kind
        (0 forward, 1 differential) since the last reset."""
        ms = C.c_double()
        n = C.c_int64()
        st = capi.dwos_stats()
        check(capi.dwos_walk_timing(self._ctx, int(kind), 1 if reset else 0, C.byref(ms), C.byref(n),
                                    C.byref(st)))
        return ms.value, n.value, st.as_dict()
