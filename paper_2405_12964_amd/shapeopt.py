"""The paper's shape-optimisation loop for mesh vertices (Sec. 6, Sec. 7.2):
forward walks at the measurement points, the squared loss against a
reference, reverse-mode differential walks for dJ/dx of every movable
vertex, one vector-Adam step on the Laplacian-preconditioned variable
(dwos_opt_step), and the boundary moved to the new vertices (BVH refit),
with the walks per point annealed by eq. (update_rule) and the movable part
remeshed periodically (dwos_remesh; the paper remeshes every 100
iterations).

Orchestration only: every walk, solve, update and remesh runs in the
library.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .opt import LargeSteps
from .solver import Solver, make_problem


def wpp(W0: int, WT: int, t: int, T: int) -> int:
    """Walks per point at iteration t of T (eq. update_rule, denominator T)."""
    return int(round(W0 * math.exp(math.log(WT / W0) * t / T)))


def vertex_jacobian(nv: int, dim: int, movable: np.ndarray):
    """CSR of dv_i/dpi for pi = the coordinates of the movable vertices in
    vertex order (pi[dim k + c] = coordinate c of the k-th movable vertex)."""
    mv = np.asarray(movable, bool)
    counts = np.where(mv, dim, 0).astype(np.int64)
    rowptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    k = np.cumsum(mv) - 1
    pid = (np.repeat(k[mv], dim) * dim + np.tile(np.arange(dim), int(mv.sum()))).astype(np.int32)
    vel = np.tile(np.eye(dim), (int(mv.sum()), 1))
    return int(mv.sum()) * dim, rowptr, pid, vel


class VertexShapeOptimizer:
    """Optimise the movable vertices of a scene's Dirichlet boundary."""

    def __init__(self, scene, movable, lam=20.0, lr=1e-3, W0=8, WT=64, T=100, precision="fp32",
                 device="cuda", cg_tol=1e-7, remesh_every=0, remesh_len=None, remesh_iters=5):
        self.scene, self.dim = scene, scene.dim
        self.device, self.lam = device, lam
        self.solver = Solver(scene.dim, precision)
        self.solver.set_problem(make_problem(scene.sigma, scene.eps, scene.delta, scene.K, scene.kmax,
                                             scene.rr, scene.src_c0, scene.gauss, scene.bc, scene.dim))
        self.lr, self.W0, self.WT, self.T = lr, W0, WT, T
        # relative residual of the two solves: far below the gradient noise
        # of a few walks per point
        self.cg_tol = cg_tol
        self.t = 0
        mv = np.asarray(movable, bool)
        if remesh_len is None:
            P = np.asarray(scene.prims)
            e = P[mv[P].all(1)]
            e = np.concatenate([e[:, [k, (k + 1) % self.dim]] for k in range(self.dim)]) if self.dim == 3 else e
            remesh_len = float(np.linalg.norm(scene.V[e[:, 0]] - scene.V[e[:, 1]], axis=1).mean()) if len(e) else 0.0
        self.remesh_every, self.remesh_len, self.remesh_iters = remesh_every, remesh_len, remesh_iters
        self._load(np.asarray(scene.V, float), np.asarray(scene.prims, np.int32), np.asarray(scene.label, np.int32),
                   np.asarray(scene.gvert, float), mv)

    def _load(self, V, P, label, gvert, mv):
        """(Re)build the boundary, the vertex Jacobian and the optimiser for a
        mesh; the optimiser's moments start from zero."""
        self.V, self.P, self.label, self.gvert, self.mv = V, P, label, gvert, mv
        self.solver.set_boundary(V, P, label, gvert)
        N, rowptr, pid, vel = vertex_jacobian(len(V), self.dim, mv)
        self.solver.set_parameters(N, rowptr, pid, vel)
        self.x = torch.tensor(V, dtype=torch.float64, device=self.device).contiguous()
        self.idx = torch.tensor(np.nonzero(mv)[0], dtype=torch.int64, device=self.device)
        self.opt = LargeSteps(self.dim, len(V), P, self.lam, mv.astype(np.int32))
        self.opt.reset(self.x)
        self.gx = torch.zeros_like(self.x)

    def remesh(self, target=None, iters=None):
        """Remesh the primitives that touch a movable vertex toward edge
        length ``target`` (dwos_remesh); fixed vertices keep their place, the
        rest of the boundary is carried over.  The remeshed primitives must
        share one label with restricted data.  Restarts the optimiser's
        moments on the new mesh."""
        from .remesh import remesh as _remesh
        target = self.remesh_len if target is None else target
        iters = self.remesh_iters if iters is None else iters
        X = self.x.cpu().numpy()
        P, mv, lab = self.P, self.mv, self.label
        touch = mv[P].any(1)
        labs = np.unique(lab[touch])
        if len(labs) != 1:
            raise ValueError("remesh: the movable primitives must share one label")
        if self.scene.bc[int(labs[0])].get("kind", "restricted") != "restricted":
            raise ValueError("remesh: mapped boundary data is not carried over")
        used = np.unique(P[touch])
        loc = -np.ones(len(X), np.int64)
        loc[used] = np.arange(len(used))
        V2, P2, src = _remesh(X[used], loc[P[touch]], target, iters, fixed=~mv[used])
        # vertices of the untouched primitives: kept ones are found through
        # src, the others appended
        rest = P[~touch]
        newidx = -np.ones(len(X), np.int64)
        kept = src >= 0
        newidx[used[src[kept]]] = np.nonzero(kept)[0]
        only = np.setdiff1d(np.unique(rest), used) if len(rest) else np.zeros(0, np.int64)
        newidx[only] = len(V2) + np.arange(len(only))
        assert np.all(newidx[rest] >= 0) if len(rest) else True
        Vn = np.concatenate([V2, X[only]])
        Pn = np.concatenate([P2, newidx[rest]]).astype(np.int32)
        labn = np.concatenate([np.full(len(P2), labs[0], np.int32), lab[~touch]])
        mvn = np.zeros(len(Vn), bool)
        mvn[:len(V2)] = True
        mvn[np.nonzero(kept)[0]] = mv[used[src[kept]]]
        gv = np.zeros(len(Vn))
        gv[len(V2):] = self.gvert[only]
        self._load(Vn, Pn, labn, gv, mvn)

    def step(self, X: torch.Tensor, uref: torch.Tensor, seed: int):
        """One iteration; returns (loss from the forward walks, W used, CG
        iterations of the two solves).  Every ``remesh_every`` iterations
        (0: never) the movable part is remeshed first."""
        if self.remesh_every and self.t > 0 and self.t % self.remesh_every == 0:
            self.remesh()
        W = wpp(self.W0, self.WT, self.t, self.T)
        u, _ = self.solver.solve(X, W, 2 * seed, var=False)
        w = (u - uref).contiguous()
        g, _ = self.solver.grad(X, w, W, 2 * seed + 1, u_mean=False)
        self.gx.zero_()
        self.gx[self.idx] = g.view(-1, self.dim)
        its = self.opt.step(self.gx, self.x, lr=self.lr, tol=self.cg_tol)
        self.solver.update_vertices(self.x)
        self.t += 1
        return 0.5 * float(((u - uref) ** 2).sum()), W, its


class ImplicitShapeOptimizer:
    """Curve inflation on an implicit boundary (Sec. 7.4): the monopoles
    (a_n, p_n) of h = c + sum_n a_n / |x - p_n| fitted so that the height
    field matches a reference uref at the pixel centres X (each of area dA)
    over the whole image, the height being u inside the domain and 0
    outside it.

    The derivative takes the paper's two parts: the volume term over the
    pixels inside the domain beyond the band (squared-loss U-statistic, W
    walks per pixel in one batch), and the band term (one-sided band of
    width eps_band, weight dA / eps_band).  A pixel that the boundary sweeps
    over trades its outside loss uref^2/2 for l(u) = (u - uref)^2/2, so the
    band integrand is l(u) - uref^2/2 = u^2/2 - u uref, with u at the band
    pixels from W forward walks (u^2 taken as mean^2 minus the variance of
    the mean, which is unbiased).  With zero boundary data this term is of
    the order of the band width.  After each Adam step on the 3n
    coordinates the scales are kept >= a_min and the new monopoles are
    uploaded (dwos_set_implicit)."""

    def __init__(self, scene, X: torch.Tensor, uref: torch.Tensor, dA: float, eps_band: float,
                 lr=2e-3, W=4, a_min=1e-3, precision="fp32"):
        self.solver = Solver.from_scene(scene, precision)
        # the band pixels' forward walks run on a second context and stream
        # (default priority), overlapping the differential walks: the two
        # launches are small and independent given the monopoles
        self.band_stream = torch.cuda.Stream(device=X.device)
        self.band_solver = Solver.from_scene(scene, precision, stream=self.band_stream)
        self.c = float(scene.mono_c)
        self.X, self.uref, self.dA, self.eps_band = X, uref, float(dA), float(eps_band)
        self.W, self.a_min = int(W), float(a_min)
        self.pi = torch.tensor(np.asarray(scene.mono, float).ravel(), dtype=torch.float64, device=X.device,
                               requires_grad=True)
        self.opt = torch.optim.Adam([self.pi], lr=lr)
        self._zero = torch.zeros(X.shape[0], dtype=torch.float64, device=X.device)
        self.region = None
        self.t = 0

    @property
    def mono(self) -> np.ndarray:
        return self.pi.detach().view(-1, 3).cpu().numpy()

    def regions(self) -> torch.Tensor:
        """Per pixel: 0 outside the domain, 1 in the band, 2 inside beyond it."""
        return self.solver.implicit_band_grad(self.X, self._zero, self.eps_band, want_mask=True)[1]

    def step(self, seed: int):
        """One iteration; returns (image loss, pixels inside beyond the band)."""
        region = self.regions()
        inner = torch.nonzero(region == 2).squeeze(1)
        band = torch.nonzero(region == 1).squeeze(1)
        out = self.uref[region == 0]
        main = torch.cuda.current_stream(self.X.device)
        if band.numel():
            Xb = self.X[band].contiguous()
            self.band_stream.wait_stream(main)
            with torch.cuda.stream(self.band_stream):
                ub, vb = self.band_solver.solve(Xb, self.W, (seed * 0x9E3779B1 + 0x7F4A7C15) & 0xFFFFFFFF)
        L, gd, _ = self.solver.grad_sqloss(self.X[inner].contiguous(), self.uref[inner].contiguous(), self.W,
                                           self.W, seed)
        grad = self.dA * gd
        lb = 0.0
        if band.numel():
            main.wait_stream(self.band_stream)
            for t in (Xb, ub, vb):
                t.record_stream(main)
            ub_ref = self.uref[band]
            coef = (self.dA / self.eps_band) * (0.5 * (ub * ub - vb) - ub * ub_ref)
            self.solver.implicit_band_grad(Xb, coef.contiguous(), self.eps_band, grad=grad)
            lb = 0.5 * float(((ub - ub_ref) ** 2).sum())
        loss = self.dA * (float(L) + lb + 0.5 * float((out * out).sum()))
        self.pi.grad = grad
        self.opt.step()
        with torch.no_grad():
            self.pi.view(-1, 3)[:, 0].clamp_(min=self.a_min)
        mono = self.mono
        self.solver.set_implicit(mono, self.c)
        self.band_solver.set_implicit(mono, self.c)
        self.region = region
        self.t += 1
        return loss, int(inner.numel())
