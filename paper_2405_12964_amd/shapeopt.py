"""The paper's shape-optimisation loop for mesh vertices (Sec. 6, Sec. 7.2):
forward walks at the measurement points, the squared loss against a
reference, reverse-mode differential walks for dJ/dx of every movable
vertex, one vector-Adam step on the Laplacian-preconditioned variable
(dwos_opt_step), and the boundary moved to the new vertices (BVH refit),
with the walks per point annealed by eq. (update_rule).

Orchestration only: every walk, solve and update runs in the HIP library.
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
                 device="cuda", cg_tol=1e-7):
        self.scene, self.dim = scene, scene.dim
        self.mv = np.asarray(movable, bool)
        self.solver = Solver(scene.dim, precision)
        self.solver.set_boundary(scene.V, scene.prims, scene.label, scene.gvert)
        self.solver.set_problem(make_problem(scene.sigma, scene.eps, scene.delta, scene.K, scene.kmax,
                                             scene.rr, scene.src_c0, scene.gauss, scene.bc, scene.dim))
        N, rowptr, pid, vel = vertex_jacobian(scene.nv, scene.dim, self.mv)
        self.solver.set_parameters(N, rowptr, pid, vel)
        self.x = torch.tensor(scene.V, dtype=torch.float64, device=device).contiguous()
        self.idx = torch.tensor(np.nonzero(self.mv)[0], dtype=torch.int64, device=device)
        self.opt = LargeSteps(scene.dim, scene.nv, scene.prims, lam, self.mv.astype(np.int32))
        self.opt.reset(self.x)
        self.lr, self.W0, self.WT, self.T = lr, W0, WT, T
        # relative residual of the two solves: far below the gradient noise
        # of a few walks per point
        self.cg_tol = cg_tol
        self.t = 0
        self.gx = torch.zeros_like(self.x)

    def step(self, X: torch.Tensor, uref: torch.Tensor, seed: int):
        """One iteration; returns (loss from the forward walks, W used, CG
        iterations of the two solves)."""
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
