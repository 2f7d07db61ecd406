"""Shape-optimisation step of the paper's experiments -- TEST INFRASTRUCTURE ONLY.

Only ``tests/`` and ``bench.py``'s CPU baseline may import this module.  It is
a plain FP64 numpy/scipy statement of the optimiser the paper uses for mesh
vertices (Sec. 6, "Implementation and evaluation"; Sec. 7.2, "Gradient
preconditioning"):

* Vector Adam (Ling et al., "VectorAdam for rotation equivariant geometry
  optimization", NeurIPS 2022): the first moment per coordinate, the second
  moment per vertex from the squared norm of the vertex's gradient vector.
* The Laplacian preconditioner of Nicolet et al. ("Large steps in inverse
  rendering of geometry", TOG 2021): the optimiser works on
  u = (I + lambda L) x, L the combinatorial Laplacian of the mesh; the
  gradient with respect to u is (I + lambda L)^-1 dJ/dx, and after the
  update x = (I + lambda L)^-1 u.
* The step size is adapted with the largest second moment over all vertices
  (the suggestion of Nicolet et al. the paper follows): every vertex moves by
  lr m_hat / (sqrt(max v_hat) + eps).
* The walks-per-point schedule of eq. (update_rule),
  WPP_t = WPP_0 exp(log(WPP_T / WPP_0) t / T) (the printed denominator N is
  read as the iteration count T).

The linear solves use scipy's sparse direct solver (a library primitive).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import sparse
from scipy.sparse import linalg as spla


def mesh_edges(prims, movable=None):
    """Undirected edges of the primitives (segments, or the three sides of
    each triangle) whose two vertices are both movable, as a sorted unique
    (E, 2) array with i < j."""
    prims = np.asarray(prims, dtype=np.int64)
    D = prims.shape[1]
    if D == 2:
        e = prims.copy()
    else:
        e = np.concatenate([prims[:, [0, 1]], prims[:, [1, 2]], prims[:, [2, 0]]])
    e = np.sort(e, axis=1)
    e = e[e[:, 0] != e[:, 1]]
    if movable is not None:
        mv = np.asarray(movable, bool)
        e = e[mv[e[:, 0]] & mv[e[:, 1]]]
    return np.unique(e, axis=0)


def laplacian(nv, prims, movable=None):
    """Combinatorial Laplacian L = Deg - Adj over the movable-movable edges."""
    e = mesh_edges(prims, movable)
    A = sparse.coo_matrix((np.ones(2 * len(e)), (np.concatenate([e[:, 0], e[:, 1]]),
                                                  np.concatenate([e[:, 1], e[:, 0]]))),
                          shape=(nv, nv)).tocsr()
    deg = np.asarray(A.sum(axis=1)).ravel()
    return (sparse.diags(deg) - A).tocsr()


def system_matrix(nv, prims, lam, movable=None):
    """M = I + lambda L."""
    return (sparse.identity(nv, format="csr") + lam * laplacian(nv, prims, movable)).tocsc()


def wpp(W0, WT, t, T):
    """Walks per point at iteration t of T, rounded to the nearest integer."""
    return int(round(W0 * math.exp(math.log(WT / W0) * t / T)))


class LargeSteps:
    """Vector Adam on u = M x with the max second moment; M = I + lambda L."""

    def __init__(self, x, prims, lam, movable=None, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        x = np.asarray(x, dtype=np.float64)
        self.nv, self.D = x.shape
        self.M = system_matrix(self.nv, prims, lam, movable)
        self.solve = spla.factorized(self.M)
        self.u = self.M @ x
        self.x = x.copy()
        self.mv = np.ones(self.nv, bool) if movable is None else np.asarray(movable, bool)
        self.m = np.zeros_like(x)
        self.v = np.zeros(self.nv)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps

    def grad_u(self, gx):
        """dJ/du = M^-1 dJ/dx (M is symmetric)."""
        gx = np.asarray(gx, dtype=np.float64)
        return np.stack([self.solve(gx[:, c]) for c in range(self.D)], axis=1)

    def step(self, gx):
        """One step; fixed vertices (movable False) keep their moments at
        zero and do not move."""
        g = self.grad_u(gx)
        g[~self.mv] = 0.0
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * np.sum(g * g, axis=1)
        mhat = self.m / (1 - self.b1 ** self.t)
        vhat = self.v / (1 - self.b2 ** self.t)
        self.u = self.u - self.lr * mhat / (math.sqrt(vhat[self.mv].max()) + self.eps)
        self.x = np.stack([self.solve(self.u[:, c]) for c in range(self.D)], axis=1)
        return self.x
