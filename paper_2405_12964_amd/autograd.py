"""torch.autograd integration: u(X; pi) with a differential-walk backward.

forward(pi)   : move the boundary to V(pi) = V_base + J pi and refit the BVH
                (library kernels), then estimate u at the query points with W
                forward walks (Algorithm 1) from Philox stream `seed`.
backward(g_u) : reverse mode sum_p g_u[p] * udot(x_p) (Sec. 4, eq.
                (functional_deriv), domain term) with one differential walk
                per (point, walk) (Algorithm 2) from a different stream
                `seed_bwd`.  Because the walks of the forward and backward
                passes are independent, a loss gradient that multiplies them
                (e.g. the squared loss, eq. (squared_loss_deriv)) is the
                uncorrelated product estimator of Sec. 5.3, which is unbiased.
"""
from __future__ import annotations

import torch

from .solver import Solver


class ShapeModel:
    """A Solver whose vertices are linear in the parameters:
    V(pi) = V_base + J pi, with J the Jacobian given to dwos_set_parameters."""

    def __init__(self, scene, precision: str = "fp32", device="cuda"):
        self.solver = Solver.from_scene(scene, precision)
        self.V_base = torch.as_tensor(scene.V_base, dtype=torch.float64, device=device).contiguous()
        self.N = int(scene.N)
        self.version = 0
        self._pi = None

    def apply(self, pi: torch.Tensor):
        """Move the boundary to V(pi) (device kernels: V = V_base + J pi, refit)."""
        pi = pi.detach().to(torch.float64).contiguous()
        if self._pi is not None and self._pi.shape == pi.shape and torch.equal(self._pi, pi):
            return
        self.solver.apply_parameters(self.V_base, pi)
        self._pi = pi.clone()
        self.version += 1


class DWoSFunction(torch.autograd.Function):
    """u = DWoSFunction.apply(pi, X, model, W, seed, W_bwd, seed_bwd)."""

    @staticmethod
    def forward(ctx, pi, X, model: ShapeModel, W: int, seed: int, W_bwd: int, seed_bwd: int):
        model.apply(pi)
        u, _ = model.solver.solve(X, W, seed, var=False)
        ctx.model = model
        ctx.save_for_backward(pi, X)
        ctx.W_bwd = int(W_bwd)
        ctx.seed_bwd = int(seed_bwd)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        pi, X = ctx.saved_tensors
        model = ctx.model
        model.apply(pi)   # no-op unless the boundary moved since forward
        w = grad_u.detach().to(torch.float64).contiguous()
        g, _ = model.solver.grad(X, w, ctx.W_bwd, ctx.seed_bwd, u_mean=False)
        return g.to(pi.dtype), None, None, None, None, None, None
