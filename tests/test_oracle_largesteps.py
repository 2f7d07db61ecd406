"""Pins of the oracle's shape-optimisation step (vector Adam with the
Laplacian preconditioner and the max second moment; the walks-per-point
schedule of eq. update_rule).

* The Laplacian of a closed ring is circulant: M^-1 = (I + lambda L)^-1
  scales the Fourier mode k by 1 / (1 + lambda (2 - 2 cos(2 pi k / n))).
* The 3D combinatorial Laplacian of an icosphere: rows sum to zero, the
  diagonal is the vertex valence (5 or 6).
* Vector Adam is rotation equivariant: rotating every gradient rotates the
  update (the defining property of Ling et al.); with lambda = 0 and one
  vertex it is Adam on that vertex's vector with the norm's moment.
* A constant gradient moves every vertex by exactly lr per step in the
  first step (bias correction), along -g / |g|.
* The schedule hits its endpoints and is geometric.
"""
import math

import numpy as np
import pytest
import torch

import scenes
from oracle import largesteps as ls


def test_ring_fourier_modes():
    n, lam = 64, 7.0
    prims = np.stack([np.arange(n), (np.arange(n) + 1) % n], 1)
    M = ls.system_matrix(n, prims, lam)
    solve = __import__("scipy.sparse.linalg", fromlist=["x"]).factorized(M)
    i = np.arange(n)
    for k in (0, 1, 5, 31, 32):
        f = np.cos(2 * np.pi * k * i / n)
        expect = f / (1 + lam * (2 - 2 * np.cos(2 * np.pi * k / n)))
        assert np.allclose(solve(f), expect, rtol=1e-12, atol=1e-12)


def test_icosphere_laplacian_structure():
    V, F = scenes.icosphere(4)
    L = ls.laplacian(len(V), F)
    assert np.allclose(np.asarray(L.sum(axis=1)).ravel(), 0)
    deg = L.diagonal()
    assert set(np.unique(deg).astype(int)) == {5, 6}
    assert (deg == 5).sum() == 12
    # a non-movable vertex decouples: its row and column are zero in L
    mv = np.ones(len(V), bool)
    mv[0] = False
    L2 = ls.laplacian(len(V), F, mv)
    assert L2[0].nnz == 0 and L2[:, 0].nnz == 0


def _rot(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s], [s, c]])


def test_vector_adam_rotation_equivariance():
    n = 32
    th = 2 * np.pi * np.arange(n) / n
    x0 = np.stack([np.cos(th), np.sin(th)], 1)
    prims = np.stack([np.arange(n), (np.arange(n) + 1) % n], 1)
    rng = np.random.default_rng(0)
    G = rng.normal(size=(5, n, 2))
    Rm = _rot(0.7)
    a = ls.LargeSteps(x0, prims, 3.0, lr=0.01)
    b = ls.LargeSteps(x0 @ Rm.T, prims, 3.0, lr=0.01)
    for g in G:
        xa = a.step(g)
        xb = b.step(g @ Rm.T)
    assert np.allclose(xa @ Rm.T, xb, atol=1e-12)


def test_vector_adam_single_vertex_matches_norm_moment_adam():
    """lambda = 0, one vertex: u = x and the update is Adam on the vector
    with the second moment of |g|^2 (compare a scalar torch Adam run on |g|
    along a fixed direction)."""
    x0 = np.array([[0.3, -0.2]])
    opt = ls.LargeSteps(x0, np.zeros((0, 2), np.int64), 0.0, lr=0.05)
    d = np.array([0.6, 0.8])
    mags = [1.0, 0.5, 2.0, -1.0, 0.1]
    p = torch.zeros(1, dtype=torch.float64, requires_grad=True)
    tadam = torch.optim.Adam([p], lr=0.05, betas=(0.9, 0.999), eps=1e-8)
    for s in mags:
        x = opt.step(np.array([s * d]))
        tadam.zero_grad()
        p.grad = torch.tensor([s], dtype=torch.float64)
        tadam.step()
        assert np.allclose(x[0], x0[0] + p.item() * d, atol=1e-12)


def test_constant_gradient_first_step_moves_by_lr():
    n = 16
    th = 2 * np.pi * np.arange(n) / n
    x0 = np.stack([np.cos(th), np.sin(th)], 1)
    prims = np.stack([np.arange(n), (np.arange(n) + 1) % n], 1)
    opt = ls.LargeSteps(x0, prims, 5.0, lr=0.02, eps=0.0)
    g = np.tile([[3.0, -4.0]], (n, 1))
    # a constant field is in the Laplacian's kernel: M^-1 g = g, and x moves
    # rigidly by lr along -g/|g|
    x = opt.step(g)
    assert np.allclose(x - x0, -0.02 * g / 5.0, atol=1e-12)


def test_wpp_schedule():
    assert ls.wpp(2, 128, 0, 100) == 2
    assert ls.wpp(2, 128, 100, 100) == 128
    assert ls.wpp(2, 128, 50, 100) == 16
    w = [ls.wpp(4, 4096, t, 10) for t in range(11)]
    assert w == sorted(w) and w[5] == 128


def test_max_second_moment_sets_one_step_size():
    """lambda = 0, first step: m_hat = g and v_hat = |g|^2, so with the max
    second moment the vertex with the largest gradient moves by lr and the
    others by lr |g_i| / max |g| (per-vertex Adam would move all by lr)."""
    x0 = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    opt = ls.LargeSteps(x0, np.zeros((0, 2), np.int64), 0.0, lr=0.1, eps=0.0)
    g = np.array([[4.0, 0.0], [0.0, 1.0], [0.6, 0.8]])
    x = opt.step(g)
    assert np.allclose(np.linalg.norm(x - x0, axis=1), [0.1, 0.025, 0.025], atol=1e-12)
