"""Seeded synthetic scenes and query points for differential walk on spheres.

This module builds inputs only: boundary geometry, boundary-data and source
specifications, the parameter Jacobian dv/dpi of the boundary vertices, and
query points.  It holds none of the estimator's arithmetic, so both the FP64
oracle and the GPU library can consume the same inputs.

The paper's own scenes (bunny, pose mesh, toaster, heightfields, images) are
not available; these generators stand in for them with the shapes and sizes of
the paper's workloads (Sec. 6-7, Table 1):

* ``c1_polygon``   2D Laplace on a regular n-gon inscribed in a disk, parameter
                   = radius (Sec. 6.3 ablation-style 2D scene).
* ``c2_star``      2D screened Poisson on a Fourier star polygon with a Gaussian
                   source; 64 shape coefficients (Sec. 7 polyline examples).
* ``c3_icosphere`` 3D shape from diffusion: displaced icosphere inside a box,
                   radial-basis vertex displacement parameters (Sec. 7.2).
* ``c4_batch``     many C3-like instances of uneven size.

Every array is float64 / int32 / int64 numpy.  Vertex positions are linear in
the parameters: ``V(pi) = V_base + sum_j pi_j * J_j`` with the Jacobian stored
as CSR by vertex (``rowptr``, ``pid``, ``vel``).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

__all__ = [
    "Scene", "c1_polygon", "c2_star", "c3_icosphere", "c4_batch",
    "disk_polygon", "icosphere", "box_triangles", "sphere_scene",
    "shell_scene", "annulus_scene", "points_in_disk", "points_on_box_faces",
    "points_in_ball", "vertices_at", "lshape_scene", "half_disk_scene",
    "annulus_reflecting_scene", "points_in_lshape", "points_in_half_disk",
    "points_on_segments", "thermal_scene", "monopole_scene", "inflation_scene",
    "lprism_scene", "points_in_lprism", "box_wall_scene", "half_ball_scene",
    "points_in_half_ball", "points_on_triangles", "thermal3d_scene",
]


@dataclass
class Scene:
    """A Dirichlet screened-Poisson problem on an explicit boundary.

    Boundary data per label is either a restricted quadratic field
    ``g(x) = c + b.x + x^T A x`` (``kind='restricted'``) or values mapped from
    the reference surface, given per vertex and interpolated linearly over a
    primitive (``kind='mapped'``, values in ``gvert``).

    The source is ``f(x) = c0 + sum_i a_i exp(-|x - m_i|^2 / (2 s_i^2))`` with
    rows ``(a_i, m_i[dim], s_i)`` in ``gauss``.
    """
    dim: int
    V: np.ndarray                 # (nv, dim) float64 vertex positions
    prims: np.ndarray             # (np, dim) int32 vertex indices
    label: np.ndarray             # (np,) int32 boundary-data label
    bc: list                      # per label: dict(kind=..., c=, b=, A=)
    gvert: np.ndarray             # (nv,) float64 values for mapped labels
    sigma: float = 0.0
    eps: float = 1e-3
    delta: float = 1e-2
    K: int = 1
    kmax: int = 65536
    rr: int = 1
    src_c0: float = 0.0
    gauss: np.ndarray = field(default_factory=lambda: np.zeros((0, 4)))
    # parameters: dv_i/dpi_j as CSR by vertex
    N: int = 0
    rowptr: Optional[np.ndarray] = None   # (nv+1,) int64
    pid: Optional[np.ndarray] = None      # (nnz,) int32
    vel: Optional[np.ndarray] = None      # (nnz, dim) float64
    bc_pid: Optional[np.ndarray] = None   # (nv,) int32, -1 = none
    V_base: Optional[np.ndarray] = None   # V(pi) = V_base + J pi
    pi0: Optional[np.ndarray] = None      # parameter values giving V
    name: str = ""
    # reflecting part of the boundary: segments (2D) or triangles (3D) over
    # their own vertices, independent of the parameters; walks start on
    # primitive s with the domain on its left normal (2D: left of the
    # segment from its first to its second vertex; 3D: the side
    # (b - a) x (c - a) points to)
    NV: Optional[np.ndarray] = None       # (n_nv, dim) float64
    nsegs: Optional[np.ndarray] = None    # (n_ns, dim) int32
    # implicit Dirichlet boundary (2D): zero set of
    # h(x) = mono_c + sum_n a_n / |x - p_n|, rows (a_n, p_n); domain h > 0
    mono: Optional[np.ndarray] = None     # (n, 3) float64
    mono_c: float = -1.0
    # normal-derivative estimator of the differential walks: 0 backward
    # difference, 1 offset-point gradient estimator (Laplace only)
    dudn: int = 0
    # Robin condition du/dn - robin_mu u = h on the reflecting part (n into
    # the domain): robin_mu >= 0 and h a restricted field dict(c=, b=, A=)
    # (None: h = 0)
    robin_mu: float = 0.0
    robin_h: Optional[dict] = None

    @property
    def nv(self) -> int:
        return int(self.V.shape[0])

    @property
    def np_(self) -> int:
        return int(self.prims.shape[0])

    def with_(self, **kw) -> "Scene":
        d = dict(self.__dict__)
        d.update(kw)
        return Scene(**d)


def vertices_at(scene: Scene, pi: np.ndarray) -> np.ndarray:
    """Vertex positions for parameter vector ``pi`` (vertices are linear in pi)."""
    pi = np.asarray(pi, dtype=np.float64)
    nv = scene.nv
    rows = np.repeat(np.arange(nv), np.diff(scene.rowptr))
    V = scene.V_base.copy()
    np.add.at(V, rows, scene.vel * pi[scene.pid][:, None])
    return V


def _restricted(c=0.0, b=None, A=None, dim=2):
    b = np.zeros(dim) if b is None else np.asarray(b, float)
    A = np.zeros((dim, dim)) if A is None else np.asarray(A, float)
    return dict(kind="restricted", c=float(c), b=b, A=A)


def _mapped():
    return dict(kind="mapped")


def _dense_csr(J: np.ndarray):
    """CSR of a dense Jacobian J[nv, N, dim]."""
    nv, N, dim = J.shape
    rowptr = (np.arange(nv + 1, dtype=np.int64) * N)
    pid = np.tile(np.arange(N, dtype=np.int32), nv)
    vel = J.reshape(nv * N, dim).astype(np.float64)
    return rowptr, pid, vel


# --------------------------------------------------------------------------
# 2D geometry
# --------------------------------------------------------------------------

def disk_polygon(n: int, R: float = 1.0):
    """Regular n-gon with vertices R(cos 2 pi i/n, sin 2 pi i/n), CCW."""
    th = 2.0 * np.pi * np.arange(n) / n
    U = np.stack([np.cos(th), np.sin(th)], axis=1)
    prims = np.stack([np.arange(n), (np.arange(n) + 1) % n], axis=1).astype(np.int32)
    return R * U, U, prims


def c1_polygon(n: int = 128, R: float = 1.0, mapped: bool = False,
               eps: float = 1e-4, delta: float = 1e-3, sigma: float = 0.0,
               g: str = "x2-y2", K: int = 1) -> Scene:
    """Regular n-gon, one parameter pi = R with dv_i/dR = v_i / R.

    ``g='x2-y2'`` gives the harmonic field x^2 - y^2; ``g='one'`` gives g = 1.
    With ``mapped=True`` the field is sampled at the vertices and interpolated
    along edges instead of being restricted.
    """
    V, U, prims = disk_polygon(n, R)
    if g == "x2-y2":
        fld = _restricted(0.0, None, [[1.0, 0.0], [0.0, -1.0]], 2)
        gv = V[:, 0] ** 2 - V[:, 1] ** 2
    elif g == "one":
        fld = _restricted(1.0, None, None, 2)
        gv = np.ones(n)
    else:
        raise ValueError(g)
    bc = [_mapped() if mapped else fld]
    rowptr = np.arange(n + 1, dtype=np.int64)
    pid = np.zeros(n, dtype=np.int32)
    return Scene(dim=2, V=V, prims=prims, label=np.zeros(n, np.int32), bc=bc,
                 gvert=gv, sigma=sigma, eps=eps, delta=delta, K=K,
                 N=1, rowptr=rowptr, pid=pid, vel=U.copy(),
                 V_base=np.zeros_like(V), pi0=np.array([R]),
                 name=f"c1_polygon{n}{'_mapped' if mapped else ''}")


def points_in_disk(P: int, rmax: float, seed: int, centre=(0.0, 0.0)) -> np.ndarray:
    """P points area-uniform in the disk r < rmax."""
    rng = np.random.default_rng(seed)
    r = rmax * np.sqrt(rng.random(P))
    th = 2 * np.pi * rng.random(P)
    return np.stack([centre[0] + r * np.cos(th), centre[1] + r * np.sin(th)], axis=1)


def star_coefficients(seed: int, kmax: int = 32, scale: float = 0.02):
    """a_k, b_k ~ N(0, (scale/k)^2), k = 1..kmax; returned as [a_1..a_K, b_1..b_K]."""
    rng = np.random.default_rng(seed)
    k = np.arange(1, kmax + 1)
    a = rng.normal(0.0, scale / k)
    b = rng.normal(0.0, scale / k)
    return np.concatenate([a, b])


def c2_star(n: int = 4096, coef: Optional[np.ndarray] = None, coef_seed: int = 0,
            kmax: int = 32, sigma: float = 10.0, eps: float = 1e-3,
            delta: float = 1e-2, K: int = 1, source: bool = True) -> Scene:
    """Star polygon r(th) = 1 + sum_k a_k cos k th + b_k sin k th, n vertices.

    Parameters are the 2*kmax Fourier coefficients; dv_i/da_k = cos(k th_i) u_i,
    dv_i/db_k = sin(k th_i) u_i with u_i the radial unit vector (dense rows).
    """
    if coef is None:
        coef = star_coefficients(coef_seed, kmax)
    coef = np.asarray(coef, float)
    th = 2.0 * np.pi * np.arange(n) / n
    U = np.stack([np.cos(th), np.sin(th)], axis=1)
    k = np.arange(1, kmax + 1)
    C = np.cos(np.outer(th, k))
    S = np.sin(np.outer(th, k))
    basis = np.concatenate([C, S], axis=1)            # (n, 2kmax)
    J = basis[:, :, None] * U[:, None, :]              # (n, N, 2)
    V = U * (1.0 + basis @ coef)[:, None]
    prims = np.stack([np.arange(n), (np.arange(n) + 1) % n], axis=1).astype(np.int32)
    rowptr, pid, vel = _dense_csr(J)
    gauss = np.array([[100.0, 0.25, 0.1, 0.15]]) if source else np.zeros((0, 4))
    return Scene(dim=2, V=V, prims=prims, label=np.zeros(n, np.int32),
                 bc=[_restricted(0.0, None, [[1.0, 0.0], [0.0, -1.0]], 2)],
                 gvert=V[:, 0] ** 2 - V[:, 1] ** 2, sigma=sigma, eps=eps,
                 delta=delta, K=K, src_c0=0.0, gauss=gauss,
                 N=2 * kmax, rowptr=rowptr, pid=pid, vel=vel,
                 V_base=U.copy(), pi0=coef.copy(), name=f"c2_star{n}")


def star_points(P: int, seed: int, rmax: float = 0.8) -> np.ndarray:
    return points_in_disk(P, rmax, seed)


def annulus_scene(a: float, b: float, n: int = 1024, sigma: float = 0.0,
                  eps: float = 1e-4, delta: float = 1e-3) -> Scene:
    """Two concentric n-gons: u = 1 on r = a (label 1), 0 on r = b (label 0).

    One parameter: the inner radius a (dv/da = v/a on the inner polygon).
    Inner polygon is listed clockwise so that, like the outer one, the domain
    lies on the left of each directed edge.
    """
    Vo, Uo, po = disk_polygon(n, b)
    Vi, Ui, pi_ = disk_polygon(n, a)
    pi_ = pi_[:, ::-1].copy() + n
    V = np.concatenate([Vo, Vi])
    prims = np.concatenate([po, pi_]).astype(np.int32)
    label = np.concatenate([np.zeros(n, np.int32), np.ones(n, np.int32)])
    rowptr = np.concatenate([np.zeros(n, np.int64), np.arange(n + 1, dtype=np.int64)])
    pid = np.zeros(n, np.int32)
    vel = Ui.copy()
    Vb = np.concatenate([Vo, np.zeros_like(Vi)])
    return Scene(dim=2, V=V, prims=prims, label=label,
                 bc=[_restricted(0.0, dim=2), _restricted(1.0, dim=2)],
                 gvert=np.zeros(2 * n), sigma=sigma, eps=eps, delta=delta,
                 N=1, rowptr=rowptr, pid=pid, vel=vel, V_base=Vb,
                 pi0=np.array([a]), name=f"annulus{n}")


# --------------------------------------------------------------------------
# 2D mixed problems: Dirichlet boundary plus a reflecting (zero-flux) part
# --------------------------------------------------------------------------

def _subdivide(points, h: float) -> np.ndarray:
    """Points along the polyline through ``points``, every edge split into
    equal pieces no longer than h (the given points are kept)."""
    P = np.asarray(points, float)
    out = [P[0]]
    for a, b in zip(P[:-1], P[1:]):
        n = max(1, int(math.ceil(np.linalg.norm(b - a) / h - 1e-9)))
        t = np.arange(1, n + 1)[:, None] / n
        out.extend(list(a + t * (b - a)))
    return np.array(out)


def _chain(n_pts: int, closed: bool = False) -> np.ndarray:
    """Segments joining consecutive points (and the last to the first if closed)."""
    i = np.arange(n_pts if closed else n_pts - 1)
    return np.stack([i, (i + 1) % n_pts], axis=1).astype(np.int32)


def corner_harmonic(r, theta):
    """r^(2/3) cos(2 theta / 3): harmonic, with zero normal derivative on the
    rays theta = 0 and theta = 3 pi / 2."""
    return np.power(r, 2.0 / 3.0) * np.cos(2.0 * theta / 3.0)


def lshape_scene(h: float = 1.0 / 128, n_arm: int = 16, sigma: float = 0.0,
                 eps: float = 1e-4, delta: float = 1e-3, gfun=None) -> Scene:
    """L-shaped domain [-1,1]^2 minus [0,1]x[-1,0].

    The two edges at the re-entrant corner (the origin) are reflecting walls
    (n_arm segments each); the outer edges are Dirichlet, split into pieces of
    length <= h, with mapped vertex values gfun(r, theta), theta in
    [0, 3 pi/2] measured from the +x axis (default: ``corner_harmonic``, the
    solution for sigma = 0).
    """
    gfun = corner_harmonic if gfun is None else gfun
    V = _subdivide([[1, 0], [1, 1], [-1, 1], [-1, -1], [0, -1]], h)
    th = np.mod(np.arctan2(V[:, 1], V[:, 0]), 2 * np.pi)
    gv = gfun(np.hypot(V[:, 0], V[:, 1]), th)
    NV = _subdivide([[0, -1], [0, 0], [1, 0]], 1.0 / n_arm)
    return Scene(dim=2, V=V, prims=_chain(len(V)), label=np.zeros(len(V) - 1, np.int32),
                 bc=[_mapped()], gvert=gv, sigma=sigma, eps=eps, delta=delta,
                 NV=NV, nsegs=_chain(len(NV)), name="lshape")


def points_in_lshape(P: int, seed: int, lim: float = 0.95) -> np.ndarray:
    """P points uniform in [-lim, lim]^2 minus the quadrant x >= 0, y <= 0."""
    rng = np.random.default_rng(seed)
    out = np.zeros((0, 2))
    while len(out) < P:
        X = rng.uniform(-lim, lim, (2 * P, 2))
        X = X[~((X[:, 0] >= 0) & (X[:, 1] <= 0))]
        out = np.concatenate([out, X])
    return out[:P]


def half_disk_scene(n_arc: int = 256, n_diam: int = 64, R: float = 1.0, sigma: float = 0.0,
                    g: str = "x2-y2", eps: float = 1e-4, delta: float = 1e-3,
                    K: int = 1) -> Scene:
    """Upper half of the disk of radius R: Dirichlet arc (n_arc segments,
    vertices on the circle), reflecting diameter (n_diam segments).  Data
    restricted x^2 - y^2 (``g='x2-y2'``) or 1 (``g='one'``), both even in y,
    so the solution is the full disk's (``g='zero'`` for source tests;
    ``g='x2-y2+y'``, harmonic with du/dy = 1 on the diameter, for Neumann and
    Robin data there).  One
    parameter pi = R with
    dv/dR = v/R on the arc (the diameter has no normal motion)."""
    th = np.pi * np.arange(n_arc + 1) / n_arc
    U = np.stack([np.cos(th), np.sin(th)], axis=1)
    fld = {"x2-y2": _restricted(0.0, None, [[1.0, 0.0], [0.0, -1.0]], 2),
           "x2-y2+y": _restricted(0.0, [0.0, 1.0], [[1.0, 0.0], [0.0, -1.0]], 2),
           "one": _restricted(1.0, None, None, 2), "zero": _restricted(0.0, None, None, 2)}[g]
    NV = _subdivide([[-R, 0.0], [R, 0.0]], 2 * R / n_diam)
    return Scene(dim=2, V=R * U, prims=_chain(n_arc + 1), label=np.zeros(n_arc, np.int32),
                 bc=[fld], gvert=np.zeros(n_arc + 1), sigma=sigma, eps=eps, delta=delta, K=K,
                 N=1, rowptr=np.arange(n_arc + 2, dtype=np.int64),
                 pid=np.zeros(n_arc + 1, np.int32), vel=U.copy(),
                 V_base=np.zeros((n_arc + 1, 2)), pi0=np.array([R]),
                 NV=NV, nsegs=_chain(len(NV)), name="half_disk")


def points_in_half_disk(P: int, seed: int, rmax: float = 0.9) -> np.ndarray:
    """P points area-uniform in the half disk r < rmax, y > 0."""
    rng = np.random.default_rng(seed)
    r = rmax * np.sqrt(rng.random(P))
    th = np.pi * rng.random(P)
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=1)


def annulus_reflecting_scene(a: float = 0.4, b: float = 1.0, n_in: int = 256, n_out: int = 512,
                             sigma: float = 4.0, eps: float = 1e-4, delta: float = 1e-3,
                             K: int = 1) -> Scene:
    """Dirichlet inner n_in-gon of radius a with g = 1 inside a reflecting
    outer n_out-gon of radius b (CCW: the domain on its left).  One
    parameter: the inner radius a (dv/da = v/a)."""
    Vi, Ui, pi_ = disk_polygon(n_in, a)
    NV, _, nsegs = disk_polygon(n_out, b)
    return Scene(dim=2, V=Vi, prims=pi_, label=np.zeros(n_in, np.int32),
                 bc=[_restricted(1.0, dim=2)], gvert=np.ones(n_in), sigma=sigma, eps=eps,
                 delta=delta, K=K, N=1, rowptr=np.arange(n_in + 1, dtype=np.int64),
                 pid=np.zeros(n_in, np.int32), vel=Ui.copy(), V_base=np.zeros_like(Vi),
                 pi0=np.array([a]), NV=NV, nsegs=nsegs.astype(np.int32), name="annulus_reflecting")


def thermal_scene(n_slice: int = 65536, n_wire: int = 125, n_modes: int = 8,
                  coef: Optional[np.ndarray] = None, coef_seed: int = 0, sigma: float = 0.0,
                  eps: float = 1e-3, delta: float = 1e-2, K: int = 1) -> Scene:
    """2D stand-in for the paper's thermal-design example (Sec. 7.3): four
    heating wires -- closed loops of n_wire segments each (500 in all), g = 1
    (label 1) -- whose shapes are the parameters, a fixed zero-flux slice
    between them (n_slice segments), inside a cold box [-2, 2]^2 (g = 0,
    label 0).

    Wire w has centre c_w = (+-1.35, +-0.45) and radius
    r(phi) = 0.15 + sum_{k < n_modes} (a_k cos k phi + b_k sin k phi); its
    2 n_modes coefficients are parameters (64 in all) with
    dv/da_k = cos(k phi) u, dv/db_k = sin(k phi) u (u the radial unit
    vector).  The slice is the superellipse |x/0.9|^4 + |y/0.6|^4 = 1 with a
    crust ripple of 1% at 24 lobes, listed clockwise so that the domain (the
    outside) is on the left of each segment.  coef: all 64 coefficients
    (default: N(0, 0.01^2) draws of seed coef_seed, mode 0 of each wire
    shifted by 0)."""
    n_wires = 4
    N = 2 * n_modes * n_wires
    if coef is None:
        coef = np.random.default_rng(coef_seed).normal(0.0, 0.01, N)
    coef = np.asarray(coef, float)
    centres = np.array([[-1.35, -0.45], [-1.35, 0.45], [1.35, -0.45], [1.35, 0.45]])
    box = np.array([[-2.0, -2.0], [2.0, -2.0], [2.0, 2.0], [-2.0, 2.0]])
    V = [box]
    prims = [_chain(4, closed=True)]
    label = [np.zeros(4, np.int32)]
    Vb = [box.copy()]
    rows, pids, vels = [np.zeros(4, np.int64)], [], []
    k = np.arange(n_modes)
    nv = 4
    for w in range(n_wires):
        phi = 2 * np.pi * np.arange(n_wire) / n_wire
        U = np.stack([np.cos(phi), np.sin(phi)], 1)
        basis = np.concatenate([np.cos(np.outer(phi, k)), np.sin(np.outer(phi, k))], 1)
        cw = coef[w * 2 * n_modes:(w + 1) * 2 * n_modes]
        V.append(centres[w] + U * (0.15 + basis @ cw)[:, None])
        Vb.append(centres[w] + 0.15 * U)
        prims.append(_chain(n_wire, closed=True) + nv)
        label.append(np.ones(n_wire, np.int32))
        rows.append(np.full(n_wire, 2 * n_modes, np.int64))
        pids.append(np.tile(np.arange(2 * n_modes, dtype=np.int32) + w * 2 * n_modes, n_wire))
        vels.append((basis[:, :, None] * U[:, None, :]).reshape(-1, 2))
        nv += n_wire
    th = -2 * np.pi * np.arange(n_slice) / n_slice          # clockwise
    c, s_ = np.cos(th), np.sin(th)
    rs = 1.0 / (np.abs(c / 0.9) ** 4 + np.abs(s_ / 0.6) ** 4) ** 0.25 * (1 + 0.01 * np.cos(24 * th))
    NV = np.stack([rs * c, rs * s_], 1)
    rowptr = np.concatenate([[0], np.cumsum(np.concatenate(rows))]).astype(np.int64)
    return Scene(dim=2, V=np.concatenate(V), prims=np.concatenate(prims).astype(np.int32),
                 label=np.concatenate(label), bc=[_restricted(0.0, dim=2), _restricted(1.0, dim=2)],
                 gvert=np.zeros(nv), sigma=sigma, eps=eps, delta=delta, K=K, N=N,
                 rowptr=rowptr, pid=np.concatenate(pids), vel=np.concatenate(vels),
                 V_base=np.concatenate(Vb), pi0=coef.copy(), NV=NV,
                 nsegs=_chain(n_slice, closed=True), name=f"thermal{n_slice}")


def monopole_scene(mono, c: float = -1.0, sigma: float = 0.0, src_c0: float = 0.0, g=(0.0, None, None),
                   eps: float = 1e-4, delta: float = 1e-3, K: int = 1) -> Scene:
    """Implicit boundary of Sec. 7.4: the zero set of
    h(x) = c + sum_n a_n / |x - p_n| (rows (a_n, p_x, p_y) of mono, a_n > 0,
    c < 0), domain {h > 0}; restricted data g = (c0, b, A); parameters
    (a_n, p_n) per monopole."""
    mono = np.asarray(mono, float).reshape(-1, 3)
    c0, b, A = g
    return Scene(dim=2, V=np.zeros((0, 2)), prims=np.zeros((0, 2), np.int32),
                 label=np.zeros(0, np.int32), bc=[_restricted(c0, b, A, 2)], gvert=np.zeros(0),
                 sigma=sigma, eps=eps, delta=delta, K=K, src_c0=src_c0, N=3 * len(mono),
                 mono=mono, mono_c=float(c), pi0=mono.ravel().copy(), name="monopoles")


def inflation_scene(n: int = 16, seed: int = 0, c: float = -1.0, eps: float = 1e-3,
                    delta: float = 1e-2) -> Scene:
    """Curve inflation (Sec. 7.4): -Lap u = 4, g = 0 inside the zero set of
    n monopoles with scales a_n ~ U(0.02, 0.06) * 16 / n (their sum stays
    near 0.64, so the far-field zero set has radius ~0.64) and positions in
    [-0.6, 0.6]^2 (seed), c = -1: a blob domain that may split."""
    rng = np.random.default_rng(seed)
    mono = np.stack([rng.uniform(0.02, 0.06, n) * 16.0 / n, rng.uniform(-0.6, 0.6, n),
                     rng.uniform(-0.6, 0.6, n)], 1)
    return monopole_scene(mono, c=c, src_c0=4.0, eps=eps, delta=delta).with_(name=f"inflation{n}")


def points_on_segments(NV: np.ndarray, nsegs: np.ndarray, P: int, seed: int, segs=None):
    """P points on reflecting segments (uniform segment from ``segs`` or all,
    uniform parameter in [0.05, 0.95]): returns (X, start_seg)."""
    rng = np.random.default_rng(seed)
    pool = np.arange(len(nsegs)) if segs is None else np.asarray(segs)
    s = pool[rng.integers(0, len(pool), P)]
    t = rng.uniform(0.05, 0.95, P)[:, None]
    a, b = NV[nsegs[s, 0]], NV[nsegs[s, 1]]
    return a + t * (b - a), s.astype(np.int32)


# --------------------------------------------------------------------------
# 3D geometry
# --------------------------------------------------------------------------

def _icosahedron():
    t = (1.0 + 5 ** 0.5) / 2.0
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], float)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]])
    return v, f


def icosphere(nu: int):
    """Class-I geodesic icosphere of frequency nu: 20 nu^2 triangles,
    10 nu^2 + 2 unit-length vertices, outward (CCW seen from outside) winding."""
    v0, f0 = _icosahedron()
    pts = []
    tris = []
    # barycentric lattice on each face
    idx = {}
    for (i, j) in [(i, j) for i in range(nu + 1) for j in range(nu + 1 - i)]:
        idx[(i, j)] = len(idx)
    lat = np.array(list(idx.keys()), float) / nu            # (m, 2): (i/nu, j/nu)
    loc_tris = []
    for i in range(nu):
        for j in range(nu - i):
            a, b, c = idx[(i, j)], idx[(i + 1, j)], idx[(i, j + 1)]
            loc_tris.append((a, b, c))
            if j + i + 1 < nu:
                d = idx[(i + 1, j + 1)]
                loc_tris.append((b, d, c))
    loc_tris = np.array(loc_tris)
    m = lat.shape[0]
    for fi, (A, B, C) in enumerate(f0):
        P = (v0[A][None, :] * (1 - lat[:, :1] - lat[:, 1:]) + v0[B][None, :] * lat[:, :1]
             + v0[C][None, :] * lat[:, 1:])
        pts.append(P)
        tris.append(loc_tris + fi * m)
    P = np.concatenate(pts)
    T = np.concatenate(tris)
    P /= np.linalg.norm(P, axis=1, keepdims=True)
    key = np.round(P * 1e9).astype(np.int64)
    _, first, inv = np.unique(key, axis=0, return_index=True, return_inverse=True)
    inv = inv.reshape(-1)
    Vu = P[first]
    T = inv[T]
    # orient outward
    a, b, c = Vu[T[:, 0]], Vu[T[:, 1]], Vu[T[:, 2]]
    nrm = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", nrm, a + b + c) < 0
    T[flip] = T[flip][:, [0, 2, 1]]
    return Vu, T.astype(np.int32)


def box_triangles(h: float = 2.0):
    """Axis-aligned cube [-h, h]^3 as 12 triangles with outward winding."""
    V = np.array([[x, y, z] for x in (-h, h) for y in (-h, h) for z in (-h, h)], float)
    quads = [(0, 1, 3, 2), (4, 6, 7, 5), (0, 4, 5, 1), (2, 3, 7, 6), (0, 2, 6, 4), (1, 5, 7, 3)]
    T = []
    for q in quads:
        T.append((q[0], q[1], q[2]))
        T.append((q[0], q[2], q[3]))
    T = np.array(T, np.int32)
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    nrm = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", nrm, a + b + c) < 0
    T[flip] = T[flip][:, [0, 2, 1]]
    return V, T


def fibonacci_sphere(n: int):
    i = np.arange(n) + 0.5
    z = 1.0 - 2.0 * i / n
    phi = np.pi * (1.0 + 5 ** 0.5) * i
    r = np.sqrt(1 - z * z)
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def radial_basis(Vu: np.ndarray, centres: np.ndarray, h: float, cut: float = 3.0):
    """Angular Gaussian bumps exp(-theta^2/(2h^2)), truncated at theta > cut*h.

    Returns CSR (rowptr, cols, vals) of phi_j(v_i)."""
    rows, cols, vals = [], [], []
    cosc = math.cos(cut * h)
    for s in range(0, Vu.shape[0], 8192):
        blk = Vu[s:s + 8192]
        dots = blk @ centres.T
        ii, jj = np.nonzero(dots >= cosc)
        th = np.arccos(np.clip(dots[ii, jj], -1.0, 1.0))
        rows.append(ii + s)
        cols.append(jj)
        vals.append(np.exp(-th ** 2 / (2 * h * h)))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(Vu.shape[0] + 1, np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr, cols.astype(np.int32), vals


def c3_icosphere(nu: int = 100, n_basis: int = 1024, h: float = 0.1,
                 coef: Optional[np.ndarray] = None, coef_seed: int = 0,
                 coef_std: float = 0.05, R0: float = 1.0, box: float = 2.0,
                 sigma: float = 4.0, eps: float = 4e-3, delta: float = 4e-2,
                 K: int = 1) -> Scene:
    """Displaced icosphere (label 1, g = 1) inside the box [-box, box]^3
    (label 0, g = 0).  v_i = u_i (R0 + sum_j c_j phi_j(u_i)); parameters c_j."""
    Vu, T = icosphere(nu)
    centres = fibonacci_sphere(n_basis)
    rp, cols, vals = radial_basis(Vu, centres, h)
    if coef is None:
        coef = np.random.default_rng(coef_seed).normal(0.0, coef_std, n_basis)
    coef = np.asarray(coef, float)
    rows = np.repeat(np.arange(Vu.shape[0]), np.diff(rp))
    disp = np.zeros(Vu.shape[0])
    np.add.at(disp, rows, vals * coef[cols])
    Vobj = Vu * (R0 + disp)[:, None]
    Vb, Tb = box_triangles(box)
    nb = Vb.shape[0]
    V = np.concatenate([Vb, Vobj])
    # object winding flipped: its stored normal points into the object,
    # i.e. out of the domain between object and box
    prims = np.concatenate([Tb, T[:, [0, 2, 1]] + nb]).astype(np.int32)
    label = np.concatenate([np.zeros(len(Tb), np.int32), np.ones(len(T), np.int32)])
    rowptr = np.concatenate([np.zeros(nb, np.int64), rp])
    vel = Vu[rows] * vals[:, None]
    Vbase = np.concatenate([Vb, Vu * R0])
    return Scene(dim=3, V=V, prims=prims, label=label,
                 bc=[_restricted(0.0, dim=3), _restricted(1.0, dim=3)],
                 gvert=np.zeros(V.shape[0]), sigma=sigma, eps=eps, delta=delta,
                 K=K, N=n_basis, rowptr=rowptr, pid=cols, vel=vel,
                 V_base=Vbase, pi0=coef.copy(), name=f"c3_icosphere{nu}")


def points_on_box_faces(P: int, seed: int, inset: float = 1.9) -> np.ndarray:
    """P points uniform on the six faces |coord| = inset of a cube (face uniform)."""
    rng = np.random.default_rng(seed)
    face = rng.integers(0, 6, P)
    uv = rng.uniform(-inset, inset, (P, 2))
    X = np.zeros((P, 3))
    ax = face // 2
    sgn = np.where(face % 2 == 0, -1.0, 1.0)
    for a in range(3):
        m = ax == a
        others = [o for o in range(3) if o != a]
        X[m, a] = sgn[m] * inset
        X[m, others[0]] = uv[m, 0]
        X[m, others[1]] = uv[m, 1]
    return X


def points_in_ball(P: int, rmin: float, rmax: float, seed: int) -> np.ndarray:
    """P points volume-uniform in the spherical shell rmin < r < rmax."""
    rng = np.random.default_rng(seed)
    r = (rmin ** 3 + (rmax ** 3 - rmin ** 3) * rng.random(P)) ** (1.0 / 3.0)
    d = rng.normal(size=(P, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return d * r[:, None]


def sphere_scene(nu: int, R: float = 1.0, g: str = "one", sigma: float = 0.0,
                 eps: float = 1e-3, delta: float = 1e-2, source_c0: float = 0.0) -> Scene:
    """Ball of radius R as an icosphere mesh (domain inside), parameter pi = R.

    The stored triangle normal points away from the centre, i.e. out of the
    domain."""
    Vu, T = icosphere(nu)
    fld = _restricted(1.0, dim=3) if g == "one" else _restricted(0.0, dim=3)
    n = Vu.shape[0]
    return Scene(dim=3, V=R * Vu, prims=T, label=np.zeros(len(T), np.int32), bc=[fld],
                 gvert=np.zeros(n), sigma=sigma, eps=eps, delta=delta,
                 src_c0=source_c0, N=1, rowptr=np.arange(n + 1, dtype=np.int64),
                 pid=np.zeros(n, np.int32), vel=Vu.copy(), V_base=np.zeros_like(Vu),
                 pi0=np.array([R]), name=f"sphere{nu}")


def shell_scene(nu_in: int, nu_out: int, a: float, b: float, sigma: float,
                eps: float = 1e-3, delta: float = 1e-2) -> Scene:
    """Spherical shell a < r < b: g = 1 on the inner icosphere (label 1,
    parameter pi = a), g = 0 on the outer icosphere (label 0)."""
    Vo, To = icosphere(nu_out)
    Vi, Ti = icosphere(nu_in)
    no = Vo.shape[0]
    V = np.concatenate([b * Vo, a * Vi])
    prims = np.concatenate([To, Ti[:, [0, 2, 1]] + no]).astype(np.int32)
    label = np.concatenate([np.zeros(len(To), np.int32), np.ones(len(Ti), np.int32)])
    rowptr = np.concatenate([np.zeros(no, np.int64), np.arange(Vi.shape[0] + 1, dtype=np.int64)])
    return Scene(dim=3, V=V, prims=prims, label=label,
                 bc=[_restricted(0.0, dim=3), _restricted(1.0, dim=3)],
                 gvert=np.zeros(V.shape[0]), sigma=sigma, eps=eps, delta=delta,
                 N=1, rowptr=rowptr, pid=np.zeros(Vi.shape[0], np.int32),
                 vel=Vi.copy(), V_base=np.concatenate([b * Vo, np.zeros_like(Vi)]),
                 pi0=np.array([a]), name=f"shell{nu_in}_{nu_out}")


def c4_batch(n_inst: int = 256, seed0: int = 100, tri_lo: float = 1e3,
             tri_hi: float = 1e5, p_lo: float = 512, p_hi: float = 16384,
             n_basis: int = 256, sigma_hi: float = 20.0):
    """Instances of the C3 generator with log-uniform triangle and point counts.

    Returns a list of (Scene, X) pairs; instance i draws from seed seed0 + i."""
    out = []
    for i in range(n_inst):
        rng = np.random.default_rng(seed0 + i)
        T = math.exp(rng.uniform(math.log(tri_lo), math.log(tri_hi)))
        nu = max(1, int(round(math.sqrt(T / 20.0))))
        P = int(round(math.exp(rng.uniform(math.log(p_lo), math.log(p_hi)))))
        sigma = float(rng.uniform(0.0, sigma_hi))
        sc = c3_icosphere(nu=nu, n_basis=n_basis, coef_seed=seed0 + i, sigma=sigma)
        X = points_on_box_faces(P, seed0 + i)
        out.append((sc, X))
    return out


# --------------------------------------------------------------------------
# 3D reflecting boundaries (walk on stars)
# --------------------------------------------------------------------------

def _grid_rect(p0, e1, e2, n1: int, n2: int):
    """Rectangle p0 + s e1 + t e2 (s, t in [0, 1]) as an n1 x n2 grid of
    cells, two triangles each, wound so that e1 x e2 is the left normal."""
    p0, e1, e2 = (np.asarray(a, float) for a in (p0, e1, e2))
    i, j = np.meshgrid(np.arange(n1 + 1), np.arange(n2 + 1), indexing="ij")
    V = p0 + (i.reshape(-1, 1) / n1) * e1 + (j.reshape(-1, 1) / n2) * e2
    idx = lambda a, b: a * (n2 + 1) + b
    T = []
    for a in range(n1):
        for b in range(n2):
            T.append((idx(a, b), idx(a + 1, b), idx(a + 1, b + 1)))
            T.append((idx(a, b), idx(a + 1, b + 1), idx(a, b + 1)))
    return V, np.array(T, np.int32)


def _graded_rect(p0, e1, e2, n1: int, n2: int, power: float):
    """As _grid_rect with the grid lines at (i/n)^power along both edges, so
    the cells (and triangles) have unequal areas."""
    p0, e1, e2 = (np.asarray(a, float) for a in (p0, e1, e2))
    s1 = (np.arange(n1 + 1) / n1) ** power
    s2 = (np.arange(n2 + 1) / n2) ** power
    i, j = np.meshgrid(np.arange(n1 + 1), np.arange(n2 + 1), indexing="ij")
    V = p0 + s1[i.reshape(-1)][:, None] * e1 + s2[j.reshape(-1)][:, None] * e2
    _, T = _grid_rect(p0, e1, e2, n1, n2)
    return V, T


def _weld(parts, tol: float = 1e-9):
    """Concatenate (V, T) meshes and merge vertices closer than tol."""
    V = np.concatenate([v for v, _ in parts])
    offs = np.cumsum([0] + [len(v) for v, _ in parts])[:-1]
    T = np.concatenate([t + o for (_, t), o in zip(parts, offs)])
    key = np.round(V / tol).astype(np.int64)
    _, first, inv = np.unique(key, axis=0, return_index=True, return_inverse=True)
    inv = inv.ravel()
    return V[first], inv[T].astype(np.int32)


def lprism_scene(n: int = 8, n_wall: int = 8, H: float = 1.0, sigma: float = 0.0,
                 eps: float = 1e-4, delta: float = 1e-3, gfun=None) -> Scene:
    """L-shaped prism: the L-shaped domain [-1,1]^2 minus [0,1]x[-1,0]
    extruded over z in [-H, H].  The two faces at the re-entrant edge (the z
    axis) are reflecting walls (n_wall cells per unit, sharing the edge's
    vertices); the outer faces and the caps z = +-H are Dirichlet (n cells
    per unit) with mapped vertex values gfun(r, theta), theta in [0, 3 pi/2]
    from the +x axis (default ``corner_harmonic``: the z-independent solution
    for sigma = 0).  Wall A is y = 0, x in [0, 1] (domain side +y); wall B is
    x = 0, y in [-1, 0] (domain side -x); both are wound with the domain on
    their left normal."""
    gfun = corner_harmonic if gfun is None else gfun
    parts = []
    path = [[1, 0], [1, 1], [-1, 1], [-1, -1], [0, -1]]
    for a, b in zip(path[:-1], path[1:]):
        a3, b3 = np.array([a[0], a[1], -H]), np.array([b[0], b[1], -H])
        L = float(np.hypot(b[0] - a[0], b[1] - a[1]))
        parts.append(_grid_rect(a3, b3 - a3, [0, 0, 2 * H], max(1, int(round(n * L))),
                                max(1, int(round(2 * H * n)))))
    for z in (-H, H):
        for x0, y0 in ((-1, 0), (0, 0), (-1, -1)):
            parts.append(_grid_rect([x0, y0, z], [1, 0, 0], [0, 1, 0], n, n))
    V, T = _weld(parts)
    th = np.mod(np.arctan2(V[:, 1], V[:, 0]), 2 * np.pi)
    gv = gfun(np.hypot(V[:, 0], V[:, 1]), th)
    nz = max(1, int(round(2 * H * n_wall)))
    wa = _grid_rect([0, 0, -H], [1, 0, 0], [0, 0, 2 * H], n_wall, nz)    # left normal -y
    wb = _grid_rect([0, -1, -H], [0, 1, 0], [0, 0, 2 * H], n_wall, nz)   # left normal +x
    wa = (wa[0], wa[1][:, [0, 2, 1]])   # domain y > 0 on the left
    wb = (wb[0], wb[1][:, [0, 2, 1]])   # domain x < 0 on the left
    NV, NT = _weld([wa, wb])
    return Scene(dim=3, V=V, prims=T, label=np.zeros(len(T), np.int32), bc=[_mapped()], gvert=gv,
                 sigma=sigma, eps=eps, delta=delta, NV=NV, nsegs=NT, name="lprism")


def points_in_lprism(P: int, seed: int, lim: float = 0.95, zlim: float = 0.5) -> np.ndarray:
    """P points uniform in [-lim, lim]^2 x [-zlim, zlim] minus x >= 0, y <= 0."""
    rng = np.random.default_rng(seed)
    out = np.zeros((0, 3))
    while len(out) < P:
        X = np.concatenate([rng.uniform(-lim, lim, (2 * P, 2)), rng.uniform(-zlim, zlim, (2 * P, 1))], 1)
        X = X[~((X[:, 0] >= 0) & (X[:, 1] <= 0))]
        out = np.concatenate([out, X])
    return out[:P]


def box_wall_scene(n_wall: int = 4, sigma: float = 0.0, eps: float = 1e-4, delta: float = 1e-3,
                   g=None, robin_mu: float = 0.0, robin_h=None, graded: float = 1.0) -> Scene:
    """Cube [-1, 1]^3: the face x = -1 is a reflecting wall (n_wall x n_wall
    cells, domain side +x; graded != 1: grid lines at (i/n)^graded, cells of
    unequal areas), the other five faces are Dirichlet (two triangles each)
    with the restricted field g (dict of _restricted; default 0)."""
    Vb, Tb = box_triangles(1.0)
    c = (Vb[Tb[:, 0]] + Vb[Tb[:, 1]] + Vb[Tb[:, 2]]) / 3
    keep = ~(c[:, 0] < -0.999)
    used = np.unique(Tb[keep])
    remap = -np.ones(len(Vb), np.int64)
    remap[used] = np.arange(len(used))
    V, T = Vb[used], remap[Tb[keep]].astype(np.int32)
    NV, NT = _graded_rect([-1, -1, -1], [0, 2, 0], [0, 0, 2], n_wall, n_wall, graded)   # left normal +x
    return Scene(dim=3, V=V, prims=T, label=np.zeros(len(T), np.int32),
                 bc=[g if g is not None else _restricted(0.0, dim=3)], gvert=np.zeros(len(V)),
                 sigma=sigma, eps=eps, delta=delta, NV=NV, nsegs=NT, robin_mu=robin_mu,
                 robin_h=robin_h, name="box_wall")


def half_ball_scene(n_az: int = 48, n_pol: int = 12, n_rad: int = 12, R: float = 1.0,
                    sigma: float = 0.0, g: str = "one", eps: float = 1e-3, delta: float = 1e-2,
                    K: int = 1) -> Scene:
    """Upper half (y > 0) of the ball of radius R: a Dirichlet hemisphere
    (latitude-longitude mesh, n_pol rings from the pole to the equator,
    n_az vertices per ring) and a reflecting flat disk y = 0 (n_rad rings
    sharing the equator's n_az vertices), domain side +y.  Data restricted:
    1 (``g='one'``) or x^2 - z^2 (``g='x2-z2'``), both even in y, so the
    solution is the full ball's.  One parameter pi = R with dv/dR = v/R on
    the hemisphere; the disk is fixed (its motion is tangential)."""
    az = 2 * np.pi * np.arange(n_az) / n_az
    pts = [[0.0, 1.0, 0.0]]
    for j in range(1, n_pol + 1):
        ph = 0.5 * np.pi * j / n_pol
        pts += [[np.sin(ph) * np.cos(a), np.cos(ph), np.sin(ph) * np.sin(a)] for a in az]
    U = np.array(pts)
    ring = lambda j, k: 1 + (j - 1) * n_az + (k % n_az)
    T = []
    for k in range(n_az):
        T.append((0, ring(1, k + 1), ring(1, k)))
    for j in range(1, n_pol):
        for k in range(n_az):
            T.append((ring(j, k), ring(j, k + 1), ring(j + 1, k + 1)))
            T.append((ring(j, k), ring(j + 1, k + 1), ring(j + 1, k)))
    T = np.array(T, np.int32)
    a, b, c = U[T[:, 0]], U[T[:, 1]], U[T[:, 2]]
    flip = np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c) < 0
    T[flip] = T[flip][:, [0, 2, 1]]
    dpts = [[0.0, 0.0, 0.0]]
    for i in range(1, n_rad + 1):
        rho = R * i / n_rad
        dpts += [[rho * np.cos(a_), 0.0, rho * np.sin(a_)] for a_ in az]
    NV = np.array(dpts)
    dring = lambda i, k: 1 + (i - 1) * n_az + (k % n_az)
    NT = []
    for k in range(n_az):
        NT.append((0, dring(1, k), dring(1, k + 1)))
    for i in range(1, n_rad):
        for k in range(n_az):
            NT.append((dring(i, k), dring(i + 1, k), dring(i + 1, k + 1)))
            NT.append((dring(i, k), dring(i + 1, k + 1), dring(i, k + 1)))
    NT = np.array(NT, np.int32)
    e1 = NV[NT[:, 1]] - NV[NT[:, 0]]
    e2 = NV[NT[:, 2]] - NV[NT[:, 0]]
    up = np.cross(e1, e2)[:, 1] < 0
    NT[up] = NT[up][:, [0, 2, 1]]   # left normal +y (the domain side)
    fld = {"one": _restricted(1.0, dim=3),
           "x2-z2": _restricted(0.0, None, np.diag([1.0, 0.0, -1.0]), 3)}[g]
    n = len(U)
    return Scene(dim=3, V=R * U, prims=T, label=np.zeros(len(T), np.int32), bc=[fld],
                 gvert=np.zeros(n), sigma=sigma, eps=eps, delta=delta, K=K, N=1,
                 rowptr=np.arange(n + 1, dtype=np.int64), pid=np.zeros(n, np.int32), vel=U.copy(),
                 V_base=np.zeros_like(U), pi0=np.array([R]), NV=NV, nsegs=NT, name="half_ball")


def points_in_half_ball(P: int, seed: int, rmax: float = 0.8, ymin: float = 0.0) -> np.ndarray:
    """P points uniform in the half ball r < rmax, y > ymin."""
    rng = np.random.default_rng(seed)
    out = np.zeros((0, 3))
    while len(out) < P:
        X = rng.uniform(-rmax, rmax, (4 * P, 3))
        X = X[(np.linalg.norm(X, axis=1) < rmax) & (X[:, 1] > ymin)]
        out = np.concatenate([out, X])
    return out[:P]


def thermal3d_scene(nu_slice: int = 57, nu_wire: int = 8, n_basis: int = 16, h: float = 0.6,
                    coef: Optional[np.ndarray] = None, coef_seed: int = 0, sigma: float = 0.0,
                    eps: float = 1e-3, delta: float = 1e-2, K: int = 1) -> Scene:
    """3D stand-in for the paper's thermal-design example (Sec. 7.3): four
    heating elements -- displaced icospheres of frequency nu_wire, radius
    0.15, g = 1 (label 1) -- whose shapes are the parameters, a fixed
    zero-flux slice between them, inside a cold box [-2, 2]^3 (g = 0, label
    0).

    Element w has centre (+-1.35, +-0.45, 0) and radius
    0.15 (1 + sum_j c_j phi_j(u)) with n_basis angular Gaussian bumps of
    width h at Fibonacci-sphere centres (4 n_basis parameters in all).  The
    slice is the superellipsoid |x/0.9|^4 + |y/0.6|^4 + |z/0.6|^4 = 1 with a
    1% ripple of 24 lobes about the z axis, an icosphere of frequency
    nu_slice projected onto it (20 nu_slice^2 triangles, 64,980 at 57), wound
    outward: the domain (outside) is on each triangle's left normal."""
    n_wires = 4
    N = n_basis * n_wires
    if coef is None:
        coef = np.random.default_rng(coef_seed).normal(0.0, 0.05, N)
    coef = np.asarray(coef, float)
    Vb, Tb = box_triangles(2.0)
    V, prims, label, Vbase = [Vb], [Tb], [np.zeros(len(Tb), np.int32)], [Vb.copy()]
    rows = [np.zeros(len(Vb), np.int64)]
    pids, vels = [], []
    nv = len(Vb)
    Vu, Tw = icosphere(nu_wire)
    centres = fibonacci_sphere(n_basis)
    rp, cols, vals = radial_basis(Vu, centres, h)
    vrows = np.repeat(np.arange(Vu.shape[0]), np.diff(rp))
    for w, cw in enumerate([[-1.35, -0.45, 0.0], [-1.35, 0.45, 0.0], [1.35, -0.45, 0.0], [1.35, 0.45, 0.0]]):
        cw = np.array(cw)
        c_w = coef[w * n_basis:(w + 1) * n_basis]
        disp = np.zeros(Vu.shape[0])
        np.add.at(disp, vrows, vals * c_w[cols])
        V.append(cw + 0.15 * Vu * (1.0 + disp)[:, None])
        Vbase.append(cw + 0.15 * Vu)
        # element winding flipped: its stored normal points into the element
        prims.append(Tw[:, [0, 2, 1]] + nv)
        label.append(np.ones(len(Tw), np.int32))
        rows.append(np.diff(rp).astype(np.int64))
        pids.append((cols + w * n_basis).astype(np.int32))
        vels.append(0.15 * Vu[vrows] * vals[:, None])
        nv += Vu.shape[0]
    Us, Ts = icosphere(nu_slice)
    rs = 1.0 / (np.abs(Us[:, 0] / 0.9) ** 4 + np.abs(Us[:, 1] / 0.6) ** 4 + np.abs(Us[:, 2] / 0.6) ** 4) ** 0.25
    phi = np.arctan2(Us[:, 1], Us[:, 0])
    NV = Us * (rs * (1 + 0.01 * np.cos(24 * phi)))[:, None]
    rowptr = np.concatenate([[0], np.cumsum(np.concatenate(rows))]).astype(np.int64)
    return Scene(dim=3, V=np.concatenate(V), prims=np.concatenate(prims).astype(np.int32),
                 label=np.concatenate(label), bc=[_restricted(0.0, dim=3), _restricted(1.0, dim=3)],
                 gvert=np.zeros(nv), sigma=sigma, eps=eps, delta=delta, K=K, N=N, rowptr=rowptr,
                 pid=np.concatenate(pids), vel=np.concatenate(vels), V_base=np.concatenate(Vbase),
                 pi0=coef.copy(), NV=NV, nsegs=Ts.astype(np.int32), name=f"thermal3d_{nu_slice}")


def points_on_triangles(NV: np.ndarray, ntris: np.ndarray, P: int, seed: int, tris=None):
    """P points on reflecting triangles (a uniform triangle from ``tris`` or
    all, barycentrics uniform on the triangle shrunk by 10% about its
    centroid): returns (X, start triangle)."""
    rng = np.random.default_rng(seed)
    pool = np.arange(len(ntris)) if tris is None else np.asarray(tris)
    s = pool[rng.integers(0, len(pool), P)]
    r1, r2 = np.sqrt(rng.random(P))[:, None], rng.random(P)[:, None]
    a, b, c = NV[ntris[s, 0]], NV[ntris[s, 1]], NV[ntris[s, 2]]
    X = (1 - r1) * a + r1 * (1 - r2) * b + r1 * r2 * c
    cen = (a + b + c) / 3
    return cen + 0.9 * (X - cen), s.astype(np.int32)


# ---------------------------------------------------------------------------
# Initial parameters of the control-variate network (inputs, not arithmetic):
# F random Fourier frequencies B ~ N(0, freq_scale^2) and Glorot-uniform
# weights for four 64-wide layers and the scalar output, zero biases.  The
# flat layout is, for each layer, W (64 x 64, row = output unit) then b (64),
# followed by the output weights (64) and output bias.
# ---------------------------------------------------------------------------
MLP_WIDTH = 64
MLP_LAYERS = 4
MLP_FREQS = 16
MLP_THETA_SIZE = MLP_LAYERS * (MLP_WIDTH * MLP_WIDTH + MLP_WIDTH) + MLP_WIDTH + 1


def mlp_init(dim: int, seed: int, freq_scale: float = 1.0, F: int = MLP_FREQS):
    """(B [F x dim], theta [MLP_THETA_SIZE]) as float64."""
    assert 2 * F + dim <= MLP_WIDTH
    rng = np.random.default_rng(seed)
    B = rng.normal(0.0, freq_scale, size=(F, dim))
    theta = np.zeros(MLP_THETA_SIZE)
    H = MLP_WIDTH
    lim = math.sqrt(6.0 / (H + H))
    for l in range(MLP_LAYERS):
        off = l * (H * H + H)
        W = rng.uniform(-lim, lim, size=(H, H))
        if l == 0:
            W[:, 2 * F + dim:] = 0.0          # padding inputs
        theta[off:off + H * H] = W.ravel()
    off = MLP_LAYERS * (H * H + H)
    theta[off:off + H] = rng.uniform(-math.sqrt(6.0 / (H + 1)), math.sqrt(6.0 / (H + 1)), size=H)
    return B, theta


def _winding(scene: Scene, x: np.ndarray) -> np.ndarray:
    """Generalised winding number of the boundary mesh at points x (about 1
    inside a closed, outward-oriented boundary, 0 outside; its sign flips with
    the orientation): angles subtended by the segments / 2 pi in 2D, solid
    angles of the triangles / 4 pi in 3D (Van Oosterom and Strackee)."""
    V, F = scene.V, scene.prims
    out = np.zeros(len(x))
    for i, p in enumerate(x):
        if scene.dim == 2:
            a, b = V[F[:, 0]] - p, V[F[:, 1]] - p
            ang = np.arctan2(a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0], np.einsum("ij,ij->i", a, b))
            out[i] = ang.sum() / (2 * np.pi)
        else:
            a, b, c = V[F[:, 0]] - p, V[F[:, 1]] - p, V[F[:, 2]] - p
            la, lb, lc = (np.linalg.norm(v, axis=1) for v in (a, b, c))
            num = np.einsum("ij,ij->i", a, np.cross(b, c))
            den = la * lb * lc + np.einsum("ij,ij->i", a, b) * lc + np.einsum("ij,ij->i", b, c) * la \
                + np.einsum("ij,ij->i", c, a) * lb
            out[i] = 2 * np.arctan2(num, den).sum() / (4 * np.pi)
    return out


def boundary_samples(scene: Scene, S: int, seed: int, h: float = 1e-6):
    """S points on the boundary mesh, uniform by length (2D) or area (3D):
    (code = prim * 2 + flip, barycentrics b1 (, b2), quadrature weight
    |boundary| / S).  flip = 0 when the domain lies on the side opposite the
    primitive's geometric normal (segment a->b: (b - a) turned clockwise;
    triangle: (b - a) x (c - a)), decided by the winding number of a point a
    distance h along that normal."""
    rng = np.random.default_rng(seed)
    V, F, D = scene.V, scene.prims, scene.dim
    if D == 2:
        t = V[F[:, 1]] - V[F[:, 0]]
        meas = np.linalg.norm(t, axis=1)
        nrm = np.stack([t[:, 1], -t[:, 0]], 1) / meas[:, None]
    else:
        cr = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
        meas = 0.5 * np.linalg.norm(cr, axis=1)
        nrm = cr / (2 * meas[:, None])
    prim = rng.choice(len(F), size=S, p=meas / meas.sum())
    if D == 2:
        b = rng.random((S, 1))
        bary = np.concatenate([1 - b, b], 1)
    else:
        u, v = rng.random(S), rng.random(S)
        fold = u + v > 1
        u[fold], v[fold] = 1 - u[fold], 1 - v[fold]
        bary = np.stack([1 - u - v, u, v], 1)
    y = np.einsum("sk,skc->sc", bary, V[F[prim]])
    inside = np.abs(_winding(scene, y + h * nrm[prim])) > 0.5
    code = (prim * 2 + inside.astype(np.int64)).astype(np.int32)
    return code, np.ascontiguousarray(bary[:, 1:]), np.full(S, meas.sum() / S)
