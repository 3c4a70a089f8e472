"""Seeded synthetic inputs for the space-time BEM heat solver.

This module holds no part of the boundary element method: it only builds
meshes (a closed CCW polygon for Gamma, a time grid, a triangulation of
Omega) and samples the manufactured heat solution u = exp(k.x + |k|^2 t/alpha)
on them.  Both the CPU oracle and the GPU path read their inputs from here.

Paper context (arXiv:1811.05224): model problem eq.(1); tensor space-time
mesh Sigma_h = Gamma_h x I_h (Sec. 1); Dirichlet datum g in X_h^{1,0}
(continuous piecewise linear in space, piecewise constant in time), initial
datum u0 in S_h^1(Omega_h) (Sec. 1, discrete spaces).  The paper's own
experiment (Sec. 4) uses a different exact solution; the manufactured
exponential here has the same role and a closed-form Neumann datum.

Conventions
-----------
* DOF order is time-major: l = m * N_Gamma + i, element sigma = gamma_i x tau_m.
* Segment i runs from vertex i to vertex (i+1) % N_Gamma; P1 node n is vertex n.
* Times t_0 = 0 < t_1 < ... < t_{N_I} = T; tau_m = (t_m, t_{m+1}].
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Workload", "square_polygon", "lshape_polygon", "polygon_from_corners",
    "uniform_times", "graded_times", "square_grid", "lshape_grid",
    "manufactured", "make", "CONFIGS",
]


@dataclasses.dataclass
class Workload:
    name: str
    alpha: float
    t_nodes: np.ndarray          # (N_I+1,) float64
    bnd_xy: np.ndarray           # (N_Gamma, 2) float64, closed CCW polygon
    vtx_xy: np.ndarray           # (M_Omega, 2) float64
    tri: np.ndarray              # (N_tri, 3) int32, CCW
    kvec: np.ndarray             # (2,) wave vector of the manufactured solution
    g: np.ndarray                # (N,) Dirichlet data, time-major nodal x time average
    u0: np.ndarray               # (M_Omega,) nodal initial data
    w_ref: np.ndarray            # (N,) L2 projection of the exact Neumann datum
    extra: dict = dataclasses.field(default_factory=dict)

    @property
    def n_gamma(self) -> int:
        return int(self.bnd_xy.shape[0])

    @property
    def n_t(self) -> int:
        return int(self.t_nodes.shape[0] - 1)

    @property
    def n(self) -> int:
        return self.n_gamma * self.n_t


# ----------------------------------------------------------------- geometry
def polygon_from_corners(corners, seg_per_edge):
    """Subdivide the closed polygon through `corners` (CCW) uniformly."""
    corners = np.asarray(corners, dtype=np.float64)
    pts = []
    nc = corners.shape[0]
    for c in range(nc):
        a, b = corners[c], corners[(c + 1) % nc]
        n = int(seg_per_edge[c])
        for s in range(n):
            lam = s / n
            # exact endpoints; interior points as a + lam (b - a)
            pts.append(a + lam * (b - a) if s else a.copy())
    return np.ascontiguousarray(np.array(pts, dtype=np.float64))


def square_polygon(n_per_side: int):
    """Unit square (0,1)^2, CCW from the origin, n_per_side segments per side."""
    return polygon_from_corners([(0, 0), (1, 0), (1, 1), (0, 1)], [n_per_side] * 4)


def lshape_polygon(n_segments: int = 384):
    """[0,1]^2 minus [0.5,1]^2 with equal segment lengths (perimeter 4)."""
    if n_segments % 8:
        raise ValueError("L-shape needs n_segments divisible by 8")
    u = n_segments // 8     # segments per half unit
    corners = [(0, 0), (1, 0), (1, .5), (.5, .5), (.5, 1), (0, 1)]
    return polygon_from_corners(corners, [2 * u, u, u, u, u, 2 * u])


def uniform_times(n_t: int, T: float = 1.0):
    t = np.arange(n_t + 1, dtype=np.float64) * (T / n_t)
    t[-1] = T
    return t


def graded_times(n_t: int, ratio: float, T: float = 1.0):
    """t_j = T (ratio^j - 1)/(ratio^n_t - 1): finest step at t = 0."""
    j = np.arange(n_t + 1, dtype=np.float64)
    t = T * (ratio ** j - 1.0) / (ratio ** n_t - 1.0)
    t[0], t[-1] = 0.0, T
    return t


def _grid(n, keep):
    xs = np.arange(n + 1, dtype=np.float64) / n
    vid = -np.ones((n + 1, n + 1), dtype=np.int64)
    verts, tris = [], []

    def v(i, j):
        if vid[i, j] < 0:
            vid[i, j] = len(verts)
            verts.append((xs[i], xs[j]))
        return vid[i, j]

    for j in range(n):
        for i in range(n):
            if not keep(i, j):
                continue
            a, b, c, d = v(i, j), v(i + 1, j), v(i + 1, j + 1), v(i, j + 1)
            tris.append((a, b, c))      # diagonal (i,j)-(i+1,j+1), CCW
            tris.append((a, c, d))
    return (np.ascontiguousarray(np.array(verts, dtype=np.float64)),
            np.ascontiguousarray(np.array(tris, dtype=np.int32)))


def square_grid(n: int):
    """Uniform right-triangle grid of the unit square: 2 n^2 triangles."""
    return _grid(n, lambda i, j: True)


def lshape_grid(n: int):
    """Uniform grid of [0,1]^2 minus [0.5,1]^2 (n even)."""
    h = n // 2
    return _grid(n, lambda i, j: not (i >= h and j >= h))


# ----------------------------------------------------------------- data
def manufactured(bnd_xy, t_nodes, vtx_xy, alpha, kvec):
    """Data of u(x,t) = exp(k.x + |k|^2 t / alpha).

    Returns (g, u0, w_ref):
      g[m*NG + n]  = u(x_n) in space times the exact mean of u over tau_m,
      u0[j]        = u(y_j, 0),
      w_ref[m*NG+i]= mean of the exact flux (k.n_i) u over gamma_i x tau_m.
    """
    k = np.asarray(kvec, dtype=np.float64)
    k2 = float(k @ k)
    t = np.asarray(t_nodes, dtype=np.float64)
    h = np.diff(t)
    if k2 == 0.0:
        tavg = np.ones_like(h)
    else:
        c = k2 / alpha
        # mean of exp(c t) over (t_m, t_{m+1}] without cancellation
        tavg = np.exp(c * t[:-1]) * np.expm1(c * h) / (c * h)
    xb = np.asarray(bnd_xy, dtype=np.float64)
    ng = xb.shape[0]
    nodal = np.exp(xb @ k)
    g = (tavg[:, None] * nodal[None, :]).reshape(-1)
    u0 = np.exp(np.asarray(vtx_xy, dtype=np.float64) @ k)
    d = np.roll(xb, -1, axis=0) - xb
    L = np.hypot(d[:, 0], d[:, 1])
    e = d / L[:, None]
    nrm = np.stack([e[:, 1], -e[:, 0]], axis=1)
    ke = (e @ k) * L
    with np.errstate(invalid="ignore", divide="ignore"):
        savg = np.where(np.abs(ke) > 0, np.expm1(ke) / np.where(ke == 0, 1, ke), 1.0)
    flux = (nrm @ k) * nodal * savg
    w_ref = (tavg[:, None] * flux[None, :]).reshape(-1)
    return g, u0, w_ref


def sine_solution(bnd_xy, t_nodes, vtx_xy, alpha, theta=math.pi / 8):
    """Data of u(x,t) = exp(-t/alpha) sin(x1 cos(theta) + x2 sin(theta)),
    the exact solution of the paper's experiments (Sec. 4).  Same
    discretisation as manufactured(): nodal in space x exact time mean."""
    t = np.asarray(t_nodes, dtype=np.float64)
    h = np.diff(t)
    tavg = alpha * (np.exp(-t[:-1] / alpha) - np.exp(-t[1:] / alpha)) / h
    kh = np.array([math.cos(theta), math.sin(theta)])
    xb = np.asarray(bnd_xy, dtype=np.float64)
    g = (tavg[:, None] * np.sin(xb @ kh)[None, :]).reshape(-1)
    u0 = np.sin(np.asarray(vtx_xy, dtype=np.float64) @ kh)
    d = np.roll(xb, -1, axis=0) - xb
    L = np.hypot(d[:, 0], d[:, 1])
    e = d / L[:, None]
    nrm = np.stack([e[:, 1], -e[:, 0]], axis=1)
    # mean over gamma_i of cos(kh.x) (kh.n_i): kh.x is linear along the segment
    a, b = xb @ kh, np.roll(xb, -1, axis=0) @ kh
    with np.errstate(invalid="ignore", divide="ignore"):
        cavg = np.where(np.abs(b - a) > 1e-14, (np.sin(b) - np.sin(a)) / np.where(b == a, 1, b - a), np.cos(a))
    w_ref = (tavg[:, None] * ((nrm @ kh) * cavg)[None, :]).reshape(-1)
    return g, u0, w_ref


def paper_level(L: int) -> "Workload":
    """The experiment of Sec. 4: Q = (0,1)^3, alpha = 10, uniform meshes with
    h_x = h_t = 2^-L (N_Gamma = 4 * 2^L segments, N_I = 2^L steps, N = 4 * 4^L,
    as in Table 1); Omega_h is the matching 2^L grid."""
    n = 2 ** L
    bnd, t, (vx, tr), alpha = square_polygon(n), uniform_times(n), square_grid(n), 10.0
    g, u0, w_ref = sine_solution(bnd, t, vx, alpha)
    return Workload(name=f"paper_L{L}", alpha=alpha, t_nodes=t, bnd_xy=bnd, vtx_xy=vx, tri=tr,
                    kvec=np.array([math.cos(math.pi / 8), math.sin(math.pi / 8)]), g=g, u0=u0, w_ref=w_ref)


# ----------------------------------------------------------------- configs
CONFIGS = ("tiny", "medium", "precision", "lshape", "diff")


def make(name: str, seed: int = 0, **over) -> Workload:
    """Build one of the named workloads (or a custom square one via overrides).

    tiny      : square, 16 segments, 16 steps, alpha=1, Omega 8x8 grid, k=(.5,.5)
    medium    : square, 256 segments, 128 steps, alpha=1, Omega 64^2, k=(1,0)
    precision : square, 512 segments, 256 steps, alpha=1, Omega 128^2, k=(.7,-.7)
    lshape    : L-shape, 384 segments, 200 graded steps (ratio 1.02), alpha=0.1,
                Omega 96-grid, k seeded (angle U[0,2pi), |k| U[.5,2])
    diff      : square, 128 segments, 128 steps, Omega 32^2; data from
                alpha*=1.5, k=(1,0); observed flux with N(0,1e-3^2) noise;
                the functional is evaluated at alpha = 1
    custom    : square with keys n_side, n_t, alpha, n_omega, k
    """
    rng = np.random.default_rng(seed)
    extra = {}
    if name == "tiny":
        bnd, t, (vx, tr), alpha, k = square_polygon(4), uniform_times(16), square_grid(8), 1.0, (0.5, 0.5)
    elif name == "medium":
        bnd, t, (vx, tr), alpha, k = square_polygon(64), uniform_times(128), square_grid(64), 1.0, (1.0, 0.0)
    elif name == "precision":
        bnd, t, (vx, tr), alpha, k = square_polygon(128), uniform_times(256), square_grid(128), 1.0, (0.7, -0.7)
    elif name == "lshape":
        bnd, t, (vx, tr), alpha = lshape_polygon(384), graded_times(200, 1.02), lshape_grid(96), 0.1
        th = rng.uniform(0.0, 2.0 * math.pi)
        mag = rng.uniform(0.5, 2.0)
        k = (mag * math.cos(th), mag * math.sin(th))
    elif name == "diff":
        bnd, t, (vx, tr) = square_polygon(32), uniform_times(128), square_grid(32)
        alpha, k = 1.0, (1.0, 0.0)
        extra["alpha_star"] = 1.5
        extra["sigma"] = 1e-3
    elif name == "custom":
        bnd = square_polygon(int(over.get("n_side", 4)))
        t = over.get("t_nodes")
        t = uniform_times(int(over.get("n_t", 4))) if t is None else np.asarray(t, np.float64)
        vx, tr = square_grid(int(over.get("n_omega", 4)))
        alpha = float(over.get("alpha", 1.0))
        k = tuple(over.get("k", (0.5, 0.5)))
    else:
        raise ValueError(f"unknown workload {name!r}")
    if name != "custom":
        if "alpha" in over:
            alpha = float(over["alpha"])
    kv = np.asarray(k, dtype=np.float64)
    if name == "diff":
        g, u0, w_ref = manufactured(bnd, t, vx, extra["alpha_star"], kv)
        extra["noise"] = rng.standard_normal(w_ref.shape[0])
    else:
        g, u0, w_ref = manufactured(bnd, t, vx, alpha, kv)
    return Workload(name=name, alpha=alpha, t_nodes=np.ascontiguousarray(t),
                    bnd_xy=bnd, vtx_xy=vx, tri=tr, kvec=kv, g=g, u0=u0,
                    w_ref=w_ref, extra=extra)
