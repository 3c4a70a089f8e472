"""Brute-force Galerkin integrals of the raw heat kernel on tiny meshes.

Test infrastructure, independent of ``oracle/`` (shares no code with it and
with the GPU library): plain numpy float64.

Time.  The double integral over tau_k x tau_m of a kernel of the lag
s = t - tau is reduced exactly to one integral in s with the trapezoid weight
w(s) = |tau_k intersected with (tau_m + s)| (Sec. 1: the Galerkin entries of
eq.(4) are integrals over pairs of space-time elements).  That integral is
taken numerically in sigma = ln s on panels of width <= 1 between the kinks of
w, against the raw fundamental solution k(r, s) = exp(-alpha r^2/(4 s))/(4 pi s)
(the 1/alpha-scaled U* of the representation formula).  No time primitive
and no exponential integral enters V, K or D.

Space.  hp-graded composite Gauss-Legendre: geometric meshes (ratio 0.25, 16 nodes per panel)
toward the singular point, in the difference variable for coincident pieces
and in Duffy coordinates about the shared vertex for pieces that share one.

D_h uses the integration-by-parts form of Sec. 2 on every pair (the raw
hypersingular kernel is not integrable over overlapping supports):
curl part psi_i' psi_j' (V-type kernel) plus alpha n_x.n_y psi_i psi_j
(d/dt of the kernel), the time derivative integrated by parts in s:
int w(s) dk/ds ds = -int w'(s) k(s) ds.

M_h^0 rows use the time integral of U* over tau_k through scipy's
exponential integral (that closed form is itself pinned against quadrature
of U* in the oracle tests); Omega's triangles are integrated in Duffy
coordinates about the test point, summed with signed areas over the three
edges.
"""
from __future__ import annotations

import functools

import numpy as np
from scipy.special import exp1

FOUR_PI = 4.0 * np.pi


@functools.lru_cache(maxsize=None)
def gl01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def composite(a, b, npan, n):
    """Gauss-Legendre with n nodes on each of npan equal panels of [a, b]."""
    x, w = gl01(n)
    e = np.linspace(a, b, npan + 1)
    h = np.diff(e)
    return (e[:-1, None] + h[:, None] * x[None, :]).ravel(), (h[:, None] * w[None, :]).ravel()


def graded(L, n=16, ratio=0.25, tiny=1e-17):
    """Nodes/weights on [0, L] on a geometric mesh toward 0: panels
    [L r^(l+1), L r^l] down to L*tiny, then one panel [0, L r^lmax]."""
    x, w = gl01(n)
    edges = [L]
    while edges[-1] > L * tiny:
        edges.append(edges[-1] * ratio)
    edges.append(0.0)
    e = np.array(edges[::-1])
    h = np.diff(e)
    return (e[:-1, None] + h[:, None] * x[None, :]).ravel(), (h[:, None] * w[None, :]).ravel()


# ------------------------------------------------------------------ time
class Lag:
    """The lag weight of tau_k x tau_m: w(s) = |(t_k, t_k+1) ^ (t_m + s, t_m+1 + s)|
    = min(h_k, h_m, s - c0, c1 - s) clipped at 0, c0 = t_k - t_m+1,
    c1 = t_k+1 - t_m (written as a minimum of differences so that w keeps its
    relative accuracy for tiny s)."""

    def __init__(self, t, k, m):
        tk0, tk1, tm0, tm1 = float(t[k]), float(t[k + 1]), float(t[m]), float(t[m + 1])
        self.hk, self.hm = tk1 - tk0, tm1 - tm0
        self.c0, self.c1 = tk0 - tm1, tk1 - tm0
        kinks = {self.c0, self.c0 + min(self.hk, self.hm), self.c1 - min(self.hk, self.hm), self.c1}
        self.kinks = sorted(c for c in kinks if c > 0)
        self.smax = self.c1

    def w(self, s):
        return np.maximum(0.0, np.minimum(np.minimum(self.hk, self.hm), np.minimum(s - self.c0, self.c1 - s)))

    def dw(self, s):
        """w'(s): +1 on the rising side (c0, c0 + min h), -1 on the falling
        side (c1 - min h, c1), 0 on the flat top and outside the support
        (decided by comparing s with the kinks, not with rounded w)."""
        flat = min(self.hk, self.hm)
        up = (s > self.c0) & (s < self.c0 + flat)
        down = (s > self.c1 - flat) & (s < self.c1)
        return up.astype(float) - down.astype(float)


def _sigma_rule(lag, amin, width=1.0, n=16):
    lo = np.log(max(amin, 1e-300) / 750.0)
    hi = np.log(lag.smax)
    cuts = sorted({lo, hi} | {np.log(c) for c in lag.kinks if lo < np.log(c) < hi})
    xs, ws = [], []
    for a, b in zip(cuts[:-1], cuts[1:]):
        npan = max(1, int(np.ceil((b - a) / width)))
        x, w = composite(a, b, npan, n)
        xs.append(x)
        ws.append(w)
    return np.concatenate(xs), np.concatenate(ws)


def time_integrals(lag, alpha, r2, kinds, chunk=4096):
    """For squared distances r2 (array) the lag integrals
      'V'  int w(s) k(r, s) ds,           k = exp(-alpha r^2/(4s))/(4 pi s)
      'K'  int w(s) k(r, s)/(2 s) ds      (times alpha (x-y).n_y: d k/d n_y)
      'Dn' -int w'(s) k(r, s) ds          (= int w(s) dk/ds ds)
    as a dict of arrays."""
    r2 = np.asarray(r2, dtype=float)
    out = {kd: np.empty_like(r2) for kd in kinds}
    flat = r2.ravel()
    order = np.argsort(flat)
    res = {kd: np.empty_like(flat) for kd in kinds}
    for c0 in range(0, flat.size, chunk):
        idx = order[c0:c0 + chunk]
        a = 0.25 * alpha * flat[idx]
        sg, wg = _sigma_rule(lag, a.min())
        s = np.exp(sg)
        e = np.exp(-a[:, None] / s[None, :])             # (n, q)
        base = e / FOUR_PI                                # k(r, s) * s (ds = s dsigma)
        for kd in kinds:
            if kd == "V":
                f = base * (lag.w(s) * wg)[None, :]
            elif kd == "K":
                f = base * (lag.w(s) * wg / (2.0 * s))[None, :]
            elif kd == "Dn":
                f = -base * (lag.dw(s) * wg)[None, :]
            else:
                raise ValueError(kd)
            res[kd][idx] = f.sum(axis=1)
    for kd in kinds:
        out[kd] = res[kd].reshape(r2.shape)
    return out


# ----------------------------------------------------------------- space
class Piece:
    """A straight piece from a with unit tangent e and length L; outward
    normal n = (e_y, -e_x) of a counter-clockwise polygon."""

    def __init__(self, a, e, L):
        self.a = np.asarray(a, float)
        self.e = np.asarray(e, float)
        self.L = float(L)
        self.n = np.array([self.e[1], -self.e[0]])
        self.b = self.a + self.L * self.e


def _same_point(p, q):
    return np.hypot(*(np.asarray(p) - np.asarray(q))) <= 1e-14


def pair_rule(P, Q, nsep=4, n=12):
    """Quadrature over P x Q: returns sP, sQ (arclength from each start),
    dx, dy (components of x - y, formed from small offsets near a shared
    point) and weights."""
    if _same_point(P.a, Q.a) and _same_point(P.b, Q.b):
        eps, we = graded(P.L, n)
        xs, ws = gl01(6)                                   # polynomial in s for fixed eps
        s = (P.L - eps)[:, None] * xs[None, :]
        w = (we * (P.L - eps))[:, None] * ws[None, :]
        e = np.broadcast_to(eps[:, None], s.shape)
        # x ahead of y and y ahead of x
        sP = np.concatenate([(s + e).ravel(), s.ravel()])
        sQ = np.concatenate([s.ravel(), (s + e).ravel()])
        d = np.concatenate([e.ravel(), -e.ravel()])
        W = np.concatenate([w.ravel(), w.ravel()])
        return sP, sQ, d * P.e[0], d * P.e[1], W
    shared = None
    for pa, pend in ((P.a, False), (P.b, True)):
        for qa, qend in ((Q.a, False), (Q.b, True)):
            if _same_point(pa, qa):
                shared = (pend, qend)
    if shared is not None:
        pend, qend = shared
        e1 = -P.e if pend else P.e                         # away from the shared vertex
        e2 = -Q.e if qend else Q.e
        xi, wxi = graded(1.0, n)
        eta, weta = gl01(20)
        parts = []
        for tri in (0, 1):
            X, E = np.meshgrid(xi, eta, indexing="ij")
            WX, WE = np.meshgrid(wxi, weta, indexing="ij")
            if tri == 0:
                u, v = P.L * X, Q.L * X * E
            else:
                u, v = P.L * X * E, Q.L * X
            W = WX * WE * P.L * Q.L * X
            parts.append((u.ravel(), v.ravel(), W.ravel()))
        u = np.concatenate([p[0] for p in parts])
        v = np.concatenate([p[1] for p in parts])
        W = np.concatenate([p[2] for p in parts])
        sP = P.L - u if pend else u
        sQ = Q.L - v if qend else v
        dx = u * e1[0] - v * e2[0]
        dy = u * e1[1] - v * e2[1]
        return sP, sQ, dx, dy, W
    sp, wp = composite(0.0, P.L, nsep, n)
    sq, wq = composite(0.0, Q.L, nsep, n)
    SP, SQ = np.meshgrid(sp, sq, indexing="ij")
    WP, WQ = np.meshgrid(wp, wq, indexing="ij")
    X = P.a[None, None, :] + SP[..., None] * P.e
    Y = Q.a[None, None, :] + SQ[..., None] * Q.e
    Z = X - Y
    return SP.ravel(), SQ.ravel(), Z[..., 0].ravel(), Z[..., 1].ravel(), (WP * WQ).ravel()


# ------------------------------------------------------------- the mesh
class Mesh:
    """Closed counter-clockwise polygon (vertices bnd, segment i from vertex i
    to i+1), time nodes t, alpha."""

    def __init__(self, alpha, t, bnd):
        self.alpha = float(alpha)
        self.t = np.asarray(t, float)
        self.bnd = np.asarray(bnd, float)
        self.ng = self.bnd.shape[0]
        d = np.roll(self.bnd, -1, axis=0) - self.bnd
        self.Ls = np.hypot(d[:, 0], d[:, 1])
        self.es = d / self.Ls[:, None]

    def seg(self, i):
        i %= self.ng
        return Piece(self.bnd[i], self.es[i], self.Ls[i])

    def dual_support(self, i):
        """The dual hat psi_i (1 at the midpoint of segment i, 0 at the
        midpoints of segments i-1 and i+1, linear in arclength between) on
        its four half-segment pieces: (piece, psi at start, psi at end,
        d psi/ds)."""
        ng = self.ng
        im, ip = (i - 1) % ng, (i + 1) % ng
        L, e, b = self.Ls, self.es, self.bnd
        Lt0, Lt1 = 0.5 * (L[im] + L[i]), 0.5 * (L[i] + L[ip])
        mid = lambda j: b[j] + 0.5 * L[j] * e[j]
        return [
            (Piece(mid(im), e[im], 0.5 * L[im]), 0.0, 0.5 * L[im] / Lt0, 1.0 / Lt0),
            (Piece(b[i], e[i], 0.5 * L[i]), 0.5 * L[im] / Lt0, 1.0, 1.0 / Lt0),
            (Piece(mid(i), e[i], 0.5 * L[i]), 1.0, 1.0 - 0.5 * L[i] / Lt1, -1.0 / Lt1),
            (Piece(b[ip], e[ip], 0.5 * L[ip]), 1.0 - 0.5 * L[i] / Lt1, 0.0, -1.0 / Lt1),
        ]

    # ---------------------------------------------------------- entries
    def V(self, k, m, i, j):
        if k < m:
            return 0.0
        lag = Lag(self.t, k, m)
        sP, sQ, dx, dy, W = pair_rule(self.seg(i), self.seg(j))
        T = time_integrals(lag, self.alpha, dx * dx + dy * dy, ["V"])
        return float(np.sum(W * T["V"]))

    def K(self, k, m, i, n):
        """Column n: the hat of polygon vertex n, rising on segment n-1 and
        falling on segment n; kernel d k / d n_y = alpha (x-y).n_y k / (2 s)."""
        if k < m:
            return 0.0
        lag = Lag(self.t, k, m)
        P = self.seg(i)
        acc = 0.0
        for Q, rising in ((self.seg(n - 1), True), (self.seg(n), False)):
            sP, sQ, dx, dy, W = pair_rule(P, Q)
            zn = dx * Q.n[0] + dy * Q.n[1]
            if not np.any(zn != 0.0):
                continue
            T = time_integrals(lag, self.alpha, dx * dx + dy * dy, ["K"])
            hat = sQ / Q.L if rising else 1.0 - sQ / Q.L
            acc += float(np.sum(W * self.alpha * zn * hat * T["K"]))
        return acc

    def D(self, k, m, i, j):
        if k < m:
            return 0.0
        lag = Lag(self.t, k, m)
        acc = 0.0
        for (P, p0, p1, dp) in self.dual_support(i):
            for (Q, q0, q1, dq) in self.dual_support(j):
                sP, sQ, dx, dy, W = pair_rule(P, Q)
                T = time_integrals(lag, self.alpha, dx * dx + dy * dy, ["V", "Dn"])
                psi_i = p0 + (p1 - p0) * sP / P.L
                psi_j = q0 + (q1 - q0) * sQ / Q.L
                nn = float(P.n @ Q.n)
                acc += dp * dq * float(np.sum(W * T["V"]))
                acc += self.alpha * nn * float(np.sum(W * psi_i * psi_j * T["Dn"]))
        return acc


# ----------------------------------------------------------------- M_h^0
def m0_kernel(alpha, t, k, r2):
    """int_{tau_k} U*(r, t) dt, U* = alpha/(4 pi t) exp(-alpha r^2/(4 t))
    (the semigroup kernel of alpha u_t = Laplace u)."""
    a = 0.25 * alpha * np.asarray(r2, float)
    t0, t1 = float(t[k]), float(t[k + 1])
    v = exp1(a / t1)
    if t0 > 0:
        v = v - exp1(a / t0)
    return alpha / FOUR_PI * v


def _graded_around(c, dist, n=16):
    """Nodes/weights on [0, 1] graded geometrically toward c in [0, 1] from
    both sides, down to panels of about dist (the distance of a nearby
    singularity from the real axis)."""
    xs, ws = [], []
    for length, sign in ((c, -1.0), (1.0 - c, 1.0)):
        if length <= 0:
            continue
        g, w = graded(length, n, tiny=max(0.25 * dist / length, 1e-13))
        xs.append(c + sign * g)
        ws.append(w)
    return np.concatenate(xs), np.concatenate(ws)


def _tri_polar(xp, A, B, n=16, neta=16):
    """Duffy rule on the triangle (xp, A, B) about xp: y = xp + xi (A - xp) +
    xi eta (B - A); weight carries the signed area (positive if CCW).  In
    eta, |y - xp| / xi = |A - xp + eta (B - A)| vanishes at a complex eta
    whose real part is the projection of xp on the line AB and whose
    imaginary part is dist(xp, AB)/|B - A|: when that is close to [0, 1] the
    eta rule is graded toward the projection."""
    xi, wxi = graded(1.0, n, tiny=1e-12)
    d = B - A
    dd = float(d @ d)
    ep = float(-(A - xp) @ d) / dd
    u = A - xp
    area2 = u[0] * d[1] - u[1] * d[0]
    dperp = abs(area2) / dd
    if -0.5 < ep < 1.5 and dperp < 0.5:
        eta, weta = _graded_around(min(max(ep, 0.0), 1.0), max(dperp, abs(ep - min(max(ep, 0.0), 1.0))))
    else:
        eta, weta = gl01(neta)
    X, E = np.meshgrid(xi, eta, indexing="ij")
    WX, WE = np.meshgrid(wxi, weta, indexing="ij")
    y = xp[None, None, :] + X[..., None] * u + (X * E)[..., None] * d
    return y.reshape(-1, 2), (WX * WE * X).ravel() * area2


def m0_entry(alpha, t, k, seg, tris, vtx, j):
    """M_h^0[(k, i), j] = int_{gamma_i} int_Omega phi_j(y) int_{tau_k} U* dt dy ds_x
    over the triangles containing vertex j (tris: (ntri, 3) vertex indices).
    The segment is split at the projections of the triangles' vertices and
    graded toward each split point."""
    acc = 0.0
    for tri in tris:
        if j not in tri:
            continue
        V = vtx[list(tri)]
        cuts = {0.0, seg.L}
        for p in V:
            s = float((p - seg.a) @ seg.e)
            if 1e-12 * seg.L < s < seg.L * (1 - 1e-12):
                cuts.add(s)
        cuts = sorted(cuts)
        # barycentric hat of j on this triangle
        lj = list(tri).index(j)
        Bv, Cv = V[(lj + 1) % 3], V[(lj + 2) % 3]
        det = (V[1, 0] - V[0, 0]) * (V[2, 1] - V[0, 1]) - (V[1, 1] - V[0, 1]) * (V[2, 0] - V[0, 0])
        hat = lambda y: ((Cv[0] - Bv[0]) * (y[:, 1] - Bv[1]) - (Cv[1] - Bv[1]) * (y[:, 0] - Bv[0])) / det
        s_nodes, s_w = [], []
        for a, b in zip(cuts[:-1], cuts[1:]):
            # graded toward both ends of [a, b]
            g, wg = graded(0.5 * (b - a), 16, tiny=1e-10)
            s_nodes += [a + g, b - g]
            s_w += [wg, wg]
        s_nodes, s_w = np.concatenate(s_nodes), np.concatenate(s_w)
        part = 0.0
        for s, ws in zip(s_nodes, s_w):
            xp = seg.a + s * seg.e
            for q in range(3):
                A, Bq = V[q], V[(q + 1) % 3]
                ar = (A[0] - xp[0]) * (Bq[1] - A[1]) - (A[1] - xp[1]) * (Bq[0] - A[0])
                if abs(ar) <= 1e-15 * float((Bq - A) @ (Bq - A)):
                    continue                  # xp on this edge's line: no area
                y, wy = _tri_polar(xp, A, Bq)
                r2 = ((y - xp) ** 2).sum(1)
                part += ws * float(np.sum(wy * hat(y) * m0_kernel(alpha, t, k, r2)))
        acc += part * np.sign(det)
    return acc


def m0_entry_packed(args):
    """m0_entry for a worker process: (alpha, t, k, segment start, tangent,
    length, triangles, vertices, j)."""
    alpha, t, k, a, e, L, tris, vtx, j = args
    return m0_entry(alpha, t, k, Piece(a, e, L), tris, vtx, j)


def entry_packed(args):
    """One V, K or D entry for a worker process: (alpha, t, bnd, op, k, m, i, j)."""
    alpha, t, bnd, op, k, m, i, j = args
    return getattr(Mesh(alpha, t, bnd), op)(k, m, i, j)
