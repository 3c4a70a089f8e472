"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Nothing here compares the oracle with itself: every check is a table of
independent values, a brute-force integral of the raw fundamental solution,
an exact identity of the continuous problem (affine solutions, constants),
or an invariance of the kernel (causality, time translation, scaling).
"""
import os

import mpmath as mp
import numpy as np
import pytest

import workloads as W
from oracle import oracle as O
from oracle.oracle import Oracle, packed_apply, packed_index

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _normals(bnd):
    d = np.roll(bnd, -1, axis=0) - bnd
    L = np.hypot(d[:, 0], d[:, 1])
    e = d / L[:, None]
    return L, e, np.stack([e[:, 1], -e[:, 0]], 1)


# --------------------------------------------------------------- E1 table
def test_e1_table():
    rows = [l.split() for l in open(os.path.join(GOLD, "e1_table.txt")) if not l.startswith("#")]
    for z, v in rows:
        assert O.e1(float(z)) == pytest.approx(float(v), rel=2e-16, abs=0)


# ------------------------------------------- time integrals vs brute force
@pytest.mark.parametrize("d,r", [(0, 0.4), (1, 0.05), (2, 0.03), (5, 1.3), (1, 1.3)])
def test_time_integrals_vs_quadrature(d, r):
    """Closed forms of the double time integrals (Sec. 1, U*) against mpmath
    2-D quadrature of the raw kernels over tau_k x tau_m (split at t = tau)."""
    mp.mp.dps = 20
    alpha = 1.7
    t = np.array([0.0, 0.11, 0.2, 0.37, 0.5, 0.66, 0.8, 0.97, 1.1])    # graded on purpose
    o = Oracle(alpha, t, W.square_polygon(1))
    k, m = 1 + d, 1
    a = mp.mpf(alpha) * mp.mpf(r) ** 2 / 4
    kern = {
        "V": lambda s: mp.exp(-a / s) / (4 * mp.pi * s),
        "K": lambda s: a * mp.exp(-a / s) / s ** 2,                   # F_K'' (times (x-y).n/(2 pi r^2))
        "D": lambda s: mp.exp(-a / s) * (a - s) / (4 * mp.pi * s ** 3),   # d/ds of the V kernel
        "dV": lambda s: -(mp.mpf(r) ** 2 / (4 * s)) * mp.exp(-a / s) / (4 * mp.pi * s),
        # dK_h/dalpha: at fixed r the alpha-derivative of the K kernel
        # alpha (x-y).n_y e^{-a/s}/(8 pi s^2) is -(x-y).n_y/(8 pi) times
        # e^{-a/s}(a - s)/s^3 (the four-point difference of E1(a/delta))
        "E1": lambda s: mp.exp(-a / s) * (a - s) / s ** 3,
    }
    tk0, tk1, tm0, tm1 = map(mp.mpf, (t[k], t[k + 1], t[m], t[m + 1]))
    for name, f in kern.items():
        def inner(tt):
            hi = min(tt, tm1)
            if hi <= tm0:
                return mp.mpf(0)
            return mp.quad(lambda tau: f(tt - tau) if tt > tau else mp.mpf(0), [tm0, hi])
        ref = mp.quad(inner, [tk0, tk1])
        val = o.time_integral(name, r, k, m)
        assert val == pytest.approx(float(ref), rel=1e-12, abs=1e-300), name


@pytest.mark.parametrize("k", [0, 3])
def test_m0_time_integral(k):
    mp.mp.dps = 30
    alpha, r = 2.3, 0.21
    t = W.uniform_times(6)
    o = Oracle(alpha, t, W.square_polygon(1))
    a = mp.mpf(alpha) * mp.mpf(r) ** 2 / 4
    f = lambda s: alpha / (4 * mp.pi * s) * mp.exp(-a / s)
    ref = mp.quad(f, [t[k], t[k + 1]])
    assert o.m0_time(r, k) == pytest.approx(float(ref), rel=1e-13)
    g = lambda al: mp.quad(lambda s: al / (4 * mp.pi * s) * mp.exp(-al * mp.mpf(r) ** 2 / (4 * s)), [t[k], t[k + 1]])
    dref = mp.diff(g, mp.mpf(alpha))
    assert o.m0_time(r, k, deriv=True) == pytest.approx(float(dref), rel=1e-11)


# ------------------------------------------------ brute-force entries
def _time_weight_nodes(t, k, m, n=48):
    """Nodes/weights for int_{tau_k} int_{tau_m} f(t - tau) = int w(s) f(s) ds."""
    br = sorted({t[k] - t[m + 1], t[k] - t[m], t[k + 1] - t[m + 1], t[k + 1] - t[m]})
    br = [max(b, 0.0) for b in br]
    x, wq = np.polynomial.legendre.leggauss(n)
    S, Wt = [], []
    for a, b in zip(br[:-1], br[1:]):
        if b <= a:
            continue
        s = 0.5 * (b - a) * (x + 1) + a
        w = np.maximum(0, np.minimum(t[k + 1], t[m + 1] + s) - np.maximum(t[k], t[m] + s))
        S.append(s)
        Wt.append(0.5 * (b - a) * wq * w)
    return np.concatenate(S), np.concatenate(Wt)


def _gauss_on(a, e, L, n):
    x, w = np.polynomial.legendre.leggauss(n)
    s = 0.5 * L * (x + 1)
    return a[None, :] + s[:, None] * e[None, :], 0.5 * L * w, s


def _brute_pair(alpha, t, k, m, P, Q, kernel, n=24):
    """4-D brute force of a separated piece pair: Gauss in x, y and in the
    time lag s with the exact trapezoid weight of tau_k x tau_m."""
    S, Ws = _time_weight_nodes(t, k, m)
    X, wx, sx = _gauss_on(*P, n)
    Y, wy, sy = _gauss_on(*Q, n)
    Z = X[:, None, :] - Y[None, :, :]
    r2 = (Z ** 2).sum(-1)
    s = S[None, None, :]
    kv = np.exp(-alpha * r2[..., None] / (4 * s)) / (4 * np.pi * s)
    val = kernel(kv, s, Z, sx, sy)
    return np.einsum("i,j,ijs,s->", wx, wy, val, Ws)


@pytest.mark.parametrize("d", [0, 1, 3])
def test_V_K_entries_brute_force(d):
    """V_h and K_h entries of separated segments (Sec. 1, eq.(4)) from the raw
    U* and its normal derivative, integrated in x, y and t - tau."""
    alpha = 1.3
    bnd = W.square_polygon(3)
    t = W.graded_times(6, 1.3)
    o = Oracle(alpha, t, bnd)
    L, e, nrm = _normals(bnd)
    k, m = 1 + d, 1
    for i, j in [(0, 4), (1, 7), (2, 9)]:
        P = (bnd[i], e[i], L[i])
        Q = (bnd[j], e[j], L[j])
        ref = _brute_pair(alpha, t, k, m, P, Q, lambda kv, s, Z, sx, sy: kv)
        assert o.entries("V", [(k, m, i, j)])[0] == pytest.approx(ref, rel=1e-11)
        # K: hat of node j+1 restricted to segment j (rising part, shape s/L)
        nq = nrm[j]
        kk = lambda kv, s, Z, sx, sy: kv * alpha * (Z @ nq)[..., None] / (2 * s) * (sy / L[j])[None, :, None]
        ref_k_rise = _brute_pair(alpha, t, k, m, P, Q, kk)
        Q2 = (bnd[(j + 1) % 12], e[(j + 1) % 12], L[(j + 1) % 12])
        nq2 = nrm[(j + 1) % 12]
        kk2 = lambda kv, s, Z, sx, sy: kv * alpha * (Z @ nq2)[..., None] / (2 * s) * (1 - sy / L[j])[None, :, None]
        ref_k_fall = _brute_pair(alpha, t, k, m, P, Q2, kk2)
        got = o.entries("K", [(k, m, i, (j + 1) % 12)])[0]
        assert got == pytest.approx(ref_k_rise + ref_k_fall, rel=1e-10, abs=1e-15 * abs(ref_k_rise))


@pytest.mark.parametrize("d", [0, 1, 2])
def test_D_entries_vs_raw_hypersingular_kernel(d):
    """D_h from the integration-by-parts form equals the Galerkin integral of
    the raw kernel -d_nx d_ny (1/alpha)U* when the supports of psi_i, psi_j
    are disjoint (Sec. 2: D = -d_n W).  Covers same-side, perpendicular and
    opposite-side pairs (n_x.n_y = 1, 0, -1)."""
    alpha = 0.9
    bnd = W.square_polygon(4)
    ng = 16
    t = W.uniform_times(5)
    o = Oracle(alpha, t, bnd)
    L, e, nrm = _normals(bnd)
    mid = bnd + 0.5 * L[:, None] * e

    def pieces(i):
        im, ip = (i - 1) % ng, (i + 1) % ng
        Lt0, Lt1 = 0.5 * (L[im] + L[i]), 0.5 * (L[i] + L[ip])
        return [  # (start, e, length, normal, psi at start, psi at end)
            (mid[im], e[im], L[im] / 2, nrm[im], 0.0, 0.5 * L[im] / Lt0),
            (bnd[i], e[i], L[i] / 2, nrm[i], 0.5 * L[im] / Lt0, 1.0),
            (mid[i], e[i], L[i] / 2, nrm[i], 1.0, 1 - 0.5 * L[i] / Lt1),
            (bnd[ip], e[ip], L[ip] / 2, nrm[ip], 1 - 0.5 * L[i] / Lt1, 0.0)]

    k, m = 1 + d, 1
    for i, j in [(0, 5), (1, 8), (2, 11), (5, 10)]:
        ref = 0.0
        for (pa, pe, pl, pn, p0, p1) in pieces(i):
            for (qa, qe, ql, qn, q0, q1) in pieces(j):
                def kern(kv, s, Z, sx, sy, pn=pn, qn=qn, pl=pl, ql=ql, p0=p0, p1=p1, q0=q0, q1=q1):
                    zx = (Z @ pn)[..., None]
                    zy = (Z @ qn)[..., None]
                    raw = kv * ((alpha ** 2 / (4 * s ** 2)) * zx * zy - (alpha / (2 * s)) * (pn @ qn))
                    psx = (p0 + (p1 - p0) * sx / pl)[:, None, None]
                    psy = (q0 + (q1 - q0) * sy / ql)[None, :, None]
                    return raw * psx * psy
                ref += _brute_pair(alpha, t, k, m, (pa, pe, pl), (qa, qe, ql), kern, n=16)
        got = o.entries("D", [(k, m, i, j)])[0]
        assert got == pytest.approx(ref, rel=1e-9, abs=1e-12 * abs(ref) + 1e-16)


def test_D_time_primitive_is_step_derivative_of_V():
    """F_D is the first antiderivative of the kernel and F_V the second, so on
    one time element (d = 0) the D-type time integral is the h-derivative of
    the V-type one (central difference in h, step 1e-4 h)."""
    alpha, h, eps = 1.0, 0.2, 2e-5
    bnd = W.square_polygon(2)
    o = Oracle(alpha, np.array([0.0, h]), bnd)
    fv = lambda hh, r: Oracle(alpha, np.array([0.0, hh]), bnd).time_integral("V", r, 0, 0)
    for r in (0.01, 0.37, 1.2):
        fd = o.time_integral("D", r, 0, 0)
        assert fd == pytest.approx((fv(h + eps, r) - fv(h - eps, r)) / (2 * eps), rel=1e-7)


# ------------------------------------------------ exact discrete identities
@pytest.fixture(scope="module")
def small():
    wl = W.make("custom", n_side=2, n_t=3, n_omega=2, alpha=1.0)
    o = Oracle.from_workload(wl)
    return wl, o, o.packed("V"), o.packed("K"), o.m0()


def test_affine_exactness(small):
    """u = c0 + c.x solves the heat equation; g, u0 are then exactly in the
    discrete spaces and w = c.n_i is exactly piecewise constant, so eq.(4)
    holds exactly: V_h w = (1/2 M_h + K_h) g - M_h^0 u0 (V, K, M, M0 together)."""
    wl, o, V, K, M0 = small
    c0, c = 0.7, np.array([0.3, -1.1])
    g = np.tile(c0 + wl.bnd_xy @ c, o.nt)
    u0 = c0 + wl.vtx_xy @ c
    _, _, nrm = _normals(wl.bnd_xy)
    w = np.tile(nrm @ c, o.nt)
    f = o.rhs(K, M0, g, u0)
    r = packed_apply(V, w, o.nt, o.ng) - f
    assert np.linalg.norm(r) / np.linalg.norm(f) < 1e-14
    wd = o.solve_direct(V, f)
    assert np.linalg.norm(wd - w) / np.linalg.norm(w) < 1e-13


def test_constant_identity(small):
    """u = 1: w = 0, so (1/2 M_h + K_h) 1 = M_h^0 1."""
    wl, o, V, K, M0 = small
    lhs = 0.5 * o.mass_apply(np.ones(o.n)) + packed_apply(K, np.ones(o.n), o.nt, o.ng)
    rhs = M0 @ np.ones(o.nv)
    assert np.linalg.norm(lhs - rhs) / np.linalg.norm(rhs) < 1e-14


def test_causality_toeplitz_symmetry(small):
    """Blocks with tau_k before tau_m vanish (Sec. 3, block lower triangular);
    uniform steps make block (k,m) depend on k - m only; diagonal time blocks
    of V_h are symmetric and V_h has a positive definite symmetric part."""
    wl, o, V, K, M0 = small
    assert np.all(o.entries("V", [(0, 1, 0, 0), (1, 2, 3, 5)]) == 0.0)
    assert np.all(o.entries("D", [(0, 2, 1, 1)]) == 0.0)
    for op, P in (("V", V), ("K", K)):
        assert np.abs(P[packed_index(2, 1)] - P[packed_index(1, 0)]).max() <= 1e-14 * np.abs(P[packed_index(1, 0)]).max()
    B = V[packed_index(1, 1)]
    assert np.abs(B - B.T).max() <= 1e-15 * np.abs(B).max()
    A = o.dense(V)
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0


def test_scaling_laws():
    """A(alpha, t) = alpha A(1, t/alpha) for V, K, D; parabolic scaling
    V(lam x, lam^2 t) = lam^4 V(x, t), K ~ lam^3, D ~ lam^2."""
    bnd = W.square_polygon(2)
    t = W.uniform_times(3)
    al, lam = 2.5, 1.7
    idx = [(0, 0, 0, 0), (1, 0, 0, 1), (2, 0, 1, 4), (2, 1, 3, 4)]
    a1 = Oracle(al, t, bnd)
    a2 = Oracle(1.0, t / al, bnd)
    s1 = Oracle(1.0, t, bnd)
    s2 = Oracle(1.0, lam ** 2 * t, lam * bnd)
    for op, p in (("V", 4), ("K", 3), ("D", 2)):
        x1, x2 = a1.entries(op, idx), a2.entries(op, idx)
        np.testing.assert_allclose(x1, al * x2, rtol=1e-13, atol=1e-15 * np.abs(x1).max())
        y1, y2 = s1.entries(op, idx), s2.entries(op, idx)
        np.testing.assert_allclose(y2, lam ** p * y1, rtol=1e-13, atol=1e-15 * np.abs(y2).max())


def test_gmres_matches_block_forward_substitution():
    wl = W.make("custom", n_side=2, n_t=4, n_omega=2, alpha=1.0, k=(0.6, 0.2))
    o = Oracle.from_workload(wl)
    V, K, D, M0 = o.packed("V"), o.packed("K"), o.packed("D"), o.m0()
    f = o.rhs(K, M0, wl.g, wl.u0)
    wd = o.solve_direct(V, f)
    wg, it, _ = o.solve_gmres(V, D, f, tol=1e-14)
    assert np.linalg.norm(wg - wd) / np.linalg.norm(wd) < 1e-12
    wn, itn, _ = o.solve_gmres(V, D, f, tol=1e-14, precondition=False)
    assert np.linalg.norm(wn - wd) / np.linalg.norm(wd) < 1e-12


def _affine_data(wl, c0, c):
    """Cauchy data of u = c0 + c.x (a stationary solution of alpha u_t = Lap u):
    g nodal and constant in time, w = c.n per segment, u0 nodal; all exact in
    the discrete spaces."""
    bnd = wl.bnd_xy
    d = np.roll(bnd, -1, axis=0) - bnd
    L = np.hypot(d[:, 0], d[:, 1])
    e = d / L[:, None]
    nrm = np.stack([e[:, 1], -e[:, 0]], 1)
    nt = wl.n_t
    return np.tile(nrm @ c, nt), np.tile(c0 + bnd @ c, nt), c0 + wl.vtx_xy @ c


@pytest.mark.parametrize("name", ["tiny", "lshape_small"])
def test_representation_formula_reproduces_affine_solutions(name):
    """Sec. 1, eq. (2): u = M~0 u0 + V~ w - W g holds for the exact Cauchy data
    of any solution; for u = c0 + c.x those data are exact in the discrete
    spaces, so the oracle's three potentials must return u at interior
    points and times to rounding (a dropped 1/alpha, a wrong sign of the
    double layer or of a time limit, or a missing hat would break it)."""
    if name == "tiny":
        wl = W.make("tiny")
    else:
        bnd = W.lshape_polygon(16)
        t = W.uniform_times(5)
        vx, tr = W.lshape_grid(6)
        wl = W.Workload(name="ls", alpha=0.3, t_nodes=t, bnd_xy=bnd, vtx_xy=vx, tri=tr,
                        kvec=np.array([1.0, 0.0]), g=None, u0=None, w_ref=None)
    o = Oracle.from_workload(wl)
    c0, c = 0.7, np.array([0.3, -1.1])
    w, g, u0 = _affine_data(wl, c0, c)
    pts = np.array([[0.25, 0.25, 1.0], [0.2, 0.7, 0.3], [0.4, 0.1, 0.05], [0.05, 0.3, 0.5], [0.3, 0.3, 0.01],
                    [0.33, 0.4, 0.0625], [0.45, 0.45, 0.9]])
    P = o.potential(pts, w, g, u0)
    u = P[:, 0] + P[:, 1] - P[:, 2]
    assert np.abs(u - (c0 + pts[:, :2] @ c)).max() <= 1e-14
    # the constant u = 1: only the initial and the double-layer potential
    P1 = o.potential(pts, 0 * w, 0 * g + 1, 0 * u0 + 1)
    assert np.abs(P1[:, 0] - P1[:, 2] - 1).max() <= 1e-14


# ------------------------------------------- alpha-derivatives by differences
def test_alpha_derivatives_vs_central_differences():
    """dV_h/dalpha, dK_h/dalpha (entries, touching and separated time
    elements, singular pairs included) and dM_h^0/dalpha (rows of the first
    steps) equal central differences in alpha of the oracle's own V_h, K_h,
    M_h^0, Richardson-extrapolated from steps 1e-3 alpha and 5e-4 alpha
    (truncation O(h^4) ~ 1e-12): the derivative formulas are pinned by the
    definition of a derivative, not by themselves."""
    alpha = 1.3
    wl = W.make("custom", n_side=2, n_t=4, n_omega=2, alpha=alpha)
    t, bnd, vx, tr = wl.t_nodes, wl.bnd_xy, wl.vtx_xy, wl.tri
    mk = lambda al: Oracle(al, t, bnd, vx, tr)
    o = mk(alpha)
    idx = [(0, 0, 1, 1), (0, 0, 1, 2), (1, 0, 1, 2), (1, 0, 2, 5), (3, 1, 0, 6), (2, 0, 3, 3), (3, 0, 7, 1)]

    def cdiff(fn, h):
        return (fn(mk(alpha + h)) - fn(mk(alpha - h))) / (2 * h)

    def richardson(fn):
        h = 1e-3 * alpha
        return (4 * cdiff(fn, h / 2) - cdiff(fn, h)) / 3

    for op, dop in (("V", "dV"), ("K", "dK")):
        fd = richardson(lambda oo: oo.entries(op, idx))
        got = o.entries(dop, idx)
        np.testing.assert_allclose(got, fd, rtol=1e-9, atol=1e-11 * np.abs(fd).max(), err_msg=dop)
    rows = [(0, 0), (0, 3), (1, 5), (3, 2)]
    fd = richardson(lambda oo: oo.m0_rows(rows))
    got = o.m0_rows(rows, deriv=True)
    np.testing.assert_allclose(got, fd, rtol=1e-9, atol=1e-11 * np.abs(fd).max(), err_msg="dM0")


# ------------------------------------------------- D_h: symmetry, positivity
def test_D_symmetric_blocks_and_positive_definite():
    """The kernel of every time block of D_h is symmetric in x and y
    (it depends on |x - y| and n_x.n_y only), so every block D_(k,m) is a
    symmetric matrix; the causal matrix has a positive definite symmetric
    part (the hypersingular operator is elliptic, Sec. 2, Theorem 1).  The
    oracle computes (i, j) and (j, i) with the pieces in swapped roles."""
    wl = W.make("custom", n_side=2, n_t=4, n_omega=2, alpha=0.7,
                t_nodes=W.graded_times(4, 1.5))
    o = Oracle.from_workload(wl)
    D = o.packed("D")
    for b in range(D.shape[0]):
        B_ = D[b]
        assert np.abs(B_ - B_.T).max() <= 1e-14 * np.abs(B_).max(), b
    A = o.dense(D)
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0


# ------------------------------------------------ lumped dual mass matrix
def test_lumped_dual_mass_vs_quadrature():
    """The lumped mass of the preconditioner (Sec. 4): for each dual hat
    psi_i, the sum over the primal indicators phi_k of <phi_k, psi_i> is the
    integral of psi_i over Gamma times h_m.  Computed here by Gauss
    quadrature of the dual hat from its definition (1 at the midpoint of
    segment i, 0 at the midpoints of segments i -/+ 1, linear in arclength)
    on a polygon with unequal segments; the row sums over the dual hats give
    |gamma_k| (the dual hats are a partition of unity)."""
    rng = np.random.default_rng(3)
    ang = np.sort(rng.uniform(0, 2 * np.pi, 9))
    rad = rng.uniform(0.7, 1.3, 9)
    bnd = np.stack([rad * np.cos(ang), rad * np.sin(ang)], 1)
    t = W.graded_times(3, 1.4)
    o = Oracle(1.0, t, bnd)
    ng = bnd.shape[0]
    L, e, _ = _normals(bnd)
    cum = np.concatenate([[0.0], np.cumsum(L)])          # arclength of vertex i
    P = cum[-1]
    mids = cum[:-1] + 0.5 * L

    def psi(i, s):
        """Dual hat i at arclength s (periodic)."""
        c, lo, hi = mids[i], mids[i - 1] - (P if i == 0 else 0), mids[(i + 1) % ng] + (P if i == ng - 1 else 0)
        s = np.where(s < lo, s + P, np.where(s > hi, s - P, s))
        return np.clip(np.where(s <= c, (s - lo) / (c - lo), (hi - s) / (hi - c)), 0, 1)

    x, w = np.polynomial.legendre.leggauss(8)
    Mk = np.zeros((ng, ng))
    for k in range(ng):
        for half in (0, 1):                                  # psi is linear on each half segment
            a = cum[k] + half * 0.5 * L[k]
            s = a + 0.25 * L[k] * (x + 1)
            for i in range(ng):
                Mk[k, i] = Mk[k, i] + np.sum(0.25 * L[k] * w * psi(i, s))
    np.testing.assert_allclose(Mk.sum(1), L, rtol=1e-14)
    h = np.diff(t)
    lump = (h[:, None] * Mk.sum(0)[None, :]).reshape(-1)
    np.testing.assert_allclose(o.lumped_dual_mass(), lump, rtol=1e-14)


# ----------------------------------------------- convergence of the flux
def test_neumann_datum_converges_for_manufactured_solution():
    """u = exp(k.x + |k|^2 t/alpha) solves alpha u_t = Laplace u; its Neumann
    datum w = (k.n) u.  With h_x = h_t halved per level (square, Omega_h the
    matching grid), the oracle's discrete flux (eq.(4) solved by block
    forward substitution) approaches the exact flux: the L2(Sigma) error of
    w_h against the element means of w falls at every level, with an
    observed order above 1."""
    errs = []
    for L in (1, 2, 3):
        n = 2 ** L
        wl = W.make("custom", n_side=n, n_t=n, n_omega=n, alpha=1.0, k=(0.5, 0.5))
        o = Oracle.from_workload(wl)
        V, K, M0 = o.packed("V"), o.packed("K"), o.m0()
        w = o.solve_direct(V, o.rhs(K, M0, wl.g, wl.u0))
        wt = np.repeat(o.h, o.ng) * np.tile(o.L, o.nt)
        errs.append(np.sqrt(np.sum(wt * (w - wl.w_ref) ** 2) / np.sum(wt * wl.w_ref ** 2)))
    eoc = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    print("flux errors", errs, "observed orders", eoc)
    assert errs[0] < 0.1
    assert np.all(eoc > 1.0), (errs, eoc)


def test_toeplitz_mode_equals_packed():
    """Uniform steps: the oracle's block-Toeplitz blocks (d, 0) reproduce the
    packed lower block triangle, and its Toeplitz product and forward
    substitution equal the packed ones (the reference solutions of larger
    meshes are computed this way)."""
    from oracle.oracle import toeplitz_apply, toeplitz_forward_solve, block_forward_solve
    wl = W.make("custom", n_side=2, n_t=5, n_omega=2, alpha=0.8)
    o = Oracle.from_workload(wl)
    V = o.packed("V")
    T = o.toeplitz_blocks("V")
    for k in range(o.nt):
        for m in range(k + 1):
            B_ = V[packed_index(k, m)]
            assert np.abs(B_ - T[k - m]).max() <= 1e-14 * np.abs(B_).max()
    x = np.random.default_rng(1).standard_normal(o.n)
    np.testing.assert_allclose(toeplitz_apply(T, x, o.nt, o.ng), packed_apply(V, x, o.nt, o.ng), rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(toeplitz_forward_solve(T, x, o.nt, o.ng), block_forward_solve(V, x, o.nt, o.ng),
                               rtol=1e-11)
