"""Python driver of the CPU oracle (arXiv:1811.05224, space-time BEM, 2D heat).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product path.

The entries come from ``liboracle.so`` (long-double C, adaptive quadrature,
built from ``stbem_oracle.c``).  This module assembles them into the packed
block-lower-triangular layout, builds the sparse/diagonal mass matrices, the
right-hand side of eq.(4) and solves the system two independent ways:
block forward substitution in time (Cholesky of the SPD diagonal blocks) and
left-preconditioned GMRES with C_V^{-1} = M~^{-1} D_h M~^{-1} (Thm 1, with the
lumped mass of Sec. 4).  Everything here is plain numpy float64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "stbem_oracle.c")

OP_V, OP_K, OP_D, OP_M0, OP_DV, OP_DK, OP_DM0 = range(7)
_OPNAME = {"V": OP_V, "K": OP_K, "D": OP_D, "dV": OP_DV, "dK": OP_DK}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no GPU toolchain involved)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
               "-Wno-unused-function", "-Wno-misleading-indentation",
               _SRC, "-o", _LIB_PATH + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.or_create.restype = ctypes.c_void_p
        L.or_create.argtypes = [ctypes.c_double, ctypes.c_int, dp, ctypes.c_int, dp,
                                ctypes.c_int, dp, ctypes.c_int, ip]
        L.or_destroy.argtypes = [ctypes.c_void_p]
        L.or_entries.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_long, ip, dp, ctypes.c_int]
        L.or_m0_rows.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_long, ip, dp, ctypes.c_int]
        L.or_potential.argtypes = [ctypes.c_void_p, ctypes.c_long, dp, dp, dp, dp, dp, ctypes.c_int]
        L.or_e1.restype = ctypes.c_double
        L.or_e1.argtypes = [ctypes.c_double]
        L.or_e1l.restype = ctypes.c_longdouble
        L.or_e1l.argtypes = [ctypes.c_longdouble]
        L.or_time_integral.restype = ctypes.c_double
        L.or_time_integral.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int]
        L.or_m0_time.restype = ctypes.c_double
        L.or_m0_time.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_int]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def e1(z: float) -> float:
    return lib().or_e1(float(z))


def nthreads_default() -> int:
    return int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1))


class Oracle:
    """Oracle for one problem (mesh, times, alpha)."""

    def __init__(self, alpha, t_nodes, bnd_xy, vtx_xy=None, tri=None, nthreads=None):
        self.alpha = float(alpha)
        self.t = np.ascontiguousarray(t_nodes, dtype=np.float64)
        self.bnd = np.ascontiguousarray(bnd_xy, dtype=np.float64)
        self.vtx = np.ascontiguousarray(np.zeros((0, 2)) if vtx_xy is None else vtx_xy, dtype=np.float64)
        self.tri = np.ascontiguousarray(np.zeros((0, 3)) if tri is None else tri, dtype=np.int32)
        self.ng = self.bnd.shape[0]
        self.nt = self.t.shape[0] - 1
        self.nv = self.vtx.shape[0]
        self.n = self.ng * self.nt
        self.nthreads = nthreads or nthreads_default()
        self._h = lib().or_create(self.alpha, self.nt, _dp(self.t), self.ng, _dp(self.bnd),
                                  self.nv, _dp(self.vtx), self.tri.shape[0], _ip(self.tri))
        if not self._h:
            raise ValueError("oracle rejected the problem")
        d = np.roll(self.bnd, -1, axis=0) - self.bnd
        self.L = np.hypot(d[:, 0], d[:, 1])
        self.h = np.diff(self.t)

    @classmethod
    def from_workload(cls, wl, **kw):
        return cls(wl.alpha, wl.t_nodes, wl.bnd_xy, wl.vtx_xy, wl.tri, **kw)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().or_destroy(h)
            self._h = None

    # ------------------------------------------------------------ entries
    def entries(self, op: str, idx) -> np.ndarray:
        """Entries A[(k,i),(m,j)] for quadruples (k, m, i, j)."""
        idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int32).reshape(-1, 4))
        out = np.empty(idx.shape[0], dtype=np.float64)
        rc = lib().or_entries(self._h, _OPNAME[op], idx.shape[0], _ip(idx), _dp(out), self.nthreads)
        if rc:
            raise ValueError(f"or_entries failed ({rc})")
        return out

    def block(self, op: str, k: int, m: int) -> np.ndarray:
        ng = self.ng
        ii, jj = np.meshgrid(np.arange(ng), np.arange(ng), indexing="ij")
        idx = np.stack([np.full(ng * ng, k), np.full(ng * ng, m), ii.ravel(), jj.ravel()], axis=1)
        return self.entries(op, idx).reshape(ng, ng)

    def packed(self, op: str) -> np.ndarray:
        """Lower block triangle, block (k,m) (k >= m) at index k(k+1)/2 + m."""
        ng, nt = self.ng, self.nt
        ks, ms = np.tril_indices(nt)
        nb = ks.shape[0]
        ii, jj = np.meshgrid(np.arange(ng), np.arange(ng), indexing="ij")
        idx = np.empty((nb, ng * ng, 4), dtype=np.int32)
        idx[:, :, 0] = ks[:, None]
        idx[:, :, 1] = ms[:, None]
        idx[:, :, 2] = ii.ravel()[None, :]
        idx[:, :, 3] = jj.ravel()[None, :]
        # np.tril_indices orders (k, m) row by row: index = k(k+1)/2 + m
        return self.entries(op, idx.reshape(-1, 4)).reshape(nb, ng, ng)

    def toeplitz_blocks(self, op: str) -> np.ndarray:
        """Uniform time steps only: block (k, m) of a causal operator depends
        on k - m alone (the kernel is a function of t - tau), so the blocks
        (d, 0), d = 0..nt-1, determine the whole matrix."""
        h = np.diff(self.t)
        if np.abs(h - h[0]).max() > 1e-12 * h[0]:
            raise ValueError("Toeplitz blocks need uniform time steps")
        ng, nt = self.ng, self.nt
        ii, jj = np.meshgrid(np.arange(ng), np.arange(ng), indexing="ij")
        idx = np.empty((nt, ng * ng, 4), dtype=np.int32)
        idx[:, :, 0] = np.arange(nt)[:, None]
        idx[:, :, 1] = 0
        idx[:, :, 2] = ii.ravel()[None, :]
        idx[:, :, 3] = jj.ravel()[None, :]
        return self.entries(op, idx.reshape(-1, 4)).reshape(nt, ng, ng)

    def m0_rows(self, rows, deriv: bool = False) -> np.ndarray:
        rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int32).reshape(-1, 2))
        out = np.empty((rows.shape[0], self.nv), dtype=np.float64)
        rc = lib().or_m0_rows(self._h, int(bool(deriv)), rows.shape[0], _ip(rows), _dp(out), self.nthreads)
        if rc:
            raise ValueError(f"or_m0_rows failed ({rc})")
        return out

    def potential(self, pts, w, g, u0=None) -> np.ndarray:
        """The three potentials of the representation formula (Sec. 1, eq. (2))
        at points (x, y, t), t > 0: columns M~0 u0, V~ w, W g (u = c0 + c1 - c2)."""
        pts = np.ascontiguousarray(np.asarray(pts, dtype=np.float64).reshape(-1, 3))
        w = np.ascontiguousarray(w, dtype=np.float64); g = np.ascontiguousarray(g, dtype=np.float64)
        u0a = np.ascontiguousarray(u0, dtype=np.float64) if u0 is not None else None
        u0p = _dp(u0a) if u0a is not None else None
        out = np.empty((pts.shape[0], 3), dtype=np.float64)
        rc = lib().or_potential(self._h, pts.shape[0], _dp(pts), _dp(w), _dp(g), u0p, _dp(out), self.nthreads)
        if rc:
            raise ValueError(f"or_potential failed ({rc})")
        return out

    def m0(self, deriv: bool = False) -> np.ndarray:
        kk, ii = np.meshgrid(np.arange(self.nt), np.arange(self.ng), indexing="ij")
        return self.m0_rows(np.stack([kk.ravel(), ii.ravel()], axis=1), deriv)

    def time_integral(self, which: str, r: float, k: int, m: int) -> float:
        w = {"V": 0, "K": 1, "D": 2, "dV": 3, "E1": 4}[which]
        return lib().or_time_integral(self._h, w, float(r), int(k), int(m))

    def m0_time(self, r: float, k: int, deriv: bool = False) -> float:
        return lib().or_m0_time(self._h, float(r), int(k), int(bool(deriv)))

    # ------------------------------------------------------------ algebra
    def dense(self, packed: np.ndarray) -> np.ndarray:
        return packed_to_dense(packed, self.nt, self.ng)

    def mass_apply(self, g: np.ndarray) -> np.ndarray:
        """M_h g: <phi^{10}_{(m,n)}, phi^0_{(k,i)}> = delta_km h_k L_i / 2 for n in {i, i+1}."""
        G = g.reshape(self.nt, self.ng)
        out = 0.5 * self.h[:, None] * self.L[None, :] * (G + np.roll(G, -1, axis=1))
        return out.reshape(-1)

    def mass_matrix(self) -> np.ndarray:
        n = self.n
        M = np.zeros((n, n))
        for k in range(self.nt):
            for i in range(self.ng):
                r = k * self.ng + i
                c = 0.5 * self.h[k] * self.L[i]
                M[r, k * self.ng + i] += c
                M[r, k * self.ng + (i + 1) % self.ng] += c
        return M

    def lumped_dual_mass(self) -> np.ndarray:
        """Row sums of <phi^0_{(m,i)}, psi_{(m,i')}>: h_m (L_{i-1} + 2 L_i + L_{i+1}) / 4."""
        Lm, Lp = np.roll(self.L, 1), np.roll(self.L, -1)
        return (self.h[:, None] * ((Lm + 2 * self.L + Lp) / 4)[None, :]).reshape(-1)

    def rhs(self, K_packed, M0, g, u0) -> np.ndarray:
        """Right-hand side of eq.(4): (1/2 M_h + K_h) g - M_h^0 u0."""
        return 0.5 * self.mass_apply(g) + packed_apply(K_packed, g, self.nt, self.ng) - M0 @ u0

    def solve_direct(self, V_packed, f) -> np.ndarray:
        return block_forward_solve(V_packed, f, self.nt, self.ng)

    def solve_gmres(self, V_packed, D_packed, f, tol=1e-12, maxit=500, precondition=True):
        nt, ng = self.nt, self.ng
        mt = self.lumped_dual_mass()
        A = lambda x: packed_apply(V_packed, x, nt, ng)
        if precondition:
            P = lambda r: packed_apply(D_packed, r / mt, nt, ng) / mt
        else:
            P = lambda r: r
        return gmres_left(A, P, f, tol=tol, maxit=maxit)


# ---------------------------------------------------------------- helpers
def packed_index(k, m):
    return k * (k + 1) // 2 + m


def packed_to_dense(P, nt, ng):
    A = np.zeros((nt * ng, nt * ng))
    for k in range(nt):
        for m in range(k + 1):
            A[k * ng:(k + 1) * ng, m * ng:(m + 1) * ng] = P[packed_index(k, m)]
    return A


def packed_apply(P, x, nt, ng, trans=False):
    X = x.reshape(nt, ng)
    Y = np.zeros((nt, ng))
    for k in range(nt):
        for m in range(k + 1):
            B = P[packed_index(k, m)]
            if trans:
                Y[m] += B.T @ X[k]
            else:
                Y[k] += B @ X[m]
    return Y.reshape(-1)


def toeplitz_apply(T, x, nt, ng, trans=False):
    """y = A x (or A^T x) for a causal block-Toeplitz A with blocks
    T[d] = A_(k, k-d)."""
    X = x.reshape(nt, ng)
    Y = np.zeros((nt, ng))
    for k in range(nt):
        for m in range(k + 1):
            if trans:
                Y[m] += T[k - m].T @ X[k]
            else:
                Y[k] += T[k - m] @ X[m]
    return Y.reshape(-1)


def toeplitz_forward_solve(T, f, nt, ng):
    """Block forward substitution for a causal block-Toeplitz A:
    T[0] w_k = f_k - sum_{m<k} T[k-m] w_m (T[0] symmetric positive definite)."""
    import scipy.linalg as sla
    F = f.reshape(nt, ng)
    W = np.zeros((nt, ng))
    c = sla.cho_factor(0.5 * (T[0] + T[0].T))
    for k in range(nt):
        rhs = F[k].copy()
        for m in range(k):
            rhs -= T[k - m] @ W[m]
        W[k] = sla.cho_solve(c, rhs)
    return W.reshape(-1)


def block_forward_solve(P, f, nt, ng, trans=False):
    """Solve A w = f (or A^T w = f) with A block lower triangular.

    The diagonal blocks are symmetric positive definite (Galerkin matrices of
    a single-layer/hypersingular kernel over the same time element), so each
    step uses a Cholesky factorisation."""
    import scipy.linalg as sla
    F = f.reshape(nt, ng).copy()
    W = np.zeros((nt, ng))
    order = range(nt) if not trans else range(nt - 1, -1, -1)
    for k in order:
        rhs = F[k].copy()
        if not trans:
            for m in range(k):
                rhs -= P[packed_index(k, m)] @ W[m]
        else:
            for j in range(k + 1, nt):
                rhs -= P[packed_index(j, k)].T @ W[j]
        Dk = P[packed_index(k, k)]
        c = sla.cho_factor(0.5 * (Dk + Dk.T))
        W[k] = sla.cho_solve(c, rhs)
    return W.reshape(-1)


def gmres_left(A, P, f, tol=1e-12, maxit=500):
    """Left-preconditioned GMRES, x0 = 0, no restart, modified Gram-Schmidt
    with one re-orthogonalisation, Givens rotations.  Stops when
    ||P(f - A x)|| <= tol ||P f||.  Returns (x, iterations, history)."""
    r0 = P(f)
    beta = np.linalg.norm(r0)
    n = f.shape[0]
    if beta == 0:
        return np.zeros(n), 0, [0.0]
    Q = np.zeros((maxit + 1, n))
    H = np.zeros((maxit + 1, maxit))
    cs, sn = np.zeros(maxit), np.zeros(maxit)
    gvec = np.zeros(maxit + 1)
    gvec[0] = beta
    Q[0] = r0 / beta
    hist = [1.0]
    j = 0
    for j in range(maxit):
        v = P(A(Q[j]))
        for _ in range(2):
            for i in range(j + 1):
                hij = Q[i] @ v
                H[i, j] += hij
                v -= hij * Q[i]
        H[j + 1, j] = np.linalg.norm(v)
        if H[j + 1, j] > 0:
            Q[j + 1] = v / H[j + 1, j]
        for i in range(j):
            a, b = H[i, j], H[i + 1, j]
            H[i, j] = cs[i] * a + sn[i] * b
            H[i + 1, j] = -sn[i] * a + cs[i] * b
        a, b = H[j, j], H[j + 1, j]
        rr = np.hypot(a, b)
        cs[j], sn[j] = a / rr, b / rr
        H[j, j] = rr
        H[j + 1, j] = 0.0
        gvec[j + 1] = -sn[j] * gvec[j]
        gvec[j] = cs[j] * gvec[j]
        hist.append(abs(gvec[j + 1]) / beta)
        if abs(gvec[j + 1]) <= tol * beta:
            j += 1
            break
    else:
        j = maxit
    y = np.linalg.solve(np.triu(H[:j, :j]), gvec[:j])
    x = Q[:j].T @ y
    return x, j, hist
