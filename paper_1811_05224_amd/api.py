"""Context object over the C ABI (argument marshalling only)."""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np
import torch

from . import _lib as L


class StbemError(RuntimeError):
    pass


@dataclasses.dataclass
class SolveInfo:
    iters: int
    outer: int
    relres: float
    true_relres: float
    status: int


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def check_entry_indices(idx, nt, ng):
    """Entry quadruples (k, m, i, j) as an (n, 4) int32 array, all inside the
    matrix (0 <= k, m < nt, 0 <= i, j < ng); raises ValueError otherwise."""
    a = np.asarray(idx)
    if a.size % 4:
        raise ValueError("entry indices come in quadruples (k, m, i, j)")
    a = a.reshape(-1, 4)
    if a.size and (a.min() < 0 or a[:, :2].max() >= nt or a[:, 2:].max() >= ng):
        raise ValueError(f"entry index outside the matrix (n_t = {nt}, n_bnd = {ng})")
    return np.ascontiguousarray(a, dtype=np.int32)


class Context:
    """One problem (Gamma_h polygon, time grid, alpha, Omega_h) on one GPU.

    Matrices live in torch tensors allocated through the library's allocator
    callback; vectors are float64 torch tensors on the same device."""

    def __init__(self, alpha, t_nodes, bnd_xy, vtx_xy=None, tri=None, device="cuda:0"):
        if not torch.cuda.is_available():
            raise StbemError("no HIP device: this library runs only on the GPU")
        self.lib = L.load()
        self.alpha_value = float(alpha)
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        t = np.ascontiguousarray(t_nodes, dtype=np.float64)
        b = np.ascontiguousarray(bnd_xy, dtype=np.float64).reshape(-1, 2)
        v = np.ascontiguousarray(np.zeros((0, 2)) if vtx_xy is None else vtx_xy, dtype=np.float64).reshape(-1, 2)
        tr = np.ascontiguousarray(np.zeros((0, 3)) if tri is None else tri, dtype=np.int32).reshape(-1, 3)
        self._keep = (t, b, v, tr)
        prob = L.stbem_problem(float(alpha), t.shape[0] - 1, _dp(t), b.shape[0], _dp(b), v.shape[0], _dp(v),
                               tr.shape[0], tr.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
        h = ctypes.c_void_p()
        rc = self.lib.stbem_create(ctypes.byref(prob), ctypes.byref(h))
        if rc:
            raise StbemError(f"stbem_create failed: {L.ERRORS.get(rc, rc)}")
        self._h = h
        self._tensors = {}
        self._alloc_cb = L.ALLOC_FN(self._alloc)
        self._free_cb = L.FREE_FN(self._free)
        self._check(self.lib.stbem_set_allocator(h, self._alloc_cb, self._free_cb, None), "stbem_set_allocator")
        n, ng, nt, nv, packed = ctypes.c_longlong(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_longlong()
        self.lib.stbem_sizes(h, ctypes.byref(n), ctypes.byref(ng), ctypes.byref(nt), ctypes.byref(nv), ctypes.byref(packed))
        self.n, self.ng, self.nt, self.nv, self.packed_entries = n.value, ng.value, nt.value, nv.value, packed.value
        self.toeplitz = False

    @classmethod
    def from_workload(cls, wl, **kw):
        return cls(wl.alpha, wl.t_nodes, wl.bnd_xy, wl.vtx_xy, wl.tri, **kw)

    # allocator callbacks: torch owns the matrix memory
    def _alloc(self, nbytes, user):
        try:
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        except RuntimeError:
            return None
        self._tensors[t.data_ptr()] = t
        return t.data_ptr()

    def _free(self, ptr, user):
        self._tensors.pop(ptr, None)

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self.lib.stbem_destroy(h)
            self._h = None
        self._tensors = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc < 0:
            msg = self.lib.stbem_last_error(self._h).decode() if getattr(self, "_h", None) else ""
            raise StbemError(f"{what} failed: {L.ERRORS.get(rc, rc)} {msg}")
        return rc

    @staticmethod
    def _stream():
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def vec(self, x=None, n=None):
        if x is None:
            return torch.zeros(n if n is not None else self.n, dtype=torch.float64, device=self.device)
        return torch.as_tensor(x, dtype=torch.float64, device=self.device).contiguous()

    def _in(self, x, n, name):
        """x as a contiguous float64 tensor on the context's device with n entries."""
        t = self.vec(x)
        if t.numel() != n:
            raise ValueError(f"{name} needs {n} entries, got {t.numel()}")
        return t

    def _out(self, out, n, name):
        if out is None:
            return self.vec(n=n)
        if (out.dtype != torch.float64 or out.device != self.device or not out.is_contiguous()
                or out.numel() != n):
            raise ValueError(f"{name}: a contiguous float64 tensor of {n} entries on {self.device} is needed")
        return out

    # ---------------------------------------------------------------- calls
    def assemble(self, mask, precision=L.FP64):
        """Assemble the operators in mask; precision FP32_IR (V, D only) keeps
        V_h as an FP32 hi + lo pair and D_h as FP32 instead of FP64."""
        self._check(self.lib.stbem_assemble(self._h, int(mask), int(precision), self._stream()), "stbem_assemble")

    def release(self, mask):
        torch.cuda.current_stream().synchronize()
        self._check(self.lib.stbem_release(self._h, int(mask)), "stbem_release")

    def matrix(self, op):
        """The operator's FP64 storage as a float64 tensor (packed blocks or dense M0)."""
        p, nb = ctypes.c_void_p(), ctypes.c_size_t()
        self._check(self.lib.stbem_matrix(self._h, int(op), ctypes.byref(p), ctypes.byref(nb)), "stbem_matrix")
        t = self._tensors[p.value]
        return t[: nb.value].view(torch.float64)

    def _nblocks(self):
        return self.nt if self.toeplitz else self.nt * (self.nt + 1) // 2

    def packed(self, op):
        """Stored blocks of a causal operator: [k(k+1)/2 + m] packed, or [k - m] in block-Toeplitz mode."""
        return self.matrix(op).view(self._nblocks(), self.ng, self.ng)

    def packed_f32(self, op):
        """FP32 storage of V_h (hi, lo) or D_h (hi, None) as [block, ng, ng] float32 tensors."""
        hi, lo, nb = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_size_t()
        self._check(self.lib.stbem_matrix_f32(self._h, int(op), ctypes.byref(hi), ctypes.byref(lo), ctypes.byref(nb)),
                    "stbem_matrix_f32")
        shape = (self._nblocks(), self.ng, self.ng)
        view = lambda p: self._tensors[p][: nb.value].view(torch.float32).view(shape)
        return view(hi.value), (view(lo.value) if lo.value else None)

    def set_toeplitz(self, on=True):
        """Block-Toeplitz storage (uniform time steps only); frees the assembled causal operators."""
        self._check(self.lib.stbem_set_toeplitz(self._h, 1 if on else 0), "stbem_set_toeplitz")
        self.toeplitz = bool(on)

    def apply(self, op, x, trans=False, out=None):
        dense = op in (L.M0, L.DM0)
        nin = self.nv if (dense and not trans) else self.n
        nout = self.nv if (dense and trans) else self.n
        x = self._in(x, nin, "x")
        y = self._out(out, nout, "out")
        self._check(self.lib.stbem_apply(self._h, int(op), int(bool(trans)), _ptr(x), _ptr(y), self._stream()), "stbem_apply")
        return y

    def mass(self, x, trans=False):
        x = self._in(x, self.n, "x")
        y = self.vec(n=self.n)
        self._check(self.lib.stbem_mass(self._h, int(bool(trans)), _ptr(x), _ptr(y), self._stream()), "stbem_mass")
        return y

    def precondition(self, r, trans=False):
        r = self._in(r, self.n, "r")
        z = self.vec(n=self.n)
        self._check(self.lib.stbem_precondition(self._h, int(bool(trans)), _ptr(r), _ptr(z), self._stream()), "stbem_precondition")
        return z

    def rhs(self, g, u0=None):
        g = self._in(g, self.n, "g")
        u0 = self._in(u0, self.nv, "u0") if u0 is not None else None
        f = self.vec(n=self.n)
        self._check(self.lib.stbem_rhs(self._h, _ptr(g), _ptr(u0), _ptr(f), self._stream()), "stbem_rhs")
        return f

    def rhs_adjoint(self, lam):
        """(1/2 M_h + K_h)^T lam: the gradient in g for an adjoint state lam."""
        lam = self._in(lam, self.n, "lam")
        out = self.vec(n=self.n)
        self._check(self.lib.stbem_rhs_adjoint(self._h, _ptr(lam), _ptr(out), self._stream()), "stbem_rhs_adjoint")
        return out

    def prepare_ir(self):
        self._check(self.lib.stbem_prepare_ir(self._h, self._stream()), "stbem_prepare_ir")

    def solve(self, f, tol=1e-12, max_it=300, mode=L.FP64, trans=False, precondition=True,
              inner_tol=1e-5, max_outer=10, ir_tol=1e-12, out=None):
        f = self._in(f, self.n, "f")
        w = self._out(out, self.n, "out")
        if w.data_ptr() == f.data_ptr():
            raise ValueError("out must not be the right-hand side")
        o = L.stbem_solve_opts(float(tol), int(max_it), int(mode), int(bool(trans)), int(bool(precondition)),
                               float(inner_tol), int(max_outer), float(ir_tol))
        info = L.stbem_solve_info()
        rc = self._check(self.lib.stbem_solve(self._h, _ptr(f), _ptr(w), ctypes.byref(o), ctypes.byref(info),
                                              self._stream()), "stbem_solve")
        return w, SolveInfo(info.iters, info.outer, info.relres, info.true_relres, rc)

    def grad_alpha(self, lam, w, g, u0=None):
        lam, w, g = self._in(lam, self.n, "lam"), self._in(w, self.n, "w"), self._in(g, self.n, "g")
        u0 = self._in(u0, self.nv, "u0") if u0 is not None else None
        out = self.vec(n=1)
        self._check(self.lib.stbem_grad_alpha(self._h, _ptr(lam), _ptr(w), _ptr(g), _ptr(u0), _ptr(out),
                                              self._stream()), "stbem_grad_alpha")
        return out

    def potential(self, pts, w, g, u0=None):
        """(M~0 u0, V~ w, W g) at points (x, y, t) of Q as an (n, 3) tensor; u = c0 + c1 - c2."""
        pts = torch.as_tensor(np.asarray(pts, dtype=np.float64).reshape(-1, 3), device=self.device).contiguous()
        out = self.vec(n=3 * pts.shape[0])
        w, g = self.vec(w), self.vec(g)
        u0t = self.vec(u0) if u0 is not None else None
        if w.numel() != self.n or g.numel() != self.n or (u0t is not None and u0t.numel() != self.nv):
            raise ValueError("w and g need N entries, u0 one per Omega vertex")
        self._check(self.lib.stbem_potential(self._h, pts.shape[0], _ptr(pts), _ptr(w), _ptr(g),
                                             _ptr(u0t) if u0t is not None else None, _ptr(out), self._stream()),
                    "stbem_potential")
        return out.view(-1, 3)

    def set_timing(self, on=True):
        self._check(self.lib.stbem_set_timing(self._h, 1 if on else 0), "stbem_set_timing")

    def kernel_times(self):
        """{kernel name: (launches, event ms, work units, algorithmic flops)} recorded since timing was switched on."""
        cap = 64
        buf = (L.stbem_kernel_time * cap)()
        n = self.lib.stbem_kernel_times(self._h, buf, cap)
        self._check(min(n, 0), "stbem_kernel_times")
        return {buf[e].name.decode(): (buf[e].launches, buf[e].ms, buf[e].units, buf[e].flops) for e in range(min(n, cap))}

    def entries(self, op, idx):
        idx = check_entry_indices(idx, self.nt, self.ng)
        idx = torch.as_tensor(idx, device=self.device).contiguous()
        out = self.vec(n=idx.shape[0])
        self._check(self.lib.stbem_entries(self._h, int(op), idx.shape[0], _ptr(idx), _ptr(out), self._stream()),
                    "stbem_entries")
        return out
