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

    # ---------------------------------------------------------------- calls
    def assemble(self, mask):
        self._check(self.lib.stbem_assemble(self._h, int(mask), self._stream()), "stbem_assemble")

    def release(self, mask):
        torch.cuda.current_stream().synchronize()
        self._check(self.lib.stbem_release(self._h, int(mask)), "stbem_release")

    def matrix(self, op):
        """The operator's storage as a float64 tensor (packed blocks or dense M0)."""
        p, nb = ctypes.c_void_p(), ctypes.c_size_t()
        self._check(self.lib.stbem_matrix(self._h, int(op), ctypes.byref(p), ctypes.byref(nb)), "stbem_matrix")
        t = self._tensors[p.value]
        return t[: nb.value].view(torch.float64)

    def packed(self, op):
        """Stored blocks of a causal operator: [k(k+1)/2 + m] packed, or [k - m] in block-Toeplitz mode."""
        nb = self.nt if self.toeplitz else self.nt * (self.nt + 1) // 2
        return self.matrix(op).view(nb, self.ng, self.ng)

    def set_toeplitz(self, on=True):
        """Block-Toeplitz storage (uniform time steps only); frees the assembled causal operators."""
        self._check(self.lib.stbem_set_toeplitz(self._h, 1 if on else 0), "stbem_set_toeplitz")
        self.toeplitz = bool(on)

    def apply(self, op, x, trans=False, out=None):
        x = self.vec(x)
        rows = self.n if (op not in (L.M0, L.DM0) or trans) else self.n
        if op in (L.M0, L.DM0) and trans:
            rows = self.nv
        y = out if out is not None else self.vec(n=rows)
        self._check(self.lib.stbem_apply(self._h, int(op), int(bool(trans)), _ptr(x), _ptr(y), self._stream()), "stbem_apply")
        return y

    def mass(self, x, trans=False):
        x = self.vec(x)
        y = self.vec(n=self.n)
        self._check(self.lib.stbem_mass(self._h, int(bool(trans)), _ptr(x), _ptr(y), self._stream()), "stbem_mass")
        return y

    def precondition(self, r, trans=False):
        r = self.vec(r)
        z = self.vec(n=self.n)
        self._check(self.lib.stbem_precondition(self._h, int(bool(trans)), _ptr(r), _ptr(z), self._stream()), "stbem_precondition")
        return z

    def rhs(self, g, u0=None):
        g = self.vec(g)
        u0 = self.vec(u0) if u0 is not None else None
        f = self.vec(n=self.n)
        self._check(self.lib.stbem_rhs(self._h, _ptr(g), _ptr(u0), _ptr(f), self._stream()), "stbem_rhs")
        return f

    def prepare_ir(self):
        self._check(self.lib.stbem_prepare_ir(self._h, self._stream()), "stbem_prepare_ir")

    def solve(self, f, tol=1e-12, max_it=300, mode=L.FP64, trans=False, precondition=True,
              inner_tol=1e-5, max_outer=10, ir_tol=1e-12, out=None):
        f = self.vec(f)
        w = out if out is not None else self.vec(n=self.n)
        o = L.stbem_solve_opts(float(tol), int(max_it), int(mode), int(bool(trans)), int(bool(precondition)),
                               float(inner_tol), int(max_outer), float(ir_tol))
        info = L.stbem_solve_info()
        rc = self._check(self.lib.stbem_solve(self._h, _ptr(f), _ptr(w), ctypes.byref(o), ctypes.byref(info),
                                              self._stream()), "stbem_solve")
        return w, SolveInfo(info.iters, info.outer, info.relres, info.true_relres, rc)

    def grad_alpha(self, lam, w, g, u0=None):
        out = self.vec(n=1)
        self._check(self.lib.stbem_grad_alpha(self._h, _ptr(self.vec(lam)), _ptr(w), _ptr(g),
                                              _ptr(self.vec(u0)) if u0 is not None else None, _ptr(out),
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
        """{kernel name: (launches, event ms, work units)} recorded since timing was switched on."""
        cap = 64
        buf = (L.stbem_kernel_time * cap)()
        n = self.lib.stbem_kernel_times(self._h, buf, cap)
        self._check(min(n, 0), "stbem_kernel_times")
        return {buf[e].name.decode(): (buf[e].launches, buf[e].ms, buf[e].units) for e in range(min(n, cap))}

    def entries(self, op, idx):
        idx = torch.as_tensor(np.asarray(idx, dtype=np.int32).reshape(-1, 4), device=self.device).contiguous()
        out = self.vec(n=idx.shape[0])
        self._check(self.lib.stbem_entries(self._h, int(op), idx.shape[0], _ptr(idx), _ptr(out), self._stream()),
                    "stbem_entries")
        return out
