"""ctypes declarations of the C ABI in include/stbem.h (names unchanged)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstbem.so")

V, K, D, M0, DV, DK, DM0 = 1, 2, 4, 8, 16, 32, 64
FP64, FP32_IR = 0, 1
WARN_NOT_CONVERGED, WARN_IR_STAGNATION = 1, 2
ERRORS = {-1: "EINVAL", -2: "EMESH", -3: "EALPHA", -4: "ETIME", -5: "ENOMEM", -6: "ENOTASSEMBLED", -7: "EHIP"}


class stbem_problem(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("n_t", ctypes.c_int), ("t_nodes", ctypes.POINTER(ctypes.c_double)),
                ("n_bnd", ctypes.c_int), ("bnd_xy", ctypes.POINTER(ctypes.c_double)),
                ("n_vtx", ctypes.c_int), ("vtx_xy", ctypes.POINTER(ctypes.c_double)),
                ("n_tri", ctypes.c_int), ("tri", ctypes.POINTER(ctypes.c_int))]


class stbem_solve_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_it", ctypes.c_int), ("mode", ctypes.c_int), ("trans", ctypes.c_int),
                ("precondition", ctypes.c_int), ("inner_tol", ctypes.c_double), ("max_outer", ctypes.c_int),
                ("ir_tol", ctypes.c_double)]


class stbem_kernel_time(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_longlong), ("ms", ctypes.c_double),
                ("units", ctypes.c_double), ("flops", ctypes.c_double)]


class stbem_solve_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer", ctypes.c_int), ("relres", ctypes.c_double),
                ("true_relres", ctypes.c_double)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_lib = None


def load():
    """Load libstbem.so; raises if it is missing (there is no other path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1811_05224_amd/build.py "
                           "(hipcc, gfx950); there is no fallback implementation")
    L = ctypes.CDLL(LIB_PATH)
    vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
    sig = {
        "stbem_create": (ctypes.c_int, [ctypes.POINTER(stbem_problem), ctypes.POINTER(vp)]),
        "stbem_destroy": (ctypes.c_int, [vp]),
        "stbem_last_error": (ctypes.c_char_p, [vp]),
        "stbem_set_allocator": (ctypes.c_int, [vp, ALLOC_FN, FREE_FN, vp]),
        "stbem_sizes": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_longlong), ip, ip, ip, ctypes.POINTER(ctypes.c_longlong)]),
        "stbem_assemble": (ctypes.c_int, [vp, ctypes.c_uint, ctypes.c_int, vp]),
        "stbem_release": (ctypes.c_int, [vp, ctypes.c_uint]),
        "stbem_matrix": (ctypes.c_int, [vp, ctypes.c_uint, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_size_t)]),
        "stbem_matrix_f32": (ctypes.c_int, [vp, ctypes.c_uint, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_size_t)]),
        "stbem_apply": (ctypes.c_int, [vp, ctypes.c_uint, ctypes.c_int, vp, vp, vp]),
        "stbem_apply_noalloc": (ctypes.c_int, [vp, ctypes.c_uint, ctypes.c_int, vp, vp, vp]),
        "stbem_mass": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, vp]),
        "stbem_precondition": (ctypes.c_int, [vp, ctypes.c_int, vp, vp, vp]),
        "stbem_rhs": (ctypes.c_int, [vp, vp, vp, vp, vp]),
        "stbem_rhs_adjoint": (ctypes.c_int, [vp, vp, vp, vp]),
        "stbem_prepare_ir": (ctypes.c_int, [vp, vp]),
        "stbem_solve": (ctypes.c_int, [vp, vp, vp, ctypes.POINTER(stbem_solve_opts), ctypes.POINTER(stbem_solve_info), vp]),
        "stbem_grad_alpha": (ctypes.c_int, [vp, vp, vp, vp, vp, vp, vp]),
        "stbem_entries": (ctypes.c_int, [vp, ctypes.c_uint, ctypes.c_longlong, vp, vp, vp]),
        "stbem_set_timing": (ctypes.c_int, [vp, ctypes.c_int]),
        "stbem_set_toeplitz": (ctypes.c_int, [vp, ctypes.c_int]),
        "stbem_potential": (ctypes.c_int, [vp, ctypes.c_longlong, vp, vp, vp, vp, vp, vp]),
        "stbem_kernel_times": (ctypes.c_int, [vp, ctypes.POINTER(stbem_kernel_time), ctypes.c_int]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype, f.argtypes = res, args
    _lib = L
    return L


EXPORTED = ["stbem_create", "stbem_destroy", "stbem_last_error", "stbem_set_allocator", "stbem_sizes",
            "stbem_assemble", "stbem_release", "stbem_matrix", "stbem_matrix_f32", "stbem_apply", "stbem_apply_noalloc", "stbem_mass",
            "stbem_precondition", "stbem_rhs", "stbem_rhs_adjoint",
            "stbem_prepare_ir", "stbem_solve", "stbem_grad_alpha", "stbem_entries", "stbem_set_timing",
            "stbem_kernel_times", "stbem_set_toeplitz", "stbem_potential"]
