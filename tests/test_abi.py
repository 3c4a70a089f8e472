"""C ABI: the shared library loads without a GPU and exports every function
that include/stbem.h declares; the Python layer has no CPU fallback."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stbem.h")
LIB = os.path.join(ROOT, "paper_1811_05224_amd", "libstbem.so")


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(stbem_\w+)\s*\(", src, re.M)))


def test_header_declares_the_entry_points():
    names = declared()
    for n in ("stbem_create", "stbem_destroy", "stbem_assemble", "stbem_apply", "stbem_precondition",
              "stbem_rhs", "stbem_solve", "stbem_grad_alpha", "stbem_last_error"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libstbem.so not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared():
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (stbem_\w+)", out))
    assert set(declared()) <= exported
    from paper_1811_05224_amd import _lib
    assert set(_lib.EXPORTED) == set(declared())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libstbem.so not built")
def test_invalid_problems_rejected_on_the_host():
    """stbem_create validates before touching the device: these calls return
    the documented error codes without a GPU."""
    from paper_1811_05224_amd import _lib as L
    import numpy as np
    lib = L.load()

    def create(alpha=1.0, t=(0.0, 0.5, 1.0), bnd=((0, 0), (1, 0), (1, 1), (0, 1))):
        t = np.ascontiguousarray(t, dtype=np.float64)
        b = np.ascontiguousarray(bnd, dtype=np.float64)
        dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        p = L.stbem_problem(alpha, t.shape[0] - 1, dp(t), b.shape[0], dp(b), 0, None, 0, None)
        h = ctypes.c_void_p()
        return lib.stbem_create(ctypes.byref(p), ctypes.byref(h))

    assert create(alpha=0.0) == -3
    assert create(alpha=float("nan")) == -3
    assert create(t=(0.0, 0.5, 0.5)) == -4
    assert create(t=(0.1, 0.5)) == -4
    assert create(bnd=((0, 0), (0, 1), (1, 1), (1, 0))) == -2      # clockwise
    assert create(bnd=((0, 0), (1, 0))) == -2
    assert create(bnd=((0, 0), (1, 0), (1, 0), (0, 1))) == -2       # zero-length segment
    assert lib.stbem_create(None, None) == -1
    assert lib.stbem_destroy(None) == 0


def test_no_cpu_fallback_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    import paper_1811_05224_amd as P
    import workloads as W
    with pytest.raises(P.StbemError):
        P.Context.from_workload(W.make("custom"))


@pytest.mark.skipif(not os.path.exists(LIB), reason="libstbem.so not built")
def test_null_context_rejected():
    """Entry points given no context return STBEM_EINVAL without touching a device."""
    from paper_1811_05224_amd import _lib as L
    lib = L.load()
    assert lib.stbem_set_timing(None, 1) == -1
    assert lib.stbem_kernel_times(None, None, 0) == -1
    assert lib.stbem_destroy(None) == 0


def test_bench_refuses_several_gpus():
    """The benchmark runs on one GPU; asked for more it stops with a message
    (before touching any device)."""
    import subprocess, sys, os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0 and "one GPU only" in r.stderr and r.stdout == ""
