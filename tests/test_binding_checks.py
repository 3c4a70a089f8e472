"""Argument checks of the Python binding and the C ABI that run without a
GPU: vectors of the wrong length and entry indices outside the matrix are
refused before any device call; entry points given no context return
STBEM_EINVAL."""
import os

import numpy as np
import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1811_05224_amd", "libstbem.so")


def test_entry_indices_checked():
    from paper_1811_05224_amd.api import check_entry_indices
    ok = check_entry_indices([[2, 1, 0, 7], [0, 0, 3, 3]], nt=3, ng=8)
    assert ok.dtype == np.int32 and ok.shape == (2, 4)
    for bad in ([[3, 0, 0, 0]], [[0, -1, 0, 0]], [[0, 0, 8, 0]], [[0, 0, 0, -1]], [1, 2, 3]):
        with pytest.raises(ValueError):
            check_entry_indices(bad, nt=3, ng=8)


def _stub(n=12, nv=5):
    """A Context shell with sizes and a CPU device, to exercise the checks."""
    from paper_1811_05224_amd.api import Context
    c = object.__new__(Context)
    c.n, c.nv, c.device = n, nv, torch.device("cpu")
    return c


def test_vector_lengths_checked():
    c = _stub()
    assert c._in(np.zeros(12), 12, "x").dtype == torch.float64
    with pytest.raises(ValueError):
        c._in(np.zeros(11), 12, "x")
    with pytest.raises(ValueError):
        c._out(torch.zeros(12, dtype=torch.float32), 12, "out")
    with pytest.raises(ValueError):
        c._out(torch.zeros(13, dtype=torch.float64), 12, "out")
    with pytest.raises(ValueError):
        c._out(torch.zeros(24, dtype=torch.float64)[::2], 12, "out")
    assert c._out(None, 5, "out").numel() == 5


@pytest.mark.skipif(not os.path.exists(LIB), reason="libstbem.so not built")
def test_null_context_rejected_by_new_entry_points():
    import ctypes
    from paper_1811_05224_amd import _lib as L
    lib = L.load()
    assert lib.stbem_assemble(None, L.V, L.FP64, None) == -1
    assert lib.stbem_rhs_adjoint(None, None, None, None) == -1
    hi, lo, nb = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_size_t()
    assert lib.stbem_matrix_f32(None, L.V, ctypes.byref(hi), ctypes.byref(lo), ctypes.byref(nb)) == -1
    assert lib.stbem_precondition(None, 0, None, None, None) == -1
