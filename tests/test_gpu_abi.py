"""C ABI behaviour on the GPU that the host alone cannot show: allocation
failure through the allocator callback, and index checks of sampled
entries."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def test_enomem_from_the_allocator_callback():
    """An allocator that returns NULL makes stbem_assemble fail with
    STBEM_ENOMEM and a message, in FP64 and in FP32 storage; nothing is
    assembled, and the context works again with a working allocator."""
    import paper_1811_05224_amd as P
    from paper_1811_05224_amd import _lib as L
    wl = W.make("custom", n_side=2, n_t=3, n_omega=2)
    c = P.Context.from_workload(wl)
    lib = c.lib
    null_alloc = L.ALLOC_FN(lambda nbytes, user: None)
    no_free = L.FREE_FN(lambda ptr, user: None)
    assert lib.stbem_set_allocator(c._h, null_alloc, no_free, None) == 0
    for mask, prec in ((L.V, L.FP64), (L.K | L.M0, L.FP64), (L.V | L.D, L.FP32_IR)):
        rc = lib.stbem_assemble(c._h, mask, prec, None)
        assert rc == -5, (mask, prec, rc)
        assert b"bytes" in lib.stbem_last_error(c._h)
    with pytest.raises(P.StbemError):
        c.matrix(L.V)
    assert lib.stbem_set_allocator(c._h, c._alloc_cb, c._free_cb, None) == 0
    c.assemble(L.V)
    assert c.packed(L.V).shape == (c.nt * (c.nt + 1) // 2, c.ng, c.ng)
    c.close()


def test_sampled_entries_outside_the_matrix_give_nan():
    """The device kernel behind stbem_entries writes NaN for a quadruple
    outside the matrix (the Python layer refuses such indices before the
    call, so the kernel is reached here through the C ABI directly)."""
    import torch
    import paper_1811_05224_amd as P
    from paper_1811_05224_amd import _lib as L
    wl = W.make("custom", n_side=2, n_t=3, n_omega=2)
    c = P.Context.from_workload(wl)
    idx = torch.tensor([[1, 0, 0, 1], [-1, 0, 0, 0], [3, 0, 0, 0], [1, 0, 8, 0], [1, 0, 0, -2], [0, 1, 0, 0]],
                       dtype=torch.int32, device=c.device)
    out = torch.zeros(idx.shape[0], dtype=torch.float64, device=c.device)
    rc = c.lib.stbem_entries(c._h, L.V, idx.shape[0], ctypes.c_void_p(idx.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    o = out.cpu().numpy()
    assert np.isfinite(o[0]) and o[0] != 0.0
    assert np.all(np.isnan(o[1:5]))
    assert o[5] == 0.0                  # above the block diagonal: causal zero
    with pytest.raises(ValueError):
        c.entries(L.V, [[1, 0, 0, 8]])
    c.close()


def test_adjoint_rhs_in_the_library():
    """(1/2 M_h + K_h)^T lam from stbem_rhs_adjoint equals the transposed
    products of the mass and the double-layer matrix."""
    import paper_1811_05224_amd as P
    from paper_1811_05224_amd import _lib as L
    from oracle.oracle import Oracle, packed_apply
    wl = W.make("custom", n_side=5, n_t=4, n_omega=2, alpha=0.7)
    o = Oracle.from_workload(wl)
    c = P.Context.from_workload(wl)
    c.assemble(L.K)
    rng = np.random.default_rng(2)
    lam = rng.standard_normal(c.n)
    got = c.rhs_adjoint(lam).cpu().numpy()
    K = o.packed("K")
    M = o.mass_matrix()
    ref = 0.5 * M.T @ lam + packed_apply(K, lam, c.nt, c.ng, trans=True)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    c.close()
