"""FP32 storage of V_h and D_h for the iterative-refinement solve.

Assembled with precision STBEM_FP32_IR, V_h is stored as the float pair
hi = fl32(V), lo = fl32(V - hi) and D_h as float; no FP64 copy of either is
kept.  V_h is computed in FP64 everywhere; D_h in FP64 on touching time
blocks and in FP32 arithmetic (float Laguerre series, one Gauss point fewer
per direction than the FP64 rule) on separated ones.  The pair must
reproduce the oracle's V_h to the FP64 bar (it carries about 48 bits), D_h's
touching blocks to FP32 rounding and its separated blocks to 1e-6 of the
block maximum (measured 2.4e-7), and the refinement solve with only this
storage must reach the oracle's solution within 1e-10.  Assembling V_h or D_h
again in FP64 drops FP32 copies made from the old FP64 storage.
"""
import numpy as np
import pytest

import workloads as W
from oracle.oracle import Oracle, packed_apply

pytestmark = pytest.mark.gpu


def block_err(gpu, ref):
    mx = np.abs(ref).reshape(ref.shape[0], -1).max(axis=1)[:, None, None]
    return np.abs(gpu - ref) / np.maximum(np.abs(ref), 1e-8 * mx + 1e-300)


@pytest.fixture(scope="module")
def small_ir():
    import paper_1811_05224_amd as P
    from paper_1811_05224_amd import _lib as L
    # 20 segments: two 16-wide tiles per block side, the second one ragged
    wl = W.make("custom", n_side=5, n_t=6, n_omega=3, alpha=1.3, k=(0.4, -0.3))
    o = Oracle.from_workload(wl)
    c = P.Context.from_workload(wl)
    c.assemble(L.K | L.M0)
    c.assemble(L.V | L.D, precision=L.FP32_IR)
    return wl, o, c, L, o.packed("V"), o.packed("D")


def test_fp32_storage_entries(small_ir):
    wl, o, c, L, V, D = small_ir
    hi, lo = c.packed_f32(L.V)
    assert lo is not None
    pair = hi.double().cpu().numpy() + lo.double().cpu().numpy()
    e_pair = block_err(pair, V).max()
    e_hi = block_err(hi.double().cpu().numpy(), V).max()
    d32, dlo = c.packed_f32(L.D)
    assert dlo is None
    d32 = d32.double().cpu().numpy()
    # touching time blocks (k - m <= 1) are computed in FP64 and rounded once;
    # separated blocks in FP32 arithmetic (float series), checked against the
    # block's largest entry: the preconditioner needs normwise accuracy only
    near = np.array([k - m <= 1 for k in range(c.nt) for m in range(k + 1)])
    e_d_near = block_err(d32[near], D[near]).max()
    dmax = np.abs(D[~near]).reshape((~near).sum(), -1).max(axis=1)[:, None, None]
    e_d_far = (np.abs(d32[~near] - D[~near]) / dmax).max()
    print("V hi+lo", e_pair, "V hi", e_hi, "D touching (FP64, stored FP32)", e_d_near,
          "D separated (FP32 arithmetic), relative to the block maximum", e_d_far)
    assert e_pair <= 1e-12
    assert e_hi <= 1e-7
    assert e_d_near <= 2e-6
    assert e_d_far <= 1e-6
    # stored blocks stay exactly symmetric
    h = hi.cpu().numpy()
    assert np.array_equal(h, np.transpose(h, (0, 2, 1)))


def test_no_fp64_copy_kept(small_ir):
    wl, o, c, L, V, D = small_ir
    import paper_1811_05224_amd as P
    with pytest.raises(P.StbemError):
        c.matrix(L.V)
    with pytest.raises(P.StbemError):
        c.matrix(L.D)
    f = c.rhs(wl.g, wl.u0)
    with pytest.raises(P.StbemError):
        c.solve(f, tol=1e-12, max_it=100, mode=L.FP64)


def test_products_from_fp32_storage(small_ir):
    wl, o, c, L, V, D = small_ir
    rng = np.random.default_rng(1)
    x = rng.standard_normal(c.n)
    for trans in (False, True):
        y = c.apply(L.V, x, trans=trans).cpu().numpy()
        ref = packed_apply(V, x, c.nt, c.ng, trans=trans)
        assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
        z = c.apply(L.D, x, trans=trans).cpu().numpy()
        refd = packed_apply(D, x, c.nt, c.ng, trans=trans)
        assert np.abs(z - refd).max() <= 1e-5 * np.abs(refd).max()
    # the preconditioner reads the FP32 D_h
    mt = o.lumped_dual_mass()
    p = c.precondition(x).cpu().numpy()
    pref = packed_apply(D, x / mt, c.nt, c.ng) / mt
    assert np.abs(p - pref).max() <= 1e-5 * np.abs(pref).max()


def test_refinement_with_fp32_storage_only(small_ir):
    wl, o, c, L, V, D = small_ir
    K, M0 = o.packed("K"), o.m0()
    f_ref = o.rhs(K, M0, wl.g, wl.u0)
    w_ref = o.solve_direct(V, f_ref)
    w, info = c.solve(f_ref, tol=1e-13, max_it=200, mode=L.FP32_IR, inner_tol=1e-6, ir_tol=1e-13)
    err = np.linalg.norm(w.cpu().numpy() - w_ref) / np.linalg.norm(w_ref)
    print("IR (FP32 storage only): inner", info.iters, "outer", info.outer, "err", err, "relres", info.true_relres)
    assert info.status == 0
    assert err < 1e-10
    # adjoint direction with the same storage
    import scipy.linalg as sla
    lam, info = c.solve(f_ref, tol=1e-13, max_it=200, mode=L.FP32_IR, trans=True, inner_tol=1e-6, ir_tol=1e-13)
    lam_ref = sla.solve(o.dense(V).T, f_ref)
    assert np.linalg.norm(lam.cpu().numpy() - lam_ref) / np.linalg.norm(lam_ref) < 1e-10


def test_fp64_reassembly_drops_stale_fp32_copies():
    """FP32 copies made from FP64 storage (first refinement solve) are freed
    when V_h or D_h is assembled again, so a later refinement solve converts
    the new storage instead of reading the old copies."""
    import paper_1811_05224_amd as P
    from paper_1811_05224_amd import _lib as L
    wl = W.make("custom", n_side=3, n_t=4, n_omega=2, alpha=0.8)
    c = P.Context.from_workload(wl)
    c.assemble(L.V | L.K | L.D)
    f = c.rhs(wl.g)
    w1, i1 = c.solve(f, tol=1e-13, max_it=100, mode=L.FP32_IR, ir_tol=1e-13)
    hi, lo = c.packed_f32(L.V)
    assert lo is None                  # the FP64 V_h serves the outer residual
    c.assemble(L.V)
    with pytest.raises(P.StbemError):
        c.packed_f32(L.V)
    c.assemble(L.D)
    with pytest.raises(P.StbemError):
        c.packed_f32(L.D)
    w2, i2 = c.solve(f, tol=1e-13, max_it=100, mode=L.FP32_IR, ir_tol=1e-13)
    assert i1.status == 0 and i2.status == 0
    assert float((w1 - w2).norm() / w1.norm()) < 1e-12
    c.close()


def test_fp32_assembly_only_for_v_and_d():
    import paper_1811_05224_amd as P
    from paper_1811_05224_amd import _lib as L
    wl = W.make("custom", n_side=2, n_t=3, n_omega=2)
    c = P.Context.from_workload(wl)
    with pytest.raises(P.StbemError):
        c.assemble(L.K, precision=L.FP32_IR)
    with pytest.raises(P.StbemError):
        c.assemble(L.V, precision=7)
    c.close()
