"""The far-field tile kernels (separated time elements) against the
per-entry kernel of the same library on meshes of 384 and 512 segments
(both code paths run the same integrals; summation orders differ), all
entries of every separated block, for V_h, K_h, D_h and the
alpha-derivatives dV_h, dK_h (whose tiles evaluate the derivative series
dV ~ -(z/alpha) e^{-z} S1, dK ~ e^{-z} SD, while the per-entry kernel takes
them from the same series through another route)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nside", [96, 128])
def test_far_tiles_match_per_entry_kernel(nside):
    import paper_1811_05224_amd as P
    from paper_1811_05224_amd import _lib as L
    wl = W.make("custom", n_side=nside, n_t=5, n_omega=2, alpha=1.0)
    c = P.Context.from_workload(wl)
    c.assemble(L.V | L.K | L.D | L.DV | L.DK)
    ng = c.ng
    for code, name in ((L.V, "V"), (L.K, "K"), (L.D, "D"), (L.DV, "dV"), (L.DK, "dK")):
        Pm = c.packed(code).cpu().numpy()
        for (k, m) in [(2, 0), (4, 1), (4, 0)]:
            ii, jj = np.meshgrid(np.arange(ng), np.arange(ng), indexing="ij")
            idx = np.stack([np.full(ng * ng, k), np.full(ng * ng, m), ii.ravel(), jj.ravel()], 1)
            ref = c.entries(code, idx).cpu().numpy().reshape(ng, ng)
            got = Pm[k * (k + 1) // 2 + m]
            scale = np.abs(ref).max()
            bad = np.argwhere(np.abs(got - ref) > 1e-13 * scale)
            print(name, (k, m), "max diff / scale", np.abs(got - ref).max() / scale, "bad entries", len(bad), bad[:5])
            assert len(bad) == 0
