"""Floor of the relative error for sampled matrix entries.

An entry is compared relative to max(|oracle value|, 1e-8 * scale of its
block), so entries far below the block's largest values need only absolute
accuracy.  The scale of a block is the oracle's largest |entry| among the
samples of that block; K_h vanishes on collinear segment pairs, so for K_h
the oracle's whole sampled row of the block is added (a row of a block on
one straight side may otherwise hold only tiny values).
"""
import numpy as np


def block_floor(o, op, idx, ref, ng):
    scale = {}
    for n, (k, m) in enumerate(zip(idx[:, 0], idx[:, 1])):
        scale[(k, m)] = max(scale.get((k, m), 0.0), abs(ref[n]))
    if op in ("K", "dK"):
        rows = sorted(set((int(k), int(m), int(i)) for k, m, i in idx[:, :3]))
        full = np.array([(k, m, i, j) for (k, m, i) in rows for j in range(ng)], dtype=np.int32)
        vals = np.abs(o.entries(op, full)).reshape(len(rows), ng).max(axis=1)
        for (k, m, i), v in zip(rows, vals):
            scale[(k, m)] = max(scale[(k, m)], v)
    return np.array([1e-8 * scale[(k, m)] for k, m in zip(idx[:, 0], idx[:, 1])])
