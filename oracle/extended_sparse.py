"""Second, independent route to x = A^{-1} b — TEST INFRASTRUCTURE ONLY.

The HODLR system is embedded in a larger block-sparse system (Section III-E,
"Extended sparse linear system"): for every non-root node a introduce
w_a = V_{s(a)}^T x(I_{s(a)}), where s(a) is the sibling of a.  Then

    row block of leaf l:  D_l x_l + sum_{a contains l, a != root} U_a(I_l,:) w_a = b_l
    constraint of node a: V_{s(a)}^T x(I_{s(a)}) - w_a = 0,

which the paper shows (two-level example) eliminates to the same coupling
systems.  Here it is generalised to all levels and handed to a general
sparse LU (SuperLU via SciPy), so it shares no algebra with the recursion.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def extended_sparse_solve(offsets, ranks, D, U, V, B):
    offsets = np.asarray(offsets, dtype=np.int64)
    L = len(ranks)
    N = int(offsets[-1])
    nleaf = 1 << L
    colstart = np.concatenate([[0], np.cumsum(ranks)]).astype(int)

    def rng(level, i):
        per = 1 << (L - level)
        return int(offsets[i * per]), int(offsets[(i + 1) * per])

    rows, cols, vals = [], [], []

    def put(r0, c0, blk):
        rr, cc = np.meshgrid(np.arange(blk.shape[0]) + r0, np.arange(blk.shape[1]) + c0, indexing="ij")
        rows.append(rr.ravel())
        cols.append(cc.ravel())
        vals.append(np.asarray(blk, dtype=np.float64).ravel())

    for i in range(nleaf):
        s, e = rng(L, i)
        put(s, s, D[s:e, :e - s])
    woff = N
    for level in range(1, L + 1):
        r = int(ranks[level - 1])
        if r == 0:
            continue
        c0 = colstart[level - 1]
        for a in range(1 << level):
            sa, ea = rng(level, a)
            sb, eb = rng(level, a ^ 1)
            put(sa, woff, U[sa:ea, c0:c0 + r])              # U_a w_a in rows I_a
            put(woff, sb, V[sb:eb, c0:c0 + r].T)            # V_{s(a)}^T x_{s(a)}
            put(woff, woff, -np.eye(r))                     # - w_a
            woff += r
    M = sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(woff, woff))
    B2 = np.asarray(B, dtype=np.float64).reshape(N, -1)
    rhs = np.zeros((woff, B2.shape[1]))
    rhs[:N] = B2
    lu = spla.splu(M)
    X = lu.solve(rhs)[:N]
    return X[:, 0] if np.asarray(B).ndim == 1 else X
