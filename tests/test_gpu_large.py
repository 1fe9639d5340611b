"""The large mixed-precision workload at full size: N = 2^22 (leaf 256, 14
levels, rank 64 on every level), D, U, V stored in FP32, a BF16
factorization with FP64 iterative refinement of 32 right-hand sides to a
1e-10 residual, and the adjoint refined the same way on the same factors.

The oracle cannot factor a 4M-row system on the host in test time, so the
checks are:
  * the refined residuals (the library's FP64 residual), re-evaluated with
    the FP64 GPU product and cross-checked on sampled leaves against a host
    FP64 evaluation of A x from its definition (leaf block plus, per level,
    U_a (V_b^T x_b) for the sibling b of the leaf's ancestor a);
  * a level-6 node (65536 rows, 8 levels) as a system of its own: the same
    BF16 + FP64 refinement path against the oracle's FP64 solve;
  * the memory the factors own, against the storage count of the factors."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _hd():
    from paper_2208_06290_amd import hodlr
    return hodlr


def _rows_of_product(inp, X, leaf):
    """(A X)(I_leaf, :) in FP64 on the host from the stored D, U, V (uniform tree)."""
    L, n = inp.levels, inp.n
    m = n >> L
    s0, e0 = leaf * m, (leaf + 1) * m
    Da = inp.D[:m, s0:e0].double().cpu().numpy().T            # D_a[p, q] = D[q, s0 + p]
    out = Da @ X[s0:e0]
    Rp = np.concatenate([[0], np.cumsum(inp.ranks)])
    for lv in range(1, L + 1):
        c0, c1 = int(Rp[lv - 1]), int(Rp[lv])
        sz = n >> lv
        anc = leaf >> (L - lv)
        sib = anc ^ 1
        Ua = inp.U[c0:c1, s0:e0].double().cpu().numpy().T     # U_anc restricted to the leaf's rows
        Vb = inp.V[c0:c1, sib * sz:(sib + 1) * sz].double().cpu().numpy().T
        out = out + Ua @ (Vb.T @ X[sib * sz:(sib + 1) * sz])
    return out


def _relres_cols(R, B):
    return float(np.max(np.linalg.norm(R, axis=0) / np.linalg.norm(B, axis=0)))


def test_large_bf16_refined_32_rhs_and_adjoint():
    hd = _hd()
    _say("large N=2^22 r=64 FP32 storage: generating on the GPU")
    inp = W.make_config(4, device=DEV)
    assert inp.D.dtype == torch.float32 and inp.levels == 14 and set(inp.ranks) == {64}
    A = hd.HODLRMatrix.from_inputs(inp)
    B = W.gaussian_rhs(inp.n, 32, seed=0, device=DEV)
    free0 = torch.cuda.mem_get_info()[0]
    F = hd.factor(A, "bf16")
    torch.cuda.synchronize()
    used = free0 - torch.cuda.mem_get_info()[0]
    R = sum(inp.ranks)
    # factors: FP32 leaf LU (256 x 256 per leaf) and Y_big (N x R); besides
    # them the factorization's workspace (tile partials, segment sums and W of
    # the widest level, each about 2^14 x 64 x R_13 FP32 values) and the
    # small pivots and K factors
    floor = 4 * (inp.n * 256 + inp.n * R)
    work = 3 * 4 * (inp.n // 256) * 64 * (R - 64)
    _say(f"  factor bytes {F.nbytes / 1e9:.2f} GB (device {used / 1e9:.2f} GB); LU + Y_big {floor / 1e9:.2f} GB, "
         f"workspace bound {work / 1e9:.2f} GB; matrix {4 * (inp.n * 256 + 2 * inp.n * R) / 1e9:.2f} GB")
    assert floor <= F.nbytes <= 1.05 * (floor + work)
    assert abs(used - F.nbytes) <= 0.02 * F.nbytes
    st = {}
    X = F.solve(B, refine=True, tol=1e-10, stats=st)
    sta = {}
    Lam = F.solve_adjoint(B, refine=True, tol=1e-10, stats=sta)
    _say(f"  forward refinement {st}; adjoint refinement {sta}")
    assert st["converged"] and st["relres"] <= 1e-10
    assert sta["converged"] and sta["relres"] <= 1e-10
    # the residuals again, by the FP64 GPU product
    AX = A.matvec(X)
    ATL = A.matvec(Lam, trans=True)
    rr = (torch.linalg.vector_norm(B - AX, dim=1) / torch.linalg.vector_norm(B, dim=1)).max().item()
    rra = (torch.linalg.vector_norm(B - ATL, dim=1) / torch.linalg.vector_norm(B, dim=1)).max().item()
    _say(f"  FP64 GPU product: forward relres {rr:.3e}, adjoint relres {rra:.3e}")
    assert rr <= 1e-10 and rra <= 1e-10
    # the GPU product on sampled leaves against the host evaluation
    Xh = X.cpu().numpy().T
    AXh = AX.cpu().numpy().T
    m = inp.n >> inp.levels
    nleaf = 1 << inp.levels
    worst = 0.0
    for leaf in [0, nleaf - 1] + [int(v) for v in np.random.default_rng(80).choice(nleaf, 2, replace=False)]:
        ref = _rows_of_product(inp, Xh, leaf)
        got = AXh[leaf * m:(leaf + 1) * m]
        worst = max(worst, float(np.max(np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0))))
    _say(f"  GPU product vs host definition on 4 sampled leaves: max rel {worst:.3e}")
    assert worst < 1e-13


def test_large_level6_node_against_oracle():
    """A level-6 node of the large workload (65536 rows, 8 levels, r = 64) as a
    system of its own: BF16 factors + FP64 refinement on the GPU against the
    oracle's FP64 solve, forward and adjoint."""
    hd = _hd()
    _say("large workload, level-6 node: generating")
    full = W.make_config(4, device=DEV)
    k = 6
    n_s = full.n >> k
    c0 = sum(full.ranks[:k])
    inp = W.HodlrInputs(n_s, full.levels - k, full.leaf_offsets[:(1 << (full.levels - k)) + 1],
                        full.ranks[k:], full.D[:, :n_s].contiguous(), full.U[c0:, :n_s].contiguous(),
                        full.V[c0:, :n_s].contiguous())
    del full
    torch.cuda.empty_cache()
    H = O.from_inputs(inp)
    B = np.random.default_rng(81).standard_normal((n_s, 4))
    _say(f"  oracle factorization ({n_s} rows)")
    Fo = O.factor(H)
    Xo = O.solve(Fo, B)
    Lo = O.solve_adjoint(H, B)
    F = hd.factor(hd.HODLRMatrix.from_inputs(inp), "bf16")
    Bd = torch.as_tensor(np.ascontiguousarray(B.T), device=DEV)
    st, sta = {}, {}
    X = F.solve(Bd, refine=True, stats=st).cpu().numpy().T
    Lm = F.solve_adjoint(Bd, refine=True, stats=sta).cpu().numpy().T
    ex = float(np.max(np.linalg.norm(X - Xo, axis=0) / np.linalg.norm(Xo, axis=0)))
    el = float(np.max(np.linalg.norm(Lm - Lo, axis=0) / np.linalg.norm(Lo, axis=0)))
    _say(f"  BF16+IR vs oracle: forward {ex:.3e} ({st}), adjoint {el:.3e} ({sta})")
    assert st["converged"] and sta["converged"]
    assert ex < 1e-9 and el < 1e-9
    assert O.relres(H, X, B) <= 1e-10
