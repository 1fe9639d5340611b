"""GPU construction (hodlr_construct: exact leaf blocks, fixed-rank cross
approximation with partial pivoting of every sibling block) against the
construction oracle.

Pivot columns are integer decisions taken from floating-point moduli: both
sides take them in FP64.  The cases keep the steps where the residual is far
above rounding (no near-ties), so the pivots must agree exactly: the GPU's
normalized v_k holds exactly 1.0 at the oracle's pivot column.  Each block's
approximant U_a V_b^T is then compared with the oracle's, and the leaf
blocks entry by entry.  At full size (the N = 2^20 double-layer workload,
rank 32) late pivots may legitimately differ, so that case checks properties
that hold for any pivots."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import oracle.construct as OC
import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _hd():
    from paper_2208_06290_amd import hodlr
    return hodlr


def _ragged(n, L, seed):
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.6, 1.4, 1 << L)
    s = np.maximum(8, np.round(w / w.sum() * n)).astype(np.int64)
    s[-1] += n - s.sum()
    return np.concatenate([[0], np.cumsum(s)])


def _spec(kind, n, dim, seed, shift):
    if kind == "laplace_dl":
        g = W.star_curve(n)
        return O.KernelSpec(kind, g["points"].numpy(), shift=shift, normals=g["normals"].numpy(),
                            weights=g["weights"].numpy(), curvature=g["curvature"].numpy())
    ell = 0.2 if kind == "gauss" else 0.3
    return O.KernelSpec(kind, W.kernel_points(n, dim, 128, seed), ell=ell, shift=shift)


def _gpu_build(spec, ranks, off, dtype=torch.float64):
    hd = _hd()
    P = torch.as_tensor(spec.points, device=DEV)
    kw = {}
    if spec.kind == "laplace_dl":
        kw = dict(normals=torch.as_tensor(spec.normals, device=DEV), weights=torch.as_tensor(spec.weights, device=DEV),
                  curvature=torch.as_tensor(spec.curvature, device=DEV))
    return hd.construct(spec.kind, P, ranks, leaf_offsets=off, ell=spec.ell, shift=spec.shift, dtype=dtype, **kw)


CASES = {
    "gauss_2d_L3": dict(kind="gauss", n=2048, dim=2, L=3, ranks=[8, 8, 8], shift=1e-2),
    "matern_3d_mixed": dict(kind="matern32", n=1024, dim=3, L=2, ranks=[6, 12], shift=1e-3),
    "double_layer_L4": dict(kind="laplace_dl", n=1024, dim=2, L=4, ranks=[6, 6, 6, 6], shift=0.5),
    "gauss_ragged_rank0": dict(kind="gauss", n=1000, dim=2, L=3, ranks=[5, 0, 7], shift=0.0, ragged=True),
    "gauss_1d_one_leaf": dict(kind="gauss", n=200, dim=1, L=0, ranks=[], shift=1.0),
    "double_layer_ragged": dict(kind="laplace_dl", n=1500, dim=2, L=4, ranks=[4, 6, 3, 5], shift=0.5, ragged=True),
}


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("name", list(CASES))
def test_construct_matches_oracle(name, dtype):
    c = CASES[name]
    _say(f"construct {name} {dtype}")
    spec = _spec(c["kind"], c["n"], c["dim"], 5, c["shift"])
    off = _ragged(c["n"], c["L"], 9) if c.get("ragged") else W.uniform_offsets(c["n"], c["L"])
    A = _gpu_build(spec, c["ranks"], off, dtype)
    Dg = A.D.double().cpu().numpy().T          # N x m_max
    Ug = A.U.double().cpu().numpy().T          # N x R
    Vg = A.V.double().cpu().numpy().T
    Do, Uo, Vo = O.construct_hodlr(spec, off, c["ranks"])
    tolD = 1e-14 if dtype == torch.float64 else 1e-7
    assert np.max(np.abs(Dg - Do)) <= tolD * np.max(np.abs(Do))
    col = 0
    for lvl, r in enumerate(c["ranks"], start=1):
        if r == 0:
            continue
        for a, (s0, e0) in enumerate(OC.node_ranges(off, lvl)):
            t0, f0 = OC.node_ranges(off, lvl)[a ^ 1]
            M = O.kernel_entries(spec, np.arange(s0, e0), np.arange(t0, f0))
            _, _, I, J = O.aca(lambda ri, cj: M[np.ix_(ri, cj)], e0 - s0, f0 - t0, r)
            Vb = Vg[t0:f0, col:col + r]
            for k, j in enumerate(J):
                assert j >= 0
                if dtype == torch.float64:
                    assert Vb[j, k] == 1.0, (lvl, a, k)      # the same pivot column
                else:
                    assert Vb[j, k] == np.float32(1.0)
            Ag = Ug[s0:e0, col:col + r] @ Vb.T
            Ao = Uo[s0:e0, col:col + r] @ Vo[t0:f0, col:col + r].T
            tol = 1e-12 if dtype == torch.float64 else 1e-6
            assert np.linalg.norm(Ag - Ao) <= tol * np.linalg.norm(M), (lvl, a)
        col += r


def test_construct_is_deterministic_and_rejects_bad_input():
    c = CASES["double_layer_L4"]
    spec = _spec(c["kind"], c["n"], c["dim"], 5, c["shift"])
    off = W.uniform_offsets(c["n"], c["L"])
    A1 = _gpu_build(spec, c["ranks"], off)
    A2 = _gpu_build(spec, c["ranks"], off)
    assert torch.equal(A1.U, A2.U) and torch.equal(A1.V, A2.V) and torch.equal(A1.D, A2.D)
    hd = _hd()
    P = torch.as_tensor(spec.points, device=DEV)
    with pytest.raises(ValueError):         # the double layer needs normals, weights and curvature
        hd.construct("laplace_dl", P, c["ranks"], leaf_offsets=off)
    with pytest.raises(hd.HodlrError):      # rank above a node size
        hd.construct("gauss", P, [600, 8, 8, 8], leaf_offsets=off, ell=0.1)
    with pytest.raises(hd.HodlrError):      # ell must be positive
        hd.construct("gauss", P, c["ranks"], leaf_offsets=off, ell=0.0)


def test_constructed_matrix_factors_and_solves():
    """The GPU-built double-layer matrix through the FP64 factorization: the
    solve matches the oracle's solve of the oracle-built matrix."""
    n, L, r = 4096, 4, 16
    spec = _spec("laplace_dl", n, 2, 0, 0.5)
    off = W.uniform_offsets(n, L)
    A = _gpu_build(spec, [r] * L, off)
    D, U, V = O.construct_hodlr(spec, off, [r] * L)
    H = O.Hodlr(off, [r] * L, D, U, V)
    B = np.random.default_rng(3).standard_normal((n, 2))
    X = _hd().factor(A, "fp64").solve(torch.as_tensor(np.ascontiguousarray(B.T), device=DEV)).cpu().numpy().T
    Xo = O.solve(O.factor(H), B)
    assert np.linalg.norm(X - Xo) <= 1e-11 * np.linalg.norm(Xo)


def test_full_size_double_layer_construction():
    """The N = 2^20 double-layer workload (leaf 256, 12 levels, rank 32) as
    built for the benchmark.  Late pivots of 32-step approximations of
    blocks this large can differ from the oracle's at rounding level, so the
    checks hold for any valid pivots: exact leaf blocks; every normalized
    v_k peaks at exactly 1 in modulus (or the step was exhausted); sampled
    sibling blocks of three levels approximated within 10x the oracle's own
    cross-approximation error of the same block; and the built matrix
    factors and solves consistently."""
    hd = _hd()
    n, L, r = 1 << 20, 12, 32
    g = W.star_curve(n, device=DEV)
    _say("full-size construction N=2^20")
    A = hd.construct("laplace_dl", g["points"], [r] * L, shift=0.5, normals=g["normals"], weights=g["weights"],
                     curvature=g["curvature"])
    spec = O.KernelSpec("laplace_dl", g["points"].cpu().numpy(), shift=0.5, normals=g["normals"].cpu().numpy(),
                        weights=g["weights"].cpu().numpy(), curvature=g["curvature"].cpu().numpy())
    rng = np.random.default_rng(11)
    for a in [0, (1 << L) - 1] + [int(x) for x in rng.choice(1 << L, 2, replace=False)]:
        idx = np.arange(a * 256, (a + 1) * 256)
        Dg = A.D[:, idx[0]:idx[-1] + 1].double().cpu().numpy().T
        De = O.kernel_entries(spec, idx, idx)
        assert np.max(np.abs(Dg - De)) <= 1e-14 * np.max(np.abs(De))
    # normalization of every v_k in every block
    for lvl in range(1, L + 1):
        sz = n >> lvl
        Vl = A.V[(lvl - 1) * r:lvl * r].reshape(r, 1 << lvl, sz)
        peak = Vl.abs().amax(dim=2)
        ok = (peak == 1.0) | ((peak == 0.0) & (Vl.abs().amax(dim=2) == 0.0))
        assert bool(ok.all()), lvl
    # sampled blocks of levels 12, 10 and 9 against the oracle's approximation of the same block
    Ug, Vg = A.U, A.V
    for lvl, nodes in ((12, [0, 1, 2047, 4094]), (10, [0, 777]), (9, [300])):
        sz = n >> lvl
        col = (lvl - 1) * r
        for a in nodes:
            s0, t0 = a * sz, (a ^ 1) * sz
            M = O.kernel_entries(spec, np.arange(s0, s0 + sz), np.arange(t0, t0 + sz))
            Uo, Vo, _, _ = O.aca(lambda ri, cj: M[np.ix_(ri, cj)], sz, sz, r)
            eo = np.linalg.norm(M - Uo @ Vo.T)
            Ua = Ug[col:col + r, s0:s0 + sz].double().cpu().numpy().T
            Vb = Vg[col:col + r, t0:t0 + sz].double().cpu().numpy().T
            eg = np.linalg.norm(M - Ua @ Vb.T)
            _say(f"  level {lvl} node {a}: gpu err {eg / np.linalg.norm(M):.2e}, oracle err {eo / np.linalg.norm(M):.2e}")
            assert eg <= 10.0 * eo + 1e-14 * np.linalg.norm(M)
    # the built matrix through the FP64 factorization: residual against its own product
    B = W.gaussian_rhs(n, 1, seed=3, device=DEV)
    X = hd.factor(A, "fp64").solve(B)
    rr = (torch.linalg.vector_norm(B - A.matvec(X)) / torch.linalg.vector_norm(B)).item()
    _say(f"  factor+solve of the built matrix: relres {rr:.2e}")
    assert rr < 1e-12
