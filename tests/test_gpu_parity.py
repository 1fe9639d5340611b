"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Every comparison is column by column on the same seeded inputs: the largest
relative error over the columns (each column's error norm over its own
norm), so a wrong narrow tail of columns cannot hide in a norm over the
block.  FP64 bar: 1e-12 relative (the stated target for the FP64 path);
mixed precision: the FP64 residual after refinement must reach 1e-10,
checked on the host by the oracle's own matrix product, and the refined
solution must match the oracle's to 1e-9."""
import math
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


def H_():
    from paper_2208_06290_amd import hodlr
    return hodlr


def _rel(a, b):
    """max over columns of ||a_j - b_j|| / ||b_j|| (vectors: one column)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if b.ndim == 1:
        a, b = a[:, None], b[:, None]
    nb = np.linalg.norm(b, axis=0)
    return float(np.max(np.linalg.norm(a - b, axis=0) / np.where(nb > 0, nb, 1.0)))


def _nonuniform_offsets(n, L, seed, lo=0.5, hi=1.5, min_leaf=5, max_leaf=256):
    rng = np.random.default_rng(seed)
    for _ in range(100):
        w = rng.uniform(lo, hi, 1 << L)
        sizes = np.maximum(min_leaf, np.round(w / w.sum() * n)).astype(np.int64)
        sizes[-1] += n - sizes.sum()
        if sizes.min() >= min_leaf and sizes.max() <= max_leaf:
            return np.concatenate([[0], np.cumsum(sizes)])
    raise RuntimeError("could not draw offsets")


def _case(n, leaf, ranks, seed, offsets=None, dtype=torch.float64, shift=4.0):
    inp = W.synthetic(n, leaf, ranks, seed=seed, leaf_offsets=offsets, dtype=dtype, shift=shift)
    H = O.from_inputs(inp)
    A = H_().HODLRMatrix.from_inputs(inp.to(DEV))
    return inp, H, A


def _rhs(n, k, seed):
    return np.random.default_rng(seed).standard_normal((n, k))


def _to_dev(X):  # N x k numpy -> (k, N) device tensor
    return torch.as_tensor(np.ascontiguousarray(X.T), device=DEV)


def _from_dev(t):  # (k, N) tensor -> N x k numpy
    return t.detach().cpu().numpy().T


# ---------------------------------------------------------------------------
CASES = {
    "L0_leaf200": dict(n=200, leaf=200, ranks=[]),
    "L1_r10": dict(n=128, leaf=64, ranks=[10]),
    "cfg0_like": dict(n=4096, leaf=64, ranks=16),
    "ragged_L4": dict(n=1000, leaf=None, L=4, ranks=[7, 0, 13, 5]),
    "ragged_L6": dict(n=3001, leaf=None, L=6, ranks=[33, 20, 64, 9, 1, 17]),
    "leaf256_L3": dict(n=2048, leaf=256, ranks=[32, 32, 32]),
    "leaf256_L5_mixed": dict(n=8192, leaf=256, ranks=[16, 48, 32, 32, 32]),
    "leaf128_L5_r64": dict(n=4096, leaf=128, ranks=64),
    "deep_L8": dict(n=4096, leaf=16, ranks=[4, 8, 3, 5, 6, 2, 7, 3]),
}


def _build(name, seed=0):
    c = CASES[name]
    off = _nonuniform_offsets(c["n"], c["L"], seed + 11) if c.get("leaf") is None else None
    return _case(c["n"], c.get("leaf") or 0, c["ranks"], seed, offsets=off)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("nrhs", [1, 3, 70])
def test_fp64_solve_matches_oracle(name, nrhs):
    _say(f"case {name} nrhs={nrhs}")
    inp, H, A = _build(name)
    hd = H_()
    B = _rhs(H.N, nrhs, 1)
    F = hd.factor(A, "fp64")
    X = _from_dev(F.solve(_to_dev(B)))
    Xo = O.solve(O.factor(H), B)
    assert _rel(X, Xo) < 1e-12


@pytest.mark.parametrize("name", ["cfg0_like", "ragged_L6", "leaf128_L5_r64", "deep_L8", "leaf256_L3",
                                  "leaf256_L5_mixed"])
def test_Y_big_matches_oracle(name):
    _say(f"Y case {name}")
    inp, H, A = _build(name, seed=2)
    F = H_().factor(A, "fp64")
    Y = _from_dev(F.y_big())
    Yo = O.y_big(O.factor(H))
    for level in range(1, H.L + 1):
        c0, c1 = H.colrange(level)
        if c1 > c0:
            assert _rel(Y[:, c0:c1], Yo[:, c0:c1]) < 1e-12, level


def test_cfg0_manufactured_solution():
    """Workload 0: b = A x_true with x_true ~ N(0,1); recover x_true."""
    _say("cfg0 manufactured")
    inp = W.make_config(0)
    H = O.from_inputs(inp)
    A = H_().HODLRMatrix.from_inputs(inp.to(DEV))
    xt = W.gaussian_rhs(H.N, 1, seed=0).numpy().T
    b = O.matvec(H, xt)
    x = _from_dev(H_().factor(A).solve(_to_dev(b)))
    assert _rel(x, np.linalg.solve(O.assemble_dense(H), b)) < 1e-12
    assert _rel(x, xt) < 1e-12


@pytest.mark.parametrize("name", ["cfg0_like", "ragged_L4", "ragged_L6", "deep_L8"])
def test_adjoint_matches_oracle(name):
    _say(f"adjoint {name}")
    inp, H, A = _build(name, seed=3)
    G = _rhs(H.N, 2, 4)
    F = H_().factor(A)
    lam = _from_dev(F.solve_adjoint(_to_dev(G)))
    assert _rel(lam, O.solve_adjoint(H, G)) < 1e-12
    b = _rhs(H.N, 2, 5)
    x = _from_dev(F.solve(_to_dev(b)))
    assert abs(np.sum(x * G) - np.sum(b * lam)) < 1e-12 * abs(np.sum(x * G)) + 1e-12


@pytest.mark.parametrize("nrhs", [5, 20, 70])
@pytest.mark.parametrize("name", ["cfg0_like", "ragged_L6", "L0_leaf200"])
@pytest.mark.parametrize("trans", [False, True])
def test_matvec_matches_oracle(name, trans, nrhs):
    _say(f"matvec {name} trans={trans} nrhs={nrhs}")
    inp, H, A = _build(name, seed=4)
    X = _rhs(H.N, nrhs, 6)
    Y = _from_dev(A.matvec(_to_dev(X), trans=trans))
    assert _rel(Y, O.matvec(H, X, trans=trans)) < 1e-13


def _build_st(name, seed, storage):
    """A case of CASES with its D, U, V stored in `storage`; the oracle gets the
    stored values (exactly representable in FP64)."""
    c = CASES[name]
    off = _nonuniform_offsets(c["n"], c["L"], seed + 11) if c.get("leaf") is None else None
    return _case(c["n"], c.get("leaf") or 0, c["ranks"], seed, offsets=off, dtype=storage)


@pytest.mark.parametrize("storage", [torch.float64, torch.float32])
@pytest.mark.parametrize("name", ["cfg0_like", "ragged_L6", "deep_L8"])
def test_gradients_match_oracle(name, storage):
    _say(f"grad {name} storage {storage}")
    inp, H, A = _build_st(name, 5, storage)
    X = _rhs(H.N, 3, 7)
    Lam = _rhs(H.N, 3, 8)
    F = H_().factor(A, "fp64" if storage == torch.float64 else "fp32")
    dD, dU, dV = F.grad(_to_dev(X), _to_dev(Lam))
    assert dD.dtype == storage and dU.dtype == storage and dV.dtype == storage
    rD, rU, rV = O.grad_structured(H, X, Lam)
    # the gradients are formed in FP64 and rounded once to the storage type
    tol = 1e-13 if storage == torch.float64 else 1e-6
    dDn = dD.double().cpu().numpy().T
    for i in range(1 << H.L):
        s0, e = O.node_range(H, H.L, i)
        assert _rel(dDn[s0:e, :e - s0], rD[s0:e, :e - s0]) < tol
    assert _rel(dU.double().cpu().numpy().T, rU) < tol
    assert _rel(dV.double().cpu().numpy().T, rV) < tol


@pytest.mark.parametrize("variant", ["fp64", "fp32", "fp32_refined"])
def test_autograd_function_matches_oracle(variant):
    _say(f"autograd {variant}")
    storage = torch.float64 if variant == "fp64" else torch.float32
    inp, H, A = _build_st("ragged_L4", 6, storage)
    hd = H_()
    b = torch.as_tensor(_rhs(H.N, 1, 9)[:, 0], device=DEV)
    t = torch.as_tensor(_rhs(H.N, 1, 10)[:, 0], device=DEV)
    D = inp.D.to(DEV).clone().requires_grad_(True)
    U = inp.U.to(DEV).clone().requires_grad_(True)
    V = inp.V.to(DEV).clone().requires_grad_(True)
    bb = b.clone().requires_grad_(True)
    x = hd.HodlrSolve.apply(bb, D, U, V, inp.ranks, inp.leaf_offsets, "fp64" if variant == "fp64" else "fp32",
                            variant == "fp32_refined")
    loss = ((x - t) ** 2).sum()
    loss.backward()
    L0, xo, lam, rD, rU, rV = O.loss_and_grads(H, b.cpu().numpy(), t.cpu().numpy())
    errs = dict(loss=abs(loss.item() - L0) / abs(L0), b=_rel(bb.grad.cpu().numpy(), lam),
                U=_rel(U.grad.double().cpu().numpy().T, rU), V=_rel(V.grad.double().cpu().numpy().T, rV))
    dDn = D.grad.double().cpu().numpy().T
    errs["D"] = max(_rel(dDn[s0:e, :e - s0], rD[s0:e, :e - s0])
                    for s0, e in (O.node_range(H, H.L, i) for i in range(1 << H.L)))
    _say(f"  {variant} gradient errors vs the FP64 oracle: " + ", ".join(f"{k} {v:.1e}" for k, v in errs.items()))
    # FP64: 1e-12; FP32 factors without refinement: the FP32 solve's error,
    # about kappa * 6e-8; refined: FP64 solves, gradients rounded once to FP32
    tol = {"fp64": 1e-12, "fp32": 1e-4, "fp32_refined": 1e-6}[variant]
    assert max(errs.values()) < tol, errs


CASES_FP32 = ["cfg0_like", "L1_r10", "ragged_L4", "ragged_L6", "deep_L8", "leaf128_L5_r64", "leaf256_L3",
              "leaf256_L5_mixed"]


@pytest.mark.parametrize("storage", [torch.float64, torch.float32])
@pytest.mark.parametrize("name", CASES_FP32)
def test_fp32_factor_with_refinement(name, storage):
    """FP32 factorization (all coupling routes: explicit inverse for r in
    {8, 16, 24, 32}, LU for the others, rank-0 levels, ragged and deep trees,
    r = 64) refined in FP64 to a 1e-10 residual, forward and adjoint."""
    _say(f"fp32 factor {name}, storage {storage}")
    inp, H, A = _build_st(name, 7, storage)
    B = _rhs(H.N, 3, 11)
    F = H_().factor(A, "fp32")
    x0 = _from_dev(F.solve(_to_dev(B)))
    Xo = O.solve(O.factor(H), B)
    e32 = _rel(x0, Xo)
    _say(f"  plain fp32 solve rel error {e32:.2e}")
    assert e32 < 1e-3
    st = {}
    x = _from_dev(F.solve(_to_dev(B), refine=True, tol=1e-10, stats=st))
    _say(f"  refined: {st}")
    assert st["converged"] and st["relres"] <= 1e-10
    assert O.relres(H, x, B) <= 1e-10
    assert _rel(x, Xo) < 1e-9
    sta = {}
    lam = _from_dev(F.solve_adjoint(_to_dev(B), refine=True, tol=1e-10, stats=sta))
    assert sta["converged"] and O.relres(O.transpose(H), lam, B) <= 1e-10
    assert _rel(lam, O.solve_adjoint(H, B)) < 1e-9


CASES_BF16 = ["cfg0_like", "ragged_L6", "deep_L8", "leaf128_L5_r64", "leaf256_L3"]
# deep_L8 (16-row leaves, every rank below 16) has no contraction that fills a
# 16 x 16 x 16 bfloat16 block: its leaf LU has no trailing block updates, its
# leaf solves one row block per wave and its level passes take the general
# (FP32) kernel, so its BF16 factorization is the FP32 one exactly
BF16_FP32_ONLY = {"deep_L8"}


@pytest.mark.parametrize("storage", [torch.float64, torch.float32])
@pytest.mark.parametrize("name", CASES_BF16)
def test_bf16_factor_with_refinement(name, storage):
    """BF16 factorization (bfloat16 operands, FP32 accumulation, FP32 panels and
    K) refined in FP64 to a 1e-10 residual, forward and adjoint.  The unrefined
    BF16 solve must be measurably less accurate than the FP32 one (the operands
    really are rounded) yet within kappa * u_bf16 of the oracle."""
    _say(f"bf16 factor {name}, storage {storage}")
    inp, H, A = _build_st(name, 17, storage)
    B = _rhs(H.N, 3, 18)
    hd = H_()
    Xo = O.solve(O.factor(H), B)
    F32 = hd.factor(A, "fp32")
    e32 = _rel(_from_dev(F32.solve(_to_dev(B))), Xo)
    del F32
    F = hd.factor(A, "bf16")
    ebf = _rel(_from_dev(F.solve(_to_dev(B))), Xo)
    _say(f"  plain solve rel error: fp32 {e32:.2e}, bf16 {ebf:.2e}")
    assert ebf < 5e-2
    if name in BF16_FP32_ONLY:
        assert ebf == e32
    else:
        assert ebf > 4 * e32
    st = {}
    x = _from_dev(F.solve(_to_dev(B), refine=True, tol=1e-10, stats=st))
    _say(f"  refined: {st}")
    assert st["converged"] and st["relres"] <= 1e-10
    assert O.relres(H, x, B) <= 1e-10
    assert _rel(x, Xo) < 1e-9
    sta = {}
    lam = _from_dev(F.solve_adjoint(_to_dev(B), refine=True, tol=1e-10, stats=sta))
    _say(f"  adjoint refined: {sta}")
    assert sta["converged"] and O.relres(O.transpose(H), lam, B) <= 1e-10
    assert _rel(lam, O.solve_adjoint(H, B)) < 1e-9


def test_refinement_reports_non_convergence():
    """kappa * u_fp32 >> 1: refinement must not claim success."""
    _say("refine non-convergence")
    inp = W.synthetic(256, 32, 4, seed=8)
    # columns 3 and 4 of A equal up to 1e-11 e_3: leaf 0 columns and V rows copied
    inp.D[3, 0:32] = inp.D[4, 0:32]
    inp.D[3, 3] += 1e-11
    inp.V[:, 3] = inp.V[:, 4]
    H = O.from_inputs(inp)
    assert np.linalg.cond(O.assemble_dense(H)) > 1e9
    A = H_().HODLRMatrix.from_inputs(inp.to(DEV))
    F = H_().factor(A, "fp32")
    st = {}
    F.solve(_to_dev(_rhs(H.N, 1, 12)), refine=True, tol=1e-10, max_iter=8, stats=st)
    _say(f"  {st}")
    assert not st["converged"] and st["relres"] > 1e-10


def test_singular_leaf_is_reported():
    _say("singular leaf")
    inp = W.synthetic(512, 64, 8, seed=9)
    inp.D[5, 64 * 3:64 * 4] = 0.0   # leaf 3, column 5 of its block is zero
    A = H_().HODLRMatrix.from_inputs(inp.to(DEV))
    with pytest.raises(H_().HodlrError) as e:
        H_().factor(A)
    assert e.value.status == 1
    assert e.value.info["level"] == 3 and e.value.info["node"] == 3 and e.value.info["column"] <= 5


def test_singular_coupling_matrix_is_reported():
    _say("singular K")
    D = torch.ones(1, 2, dtype=torch.float64, device=DEV)
    U = torch.ones(1, 2, dtype=torch.float64, device=DEV)
    A = H_().HODLRMatrix(D, U, U.clone(), [1], [0, 1, 2])
    with pytest.raises(H_().HodlrError) as e:
        H_().factor(A)
    assert e.value.status == 1 and e.value.info["level"] == 0


@pytest.mark.parametrize("rank,leaf", [(16, 64), (64, 128)])
def test_coupling_matrices_with_zero_generators(rank, leaf):
    """V generators of level 2 set to zero: the two coupling matrices of
    level 1 are [[0, I], [I, 0]] (eq. "e:k" with V_a^T Y_a = 0), so every
    elimination step takes its pivot from the other half of the rows.  2r = 32
    runs the four-wave Gauss-Jordan inverse, 2r = 128 the eight-wave one.
    Solve, adjoint solve and log|det A| against the oracle and LAPACK."""
    _say(f"zero generators rank {rank}")
    n = 4096
    inp = W.synthetic(n, leaf, rank, seed=21)
    inp.V[rank:2 * rank, :] = 0.0   # columns [R_1, R_2) of V_big: level 2
    H = O.from_inputs(inp)
    A = H_().HODLRMatrix.from_inputs(inp.to(DEV))
    F = H_().factor(A, "fp64")
    B = _rhs(n, 2, 22)
    assert _rel(_from_dev(F.solve(_to_dev(B))), O.solve(O.factor(H), B)) < 1e-12
    assert _rel(_from_dev(F.solve_adjoint(_to_dev(B))), O.solve_adjoint(H, B)) < 1e-12
    sign, la = F.slogdet()
    s_o, l_o = np.linalg.slogdet(O.assemble_dense(H))
    assert sign == s_o and abs(la - l_o) <= 1e-12 * max(1.0, abs(l_o))


def test_bitwise_determinism():
    _say("determinism")
    inp, H, A = _build("leaf256_L3", seed=10)
    B = _to_dev(_rhs(H.N, 2, 13))
    hd = H_()
    for prec in ("fp64", "fp32", "bf16"):
        F1 = hd.factor(A, prec)
        F2 = hd.factor(A, prec)
        assert torch.equal(F1.y_big(), F2.y_big())
        assert torch.equal(F1.solve(B), F2.solve(B))
        assert torch.equal(F1.solve_adjoint(B), F2.solve_adjoint(B))


def test_refactor_reuses_storage():
    _say("refactor")
    inp, H, A = _build("cfg0_like", seed=11)
    inp2 = W.synthetic(4096, 64, 16, seed=12)
    hd = H_()
    F = hd.factor(A)
    nb = F.nbytes
    A2 = hd.HODLRMatrix.from_inputs(inp2.to(DEV))
    F.refactor(A2)
    assert F.nbytes == nb
    B = _rhs(4096, 1, 14)
    assert _rel(_from_dev(F.solve(_to_dev(B))), O.solve(O.factor(O.from_inputs(inp2)), B)) < 1e-12


def test_concurrent_solves_on_two_streams():
    """Solves and adjoint solves issued on two streams without waiting in
    between share one factorization but not its workspace: every result must
    match the oracle."""
    _say("two streams")
    inp, H, A = _build("leaf256_L3", seed=14)
    hd = H_()
    F = hd.factor(A)
    Fo = O.factor(H)
    Bs = [_rhs(H.N, 2 + k, 20 + k) for k in range(6)]
    dev_B = [_to_dev(B) for B in Bs]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    cur = torch.cuda.current_stream()
    s1.wait_stream(cur)
    s2.wait_stream(cur)
    outs = []
    for k, B in enumerate(dev_B):
        st = s1 if k % 2 == 0 else s2
        with torch.cuda.stream(st):
            outs.append(F.solve(B) if k % 3 else F.solve_adjoint(B))
    cur.wait_stream(s1)
    cur.wait_stream(s2)
    torch.cuda.synchronize()
    for k, (B, X) in enumerate(zip(Bs, outs)):
        want = O.solve(Fo, B) if k % 3 else O.solve_adjoint(H, B)
        assert _rel(_from_dev(X), want) < 1e-12, k


def test_concurrent_refined_solves_from_two_threads():
    """Two host threads, each refining FP32 solves on its own stream (every
    refinement step synchronises its stream), on one factorization."""
    import threading
    _say("two threads")
    inp, H, A = _build_st("cfg0_like", 15, torch.float32)
    hd = H_()
    F = hd.factor(A, "fp32")
    Bs = [_rhs(H.N, 2, 30 + k) for k in range(4)]
    dev_B = [_to_dev(B) for B in Bs]
    torch.cuda.synchronize()
    res = {}

    def work(tid):
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            for k in range(tid, len(Bs), 2):
                stats = {}
                x = F.solve(dev_B[k], refine=True, stats=stats) if k < 2 else \
                    F.solve_adjoint(dev_B[k], refine=True, stats=stats)
                st.synchronize()
                res[k] = (_from_dev(x), stats)

    th = [threading.Thread(target=work, args=(t,)) for t in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    Fo = O.factor(H)
    for k, B in enumerate(Bs):
        x, stats = res[k]
        want = O.solve(Fo, B) if k < 2 else O.solve_adjoint(H, B)
        assert stats["converged"], (k, stats)
        assert _rel(x, want) < 1e-9, k


def _offsets16(n, L, seed):
    """Non-uniform leaves whose sizes are multiples of 16 (in-place factors)."""
    rng = np.random.default_rng(seed)
    sizes = 16 * rng.integers(2, 9, 1 << L)
    sizes[-1] += n - sizes.sum()
    assert sizes[-1] > 0 and sizes[-1] % 16 == 0 and sizes.max() <= 256
    return np.concatenate([[0], np.cumsum(sizes)])


@pytest.mark.parametrize("name,storage", [("cfg0_like", torch.float64), ("leaf256_L3", torch.float64),
                                          ("ragged16_L5", torch.float64), ("cfg0_like", torch.float32)])
def test_inplace_factorization(name, storage):
    """HODLR_INPLACE: the leaf factors overwrite D and Y_big overwrites U (the
    paper's in-place algorithm); solves match the oracle, U afterwards holds
    Y_big, and the factorization owns fewer bytes."""
    _say(f"in place {name} {storage}")
    if name == "ragged16_L5":
        off = _offsets16(16 * 5 * 32, 5, 3)
        inp = W.synthetic(int(off[-1]), 0, [6, 13, 16, 3, 9], seed=16, leaf_offsets=off, dtype=storage)
        H = O.from_inputs(inp)
    else:
        inp, H, A = _build_st(name, 16, storage)
    hd = H_()
    prec = "fp64" if storage == torch.float64 else "fp32"
    A_ref = hd.HODLRMatrix.from_inputs(inp.to(DEV))
    F_ref = hd.factor(A_ref, prec)
    D2, U2, V2 = inp.D.to(DEV).clone(), inp.U.to(DEV).clone(), inp.V.to(DEV).clone()
    A2 = hd.HODLRMatrix(D2, U2, V2, inp.ranks, inp.leaf_offsets)
    F = hd.factor(A2, prec, inplace=True)
    assert F.nbytes < F_ref.nbytes
    _say(f"  factor bytes: in place {F.nbytes}, separate {F_ref.nbytes}")
    B = _rhs(H.N, 3, 17)
    X = _from_dev(F.solve(_to_dev(B)))
    Xr = _from_dev(F_ref.solve(_to_dev(B)))
    tol = 1e-12 if storage == torch.float64 else 1e-3
    assert _rel(X, O.solve(O.factor(H), B)) < tol
    assert torch.equal(F.y_big(), F_ref.y_big())
    assert torch.equal(U2.double(), F_ref.y_big())  # Y_big now lives in U
    assert np.array_equal(X, Xr)
    G = _from_dev(F.solve_adjoint(_to_dev(B)))
    assert _rel(G, O.solve_adjoint(H, B)) < tol
    with pytest.raises(hd.HodlrError) as e:
        F.solve(_to_dev(B), refine=True)
    assert e.value.status == -1
    # refactor in place on a fresh copy of the same matrix
    A3 = hd.HODLRMatrix(inp.D.to(DEV).clone(), inp.U.to(DEV).clone(), V2, inp.ranks, inp.leaf_offsets)
    F.refactor(A3)
    assert np.array_equal(_from_dev(F.solve(_to_dev(B))), Xr)


def test_many_tiles_and_segments():
    """N = 65536, leaf 256, r = 32: nodes of the top levels span 128 tiles,
    so the products go through the segment reduction."""
    _say("many tiles N=65536")
    inp, H, A = _case(65536, 256, 32, seed=13)
    B = _rhs(H.N, 2, 15)
    F = H_().factor(A)
    X = _from_dev(F.solve(_to_dev(B)))
    assert _rel(X, O.solve(O.factor(H), B)) < 1e-12
    G = _from_dev(F.solve_adjoint(_to_dev(B)))
    assert _rel(G, O.solve_adjoint(H, B)) < 1e-12


def _subtree(H, k, i=0):
    """Node i of level k as a HODLR matrix of its own (its leaves, the
    generators of levels k+1..L on its rows): an independent system with the
    same leaf size and ranks."""
    s0, e0 = O.node_range(H, k, i)
    per = 1 << (H.L - k)
    off = H.offsets[i * per:(i + 1) * per + 1] - s0
    c0 = int(sum(H.ranks[:k]))
    return O.Hodlr(off.copy(), list(H.ranks[k:]), H.D[s0:e0].copy(), H.U[s0:e0, c0:].copy(),
                   H.V[s0:e0, c0:].copy()), s0, e0


def test_full_size_bie_in_bench_configuration():
    """The benchmark workload itself (Laplace double-layer BIE on the star
    curve, N = 2^20, leaf 256, 12 levels, rank 32) in the launch configuration
    that bench.py times, checked at full size by what the oracle can evaluate:
      * the FP64 residual of the whole solve through the oracle's own HODLR
        product (host, FP64);
      * Y_big of levels 5..12 on the leftmost level-4 node (65536 rows):
        those columns equal the Y of that node as a HODLR matrix of its own,
        factored by the oracle;
      * Y_big of levels 1..4 on the leftmost node of each level by the
        defining property A_a Y_a = U_a (oracle product on the node);
      * the solution of that level-4 node as a system of its own (GPU, same
        kernels and shapes) against the oracle's;
      * the FP32 factorization refined to a 1e-10 residual, at full size and
        on the level-4 node against the oracle."""
    _say("full-size BIE N=2^20: generating")
    inp = W.make_config(2, device=DEV)
    A = H_().HODLRMatrix.from_inputs(inp)
    b = W.gaussian_rhs(inp.n, 1, seed=0, device=DEV)
    F = H_().factor(A, "fp64")
    x = F.solve(b)
    Y = F.y_big()
    torch.cuda.synchronize()
    _say("full-size BIE: oracle checks")
    H = O.from_inputs(inp)
    bh = b.detach().cpu().numpy().T
    xh = x.detach().cpu().numpy().T
    relres = O.relres(H, xh, bh)
    _say(f"full-size BIE FP64 relres {relres:.3e}")
    assert relres < 1e-12
    Yh = Y.detach().cpu().numpy().T
    del Y
    # levels 1..4: A_a Y_a = U_a on the leftmost node of each level
    for lv in range(1, 5):
        Ha, s0, e0 = _subtree(H, lv)
        c0, c1 = H.colrange(lv)
        res = _rel(O.matvec(Ha, Yh[s0:e0, c0:c1]), H.U[s0:e0, c0:c1])
        _say(f"full-size BIE Y level {lv}: ||A_a Y_a - U_a|| / ||U_a|| = {res:.3e}")
        assert res < 1e-12
    # levels 5..12 on the leftmost level-4 node, against the oracle's factorization of that node
    k = 4
    Hs, s0, e0 = _subtree(H, k)
    _say(f"full-size BIE: oracle factorization of the level-{k} node ({e0 - s0} rows)")
    Fs = O.factor(Hs)
    Ys = O.y_big(Fs)
    c0 = int(sum(H.ranks[:k]))
    for lv in range(1, Hs.L + 1):
        a0, a1 = Hs.colrange(lv)
        err = _rel(Yh[s0:e0, c0 + a0:c0 + a1], Ys[:, a0:a1])
        _say(f"full-size BIE Y level {k + lv}: rel err {err:.3e}")
        assert err < 1e-12
    # the level-4 node as a system of its own on the GPU
    inp_s = W.HodlrInputs(e0 - s0, Hs.L, Hs.offsets, Hs.ranks, inp.D[:, s0:e0], inp.U[c0:, s0:e0],
                          inp.V[c0:, s0:e0])
    As = H_().HODLRMatrix.from_inputs(inp_s)
    bs = _rhs(e0 - s0, 2, 40)
    xs = _from_dev(H_().factor(As, "fp64").solve(_to_dev(bs)))
    xso = O.solve(Fs, bs)
    err = _rel(xs, xso)
    _say(f"full-size BIE level-{k} node solve vs oracle: {err:.3e}")
    assert err < 1e-12
    del F
    F32 = H_().factor(A, "fp32")
    stats = {}
    x32 = F32.solve(b, refine=True, tol=1e-10, stats=stats)
    x32h = x32.detach().cpu().numpy().T
    relres32 = O.relres(H, x32h, bh)
    _say(f"full-size BIE FP32+IR relres {relres32:.3e} after {stats.get('iters')} steps")
    assert relres32 <= 1e-10
    assert _rel(x32h, xh) < 1e-10
    del F32
    st = {}
    xs32 = _from_dev(H_().factor(As, "fp32").solve(_to_dev(bs), refine=True, stats=st))
    err = _rel(xs32, xso)
    _say(f"full-size BIE level-{k} node FP32+IR vs oracle: {err:.3e} ({st})")
    assert err < 1e-10
