"""Complex HODLR matrices on the GPU (the real embedding of the factor/solve
path) against the complex oracle, which the CPU pins tie to the real
recursion through the same embedding and to dense LAPACK.  Comparisons are
per column (max over columns of the relative 2-norm error)."""
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


def _offsets(n, L, seed):
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.6, 1.4, 1 << L)
    s = np.maximum(6, np.round(w / w.sum() * n)).astype(np.int64)
    s[-1] += n - s.sum()
    return np.concatenate([[0], np.cumsum(s)])


CASES = {
    "uniform_L4": dict(n=512, leaf=32, ranks=6),
    "ragged_L3_rank0": dict(n=300, L=3, ranks=[5, 0, 4]),
    "deep_L6": dict(n=640, leaf=10, ranks=[2, 3, 1, 4, 2, 3]),
    "leaf128_L3_r32": dict(n=1024, leaf=128, ranks=32),       # embedded: leaf 256, rank 64 (the limits)
    "helmholtz_L6": dict(helmholtz=True, n=4096, leaf=64, ranks=16),
}


def _build(name, seed=0):
    c = CASES[name]
    if c.get("helmholtz"):
        inp = W.helmholtz_matrix(c["n"], c["leaf"], c["ranks"], kappa=20.0, seed=seed)
    else:
        off = _offsets(c["n"], c["L"], seed + 3) if "L" in c else None
        inp = W.synthetic(c["n"], c.get("leaf", 0), c["ranks"], seed=seed, leaf_offsets=off, dtype=torch.complex128)
    return inp, O.from_inputs(inp), _hd().HODLRMatrix.from_inputs(inp.to(DEV))


def _rhs(n, k, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k))


def _dev(X):
    return torch.as_tensor(np.ascontiguousarray(X.T), device=DEV)


def _host(t):
    return t.detach().cpu().numpy().T


def _rel(X, Xo):
    return float(np.max(np.linalg.norm(X - Xo, axis=0) / np.linalg.norm(Xo, axis=0)))


@pytest.mark.parametrize("nrhs", [1, 3])
@pytest.mark.parametrize("name", list(CASES))
def test_complex_solve_and_adjoint_match_oracle(name, nrhs):
    _say(f"complex {name} nrhs={nrhs}")
    inp, H, A = _build(name)
    B = _rhs(H.N, nrhs, 1)
    F = _hd().factor(A, "fp64")
    X = _host(F.solve(_dev(B)))
    assert X.dtype == np.complex128
    assert _rel(X, O.solve(O.factor(H), B)) < 1e-12
    L = _host(F.solve_adjoint(_dev(B)))
    assert _rel(L, O.solve_adjoint(H, B)) < 1e-12


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("name", ["uniform_L4", "ragged_L3_rank0", "helmholtz_L6"])
def test_complex_low_precision_with_refinement(name, precision):
    inp, H, A = _build(name, seed=4)
    B = _rhs(H.N, 2, 5)
    F = _hd().factor(A, precision)
    st, sta = {}, {}
    X = _host(F.solve(_dev(B), refine=True, stats=st))
    L = _host(F.solve_adjoint(_dev(B), refine=True, stats=sta))
    _say(f"  {name} {precision}: {st} adjoint {sta}")
    assert st["converged"] and sta["converged"]
    assert _rel(X, O.solve(O.factor(H), B)) < 1e-9
    assert _rel(L, O.solve_adjoint(H, B)) < 1e-9
    assert O.relres(H, X, B) <= 1e-10


@pytest.mark.parametrize("name", ["uniform_L4", "ragged_L3_rank0", "deep_L6"])
def test_complex_matvec_y_and_logdet(name):
    inp, H, A = _build(name, seed=6)
    X = _rhs(H.N, 2, 7)
    assert _rel(_host(A.matvec(_dev(X))), O.matvec(H, X)) < 1e-13
    assert _rel(_host(A.matvec(_dev(X), trans=True)), O.matvec(H, X, trans=True)) < 1e-13
    F = _hd().factor(A, "fp64")
    Y = _host(F.y_big())
    Yo = O.y_big(O.factor(H))
    for level in range(1, H.L + 1):
        c0, c1 = H.colrange(level)
        if c1 > c0:
            assert np.linalg.norm(Y[:, c0:c1] - Yo[:, c0:c1]) <= 1e-12 * np.linalg.norm(Yo[:, c0:c1]), level
    sign, la = F.slogdet()
    _, ld = np.linalg.slogdet(O.assemble_dense(H))
    assert sign == 1.0 and abs(la - ld) <= 1e-12 * max(1.0, abs(ld))


def test_complex_refactor_noalloc_and_determinism():
    inp, H, A = _build("uniform_L4", seed=8)
    hd = _hd()
    B = _rhs(H.N, 2, 9)
    F = hd.factor(A, "fp64")
    X1 = F.solve(_dev(B))
    F2 = hd.factor(hd.HODLRMatrix.from_inputs(inp.to(DEV)), "fp64")
    assert torch.equal(X1, F2.solve(_dev(B)))
    Bd = _dev(B).contiguous()
    assert torch.equal(F.solve_noalloc_(Bd.clone()), X1)
    assert torch.equal(F.solve_noalloc_(Bd.clone(), adjoint=True), F.solve_adjoint(Bd))
    # new values through refactor: the same bits as a fresh factorization
    inp2, H2, A2 = _build("uniform_L4", seed=10)
    F.refactor(A2)
    X2 = F.solve(_dev(B))
    assert torch.equal(X2, hd.factor(A2, "fp64").solve(_dev(B)))
    assert _rel(_host(X2), O.solve(O.factor(H2), B)) < 1e-12


def test_complex_unsupported_calls():
    hd = _hd()
    inp, H, A = _build("uniform_L4")
    F = hd.factor(A, "fp64")
    X = F.solve(_dev(_rhs(H.N, 1, 2)))
    with pytest.raises(hd.HodlrError) as e:
        F.slogdet_grad()
    assert e.value.status == -4
    with pytest.raises(hd.HodlrError) as e:
        hd.factor(hd.HODLRMatrix.from_inputs(inp.to(DEV)), "fp64", inplace=True)
    assert e.value.status == -4
    big = W.synthetic(1024, 256, 4, seed=1, dtype=torch.complex128)          # leaf 256 > 128
    with pytest.raises(hd.HodlrError) as e:
        hd.factor(hd.HODLRMatrix.from_inputs(big.to(DEV)), "fp64")
    assert e.value.status == -4
    wide = W.synthetic(1024, 128, 40, seed=1, dtype=torch.complex128)        # rank 40 > 32
    with pytest.raises(hd.HodlrError) as e:
        hd.factor(hd.HODLRMatrix.from_inputs(wide.to(DEV)), "fp64")
    assert e.value.status == -4
    del X
