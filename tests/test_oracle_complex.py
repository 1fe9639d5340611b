"""Pins of the oracle on complex HODLR matrices (the field F = C of the
paper; A(I_a, I_b) = U_a V_b^*, eq. "e:rank").

The independent route is the real embedding: a complex entry p + i q becomes
the real 2x2 block [[p, -q], [q, p]] and index i the rows 2i, 2i+1.  The
embedding maps products to products and M^* to emb(M)^T, so the embedded
matrix is a real HODLR matrix on the same tree (leaf sizes and ranks
doubled, U~ = emb(U), V~ = emb(V)).  Its solution by the real recursion,
which the real pins tie to LAPACK, read back as complex numbers, must equal
the complex oracle's solution.  Dense LAPACK solves of the assembled complex
matrix are a second check."""
import numpy as np
import pytest
import torch

import oracle as O
import oracle.hodlr_oracle as OH
import workloads as W


def _emb(M: np.ndarray) -> np.ndarray:
    """Real embedding of a complex matrix, interleaved (entry (i, j) -> rows 2i, 2i+1, cols 2j, 2j+1)."""
    m, n = M.shape
    E = np.zeros((2 * m, 2 * n))
    E[0::2, 0::2] = M.real
    E[0::2, 1::2] = -M.imag
    E[1::2, 0::2] = M.imag
    E[1::2, 1::2] = M.real
    return E


def _embed_hodlr(H: O.Hodlr) -> O.Hodlr:
    D = np.zeros((2 * H.N, 2 * H.D.shape[1]))
    for i in range(1 << H.L):
        s, e = O.node_range(H, H.L, i)
        D[2 * s:2 * e, :2 * (e - s)] = _emb(H.D[s:e, :e - s])
    return O.Hodlr(2 * H.offsets, [2 * r for r in H.ranks], D, _emb(H.U), _emb(H.V))


def _interleave(X: np.ndarray) -> np.ndarray:
    R = np.zeros((2 * X.shape[0], X.shape[1]))
    R[0::2], R[1::2] = X.real, X.imag
    return R


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
}


def _build(name, seed=0):
    c = CASES[name]
    off = _offsets(c["n"], c["L"], seed + 3) if "L" in c else None
    inp = W.synthetic(c["n"], c.get("leaf", 0), c["ranks"], seed=seed, leaf_offsets=off, dtype=torch.complex128)
    return O.from_inputs(inp)


def _rhs(n, k, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k))


def test_embedding_is_a_real_hodlr_of_the_embedded_matrix():
    H = _build("uniform_L4")
    A = O.assemble_dense(H)
    assert np.iscomplexobj(A) and np.abs(A.imag).max() > 0.1
    assert np.allclose(O.assemble_dense(_embed_hodlr(H)), _emb(A), rtol=0, atol=1e-13)


@pytest.mark.parametrize("name", list(CASES))
def test_complex_solve_matches_real_embedding_and_dense(name):
    H = _build(name)
    B = _rhs(H.N, 3, 1)
    X = O.solve(O.factor(H), B)
    Xr = O.solve(O.factor(_embed_hodlr(H)), _interleave(B))
    assert np.linalg.norm(_interleave(X) - Xr) <= 1e-12 * np.linalg.norm(Xr)
    Xd = np.linalg.solve(O.assemble_dense(H), B)
    assert np.linalg.norm(X - Xd) <= 1e-12 * np.linalg.norm(Xd)


@pytest.mark.parametrize("name", list(CASES))
def test_complex_adjoint_is_the_conjugate_transpose_inverse(name):
    """solve_adjoint gives A^{-*} G: through the embedding that is the
    inverse transpose of the real embedded matrix."""
    H = _build(name, seed=2)
    G = _rhs(H.N, 2, 5)
    Lam = O.solve_adjoint(H, G)
    Lr = O.solve_adjoint(_embed_hodlr(H), _interleave(G))
    assert np.linalg.norm(_interleave(Lam) - Lr) <= 1e-12 * np.linalg.norm(Lr)
    # <A x, g> = <x, A^* g> with the conjugate-linear inner product
    x = _rhs(H.N, 1, 6)[:, 0]
    g = _rhs(H.N, 1, 7)[:, 0]
    lhs = np.vdot(O.matvec(H, x), g)
    rhs = np.vdot(x, O.matvec(H, g, trans=True))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_complex_matvec_matches_the_embedding():
    H = _build("ragged_L3_rank0", seed=4)
    X = _rhs(H.N, 2, 8)
    Y = O.matvec(H, X)
    Yr = O.matvec(_embed_hodlr(H), _interleave(X))
    assert np.linalg.norm(_interleave(Y) - Yr) <= 1e-13 * np.linalg.norm(Yr)


def test_planted_missing_conjugate_fails(monkeypatch):
    """V^T in place of V^* everywhere in the oracle (a consistent mistake the
    dense check alone would not see) breaks the embedding pin."""
    H = _build("uniform_L4", seed=9)
    B = _rhs(H.N, 2, 10)
    Xr = O.solve(O.factor(_embed_hodlr(H)), _interleave(B))
    monkeypatch.setattr(OH, "_adj", lambda M: M.T)
    X = O.solve(O.factor(H), B)
    assert np.linalg.norm(_interleave(X) - Xr) > 1e-6 * np.linalg.norm(Xr)


def test_helmholtz_workload_is_complex_symmetric_and_close_to_its_kernel():
    """The Helmholtz-style workload: A^T = A exactly (U_b = conj(V_b),
    V_a = conj(U_a)), and the HODLR approximant close to the kernel matrix."""
    n = 1024
    inp = W.helmholtz_matrix(n, 64, 16, kappa=20.0)
    A = O.assemble_dense(O.from_inputs(inp))
    assert np.array_equal(A, A.T)
    P = W.kernel_points(n, 3, 64, 0)
    d = np.sqrt(((P[:, None, :] - P[None, :, :]) ** 2).sum(-1))
    np.fill_diagonal(d, 1.0)
    G = (4.0 / n) * np.exp(1j * 20.0 * d) / (4 * np.pi * d)
    np.fill_diagonal(G, 1.0)
    assert np.linalg.norm(A - G) <= 2e-2 * np.linalg.norm(G)
