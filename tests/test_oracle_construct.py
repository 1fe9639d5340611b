"""Pins of the construction oracle (cross approximation of the sibling blocks
and the kernel entries) against facts that do not come from the oracle:
closed-form kernel values, Gauss's lemma for the double layer, the skeleton
(CUR) form that Gaussian elimination with the same pivots gives, the cross
interpolation property, exact recovery of exactly low-rank blocks, and the
pivot rules on hand-made blocks."""
import math

import numpy as np
import pytest

import oracle as O
import oracle.construct as OC
import workloads as W


def _curve_spec(n, shift=0.0):
    g = W.star_curve(n)
    return O.KernelSpec("laplace_dl", g["points"].numpy(), shift=shift, normals=g["normals"].numpy(),
                        weights=g["weights"].numpy(), curvature=g["curvature"].numpy())


def _circle_spec(n, rho):
    t = 2 * np.pi * np.arange(n) / n
    pts = rho * np.stack([np.cos(t), np.sin(t)], 1)
    return O.KernelSpec("laplace_dl", pts, normals=-pts / rho, weights=np.full(n, 2 * np.pi * rho / n),
                        curvature=np.full(n, 1.0 / rho))


# --------------------------------------------------------------------------- entries

def test_radial_kernel_closed_values():
    ell = 0.3
    pts = np.array([[0.0, 0.0], [ell, 0.0], [0.0, 2 * ell]])
    g = O.kernel_entries(O.KernelSpec("gauss", pts, ell=ell, shift=0.25), np.arange(3), np.arange(3))
    assert g[0, 1] == pytest.approx(math.exp(-0.5), rel=1e-15)
    assert g[0, 2] == pytest.approx(math.exp(-2.0), rel=1e-15)
    assert np.allclose(np.diag(g), 1.25, rtol=0, atol=0) and np.array_equal(g, g.T)
    m = O.kernel_entries(O.KernelSpec("matern32", pts, ell=ell), np.arange(3), np.arange(3))
    s3 = math.sqrt(3.0)
    assert m[0, 1] == pytest.approx((1 + s3) * math.exp(-s3), rel=1e-15)
    assert m[1, 2] == pytest.approx((1 + s3 * math.sqrt(5)) * math.exp(-s3 * math.sqrt(5)), rel=1e-14)
    assert np.all(np.diag(m) == 1.0) and np.array_equal(m, m.T)


def test_double_layer_on_a_circle_is_constant():
    """On a circle of radius rho with the inward normal, n(y).(x-y) /
    (2 pi |x-y|^2) = 1/(4 pi rho) for every x != y, and the curvature limit
    on the diagonal is the same constant."""
    rho, n = 1.7, 64
    A = O.kernel_dense(_circle_spec(n, rho), n)
    w = 2 * np.pi * rho / n
    assert np.allclose(A, w / (4 * np.pi * rho), rtol=1e-13, atol=0)


@pytest.mark.parametrize("n", [256, 1024])
def test_double_layer_gauss_lemma_on_the_star(n):
    """Gauss's lemma: the double layer of the constant density is 1/2 on the
    curve (inward normal); the trapezoidal rule with the curvature limit on
    the diagonal is spectrally accurate for the smooth star curve."""
    A = O.kernel_dense(_curve_spec(n), n)
    assert np.max(np.abs(A.sum(1) - 0.5)) < 1e-10
    # with the second-kind shift 1/2 the constant is an eigenvector of eigenvalue 1
    A2 = O.kernel_dense(_curve_spec(n, shift=0.5), n)
    assert np.max(np.abs(A2.sum(1) - 1.0)) < 1e-10


# --------------------------------------------------------------------------- cross approximation

def _cauchy_block(m, n, seed):
    """1/(x_i - y_j + 3) with x, y in [0, 1]: smooth, numerically low rank."""
    rng = np.random.default_rng(seed)
    x, y = rng.random(m), rng.random(n)
    M = 1.0 / (x[:, None] - y[None, :] + 3.0)
    return M, lambda ri, cj: M[np.ix_(ri, cj)]


@pytest.mark.parametrize("k", [1, 3, 6])
def test_aca_equals_skeleton_form(k):
    """k steps of cross approximation equal Gaussian elimination with the
    same pivots: U V^T = M(:, J) M(I, J)^{-1} M(I, :)."""
    M, ent = _cauchy_block(40, 35, 1)
    U, V, I, J = O.aca(ent, 40, 35, k)
    assert len(set(I)) == k and min(J) >= 0
    S = M[:, J] @ np.linalg.solve(M[np.ix_(I, J)], M[I, :])
    assert np.linalg.norm(U @ V.T - S) <= 1e-12 * np.linalg.norm(M)


def test_aca_interpolates_its_crosses():
    M, ent = _cauchy_block(50, 60, 2)
    U, V, I, J = O.aca(ent, 50, 60, 5)
    R = M - U @ V.T
    assert np.max(np.abs(R[I, :])) < 1e-13 and np.max(np.abs(R[:, J])) < 1e-13
    # the error drops with the steps (smooth kernel)
    errs = []
    for s in (1, 2, 4, 8):
        Us, Vs, _, _ = O.aca(ent, 50, 60, s)
        errs.append(np.linalg.norm(M - Us @ Vs.T))
    assert all(b < a for a, b in zip(errs, errs[1:])) and errs[-1] < 1e-9 * np.linalg.norm(M)


def test_aca_recovers_an_exactly_low_rank_block():
    """(1 + x.y)^2 in 2-D spans the six monomials of degree <= 2: six steps
    reproduce the block; a rank-1 integer block is exhausted after one step
    (its residual is exactly zero), giving zero further columns."""
    rng = np.random.default_rng(3)
    X, Y = rng.random((30, 2)), rng.random((25, 2))
    M = (1.0 + X @ Y.T) ** 2
    U, V, I, J = O.aca(lambda ri, cj: M[np.ix_(ri, cj)], 30, 25, 6)
    assert np.linalg.norm(M - U @ V.T) <= 1e-12 * np.linalg.norm(M)
    a = np.array([1.0, -2.0, 3.0, 4.0])
    b = np.array([2.0, 1.0, -1.0])
    M1 = np.outer(a, b)
    U, V, I, J = O.aca(lambda ri, cj: M1[np.ix_(ri, cj)], 4, 3, 3)
    assert np.array_equal(U @ V.T, M1)
    assert J[1:] == [-1, -1] and not U[:, 1:].any() and not V[:, 1:].any()
    # after the exhausted steps the unused rows are taken in index order
    assert I == [0, 3, 1]


def test_aca_pivot_rules_on_a_hand_block():
    """First pivot row 0; the column of largest modulus in it, the lowest on
    ties; the next row the largest modulus of the new column among the rows
    not used yet."""
    M = np.array([[1.0, -2.0, 2.0],
                  [0.5, 1.0, 0.0],
                  [4.0, 0.0, 1.0],
                  [-3.0, 9.0, 0.0]])
    U, V, I, J = O.aca(lambda ri, cj: M[np.ix_(ri, cj)], 4, 3, 2)
    assert I[0] == 0 and J[0] == 1              # |-2| = |2|: lowest index
    # column 1 of M is [-2, 1, 0, 9]: row 3 is next
    assert I[1] == 3
    # residual row 3: [-3, 9, 0] - u(3) v with v = M[0]/(-2), u(3) = 9
    v = M[0] / -2.0
    r3 = M[3] - 9.0 * v
    assert J[1] == int(np.argmax(np.abs(r3)))
    assert np.allclose(V[:, 0], v) and np.allclose(U[:, 0], M[:, 1])


@pytest.mark.parametrize("mistake", ["row_sign", "col_dropped_term", "next_row_reuses"])
def test_planted_aca_mistakes_fail(monkeypatch, mistake):
    """A flipped sign in the residual row, a dropped term in the residual
    column, or a pivot row chosen again each break the skeleton pin."""
    if mistake == "row_sign":
        monkeypatch.setattr(OC, "_residual_row",
                            lambda e, i, U, V, k, n: e(np.array([i]), np.arange(n))[0] + V[:, :k] @ U[i, :k])
    elif mistake == "col_dropped_term":
        monkeypatch.setattr(OC, "_residual_col",
                            lambda e, j, U, V, k, m: e(np.arange(m), np.array([j]))[:, 0]
                            - U[:, :max(k - 1, 0)] @ V[j, :max(k - 1, 0)])
    else:
        monkeypatch.setattr(OC, "_next_row", lambda u, used: int(np.argmax(np.abs(u))))
    M, ent = _cauchy_block(40, 35, 1)
    U, V, I, J = O.aca(ent, 40, 35, 4)
    ok = len(set(I)) == 4 and len(set(J)) == 4 and min(J) >= 0
    if ok:
        try:
            S = M[:, J] @ np.linalg.solve(M[np.ix_(I, J)], M[I, :])
            ok = np.linalg.norm(U @ V.T - S) <= 1e-12 * np.linalg.norm(M)
        except np.linalg.LinAlgError:
            ok = False
    assert not ok


# --------------------------------------------------------------------------- whole construction

def _assembled_blocks_are_skeletons(spec, off, ranks, Ah, A):
    """Every sibling block of the assembled matrix is the skeleton form of
    the exact block with the pivots its cross approximation chose."""
    for lvl in range(1, len(ranks) + 1):
        nodes = OC.node_ranges(off, lvl)
        for a, (s0, e0) in enumerate(nodes):
            t0, f0 = nodes[a ^ 1]
            M = A[s0:e0, t0:f0]
            _, _, I, J = O.aca(lambda ri, cj: M[np.ix_(ri, cj)], e0 - s0, f0 - t0, ranks[lvl - 1])
            S = M[:, J] @ np.linalg.solve(M[np.ix_(I, J)], M[I, :])
            assert np.linalg.norm(Ah[s0:e0, t0:f0] - S) <= 1e-10 * np.linalg.norm(M), (lvl, a)


def test_construction_of_the_double_layer_matrix():
    """Exact leaf blocks, skeleton sibling blocks, and an error that falls
    with the rank (star-curve double layer with the 1/2 shift, halving tree)."""
    n, L = 1024, 4
    spec = _curve_spec(n, shift=0.5)
    off = W.uniform_offsets(n, L)
    A = O.kernel_dense(spec, n)
    errs = []
    for r in (4, 8, 16):
        D, U, V = O.construct_hodlr(spec, off, [r] * L)
        Ah = O.assemble_dense(O.Hodlr(off, [r] * L, D, U, V))
        for a in range(1 << L):
            s0, e0 = int(off[a]), int(off[a + 1])
            assert np.array_equal(Ah[s0:e0, s0:e0], A[s0:e0, s0:e0])
        if r == 8:
            _assembled_blocks_are_skeletons(spec, off, [r] * L, Ah, A)
        errs.append(np.linalg.norm(Ah - A) / np.linalg.norm(A))
    assert errs[0] > errs[1] > errs[2]


@pytest.mark.parametrize("kind,dim,ell", [("gauss", 2, 0.2), ("matern32", 3, 0.1)])
def test_construction_of_kernel_matrices(kind, dim, ell):
    n, L = 1024, 3
    spec = O.KernelSpec(kind, W.kernel_points(n, dim, n >> L, seed=4), ell=ell, shift=1e-2)
    off = W.uniform_offsets(n, L)
    A = O.kernel_dense(spec, n)
    errs = []
    for r in (4, 12):
        D, U, V = O.construct_hodlr(spec, off, [r] * L)
        Ah = O.assemble_dense(O.Hodlr(off, [r] * L, D, U, V))
        if r == 4:
            _assembled_blocks_are_skeletons(spec, off, [r] * L, Ah, A)
        errs.append(np.linalg.norm(Ah - A) / np.linalg.norm(A))
    assert errs[1] < errs[0]
