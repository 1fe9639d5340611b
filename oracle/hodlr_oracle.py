"""Plain recursive HODLR factor/solve in FP64 — TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's CPU-baseline leg may use
this module; the product library never does.

What it follows (Chen & Martinsson, "Solving linear systems on a GPU with
hierarchically off-diagonal low-rank approximations"):

* cluster tree / tessellation: Definition "Cluster tree" and the HODLR
  tessellation of Section II-A (leaves give diagonal blocks, sibling pairs
  give off-diagonal blocks);
* generators: A(I_a, I_b) = U_a V_b^* for siblings a, b (eq. "e:rank"), V^*
  the conjugate transpose (V^T for real matrices; complex matrices, the
  field F = C of the paper, take the same recursion with V^*);
* recursion (Section III-A): solve A_a [z_a | Y_a] = [b_a | U_a] on each
  child (eq. "e:recursion"), then the coupling system with
  K = [[V_a^T Y_a, I], [I, V_b^T Y_b]] (eqs. "e:node", "e:k"), then
  x = z - Y w (eq. "e:solution"); correctness is Theorem "Correctness of
  recursion"; factorization = everything independent of b (Y's and LU of K);
* leaves are factored by LU with partial pivoting (LAPACK getrf via SciPy).

The matrix is given as plain logical arrays (no device layout):
``D`` (N x m_max, leaf block a = D[o:o+m, :m]), ``U``/``V`` (N x R, level l in
columns [R_{l-1}, R_l)).
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional

import numpy as np
import scipy.linalg as sla


@dataclasses.dataclass
class Hodlr:
    offsets: np.ndarray   # int64, 2**L + 1 leaf boundaries
    ranks: List[int]      # r_1 .. r_L
    D: np.ndarray         # N x m_max
    U: np.ndarray         # N x R
    V: np.ndarray         # N x R

    @property
    def L(self) -> int:
        return len(self.ranks)

    @property
    def N(self) -> int:
        return int(self.offsets[-1])

    def colrange(self, level: int):
        """Columns of U_big / V_big that hold the level-`level` generators."""
        c0 = int(sum(self.ranks[:level - 1]))
        return c0, c0 + int(self.ranks[level - 1])

    def astype(self, dt) -> "Hodlr":
        return Hodlr(self.offsets, list(self.ranks), self.D.astype(dt), self.U.astype(dt), self.V.astype(dt))


def from_inputs(inp) -> Hodlr:
    """Build from a ``workloads.HodlrInputs`` (copies to host float64)."""
    off, ranks, D, U, V = inp.numpy64()
    return Hodlr(np.asarray(off, np.int64), list(ranks), np.ascontiguousarray(D),
                 np.ascontiguousarray(U), np.ascontiguousarray(V))


def node_range(H: Hodlr, level: int, i: int):
    """Half-open row range [start, stop) of node i at `level` (0-based, left to right).

    A level-`level` node is the union of 2**(L-level) consecutive leaves.
    """
    per = 1 << (H.L - level)
    return int(H.offsets[i * per]), int(H.offsets[(i + 1) * per])


def _adj(M: np.ndarray) -> np.ndarray:
    """M^* (the transpose for real M)."""
    return M.conj().T


def _gen(H: Hodlr, which: str, level: int, i: int) -> np.ndarray:
    s, e = node_range(H, level, i)
    c0, c1 = H.colrange(level)
    M = H.U if which == "U" else H.V
    return M[s:e, c0:c1]


def _leaf(H: Hodlr, i: int) -> np.ndarray:
    s, e = node_range(H, H.L, i)
    return H.D[s:e, :e - s]


def assemble_dense(H: Hodlr) -> np.ndarray:
    """The plain definition: leaves on the diagonal, U_a V_b^* on sibling blocks."""
    N = H.N
    A = np.zeros((N, N), dtype=H.D.dtype)
    for i in range(1 << H.L):
        s, e = node_range(H, H.L, i)
        A[s:e, s:e] = _leaf(H, i)
    for level in range(1, H.L + 1):
        for p in range(1 << (level - 1)):
            a, b = 2 * p, 2 * p + 1
            sa, ea = node_range(H, level, a)
            sb, eb = node_range(H, level, b)
            A[sa:ea, sb:eb] = _gen(H, "U", level, a) @ _adj(_gen(H, "V", level, b))
            A[sb:eb, sa:ea] = _gen(H, "U", level, b) @ _adj(_gen(H, "V", level, a))
    return A


# ---------------------------------------------------------------------------
# recursion (Section III-A)
# ---------------------------------------------------------------------------

def _coupling_matrix(Va, Ya, Vb, Yb):
    """K = [[V_a^* Y_a, I], [I, V_b^* Y_b]]  (eq. "e:k")."""
    r = Ya.shape[1]
    I = np.eye(r, dtype=Ya.dtype)
    return np.block([[_adj(Va) @ Ya, I], [I, _adj(Vb) @ Yb]])


def _combine(Za, Zb, Ya, Yb, W):
    """x = z - Y w on both children (eq. "e:solution")."""
    r = Ya.shape[1]
    return np.vstack([Za - Ya @ W[:r], Zb - Yb @ W[r:]])


def _factor(H: Hodlr, level: int, i: int) -> dict:
    if level == H.L:
        D = _leaf(H, i)
        lu, piv = sla.lu_factor(D, check_finite=True)
        if np.any(np.diag(lu) == 0):
            raise np.linalg.LinAlgError(f"singular leaf {i}")
        return dict(leaf=True, lu=(lu, piv), level=level, i=i)
    a, b = 2 * i, 2 * i + 1
    Fa = _factor(H, level + 1, a)
    Fb = _factor(H, level + 1, b)
    Ua, Ub = _gen(H, "U", level + 1, a), _gen(H, "U", level + 1, b)
    Va, Vb = _gen(H, "V", level + 1, a), _gen(H, "V", level + 1, b)
    Ya = _solve(Fa, Ua)          # A_a Y_a = U_a  (eq. "e:recursion")
    Yb = _solve(Fb, Ub)
    node = dict(leaf=False, a=Fa, b=Fb, Ya=Ya, Yb=Yb, Va=Va, Vb=Vb, level=level, i=i,
                na=Ua.shape[0], Klu=None)
    if Ya.shape[1]:
        K = _coupling_matrix(Va, Ya, Vb, Yb)
        lu, piv = sla.lu_factor(K)
        if np.any(np.diag(lu) == 0):
            raise np.linalg.LinAlgError(f"singular coupling matrix at level {level} node {i}")
        node["Klu"] = (lu, piv)
    return node


def _solve(F: dict, B: np.ndarray) -> np.ndarray:
    if F["leaf"]:
        return sla.lu_solve(F["lu"], B)
    na = F["na"]
    Za = _solve(F["a"], B[:na])
    Zb = _solve(F["b"], B[na:])
    if F["Klu"] is None:
        return np.vstack([Za, Zb])
    rhs = np.vstack([_adj(F["Va"]) @ Za, _adj(F["Vb"]) @ Zb])   # right side of eq. "e:node"
    W = sla.lu_solve(F["Klu"], rhs)
    return _combine(Za, Zb, F["Ya"], F["Yb"], W)


def factor(H: Hodlr) -> dict:
    """Factorization stage: every Y_a = A_a^{-1} U_a, the leaf LUs and the LU of every K."""
    F = _factor(H, 0, 0)
    F["H"] = H
    return F


def solve(F: dict, B: np.ndarray) -> np.ndarray:
    """Solution stage: x = A^{-1} B (B is N or N x k)."""
    vec = B.ndim == 1
    X = _solve(F, B.reshape(B.shape[0], -1))
    return X[:, 0] if vec else X


def y_big(F: dict) -> np.ndarray:
    """The N x R matrix whose level-l columns at rows I_a hold Y_a = A_a^{-1} U_a."""
    H = F["H"]
    Y = np.zeros_like(H.U)

    def walk(node):
        if node["leaf"]:
            return
        lvl = node["level"] + 1
        c0, c1 = H.colrange(lvl)
        sa, ea = node_range(H, lvl, 2 * node["i"])
        sb, eb = node_range(H, lvl, 2 * node["i"] + 1)
        Y[sa:ea, c0:c1] = node["Ya"]
        Y[sb:eb, c0:c1] = node["Yb"]
        walk(node["a"])
        walk(node["b"])

    walk(F)
    return Y


def _lu_slogdet(lu_piv):
    """(sign, log|det|) of a matrix from its LAPACK LU: the product of U's
    diagonal, with one sign change per row interchange."""
    lu, piv = lu_piv
    d = np.diag(lu)
    swaps = int(np.sum(piv != np.arange(len(piv))))
    sign = (-1.0) ** swaps * float(np.prod(np.sign(d)))
    return sign, float(np.sum(np.log(np.abs(d))))


def slogdet(F: dict):
    """(sign, log|det A|) from the factorization (the appendix's product form
    A = A^(L+1) A^(L) ... A^(1): leaf blocks, then per level block-diagonal
    2x2 factors [[I, Y_a V_b^T], [Y_b V_a^T, I]]).  By Sylvester's determinant
    theorem each 2x2 factor has the determinant of [[I, T_b], [T_a, I]] with
    T = V^T Y, which is K = [[T_a, I], [I, T_b]] with its two r-row blocks
    swapped: det = (-1)^r det K."""
    sign, logabs = 1.0, 0.0

    def walk(node):
        nonlocal sign, logabs
        if node["leaf"]:
            sg, la = _lu_slogdet(node["lu"])
            sign *= sg
            logabs += la
            return
        walk(node["a"])
        walk(node["b"])
        if node["Klu"] is not None:
            r = node["Ya"].shape[1]
            sg, la = _lu_slogdet(node["Klu"])
            sign *= sg * (-1.0) ** r
            logabs += la

    walk(F)
    return sign, logabs


# ---------------------------------------------------------------------------
# transpose, adjoint, matvec, gradients
# ---------------------------------------------------------------------------

def transpose(H: Hodlr) -> Hodlr:
    """A^* (A^T for real matrices) is HODLR on the same tree: leaf blocks
    conjugate-transposed and U <-> V, because
    A^*(I_a, I_b) = (U_b V_a^*)^* = V_a U_b^*."""
    Dt = np.zeros_like(H.D)
    for i in range(1 << H.L):
        s, e = node_range(H, H.L, i)
        Dt[s:e, :e - s] = _adj(H.D[s:e, :e - s])
    return Hodlr(H.offsets, list(H.ranks), Dt, H.V.copy(), H.U.copy())


def solve_adjoint(H: Hodlr, G: np.ndarray) -> np.ndarray:
    """lambda = A^{-T} G (A^{-*} G for complex A), by factoring the transposed
    HODLR matrix independently."""
    return solve(factor(transpose(H)), G)


def matvec(H: Hodlr, X: np.ndarray, trans: bool = False) -> np.ndarray:
    """Y = A X (or A^T X; A^* X for complex A) block by block, without assembling A."""
    if trans:
        H = transpose(H)
    vec = X.ndim == 1
    X2 = X.reshape(X.shape[0], -1)
    Y = np.zeros_like(X2, dtype=np.result_type(H.D.dtype, X2.dtype))
    for i in range(1 << H.L):
        s, e = node_range(H, H.L, i)
        Y[s:e] += _leaf(H, i) @ X2[s:e]
    for level in range(1, H.L + 1):
        for p in range(1 << (level - 1)):
            a, b = 2 * p, 2 * p + 1
            sa, ea = node_range(H, level, a)
            sb, eb = node_range(H, level, b)
            Y[sa:ea] += _gen(H, "U", level, a) @ (_adj(_gen(H, "V", level, b)) @ X2[sb:eb])
            Y[sb:eb] += _gen(H, "U", level, b) @ (_adj(_gen(H, "V", level, a)) @ X2[sa:ea])
    return Y[:, 0] if vec else Y


def grad_structured(H: Hodlr, X: np.ndarray, Lam: np.ndarray):
    """dL/dA = -Lam X^T restricted to the HODLR parameters.

    With A(I_a, I_b) = U_a V_b^T the chain rule gives
    dD_a = -Lam_a X_a^T,  dU_a = -Lam_a X_b^T V_b,  dV_b = -X_b Lam_a^T U_a.
    Returns (dD, dU, dV) in the layouts of D, U, V.
    """
    X = X.reshape(X.shape[0], -1)
    Lam = Lam.reshape(Lam.shape[0], -1)
    dD = np.zeros_like(H.D)
    dU = np.zeros_like(H.U)
    dV = np.zeros_like(H.V)
    for i in range(1 << H.L):
        s, e = node_range(H, H.L, i)
        dD[s:e, :e - s] = -Lam[s:e] @ X[s:e].T
    for level in range(1, H.L + 1):
        c0, c1 = H.colrange(level)
        for p in range(1 << (level - 1)):
            for a, b in ((2 * p, 2 * p + 1), (2 * p + 1, 2 * p)):
                sa, ea = node_range(H, level, a)
                sb, eb = node_range(H, level, b)
                Vb = H.V[sb:eb, c0:c1]
                Ua = H.U[sa:ea, c0:c1]
                dU[sa:ea, c0:c1] = -Lam[sa:ea] @ (X[sb:eb].T @ Vb)
                dV[sb:eb, c0:c1] = -X[sb:eb] @ (Lam[sa:ea].T @ Ua)
    return dD, dU, dV


def logdet_grad_structured(H: Hodlr):
    """Gradient of log|det A| with respect to the HODLR parameters D, U, V.

    Jacobi's formula gives d log|det A| = trace(A^{-1} dA), so the gradient
    with respect to the entries of A is A^{-T}; restricted to the parameters
    through A(I_a, I_a) = D_a and A(I_a, I_b) = U_a V_b^T (as in
    grad_structured with -Lam X^T replaced by G = A^{-T}):
    dD_a = G_aa,  dU_a = G_ab V_b,  dV_b = G_ab^T U_a.  Dense: small N only.
    """
    G = np.linalg.inv(assemble_dense(H)).T
    dD = np.zeros_like(H.D)
    dU = np.zeros_like(H.U)
    dV = np.zeros_like(H.V)
    for i in range(1 << H.L):
        s, e = node_range(H, H.L, i)
        dD[s:e, :e - s] = G[s:e, s:e]
    for level in range(1, H.L + 1):
        c0, c1 = H.colrange(level)
        for p in range(1 << (level - 1)):
            for a, b in ((2 * p, 2 * p + 1), (2 * p + 1, 2 * p)):
                sa, ea = node_range(H, level, a)
                sb, eb = node_range(H, level, b)
                dU[sa:ea, c0:c1] = G[sa:ea, sb:eb] @ H.V[sb:eb, c0:c1]
                dV[sb:eb, c0:c1] = G[sa:ea, sb:eb].T @ H.U[sa:ea, c0:c1]
    return dD, dU, dV


def loss_and_grads(H: Hodlr, b: np.ndarray, t: np.ndarray):
    """L = ||x - t||_F^2 with x = A^{-1} b.  Returns (L, x, dL/db, dD, dU, dV)."""
    F = factor(H)
    x = solve(F, b)
    G = 2.0 * (x - t)
    lam = solve_adjoint(H, G)
    dD, dU, dV = grad_structured(H, x, lam)
    return float(np.sum((x - t) ** 2)), x, lam, dD, dU, dV


# ---------------------------------------------------------------------------
# mixed-precision iterative refinement
# ---------------------------------------------------------------------------

def relres(H: Hodlr, X: np.ndarray, B: np.ndarray) -> float:
    """max over columns of ||b - A x||_2 / ||b||_2 with A the HODLR matrix itself."""
    Rm = B.reshape(B.shape[0], -1) - matvec(H, X.reshape(X.shape[0], -1))
    nb = np.linalg.norm(B.reshape(B.shape[0], -1), axis=0)
    return float(np.max(np.linalg.norm(Rm, axis=0) / np.where(nb > 0, nb, 1.0)))


def _round_bf16(a: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), kept in float32."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def low_precision_solver(H: Hodlr, precision: str) -> Callable[[np.ndarray], np.ndarray]:
    """A solver for A built entirely in float32 arithmetic ('fp32'), or in float32
    on inputs rounded to bfloat16 ('bf16').  Used to emulate a low-precision
    factorization for refinement tests."""
    Hl = H.astype(np.float32)
    if precision == "bf16":
        Hl = Hodlr(Hl.offsets, Hl.ranks, _round_bf16(Hl.D), _round_bf16(Hl.U), _round_bf16(Hl.V))
    elif precision != "fp32":
        raise ValueError(precision)
    Fl = factor(Hl)
    return lambda Rhs: solve(Fl, Rhs.astype(np.float32)).astype(np.float64)


def refine(H: Hodlr, low_solve: Callable[[np.ndarray], np.ndarray], B: np.ndarray,
           tol: float = 1e-10, max_iter: int = 30):
    """FP64 iterative refinement around a low-precision solver.

    x_0 = 0, r_0 = b.  Each step scales r by its per-column max-norm s, solves
    in low precision, adds s * d to x in FP64 and recomputes r = b - A x with
    an FP64 matvec.  Stops when max_col ||r||/||b|| <= tol; fails when
    max_iter steps pass or the residual grows on two consecutive steps.
    Returns (x, iterations, relres, converged).
    """
    B2 = B.reshape(B.shape[0], -1).astype(np.float64)
    X = np.zeros_like(B2)
    Rm = B2.copy()
    nb = np.linalg.norm(B2, axis=0)
    nb = np.where(nb > 0, nb, 1.0)
    prev = np.inf
    grow = 0
    it = 0
    res = float(np.max(np.linalg.norm(Rm, axis=0) / nb))
    while res > tol and it < max_iter:
        s = np.max(np.abs(Rm), axis=0)
        s = np.where(s > 0, s, 1.0)
        Dx = low_solve(Rm / s) * s
        X = X + Dx
        Rm = B2 - matvec(H, X)
        it += 1
        res = float(np.max(np.linalg.norm(Rm, axis=0) / nb))
        grow = grow + 1 if res > prev else 0
        prev = res
        if grow >= 2:
            break
    Xo = X[:, 0] if B.ndim == 1 else X
    return Xo, it, res, res <= tol
