"""HODLR construction by cross approximation in FP64 — TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's CPU-baseline leg may use
this module; the product library never does.

What it follows:

* the matrices of Section I ("Kernel matrices": K_ij = k(y_i, y_j) for the
  Gaussian and the Matern kernel) and of Section IV-B (the Laplace
  double-layer kernel d(x, y) = n(y).(x - y) / (2 pi |x - y|^2) of eq.
  "e:laplace_int", discretized by the trapezoidal rule on a closed curve);
* Section II-B: a HODLR approximation compresses every sibling block
  A(I_a, I_b) on its own; the numerical experiments of Section IV-A compress
  them with an approximate partial-pivoted LU.  Here that is adaptive cross
  approximation with partial pivoting taken for a fixed number of steps
  (the rank of the level), which is Gaussian elimination of the block with a
  pivot row chosen from the previous cross and the pivot column chosen in
  the pivot row:
      for k = 1 .. r:
        residual row     v = A(i_k, :) - sum_{l<k} u_l(i_k) v_l
        pivot column     j_k = argmax_j |v_j|, delta = v(j_k)
        v_k = v / delta
        residual column  u_k = A(:, j_k) - sum_{l<k} v_l(j_k) u_l
        next pivot row   i_{k+1} = argmax over rows not yet used of |u_k|
  with i_1 = the block's first row, the lowest index on ties, and an
  exhausted step (delta = 0) giving u_k = v_k = 0.  Then A(I_a, I_b) is
  approximated by U_a V_b^T with U_a = [u_1 .. u_r], V_b = [v_1 .. v_r]
  (eq. "e:rank").

Entries (p != q):
  gauss      exp(-|x_p - x_q|^2 / (2 ell^2))
  matern32   (1 + s) exp(-s),  s = sqrt(3) |x_p - x_q| / ell
  laplace_dl w_q n_q . (x_p - x_q) / (2 pi |x_p - x_q|^2)
and on the diagonal the kernel's value at 0 (1 for the radial kernels; for
the double layer the smooth limit w_p kappa_p / (4 pi), kappa the
curvature) plus ``shift``.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional, Tuple

import numpy as np


@dataclasses.dataclass
class KernelSpec:
    kind: str                              # "gauss" | "matern32" | "laplace_dl"
    points: np.ndarray                     # N x dim
    ell: float = 1.0                       # length scale (radial kernels)
    shift: float = 0.0                     # added to every diagonal entry
    normals: Optional[np.ndarray] = None   # N x 2 (laplace_dl)
    weights: Optional[np.ndarray] = None   # N (laplace_dl)
    curvature: Optional[np.ndarray] = None  # N (laplace_dl)


def entries(spec: KernelSpec, p: np.ndarray, q: np.ndarray) -> np.ndarray:
    """The block A[p][:, q] from the definitions above (p, q index arrays)."""
    p = np.asarray(p, dtype=np.int64)
    q = np.asarray(q, dtype=np.int64)
    X = spec.points[p][:, None, :]
    Yq = spec.points[q][None, :, :]
    diff = X - Yq                                  # x_p - x_q
    d2 = np.sum(diff * diff, axis=2)
    same = p[:, None] == q[None, :]
    if spec.kind == "gauss":
        A = np.exp(-d2 / (2.0 * spec.ell ** 2))
        A = np.where(same, 1.0, A)
    elif spec.kind == "matern32":
        s = np.sqrt(3.0) * np.sqrt(d2) / spec.ell
        A = (1.0 + s) * np.exp(-s)
        A = np.where(same, 1.0, A)
    elif spec.kind == "laplace_dl":
        nq = spec.normals[q][None, :, :]
        num = np.sum(nq * diff, axis=2)
        with np.errstate(divide="ignore", invalid="ignore"):
            A = num / (2.0 * np.pi * d2) * spec.weights[q][None, :]
        lim = (spec.weights[p] * spec.curvature[p] / (4.0 * np.pi))[:, None]
        A = np.where(same, np.broadcast_to(lim, A.shape), A)
    else:
        raise ValueError(spec.kind)
    return np.where(same, A + spec.shift, A)


def _residual_row(entry, i, U, V, k, n):
    """A(i, :) - sum_{l<k} u_l(i) v_l."""
    return entry(np.array([i]), np.arange(n))[0] - V[:, :k] @ U[i, :k]


def _residual_col(entry, j, U, V, k, m):
    """A(:, j) - sum_{l<k} v_l(j) u_l."""
    return entry(np.arange(m), np.array([j]))[:, 0] - U[:, :k] @ V[j, :k]


def _next_row(u, used):
    """argmax over the rows not yet used of |u| (lowest index on ties)."""
    return int(np.argmax(np.where(used, -1.0, np.abs(u))))


def aca(entry: Callable[[np.ndarray, np.ndarray], np.ndarray], m: int, n: int, steps: int,
        ) -> Tuple[np.ndarray, np.ndarray, List[int], List[int]]:
    """Cross approximation with partial pivoting of an m x n block given by
    ``entry(rows, cols)`` (local indices), ``steps`` steps.  Returns U (m x
    steps), V (n x steps) with block ~= U V^T, and the pivot rows and
    columns (a zero pivot column is reported as -1)."""
    U = np.zeros((m, steps))
    V = np.zeros((n, steps))
    used = np.zeros(m, dtype=bool)
    piv_rows: List[int] = []
    piv_cols: List[int] = []
    i = 0
    for k in range(steps):
        piv_rows.append(i)
        used[i] = True
        v = _residual_row(entry, i, U, V, k, n)
        j = int(np.argmax(np.abs(v)))
        delta = v[j]
        if delta == 0.0:
            piv_cols.append(-1)
            u = np.zeros(m)
        else:
            piv_cols.append(j)
            V[:, k] = v / delta
            u = _residual_col(entry, j, U, V, k, m)
            U[:, k] = u
        i = _next_row(u, used)
    return U, V, piv_rows, piv_cols


def node_ranges(offsets: np.ndarray, level: int):
    """Index ranges of the 2^level nodes of a level (leaf boundaries given)."""
    L = int(round(np.log2(len(offsets) - 1)))
    per = 1 << (L - level)
    return [(int(offsets[i * per]), int(offsets[(i + 1) * per])) for i in range(1 << level)]


def build(spec: KernelSpec, offsets: np.ndarray, ranks: List[int]):
    """D (N x m_max), U, V (N x R) of the HODLR approximation: exact leaf
    blocks, and for every node a of level l with sibling b the block
    A(I_a, I_b) by ``aca`` with r_l steps, U_a into the rows I_a and V_b into
    the rows I_b of the level's columns."""
    offsets = np.asarray(offsets, dtype=np.int64)
    N = int(offsets[-1])
    L = len(ranks)
    sizes = np.diff(offsets)
    m_max = int(sizes.max())
    D = np.zeros((N, m_max))
    for a in range(1 << L):
        s0, e0 = int(offsets[a]), int(offsets[a + 1])
        idx = np.arange(s0, e0)
        D[s0:e0, :e0 - s0] = entries(spec, idx, idx)
    R = int(sum(ranks))
    U = np.zeros((N, R))
    V = np.zeros((N, R))
    c0 = 0
    for lvl in range(1, L + 1):
        r = int(ranks[lvl - 1])
        nodes = node_ranges(offsets, lvl)
        for a, (s0, e0) in enumerate(nodes):
            t0, f0 = nodes[a ^ 1]
            Ua, Vb, _, _ = aca(lambda ri, cj: entries(spec, s0 + ri, t0 + cj), e0 - s0, f0 - t0, r)
            U[s0:e0, c0:c0 + r] = Ua
            V[t0:f0, c0:c0 + r] = Vb
        c0 += r
    return D, U, V


def dense(spec: KernelSpec, N: int) -> np.ndarray:
    """The whole N x N matrix from the definitions (small N only)."""
    idx = np.arange(N)
    return entries(spec, idx, idx)
