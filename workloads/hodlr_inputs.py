"""Seeded input generators for the five HODLR workloads.

Storage convention (shared with the C ABI): every matrix is column-major and
is held in a torch tensor whose *row-major* shape is the transpose, i.e.

* ``D`` — tensor ``(m_max, N)``: the N x m_max stack of leaf blocks (the
  paper's D_big of the data-structure section, Fig. "f:dk"); leaf alpha with
  rows ``[o, o+m)`` is ``D[:m, o:o+m].T``.
* ``U``, ``V`` — tensors ``(R, N)``: the N x R concatenations U_big and
  V_big (Fig. "f:cat", eq. "e:u"); level l occupies columns
  ``[R_{l-1}, R_l)`` with ``R_l = r_1 + ... + r_l``.  Rows of a node are its
  index set; ranks vary per level and are left-aligned.

Cluster-tree nodes are consecutive index sets (Definition "Cluster tree");
level l has 2**l nodes, node i at level l spans leaves
``[i*2**(L-l), (i+1)*2**(L-l))``.  The off-diagonal block between siblings
alpha, beta is ``U_alpha V_beta^T`` (eq. "e:rank").

Randomness comes from ``torch.Generator`` objects keyed by
``(seed, stream, level)`` so each part can be regenerated on its own.
Nothing here factors or solves anything.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np
import torch

# stream ids for the keyed generators
_S_GEOM, _S_D, _S_U, _S_V, _S_RHS, _S_OMEGA, _S_TARGET = range(7)


def _gen(seed: int, stream: int, level: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed((int(seed) * 1_000_003 + stream * 10_007 + level * 101 + 12345) % (2**63 - 1))
    return g


def uniform_offsets(n: int, levels: int) -> np.ndarray:
    """Leaf offsets of a uniform halving tree (requires 2**levels | n)."""
    nl = 1 << levels
    if n % nl:
        raise ValueError(f"N={n} is not divisible by 2**L={nl}")
    return np.arange(nl + 1, dtype=np.int64) * (n // nl)


def rank_prefix(ranks: Sequence[int]) -> List[int]:
    """[R_0=0, R_1, ..., R_L] with R_l = r_1 + ... + r_l."""
    out = [0]
    for r in ranks:
        out.append(out[-1] + int(r))
    return out


@dataclasses.dataclass
class HodlrInputs:
    n: int
    levels: int
    leaf_offsets: np.ndarray          # int64, 2**L + 1
    ranks: List[int]                  # r_1..r_L
    D: torch.Tensor                   # (m_max, N)
    U: torch.Tensor                   # (R, N)
    V: torch.Tensor                   # (R, N)
    name: str = ""
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def m_max(self) -> int:
        return int(np.max(np.diff(self.leaf_offsets)))

    @property
    def R(self) -> int:
        return int(sum(self.ranks))

    def to(self, device=None, dtype=None) -> "HodlrInputs":
        return dataclasses.replace(
            self,
            D=self.D.to(device=device, dtype=dtype),
            U=self.U.to(device=device, dtype=dtype),
            V=self.V.to(device=device, dtype=dtype),
        )

    def numpy64(self):
        """(offsets, ranks, D (N x m_max), U (N x R), V (N x R)) as float64
        numpy (complex128 for complex inputs)."""
        dt = torch.complex128 if self.D.is_complex() else torch.float64
        return (self.leaf_offsets.copy(), list(self.ranks),
                self.D.detach().to("cpu", dt).numpy().T,
                self.U.detach().to("cpu", dt).numpy().T,
                self.V.detach().to("cpu", dt).numpy().T)


def _node_sizes_per_row(offsets: np.ndarray, levels: int, level: int) -> np.ndarray:
    """For each row, the size of the level-`level` node that contains it."""
    nl = 1 << levels
    per = nl >> level
    bounds = offsets[::per]
    sizes = np.diff(bounds)
    return np.repeat(sizes, sizes)


def synthetic(n: int, leaf: int, rank, seed: int = 0, shift: float = 4.0,
              dtype=torch.float64, device="cpu",
              leaf_offsets: Optional[np.ndarray] = None,
              levels: Optional[int] = None) -> HodlrInputs:
    """Synthetic HODLR matrix: D_a = G_a + shift*|I_a|*I with G_a ~ N(0,1);
    U_a, V_a ~ N(0,1)/sqrt(|I_a|) (each generator column has unit expected norm).

    ``rank`` is an int (same rank on every level) or a list r_1..r_L.
    ``leaf_offsets`` gives a non-uniform tree (then ``levels`` is implied).
    dtype=torch.complex128: real parts as for float64, imaginary parts drawn
    the same way from a second seed (without the shift), generators scaled
    by 1/sqrt(2) so their columns keep unit expected norm.
    """
    if dtype == torch.complex128:
        kw = dict(dtype=torch.float64, device=device, leaf_offsets=leaf_offsets, levels=levels)
        re = synthetic(n, leaf, rank, seed=seed, shift=shift, **kw)
        im = synthetic(n, leaf, rank, seed=seed + 7_777_777, shift=0.0, **kw)
        h = 1.0 / math.sqrt(2.0)
        return HodlrInputs(n, re.levels, re.leaf_offsets, re.ranks, torch.complex(re.D, im.D),
                           torch.complex(re.U * h, im.U * h), torch.complex(re.V * h, im.V * h),
                           name="complex " + re.name, meta=dict(kind="synthetic_complex", seed=seed, shift=shift))
    if leaf_offsets is None:
        if levels is None:
            levels = int(round(math.log2(n // leaf)))
        offsets = uniform_offsets(n, levels)
    else:
        offsets = np.asarray(leaf_offsets, dtype=np.int64)
        levels = int(round(math.log2(len(offsets) - 1)))
        assert offsets[0] == 0 and offsets[-1] == n and len(offsets) == (1 << levels) + 1
    ranks = [int(rank)] * levels if np.isscalar(rank) else [int(x) for x in rank]
    assert len(ranks) == levels
    sizes = np.diff(offsets)
    m_max = int(sizes.max())
    gen_dtype = torch.float64 if dtype == torch.float64 else torch.float32
    D = torch.zeros(m_max, n, dtype=gen_dtype, device=device)
    gD = _gen(seed, _S_D, levels, device)
    if np.all(sizes == m_max):
        nl = len(sizes)
        G = torch.randn(nl, m_max, m_max, generator=gD, dtype=gen_dtype, device=device)
        G.diagonal(dim1=1, dim2=2).add_(shift * m_max)
        # D[q, a*m + p] = D_a[p, q]
        D.copy_(G.permute(2, 0, 1).reshape(m_max, n))
        del G
    else:
        for a, m in enumerate(sizes):
            o = int(offsets[a])
            G = torch.randn(m, m, generator=gD, dtype=gen_dtype, device=device)
            G.diagonal().add_(shift * m)
            D[:m, o:o + m] = G.T
    Rp = rank_prefix(ranks)
    U = torch.empty(Rp[-1], n, dtype=gen_dtype, device=device)
    V = torch.empty(Rp[-1], n, dtype=gen_dtype, device=device)
    for lvl in range(1, levels + 1):
        r = ranks[lvl - 1]
        if r == 0:
            continue
        scale = torch.as_tensor(1.0 / np.sqrt(_node_sizes_per_row(offsets, levels, lvl)),
                                dtype=gen_dtype, device=device)
        gu = _gen(seed, _S_U, lvl, device)
        gv = _gen(seed, _S_V, lvl, device)
        U[Rp[lvl - 1]:Rp[lvl]] = torch.randn(r, n, generator=gu, dtype=gen_dtype, device=device) * scale
        V[Rp[lvl - 1]:Rp[lvl]] = torch.randn(r, n, generator=gv, dtype=gen_dtype, device=device) * scale
    return HodlrInputs(n, levels, offsets, ranks, D.to(dtype), U.to(dtype), V.to(dtype),
                       name=f"synthetic N={n} leaf={m_max} L={levels} r={ranks[0] if ranks else 0}",
                       meta=dict(kind="synthetic", seed=seed, shift=shift))


def gaussian_rhs(n: int, nrhs: int, seed: int = 0, stream: int = _S_RHS,
                 dtype=torch.float64, device="cpu") -> torch.Tensor:
    """(nrhs, N) tensor = N x nrhs column-major block of N(0,1) right-hand sides."""
    g = _gen(seed, stream, 0, device)
    return torch.randn(nrhs, n, generator=g, dtype=dtype, device=device)


# ---------------------------------------------------------------------------
# Laplace double-layer BIE on a star curve (second-kind Nystrom matrix)
# ---------------------------------------------------------------------------

def _star_geometry(n: int, device, amp=0.3, k=5):
    t = 2.0 * math.pi * torch.arange(n, dtype=torch.float64, device=device) / n
    r = 1.0 + amp * torch.cos(k * t)
    dr = -amp * k * torch.sin(k * t)
    d2r = -amp * k * k * torch.cos(k * t)
    c, s = torch.cos(t), torch.sin(t)
    x, y = r * c, r * s
    xp, yp = dr * c - r * s, dr * s + r * c
    xpp = d2r * c - 2 * dr * s - r * c
    ypp = d2r * s + 2 * dr * c - r * s
    sp = torch.sqrt(xp * xp + yp * yp)
    # inward unit normal of the counter-clockwise curve
    nx, ny = -yp / sp, xp / sp
    kappa = (xp * ypp - yp * xpp) / sp ** 3
    w = (2.0 * math.pi / n) * sp
    return x, y, nx, ny, kappa, w


def star_curve(n: int, device="cpu") -> dict:
    """The star curve's trapezoid nodes (geometry only): ``points`` (n, 2),
    inward unit ``normals`` (n, 2), quadrature ``weights`` (n,) and
    ``curvature`` (n,), float64 tensors."""
    x, y, nx, ny, kappa, w = _star_geometry(n, device)
    return dict(points=torch.stack([x, y], 1), normals=torch.stack([nx, ny], 1), weights=w, curvature=kappa)


class _BieEntries:
    """A_ij = 1/2 delta_ij + w_j d(x_i, x_j), d(x,y) = n(y).(x-y) / (2 pi |x-y|^2)
    with the inward normal; the diagonal uses the smooth limit kappa/(4 pi)."""

    def __init__(self, n, device):
        self.x, self.y, self.nx, self.ny, self.kappa, self.w = _star_geometry(n, device)

    def block(self, ri: torch.Tensor, cj: torch.Tensor) -> torch.Tensor:
        """Entries A[ri[..., :, None], cj[..., None, :]] for disjoint index sets."""
        dx = self.x[ri][..., :, None] - self.x[cj][..., None, :]
        dy = self.y[ri][..., :, None] - self.y[cj][..., None, :]
        num = self.nx[cj][..., None, :] * dx + self.ny[cj][..., None, :] * dy
        return num / (2.0 * math.pi * (dx * dx + dy * dy)) * self.w[cj][..., None, :]

    def diag_block(self, idx: torch.Tensor) -> torch.Tensor:
        """Full square block A[idx, idx] (idx: (..., m)) including the diagonal."""
        dx = self.x[idx][..., :, None] - self.x[idx][..., None, :]
        dy = self.y[idx][..., :, None] - self.y[idx][..., None, :]
        r2 = dx * dx + dy * dy
        eye = torch.eye(idx.shape[-1], dtype=torch.bool, device=idx.device)
        r2 = torch.where(eye, torch.ones_like(r2), r2)
        num = self.nx[idx][..., None, :] * dx + self.ny[idx][..., None, :] * dy
        K = num / (2.0 * math.pi * r2)
        dg = (self.kappa[idx] / (4.0 * math.pi))[..., :, None].expand_as(K)
        K = torch.where(eye, dg, K)
        A = K * self.w[idx][..., None, :]
        return A + 0.5 * eye.to(A.dtype)


def _aca_batched(entries, rows: torch.Tensor, cols: torch.Tensor, kmax: int):
    """Adaptive cross approximation with partial pivoting, batched over blocks.

    rows, cols: (B, n) index arrays.  Returns U, V of shape (B, n, kmax) with
    block ~= U V^T.  A fixed number of steps is taken; exhausted blocks get
    zero columns.
    """
    B, n = rows.shape
    dev = rows.device
    Uc = torch.zeros(B, n, kmax, dtype=torch.float64, device=dev)
    Vc = torch.zeros(B, n, kmax, dtype=torch.float64, device=dev)
    used = torch.zeros(B, n, dtype=torch.bool, device=dev)
    ip = torch.zeros(B, dtype=torch.long, device=dev)
    bi = torch.arange(B, device=dev)
    for k in range(kmax):
        ri = rows[bi, ip][:, None]                                     # (B,1)
        row = entries.block(ri, cols)[:, 0, :]                         # (B,n)
        if k:
            row = row - torch.einsum("bk,bnk->bn", Uc[bi, ip, :k], Vc[:, :, :k])
        jp = torch.argmax(row.abs(), dim=1)
        delta = row[bi, jp]
        ok = delta.abs() > 1e-300
        v = torch.where(ok[:, None], row / torch.where(ok, delta, torch.ones_like(delta))[:, None],
                        torch.zeros_like(row))
        cj = cols[bi, jp][:, None]
        col = entries.block(rows, cj)[:, :, 0]                         # (B,n)
        if k:
            col = col - torch.einsum("bnk,bk->bn", Uc[:, :, :k], Vc[bi, jp, :k])
        col = torch.where(ok[:, None], col, torch.zeros_like(col))
        Uc[:, :, k] = col
        Vc[:, :, k] = v
        used[bi, ip] = True
        score = torch.where(used, torch.full_like(col, -1.0), col.abs())
        ip = torch.argmax(score, dim=1)
    return Uc, Vc


def _recompress(Uc: torch.Tensor, Vc: torch.Tensor, r: int):
    """Truncate U V^T (B, n, k) to exactly rank r via QR + SVD (balanced split)."""
    Qu, Ru = torch.linalg.qr(Uc)
    Qv, Rv = torch.linalg.qr(Vc)
    M = Ru @ Rv.transpose(1, 2)
    P, S, Wt = torch.linalg.svd(M)
    s = torch.sqrt(S[:, :r])
    U = Qu @ (P[:, :, :r] * s[:, None, :])
    V = Qv @ (Wt.transpose(1, 2)[:, :, :r] * s[:, None, :])
    return U, V


def bie_star(n: int, leaf: int, rank: int, oversample: int = 8, dtype=torch.float64,
             device="cpu") -> HodlrInputs:
    """Second-kind Nystrom matrix of the Laplace double layer (1/2 I + D) on the
    star curve r(t) = 1 + 0.3 cos 5t, trapezoid nodes t_j = 2 pi j / N in
    natural order, halving tree; leaf blocks exact, every sibling block
    compressed to exactly ``rank`` by ACA (rank + oversample steps) followed by
    QR/SVD recompression."""
    levels = int(round(math.log2(n // leaf)))
    offsets = uniform_offsets(n, levels)
    ent = _BieEntries(n, device)
    nl = 1 << levels
    idx = torch.arange(n, device=device).view(nl, leaf)
    D = ent.diag_block(idx)                                             # (nl, m, m)
    Dt = D.permute(2, 0, 1).reshape(leaf, n).contiguous()
    del D
    R = rank * levels
    U = torch.empty(R, n, dtype=torch.float64, device=device)
    V = torch.empty(R, n, dtype=torch.float64, device=device)
    kmax = rank + oversample
    for lvl in range(1, levels + 1):
        nb = 1 << lvl
        sz = n // nb
        nodes = torch.arange(n, device=device).view(nb, sz)
        sib = torch.arange(nb, device=device) ^ 1
        Uc, Vc = _aca_batched(ent, nodes, nodes[sib], min(kmax, sz))
        if Uc.shape[2] < rank:
            raise ValueError("rank exceeds node size")
        Ub, Vb = _recompress(Uc, Vc, rank)
        del Uc, Vc
        c0 = (lvl - 1) * rank
        # block of row-node k: A(I_k, I_sib(k)) = U_k V_sib(k)^T
        U[c0:c0 + rank] = Ub.permute(2, 0, 1).reshape(rank, n)
        V[c0:c0 + rank] = Vb[sib].permute(2, 0, 1).reshape(rank, n)
    return HodlrInputs(n, levels, offsets, [rank] * levels, Dt.to(dtype), U.to(dtype), V.to(dtype),
                       name=f"Laplace double-layer BIE star N={n} leaf={leaf} r={rank}",
                       meta=dict(kind="bie_star", oversample=oversample))


# ---------------------------------------------------------------------------
# Kernel matrices on random points (Gaussian 2-D, Matern-3/2 3-D)
# ---------------------------------------------------------------------------

def rcb_order(P: np.ndarray, leaf: int) -> np.ndarray:
    """Recursive coordinate bisection: split at the median along the axis of
    largest bounding-box extent (ties -> lowest axis), stable sort, lower
    half first.  Returns the permutation (new order -> original index)."""
    out = []

    def rec(ix):
        if len(ix) <= leaf:
            out.append(ix)
            return
        Q = P[ix]
        d = int(np.argmax(Q.max(0) - Q.min(0)))
        o = ix[np.argsort(Q[:, d], kind="stable")]
        h = len(o) // 2
        rec(o[:h])
        rec(o[h:])

    rec(np.arange(len(P)))
    return np.concatenate(out)


def kernel_points(n: int, dim: int, leaf: int, seed: int = 0) -> np.ndarray:
    """n points uniform in [0,1]^dim (seeded), in RCB order with ``leaf``-point
    leaves: an (n, dim) float64 array."""
    rng = np.random.default_rng(int(seed) * 7919 + 17)
    pts = rng.random((n, dim))
    return pts[rcb_order(pts, leaf)]


def _kernel_fn(kind: str):
    if kind == "gauss":
        s2 = 2.0 * 0.05 ** 2
        return lambda d2: torch.exp(-d2 / s2)
    if kind == "matern32":
        c = math.sqrt(3.0) / 0.1

        def f(d2):
            s = c * torch.sqrt(d2)
            return (1.0 + s) * torch.exp(-s)
        return f
    raise ValueError(kind)


def _kblock(P: torch.Tensor, ri: torch.Tensor, cj: torch.Tensor, f):
    X = P[ri]               # (..., a, dim)
    Y = P[cj]               # (..., b, dim)
    d2 = ((X[..., :, None, :] - Y[..., None, :, :]) ** 2).sum(-1)
    return f(d2)


def _block_apply(P, rows, cols, M, f, budget=1 << 25):
    """(B, n, n) kernel blocks K(rows_b, cols_b) applied to M (B, n, k), chunked."""
    B, n = rows.shape
    out = torch.empty(B, n, M.shape[2], dtype=M.dtype, device=M.device)
    step = max(1, min(n, budget // max(1, B * n)))
    for i0 in range(0, n, step):
        Kc = _kblock(P, rows[:, i0:i0 + step], cols, f)
        out[:, i0:i0 + step] = Kc @ M
    return out


def kernel_matrix(n: int, leaf: int, rank: int, kind: str, dim: int, nugget: float,
                  seed: int = 0, oversample: int = 10, power_iters: int = 1,
                  dtype=torch.float64, device="cpu") -> HodlrInputs:
    """Symmetric kernel matrix K(x_i, x_j) + nugget*I on N points uniform in
    [0,1]^dim ordered by RCB; leaf blocks exact; each sibling pair compressed
    once by a randomized range finder (Gaussian test matrix, oversampling,
    power iterations, QR, truncated SVD to exactly ``rank``) so that U = V
    per node."""
    levels = int(round(math.log2(n // leaf)))
    offsets = uniform_offsets(n, levels)
    P = torch.as_tensor(kernel_points(n, dim, leaf, seed), dtype=torch.float64, device=device)
    f = _kernel_fn(kind)
    nl = 1 << levels
    idx = torch.arange(n, device=device).view(nl, leaf)
    Dblk = _kblock(P, idx, idx, f) + nugget * torch.eye(leaf, dtype=torch.float64, device=device)
    Dt = Dblk.permute(2, 0, 1).reshape(leaf, n).contiguous()
    del Dblk
    R = rank * levels
    U = torch.empty(R, n, dtype=torch.float64, device=device)
    for lvl in range(1, levels + 1):
        nb = 1 << lvl
        sz = n // nb
        nodes = torch.arange(n, device=device).view(nb, sz)
        a_rows, b_rows = nodes[0::2], nodes[1::2]          # sibling pairs
        k = min(rank + oversample, sz)
        g = _gen(seed, _S_OMEGA, lvl, device)
        Om = torch.randn(nb // 2, sz, k, generator=g, dtype=torch.float64, device=device)
        Y = _block_apply(P, a_rows, b_rows, Om, f)           # A_ab Om
        for _ in range(power_iters):
            Q, _r = torch.linalg.qr(Y)
            Z = _block_apply(P, b_rows, a_rows, Q, f)        # A_ab^T Q
            Y = _block_apply(P, a_rows, b_rows, Z, f)
        Q, _r = torch.linalg.qr(Y)                           # (B, sz, k)
        Bt = _block_apply(P, b_rows, a_rows, Q, f)           # (A_ab^T Q) = B^T, (B, sz, k)
        W, S, Zt = torch.linalg.svd(Bt, full_matrices=False)  # B^T = W S Zt  ->  B = Zt^T S W^T
        s = torch.sqrt(S[:, :rank])
        Ua = Q @ (Zt.transpose(1, 2)[:, :, :rank] * s[:, None, :])   # A_ab ~= Ua Vb^T
        Vb = W[:, :, :rank] * s[:, None, :]
        c0 = (lvl - 1) * rank
        blk = torch.empty(nb, sz, rank, dtype=torch.float64, device=device)
        blk[0::2] = Ua
        blk[1::2] = Vb
        U[c0:c0 + rank] = blk.permute(2, 0, 1).reshape(rank, n)
    V = U.clone()
    return HodlrInputs(n, levels, offsets, [rank] * levels, Dt.to(dtype), U.to(dtype), V.to(dtype),
                       name=f"{kind} kernel N={n} dim={dim} leaf={leaf} r={rank}",
                       meta=dict(kind=kind, dim=dim, nugget=nugget, seed=seed))


def helmholtz_matrix(n: int, leaf: int, rank: int, kappa: float = 20.0, seed: int = 0, oversample: int = 10,
                     power_iters: int = 1, device="cpu") -> HodlrInputs:
    """Complex symmetric matrix I + h G on N points uniform in [0,1]^3 in RCB
    order, G_pq = exp(i kappa |x_p - x_q|) / (4 pi |x_p - x_q|) (the 3-D
    Helmholtz fundamental solution, G_pp = 0), h = 4/N; leaf blocks exact;
    each sibling pair compressed once by a randomized range finder (complex
    Gaussian test matrix, oversampling, power iterations, QR, truncated SVD
    to exactly ``rank``) into A(I_a, I_b) ~= U_a V_b^*; A(I_b, I_a) =
    A(I_a, I_b)^T then gives U_b = conj(V_b) and V_a = conj(U_a)."""
    levels = int(round(math.log2(n // leaf)))
    offsets = uniform_offsets(n, levels)
    P = torch.as_tensor(kernel_points(n, 3, leaf, seed), dtype=torch.float64, device=device)
    h = 4.0 / n

    def f(d2):
        d = torch.sqrt(d2)
        return h * torch.exp(1j * kappa * d) / (4.0 * math.pi * d)

    nl = 1 << levels
    idx = torch.arange(n, device=device).view(nl, leaf)
    Dblk = _kblock(P, idx, idx, f)
    eye = torch.eye(leaf, dtype=torch.bool, device=device)
    Dblk = torch.where(eye, torch.ones((), dtype=Dblk.dtype, device=device), Dblk)
    Dt = Dblk.permute(2, 0, 1).reshape(leaf, n).contiguous()
    del Dblk
    R = rank * levels
    U = torch.empty(R, n, dtype=torch.complex128, device=device)
    V = torch.empty(R, n, dtype=torch.complex128, device=device)
    for lvl in range(1, levels + 1):
        nb = 1 << lvl
        sz = n // nb
        nodes = torch.arange(n, device=device).view(nb, sz)
        a_rows, b_rows = nodes[0::2], nodes[1::2]
        k = min(rank + oversample, sz)
        g = _gen(seed, _S_OMEGA, lvl, device)
        Om = torch.complex(torch.randn(nb // 2, sz, k, generator=g, dtype=torch.float64, device=device),
                           torch.randn(nb // 2, sz, k, generator=g, dtype=torch.float64, device=device))
        # A_ab X and A_ab^* X = conj(A_ba conj(X)) (A_ab^T = A_ba)
        Y = _block_apply(P, a_rows, b_rows, Om, f)
        for _ in range(power_iters):
            Q, _r = torch.linalg.qr(Y)
            Z = _block_apply(P, b_rows, a_rows, Q.conj(), f).conj()
            Y = _block_apply(P, a_rows, b_rows, Z, f)
        Q, _r = torch.linalg.qr(Y)                                   # (B, sz, k)
        Bs = _block_apply(P, b_rows, a_rows, Q.conj(), f).conj()     # B^* = A_ab^* Q, (B, sz, k)
        W, S, Zh = torch.linalg.svd(Bs, full_matrices=False)         # B^* = W S Zh  ->  B = Zh^* S W^*
        s = torch.sqrt(S[:, :rank]).to(torch.complex128)
        Ua = Q @ (Zh.conj().transpose(1, 2)[:, :, :rank] * s[:, None, :])   # A_ab ~= Ua Vb^*
        Vb = W[:, :, :rank] * s[:, None, :]
        c0 = (lvl - 1) * rank
        bu = torch.empty(nb, sz, rank, dtype=torch.complex128, device=device)
        bv = torch.empty(nb, sz, rank, dtype=torch.complex128, device=device)
        bu[0::2], bv[1::2] = Ua, Vb
        bu[1::2], bv[0::2] = Vb.conj(), Ua.conj()
        U[c0:c0 + rank] = bu.permute(2, 0, 1).reshape(rank, n)
        V[c0:c0 + rank] = bv.permute(2, 0, 1).reshape(rank, n)
    return HodlrInputs(n, levels, offsets, [rank] * levels, Dt, U, V,
                       name=f"Helmholtz 3-D kernel N={n} kappa={kappa} leaf={leaf} r={rank}",
                       meta=dict(kind="helmholtz", kappa=kappa, seed=seed))


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

CONFIGS = {
    0: dict(desc="synthetic HODLR FP64, N=4096, leaf 64 (L=6), r=16, one RHS b = A x_true",
            n=4096, leaf=64, rank=16, nrhs=1, storage="f64"),
    1: dict(desc="Gaussian kernel (sigma 0.05) + 1e-2 I on N=262144 points in [0,1]^2, RCB, leaf 128, r=32",
            n=262144, leaf=128, rank=32, nrhs=16, storage="f64"),
    2: dict(desc="Laplace double-layer BIE (1/2 I + D) on the star curve, N=1048576, leaf 256, r=32",
            n=1 << 20, leaf=256, rank=32, nrhs=1, storage="f64"),
    3: dict(desc="Matern-3/2 (l=0.1) + 1e-3 I on N=131072 points in [0,1]^3, RCB, leaf 128, r=24, FP32",
            n=131072, leaf=128, rank=24, nrhs=1, storage="f32"),
    4: dict(desc="synthetic HODLR N=4194304, leaf 256 (L=14), r=64, shift 4*leaf, stored FP32, 32 RHS",
            n=1 << 22, leaf=256, rank=64, nrhs=32, storage="f32"),
}


def make_config(cfg: int, device="cpu", n: Optional[int] = None, seed: int = 0) -> HodlrInputs:
    """Build workload ``cfg`` (optionally at a smaller N with the same leaf and rank)."""
    c = CONFIGS[cfg]
    n = c["n"] if n is None else n
    sdt = torch.float64 if c["storage"] == "f64" else torch.float32
    if cfg in (0, 4):
        return synthetic(n, c["leaf"], c["rank"], seed=seed, dtype=sdt, device=device)
    if cfg == 1:
        return kernel_matrix(n, c["leaf"], c["rank"], "gauss", 2, 1e-2, seed=seed, dtype=sdt, device=device)
    if cfg == 2:
        return bie_star(n, c["leaf"], c["rank"], dtype=sdt, device=device)
    if cfg == 3:
        return kernel_matrix(n, c["leaf"], c["rank"], "matern32", 3, 1e-3, seed=seed, dtype=sdt, device=device)
    raise ValueError(cfg)
