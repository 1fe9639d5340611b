"""Operation and storage counts for HODLR factor/solve (host arithmetic only).

These follow the complexity analysis of Section III-D (Theorems "Storage",
"Factorization cost" and "Solution cost"), generalised to per-level ranks
r_1..r_L and non-uniform leaves:

* storage entries       S = sum_a m_a^2 + 2 N R                   (Thm "Storage";
  the printed m N + r N L drops the factor 2 that its own derivation has)
* paper factor flops    F = 2/3 sum_a m_a^3 + 2 sum_a m_a^2 R + sum_l 4 N r_l R_l
  which for uniform m and constant r is 2/3 m^2 N + 2 m r N L + 2 r^2 N (L + L^2)
* solve flops per rhs   S_f = 2 sum_a m_a^2 + sum_l 4 N r_l       (Thm "Solution cost")

``R_l = r_1 + ... + r_l`` and ``R = R_L``.
"""
from __future__ import annotations

from typing import Dict, Sequence

import numpy as np


def _prefix(ranks):
    out = [0]
    for r in ranks:
        out.append(out[-1] + int(r))
    return out


def storage_entries(leaf_offsets: Sequence[int], ranks: Sequence[int]) -> int:
    m = np.diff(np.asarray(leaf_offsets, dtype=np.int64))
    n = int(np.asarray(leaf_offsets)[-1])
    return int(np.sum(m * m) + 2 * n * sum(int(r) for r in ranks))


def factor_flops_paper(leaf_offsets: Sequence[int], ranks: Sequence[int]) -> float:
    m = np.diff(np.asarray(leaf_offsets, dtype=np.float64))
    n = float(np.asarray(leaf_offsets)[-1])
    Rp = _prefix(ranks)
    R = Rp[-1]
    lv = sum(4.0 * n * int(ranks[l - 1]) * Rp[l] for l in range(1, len(ranks) + 1))
    return float(2.0 / 3.0 * np.sum(m ** 3) + 2.0 * np.sum(m * m) * R + lv)


def factor_flops_executed(leaf_offsets: Sequence[int], ranks: Sequence[int]) -> Dict[str, float]:
    """Flops of each factor step as this library executes them."""
    m = np.diff(np.asarray(leaf_offsets, dtype=np.float64))
    n = float(np.asarray(leaf_offsets)[-1])
    Rp = _prefix(ranks)
    R = Rp[-1]
    out = dict(leaf_lu=float(2.0 / 3.0 * np.sum(m ** 3)), leaf_trsm=float(2.0 * np.sum(m * m) * R),
               couple_product=0.0, couple_lu=0.0, couple_solve=0.0, update=0.0)
    for l in range(1, len(ranks) + 1):
        r = int(ranks[l - 1])
        parents = 1 << (l - 1)
        out["couple_product"] += 2.0 * n * r * Rp[l]
        out["couple_lu"] += parents * 2.0 / 3.0 * (2 * r) ** 3
        out["couple_solve"] += parents * 2.0 * (2 * r) ** 2 * Rp[l - 1]
        out["update"] += 2.0 * n * r * Rp[l - 1]
    out["total"] = sum(out.values())
    return out


def solve_flops(leaf_offsets: Sequence[int], ranks: Sequence[int], nrhs: int = 1) -> float:
    m = np.diff(np.asarray(leaf_offsets, dtype=np.float64))
    n = float(np.asarray(leaf_offsets)[-1])
    return float(nrhs * (2.0 * np.sum(m * m) + sum(4.0 * n * int(r) for r in ranks)))


def paper_closed_form_factor(n: int, m: int, r: int, L: int) -> float:
    return 2.0 / 3.0 * m * m * n + 2.0 * m * r * n * L + 2.0 * r * r * n * (L + L * L)
