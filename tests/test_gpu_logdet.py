"""Sign and log|det A| from the GPU factors (hodlr_logdet) against the
oracle's product-form determinant, which the CPU pins tie to LAPACK's slogdet
of the assembled matrix.  Cases cover both coupling routes (explicit inverse
for r in {8, 16, 24, 32}, LU with partial pivoting otherwise), ragged and deep
trees, rank-0 levels, a single leaf, negative determinants, FP32 factors and
an exactly singular leaf."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _hd():
    from paper_2208_06290_amd import hodlr
    return hodlr


def _offsets(n, L, seed, min_leaf=5, max_leaf=256):
    rng = np.random.default_rng(seed)
    while True:
        w = rng.uniform(0.5, 1.5, 1 << L)
        sizes = np.maximum(min_leaf, np.round(w / w.sum() * n)).astype(np.int64)
        sizes[-1] += n - sizes.sum()
        if sizes.min() >= min_leaf and sizes.max() <= max_leaf:
            return np.concatenate([[0], np.cumsum(sizes)])


CASES = {
    "cfg0_like": dict(n=4096, leaf=64, ranks=16),                                # inverse route
    "leaf128_L5_r64": dict(n=4096, leaf=128, ranks=64),                          # LU route, 2r = 128
    "ragged_L6": dict(n=3001, L=6, ranks=[33, 20, 64, 9, 1, 17]),                # LU route, mixed
    "ragged_L4_r0": dict(n=1000, L=4, ranks=[7, 0, 13, 5]),                      # a rank-0 level
    "deep_L8": dict(n=4096, leaf=16, ranks=[4, 8, 3, 5, 6, 2, 7, 3]),
    "leaf256_L5_mixed": dict(n=8192, leaf=256, ranks=[16, 48, 32, 32, 32]),      # fused bottom levels
    "L0_leaf200": dict(n=200, leaf=200, ranks=[]),
}


def _build(name, seed, dtype=torch.float64, shift=4.0):
    c = CASES[name]
    off = _offsets(c["n"], c["L"], seed + 11) if c.get("leaf") is None else None
    inp = W.synthetic(c["n"], c.get("leaf") or 0, c["ranks"], seed=seed, leaf_offsets=off, dtype=dtype, shift=shift)
    return inp, O.from_inputs(inp)


def _flip_sign(inp):
    """Negate row 0 of A (its leaf-block part in D and its generator part in
    U): det A changes sign.  D is (m_max, N) and U (R, N), so row 0 of A is
    column 0 of both tensors."""
    inp.D[:, 0] = -inp.D[:, 0]
    inp.U[:, 0] = -inp.U[:, 0]


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("negate", [False, True])
def test_logdet_matches_oracle(name, negate):
    inp, H = _build(name, 70)
    sign0, la0 = O.slogdet(O.factor(H))
    if negate:
        _flip_sign(inp)
        H = O.from_inputs(inp)
    sign_o, la_o = O.slogdet(O.factor(H))
    if negate:
        assert sign_o == -sign0 and abs(la_o - la0) <= 1e-12 * max(1.0, abs(la0))
    F = _hd().factor(_hd().HODLRMatrix.from_inputs(inp.to(DEV)), "fp64")
    sign, la = F.slogdet()
    print(f"logdet {name} negate={negate}: gpu ({sign:+.0f}, {la:.15e}) oracle ({sign_o:+.0f}, {la_o:.15e})",
          flush=True)
    assert sign == sign_o
    assert abs(la - la_o) <= 1e-12 * max(1.0, abs(la_o))
    # deterministic: a second factorization gives the same bits
    F2 = _hd().factor(_hd().HODLRMatrix.from_inputs(inp.to(DEV)), "fp64")
    assert F2.slogdet() == (sign, la)


@pytest.mark.parametrize("name", ["cfg0_like", "ragged_L6", "leaf128_L5_r64"])
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_logdet_low_precision_factors(name, precision):
    """FP32 / BF16 factors: the pivots carry the factorization's error, about
    kappa * u of the format per pivot relative, summed over N pivots."""
    inp, H = _build(name, 71, dtype=torch.float32)
    sign_o, la_o = O.slogdet(O.factor(H))
    F = _hd().factor(_hd().HODLRMatrix.from_inputs(inp.to(DEV)), precision)
    sign, la = F.slogdet()
    err = abs(la - la_o)
    print(f"logdet {precision} {name}: |logabs error| {err:.2e} (logabs {la_o:.6e})", flush=True)
    assert sign == sign_o
    u = 6e-8 if precision == "fp32" else 4e-3
    assert err <= 10 * u * H.N


def test_logdet_of_singular_leaf_is_minus_infinity():
    inp = W.synthetic(512, 64, 8, seed=72)
    inp.D[5, 64 * 3:64 * 4] = 0.0   # leaf 3, column 5 of its block is zero
    F = _hd().factor(_hd().HODLRMatrix.from_inputs(inp.to(DEV)), "fp64", raise_singular=False)
    assert F.info is not None
    sign, la = F.slogdet()
    assert sign == 0.0 and la == -np.inf


def _grad_err(got, ref, H=None, leaf_blocks=False):
    g = got.double().cpu().numpy().T
    if leaf_blocks:
        num = den = 0.0
        for i in range(1 << H.L):
            s0, e = O.node_range(H, H.L, i)
            num += float(np.sum((g[s0:e, :e - s0] - ref[s0:e, :e - s0]) ** 2))
            den += float(np.sum(ref[s0:e, :e - s0] ** 2))
        return (num / den) ** 0.5
    return float(np.linalg.norm(g - ref) / np.linalg.norm(ref))


@pytest.mark.parametrize("name", list(CASES))
def test_logdet_gradient_matches_oracle(name):
    """Gradient of log|det A| through the factorization (both coupling
    routes, ragged, rank-0, deep, single leaf) against the oracle's
    A^{-T} restricted to D, U, V (itself pinned by finite differences of
    LAPACK's slogdet)."""
    inp, H = _build(name, 73)
    rD, rU, rV = O.logdet_grad_structured(H)
    F = _hd().factor(_hd().HODLRMatrix.from_inputs(inp.to(DEV)), "fp64")
    dD, dU, dV = F.slogdet_grad()
    eD = _grad_err(dD, rD, H, leaf_blocks=True)
    eU = _grad_err(dU, rU) if H.U.size else 0.0
    eV = _grad_err(dV, rV) if H.V.size else 0.0
    print(f"logdet gradient {name}: rel err D {eD:.2e} U {eU:.2e} V {eV:.2e}", flush=True)
    assert max(eD, eU, eV) < 1e-11
    # entries of dD outside the leaf blocks stay untouched (zero)
    g = dD.double().cpu().numpy().T
    mask = np.ones_like(g, dtype=bool)
    for i in range(1 << H.L):
        s0, e = O.node_range(H, H.L, i)
        mask[s0:e, :e - s0] = False
    assert not np.any(g[mask])


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_logdet_gradient_low_precision_factors(precision):
    """FP32 storage, FP32/BF16 factors: the solves carry the factors' error."""
    inp, H = _build("cfg0_like", 74, dtype=torch.float32)
    rD, rU, rV = O.logdet_grad_structured(H)
    F = _hd().factor(_hd().HODLRMatrix.from_inputs(inp.to(DEV)), precision)
    dD, dU, dV = F.slogdet_grad()
    assert dD.dtype == torch.float32
    e = max(_grad_err(dD, rD, H, leaf_blocks=True), _grad_err(dU, rU), _grad_err(dV, rV))
    print(f"logdet gradient {precision}: max rel err {e:.2e}", flush=True)
    assert e < (1e-5 if precision == "fp32" else 5e-2)
