"""The allocation-free solve (hodlr_solve_noalloc) against hodlr_solve /
hodlr_solve_adjoint on the same factors, through the C ABI: two calls in a
row on one GPU's scratch, the second with a smaller input (fewer columns and
a smaller factorization), each equal to the workspace-based entry point bit
for bit (same kernels) and to the oracle within the FP64 bar; sizes beyond
the scratch are refused before any launch."""
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


def _rel(a, b):
    nb = np.linalg.norm(b, axis=0)
    return float(np.max(np.linalg.norm(a - b, axis=0) / np.where(nb > 0, nb, 1.0)))


def _rhs(n, k, seed):
    return np.random.default_rng(seed).standard_normal((n, k))


def _check(F, H, Fo, B, adjoint, precision):
    hd = _hd()
    Bd = torch.as_tensor(np.ascontiguousarray(B.T), device=DEV)
    want = (F.solve_adjoint(Bd) if adjoint else F.solve(Bd))
    got = F.solve_noalloc_(Bd.clone(), adjoint=adjoint)
    torch.cuda.synchronize()
    assert torch.equal(got, want), "noalloc result differs from the workspace entry point"
    ref = O.solve_adjoint(H, B) if adjoint else O.solve(Fo, B)
    err = _rel(got.cpu().numpy().T, ref)
    print(f"  noalloc {precision} adjoint={adjoint} N={H.N} nrhs={B.shape[1]}: rel err vs oracle {err:.2e}",
          flush=True)
    assert err < (1e-12 if precision == "fp64" else 1e-3)
    return hd


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_matches_solve_twice_then_smaller(precision):
    hd = _hd()
    st = torch.float64 if precision == "fp64" else torch.float32
    # first call: N = 16384, leaf 256, r = 32 (several tiles per node at the top), 5 columns
    inp1 = W.synthetic(16384, 256, 32, seed=31, dtype=st)
    H1 = O.from_inputs(inp1)
    F1 = hd.factor(hd.HODLRMatrix.from_inputs(inp1.to(DEV)), precision)
    Fo1 = O.factor(H1)
    assert 0 < F1.noalloc_bytes(5) <= 64 << 20
    _check(F1, H1, Fo1, _rhs(H1.N, 5, 32), False, precision)
    _check(F1, H1, Fo1, _rhs(H1.N, 5, 33), True, precision)
    # second call: a smaller ragged factorization and fewer columns on the same scratch
    off = np.concatenate([[0], np.cumsum(np.random.default_rng(34).integers(20, 90, 16))])
    inp2 = W.synthetic(int(off[-1]), 0, [9, 0, 17, 5], seed=35, leaf_offsets=off, dtype=st)
    H2 = O.from_inputs(inp2)
    F2 = hd.factor(hd.HODLRMatrix.from_inputs(inp2.to(DEV)), precision)
    Fo2 = O.factor(H2)
    _check(F2, H2, Fo2, _rhs(H2.N, 2, 36), False, precision)
    _check(F2, H2, Fo2, _rhs(H2.N, 2, 37), True, precision)
    # and the first factorization again, one column
    _check(F1, H1, Fo1, _rhs(H1.N, 1, 38), False, precision)


def test_noalloc_refuses_sizes_beyond_the_scratch():
    hd = _hd()
    inp = W.synthetic(65536, 256, 32, seed=39)
    F = hd.factor(hd.HODLRMatrix.from_inputs(inp.to(DEV)), "fp64")
    k = 1
    while F.noalloc_bytes(k) <= 64 << 20 and k < 32768:
        k *= 2
    assert F.noalloc_bytes(k) > 64 << 20
    B = torch.zeros(k, inp.n, dtype=torch.float64, device=DEV)
    with pytest.raises(hd.HodlrError) as e:
        F.solve_noalloc_(B)
    assert e.value.status == -1
    assert torch.count_nonzero(B).item() == 0   # nothing was launched
