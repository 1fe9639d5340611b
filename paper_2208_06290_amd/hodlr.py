"""Python binding of the HODLR C ABI (``include/hodlr.h``) over torch tensors.

Argument marshalling only: every step of factorization, solve, adjoint,
matrix product and gradient runs in ``libhodlr.so``.  Tensors must live on a
ROCm device; the library fails loudly when it is missing.

Layout convention (column-major at the ABI): a torch tensor of row-major
shape ``(k, N)`` is the N x k column-major matrix, so ``D`` is ``(m_max, N)``,
``U``/``V`` are ``(R, N)`` and right-hand sides are ``(nrhs, N)``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhodlr.so")

F64, F32, BF16, C128 = 0, 1, 2, 3
_DT = {"fp64": F64, "fp32": F32, "bf16": BF16}
INPLACE = 1  # hodlr_factor flag: the factors overwrite D and U
_STATUS = {0: "ok", -1: "invalid argument", -2: "device allocation failed", -3: "HIP runtime error",
           -4: "unsupported by this build", 1: "exactly singular pivot",
           2: "iterative refinement did not converge"}
OK, ERR_SINGULAR, ERR_NOT_CONVERGED = 0, 1, 2


class HodlrError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {_STATUS.get(status, status)} (status {status})")
        self.status = status


class _Matrix(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("levels", ctypes.c_int32),
                ("leaf_offsets", ctypes.POINTER(ctypes.c_int64)), ("ranks", ctypes.POINTER(ctypes.c_int32)),
                ("dtype", ctypes.c_int), ("D", ctypes.c_void_p), ("ldd", ctypes.c_int64),
                ("U", ctypes.c_void_p), ("ldu", ctypes.c_int64), ("V", ctypes.c_void_p), ("ldv", ctypes.c_int64)]


class _Info(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("column", ctypes.c_int32), ("node", ctypes.c_int64)]


class _Opts(ctypes.Structure):
    _fields_ = [("refine", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("tol", ctypes.c_double)]


class _Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32), ("relres", ctypes.c_double)]


class _Kernel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("dim", ctypes.c_int32), ("points", ctypes.c_void_p), ("ldp", ctypes.c_int64),
                ("normals", ctypes.c_void_p), ("weights", ctypes.c_void_p), ("curvature", ctypes.c_void_p),
                ("ell", ctypes.c_double), ("shift", ctypes.c_double)]


KERNELS = {"gauss": 0, "matern32": 1, "laplace_dl": 2}

EXPORTS = ["hodlr_factor", "hodlr_refactor", "hodlr_solve", "hodlr_solve_adjoint", "hodlr_solve_noalloc",
           "hodlr_solve_noalloc_bytes", "hodlr_matvec", "hodlr_grad", "hodlr_logdet", "hodlr_logdet_grad",
           "hodlr_factors_y", "hodlr_factor_bytes", "hodlr_destroy", "hodlr_status_string", "hodlr_timing_enable",
           "hodlr_kernel_times", "hodlr_construct"]

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libhodlr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2208_06290_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.hodlr_factor.argtypes = [ctypes.POINTER(_Matrix), ctypes.c_int, i32, vp, ctypes.POINTER(vp),
                                 ctypes.POINTER(_Info)]
    lib.hodlr_refactor.argtypes = [vp, ctypes.POINTER(_Matrix), vp, ctypes.POINTER(_Info)]
    for f in (lib.hodlr_solve, lib.hodlr_solve_adjoint):
        f.argtypes = [vp, i64, vp, i64, ctypes.POINTER(_Opts), vp, ctypes.POINTER(_Stats)]
    lib.hodlr_solve_noalloc.argtypes = [vp, i32, i64, vp, i64, vp]
    lib.hodlr_solve_noalloc_bytes.argtypes = [vp, i64]
    lib.hodlr_solve_noalloc_bytes.restype = ctypes.c_size_t
    lib.hodlr_matvec.argtypes = [ctypes.POINTER(_Matrix), i32, i64, vp, i64, vp, i64, vp]
    lib.hodlr_grad.argtypes = [vp, i64, vp, i64, vp, i64, vp, vp, vp, vp]
    lib.hodlr_factors_y.argtypes = [vp, vp, i64, vp]
    lib.hodlr_logdet.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), vp]
    lib.hodlr_logdet_grad.argtypes = [vp, vp, vp, vp, vp]
    lib.hodlr_factor_bytes.argtypes = [vp]
    lib.hodlr_factor_bytes.restype = ctypes.c_size_t
    lib.hodlr_destroy.argtypes = [vp]
    lib.hodlr_destroy.restype = None
    lib.hodlr_status_string.argtypes = [ctypes.c_int]
    lib.hodlr_status_string.restype = ctypes.c_char_p
    lib.hodlr_timing_enable.argtypes = [i32]
    lib.hodlr_timing_enable.restype = None
    lib.hodlr_kernel_times.argtypes = [ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int64), i32]
    lib.hodlr_kernel_times.restype = i32
    lib.hodlr_construct.argtypes = [ctypes.POINTER(_Kernel), i64, i32, ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(i32), ctypes.c_int, vp, i64, vp, i64, vp, i64, vp]
    for name in ("hodlr_factor", "hodlr_refactor", "hodlr_solve", "hodlr_solve_adjoint", "hodlr_solve_noalloc",
                 "hodlr_matvec", "hodlr_grad", "hodlr_logdet", "hodlr_logdet_grad", "hodlr_factors_y",
                 "hodlr_construct"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_dev(t: torch.Tensor, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")


class HODLRMatrix:
    """A HODLR matrix given by its leaf blocks and per-level generators.

    D: (m_max, N) tensor (N x m_max column-major stack of leaf blocks);
    U, V: (R, N) tensors (U_big / V_big); ranks: r_1..r_L;
    leaf_offsets: 2**L + 1 row boundaries (None = uniform).
    """

    def __init__(self, D: torch.Tensor, U: torch.Tensor, V: torch.Tensor, ranks: Sequence[int],
                 leaf_offsets: Optional[Sequence[int]] = None):
        self.ranks = [int(r) for r in ranks]
        self.levels = len(self.ranks)
        self.n = int(D.shape[1])
        self.D, self.U, self.V = D, U, V
        R = sum(self.ranks)
        for t, nm in ((D, "D"), (U, "U"), (V, "V")):
            if t.dtype not in (torch.float64, torch.float32, torch.complex128) or t.dtype != D.dtype:
                raise ValueError("D, U, V must share dtype float64, float32 or complex128")
            if t.dim() != 2 or t.shape[1] != self.n or t.stride(1) != 1 or t.stride(0) < self.n:
                raise ValueError(f"{nm} must be a (k, N) tensor with unit stride along N and row stride >= N")
        if U.shape[0] != R or V.shape[0] != R:
            raise ValueError(f"U and V need sum(ranks) = {R} rows, got {U.shape[0]} and {V.shape[0]}")
        self.leaf_offsets = None if leaf_offsets is None else np.ascontiguousarray(leaf_offsets, dtype=np.int64)
        if self.leaf_offsets is not None:
            if self.leaf_offsets.shape != ((1 << self.levels) + 1,):
                raise ValueError(f"leaf_offsets needs 2**L + 1 = {(1 << self.levels) + 1} entries")
            m_max = int(np.max(np.diff(self.leaf_offsets)))
        else:
            if self.n % (1 << self.levels):
                raise ValueError("a uniform tree needs 2**L to divide N")
            m_max = self.n >> self.levels
        if D.shape[0] < m_max:
            raise ValueError(f"D needs at least the largest leaf size {m_max} rows, got {D.shape[0]}")
        for t, nm in ((D, "D"), (U, "U"), (V, "V")):
            _check_dev(t, nm)
        self._ranks_c = (ctypes.c_int32 * max(1, self.levels))(*self.ranks)
        self._off_c = None if self.leaf_offsets is None else self.leaf_offsets.ctypes.data_as(
            ctypes.POINTER(ctypes.c_int64))

    @classmethod
    def from_inputs(cls, inp) -> "HODLRMatrix":
        return cls(inp.D, inp.U, inp.V, inp.ranks, inp.leaf_offsets)

    def c_struct(self) -> _Matrix:
        m = _Matrix()
        m.n = self.n
        m.levels = self.levels
        m.leaf_offsets = self._off_c if self._off_c is not None else ctypes.POINTER(ctypes.c_int64)()
        m.ranks = self._ranks_c
        m.dtype = {torch.float64: F64, torch.float32: F32, torch.complex128: C128}[self.D.dtype]
        m.D, m.ldd = self.D.data_ptr(), self.D.stride(0)
        m.U, m.ldu = self.U.data_ptr(), self.U.stride(0) if self.U.shape[0] > 1 else self.n
        m.V, m.ldv = self.V.data_ptr(), self.V.stride(0) if self.V.shape[0] > 1 else self.n
        return m

    @property
    def is_complex(self) -> bool:
        return self.D.dtype == torch.complex128

    @property
    def device(self):
        return self.D.device

    def matvec(self, x: torch.Tensor, trans: bool = False) -> torch.Tensor:
        """FP64 product A x (or A^T x); x is (N,) or (nrhs, N)."""
        lib = load_library()
        X, vec = _as_rhs(x, self.n, self.is_complex)
        Y = torch.empty_like(X)
        m = self.c_struct()
        st = lib.hodlr_matvec(ctypes.byref(m), int(trans), X.shape[0], X.data_ptr(), self.n, Y.data_ptr(), self.n,
                              _stream(self.device))
        if st:
            raise HodlrError(st, "hodlr_matvec")
        return Y[0] if vec else Y


def _as_rhs(b: torch.Tensor, n: int, cplx: bool = False):
    _check_dev(b, "right-hand side")
    vec = b.dim() == 1
    B = b.reshape(1, -1) if vec else b
    if B.shape[-1] != n:
        raise ValueError(f"right-hand side must have N={n} entries per column")
    if B.is_complex() and not cplx:
        raise ValueError("complex right-hand side for a real matrix")
    return B.to(torch.complex128 if cplx else torch.float64).contiguous().clone(), vec


class Factors:
    """A factorization owned by the library (freed with the object)."""

    def __init__(self, A: HODLRMatrix, handle: ctypes.c_void_p, precision: str, info: Optional[dict],
                 inplace: bool = False):
        self.A = A
        self._h = handle
        self.precision = precision
        self.info = info
        self.inplace = inplace

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.hodlr_destroy(h)
            self._h = None

    @property
    def nbytes(self) -> int:
        return int(load_library().hodlr_factor_bytes(self._h))

    def refactor(self, A: Optional[HODLRMatrix] = None):
        lib = load_library()
        A = A or self.A
        m = A.c_struct()
        info = _Info()
        st = lib.hodlr_refactor(self._h, ctypes.byref(m), _stream(A.device), ctypes.byref(info))
        if st:
            raise HodlrError(st, "hodlr_refactor")
        self.A = A

    def _solve(self, fn, b, refine, tol, max_iter, out_stats, stream=None):
        lib = load_library()
        X, vec = _as_rhs(b, self.A.n, self.A.is_complex)
        o = _Opts(int(refine), int(max_iter), float(tol))
        s = _Stats()
        sp = _stream(self.A.device) if stream is None else ctypes.c_void_p(stream.cuda_stream)
        st = fn(self._h, X.shape[0], X.data_ptr(), self.A.n, ctypes.byref(o), sp, ctypes.byref(s))
        if out_stats is not None:
            out_stats.update(iters=s.iters, converged=bool(s.converged), relres=s.relres)
        if st and not (st == ERR_NOT_CONVERGED and out_stats is not None):
            raise HodlrError(st, fn.__name__)
        return X[0] if vec else X

    def solve(self, b: torch.Tensor, refine: bool = False, tol: float = 1e-10, max_iter: int = 30,
              stats: Optional[dict] = None, stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
        """x = A^{-1} b (FP64 result); b is (N,) or (nrhs, N).  `stream`: the
        torch stream to run on (default: the current one); b must be ready on it."""
        return self._solve(load_library().hodlr_solve, b, refine, tol, max_iter, stats, stream)

    def solve_adjoint(self, g: torch.Tensor, refine: bool = False, tol: float = 1e-10, max_iter: int = 30,
                      stats: Optional[dict] = None, stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
        """lambda = A^{-T} g (FP64 result; A^{-*} g for a complex A)."""
        return self._solve(load_library().hodlr_solve_adjoint, g, refine, tol, max_iter, stats, stream)

    def solve_noalloc_(self, B: torch.Tensor, adjoint: bool = False) -> torch.Tensor:
        """In place B <- A^{-1} B (or A^{-T} B) through the allocation-free entry
        point: B must be a contiguous (nrhs, N) or (N,) float64 device tensor
        (it is overwritten and returned); no refinement."""
        lib = load_library()
        _check_dev(B, "right-hand side")
        want = torch.complex128 if self.A.is_complex else torch.float64
        if B.dtype != want or not B.is_contiguous() or B.shape[-1] != self.A.n or B.dim() > 2:
            raise ValueError(f"B must be a contiguous {want} (nrhs, N) or (N,) tensor")
        nrhs = 1 if B.dim() == 1 else B.shape[0]
        st = lib.hodlr_solve_noalloc(self._h, int(adjoint), nrhs, B.data_ptr(), self.A.n, _stream(self.A.device))
        if st:
            raise HodlrError(st, "hodlr_solve_noalloc")
        return B

    def noalloc_bytes(self, nrhs: int) -> int:
        return int(load_library().hodlr_solve_noalloc_bytes(self._h, nrhs))

    def slogdet(self):
        """(sign, log|det A|) from the stored factors (sign 0 and -inf for an
        exactly singular pivot)."""
        lib = load_library()
        sg, la = ctypes.c_double(), ctypes.c_double()
        st = lib.hodlr_logdet(self._h, ctypes.byref(sg), ctypes.byref(la), _stream(self.A.device))
        if st:
            raise HodlrError(st, "hodlr_logdet")
        return sg.value, la.value

    def _grad_buffers(self):
        # the library writes dD, dU, dV with the leading dimensions of D, U, V
        A = self.A
        return tuple(torch.empty_strided(t.shape, t.stride(), dtype=t.dtype, device=t.device).zero_()
                     for t in (A.D, A.U, A.V))

    def slogdet_grad(self):
        """(dD, dU, dV) of log|det A| in the layouts and dtype of D, U, V."""
        lib = load_library()
        dD, dU, dV = self._grad_buffers()
        st = lib.hodlr_logdet_grad(self._h, dD.data_ptr(), dU.data_ptr(), dV.data_ptr(), _stream(self.A.device))
        if st:
            raise HodlrError(st, "hodlr_logdet_grad")
        return dD, dU, dV

    def y_big(self) -> torch.Tensor:
        """Y_big as an (R, N) float64 tensor (Y_a = A_a^{-1} U_a per level)."""
        lib = load_library()
        R = sum(self.A.ranks)
        dt = torch.complex128 if self.A.is_complex else torch.float64
        Y = torch.empty(R, self.A.n, dtype=dt, device=self.A.device)
        st = lib.hodlr_factors_y(self._h, Y.data_ptr(), self.A.n, _stream(self.A.device))
        if st:
            raise HodlrError(st, "hodlr_factors_y")
        return Y

    def grad(self, x: torch.Tensor, lam: torch.Tensor):
        """(dD, dU, dV) of a loss with dL/dA = -lam x^T, in the layouts and dtype of D, U, V."""
        lib = load_library()
        X, _ = _as_rhs(x, self.A.n)
        Lm, _ = _as_rhs(lam, self.A.n)
        A = self.A
        dD, dU, dV = self._grad_buffers()
        st = lib.hodlr_grad(self._h, X.shape[0], X.data_ptr(), A.n, Lm.data_ptr(), A.n, dD.data_ptr(),
                            dU.data_ptr(), dV.data_ptr(), _stream(A.device))
        if st:
            raise HodlrError(st, "hodlr_grad")
        return dD, dU, dV


def factor(A: HODLRMatrix, precision: str = "fp64", raise_singular: bool = True, inplace: bool = False) -> Factors:
    """Factorize A (precision: 'fp64', 'fp32' or 'bf16').  inplace=True overwrites
    A.D with the leaf factors and A.U with Y_big (no refinement or gradients then)."""
    lib = load_library()
    m = A.c_struct()
    h = ctypes.c_void_p()
    info = _Info()
    st = lib.hodlr_factor(ctypes.byref(m), _DT[precision], INPLACE if inplace else 0, _stream(A.device),
                          ctypes.byref(h), ctypes.byref(info))
    if st < 0 or (st and raise_singular):
        if h:
            lib.hodlr_destroy(h)
        raise HodlrError(st, "hodlr_factor") if st != ERR_SINGULAR else _singular(info)
    inf = dict(level=info.level, column=info.column, node=info.node) if st == ERR_SINGULAR else None
    return Factors(A, h, precision, inf, inplace)


def construct(kind: str, points: torch.Tensor, ranks: Sequence[int], leaf_offsets: Optional[Sequence[int]] = None,
              ell: float = 1.0, shift: float = 0.0, normals: Optional[torch.Tensor] = None,
              weights: Optional[torch.Tensor] = None, curvature: Optional[torch.Tensor] = None,
              dtype: torch.dtype = torch.float64) -> HODLRMatrix:
    """HODLR approximation of a kernel matrix built on the GPU (hodlr_construct):
    exact leaf blocks and r_l steps of cross approximation with partial
    pivoting per sibling block.  points: (N, dim) float64 on the device
    ('gauss', 'matern32': dim 1..3; 'laplace_dl': dim 2 with (N, 2) unit
    normals, (N,) weights and curvature).  Returns D, U, V in ``dtype``."""
    if kind not in KERNELS:
        raise ValueError(f"kind must be one of {sorted(KERNELS)}")
    lib = load_library()
    n, dim = int(points.shape[0]), int(points.shape[1])
    ranks = [int(r) for r in ranks]
    L = len(ranks)
    if leaf_offsets is not None:
        off = np.ascontiguousarray(leaf_offsets, dtype=np.int64)
        m_max = int(np.max(np.diff(off)))
    else:
        if n % (1 << L):
            raise ValueError("a uniform tree needs 2**L to divide N")
        off, m_max = None, n >> L
    dev = points.device
    P = points.to(torch.float64).t().contiguous()            # N x dim column-major
    keep = [P]
    k = _Kernel()
    k.kind, k.dim, k.points, k.ldp = KERNELS[kind], dim, P.data_ptr(), n
    k.ell, k.shift = float(ell), float(shift)
    if kind == "laplace_dl":
        if normals is None or weights is None or curvature is None:
            raise ValueError("laplace_dl needs normals, weights and curvature")
        Nm = normals.to(torch.float64).t().contiguous()
        Wt = weights.to(torch.float64).contiguous()
        Kp = curvature.to(torch.float64).contiguous()
        for t, nm in ((Nm, "normals"), (Wt, "weights"), (Kp, "curvature")):
            _check_dev(t, nm)
        keep += [Nm, Wt, Kp]
        k.normals, k.weights, k.curvature = Nm.data_ptr(), Wt.data_ptr(), Kp.data_ptr()
    _check_dev(P, "points")
    R = sum(ranks)
    D = torch.empty(m_max, n, dtype=dtype, device=dev)
    U = torch.empty(max(R, 1), n, dtype=dtype, device=dev)[:R]
    V = torch.empty(max(R, 1), n, dtype=dtype, device=dev)[:R]
    rc = (ctypes.c_int32 * max(1, L))(*ranks)
    oc = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if off is not None else ctypes.POINTER(ctypes.c_int64)()
    st = lib.hodlr_construct(ctypes.byref(k), n, L, oc, rc, F64 if dtype == torch.float64 else F32,
                             D.data_ptr(), n, U.data_ptr(), n, V.data_ptr(), n, _stream(dev))
    del keep
    if st != 0:
        raise HodlrError(st, "hodlr_construct")
    return HODLRMatrix(D, U, V, ranks, off)


def _singular(info: _Info) -> HodlrError:
    e = HodlrError(ERR_SINGULAR, f"hodlr_factor (level {info.level}, node {info.node}, column {info.column})")
    e.info = dict(level=info.level, column=info.column, node=info.node)
    return e


def kernel_times(reset: bool = False) -> dict:
    """Per-kernel {name: (total_ms, launches)} recorded with HIP events."""
    lib = load_library()
    cap = 64
    names = (ctypes.c_char_p * cap)()
    ms = (ctypes.c_double * cap)()
    cnt = (ctypes.c_int64 * cap)()
    k = lib.hodlr_kernel_times(names, ms, cnt, cap)
    return {names[i].decode(): (ms[i], cnt[i]) for i in range(min(k, cap))}


def timing(enable: bool):
    load_library().hodlr_timing_enable(1 if enable else 0)


class HodlrSolve(torch.autograd.Function):
    """x = A^{-1} b with gradients for b, D, U, V (adjoint solve on the same factors).

    forward(b, D, U, V, ranks, leaf_offsets, precision, refine) -> x (float64, shape of b).
    refine=True refines the forward and the adjoint solve in FP64 (useful with
    the 'fp32' and 'bf16' factorizations).
    """

    @staticmethod
    def forward(ctx, b, D, U, V, ranks, leaf_offsets=None, precision="fp64", refine=False):
        A = HODLRMatrix(D.detach(), U.detach(), V.detach(), ranks, leaf_offsets)
        F = factor(A, precision)
        x = F.solve(b.detach(), refine=refine)
        ctx.F = F
        ctx.refine = refine
        ctx.b_dtype = b.dtype
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        F = ctx.F
        lam = F.solve_adjoint(gx.detach(), refine=ctx.refine)
        dD, dU, dV = F.grad(x, lam)
        db = lam.to(ctx.b_dtype)
        return db, dD, dU, dV, None, None, None, None
