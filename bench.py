"""Benchmark: HODLR factor + solve on one MI355X.

Workload (default): the Laplace double-layer BIE on the star curve,
N = 1,048,576 Nystrom nodes, leaf 256 (12 levels), rank 32, stored FP64,
one right-hand side ~ N(0,1), synthetic and seeded, generated on the GPU.

A step is one factorization (recomputed in the factors' existing storage)
plus one solve of the right-hand side.  Reported:
  value      factor+solve throughput of the FP64 path in TFLOP/s with the
             paper's operation count (factor: 2/3 m^2 N + 2 m r N L +
             2 r^2 N (L + L^2); solve: 2 m N + 4 r N L)
  fp64 / fp32_ir   per-path factor and solve times, TFLOP/s and the FP64
             relative residual ||b - A x|| / ||b|| (the mixed path refines
             to 1e-10)
  roofline   the dominant kernel's achieved rate from HIP events against
             the MI355X peak
  cpu_baseline  the CPU oracle on a bounded sample of the same workload

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--n N] [--no-cpu] [--no-mixed] [--no-construct]
       python bench.py --construct-only [--config 1|2|3]   (GPU construction of the kernel matrix only)
       python bench.py --copy-probe     (plain device copy, for counter calibration)
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = dict(hbm=8.0e12, f64=78.6e12, f32=157.3e12, bf16=2.5e15)

# HBM traffic of the level pass per launch (one tree level) of the FP64
# factorization at N = 2^20, leaf 256, rank 32, from two rocprofv3 counter runs
# (FETCH_SIZE x 2.0 and WRITE_SIZE x 1.0, the factors that a plain 1 GiB copy
# reads back; summary and commands in profiles/level_pass_traffic_n1m_fp64.md
# and profiles/counters_n1m_synthetic_fp64_fp32_bf16.md).
# It is reported only while the kernel source is the one it was measured on.
LEVEL_PASS_TRAFFIC = dict(
    source_sha256="000a3cfbe028865a382020c1e736d879689e56ac5eadf5b6fe90b1f86aea5e5b",
    n=1 << 20, leaf=256, rank=32, bytes_per_launch=4.2646e9)

# HBM traffic of one cross-approximation step (row + column launch) of the
# construction of the double-layer matrix at N = 2^20, leaf 256, rank 32, from
# the same two counter runs and copy calibration (summary and commands in
# profiles/construct_aca_bie_n1m_fp64.md); reported only for that source.
CONSTRUCT_TRAFFIC = dict(
    source_sha256="477a0a4d62ad1017a94fabf7db84e260b0261532df6c4fee0bca09078fe1bae9",
    n=1 << 20, leaf=256, rank=32, kind="laplace_dl", bytes_per_step=4.2422e9)


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_models(inp, nrhs, tsize):
    """Algorithmic bytes and flops of one launch of each kernel kind, summed over
    the launches of one factorization / one solve (per-launch = total / launches)."""
    N, L = inp.n, inp.levels
    off = inp.leaf_offsets
    m = [int(off[i + 1] - off[i]) for i in range(len(off) - 1)]
    r = inp.ranks
    Rp = [0]
    for x in r:
        Rp.append(Rp[-1] + x)
    R = Rp[-1]
    sb = inp.D.element_size()
    summ2 = sum(mm * mm for mm in m)
    summ3 = sum(mm ** 3 for mm in m)
    mod = {}
    # leaf LU: read D (storage), write LU (compute)
    mod["leaf_lu"] = dict(flops=2.0 / 3.0 * summ3, bytes=summ2 * (sb + tsize), launches=1, bound="mfma")
    # leaf TRSM: read LU, read U (storage), write Y
    mod["leaf_trsm"] = dict(flops=2.0 * summ2 * R, bytes=summ2 * tsize + N * R * (sb + tsize), launches=1, bound="mfma")
    # level passes of the factor: product-only at the leaves, then update + product per level p = L-1..1
    fl = 2.0 * N * r[L - 1] * R
    by = N * R * tsize + N * r[L - 1] * sb
    for p in range(L - 1, 0, -1):
        ka, kb, nz = r[p], r[p - 1], Rp[p]
        fl += 2.0 * N * ka * nz + 2.0 * N * kb * nz
        by += 2.0 * N * nz * tsize + N * ka * tsize + N * kb * sb
    mod["level_pass"] = dict(flops=fl, bytes=by, launches=L)
    # solve: leaf solve reads LU, level passes read Y and V blocks once (x traffic small)
    mod["leaf_solve"] = dict(flops=2.0 * summ2 * nrhs, bytes=summ2 * tsize + 2.0 * N * nrhs * tsize, launches=1)
    sfl = 2.0 * N * r[L - 1] * nrhs
    sby = N * r[L - 1] * sb + N * nrhs * tsize
    for p in range(L - 1, -1, -1):
        ka = r[p]
        kb = r[p - 1] if p > 0 else 0
        sfl += 2.0 * N * (ka + kb) * nrhs
        sby += N * ka * tsize + N * kb * sb + 2.0 * N * nrhs * tsize
    mod["solve_pass"] = dict(flops=sfl, bytes=sby, launches=L + 1)
    return mod


def _timed_path(hodlr, A, precision, B, refine, steps, warmup, adjoint=False):
    """Factor A in `precision` and solve B (nrhs columns), warmup + timed steps.
    A step is one refactorization (in the factors' existing storage) plus one
    solve of all columns (with refinement when `refine`), and with `adjoint` one
    adjoint solve as well.  Returns (results, per-kernel times, factors)."""
    import torch

    _say(f"{precision}: factor + warmup")
    free0 = torch.cuda.mem_get_info()[0]
    F = hodlr.factor(A, precision)
    torch.cuda.synchronize()
    dev_bytes = free0 - torch.cuda.mem_get_info()[0]
    stats, astats = {}, {}
    for _ in range(1 + warmup):
        F.refactor()
        x = F.solve(B, refine=refine, stats=stats)
        if adjoint:
            lam = F.solve_adjoint(B, refine=refine, stats=astats)
    torch.cuda.synchronize()

    def run(k):
        tf = ts = ta = 0.0
        for _ in range(k):
            torch.cuda.synchronize()
            a0 = time.perf_counter()
            F.refactor()            # ends with the singularity verdict (one sync)
            torch.cuda.synchronize()
            a1 = time.perf_counter()
            xx = F.solve(B, refine=refine, stats=stats)
            torch.cuda.synchronize()
            a2 = time.perf_counter()
            if adjoint:
                F.solve_adjoint(B, refine=refine, stats=astats)
                torch.cuda.synchronize()
            a3 = time.perf_counter()
            tf += a1 - a0
            ts += a2 - a1
            ta += a3 - a2
        return tf / k, ts / k, ta / k, xx

    # the headline figures: no per-kernel instrumentation in these steps
    _say(f"{precision}: {steps} timed steps")
    tf, ts, ta, x = run(steps)
    # per-kernel times from HIP events on the launch stream, in a second run of the same steps
    _say(f"{precision}: {steps} steps with per-kernel HIP events")
    hodlr.timing(True)
    run(steps)
    kt = hodlr.kernel_times()
    hodlr.timing(False)
    r = A.matvec(x) - B
    relres = (torch.linalg.vector_norm(r, dim=-1) / torch.linalg.vector_norm(B, dim=-1)).max().item()
    out = dict(t_factor_ms=tf * 1e3, t_solve_ms=ts * 1e3, ms_per_step=(tf + ts) * 1e3, relres=relres,
               refine_iters=stats.get("iters", 0), factor_bytes=F.nbytes, device_bytes_at_factor=int(dev_bytes))
    if adjoint:
        lam = F.solve_adjoint(B, refine=refine, stats=astats)
        ra = A.matvec(lam, trans=True) - B
        out.update(t_adjoint_ms=ta * 1e3, adjoint_relres=(torch.linalg.vector_norm(ra, dim=-1) /
                                                          torch.linalg.vector_norm(B, dim=-1)).max().item(),
                   adjoint_refine_iters=astats.get("iters", 0))
    return out, kt, F


def _kernel_table(kt, mods, steps, peak_flops):
    """Per-kernel averages from HIP events with each modelled kernel's achieved
    rate against its bound; returns (table, roofline of the kernel that takes
    the most time)."""
    per_kernel, roof = {}, None
    ranked = sorted(kt.items(), key=lambda kv: -kv[1][0])
    for name, (ms, cnt) in ranked:
        d = dict(avg_ms=ms / max(cnt, 1), launches_per_step=cnt / steps, total_ms_per_step=ms / steps)
        if name in mods:
            mdl = mods[name]
            avg_s = ms / cnt / 1e3
            fl, by = mdl["flops"] / mdl["launches"], mdl["bytes"] / mdl["launches"]
            # a kernel without a fixed bound is priced against whichever roof its
            # intensity reaches first: HBM below the ridge point, MFMA above it
            bound = mdl.get("bound") or ("mfma" if fl / by > peak_flops / PEAK["hbm"] else "hbm")
            if bound == "mfma":
                d.update(bound="mfma", achieved=fl / avg_s / 1e12, peak=peak_flops / 1e12, unit="TFLOP/s")
            else:
                d.update(bound="hbm", achieved=by / avg_s / 1e9, peak=PEAK["hbm"] / 1e9, unit="GB/s")
            d.update(frac=d["achieved"] / d["peak"], intensity_flop_per_byte=mdl["flops"] / mdl["bytes"])
            if roof is None:
                roof = dict(kernel=name, bound=d["bound"], achieved=d["achieved"], peak=d["peak"], unit=d["unit"],
                            frac=d["frac"])
        per_kernel[name] = d
    return per_kernel, roof


WORKLOADS = {
    1: ("gaussian_kernel_2d", "synthetic (seeded uniform points in [0,1]^2, RCB order, Gaussian kernel "
        "sigma 0.05 + 1e-2 I, randomized range finder to rank 32 on the GPU)"),
    2: ("laplace_dl_bie_star", "synthetic (seeded star-curve Laplace double-layer Nystrom matrix, "
        "ACA-compressed on the GPU)"),
    3: ("matern32_kernel_3d", "synthetic (seeded uniform points in [0,1]^3, RCB order, Matern-3/2 l=0.1 "
        "+ 1e-3 I, randomized range finder to rank 24 on the GPU)"),
    4: ("synthetic_hodlr_fp32_storage", "synthetic (seeded N(0,1) leaf blocks + 1024 I, N(0,1)/sqrt(node size) "
        "generators, stored FP32)"),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2, choices=[1, 2, 3, 4],
                    help="workload: 2 = the headline BIE system (default); 1 = Gaussian kernel, N = 2^18, "
                         "nrhs 1 and 16; 3 = Matern-3/2 in FP32 with the gradient; 4 = N = 2^22, r = 64, BF16 "
                         "factorization, 32 right-hand sides, FP64 refinement and the adjoint")
    ap.add_argument("--n", type=int, default=None, help="override N (same leaf and rank)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP32 and BF16 refinement paths")
    ap.add_argument("--no-construct", action="store_true", help="skip timing the GPU construction of the matrix")
    ap.add_argument("--complex", action="store_true",
                    help="only time factor + solve of the complex Helmholtz-kernel workload (N = 2^17, leaf 128, "
                         "rank 32) through the real embedding")
    ap.add_argument("--construct-only", action="store_true",
                    help="only time the GPU construction of the workload's kernel matrix (no factor / solve)")
    ap.add_argument("--synthetic", action="store_true",
                    help="random generators of the same N, leaf and rank instead of the BIE matrix (same shapes, "
                         "so the same kernels and traffic; used for counter runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU subtree sharding is a design note only)", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W
    from paper_2208_06290_amd import hodlr, model

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        _say("copy probe: 3 copies of 1 GiB (read 1 GiB + write 1 GiB each)")
        return
    cfg = args.config
    c = W.CONFIGS[cfg]
    if args.complex:
        out = complex_bench(hodlr, W, args.n or (1 << 17), args.steps, args.warmup, dev)
        print(json.dumps({"complex": out}), flush=True)
        return
    if args.construct_only:
        if cfg not in (1, 2, 3):
            print("bench.py: --construct-only needs a kernel-matrix workload (--config 1, 2 or 3)", file=sys.stderr)
            sys.exit(2)
        N = args.n or c["n"]
        L = int(round(math.log2(N // c["leaf"])))
        cons = construct_bench(hodlr, W, cfg, N, W.uniform_offsets(N, L), [c["rank"]] * L, args.steps, dev,
                               cpu=not args.no_cpu)
        print(json.dumps({"config": {"workload": WORKLOADS[cfg][0], "N": N, "leaf": c["leaf"], "levels": L,
                                     "rank": c["rank"]}, "construct": cons}), flush=True)
        return
    t0 = time.time()
    if args.synthetic and cfg == 2:
        inp = W.synthetic(args.n or c["n"], c["leaf"], c["rank"], seed=0, dtype=torch.float64, device=dev)
    else:
        inp = W.make_config(cfg, device=dev, n=args.n)
    torch.cuda.synchronize()
    _say(f"generated {inp.name} in {time.time() - t0:.1f}s")
    N = inp.n
    A = hodlr.HODLRMatrix.from_inputs(inp)
    Fp = model.factor_flops_paper(inp.leaf_offsets, inp.ranks)
    ssize = inp.D.element_size()
    paths = {}
    kts = {}

    def flops_of(res, nrhs):
        Sp = model.solve_flops(inp.leaf_offsets, inp.ranks, nrhs)
        res.update(factor_tflops=Fp / res["t_factor_ms"] * 1e-9,
                   tflops=(Fp + Sp) / res["ms_per_step"] * 1e-9)
        return res

    if cfg == 2:
        b = W.gaussian_rhs(N, 1, seed=0, device=dev)
        plan = [("fp64", "fp64", False)]
        if not args.no_mixed:
            plan += [("fp32_ir", "fp32", True), ("bf16_ir", "bf16", True)]
        for key, prec, refine in plan:
            res, kt, F = _timed_path(hodlr, A, prec, b, refine, args.steps, args.warmup)
            _say(f"{key}: releasing the factors")
            del F
            paths[key] = flops_of(res, 1)
            kts[key] = kt
            _say(f"{key}: {paths[key]}")
        head = paths["fp64"]
        nrhs, dtype = 1, "f64"
    elif cfg == 1:
        b1 = W.gaussian_rhs(N, 1, seed=0, device=dev)
        b16 = W.gaussian_rhs(N, 16, seed=1, device=dev)
        res, kt, F = _timed_path(hodlr, A, "fp64", b1, False, args.steps, args.warmup)
        paths["fp64_nrhs1"] = flops_of(res, 1)
        kts["fp64_nrhs1"] = kt
        del F
        res, kt, F = _timed_path(hodlr, A, "fp64", b16, False, args.steps, args.warmup)
        paths["fp64_nrhs16"] = flops_of(res, 16)
        del F
        for k, v in paths.items():
            _say(f"{k}: {v}")
        head = paths["fp64_nrhs1"]
        nrhs, dtype = 1, "f64"
    elif cfg == 3:
        b = W.gaussian_rhs(N, 1, seed=0, device=dev)
        t = W.gaussian_rhs(N, 1, seed=1, device=dev)
        res, kt, F = _timed_path(hodlr, A, "fp32", b, False, args.steps, args.warmup, adjoint=True)
        # one gradient of L = ||x - t||^2: adjoint solve of 2 (x - t), then dD, dU, dV
        x = F.solve(b)
        torch.cuda.synchronize()
        tg = time.perf_counter()
        for _ in range(args.steps):
            lam = F.solve_adjoint(2.0 * (x - t))
            dD, dU, dV = F.grad(x, lam)
        torch.cuda.synchronize()
        res["t_gradient_ms"] = (time.perf_counter() - tg) / args.steps * 1e3
        del F
        paths["fp32"] = flops_of(res, 1)
        kts["fp32"] = kt
        _say(f"fp32: {paths['fp32']}")
        head = paths["fp32"]
        nrhs, dtype = 1, "f32"
    else:  # cfg 4
        B = W.gaussian_rhs(N, c["nrhs"], seed=0, device=dev)
        plan = [("bf16_ir", "bf16")]
        if not args.no_mixed:
            plan.append(("fp32_ir", "fp32"))
        for key, prec in plan:
            res, kt, F = _timed_path(hodlr, A, prec, B, True, args.steps, args.warmup, adjoint=True)
            del F
            paths[key] = flops_of(res, c["nrhs"])
            kts[key] = kt
            _say(f"{key}: {paths[key]}")
        head = paths["bf16_ir"]
        nrhs, dtype = c["nrhs"], "bf16"
    for key, kt in kts.items():
        prec = key.split("_")[0]
        tsize = 8 if prec == "fp64" else 4
        peak = PEAK["f64"] if prec == "fp64" else PEAK["f32"] if prec == "fp32" else PEAK["bf16"]
        mods = kernel_models(inp, nrhs, tsize)
        paths[key]["kernels"], paths[key]["roofline"] = _kernel_table(kt, mods, args.steps, peak)
    headkey = next(iter(kts))
    roof = paths[headkey].get("roofline")
    if roof is not None:
        roof = dict(roof)
        roof["traffic"] = measured_traffic(roof["kernel"], inp) if headkey == "fp64" else None

    cons = None
    if cfg in (1, 2, 3) and not args.no_construct:
        cons = construct_bench(hodlr, W, cfg, N, inp.leaf_offsets, inp.ranks, args.steps, dev, cpu=not args.no_cpu)
        _say(f"construct: {cons}")

    cpu = None
    if not args.no_cpu and cfg == 2:
        _say("cpu baseline: loading the oracle")
        cpu = cpu_baseline(inp, b[0])

    mem = torch.cuda.mem_get_info()
    res = {
        "metric": "factor+solve s & TFLOP/s at N=1M; mixed-prec vs FP64 at rel. residual 1e-10",
        "value": head["tflops"],
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": WORKLOADS[cfg][1] if not (args.synthetic and cfg == 2) else
        "synthetic (seeded random HODLR generators with the BIE workload's N, leaf and rank)",
        "config": {"workload": WORKLOADS[cfg][0], "N": N, "leaf": int(inp.m_max), "levels": inp.levels,
                   "rank": int(inp.ranks[0]) if inp.ranks else 0, "nrhs": nrhs,
                   "storage": "f64" if ssize == 8 else "f32",
                   "flop_count": "paper (factor 2/3 m^2N + 2mrNL + 2r^2N(L+L^2), solve 2mN + 4rNL per rhs)",
                   "matrix_bytes": int(inp.D.numel() + inp.U.numel() + inp.V.numel()) * ssize,
                   "device_total_bytes": int(mem[1])},
        **paths,
        "construct": cons,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


def complex_bench(hodlr, W, n, steps, warmup, dev, leaf=128, rank=32, kappa=20.0):
    """Factor + solve of the complex Helmholtz-kernel matrix (3-D, I + h G,
    rank-`rank` HODLR approximant) in FP64 and FP32 + FP64 refinement.  The
    library factors its real embedding (2N rows, leaf 2 leaf, rank 2 rank);
    TFLOP/s use the paper's count on that real system."""
    import numpy as np
    import torch

    from paper_2208_06290_amd import model

    t0 = time.time()
    inp = W.helmholtz_matrix(n, leaf, rank, kappa=kappa, device=dev)
    torch.cuda.synchronize()
    _say(f"complex: generated {inp.name} in {time.time() - t0:.1f}s")
    A = hodlr.HODLRMatrix.from_inputs(inp)
    b = torch.complex(W.gaussian_rhs(n, 1, seed=0, device=dev), W.gaussian_rhs(n, 1, seed=1, device=dev))
    off2 = 2 * np.asarray(inp.leaf_offsets, dtype=np.int64)
    r2 = [2 * r for r in inp.ranks]
    Fp = model.factor_flops_paper(off2, r2)
    Sp = model.solve_flops(off2, r2, 1)
    out = {"workload": "helmholtz_3d_kernel", "N": n, "leaf": leaf, "levels": inp.levels, "rank": rank,
           "kappa": kappa, "storage": "c128",
           "method": f"real embedding: {2 * n} x {2 * n} real HODLR, leaf {2 * leaf}, rank {2 * rank}",
           "flop_count": "paper's factor and solve counts on the embedded real system"}
    for key, prec, refine in (("fp64", "fp64", False), ("fp32_ir", "fp32", True)):
        res, kt, F = _timed_path(hodlr, A, prec, b, refine, steps, warmup)
        del F
        res.update(factor_tflops=Fp / res["t_factor_ms"] * 1e-9, tflops=(Fp + Sp) / res["ms_per_step"] * 1e-9)
        res["kernels"] = {k: {"ms_per_step": v[0] / steps, "launches_per_step": v[1] / steps} for k, v in kt.items()}
        out[key] = res
        _say(f"complex {key}: {res['t_factor_ms']:.2f} ms factor, {res['t_solve_ms']:.2f} ms solve, "
             f"relres {res['relres']:.2e}")
    return out


def construct_model(N, ranks, m_max, dim, dl, sb):
    """Algorithmic HBM bytes of the construction: the leaf blocks written once;
    per level of rank r and step k, the residual rows read k earlier V entries
    and write one per column, the normalization reads and writes v_k once, the
    residual columns read k earlier U entries and write one per row, and every
    entry evaluated reads its point's coordinates (plus normal and weight for
    the double layer)."""
    pt = 8 * dim + (24 if dl else 0)
    leaves = N * m_max * sb + N * pt
    steps = 0.0
    for r in ranks:
        for k in range(r):
            steps += N * (8 * k + 8) + N * 16 + N * (8 * k + 8) + 2 * N * pt
    return leaves, steps


def construct_bench(hodlr, W, cfg, N, leaf_offsets, ranks, steps, dev, cpu=True):
    """Time hodlr_construct on the workload's kernel matrix (same points, tree
    and ranks as the factorized matrix); roofline of the cross-approximation
    steps against HBM; the construction oracle on a bounded sample."""
    import numpy as np
    import torch

    c = W.CONFIGS[cfg]
    L, ranks = len(ranks), list(ranks)
    m_max = int(np.max(np.diff(leaf_offsets)))
    dtype = torch.float64 if c["storage"] == "f64" else torch.float32
    if cfg == 2:
        g = W.star_curve(N, device=dev)
        kind, pts, dim = "laplace_dl", g["points"], 2
        kw = dict(shift=0.5, normals=g["normals"], weights=g["weights"], curvature=g["curvature"])
    else:
        dim = 2 if cfg == 1 else 3
        kind = "gauss" if cfg == 1 else "matern32"
        pts = torch.as_tensor(W.kernel_points(N, dim, c["leaf"], 0), device=dev)
        kw = dict(ell=0.05 if cfg == 1 else 0.1, shift=1e-2 if cfg == 1 else 1e-3)
    A = hodlr.construct(kind, pts, ranks, dtype=dtype, **kw)  # warm-up
    del A
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        A = hodlr.construct(kind, pts, ranks, dtype=dtype, **kw)
        del A
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    hodlr.timing(True)
    A = hodlr.construct(kind, pts, ranks, dtype=dtype, **kw)
    kt = hodlr.kernel_times()
    hodlr.timing(False)
    del A
    leaves_b, steps_b = construct_model(N, ranks, m_max, dim, kind == "laplace_dl", 8 if dtype == torch.float64 else 4)
    aca_ms = kt.get("aca_step", (float("nan"), 0))[0]
    nsteps = kt.get("aca_step", (0, 0))[1]
    achieved = steps_b / (aca_ms * 1e-3)
    out = {"kernel_matrix": kind, "ms": ms, "method": f"exact leaves + {ranks[0] if ranks else 0}-step cross "
           "approximation with partial pivoting per sibling block, FP64",
           "kernels": {k: {"total_ms": v[0], "launches": v[1]} for k, v in kt.items()},
           "roofline": {"kernel": "aca_step", "bound": "hbm", "achieved": achieved / 1e9, "peak": PEAK["hbm"] / 1e9,
                        "unit": "GB/s", "frac": achieved / PEAK["hbm"], "bytes_per_step": steps_b / max(nsteps, 1),
                        "traffic": construct_traffic(kind, N, m_max, ranks)}}
    if cpu:
        import oracle as O

        n2 = min(N, 8192)
        L2 = int(round(math.log2(n2 // m_max)))
        off2 = np.asarray(leaf_offsets[: (1 << L2) + 1], dtype=np.int64)
        ph = pts[:n2].double().cpu().numpy()
        if kind == "laplace_dl":
            spec = O.KernelSpec(kind, ph, shift=0.5, normals=kw["normals"][:n2].cpu().numpy(),
                                weights=kw["weights"][:n2].cpu().numpy(), curvature=kw["curvature"][:n2].cpu().numpy())
        else:
            spec = O.KernelSpec(kind, ph, ell=kw["ell"], shift=kw["shift"])
        t1 = time.perf_counter()
        O.construct_hodlr(spec, off2, ranks[L - L2:])
        t2 = time.perf_counter()
        out["cpu_oracle"] = {"seconds": t2 - t1, "kind": "oracle",
                             "sample": f"leftmost subtree, N={n2}, {L2} levels, same leaf and rank"}
    return out


def construct_traffic(kind, N, leaf, ranks):
    """Counter-measured HBM bytes per cross-approximation step, or None when no
    measurement matches this workload and the current kernel source."""
    import hashlib

    t = CONSTRUCT_TRAFFIC
    if kind != t["kind"] or N != t["n"] or leaf != t["leaf"] or any(int(r) != t["rank"] for r in ranks):
        return None
    with open(os.path.join(ROOT, "paper_2208_06290_amd", "csrc", "construct.hip"), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != t["source_sha256"]:
            return None
    return t["bytes_per_step"]


def measured_traffic(kernel, inp):
    """Counter-measured HBM bytes per launch of `kernel`, or None when no
    measurement matches this workload and the current kernel source."""
    import hashlib

    t = LEVEL_PASS_TRAFFIC
    if kernel != "level_pass" or inp.n != t["n"] or int(inp.m_max) != t["leaf"]:
        return None
    if any(int(r) != t["rank"] for r in inp.ranks):
        return None
    src = os.path.join(ROOT, "paper_2208_06290_amd", "csrc", "level_pass.hip")
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != t["source_sha256"]:
            return None
    return t["bytes_per_launch"]


def cpu_baseline(inp, b, rows=65536):
    """The oracle (unchanged) on the host: factor + solve of the leftmost subtree
    with `rows` rows (a level-k node, itself a HODLR matrix with L-k levels) of
    the same matrix; TFLOP/s with the paper's operation count."""
    import numpy as np

    import oracle as O
    from paper_2208_06290_amd import model

    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [os.cpu_count() or 1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    k = 0
    while (inp.n >> k) > rows and k < inp.levels:
        k += 1
    n2 = int(inp.leaf_offsets[1 << (inp.levels - k)])
    L2 = inp.levels - k
    off = np.asarray(inp.leaf_offsets[: (1 << L2) + 1], dtype=np.int64)
    c0 = int(sum(inp.ranks[:k]))
    H = O.Hodlr(off, list(inp.ranks[k:]),
                inp.D[:, :n2].double().cpu().numpy().T.copy(),
                inp.U[c0:, :n2].double().cpu().numpy().T.copy(),
                inp.V[c0:, :n2].double().cpu().numpy().T.copy())
    bb = b[:n2].double().cpu().numpy()
    _say(f"cpu baseline: oracle on a level-{k} subtree, N={n2}, {L2} levels, {threads} BLAS threads")
    t0 = time.perf_counter()
    F = O.factor(H)
    t1 = time.perf_counter()
    x = O.solve(F, bb)
    t2 = time.perf_counter()
    _say(f"cpu baseline: factor {t1 - t0:.2f}s solve {t2 - t1:.2f}s")
    fl = model.factor_flops_paper(off, H.ranks) + model.solve_flops(off, H.ranks, 1)
    return {"value": fl / (t2 - t0) / 1e12, "unit": "TFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": f"leftmost level-{k} subtree (N={n2}, {L2} levels, same leaf and rank) of the same matrix, "
                      f"factor + 1 solve: factor {t1 - t0:.2f}s, solve {t2 - t1:.2f}s",
            "seconds": t2 - t0}


if __name__ == "__main__":
    main()
