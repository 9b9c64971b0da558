#!/usr/bin/env python3
"""Benchmark of the mixed-precision flexible-preconditioned kernel solver.

One step = one solve of (K_hat + gamma I) w = y on the kriging-shaped workload
(N = 100,000 points, d = 3, x ~ U[0,10]^3, sigma = 0.5, gamma = 1e-3) with
flexible GMRES: FP64 outer products, Gram-Schmidt (CGS2) and Givens; exactly 10
FP32 inner CG iterations on K_hat + delta I, delta = 10 gamma; restart 100; stop
at true relative residual 1e-6.  Inputs are resident in device memory before
the timed region; the step includes point preparation.

Beside the timed steps, one solve with the paper's inner-accuracy rule (inner
tolerance ten times the outer one, section 6, capped at 100 inner iterations;
no restart) and one plain FP64 CG solve are timed on the same GPU.

Printed (one JSON line): whole-step kernel pair-evaluations per second (value),
the time to a 1e-6 residual for the mixed solver and for plain FP64 CG on the
same GPU, the roofline of the dominant kernel (the FP32 product, timed with HIP
events inside the timed region) and the FP64 CPU oracle's pair rate on a
bounded row sample of the same product.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "kernel-MVP pairs/s + time to 1e-6 residual, mixed-prec FGMRES vs FP64 CG"

# MI355X issue model, from the unit counts (256 CUs x 4 SIMDs, 16 lanes each,
# 2.4 GHz): a wave64 VALU instruction occupies its SIMD 4 cycles (FP32 and FP64
# FMA alike; packed FP32 is not used), a transcendental (v_exp_f32) 8 cycles
# (half rate), a v_mfma_f32_16x16x4f32 32 cycles and a v_mfma_f64_16x16x4f64
# 64 cycles (157.3 and 78.6 TFLOP/s dense).  Matrix-core and VALU instructions
# of one SIMD are counted one after the other: the issue-rate probe
# (krr_probe_issue_rates) measures their mix at the serial sum, not at the
# larger of the two.
SIMD_CYCLES_S = 256 * 4 * 2.4e9
VALU_LANE_OPS = SIMD_CYCLES_S * 16          # FMA lane-ops/s
C_FMA, C_EXP, C_MFMA32, C_MFMA64 = 4, 8, 32, 64
C_MFMA_H32 = 32                              # v_mfma_f32_32x32x16_f16 (1024 outputs x 16 slots)
C_SQRT = 8                                   # v_sqrt_f32, like v_exp_f32
DIMS = (1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64)


def dpad(d: int) -> int:
    """The compiled dimension the library runs d at."""
    return next(p for p in DIMS if p >= d)
C_EXP2_F64 = 15 * C_FMA                     # clamp, rint, subtract, 10 FMAs, convert, ldexp
C_EXP2_F64_TAB = 11 * C_FMA                 # rint, subtract, convert, 4 FMAs, index, shift, table product, ldexp
C_EXP2_F64_TAB4096 = 9 * C_FMA              # the 4096-entry form (d <= 3): 2 FMAs
C_SYM_STEP = 6 * C_FMA                      # symmetric products, per wave-step: the source terms summed
                                            # over the lane rows (permlane swaps, adds) and stored


def sym_group_tiles(n: int) -> int:
    """Tiles per group of the symmetric products for n points (the library's rule)."""
    nt = (n + 255) // 256
    return max(min((nt + 99) // 100, 10), (nt + 511) // 512)


def product_peak(d: int, prec: str = "fp32", n: int | None = None) -> tuple[float, str, str]:
    """Peak pairs/s of the product kernel that runs for dimension d and precision.

    Matrix-core kernels, per 1024 pairs (one wave-step) plus, per lane, 16
    exponentials and 16 FMAs: FP32 / BF16 for d <= 48 (split-f16 kernels)
    ceil((3D + 2) / 16) 32x32x16 f16 matrix-core operations; FP64 for d <= 16
    4 ceil((D + 1) / 4) 16x16x4 FP64 ones (D the compiled dimension; FP64
    exponentials from the 256-entry table, 11 instructions; 9 with the
    4096-entry table at d <= 3), the same model for
    FP64 at d > 16 (staged kernel).  Otherwise (VALU kernel) per 64 pairs: d + 1
    FMAs and one exponential per lane.  Matrix-core
    and VALU issue counted one after the other (measured by the issue probe).
    """
    tag = {"fp64": "FP64", "bf16": "BF16"}.get(prec, "FP32")
    valu = os.environ.get("KRR_KMVP_VALU", "0") == "1"
    if 16 < d <= 48 and prec != "fp64" and not valu:
        D = dpad(d)
        kc = (3 * D + 2 + 15) // 16
        cyc = kc * C_MFMA_H32 + 16 * (C_EXP + C_FMA)
        rule = (f"1024 pairs per {cyc} SIMD cycles: {kc} 32x32x16 f16 matrix-core ops + 16 x (exp2 + FMA) "
                f"per lane, serial issue; 1024 SIMDs x 2.4 GHz")
        return SIMD_CYCLES_S * 1024 / cyc, rule, f"k_kmvp_mhw<{D}, {tag}>"
    if ((16 < d and prec == "fp64") or d > 48) and not valu:
        D = dpad(d)
        dk = (D + 4) // 4
        if prec == "fp64":
            cyc = 4 * dk * C_MFMA64 + 16 * (C_EXP2_F64_TAB + C_FMA)
        else:
            cyc = 4 * dk * C_MFMA32 + 16 * (C_EXP + C_FMA)
        rule = (f"1024 pairs per {cyc} SIMD cycles: {4 * dk} 16x16x4 matrix-core ops + 16 x (exp2 + FMA) per "
                f"lane, serial issue; 1024 SIMDs x 2.4 GHz")
        return SIMD_CYCLES_S * 1024 / cyc, rule, f"k_kmvp_mgw<{D}, {tag}>"
    if d <= 16 and prec == "fp64" and not valu and os.environ.get("KRR_KMVP_SYM", "1") != "0":
        # symmetric FP64 product: per wave-step 1024 evaluated pairs serve 2048
        # terms (16 x (exp2 + 2 FMAs) per lane)
        D = dpad(d)
        dk = (D + 4) // 4
        cyc = 4 * dk * C_MFMA64 + 16 * ((C_EXP2_F64_TAB4096 if D <= 3 else C_EXP2_F64_TAB) + 2 * C_FMA) + C_SYM_STEP
        rule = (f"2048 pair terms (1024 exponentials) per {cyc} SIMD cycles: {4 * dk} 16x16x4 FP64 matrix-core ops + "
                f"16 x (exp2 + 2 FMAs) per lane + the source-term reduction, serial issue; 1024 SIMDs x 2.4 GHz")
        return SIMD_CYCLES_S * 2048 / cyc, rule, f"k_kmvp_ms<{D}>"
    sym32 = d <= 12 or (d <= 16 and n is not None and sym_group_tiles(n) >= 8)  # square products of n points
    if (sym32 and prec != "fp64" and not valu and os.environ.get("KRR_KMVP_SYM", "1") != "0"
            and os.environ.get("KRR_KMVP_MG32", "0") != "1"):
        # symmetric split-f16 product: per wave-step ceil((3D + 2) / 16) 32x32x16
        # f16 ops form 1024 exponentials that serve 2048 terms (16 x (exp2 +
        # 2 FMAs) per lane)
        D = dpad(d)
        kc = (3 * D + 2 + 15) // 16
        cyc = kc * C_MFMA_H32 + 16 * (C_EXP + 2 * C_FMA) + C_SYM_STEP
        rule = (f"2048 pair terms (1024 exponentials) per {cyc} SIMD cycles: {kc} 32x32x16 f16 matrix-core op(s) + "
                f"16 x (exp2 + 2 FMAs) per lane + the source-term reduction, serial issue; 1024 SIMDs x 2.4 GHz")
        return SIMD_CYCLES_S * 2048 / cyc, rule, f"k_kmvp_mhs<{D}, {tag}>"
    if d <= 16 and not valu:
        D = dpad(d)
        if prec != "fp64" and os.environ.get("KRR_KMVP_MG32", "0") != "1":
            kc = (3 * D + 2 + 15) // 16
            cyc = kc * C_MFMA_H32 + 16 * (C_EXP + C_FMA)
            rule = (f"1024 pairs per {cyc} SIMD cycles: {kc} 32x32x16 f16 matrix-core op(s) + 16 x (exp2 + FMA) "
                    f"per lane, serial issue; 1024 SIMDs x 2.4 GHz")
            return SIMD_CYCLES_S * 1024 / cyc, rule, f"k_kmvp_mh<{D}, {tag}>"
        dk = (D + 4) // 4
        if prec == "fp64":
            cyc = 4 * dk * C_MFMA64 + 16 * ((C_EXP2_F64_TAB4096 if D <= 3 else C_EXP2_F64_TAB) + C_FMA)
        else:
            cyc = 4 * dk * C_MFMA32 + 16 * (C_EXP + C_FMA)
        rule = (f"1024 pairs per {cyc} SIMD cycles: {4 * dk} 16x16x4 matrix-core ops + 16 x (exp2 + FMA) per "
                f"lane, serial issue; 1024 SIMDs x 2.4 GHz")
        return SIMD_CYCLES_S * 1024 / cyc, rule, f"k_kmvp_mg<{D}, {tag}>"
    if prec == "fp64":
        cyc = (d + 1) * C_FMA + C_EXP2_F64
    else:
        cyc = (d + 1) * C_FMA + C_EXP
    rule = f"64 pairs per {cyc} SIMD cycles: (d + 1) FMAs + exp2 per lane; 1024 SIMDs x 2.4 GHz"
    kname = f"k_kmvp_hd<{dpad(d)}, {tag}, gauss>" if d > 16 else f"k_kmvp<{dpad(d)}, {tag}>"
    return SIMD_CYCLES_S * 64 / cyc, rule, kname


def matern_peak(d: int) -> tuple[float, str, str]:
    """Peak pairs/s of the FP32 Matern-3/2 product.  d <= 16 (square products):
    the symmetric split-f16 kernel, per 2048 pair terms the one-sided step's
    operations with 4 FMA-class ops per pair plus the source-term reduction.
    d <= 48 (one-sided split-f16 kernels),
    per 1024 pairs: ceil((3D + 4) / 16) 32x32x16 f16 matrix-core operations and,
    per lane, 16 x (sqrt + exp2 + 2 FMAs), serial issue (v_sqrt_f32 costs 8
    cycles, as v_exp_f32).  Otherwise (VALU kernel) per 64 pairs: 2d + 3
    FMA-class operations, sqrt and exp2 per lane."""
    sym = d <= 16  # square products (the Matern form at every group size)
    if (sym and os.environ.get("KRR_KMVP_VALU", "0") != "1" and os.environ.get("KRR_KMVP_SYM", "1") != "0"
            and os.environ.get("KRR_KMVP_MG32", "0") != "1"):
        # symmetric split-f16 form (square products): per wave-step 1024 kernel
        # values serve 2048 terms, 16 x (sqrt + exp2 + 4 FMA-class ops) per lane
        D = dpad(d)
        kc = (3 * D + 4 + 15) // 16
        cyc = kc * C_MFMA_H32 + 16 * (C_SQRT + C_EXP + 4 * C_FMA) + C_SYM_STEP
        rule = (f"2048 pair terms (1024 kernel values) per {cyc} SIMD cycles: {kc} 32x32x16 f16 matrix-core op(s) + "
                f"16 x (sqrt + exp2 + 4 FMA-class ops) per lane + the source-term reduction, serial issue; "
                f"1024 SIMDs x 2.4 GHz")
        return SIMD_CYCLES_S * 2048 / cyc, rule, f"k_kmvp_mhs<{D}, FP32, matern>"
    if d <= 48 and os.environ.get("KRR_KMVP_VALU", "0") != "1":
        D = dpad(d)
        kc = (3 * D + 4 + 15) // 16
        cyc = kc * C_MFMA_H32 + 16 * (C_SQRT + C_EXP + 2 * C_FMA)
        rule = (f"1024 pairs per {cyc} SIMD cycles: {kc} 32x32x16 f16 matrix-core op(s) + 16 x (sqrt + exp2 + "
                f"2 FMA) per lane, serial issue; 1024 SIMDs x 2.4 GHz")
        kname = f"k_kmvp_mh<{D}, FP32, matern>" if d <= 16 else f"k_kmvp_mhw<{D}, FP32, matern>"
        return SIMD_CYCLES_S * 1024 / cyc, rule, kname
    cyc = (2 * d + 3) * C_FMA + C_SQRT + C_EXP
    rule = f"64 pairs per {cyc} SIMD cycles: 2d + 3 FMA-class ops + sqrt + exp2 per lane"
    kname = f"k_kmvp_hd<{dpad(d)}, FP32, matern>" if d > 16 else f"k_kmvp_matern<{dpad(d)}, FP32>"
    return SIMD_CYCLES_S * 64 / cyc, rule, kname


def multi_peak(d: int) -> tuple[float, str, str]:
    """Peak pair x RHS products/s of the FP32 16-RHS product, per 16 sources x 16
    targets x 16 RHS (one wave step), serial issue.  d <= 16 (split-f16 exponent):
    ceil(2 ceil((3D + 4) / 16) / 4) 16x16x32 f16 operations (16 cycles each),
    4 exp2 per lane and four 16x16x4 FP32 operations.  Otherwise: four FP32
    operations and, per lane, 4 x (d FMAs + exp2)."""
    if d <= 16 and os.environ.get("KRR_KMVP_MULTI_VALU", "0") != "1":
        D = dpad(d)
        kc = (2 * ((3 * D + 4 + 15) // 16) + 3) // 4
        cyc = kc * 16 + 4 * C_EXP + 4 * C_MFMA32
        rule = (f"4096 pair-RHS per {cyc} SIMD cycles: {kc} 16x16x32 f16 op(s) for the exponents, 4 exp2 per lane, "
                f"four 16x16x4 FP32 ops for 16 RHS, serial issue; 1024 SIMDs x 2.4 GHz")
        return SIMD_CYCLES_S * 4096 / cyc, rule, f"k_kmvp_multi<{D}, FP32, split-f16>"
    cyc = 4 * C_MFMA32 + 4 * (d * C_FMA + C_EXP)
    rule = (f"4096 pair x RHS per {cyc} SIMD cycles: 4 16x16x4 matrix-core ops + 4 x (d FMAs + exp2) per lane, "
            "serial issue; 1024 SIMDs x 2.4 GHz")
    return SIMD_CYCLES_S * 4096 / cyc, rule, f"k_kmvp_multi<{d}, FP32>"


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the split-f16 product kernel's source section; the committed
    counter summary is used only while it matches."""
    src = open(os.path.join(ROOT, "paper_1408_1237_amd", "csrc", "kmvp.hip")).read()
    a = src.index("// ---------------------------------------------------------------- split-f16 matrix-core exponent")
    b = src.index("// qw_j = q_j * w_j", a)
    return hashlib.sha256(src[a:b].encode()).hexdigest()[:16]


def read_traffic(name: str):
    """Per-launch HBM bytes of the product kernel from the committed counter summary."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith("traffic:"):
            for kv in line.split()[1:]:
                k, v = kv.split("=")
                vals[k] = v
    if vals.get("source_hash") != kernel_source_hash():
        return None
    try:
        return float(vals["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(p, target_s: float = 10.0) -> dict:
    """FP64 oracle kernel sum on a bounded sample of rows (OpenMP over rows), on
    all host threads and on one."""
    import numpy as np

    import oracle
    from paper_1408_1237_amd import workloads

    q = workloads.random_vector(7, p.n)
    rng = np.random.default_rng(0)

    def rate(budget_s: float):
        rows = rng.choice(p.n, 64, replace=False)
        t0 = time.perf_counter()
        oracle.mvp_rows(p.x, p.sigma, q, rows, shift=p.gamma)
        dt = time.perf_counter() - t0
        nrows = int(min(p.n, max(64, 64 * budget_s / max(dt, 1e-3))))
        rows = rng.choice(p.n, nrows, replace=False)
        t0 = time.perf_counter()
        oracle.mvp_rows(p.x, p.sigma, q, rows, shift=p.gamma)
        dt = time.perf_counter() - t0
        return float(nrows) * p.n / dt, nrows, dt

    threads = oracle.num_threads()
    v_all, nr_all, dt_all = rate(target_s)
    oracle.set_num_threads(1)
    try:
        v_one, nr_one, dt_one = rate(target_s / 2)
    finally:
        oracle.set_num_threads(threads)
    return {"value": v_all, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": f"{nr_all} rows x {p.n} sources of (K_hat + gamma I) q, FP64 on-the-fly loop, {dt_all:.1f} s "
                      f"on {threads} threads",
            "value_1thread": v_one,
            "sample_1thread": f"{nr_one} rows x {p.n} sources, {dt_one:.1f} s on 1 thread",
            "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count()}


def plain_small_block(api, torch) -> dict:
    """The small plain case (N = 2000, d = 2, sigma = 0.1, gamma = 1e-2): the
    oracle's FP64 CG and Cholesky solve on the host against the GPU's plain FP64
    CG and mixed FGMRES (delta = 0.1, 10 inner iterations), each to 1e-6."""
    import oracle
    from paper_1408_1237_amd import workloads

    p = workloads.plain_small()
    x = torch.from_numpy(p.x).cuda()
    y = torch.from_numpy(p.y).cuda()
    out = {"workload": "N=2000 d=2 x~U[0,1]^2 sigma=0.1 gamma=1e-2", "cpu_threads": oracle.num_threads()}
    t0 = time.perf_counter()
    wd = oracle.direct_solve(p.x, p.sigma, p.gamma, p.y)
    out["cpu_cholesky_s"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, st, it, rel, _ = oracle.cg(p.x, p.sigma, p.gamma, p.y, 20000, p.tol)
    out["cpu_cg64"] = {"time_s": time.perf_counter() - t0, "iters": it, "relres_true": rel}
    for label, mode, kw in (("gpu_cg64", "cg64", dict(max_outer=20000)),
                            ("gpu_fgmres", "fgmres", dict(inner_prec="fp32", inner_maxit=p.inner_maxit,
                                                          inner_tol=0.0, delta=p.delta, restart_m=100, gs="cgs2"))):
        api.krr_solve([x], [p.sigma], [p.gamma], [y], mode=mode, **kw)  # tunes the products
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        (w,), (i,) = api.krr_solve([x], [p.sigma], [p.gamma], [y], mode=mode, **kw)
        torch.cuda.synchronize()
        wn = w.cpu().numpy()
        out[label] = {"time_s": time.perf_counter() - t0, "iters": i["outer_iters"], "inner_iters": i["inner_iters"],
                      "relres_true": oracle.true_relres(p.x, p.sigma, p.gamma, p.y, wn),
                      "rel_err_vs_cholesky": float(((wn - wd) ** 2).sum() ** 0.5 / (wd ** 2).sum() ** 0.5)}
    return out


def kernel_only(api, native, workloads, torch, p, x, reps: int, prec: str = "fp32") -> int:
    """Repeated products (through the C ABI, which also prepares the points each
    call) and one plain copy of known size for counter calibration."""
    q = torch.from_numpy(workloads.random_vector(7, p.n)).cuda()
    q = q if prec == "fp64" else q.float()
    ws = api.workspace(native.workspace_size(native.KRR_WS_KMVP, [(p.n, p.d)]), x.device)
    api.kmvp_gauss(x, p.sigma, q, shift=p.delta, prec=prec, ws=ws)  # tunes the plan
    torch.cuda.synchronize()
    with native.profile() as prof:
        for _ in range(reps):
            api.kmvp_gauss(x, p.sigma, q, shift=p.delta, prec=prec, ws=ws)
        torch.cuda.synchronize()
    a = torch.ones(64 << 20, dtype=torch.float32, device=x.device)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    st = prof.stats[prec]
    ach = st["pairs"] / (st["total_ms"] * 1e-3) / 1e9
    print(json.dumps({"mode": "kernel-only", "prec": prec, "n": p.n, "d": p.d, "launches": st["launches"],
                      "avg_launch_ms": st["total_ms"] / max(st["launches"], 1), "gpair_s": ach,
                      "skipped_frac": st["pairs_skipped"] / max(st["pairs"], 1.0),
                      "copy_bytes": 2 * a.numel() * 4}), flush=True)
    return 0


def product_rates(api, native, torch, x, sigma, shift, n, reps, precs=("fp64", "fp32", "bf16")) -> dict:
    """Average product-kernel launch time and pair rate per precision (HIP
    events), with the share of pairs in far tile pairs the kernels skipped
    (exact zeros) and the rate over the pairs they evaluated."""
    out = {}
    for prec in precs:
        dt = torch.float64 if prec == "fp64" else torch.float32
        q = torch.randn(n, dtype=torch.float64, device=x.device, generator=None).to(dt)
        api.kmvp_gauss(x, sigma, q, shift=shift, prec=prec)  # tunes the plan
        torch.cuda.synchronize()
        with native.profile() as prof:
            for _ in range(reps):
                api.kmvp_gauss(x, sigma, q, shift=shift, prec=prec)
            torch.cuda.synchronize()
        st = prof.stats[prec]
        sec = st["total_ms"] * 1e-3
        out[prec] = {"gpair_s": round(st["pairs"] / sec / 1e9, 1),
                     "avg_launch_ms": round(st["total_ms"] / max(st["launches"], 1), 4), "launches": st["launches"],
                     "skipped_frac": round(st["pairs_skipped"] / max(st["pairs"], 1.0), 4),
                     "evaluated_gpair_s": round((st["pairs"] - st["pairs_skipped"]) / sec / 1e9, 1)}
    return out


def workload_clustered(args, api, native, workloads, torch) -> dict:
    """N = 1e6, d = 2 clustered points (50-component mixture, sigma = 1,
    gamma = 1e-4): product rates per precision, then the mixed solve to a true
    relative residual of 1e-6 (FP64 outer products, BF16-input inner CG on
    K_hat + 1e-3 I, inner tolerance 1e-5 and at most 10 inner iterations, or
    --inner-maxit), and plain FP64 CG given the same wall time (the residual it
    reaches is reported)."""
    p = workloads.clustered_large()
    if args.gamma > 0:  # the same points with another regulariser (delta = 10 gamma)
        p.gamma, p.delta = args.gamma, 10 * args.gamma
    x = torch.from_numpy(p.x).cuda()
    y = torch.from_numpy(p.y).cuda()
    torch.manual_seed(7)
    os.environ.setdefault("KRR_PROGRESS", "25")
    rates = product_rates(api, native, torch, x, p.sigma, p.delta, p.n, 3)
    log(f"clustered products: {rates}")
    if args.cg_only:
        # plain FP64 CG alone for --max-outer iterations (its comparison run)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        (wc,), (ic,) = api.krr_solve([x], [p.sigma], [p.gamma], [y], mode="cg64", tol=p.tol,
                                     max_outer=args.max_outer or 1000, cg_check=16)
        torch.cuda.synchronize()
        tc = time.perf_counter() - t0
        log(f"cg64 alone, {ic['outer_iters']} iterations: status {ic['status']}, relres {ic['relres_true']:.3e}, "
            f"{tc:.2f} s")
        return {"metric": METRIC, "value": tc, "unit": "s", "n_gpus": 1, "dtype": "f64", "data": "synthetic",
                "higher_is_better": False, "vs_baseline": None,
                "config": {"workload": f"clustered N=1e6 d=2 sigma=1 gamma={p.gamma:g}; plain FP64 CG for "
                                       f"{args.max_outer or 1000} iterations", "n": p.n, "d": p.d},
                "products": rates,
                "cg64": {"iters": ic["outer_iters"], "relres_true": ic["relres_true"], "time_s": tc,
                         "status": ic["status"]}}
    inner_maxit = args.inner_maxit or p.inner_maxit
    inner_prec = args.inner_prec or "bf16"
    opts = dict(inner_prec=inner_prec, inner_maxit=inner_maxit, inner_tol=p.inner_tol, delta=p.delta,
                restart_m=args.restart or 200, tol=p.tol, max_outer=args.max_outer or 3000, gs="cgs2")
    torch.cuda.synchronize()
    with native.profile(max_launches=200_000) as prof:
        t0 = time.perf_counter()
        w, info = api.fgmres_solve(x, p.sigma, p.gamma, y, **opts)
        torch.cuda.synchronize()
        tf = time.perf_counter() - t0
    log(f"fgmres bf16 inner: status {info['status']}, {info['outer_iters']} outer, {info['inner_iters']} inner, "
        f"relres {info['relres_true']:.3e}, {tf:.2f} s")
    st = prof.stats
    # plain FP64 CG with the same wall time: iterations from the FP64 product time
    t_it = rates["fp64"]["avg_launch_ms"] * 1e-3 + 1e-4
    cg_iters = max(16, int(tf / t_it) // 16 * 16)
    ic, tc = {"outer_iters": 0, "relres_true": None, "status": None}, 0.0
    if not args.no_cg:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        (wc,), (ic,) = api.krr_solve([x], [p.sigma], [p.gamma], [y], mode="cg64", tol=p.tol, max_outer=cg_iters,
                                     cg_check=16)
        torch.cuda.synchronize()
        tc = time.perf_counter() - t0
        log(f"cg64 given {cg_iters} iterations (the same wall time): status {ic['status']}, "
            f"relres {ic['relres_true']:.3e}, {tc:.2f} s")
    peak_pairs, peak_rule, kname = product_peak(p.d, prec="bf16")
    ach = rates["bf16"]["evaluated_gpair_s"]
    return {"metric": METRIC, "value": rates["bf16"]["gpair_s"] * 1e9, "unit": "pairs/s", "n_gpus": 1,
            "dtype": "bf16-input/f32 + f64", "data": "synthetic", "higher_is_better": True, "vs_baseline": None,
            "config": {"workload": f"clustered N=1e6 d=2 50-component mixture sigma=1 gamma={p.gamma:g}; FGMRES FP64 "
                                   f"outer, {inner_prec} inner CG ({inner_maxit} its, tol 1e-5) on K_hat+{p.delta:g} I, "
                                   "tol 1e-6",
                       "n": p.n, "d": p.d},
            "roofline": {"bound": "alu", "achieved": ach, "peak": round(peak_pairs / 1e9, 1), "unit": "Gpair/s",
                         "frac": round(ach * 1e9 / peak_pairs, 4), "traffic": None, "kernel": kname,
                         "peak_rule": peak_rule + "; achieved over the evaluated (not skipped) pairs"},
            "products": rates,
            "fgmres": {"status": info["status"], "outer_iters": info["outer_iters"],
                       "inner_iters": info["inner_iters"], "mvp64": info["mvp64"], "mvp16": info["mvp16"],
                       "relres_true": info["relres_true"], "time_to_solution_s": tf,
                       "t_prep_ms": info["t_prep_ms"], "t_inner_ms": info["t_inner_ms"],
                       "t_outer_ms": info["t_outer_ms"], "t_ortho_ms": info["t_ortho_ms"],
                       "product_ms": {k: round(st[k]["total_ms"], 1) for k in ("fp64", "bf16")},
                       "skipped_frac": {k: round(st[k]["pairs_skipped"] / max(st[k]["pairs"], 1.0), 4)
                                        for k in ("fp64", "bf16")}},
            "cg64_same_wall_time": {"iters": ic["outer_iters"], "relres_true": ic["relres_true"], "time_s": tc,
                                    "status": ic["status"]}}


def workload_batched(args, api, native, workloads, torch) -> dict:
    """64 systems (N_k ~ U{1000..50000}, d in {4, 8}) x 16 right-hand sides: the
    batched mixed FGMRES and the batched plain FP64 CG, each to 1e-6 on every
    column; the multi-RHS kernel rate on the largest system."""
    import numpy as np

    # the library prints a progress line every 50 outer steps (a long solve is one call)
    os.environ.setdefault("KRR_PROGRESS", "50")
    probs = workloads.batched()
    xs = [torch.from_numpy(q.x).cuda() for q in probs]
    Ys = [torch.from_numpy(np.asfortranarray(q.y)).cuda() for q in probs]
    opts = dict(inner_prec="fp32", inner_maxit=args.inner_maxit or 10, inner_tol=args.inner_tol,
                restart_m=args.restart or 30, max_outer=args.max_outer or 3000)
    torch.cuda.synchronize()
    with native.profile(max_launches=200_000) as prof:
        t0 = time.perf_counter()
        Ws, infos = api.krr_solve(xs, [q.sigma for q in probs], [q.gamma for q in probs], Ys, mode="fgmres", **opts)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
    worst = max(i["relres_true"] for i in infos)
    steps = infos[0]["batch_steps"]
    log(f"batched fgmres: {len(infos)} columns, {steps} outer steps, worst relres {worst:.3e}, {tb:.2f} s, "
        f"tile {infos[0]['batch_tiles']}, prep {infos[0]['t_prep_ms']:.0f} ms")
    ic, tcg, worst_cg = [{"batch_steps": 0, "outer_iters": 0}], float("nan"), float("nan")
    if not args.no_cg:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Wc, ic = api.krr_solve(xs, [q.sigma for q in probs], [q.gamma for q in probs], Ys, mode="cg64",
                               max_outer=args.max_outer or 20000, cg_check=16)
        torch.cuda.synchronize()
        tcg = time.perf_counter() - t0
        worst_cg = max(i["relres_true"] for i in ic)
        log(f"batched cg64: {ic[0]['batch_steps']} iterations (max column {max(i['outer_iters'] for i in ic)}), "
            f"worst relres {worst_cg:.3e}, {tcg:.2f} s")
    big = max(range(len(probs)), key=lambda k: probs[k].n)
    q = probs[big]
    rates = {}
    for prec in ("fp32", "fp64"):
        dt = torch.float64 if prec == "fp64" else torch.float32
        Q = torch.randn(16, q.n, dtype=torch.float64, device="cuda").to(dt).t()
        api.kmvp_gauss_multi(xs[big], q.sigma, Q, shift=q.gamma, prec=prec)
        torch.cuda.synchronize()
        with native.profile() as pr:
            for _ in range(5):
                api.kmvp_gauss_multi(xs[big], q.sigma, Q, shift=q.gamma, prec=prec)
            torch.cuda.synchronize()
        st = pr.stats[prec]
        rates[prec] = {"gpair_rhs_s": round(st["pairs"] / (st["total_ms"] * 1e-3) / 1e9, 1),
                       "avg_launch_ms": round(st["total_ms"] / max(st["launches"], 1), 4)}
    log(f"multi-RHS products on the largest system (n={q.n}, d={q.d}): {rates}")
    peak_pairs, peak_rule, kname = multi_peak(q.d)
    ach = rates["fp32"]["gpair_rhs_s"]
    return {"metric": METRIC, "value": tb, "unit": "s (time to 1e-6 on all 1024 columns)", "n_gpus": 1,
            "dtype": "f32+f64", "data": "synthetic", "higher_is_better": False, "vs_baseline": None,
            "config": {"workload": f"batched 64 systems N_k~U{{1000..50000}} d in {{4,8}} x 16 RHS; "
                                   f"FGMRES({opts['restart_m']}), {opts['inner_maxit']} FP32 inner CG"
                                   + (f" (tol {opts['inner_tol']:g})" if opts["inner_tol"] > 0 else "")
                                   + " on K_hat+0.1 I, tol 1e-6 per column"},
            "time_to_solution_s": tb, "outer_steps": steps, "worst_relres_true": worst,
            "max_column_outer": max(i["outer_iters"] for i in infos),
            "batch_tiles": infos[0]["batch_tiles"], "t_prep_ms": infos[0]["t_prep_ms"],
            "cg64": {"time_to_solution_s": tcg, "iterations": ic[0]["batch_steps"],
                     "max_column_iters": max(i["outer_iters"] for i in ic), "worst_relres_true": worst_cg},
            "speedup_fgmres_vs_cg64": tcg / tb,
            "roofline": {"bound": "mfma", "achieved": ach, "peak": round(peak_pairs / 1e9, 1),
                         "unit": "Gpair-RHS/s", "frac": round(ach * 1e9 / peak_pairs, 4), "traffic": None,
                         "kernel": kname, "peak_rule": peak_rule},
            "multi_products_largest_system": rates}


def workload_gp(args, api, native, workloads, torch) -> dict:
    """N = 2e5, d = 16: forward solve, then the gradient pass of y^T K^-1 y
    (lambda = w)."""
    p = workloads.gp_regression()
    x = torch.from_numpy(p.x).cuda()
    y = torch.from_numpy(p.y).cuda()
    os.environ.setdefault("KRR_PROGRESS", "100")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    w, info = api.fgmres_solve(x, p.sigma, p.gamma, y, inner_prec="fp32", inner_maxit=p.inner_maxit,
                               inner_tol=p.inner_tol, delta=p.delta, restart_m=100, gs="cgs2",
                               max_outer=args.max_outer or 3000)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    log(f"gp forward solve: {info['outer_iters']} outer, relres {info['relres_true']:.3e}, {ts:.2f} s")
    # the paper's inner rule (inner tolerance 10x the outer one, at most 100
    # inner iterations) and plain FP64 CG on the same system
    t0 = time.perf_counter()
    wp, ip = api.fgmres_solve(x, p.sigma, p.gamma, y, inner_prec="fp32", inner_maxit=100, inner_tol=10 * p.tol,
                              delta=p.delta, restart_m=1000, gs="cgs2", max_outer=args.max_outer or 1000)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    log(f"gp fgmres (paper inner rule): {ip['outer_iters']} outer, {ip['inner_iters']} inner, "
        f"relres {ip['relres_true']:.3e}, {tp:.2f} s")
    t0 = time.perf_counter()
    (wc,), (ic,) = api.krr_solve([x], [p.sigma], [p.gamma], [y], mode="cg64", tol=p.tol,
                                 max_outer=args.max_outer or 20000, cg_check=32)
    torch.cuda.synchronize()
    tc = time.perf_counter() - t0
    log(f"gp cg64: {ic['outer_iters']} iterations, relres {ic['relres_true']:.3e}, {tc:.2f} s")
    d = p.d
    times = {}
    for prec in ("fp64", "fp32"):
        api.kmvp_grad(x, p.sigma, p.gamma, w, w, prec=prec)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 3
        e0.record()
        for _ in range(reps):
            api.kmvp_grad(x, p.sigma, p.gamma, w, w, prec=prec)
        e1.record()
        torch.cuda.synchronize()
        times[prec] = e0.elapsed_time(e1) / reps
    rate = float(p.n) ** 2 / (times["fp64"] * 1e-3)
    # FP64 pair loop: 3d + 3 slots plus the exp2_f64 sequence (clamp, rint, subtract,
    # 10 FMAs, convert, ldexp: 15); FP32: 3d + 3
    peak = SIMD_CYCLES_S * 64 / ((3 * d + 3) * C_FMA + C_EXP2_F64)
    log(f"gradient pass: fp64 {times['fp64']:.2f} ms ({rate / 1e9:.1f} Gpair/s), fp32 {times['fp32']:.2f} ms")
    return {"metric": METRIC, "value": rate, "unit": "pairs/s", "n_gpus": 1, "dtype": "f64",
            "data": "synthetic", "higher_is_better": True, "vs_baseline": None,
            "config": {"workload": "gp_regression N=2e5 d=16 sigma=4 gamma=1e-2: gradient of y^T K^-1 y", "n": p.n,
                       "d": d},
            "forward_solve": {"time_s": ts, "outer_iters": info["outer_iters"], "relres_true": info["relres_true"],
                              "t_inner_ms": info["t_inner_ms"], "t_outer_ms": info["t_outer_ms"],
                              "settings": "FGMRES(100), 10 FP32 inner CG iterations on K_hat + 0.1 I"},
            "fgmres_paper_rule": {"time_s": tp, "outer_iters": ip["outer_iters"], "inner_iters": ip["inner_iters"],
                                  "relres_true": ip["relres_true"], "status": ip["status"]},
            "cg64": {"time_s": tc, "iters": ic["outer_iters"], "relres_true": ic["relres_true"],
                     "status": ic["status"]},
            "speedup_fgmres_paper_rule_vs_cg64": tc / tp,
            "gradient_pass_ms": times,
            "roofline": {"bound": "alu", "achieved": round(rate / 1e9, 1), "peak": round(peak / 1e9, 1),
                         "unit": "Gpair/s", "frac": round(rate / peak, 4), "traffic": None,
                         "kernel": f"k_grad<{d}, true, double>",
                         "peak_rule": "64 pairs per (3d + 3) FMA + exp2_f64 SIMD cycles (4 each, exp2_f64 60); "
                                      "1024 SIMDs x 2.4 GHz (time includes prep and the epilogue kernels)"}}


def workload_highd(args, api, native, workloads, torch) -> dict:
    """Regression at the regression table's largest shape (N = 44,484, d = 41):
    product rates per precision (FP64 and FP32 / BF16 on their large-d
    matrix-core kernels), the mixed FGMRES solve with the paper's inner rule and
    plain FP64 CG to 1e-6."""
    p = workloads.regression_highd()
    x = torch.from_numpy(p.x).cuda()
    y = torch.from_numpy(p.y).cuda()
    rates = {}
    for prec in ("fp64", "fp32", "bf16"):
        dt = torch.float64 if prec == "fp64" else torch.float32
        q = torch.randn(p.n, dtype=torch.float64, device="cuda").to(dt)
        api.kmvp_gauss(x, p.sigma, q, shift=p.gamma, prec=prec)
        torch.cuda.synchronize()
        with native.profile() as prof:
            for _ in range(5):
                api.kmvp_gauss(x, p.sigma, q, shift=p.gamma, prec=prec)
            torch.cuda.synchronize()
        st = prof.stats[prec]
        rates[prec] = {"gpair_s": round(st["pairs"] / (st["total_ms"] * 1e-3) / 1e9, 1),
                       "avg_launch_ms": round(st["total_ms"] / max(st["launches"], 1), 4)}
    log(f"high-d products: {rates}")
    opts = dict(inner_prec="fp32", inner_maxit=100, inner_tol=10 * p.tol, delta=p.delta, restart_m=1000,
                tol=p.tol, max_outer=args.max_outer or 1000, gs="cgs2")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    w, info = api.fgmres_solve(x, p.sigma, p.gamma, y, **opts)
    torch.cuda.synchronize()
    tf = time.perf_counter() - t0
    log(f"high-d fgmres: {info['outer_iters']} outer, {info['inner_iters']} inner, relres {info['relres_true']:.3e}, "
        f"{tf:.2f} s")
    t0 = time.perf_counter()
    (wc,), (ic,) = api.krr_solve([x], [p.sigma], [p.gamma], [y], mode="cg64", tol=p.tol,
                                 max_outer=args.max_outer or 20000, cg_check=32)
    torch.cuda.synchronize()
    tc = time.perf_counter() - t0
    log(f"high-d cg64: {ic['outer_iters']} iterations, relres {ic['relres_true']:.3e}, {tc:.2f} s")
    peak, rule, kname = product_peak(p.d)
    ach = rates["fp32"]["gpair_s"]
    return {"metric": METRIC, "value": ach * 1e9, "unit": "pairs/s", "n_gpus": 1, "dtype": "f32", "data": "synthetic",
            "higher_is_better": True, "vs_baseline": None,
            "config": {"workload": "regression N=44484 d=41 x~N(0,I) sigma=sqrt(41) gamma=1e-2; FGMRES with the "
                                   "paper's inner rule vs FP64 CG", "n": p.n, "d": p.d},
            "roofline": {"bound": "alu", "achieved": ach, "peak": round(peak / 1e9, 1), "unit": "Gpair/s",
                         "frac": round(ach * 1e9 / peak, 4), "traffic": None, "kernel": kname, "peak_rule": rule},
            "products": rates,
            "fgmres": {"time_s": tf, "outer_iters": info["outer_iters"], "inner_iters": info["inner_iters"],
                       "relres_true": info["relres_true"]},
            "cg64": {"time_s": tc, "iters": ic["outer_iters"], "relres_true": ic["relres_true"]},
            "speedup_fgmres_vs_cg64": tc / tf}


def workload_matern(args, api, native, workloads, torch) -> dict:
    """Matern-3/2 GPR (N = 1e5, d = 8): product rates per precision, the mixed
    FGMRES solve (the paper's inner rule) and plain FP64 CG to 1e-6."""
    p = workloads.matern_classification()
    x = torch.from_numpy(p.x).cuda()
    y = torch.from_numpy(p.y).cuda()
    rates = {}
    for prec in ("fp64", "fp32", "bf16"):
        dt = torch.float64 if prec == "fp64" else torch.float32
        q = torch.randn(p.n, dtype=torch.float64, device="cuda").to(dt)
        api.kmvp_matern(x, p.sigma, q, shift=p.gamma, prec=prec)
        torch.cuda.synchronize()
        with native.profile() as prof:
            for _ in range(3):
                api.kmvp_matern(x, p.sigma, q, shift=p.gamma, prec=prec)
            torch.cuda.synchronize()
        st = prof.stats[prec]
        rates[prec] = {"gpair_s": round(st["pairs"] / (st["total_ms"] * 1e-3) / 1e9, 1),
                       "avg_launch_ms": round(st["total_ms"] / max(st["launches"], 1), 4)}
    log(f"matern products: {rates}")
    opts = dict(kernel="matern32", inner_prec="fp32", inner_maxit=100, inner_tol=10 * p.tol, delta=p.delta,
                restart_m=1000, tol=p.tol, max_outer=args.max_outer or 1000, gs="cgs2")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    w, info = api.fgmres_solve(x, p.sigma, p.gamma, y, **opts)
    torch.cuda.synchronize()
    tf = time.perf_counter() - t0
    log(f"matern fgmres: {info['outer_iters']} outer, relres {info['relres_true']:.3e}, {tf:.2f} s")
    t0 = time.perf_counter()
    (wc,), (ic,) = api.krr_solve([x], [p.sigma], [p.gamma], [y], mode="cg64", kernel="matern32", tol=p.tol,
                                 max_outer=20000, cg_check=32)
    torch.cuda.synchronize()
    tc = time.perf_counter() - t0
    log(f"matern cg64: {ic['outer_iters']} iterations, relres {ic['relres_true']:.3e}, {tc:.2f} s")
    d = p.d
    peak, rule, kname = matern_peak(d)
    ach = rates["fp32"]["gpair_s"]
    return {"metric": METRIC, "value": ach * 1e9, "unit": "pairs/s", "n_gpus": 1, "dtype": "f32", "data": "synthetic",
            "higher_is_better": True, "vs_baseline": None,
            "config": {"workload": "matern32 classification N=1e5 d=8 h=sqrt(8) gamma=1e-2; FGMRES with the paper's "
                                   "inner rule vs FP64 CG", "n": p.n, "d": d},
            "roofline": {"bound": "alu", "achieved": ach, "peak": round(peak / 1e9, 1), "unit": "Gpair/s",
                         "frac": round(ach * 1e9 / peak, 4), "traffic": None, "kernel": kname, "peak_rule": rule},
            "products": rates,
            "fgmres": {"time_s": tf, "outer_iters": info["outer_iters"], "inner_iters": info["inner_iters"],
                       "relres_true": info["relres_true"]},
            "cg64": {"time_s": tc, "iters": ic["outer_iters"], "relres_true": ic["relres_true"]},
            "speedup_fgmres_vs_cg64": tc / tf}


def workload_sweep(args, api, native, workloads, torch) -> dict:
    """The preconditioner's parameter study (section 5.3-5.4): 2000 points in the
    unit cube, Gaussian kernel with three bandwidths (conditioning), flexible
    GMRES and flexible CG over the inner shift delta and the inner tolerance
    epsilon; outer and inner iteration counts and times per setting.  Then the
    plain FP64 CG over bandwidth and regulariser (section 3): iterations and
    the condition number estimated from the CG's Lanczos coefficients.  The
    paper's figures for these studies are not in its text: the tables are
    reported, not compared."""
    import numpy as np

    rng = np.random.default_rng(11)
    n = 2000
    xs = rng.random((n, 3))
    y = rng.standard_normal(n)
    x = torch.from_numpy(xs).cuda()
    yt = torch.from_numpy(y).cuda()
    gamma = 1e-6
    rows = []
    for sigma in (0.05, 0.1, 0.2):
        for mode in ("fgmres", "fcg"):
            for delta in (1e-4, 1e-3, 1e-2, 1e-1):
                for eps in (1e-2, 1e-4, 1e-6):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    (w,), (info,) = api.krr_solve([x], [sigma], [gamma], [yt], mode=mode, delta=delta, inner_tol=eps,
                                                  inner_maxit=500, restart_m=200, max_outer=200, inner_prec="fp32")
                    torch.cuda.synchronize()
                    rows.append({"sigma": sigma, "mode": mode, "delta": delta, "eps": eps, "status": info["status"],
                                 "outer": info["outer_iters"], "inner": info["inner_iters"],
                                 "relres": float(f"{info['relres_true']:.3e}"),
                                 "time_ms": round(1e3 * (time.perf_counter() - t0), 2)})
            log(f"sigma {sigma} done")
    # condition number and plain CG iterations over bandwidth and regulariser
    # (section 3): the condition number estimated from the CG's own Lanczos
    # coefficients, the iteration count to the same tolerance
    cond = []
    for sigma in (0.025, 0.05, 0.1, 0.2, 0.4):
        for gamma_c in (1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            (w,), (info,) = api.krr_solve([x], [sigma], [gamma_c], [yt], mode="cg64", max_outer=20000)
            torch.cuda.synchronize()
            lo, hi = info["lambda_min_est"], info["lambda_max_est"]
            cond.append({"sigma": sigma, "gamma": gamma_c, "status": info["status"], "cg_iters": info["outer_iters"],
                         "lambda_min_est": float(f"{lo:.4e}"), "lambda_max_est": float(f"{hi:.4e}"),
                         "cond_est": float(f"{hi / lo:.3e}") if lo > 0 else None,
                         "time_ms": round(1e3 * (time.perf_counter() - t0), 2)})
        log(f"cg sigma {sigma} done")
    return {"metric": METRIC, "value": None, "unit": "table", "n_gpus": 1, "dtype": "f32+f64", "data": "synthetic",
            "higher_is_better": True, "vs_baseline": None,
            "config": {"workload": "parameter study: N=2000 U[0,1]^3, gamma=1e-6, sigma in {0.05, 0.1, 0.2}; "
                                   "delta in {1e-4..1e-1}, inner tolerance in {1e-2, 1e-4, 1e-6}, tol 1e-6; "
                                   "FP64 CG over sigma in {0.025..0.4} x gamma in {1e-1..1e-6}"},
            "rows": rows, "cg_condition": cond}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cg", action="store_true", help="skip the FP64 CG comparator")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--n", type=int, default=100_000, help="points (default: the full workload)")
    ap.add_argument("--kernel-prec", default="fp32", choices=("fp64", "fp32", "bf16"),
                    help="precision of the --kernel-only products")
    ap.add_argument("--kernel-points", default="kriging", choices=("kriging", "gp", "clustered", "highd"),
                    help="point set of the --kernel-only products (kriging N=1e5 d=3, gp N=2e5 d=16, "
                         "clustered N=1e6 d=2, highd N=44484 d=41)")
    ap.add_argument("--workload", default="kriging", choices=("kriging", "clustered", "batched", "gp", "matern", "highd", "sweep"),
                    help="kriging (default, the headline line); the others print their own line")
    ap.add_argument("--max-outer", type=int, default=0,
                    help="outer-step budget of the secondary workloads (default: to convergence)")
    ap.add_argument("--inner-maxit", type=int, default=0,
                    help="inner CG iterations of the clustered workload (default: its 10)")
    ap.add_argument("--inner-prec", default="", choices=("", "fp32", "bf16"),
                    help="inner product precision of the clustered workload (default: its bf16)")
    ap.add_argument("--inner-tol", type=float, default=0.0,
                    help="batched workload: inner CG tolerance (default 0: the fixed iteration count)")
    ap.add_argument("--restart", type=int, default=0,
                    help="restart length of the timed solve (default 100; clustered workload: 200)")
    ap.add_argument("--gamma", type=float, default=0.0,
                    help="clustered workload: another regulariser gamma for the same points (delta = 10 gamma)")
    ap.add_argument("--cg-only", action="store_true",
                    help="clustered workload: only plain FP64 CG, for --max-outer iterations")
    ap.add_argument("--kernel-only", type=int, default=0, metavar="K",
                    help="only K FP32 products on the workload's points plus one 256 MiB copy "
                         "(the short run used for rocprofv3 counter passes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the sharded path is not built.",
              file=sys.stderr)
        return 2

    import torch

    from paper_1408_1237_amd import api, native, workloads

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    native.load()
    others = {"clustered": workload_clustered, "batched": workload_batched, "gp": workload_gp,
              "matern": workload_matern, "highd": workload_highd, "sweep": workload_sweep}
    if args.workload in others:
        out = others[args.workload](args, api, native, workloads, torch)
        print(json.dumps(out), flush=True)
        return 0
    if args.kernel_only:
        pk = {"kriging": lambda: workloads.kriging(n=args.n), "gp": workloads.gp_regression,
              "clustered": workloads.clustered_large, "highd": workloads.regression_highd}[args.kernel_points]()
        xk = torch.from_numpy(pk.x).cuda()
        return kernel_only(api, native, workloads, torch, pk, xk, args.kernel_only, args.kernel_prec)
    p = workloads.kriging(n=args.n)
    x = torch.from_numpy(p.x).cuda()
    y = torch.from_numpy(p.y).cuda()
    opts = dict(inner_prec="fp32", inner_maxit=p.inner_maxit, inner_tol=0.0, delta=p.delta,
                restart_m=args.restart or 100, tol=p.tol, max_outer=5000, gs="cgs2")
    paper_opts = dict(inner_prec="fp32", inner_maxit=100, inner_tol=10 * p.tol, delta=p.delta, restart_m=1000,
                      tol=p.tol, max_outer=1000, gs="cgs2")
    need = max(native.workspace_size(native.KRR_WS_FGMRES, [(p.n, p.d)], opts=api.make_opts(**o))
               for o in (opts, paper_opts))
    ws = api.workspace(need, x.device)
    log(f"workload kriging n={p.n} d={p.d} sigma={p.sigma} gamma={p.gamma}; workspace {need / 2**20:.0f} MiB")

    for k in range(args.warmup):
        w, info = api.fgmres_solve(x, p.sigma, p.gamma, y, ws=ws, **opts)
        log(f"warmup {k}: status={info['status']} outer={info['outer_iters']} relres={info['relres_true']:.3e}")
    torch.cuda.synchronize()

    infos = []
    with native.profile(max_launches=200_000) as prof:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            w, info = api.fgmres_solve(x, p.sigma, p.gamma, y, ws=ws, **opts)
            infos.append(info)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
    for k, info in enumerate(infos):
        log(f"step {k}: status={info['status']} outer={info['outer_iters']} inner={info['inner_iters']} "
            f"mvp64={info['mvp64']} mvp32={info['mvp32']} relres={info['relres_true']:.3e} "
            f"t={info['t_total_ms']:.1f} ms")
    if any(i["status"] != 0 or i["relres_true"] > p.tol for i in infos):
        log("FGMRES did not reach the tolerance")
    pairs_step = sum((i["mvp64"] + i["mvp32"] + i["mvp16"]) for i in infos) * float(p.n) ** 2
    value = pairs_step / elapsed
    ms_per_step = 1e3 * elapsed / args.steps

    st = prof.stats
    f32 = st["fp32"]
    f64 = st["fp64"]
    achieved = f32["pairs"] / (f32["total_ms"] * 1e-3) / 1e9
    peak_pairs, peak_rule, kname = product_peak(p.d)
    peak = peak_pairs / 1e9
    peak64, _, kname64 = product_peak(p.d, "fp64")
    ach64 = f64["pairs"] / max(f64["total_ms"], 1e-9) / 1e6
    traffic = read_traffic("kmvp_fp32_d3_kriging_counters.txt")
    probe = api.probe_issue_rates()
    # Roofline of the dominant kernel against the published FP32 vector peak
    # (157.3 TFLOP/s: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA) x 2 (packed) x 2.4 GHz)
    # at the algorithmic 3d + 1 FLOP per pair (d subtractions, d multiply-adds,
    # the accumulate; the exp2 is not counted); the FP64 product against 78.6
    # TFLOP/s.  Beside it, the issue model of the kernel's own instruction mix
    # (product_peak), which also prices the exponentials and the matrix-core work.
    flops_pair = 3 * p.d + 1
    tflops = achieved * 1e9 * flops_pair / 1e12
    tflops64 = ach64 * 1e9 * flops_pair / 1e12
    roofline = {"bound": "alu", "achieved": round(tflops, 2), "peak": 157.3, "unit": "TFLOP/s",
                "frac": round(tflops / 157.3, 4), "traffic": traffic,
                "flop_rule": f"{flops_pair} FLOP per pair (3d + 1, d = {p.d}) x pair rate; peak: published FP32 "
                             "vector rate (packed FMA, which this build does not issue)",
                "kernel": kname, "launches": f32["launches"],
                "avg_launch_ms": round(f32["total_ms"] / max(f32["launches"], 1), 4),
                "pair_rate_gpair_s": round(achieved, 1),
                "issue_model": {"achieved": round(achieved, 1), "peak": round(peak, 1), "unit": "Gpair/s",
                                "frac": round(achieved / peak, 4), "rule": peak_rule},
                "fp64": {"kernel": kname64, "achieved": round(tflops64, 3), "peak": 78.6, "unit": "TFLOP/s",
                         "frac": round(tflops64 / 78.6, 4), "pair_rate_gpair_s": round(ach64, 1),
                         "pairs_rule": "N^2 pair terms per product (the symmetric kernel evaluates each "
                                       "unordered pair once for both of its terms)",
                         "issue_model_peak_gpair_s": round(peak64 / 1e9, 1),
                         "issue_model_frac": round(ach64 * 1e9 / peak64, 4),
                         "avg_launch_ms": round(f64["total_ms"] / max(f64["launches"], 1), 4)},
                "issue_probe": {k: float(f"{v:.4g}") for k, v in probe.items()}}
    log(f"kernel fp32: {f32['launches']} launches, {roofline['avg_launch_ms']} ms avg, {achieved:.0f} Gpair/s "
        f"({100 * achieved / peak:.1f}% of {peak:.0f}; {tflops:.1f} TFLOP/s, {100 * tflops / 157.3:.1f}% of 157.3); "
        f"fp64: {ach64:.0f} Gpair/s ({100 * ach64 * 1e9 / peak64:.1f}% of {peak64 / 1e9:.0f}; "
        f"{100 * tflops64 / 78.6:.1f}% of 78.6 TFLOP/s); probe {roofline['issue_probe']}")

    out = {"metric": METRIC, "value": value, "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
           "config": {"workload": f"kriging-shaped N={p.n} d=3 x~U[0,10]^3 sigma=0.5 gamma=1e-3; "
                                  f"FGMRES({opts['restart_m']}) FP64 outer, 10 FP32 inner CG on K_hat+1e-2 I, tol 1e-6",
                      "n": p.n, "d": p.d, "parallelism": "single GPU"},
           "fgmres": {"time_to_solution_s": ms_per_step / 1e3, "outer_iters": infos[-1]["outer_iters"],
                      "inner_iters": infos[-1]["inner_iters"], "mvp64": infos[-1]["mvp64"],
                      "mvp32": infos[-1]["mvp32"], "relres_true": infos[-1]["relres_true"]},
           "roofline": roofline}

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    wp, ip = api.fgmres_solve(x, p.sigma, p.gamma, y, ws=ws, **paper_opts)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    log(f"fgmres (paper inner rule): status={ip['status']} outer={ip['outer_iters']} inner={ip['inner_iters']} "
        f"relres={ip['relres_true']:.3e} t={tp:.2f} s")
    out["fgmres_paper_rule"] = {"time_to_solution_s": tp, "outer_iters": ip["outer_iters"],
                                "inner_iters": ip["inner_iters"], "mvp64": ip["mvp64"], "mvp32": ip["mvp32"],
                                "relres_true": ip["relres_true"], "status": ip["status"],
                                "settings": "inner tol 1e-5 (10x outer), <= 100 inner its, restart 1000"}

    if not args.no_cg:
        o64 = dict(tol=p.tol, max_outer=20000, cg_check=32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        (wc,), (ic,) = api.krr_solve([x], [p.sigma], [p.gamma], [y], mode="cg64", ws=ws, **o64)
        torch.cuda.synchronize()
        tc = time.perf_counter() - t0
        log(f"cg64: status={ic['status']} iters={ic['outer_iters']} relres={ic['relres_true']:.3e} t={tc:.2f} s")
        out["cg64"] = {"time_to_solution_s": tc, "iters": ic["outer_iters"], "mvp64": ic["mvp64"],
                       "relres_true": ic["relres_true"], "status": ic["status"]}
        out["speedup_fgmres_vs_cg64"] = tc / (ms_per_step / 1e3)
        out["speedup_fgmres_paper_rule_vs_cg64"] = tc / tp

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(p)
        cb = out["cpu_baseline"]
        log(f"cpu oracle: {cb['value']:.3e} pairs/s on {cb['cores']} threads, {cb['value_1thread']:.3e} on 1 "
            f"({cb['cpu_model']})")
        out["plain_small"] = plain_small_block(api, torch)
        log(f"plain small: {out['plain_small']}")

    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
