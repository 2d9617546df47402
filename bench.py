"""Benchmark: fine-grid unknowns/s of the GMG Poisson solve to 1e-10 relative
residual on one MI355X, plus the smoother's achieved HBM bandwidth.

Default workload: 3D 7-point Poisson, 1023^3 interior (h = 1/1024, about
1.07e9 unknowns), zero Dirichlet data, f = sum of eight sine modes
a_m prod_i sin(k_{m,i} pi x_i) with a_m ~ N(0,1), k ~ U{1..32} (SplitMix64
seed 5), FP64 V(1,1) red-black Gauss-Seidel, full weighting / trilinear
interpolation, one-node coarsest level, u0 = 0, rtol = 1e-10.  A step = one
gmg_solve from u = 0 with f already in HBM.  The same line also carries the
mixed-precision solve of the same problem (FP32 V(1,1) cycles inside FP64
refinement) and the 256-problem uneven batch, each timed against plain FP64
single-problem solves.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, AMD published peak
# committed rocprofv3 counter tables of the level-0 passes: (workload, kernel class) -> file
TRAFFIC_PROFILES = {
    ("poisson3d_255_sine_noise_fp64_v22", "smooth_pre_l0"):
        os.path.join(ROOT, "profiles", "rb_pass_l0_poisson3d_255_traffic.md"),
    ("poisson3d_255_sine_noise_fp64_v22", "smooth_post_l0"):
        os.path.join(ROOT, "profiles", "rb_pass_l0_poisson3d_255_traffic.md"),
    ("poisson3d_511_uniform_fp64_v22", "smooth_pre_l0"):
        os.path.join(ROOT, "profiles", "rb_pass_l0_poisson3d_511_traffic.md"),
    ("poisson3d_511_uniform_fp64_v22", "smooth_post_l0"):
        os.path.join(ROOT, "profiles", "rb_pass_l0_poisson3d_511_traffic.md"),
    ("poisson3d_1023_sine_modes_fp64_v11", "smooth_cross_l0"):
        os.path.join(ROOT, "profiles", "cross_pass_l0_poisson3d_1023_traffic.md"),
}

WORKLOADS = {
    # name: dim, levels, right-hand side, precision, sweeps nu1 = nu2, FP32
    # cycles per refinement step (mixed)
    "poisson3d_255_sine_noise_fp64_v22": dict(dim=3, L=8, rhs="sine_noise", prec="fp64"),
    "poisson2d_127_sine_fp64_v22": dict(dim=2, L=7, rhs="sine", prec="fp64"),
    "poisson3d_511_uniform_fp64_v22": dict(dim=3, L=9, rhs="uniform", prec="fp64"),
    "poisson3d_511_uniform_mixed_v22": dict(dim=3, L=9, rhs="uniform", prec="mixed"),
    "poisson3d_511_uniform_mixed2_v22": dict(dim=3, L=9, rhs="uniform", prec="mixed", inner=2),
    # the headline: its line also carries the mixed-precision solve of the same
    # problem and the 256-problem batch, each against plain FP64 solves
    "poisson3d_1023_sine_modes_fp64_v11": dict(dim=3, L=10, rhs="sine_modes", prec="fp64", nu=1,
                                               extras=True),
    "poisson3d_1023_sine_modes_mixed_v11": dict(dim=3, L=10, rhs="sine_modes", prec="mixed",
                                                nu=1),
    "poisson3d_1023_sine_modes_mixed2_v11": dict(dim=3, L=10, rhs="sine_modes", prec="mixed",
                                                 nu=1, inner=2),
    "poisson3d_255_sine_noise_fp64_wj22": dict(dim=3, L=8, rhs="sine_noise", prec="fp64",
                                               smoother="wj"),
    "batch256_uneven_fp64_v22": dict(dim=0, L=0, rhs="batch", prec="fp64"),
    # one full-multigrid pass (Algorithm 2) on the model problem u = prod sin(pi x_i)
    "poisson3d_255_sine_fmg22": dict(dim=3, L=8, rhs="fmg", prec="fp64"),
    "poisson3d_1023_sine_fmg22": dict(dim=3, L=10, rhs="fmg", prec="fp64"),
    "poisson2d_4095_sine_fmg22": dict(dim=2, L=12, rhs="fmg", prec="fp64"),
    # the paper's own method (multicolour GS, finite-element transfers, V(1,1),
    # tol 1e-6, u = prod sin(pi x_i)): the configuration of its Tables 5, 7, 8
    "poisson2d_4095_paper_mcgs_v11": dict(dim=2, L=12, rhs="model", prec="fp64", nu=1,
                                          smoother="mcgs", flags=0x80, rtol=1e-6,
                                          paper_s=0.4339),
    "poisson3d_255_paper_mcgs_v11": dict(dim=3, L=8, rhs="model", prec="fp64", nu=1,
                                         smoother="mcgs", flags=0x80, rtol=1e-6, paper_s=0.7287),
    "poisson3d_255_paper_fmg33": dict(dim=3, L=8, rhs="fmg", prec="fp64", nu=3,
                                      smoother="mcgs", flags=0x80, paper_s=0.1456),
    "poisson2d_4095_paper_fmg12": dict(dim=2, L=12, rhs="fmg", prec="fp64", nu1=1, nu2=2,
                                       smoother="mcgs", flags=0x80, paper_s=0.09167),
    # exact solve by the sine transform (the paper's FFT comparison, Tables 12-15)
    "poisson2d_4095_sine_dst": dict(dim=2, L=12, rhs="dst", prec="fp64", paper_s=0.1364),
    "poisson3d_255_sine_dst": dict(dim=3, L=8, rhs="dst", prec="fp64", paper_s=0.1893),
    "poisson3d_1023_sine_dst": dict(dim=3, L=10, rhs="dst", prec="fp64"),
}
DEFAULT = "poisson3d_1023_sine_modes_fp64_v11"


def make_rhs(spec):
    """Host right-hand side (None for recipes built on the device)."""
    from paper_1208_4247_amd import workloads as wl

    d, m = spec["dim"], (1 << spec["L"]) - 1
    if spec["rhs"] == "sine_modes":
        return None
    if spec["rhs"] == "sine_noise":
        return wl.rhs_sine_plus_noise(d, m, 2)
    if spec["rhs"] == "sine":
        return wl.rhs_sine(d, m)
    if spec["rhs"] == "uniform":
        return wl.rhs_uniform(d, m, 3)
    if spec["rhs"] == "model":
        return d * math.pi ** 2 * wl.sine_product(d, m)
    raise ValueError(spec["rhs"])


def cpu_baseline(spec, f, gpu_iters, budget_s=30.0):
    """The FP64 CPU oracle (untuned) solving the same workload with the same
    cycle on the host cores, bounded in time: the full solve when it fits,
    else the oracle's solve loop cut after a few cycles (initial residual
    norm, then per cycle a V-cycle and the stop test's residual norm), scaled
    to unknowns/s at the GPU's cycle count."""
    import oracle

    oracle.build()
    threads = min(16, os.cpu_count() or 1)
    oracle.set_threads(threads)
    N = f.size
    nu = spec.get("nu", 2)
    smoother = {"rbgs": oracle.RBGS, "wj": oracle.WJ, "mcgs": oracle.MCGS}[
        spec.get("smoother", "rbgs")]
    variant = oracle.FE_TRANSFER if spec.get("flags", 0) & 0x80 else 0
    omega = 6.0 / 7.0 if f.ndim == 3 else 0.8
    kw = dict(nu1=nu, nu2=nu, smoother=smoother, omega=omega, variant=variant)
    rtol = spec.get("rtol", 1e-10)
    t0 = time.perf_counter()
    oracle.solve(f, rtol=rtol, maxit=1, **kw)
    t_one = time.perf_counter() - t0
    if t_one * gpu_iters <= budget_s:
        # the median of up to three full solves on every host thread, then
        # one on a single thread when it fits the budget
        ts = []
        while not ts or (len(ts) < 3 and sum(ts) + t_one * gpu_iters <= budget_s / 2):
            t0 = time.perf_counter()
            _, it, rel, st, _ = oracle.solve(f, rtol=rtol, **kw)
            ts.append(time.perf_counter() - t0)
        t = sorted(ts)[len(ts) // 2]
        out = dict(value=N / t, unit="unknowns/s", cores=oracle.num_threads(), kind="oracle",
                   sample="full solve of the same workload (%d V-cycles to relres %.1e), median "
                   "of %d: %.2f s" % (it, rel, len(ts), t))
        if t * threads <= budget_s / 2:
            oracle.set_threads(1)
            t0 = time.perf_counter()
            oracle.solve(f, rtol=rtol, **kw)
            t1 = time.perf_counter() - t0
            oracle.set_threads(threads)
            out["single_thread_value"] = N / t1
            out["sample"] += "; one thread: %.2f s" % t1
        return out
    k = max(1, min(int(budget_s / t_one), gpu_iters))
    t0 = time.perf_counter()
    oracle.solve(f, rtol=rtol, maxit=k, **kw)
    t = time.perf_counter() - t0
    return dict(value=N / (t * gpu_iters / k), unit="unknowns/s", cores=oracle.num_threads(),
                kind="oracle",
                sample="the oracle's solve loop on the same workload cut after %d of the GPU's "
                "%d cycles (initial residual norm, then per cycle a V-cycle and the stop test's "
                "residual norm): %.1f s, scaled to %d cycles" % (k, gpu_iters, t, gpu_iters))


def measured_traffic(workload, cls, tile, folded):
    """HBM bytes per launch of the level-0 pass class `cls` with tile
    (stages, variant, tz), from a committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE per dispatch, scaled by the runtime's copy of a
    known size; one entry per autotuner candidate), or None when no summary
    covers this workload and kernel source."""
    import hashlib

    path = TRAFFIC_PROFILES.get((workload, cls))
    if path is None or tile is None or not os.path.exists(path):
        return None
    line = [l for l in open(path) if l.startswith("traffic-json: ")]
    if not line:
        return None
    rec = json.loads(line[-1][len("traffic-json: "):])
    csrc = os.path.join(ROOT, "paper_1208_4247_amd", "csrc")
    for name, digest in rec.get("sources_sha256", {}).items():
        with open(os.path.join(csrc, name), "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest() != digest:
                return None
    if cls == "smooth_cross_l0":
        key = "cross|%d|%d|%d|%d" % (tile + (1 if folded else 0,))
    else:
        role = {"smooth_pre_l0": "pre", "smooth_post_l0": "post"}[cls]
        key = "%s|%d|%d|%d" % ((role,) + tuple(tile))
    return rec["tiles"].get(key)


def bench_fmg(args, spec):
    """One FMG(nu1,nu2) pass (Algorithm 2) for -Lap u = d pi^2 prod sin(pi x_i),
    u = prod sin(pi x_i): time per pass, and its L2_h error against the exact
    solution beside the discrete solution's own error (closed form), the
    comparison of the paper's FMG tables."""
    import torch

    from paper_1208_4247_amd import capi
    from paper_1208_4247_amd import workloads as wl
    from paper_1208_4247_amd.solver import Plan

    d, L = spec["dim"], spec["L"]
    nu1 = spec.get("nu1", spec.get("nu", 2)) if args.nu1 is None else args.nu1
    nu2 = spec.get("nu2", spec.get("nu", 2)) if args.nu2 is None else args.nu2
    smoother = spec.get("smoother", "rbgs")
    m = (1 << L) - 1
    N = m ** d
    n = m + 1
    h = 1.0 / (m + 1)
    torch.cuda.set_device(0)
    phi = wl.sine_product_device(d, m, "cuda")
    f = (d * math.pi ** 2) * phi
    flags = args.flags | spec.get("flags", 0) | (0 if args.no_autotune else capi.GMG_AUTOTUNE)
    plan = Plan(d, L, nu1=nu1, nu2=nu2, flags=flags, smoother=smoother)
    u = torch.empty_like(f)
    for _ in range(max(1, args.warmup)):
        plan.fmg(u, f)
    torch.cuda.synchronize()
    ts = []
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.fmg(u, f)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    ms = 1e3 * sum(ts) / len(ts)
    err = float(torch.sqrt(h ** d * torch.sum((u - phi) ** 2)))
    lam = d * (4.0 / h ** 2) * math.sin(math.pi * h / 2) ** 2
    disc = abs(d * math.pi ** 2 / lam - 1.0) * float(torch.sqrt(h ** d * torch.sum(phi ** 2)))
    line = {
        "metric": "fine-grid unknowns/s, one FMG(%d,%d) pass" % (nu1, nu2),
        "value": N / (ms * 1e-3), "unit": "unknowns/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "dim": d, "side": m, "levels": L,
                   "cycle": "FMG(%d,%d) %s" % (nu1, nu2, cycle_name(smoother, spec)),
                   "l2h_error": err, "discretisation_error": disc, "error_ratio": err / disc,
                   # the norm of the paper's FMG tables: (sum e^2 / (n+1)^d)^(1/2)
                   "paper_norm_error": err * (n / (n + 1)) ** (d / 2)},
    }
    if "paper_s" in spec:
        line["config"]["paper_gtx480_s"] = spec["paper_s"]
    print(json.dumps(line), flush=True)


def bench_dst(args, spec):
    """One exact solve by the sine transform of -Lap u = d pi^2 prod sin(pi x_i)
    (gmg_dst_solve): time per solve and the L2_h error against the exact u,
    which is the paper's FFT column (Tables 12, 14)."""
    import torch

    from paper_1208_4247_amd import workloads as wl
    from paper_1208_4247_amd.solver import DstSolver

    d, L = spec["dim"], spec["L"]
    m = (1 << L) - 1
    N = m ** d
    h = 1.0 / (m + 1)
    torch.cuda.set_device(0)
    phi = wl.sine_product_device(d, m, "cuda")
    f = (d * math.pi ** 2) * phi
    solver = DstSolver(d, L)
    u = torch.empty_like(f)
    for _ in range(max(1, args.warmup)):
        solver.solve(u, f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        solver.solve(u, f)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    err = float(torch.sqrt(h ** d * torch.sum((u - phi) ** 2)))
    line = {
        "metric": "fine-grid unknowns/s, one exact sine-transform solve",
        "value": N / (ms * 1e-3), "unit": "unknowns/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "dim": d, "side": m, "levels": L,
                   "method": "DST-I along every axis (rocFFT batched complex FFTs, two real lines "
                             "each), eigenvalue "
                             "division, inverse", "l2h_error": err,
                   "workspace_MB": solver.workspace.numel() / 1e6},
    }
    if "paper_s" in spec:
        line["config"]["paper_gtx480_cufft_s"] = spec["paper_s"]
    print(json.dumps(line), flush=True)


def cycle_name(smoother, spec):
    if smoother == "mcgs":
        return "%d-colour GS, finite-element transfers" % (4 if spec["dim"] == 2 else 8)
    return "weighted Jacobi" if smoother == "wj" else "red-black GS"


def run_batch(args, steps, warmup):
    """256 independent problems of uneven size (128 2D with side 2^k-1,
    k ~ U{6..10}; 128 3D with k ~ U{5..7}; U[-1,1] right-hand sides, seed 4),
    FP64 V(2,2) RB-GS to 1e-10 each, by one batch plan (graph-captured
    cycles, autotuned tiles), and the same 256 solves run one after another
    by autotuned single-problem plans.  Returns the timings."""
    import torch

    from paper_1208_4247_amd import capi
    from paper_1208_4247_amd import workloads as wl
    from paper_1208_4247_amd.solver import BatchPlan, Plan

    probs = wl.batch_problems(4)
    N = sum(m ** d for d, m in probs)
    fs = [torch.from_numpy(wl.batch_rhs(4, q, d, m)).cuda() for q, (d, m) in enumerate(probs)]
    us = [torch.zeros_like(f) for f in fs]
    flags = args.flags | capi.GMG_USE_GRAPH
    if not args.no_autotune:
        flags |= capi.GMG_AUTOTUNE  # the warm-up solve tunes one problem per shape
    plan = BatchPlan([(d, (m + 1).bit_length() - 1) for d, m in probs], flags=flags)
    for _ in range(max(1, warmup)):
        for u in us:
            u.zero_()
        plan.solve(us, fs)
    torch.cuda.synchronize()
    t_total = 0.0
    for _ in range(steps):
        for u in us:
            u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s, its, rels, sts = plan.solve(us, fs)
        torch.cuda.synchronize()
        t_total += time.perf_counter() - t0
    batch_ms = 1e3 * t_total / steps
    plans = {}
    for d, m in sorted(set(probs)):
        plans[(d, m)] = Plan(d, (m + 1).bit_length() - 1, flags=args.flags | capi.GMG_AUTOTUNE)
    for q, (d, m) in enumerate(probs):
        us[q].zero_()
        plans[(d, m)].solve(us[q], fs[q], rtol=1e-10)
    torch.cuda.synchronize()
    seq = []
    for _ in range(max(1, min(steps, 3))):
        for u in us:
            u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for q, (d, m) in enumerate(probs):
            plans[(d, m)].solve(us[q], fs[q], rtol=1e-10)
        torch.cuda.synchronize()
        seq.append(time.perf_counter() - t0)
    seq_ms = 1e3 * sum(seq) / len(seq)
    return {"problems": len(probs), "unknowns": N, "batch_ms_per_solve": batch_ms,
            "max_cycles": max(its), "min_cycles": min(its),
            "all_converged": all(x == 0 for x in sts),
            "sequential_single_solves_ms": seq_ms, "speedup_vs_sequential": seq_ms / batch_ms}


def bench_batch(args):
    """The 256-problem batch on its own: value = total unknowns / solve time."""
    import torch

    torch.cuda.set_device(0)
    b = run_batch(args, args.steps, args.warmup)
    line = {
        "metric": "fine-grid unknowns/s to 1e-10 rel. residual (batch of 256 uneven problems)",
        "value": b["unknowns"] / (b["batch_ms_per_solve"] * 1e-3), "unit": "unknowns/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": b["batch_ms_per_solve"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": dict({"workload": "batch256_uneven_fp64_v22"}, **b),
    }
    print(json.dumps(line), flush=True)


def mixed_vs_fp64(args, spec, f, u64, ms64, steps):
    """The mixed-precision solve (FP32 V-cycles inside FP64 refinement, the
    library's default inner-cycle count) of the same problem, timed like the
    FP64 solve it is compared with: its time, its FP64 residual (by the FP64
    residual kernel) and its distance from the FP64 iterate u64."""
    import torch

    from paper_1208_4247_amd import capi
    from paper_1208_4247_amd.solver import Plan

    d, L, nu = spec["dim"], spec["L"], spec.get("nu", 2)
    flags = args.flags | (0 if args.no_autotune else capi.GMG_AUTOTUNE)
    pm = Plan(d, L, flags=flags, nu1=nu, nu2=nu, precision="mixed")
    um = torch.zeros_like(f)
    pm.solve(um, f, rtol=1e-10)  # warm-up (autotunes)
    ts = []
    for _ in range(max(1, steps)):
        um.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, it, rel = pm.solve(um, f, rtol=1e-10)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    ms = 1e3 * sum(ts) / len(ts)
    inner = pm.cfg.inner_cycles
    del pm
    p64 = Plan(d, L, nu1=nu, nu2=nu)
    nrm = p64.op_residual(0, um, f, None, want_norm=True)
    res0 = float(torch.linalg.vector_norm(f))
    diff = float(torch.linalg.vector_norm(um - u64) / torch.linalg.vector_norm(u64))
    del p64, um
    return {"mixed_ms_per_solve": ms, "mixed_steps": it, "mixed_status": st,
            "mixed_inner_cycles": inner, "mixed_speedup_vs_fp64": ms64 / ms,
            "mixed_fp64_relres": (nrm / res0) if res0 > 0 else 0.0,
            "mixed_vs_fp64_rel_diff": diff}


def compare_fp64(args, spec, plan, u_mixed, f, mixed_ms):
    """The plain FP64 solve of the same problem in the same process: its time
    to 1e-10, and the mixed result's distance from it and FP64 residual."""
    import torch

    from paper_1208_4247_amd import capi
    from paper_1208_4247_amd.solver import Plan

    d, L, nu = spec["dim"], spec["L"], spec.get("nu", 2)
    flags = args.flags | (0 if args.no_autotune else capi.GMG_AUTOTUNE)
    p64 = Plan(d, L, flags=flags, nu1=nu, nu2=nu)
    u64 = torch.zeros_like(f)
    p64.solve(u64, f, rtol=1e-10)  # warm-up (autotunes)
    ts = []
    for _ in range(max(1, min(args.steps, 3))):
        u64.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, it64, rel64 = p64.solve(u64, f, rtol=1e-10)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    ms64 = 1e3 * sum(ts) / len(ts)
    diff = float(torch.linalg.vector_norm(u_mixed - u64) / torch.linalg.vector_norm(u64))
    # FP64 residual of the mixed result, by the FP64 plan's own residual kernel
    r = torch.empty_like(f)
    nrm = p64.op_residual(0, u_mixed, f, r, want_norm=True)
    res0 = float(torch.linalg.vector_norm(f))
    del r, p64, u64
    return {"fp64_ms_per_solve": ms64, "fp64_iters": it64,
            "speedup_vs_fp64": ms64 / mixed_ms,
            "mixed_vs_fp64_rel_diff": diff,
            "mixed_fp64_relres": (nrm / res0) if res0 > 0 else 0.0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline workload: skip the mixed-precision and batch comparisons")
    ap.add_argument("--flags", type=int, default=0)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--nu1", type=int, default=None, help="FMG workloads: pre-sweeps")
    ap.add_argument("--nu2", type=int, default=None, help="FMG workloads: post-sweeps")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: measures one GPU only (the solver runs every level of one problem on "
              "a single device); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1208_4247_amd import capi
    from paper_1208_4247_amd.solver import Plan

    spec = WORKLOADS[args.workload]
    if spec["rhs"] == "batch":
        return bench_batch(args)
    if spec["rhs"] == "fmg":
        return bench_fmg(args, spec)
    if spec["rhs"] == "dst":
        return bench_dst(args, spec)
    if args.nu1 is not None or args.nu2 is not None:
        sys.exit("bench.py: --nu1/--nu2 apply to the FMG workloads only")
    d, L = spec["dim"], spec["L"]
    nu = spec.get("nu", 2)
    inner = spec.get("inner")  # None: the library's default inner-cycle count
    m = (1 << L) - 1
    N = m ** d
    f_host = make_rhs(spec)
    torch.cuda.set_device(0)
    if f_host is None:
        from paper_1208_4247_amd import workloads as wl

        f = wl.rhs_sine_modes_device(d, m, 5, "cuda")
    else:
        f = torch.from_numpy(f_host).cuda()
    u = torch.zeros_like(f)
    flags = args.flags | capi.GMG_PROFILE | spec.get("flags", 0)
    if not args.no_autotune:
        flags |= capi.GMG_AUTOTUNE
    smoother = spec.get("smoother", "rbgs")
    rtol = spec.get("rtol", 1e-10)
    plan = Plan(d, L, precision=spec["prec"], flags=flags, nu1=nu, nu2=nu, inner_cycles=inner,
                smoother=smoother)
    print("# workload %s: %d^%d, plan workspace %.1f MB" % (args.workload, m, d,
          plan.workspace.numel() / 1e6), flush=True)

    # warm-up (the first solve also runs the tile autotuner)
    for _ in range(args.warmup):
        u.zero_()
        st, it, rel = plan.solve(u, f, rtol=rtol)
    torch.cuda.synchronize()
    # timed region: hipEvents only around the level-0 smoothing passes
    smoothers = ["smooth_pre_l0", "smooth_post_l0", "smooth_cross_l0"]
    plan.profile_only(smoothers)
    plan.profile_reset()
    iters = []
    t_total = 0.0
    t_each = []
    for k in range(args.steps):
        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, it, rel = plan.solve(u, f, rtol=rtol)
        torch.cuda.synchronize()
        t_each.append(time.perf_counter() - t0)
        t_total += t_each[-1]
        iters.append(it)
    prof = plan.profile()
    # the same solves with no dispatch events at all: what the events of the
    # timed region cost
    plan.profile_only([])
    t_plain = []
    for _ in range(max(1, min(args.steps, 5))):
        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.solve(u, f, rtol=rtol)
        torch.cuda.synchronize()
        t_plain.append(time.perf_counter() - t0)
    ms_per_step = 1e3 * t_total / args.steps
    value = N / (t_total / args.steps)
    dom = max(smoothers, key=lambda k: prof[k]["ms"])
    pv = prof[dom]
    role = {"smooth_pre_l0": 0, "smooth_post_l0": 1, "smooth_cross_l0": 2}[dom]
    tile = None if smoother == "mcgs" else plan.get_tile(0, role)
    achieved = pv["bytes"] / (pv["ms"] * 1e-3) / 1e9 if pv["ms"] > 0 else 0.0
    avg_us = 1e3 * pv["ms"] / max(pv["launches"], 1)
    bytes_per_launch = pv["bytes"] / max(pv["launches"], 1)
    print("# iters %s relres %.3e status %d; %.3f ms per solve" % (sorted(set(iters)), rel, st,
          ms_per_step), flush=True)
    # per-kernel breakdown from a separate, fully profiled run (events around
    # every launch perturb the timing, so it is not the timed region)
    plan.profile_only(plan.PROFILE_CLASSES)
    plan.profile_reset()
    for _ in range(2):
        u.zero_()
        plan.solve(u, f, rtol=rtol)
    full = plan.profile()
    # the restriction runs inside the pass when no separate restriction ran
    fused_pre = dom != "smooth_post_l0" and full["resid_restrict_l0"]["launches"] == 0
    traffic = measured_traffic(args.workload, dom, tile, fused_pre)
    if traffic is not None and dom == "smooth_pre_l0" and fused_pre:
        traffic = None  # the 255^3 and 511^3 tables cover the plain pre-smoothing pass only
    for k, v in full.items():
        if v["launches"]:
            print("#   %-22s launches %6d  avg %9.3f us  alg %8.1f GB/s" % (
                k, v["launches"], 1e3 * v["ms"] / v["launches"],
                v["bytes"] / (v["ms"] * 1e-3) / 1e9 if v["ms"] > 0 else 0.0), flush=True)
    line = {
        "metric": "fine-grid unknowns/s to %g rel. residual; smoother HBM GB/s %% of peak" % rtol,
        "value": value,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "ms_median": 1e3 * sorted(t_each)[len(t_each) // 2],
        "ms_min": 1e3 * min(t_each),
        "ms_no_events": 1e3 * sum(t_plain) / len(t_plain),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if spec["prec"] == "fp64" else "f32-in-f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "dim": d, "side": m, "levels": L,
                   "cycle": "V(%d,%d) %s" % (nu, nu, cycle_name(smoother, spec)),
                   "rtol": rtol, "iters": iters[-1]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     # traffic: rocprofv3 FETCH_SIZE + WRITE_SIZE per dispatch of this
                     # tile, from the committed counter table of the same sources
                     "traffic_source": (os.path.relpath(TRAFFIC_PROFILES[(args.workload, dom)],
                                                        ROOT) if traffic is not None else None),
                     "kernel": dom, "avg_us": avg_us, "alg_bytes_per_launch": bytes_per_launch,
                     "tile": ({"stages": tile[0], "variant": tile[1], "tz": tile[2]} if tile
                              else None),
                     "restriction_folded_in": bool(fused_pre),
                     "timer": "HIP events recorded by each dispatch of the kernel",
                     # every level-0 kernel class, from the fully profiled breakdown run
                     "level0_kernels": {
                         k: {"avg_us": 1e3 * v["ms"] / v["launches"],
                             "achieved": v["bytes"] / (v["ms"] * 1e-3) / 1e9,
                             "frac": v["bytes"] / (v["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS}
                         for k, v in full.items()
                         if k.endswith("_l0") and v["launches"] and v["ms"] > 0}},
    }
    if "paper_s" in spec:
        line["config"]["paper_gtx480_s"] = spec["paper_s"]
    if spec["prec"] == "mixed":
        line["config"].update(compare_fp64(args, spec, plan, u, f, ms_per_step))
        line["config"]["inner_cycles"] = plan.cfg.inner_cycles
    if spec.get("extras") and not args.no_extras:
        # u holds the FP64 solve's result (last breakdown solve)
        line["config"].update(mixed_vs_fp64(args, spec, f, u, ms_per_step,
                                            min(args.steps, 5)))
        print("# mixed: %(mixed_ms_per_solve).3f ms, %(mixed_steps)d steps of "
              "%(mixed_inner_cycles)d FP32 cycles, %(mixed_speedup_vs_fp64).2fx FP64, FP64 relres "
              "%(mixed_fp64_relres).2e, distance %(mixed_vs_fp64_rel_diff).2e" % line["config"],
              flush=True)
        b = run_batch(args, min(args.steps, 10), 1)
        line["config"]["batch256"] = b
        print("# batch: %.3f ms, %.2fx the sequential single solves (%.3f ms)" % (
            b["batch_ms_per_solve"], b["speedup_vs_sequential"],
            b["sequential_single_solves_ms"]), flush=True)
    if not args.no_cpu_baseline:
        if f_host is None:
            del plan, u
            torch.cuda.synchronize()
            f_host = f.cpu().numpy()
        line["cpu_baseline"] = cpu_baseline(spec, f_host, iters[-1])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
