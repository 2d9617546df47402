"""Per-kernel timings of the hot path on one GPU (the methodology of the
paper's matrix-free matvec tables, Sec. 5.2 Tables 3-4, applied to every
kernel of the cycle): each fused pass, tile shape and z-chunk is timed with
device events over repeated launches and reported as microseconds and
algorithmic HBM GB/s.

    python -m paper_1208_4247_amd.microbench --dim 3 --m 255
"""
from __future__ import annotations

import argparse
import json

import torch

from .solver import Plan


def _time(fn, reps):
    fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    b.synchronize()
    return a.elapsed_time(b) * 1e3 / reps  # microseconds


def run(dim, m, reps=20, dtype=torch.float64, smoother="rbgs", tzs=(0,), out=None, stages=None,
        variants=None, kinds=("plain", "zero", "prolong", "prolong_bwd"), transfers=True):
    L = (m + 1).bit_length() - 1
    plan = Plan(dim, L, smoother=smoother, nu1=2, nu2=2)
    n = m ** dim
    mc = (m - 1) // 2
    es = torch.finfo(dtype).bits // 8
    g = torch.Generator(device="cuda").manual_seed(0)
    f = torch.rand((m,) * dim, dtype=dtype, device="cuda", generator=g)
    u = torch.rand((m,) * dim, dtype=dtype, device="cuda", generator=g) * 1e-3
    o = torch.empty_like(u)
    e = torch.rand((mc,) * dim, dtype=dtype, device="cuda", generator=g) * 1e-3
    fc = torch.empty((mc,) * dim, dtype=dtype, device="cuda")
    rows = []
    stage_counts = stages or ((2, 4) if smoother == "rbgs" else (1, 2))
    for st in stage_counts:
        nsw = st // 2 if smoother == "rbgs" else st
        for v in range(plan.tile_variants(st)):
            if variants is not None and v not in variants:
                continue
            for tz in tzs:
                plan.set_tile(0, st, v, tz)
                for kind in kinds:
                    if kind == "plain":
                        fn = lambda: plan.op_smooth(0, nsw, False, u, f, None, o)
                        nb = 3 * n * es
                    elif kind == "norm":
                        fn = lambda: plan.op_smooth(0, nsw, False, u, f, None, o, want_norm=True)
                        nb = 3 * n * es
                    elif kind == "zero":
                        fn = lambda: plan.op_smooth(0, nsw, False, None, f, None, o)
                        nb = 2 * n * es
                    elif kind == "prolong":
                        fn = lambda: plan.op_smooth(0, nsw, False, u, f, e, o)
                        nb = 3 * n * es + mc ** dim * es
                    else:
                        fn = lambda: plan.op_smooth(0, nsw, True, u, f, e, o)
                        nb = 3 * n * es + mc ** dim * es
                    us = _time(fn, reps)
                    rows.append(dict(kernel="%s_pass" % smoother, stages=st, variant=v, tz=tz,
                                     kind=kind, us=us, gbs=nb / (us * 1e-6) / 1e9))
    if transfers:
        us = _time(lambda: plan.op_restrict_residual(0, u, f, fc), reps)
        rows.append(dict(kernel="resid_restrict", us=us,
                         gbs=(2 * n + mc ** dim) * es / (us * 1e-6) / 1e9))
        us = _time(lambda: plan.op_residual(0, u, f, o, want_norm=False), reps)
        rows.append(dict(kernel="residual", us=us, gbs=3 * n * es / (us * 1e-6) / 1e9))
    for r in rows:
        print(json.dumps(r), flush=True)
    if out:
        with open(out, "a") as fh:
            for r in rows:
                fh.write(json.dumps(dict(r, dim=dim, m=m)) + "\n")
    plan.close()
    return rows


def tuner_tz(m):
    """The z-chunks the autotuner tries on a level of side m (0: automatic):
    powers of two up to 64, the chunks that split the planes into 2, 3, 5, 6
    or 12 nearly equal runs, and the automatic choice."""
    return sorted({min(c, m) for c in (4, 8, 16, 32, 64)} |
                  {max(1, -(-m // k)) for k in (2, 3, 5, 6, 12)}) + [0]


def traffic_table(dim, m):
    """Every tile candidate the autotuner tries for the level-0 red-black
    passes of a V(2,2) cycle -- pre-smoothing with the norm partials of the
    start value, post-smoothing with the interpolated correction -- launched
    twice each in a fixed order, with one manifest line per candidate.  Under
    a hardware-counter profiler (FETCH_SIZE, WRITE_SIZE) the k_rb_pass
    dispatches map two by two onto the manifest, giving the HBM bytes of
    every candidate the cycle may run."""
    L = (m + 1).bit_length() - 1
    plan = Plan(dim, L, nu1=2, nu2=2)
    mc = (m - 1) // 2
    g = torch.Generator(device="cuda").manual_seed(0)
    f = torch.rand((m,) * dim, dtype=torch.float64, device="cuda", generator=g)
    u = torch.rand((m,) * dim, dtype=torch.float64, device="cuda", generator=g) * 1e-3
    o = torch.empty_like(u)
    e = torch.rand((mc,) * dim, dtype=torch.float64, device="cuda", generator=g) * 1e-3
    for role in ("pre", "post"):
        for st in (2, 4):
            nsw = st // 2
            for v in range(plan.tile_variants(st)):
                seen = set()
                for tz in tuner_tz(m):
                    try:
                        plan.set_tile(0, st, v, tz)
                    except Exception:
                        continue  # more workgroups than the partial-sum buffer holds
                    tzv = plan.get_tile(0, 0)[2]
                    if tzv in seen:
                        continue
                    seen.add(tzv)
                    if role == "pre":
                        fn = lambda: plan.op_smooth(0, nsw, False, u, f, None, o, want_norm=True)
                    else:
                        fn = lambda: plan.op_smooth(0, nsw, True, u, f, e, o)
                    print(json.dumps(dict(manifest=role, dim=dim, m=m, stages=st, variant=v,
                                          tz=tzv, launches=2)), flush=True)
                    fn()
                    fn()
    torch.cuda.synchronize()
    plan.close()


def cross_sweep(dim, m, strips=(0, 1, 2, 3, 4, 6, 8), variants=None, tzs=None):
    """The cross-cycle pass of FP64 red-black V(1,1) solves (three stages,
    interpolated correction in, mid-pass norm, with and without the folded
    restriction) for every tile, z-chunk and tile order, timed inside short
    solves (three cross passes each) by the plan's dispatch events: one JSON
    row per candidate with the mean pass time and the algorithmic rate."""
    from . import capi

    L = (m + 1).bit_length() - 1
    g = torch.Generator(device="cuda").manual_seed(0)
    f = torch.rand((m,) * dim, dtype=torch.float64, device="cuda", generator=g) - 0.5
    u = torch.zeros_like(f)
    for fold in (True, False):
        flags = capi.GMG_PROFILE | (0 if fold else capi.GMG_NO_FUSED_RESTRICT)
        plan = Plan(dim, L, nu1=1, nu2=1, flags=flags)
        plan.profile_only(["smooth_cross_l0", "resid_restrict_l0"])
        for v in range(plan.tile_variants(3)):
            if variants is not None and v not in variants:
                continue
            for tz in (tzs or tuner_tz(m)):
                try:
                    plan.set_tile(0, 3, v, tz)
                except capi.GmgError:
                    continue
                for sw in strips:
                    plan.set_tile_order(0, 3, sw)
                    plan.profile_reset()
                    u.zero_()
                    plan.solve(u, f, rtol=1e-30, maxit=4)
                    pr = plan.profile()
                    c, r = pr["smooth_cross_l0"], pr["resid_restrict_l0"]
                    us = 1e3 * c["ms"] / max(c["launches"], 1)
                    rus = 1e3 * r["ms"] / max(r["launches"], 1) if r["launches"] else 0.0
                    print(json.dumps(dict(kernel="cross_pass", fold=fold, variant=v,
                                          tz=plan.get_tile(0, 2)[2], strip=sw, us=us,
                                          restrict_us=rus, step_us=us + rus,
                                          gbs=c["bytes"] / max(c["ms"], 1e-9) / 1e6)),
                          flush=True)
        plan.close()


def cross_traffic_table(dim, m):
    """Every candidate the autotuner tries for the cross-cycle pass of an FP64
    red-black V(1,1) solve (three-stage tile x z-chunk, restriction folded in
    or not), two launches each inside a two-cycle solve, with one manifest
    line per candidate.  Under a counter profiler restricted to the
    three-stage kernels (FETCH_SIZE, WRITE_SIZE) the dispatches map two by
    two onto the manifest."""
    from . import capi

    L = (m + 1).bit_length() - 1
    g = torch.Generator(device="cuda").manual_seed(0)
    f = torch.rand((m,) * dim, dtype=torch.float64, device="cuda", generator=g) - 0.5
    u = torch.zeros_like(f)
    for fold in (True, False):
        plan = Plan(dim, L, nu1=1, nu2=1, flags=0 if fold else capi.GMG_NO_FUSED_RESTRICT)
        for v in range(plan.tile_variants(3)):
            seen = set()
            for tz in tuner_tz(m):
                try:
                    plan.set_tile(0, 3, v, tz)
                except capi.GmgError:
                    continue
                tzv = plan.get_tile(0, 2)[2]
                if tzv in seen:
                    continue
                seen.add(tzv)
                u.zero_()
                st, it, rel = plan.solve(u, f, rtol=1e-30, maxit=2)
                if it != 2:
                    continue
                print(json.dumps(dict(manifest="cross", dim=dim, m=m, stages=3, variant=v,
                                      tz=tzv, fold=fold, launches=2)), flush=True)
        torch.cuda.synchronize()
        plan.close()


def traffic_report(manifest_log, fetch_csv, write_csv, copy_fetch_csv, copy_write_csv,
                   kernel_regex, title):
    """The counter table of a traffic-table run as markdown: HBM bytes per
    launch of every candidate from FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch), scaled by what the same counters read for the runtime's copy
    of a 1 GiB buffer, and a last line with the table as JSON for bench.py."""
    import csv
    import re

    man = [json.loads(l) for l in open(manifest_log) if l.startswith('{"manifest"')]

    def disp(path, regex):
        rows = [r for r in csv.DictReader(open(path)) if re.search(regex, r["Kernel_Name"])]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        return rows

    fr = disp(fetch_csv, kernel_regex)
    wr = disp(write_csv, kernel_regex)
    need = sum(e["launches"] for e in man)
    if len(fr) != need or len(wr) != need:
        raise SystemExit("dispatch count %d/%d does not match the manifest (%d)" % (
            len(fr), len(wr), need))
    cf = [float(r["Counter_Value"]) for r in disp(copy_fetch_csv, "copyBuffer")]
    cw = [float(r["Counter_Value"]) for r in disp(copy_write_csv, "copyBuffer")]
    gib_kib = float(1 << 20)
    kf, kw = gib_kib / (sum(cf) / len(cf)), gib_kib / (sum(cw) / len(cw))
    out = ["# %s" % title, "",
           "Calibration: the runtime's copy of a 1 GiB buffer (`__amd_rocclr_copyBuffer`) "
           "reads %.0f KiB and writes %.0f KiB per dispatch by these counters, so bytes = "
           "FETCH_SIZE x %.4f x 1024 and WRITE_SIZE x %.4f x 1024." % (
               sum(cf) / len(cf), sum(cw) / len(cw), kf, kw), "",
           "| candidate | kernel | FETCH KiB | WRITE KiB | traffic MB | algorithmic MB | "
           "traffic / alg |", "|---|---|---|---|---|---|---|"]
    table = {}
    i = 0
    for e in man:
        n = e["launches"]
        fk = sum(float(r["Counter_Value"]) for r in fr[i:i + n]) / n
        wk = sum(float(r["Counter_Value"]) for r in wr[i:i + n]) / n
        kern = fr[i]["Kernel_Name"].split("(")[0].replace("void gmg::", "")
        i += n
        m, d = e["m"], e["dim"]
        mc = (m - 1) // 2
        traffic = 1024.0 * (fk * kf + wk * kw)
        if e["manifest"] == "cross":
            # the pass's flags are its last template argument; 16: restriction
            # folded in (a candidate asked to fold whose tile does not fit runs
            # the plain pass, and is filed under it)
            fold = (int(kern.rstrip(">").split(",")[-1]) & 16) != 0
            # w_k, f and the coarse correction read; w_{k+1} (and f_c) written
            alg = 8.0 * (3 * m ** d + mc ** d + (mc ** d if fold else 0))
            key = "%s|%d|%d|%d|%d" % (e["manifest"], e["stages"], e["variant"], e["tz"],
                                      1 if fold else 0)
        else:
            # pre: u, f read, result written; post: the coarse correction too
            alg = 8.0 * (3 * m ** d + (mc ** d if e["manifest"] == "post" else 0))
            key = "%s|%d|%d|%d" % (e["manifest"], e["stages"], e["variant"], e["tz"])
        table[key] = traffic
        out.append("| %s | `%s` | %.0f | %.0f | %.1f | %.1f | %.3f |" % (
            key, kern, fk, wk, traffic / 1e6, alg / 1e6, traffic / alg))
    import hashlib
    import os

    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    sha = {n: hashlib.sha256(open(os.path.join(csrc, n), "rb").read()).hexdigest()
           for n in ("smooth.hip", "gmg_internal.h")}
    out += ["", "traffic-json: " + json.dumps({"tiles": table, "fetch_factor": kf,
                                               "write_factor": kw, "sources_sha256": sha})]
    print("\n".join(out))


def trace_report(trace_csv, title, active_us=5.0):
    """A rocprofv3 kernel trace (--kernel-trace, CSV) as markdown: per kernel
    and grid size, the dispatches, those that did work (longer than
    active_us: the launches a solve enqueues past its stop test return at
    once) and their mean duration.  Meant for traced runs whose tile choices
    come from an autotuner cache (GMG_TUNE_CACHE), so that every dispatch
    belongs to a solve."""
    import csv
    import collections

    rows = list(csv.DictReader(open(trace_csv)))
    agg = collections.OrderedDict()
    for r in rows:
        name = r["Kernel_Name"].split("(")[0].replace("void ", "").replace("gmg::", "")
        grid = int(r.get("Grid_Size_X") or r.get("Grid_Size") or 0)
        wg = int(r.get("Workgroup_Size_X") or r.get("Workgroup_Size") or 0)
        us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        a = agg.setdefault((name, grid, wg), [0, 0, 0.0])
        a[0] += 1
        if us > active_us:
            a[1] += 1
            a[2] += us
    out = ["# %s" % title, "",
           "Dispatches that did work are those longer than %.0f us (launches enqueued past "
           "a solve's stop test return at once)." % active_us, "",
           "| kernel | grid | wg | dispatches | active | avg active (us) | total active (ms) |",
           "|---|---|---|---|---|---|---|"]
    for (name, grid, wg), (n, na, t) in sorted(agg.items(), key=lambda kv: -kv[1][2]):
        out.append("| `%s` | %d | %d | %d | %d | %.2f | %.2f |" % (
            name, grid, wg, n, na, t / na if na else 0.0, t / 1e3))
    print("\n".join(out))


def solve_run(dim, m, cycles, nu=1, precision="fp64"):
    """An autotuned solve of the bench's sine-modes right-hand side cut at
    `cycles` cycles (rtol 1e-30), after one warm-up solve that tunes (or
    reads GMG_TUNE_CACHE): the dispatches a counter profiler sees are those
    of a production solve of this size."""
    from . import capi
    from . import workloads as wl

    L = (m + 1).bit_length() - 1
    f = wl.rhs_sine_modes_device(dim, m, 5, "cuda")
    u = torch.zeros_like(f)
    plan = Plan(dim, L, nu1=nu, nu2=nu, precision=precision, flags=capi.GMG_AUTOTUNE)
    plan.solve(u, f, rtol=1e-30, maxit=2)
    torch.cuda.synchronize()
    u.zero_()
    st, it, rel = plan.solve(u, f, rtol=1e-30, maxit=cycles)
    torch.cuda.synchronize()
    print(json.dumps(dict(solve_run=True, dim=dim, m=m, cycles=it, relres=rel,
                          level0_tiles=[plan.get_tile(0, r) for r in (0, 1)])), flush=True)


def counter_report(pmc_csvs, kernel_regex, title, points, clock_ghz=2.4,
                   active_us=5.0, cus=256):
    """Counters of rocprofv3 --pmc runs, each with --kernel-trace (its
    kernel_trace CSV beside the counter CSV gives every dispatch its
    duration), for the kernels matching kernel_regex that did work (longer
    than active_us), as markdown: the mean
    of every counter per dispatch, and per fine point (points per dispatch)
    the lane-instruction counts; the time the VALU instructions alone need
    at one wave-instruction per 4 cycles per SIMD (FP64 and unpacked FP32
    run 16 lanes a cycle), the LDS bank-conflict cycles per CU, and the
    texture-address unit's busy share, against the measured duration."""
    import collections
    import csv
    import re

    def rows(path):
        return list(csv.DictReader(open(path)))

    groups = collections.OrderedDict()
    for path in pmc_csvs:
        tr = {}
        tpath = path.replace("counter_collection", "kernel_trace")
        for r in rows(tpath):
            tr[r["Dispatch_Id"]] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        for r in rows(path):
            if not re.search(kernel_regex, r["Kernel_Name"]):
                continue
            us = tr.get(r["Dispatch_Id"])
            if us is None or us < active_us:
                continue
            name = r["Kernel_Name"].split("(")[0].replace("void ", "").replace("gmg::", "")
            grid = int(r.get("Grid_Size") or r.get("Grid_Size_X") or 0)
            g = groups.setdefault((name, grid), collections.defaultdict(list))
            g[r["Counter_Name"]].append(float(r["Counter_Value"]))
            g["__us"].append((path, r["Dispatch_Id"], us))
    out = ["# %s" % title, "",
           "Means per dispatch longer than %.0f us. Per point: lane instructions "
           "(wave instructions x 64) per fine point, %d points per dispatch. Clock: "
           "GRBM_GUI_ACTIVE / (8 XCDs x duration) where counted, else %.1f GHz. VALU floor: "
           "SQ_INSTS_VALU x 4 cycles / (4 SIMDs x %d CUs) at that clock. LDS conflict: "
           "SQ_LDS_BANK_CONFLICT / %d CUs at that clock. TA busy: TA_TA_BUSY / (%d x duration "
           "x clock)." % (active_us, points, clock_ghz, cus, cus, cus), ""]
    for (name, grid), g in groups.items():
        usl = list(set(g["__us"]))  # one entry per dispatch of each run
        us = sum(v[2] for v in usl) / len(usl)
        mean = {k: sum(v) / len(v) for k, v in g.items() if k != "__us"}
        out += ["## `%s`, grid %d" % (name, grid), "",
                "duration under the counter runs: %.1f us (mean of %d dispatches in %d runs)" % (
                    us, len(usl), len(pmc_csvs)),
                "", "| counter | mean per dispatch | per fine point |", "|---|---|---|"]
        for k in sorted(mean):
            pp = mean[k] * 64 / points if k.startswith("SQ_INSTS") else mean[k] / points
            out.append("| %s | %.4g | %.3f |" % (k, mean[k], pp))
        out.append("")
        cyc = clock_ghz * 1e3  # cycles per microsecond at the rated clock
        if "GRBM_GUI_ACTIVE" in mean:
            # GRBM_GUI_ACTIVE sums the XCDs' active cycles: its rate over
            # the dispatch is 8 x the shader clock
            cyc = mean["GRBM_GUI_ACTIVE"] / (8 * us)
            out.append("- mean shader clock GRBM_GUI_ACTIVE / (8 x duration): %.2f GHz" % (
                cyc / 1e3))
        if "SQ_INSTS_VALU" in mean:
            fl = mean["SQ_INSTS_VALU"] * 4 / (4 * cus) / cyc
            out.append("- VALU floor at that clock %.1f us = %.0f%% of the duration" % (
                fl, 100 * fl / us))
        if "SQ_LDS_BANK_CONFLICT" in mean:
            lc = mean["SQ_LDS_BANK_CONFLICT"] / cus / cyc
            out.append("- LDS bank-conflict cycles per CU: %.1f us = %.0f%% of the duration" % (
                lc, 100 * lc / us))
        if "TA_TA_BUSY" in mean:
            out.append("- TA busy %.0f%%" % (100 * mean["TA_TA_BUSY"] / cus / (us * cyc)))
        out.append("")
    print("\n".join(out))


def batch_solves(nsolves, flags=0):
    """The bench's 256-problem batch (128 2D problems of side 2^k - 1,
    k ~ U{6..10}, 128 3D with k ~ U{5..7}; U[-1,1) right-hand sides, seed 4;
    FP64 V(2,2) to 1e-10 each; graph-captured cycles, autotuned): one solve
    that tunes (or reads GMG_TUNE_CACHE), then nsolves timed solves.  flags
    are added to the plan's (GMG_BATCH_ONE_STREAM: one stream)."""
    import time

    from . import capi
    from . import workloads as wl
    from .solver import BatchPlan

    probs = wl.batch_problems(4)
    fs = [torch.from_numpy(wl.batch_rhs(4, q, d, m)).cuda() for q, (d, m) in enumerate(probs)]
    us = [torch.zeros_like(f) for f in fs]
    plan = BatchPlan([(d, (m + 1).bit_length() - 1) for d, m in probs],
                     flags=capi.GMG_USE_GRAPH | capi.GMG_AUTOTUNE | flags)
    for k in range(nsolves + 1):
        for u in us:
            u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s, its, rels, sts = plan.solve(us, fs)
        torch.cuda.synchronize()
        print(json.dumps(dict(batch_solve=k, ms=1e3 * (time.perf_counter() - t0),
                              min_cycles=min(its), max_cycles=max(its),
                              all_converged=all(x == 0 for x in sts))), flush=True)


def copy_calibration(mib, reps=20):
    """A plain device copy of known size (torch's copy kernel): the yardstick
    that converts the HBM byte counters of a profiler into bytes.  Also
    torch's elementwise add of two arrays into a third, the same mix of two
    reads and one write per point as a smoothing pass: a streaming ceiling
    for that traffic pattern."""
    n = mib * (1 << 20) // 8
    src = torch.rand(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    us = _time(lambda: dst.copy_(src), reps)
    row = dict(kernel="copy", bytes_read=n * 8, bytes_written=n * 8, us=us,
               gbs=2 * n * 8 / (us * 1e-6) / 1e9)
    print(json.dumps(row), flush=True)
    src2 = torch.rand_like(src)
    us = _time(lambda: torch.add(src, src2, out=dst), reps)
    print(json.dumps(dict(kernel="elementwise_add", bytes_read=2 * n * 8, bytes_written=n * 8,
                          us=us, gbs=3 * n * 8 / (us * 1e-6) / 1e9)), flush=True)
    return row


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="only time a plain copy of this many MiB")
    ap.add_argument("--dim", type=int, default=3)
    ap.add_argument("--m", type=int, nargs="+", default=[255])
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--smoother", default="rbgs")
    ap.add_argument("--tz", type=int, nargs="+", default=[0])
    ap.add_argument("--fp32", action="store_true")
    ap.add_argument("--out", default=None)
    ap.add_argument("--stages", type=int, nargs="+", default=None)
    ap.add_argument("--variants", type=int, nargs="+", default=None)
    ap.add_argument("--kinds", nargs="+", default=["plain", "zero", "prolong", "prolong_bwd"])
    ap.add_argument("--no-transfers", action="store_true")
    ap.add_argument("--cross-sweep", action="store_true",
                    help="time the cross-cycle pass over tiles, z-chunks and tile orders")
    ap.add_argument("--strips", type=int, nargs="+", default=[0, 1, 2, 3, 4, 6, 8])
    ap.add_argument("--cross-traffic-table", action="store_true",
                    help="launch every autotuner candidate of the cross-cycle pass twice "
                    "(for a counter profiler)")
    ap.add_argument("--traffic-report", nargs=5, metavar=("MANIFEST_LOG", "FETCH_CSV",
                                                          "WRITE_CSV", "COPY_FETCH_CSV",
                                                          "COPY_WRITE_CSV"),
                    help="markdown counter table of a traffic-table run")
    ap.add_argument("--trace-report", metavar="KERNEL_TRACE_CSV",
                    help="markdown per-kernel summary of a rocprofv3 kernel trace")
    ap.add_argument("--kernel-regex", default=r"k_rb_pass<double, 3, 3,")
    ap.add_argument("--title", default="HBM traffic of the cross-cycle pass")
    ap.add_argument("--batch-flags", type=lambda v: int(v, 0), default=0,
                    help="plan flags added to the batch plan of --batch-solves")
    ap.add_argument("--batch-solves", type=int, default=0,
                    help="the 256-problem batch: a tuning solve, then this many solves")
    ap.add_argument("--solve-cycles", type=int, default=0,
                    help="one autotuned solve of the sine-modes problem cut at this many cycles")
    ap.add_argument("--counter-report", nargs="+", metavar="CSV",
                    help="counter_collection CSVs of --pmc --kernel-trace runs")
    ap.add_argument("--points", type=int, default=1023 ** 3)
    ap.add_argument("--active-us", type=float, default=5.0,
                    help="counter report: keep dispatches at least this long")
    ap.add_argument("--traffic-table", action="store_true",
                    help="launch every autotuner candidate of the level-0 passes twice "
                    "(for a counter profiler)")
    a = ap.parse_args()
    if a.batch_solves:
        batch_solves(a.batch_solves, a.batch_flags)
        return
    if a.solve_cycles:
        for m in a.m:
            solve_run(a.dim, m, a.solve_cycles)
        return
    if a.counter_report:
        counter_report(a.counter_report, a.kernel_regex, a.title, a.points,
                       active_us=a.active_us)
        return
    if a.cross_sweep:
        for m in a.m:
            cross_sweep(a.dim, m, tuple(a.strips), a.variants,
                        None if a.tz == [0] else a.tz)
        return
    if a.trace_report:
        trace_report(a.trace_report, a.title)
        return
    if a.traffic_report:
        traffic_report(*a.traffic_report, a.kernel_regex, a.title)
        return
    if a.cross_traffic_table:
        for m in a.m:
            cross_traffic_table(a.dim, m)
        return
    if a.traffic_table:
        for m in a.m:
            traffic_table(a.dim, m)
        return
    if a.copy_mib:
        copy_calibration(a.copy_mib, a.reps)
        return
    for m in a.m:
        print("# dim %d m %d" % (a.dim, m), flush=True)
        run(a.dim, m, a.reps, torch.float32 if a.fp32 else torch.float64, a.smoother, a.tz, a.out,
            a.stages, a.variants, a.kinds, not a.no_transfers)


if __name__ == "__main__":
    main()
