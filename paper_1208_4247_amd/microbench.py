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
    ap.add_argument("--traffic-table", action="store_true",
                    help="launch every autotuner candidate of the level-0 passes twice "
                    "(for a counter profiler)")
    a = ap.parse_args()
    if a.cross_sweep:
        for m in a.m:
            cross_sweep(a.dim, m, tuple(a.strips), a.variants,
                        None if a.tz == [0] else a.tz)
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
