"""GPU parity: every kernel of the hot path, one V-cycle and whole solves,
through the C ABI, against the FP64 CPU oracle on identical seeded inputs.

Bars (FP64): kernels and single cycles within 1e-13 of the oracle (relative
to the array's max-abs), full solves with the same cycle count and iterates
within 1e-12 relative (2-norm).  The oracle never contracts multiply-adds and
divides by 2d where the GPU multiplies by 1/(2d) and uses fused multiply-adds,
so the two differ by rounding only.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1208_4247_amd import workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1208_4247_amd import capi

    capi.lib()
    oracle.build()


def Plan(*a, **k):
    from paper_1208_4247_amd.solver import Plan as P

    return P(*a, **k)


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def maxrel(a, b):
    den = max(float(np.max(np.abs(b))), 1e-300)
    return float(np.max(np.abs(a - b))) / den


def rel2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def levels_of(m):
    return int(np.log2(m + 1))


# ------------------------------------------------------------------ smoother

SMOOTH_CASES = [
    (2, 7), (2, 31), (2, 127), (2, 255), (2, 1023),
    (3, 3), (3, 15), (3, 31), (3, 63), (3, 127),
]


@pytest.mark.parametrize("dim,m", SMOOTH_CASES)
@pytest.mark.parametrize("nsweeps", [1, 2, 3])
@pytest.mark.parametrize("backward", [False, True])
def test_rb_smooth_parity(dim, m, nsweeps, backward):
    L = levels_of(m)
    plan = Plan(dim, L, nu1=3, nu2=3)  # nu 3 -> plans carry the chained-pass scratch
    f = wl.rhs_uniform(dim, m, seed=100 + m)
    u0 = wl.rhs_uniform(dim, m, seed=200 + m) * 1e-3
    want = oracle.rbgs(u0, f, nsweeps, backward=backward)
    out = torch.empty((m,) * dim, dtype=torch.float64, device="cuda")
    plan.op_smooth(0, nsweeps, backward, dev(u0), dev(f), None, out)
    assert maxrel(host(out), want) <= 1e-13


@pytest.mark.parametrize("dim,m", [(2, 63), (2, 511), (3, 31), (3, 63)])
@pytest.mark.parametrize("stages", [2, 4])
def test_rb_smooth_every_tile_variant_bitwise(dim, m, stages):
    """Every tile shape and z-chunk gives the same bits (one pass of
    stages/2 sweeps)."""
    plan = Plan(dim, levels_of(m))
    f = dev(wl.rhs_uniform(dim, m, seed=7))
    u0 = dev(wl.rhs_uniform(dim, m, seed=8))
    ref = None
    for v in range(plan.tile_variants(stages)):
        for tz in (0, 5, m):
            plan.set_tile(0, stages, v, tz)
            out = torch.empty_like(f)
            plan.op_smooth(0, stages // 2, False, u0, f, None, out)
            got = host(out)
            if ref is None:
                ref = got
                assert maxrel(got, oracle.rbgs(host(u0), host(f), stages // 2)) <= 1e-13
            assert np.array_equal(got, ref), (v, tz)


@pytest.mark.parametrize("dim,m", [(2, 127), (3, 31), (3, 63)])
@pytest.mark.parametrize("backward", [False, True])
def test_rb_smooth_zero_start_and_prolong(dim, m, backward):
    """Fused variants: zero start value (coarse levels) and start value
    u + P e (the ascent's prolongation fused into the first post-sweep)."""
    L = levels_of(m)
    mc = (m - 1) // 2
    plan = Plan(dim, L)
    f = wl.rhs_uniform(dim, m, seed=11)
    w = wl.rhs_uniform(dim, m, seed=12) * 1e-3
    e = wl.rhs_uniform(dim, mc, seed=13) * 1e-3
    out = torch.empty((m,) * dim, dtype=torch.float64, device="cuda")
    plan.op_smooth(0, 2, backward, None, dev(f), None, out)
    assert maxrel(host(out), oracle.rbgs(np.zeros_like(f), f, 2, backward)) <= 1e-13
    plan.op_smooth(0, 2, backward, dev(w), dev(f), dev(e), out)
    want = oracle.rbgs(oracle.prolong_add(e, w), f, 2, backward)
    assert maxrel(host(out), want) <= 1e-13


@pytest.mark.parametrize("dim,m", [(2, 3), (2, 127), (2, 1023), (3, 3), (3, 31), (3, 127),
                                   (3, 255)])
@pytest.mark.parametrize("with_in", [False, True])
def test_prolong_add_parity(dim, m, with_in):
    """The stand-alone (bi/tri)linear interpolation (full multigrid's
    interpolation into zero, and u + P e): every fine parity, the zero coarse
    boundary on all sides, in place and out of place."""
    plan = Plan(dim, levels_of(m))
    mc = (m - 1) // 2
    e = wl.rhs_uniform(dim, mc, seed=140 + m)
    u = wl.rhs_uniform(dim, m, seed=141 + m) if with_in else np.zeros((m,) * dim)
    want = oracle.prolong_add(e, u)
    out = torch.empty((m,) * dim, dtype=torch.float64, device="cuda")
    plan.op_prolong_add(0, dev(u) if with_in else None, dev(e), out)
    assert maxrel(host(out), want) <= 1e-15
    ud = dev(u)
    plan.op_prolong_add(0, ud, dev(e), ud)
    assert maxrel(host(ud), want) <= 1e-15


@pytest.mark.parametrize("dim,m", [(2, 63), (2, 1023), (3, 31), (3, 127)])
@pytest.mark.parametrize("nsweeps", [0, 1, 2])
def test_fused_input_residual_norm(dim, m, nsweeps):
    """The pre-smoothing pass reports ||f - A u_in|| of its start value."""
    plan = Plan(dim, levels_of(m))
    f = wl.rhs_uniform(dim, m, seed=21)
    u0 = wl.rhs_uniform(dim, m, seed=22) * 1e-4
    out = torch.empty((m,) * dim, dtype=torch.float64, device="cuda")
    nrm = plan.op_smooth(0, nsweeps, False, dev(u0), dev(f), None, out, want_norm=True)
    want = oracle.norm2(oracle.residual(u0, f))
    assert abs(nrm - want) <= 1e-12 * want


@pytest.mark.parametrize("dim,m,omega", [(2, 127, 0.8), (2, 255, 2 / 3), (3, 31, 6 / 7), (3, 63, 6 / 7)])
@pytest.mark.parametrize("nsweeps", [1, 2, 3])
def test_wj_smooth_parity(dim, m, omega, nsweeps):
    plan = Plan(dim, levels_of(m), smoother="wj", omega=omega, nu1=3, nu2=3)
    f = wl.rhs_uniform(dim, m, seed=31)
    u0 = wl.rhs_uniform(dim, m, seed=32) * 1e-3
    out = torch.empty((m,) * dim, dtype=torch.float64, device="cuda")
    plan.op_smooth(0, nsweeps, False, dev(u0), dev(f), None, out)
    assert maxrel(host(out), oracle.wj(u0, f, omega, nsweeps)) <= 1e-13


# ------------------------------------------------------------------ transfers


@pytest.mark.parametrize("dim,m", [(2, 3), (2, 63), (2, 255), (2, 1023), (3, 3), (3, 15), (3, 63), (3, 127)])
def test_residual_restriction_parity(dim, m):
    plan = Plan(dim, levels_of(m))
    mc = (m - 1) // 2
    f = wl.rhs_uniform(dim, m, seed=41)
    u = wl.rhs_uniform(dim, m, seed=42) * 1e-3
    fc = torch.empty((mc,) * dim, dtype=torch.float64, device="cuda")
    plan.op_restrict_residual(0, dev(u), dev(f), fc)
    want = oracle.restrict_fw(oracle.residual(u, f))
    assert maxrel(host(fc), want) <= 1e-13


@pytest.mark.parametrize("dim,m", [(2, 1), (2, 127), (3, 1), (3, 31)])
def test_residual_and_norm_parity(dim, m):
    plan = Plan(dim, levels_of(m))
    f = wl.rhs_uniform(dim, m, seed=51)
    u = wl.rhs_uniform(dim, m, seed=52) * 1e-3
    r = torch.empty((m,) * dim, dtype=torch.float64, device="cuda")
    nrm = plan.op_residual(0, dev(u), dev(f), r)
    want = oracle.residual(u, f)
    assert maxrel(host(r), want) <= 1e-13
    assert abs(nrm - oracle.norm2(want)) <= 1e-13 * oracle.norm2(want)


# ------------------------------------------------------------------ cycles and solves

CYCLE_CASES = [(2, 1), (2, 3), (2, 7), (2, 63), (2, 127), (2, 511), (3, 1), (3, 3), (3, 7),
               (3, 15), (3, 31), (3, 63), (3, 127)]


@pytest.mark.parametrize("dim,m", CYCLE_CASES)
@pytest.mark.parametrize("nu", [(2, 2), (1, 1), (1, 0), (0, 2), (3, 1)])
def test_vcycle_parity(dim, m, nu):
    L = levels_of(m)
    plan = Plan(dim, L, nu1=nu[0], nu2=nu[1])
    f = wl.rhs_uniform(dim, m, seed=61)
    u0 = wl.rhs_uniform(dim, m, seed=62) * 1e-3
    ud = dev(u0)
    plan.vcycle(ud, dev(f))
    want = oracle.vcycle(u0, f, nu[0], nu[1])
    assert maxrel(host(ud), want) <= 1e-12


@pytest.mark.parametrize("dim,m", [(2, 63), (3, 31)])
def test_vcycle_parity_wj(dim, m):
    plan = Plan(dim, levels_of(m), smoother="wj", nu1=2, nu2=2)
    omega = 0.8 if dim == 2 else 6 / 7
    f = wl.rhs_uniform(dim, m, seed=63)
    u0 = wl.rhs_uniform(dim, m, seed=64) * 1e-3
    ud = dev(u0)
    plan.vcycle(ud, dev(f))
    want = oracle.vcycle(u0, f, 2, 2, smoother=oracle.WJ, omega=omega)
    assert maxrel(host(ud), want) <= 1e-12


@pytest.mark.parametrize("dim,m", [(2, 7), (2, 127), (2, 511), (3, 7), (3, 31), (3, 63), (3, 127)])
def test_solve_parity(dim, m):
    """Same cycle count as the oracle and iterates within 1e-12."""
    L = levels_of(m)
    f = wl.rhs_uniform(dim, m, seed=71)
    u_ref, it_ref, rel_ref, st_ref, _ = oracle.solve(f, rtol=1e-10, maxit=60)
    plan = Plan(dim, L)
    ud = torch.zeros((m,) * dim, dtype=torch.float64, device="cuda")
    st, it, rel = plan.solve(ud, dev(f), rtol=1e-10, maxit=60)
    assert (st, it) == (st_ref, it_ref)
    assert rel2(host(ud), u_ref) <= 1e-12
    assert rel <= 1e-10 and abs(rel - rel_ref) <= 1e-3 * rel_ref


def test_solve_poisson2d_127_sine():
    """2D 127^2, f = 2 pi^2 sin(pi x) sin(pi y), V(2,2) RB-GS to 1e-10."""
    f = wl.rhs_sine(2, 127)
    u_ref, it_ref, rel_ref, st_ref, _ = oracle.solve(f, rtol=1e-10)
    plan = Plan(2, 7)
    ud = torch.zeros((127, 127), dtype=torch.float64, device="cuda")
    st, it, rel = plan.solve(ud, dev(f), rtol=1e-10)
    assert st == 0 and it == it_ref
    assert rel2(host(ud), u_ref) <= 1e-12


def test_solve_poisson3d_255_sine_noise():
    """3D 255^3, f = 3 pi^2 prod sin + 1e-3 U[-1,1] (seed 2), FP64 V(2,2) to
    1e-10: the benchmark workload, full-array parity with the oracle."""
    f = wl.rhs_sine_plus_noise(3, 255, 2)
    u_ref, it_ref, rel_ref, st_ref, _ = oracle.solve(f, rtol=1e-10)
    plan = Plan(3, 8)
    ud = torch.zeros((255,) * 3, dtype=torch.float64, device="cuda")
    st, it, rel = plan.solve(ud, dev(f), rtol=1e-10)
    assert st == 0 and it == it_ref, (it, it_ref)
    assert rel2(host(ud), u_ref) <= 1e-12


def test_solve_resume_and_maxit():
    f = wl.rhs_uniform(3, 31, seed=81)
    plan = Plan(3, 5)
    fd = dev(f)
    ud = torch.zeros_like(fd)
    st, it, rel = plan.solve(ud, fd, rtol=1e-10)
    u_full = host(ud)
    ud.zero_()
    st3, it3, rel3 = plan.solve(ud, fd, rtol=1e-10, maxit=3)
    assert st3 == 1 and it3 == 3
    res0 = oracle.norm2(f)
    st4, it4, rel4 = plan.solve(ud, fd, rtol=1e-10, res0=res0)
    assert st4 == 0 and it4 == it - 3
    assert np.array_equal(host(ud), u_full)
    z = torch.zeros_like(fd)
    assert plan.solve(z.clone(), z, rtol=1e-10)[:2] == (0, 0)


def test_solve_nonfinite_rhs():
    f = wl.rhs_uniform(2, 31, seed=82)
    f[3, 4] = np.nan
    plan = Plan(2, 5)
    from paper_1208_4247_amd import capi

    with pytest.raises(capi.GmgError) as ei:
        plan.solve(torch.zeros((31, 31), dtype=torch.float64, device="cuda"), dev(f))
    assert ei.value.status == capi.GMG_ERR_NONFINITE


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_solve_reports_divergence(precision):
    """Algorithm 3's loop with a resumed reference norm far below the
    residual of the start value: after the first cycle the residual is still
    above 1e3 times that reference, so the solve stops with
    GMG_ERR_DIVERGED and still reports its cycle count and relative
    residual.  Ordinary inputs; the stop test is what is exercised."""
    import ctypes

    from paper_1208_4247_amd import capi
    from paper_1208_4247_amd.solver import _ptr

    f = wl.rhs_uniform(3, 31, seed=84)
    plan = Plan(3, 5, precision=precision)
    fd = dev(f)
    ud = torch.zeros_like(fd)
    it, rel = ctypes.c_int(-1), ctypes.c_double(-1.0)
    res0 = ctypes.c_double(1e-30)
    s = capi.lib().gmg_solve(plan.handle, _ptr(ud), _ptr(fd), 1e-10, 50, ctypes.byref(res0),
                             ctypes.byref(it), ctypes.byref(rel))
    torch.cuda.synchronize()
    assert s == capi.GMG_ERR_DIVERGED, capi.status_string(s)
    assert it.value == 1
    # relres = ||f - A u_1|| / 1e-30 with u_1 the first iterate: one cycle
    # from zero, or (mixed) one refinement step of inner_cycles FP32 cycles,
    # which equals that many cycles up to FP32 rounding of the correction
    u1 = np.zeros_like(f)
    for _ in range(1 if precision == "fp64" else plan.cfg.inner_cycles):
        u1 = oracle.vcycle(u1, f, 2, 2)
    want = oracle.norm2(oracle.residual(u1, f)) / 1e-30
    assert abs(rel.value / want - 1.0) < (1e-9 if precision == "fp64" else 1e-3)
    assert plan.solve(torch.zeros_like(fd), fd, rtol=1e-10)[0] == capi.GMG_OK


def test_run_to_run_bitwise():
    f = dev(wl.rhs_uniform(3, 63, seed=83))
    plan = Plan(3, 6)
    outs = []
    for _ in range(2):
        ud = torch.zeros_like(f)
        plan.solve(ud, f, rtol=1e-10)
        outs.append(host(ud))
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("dim,m", [(3, 31), (3, 127), (2, 255), (2, 1023)])
@pytest.mark.parametrize("nu", [(2, 2), (1, 1), (1, 2)])
@pytest.mark.parametrize("post_forward", [False, True])
def test_fused_coarse_kernels_bitwise(dim, m, nu, post_forward):
    """The LDS-tile kernels of the small coarse levels give the same bits as
    the general passes + restriction on those levels."""
    from paper_1208_4247_amd import capi

    f = dev(wl.rhs_uniform(dim, m, seed=65))
    u0 = dev(wl.rhs_uniform(dim, m, seed=66) * 1e-3)
    base = capi.GMG_POST_FORWARD if post_forward else 0
    outs = []
    for flags in (base, base | capi.GMG_NO_FUSED_COARSE):
        plan = Plan(dim, levels_of(m), nu1=nu[0], nu2=nu[1], flags=flags)
        ud = u0.clone()
        plan.vcycle(ud, f)
        outs.append(host(ud))
    assert np.array_equal(outs[0], outs[1])
    want = oracle.vcycle(host(u0), host(f), nu[0], nu[1]) if not post_forward else None
    if want is not None:
        assert maxrel(outs[0], want) <= 1e-12


@pytest.mark.parametrize("dim,m,nu,coarse_passes", [(3, 63, (2, 2), True), (3, 127, (2, 2), False),
                                                    (3, 127, (1, 1), True), (2, 255, (2, 2), True),
                                                    (3, 63, (3, 2), True), (2, 127, (1, 2), False)])
def test_fused_restriction_bitwise(dim, m, nu, coarse_passes):
    """Residual + full weighting inside the last pre-smoothing pass gives the
    same bits as the separate restriction kernel, on level 0 and (general
    passes on the coarse levels) on every level, for one cycle and a solve."""
    from paper_1208_4247_amd import capi

    f = dev(wl.rhs_uniform(dim, m, seed=71))
    u0 = dev(wl.rhs_uniform(dim, m, seed=72) * 1e-3)
    base = capi.GMG_NO_FUSED_COARSE if coarse_passes else 0
    cyc, sol = [], []
    for flags in (base, base | capi.GMG_NO_FUSED_RESTRICT):
        plan = Plan(dim, levels_of(m), nu1=nu[0], nu2=nu[1], flags=flags)
        ud = u0.clone()
        plan.vcycle(ud, f)
        cyc.append(host(ud))
        ud = torch.zeros_like(f)
        st, it, rel = plan.solve(ud, f, rtol=1e-10)
        sol.append((st, it, host(ud)))
    assert np.array_equal(cyc[0], cyc[1])
    assert sol[0][:2] == sol[1][:2] and np.array_equal(sol[0][2], sol[1][2])
    want = oracle.vcycle(host(u0), host(f), nu[0], nu[1])
    assert maxrel(cyc[0], want) <= 1e-12


@pytest.mark.parametrize("stages", [2, 4])
def test_fused_restriction_every_tile_bitwise(stages):
    """Every tile shape and z-chunk of the fused pass (where it fits) gives
    the bits of the separate restriction."""
    from paper_1208_4247_amd import capi

    m = 127
    f = dev(wl.rhs_uniform(3, m, seed=73))
    u0 = dev(wl.rhs_uniform(3, m, seed=74) * 1e-3)
    ref = Plan(3, 7, flags=capi.GMG_NO_FUSED_RESTRICT)
    ud = u0.clone()
    ref.vcycle(ud, f)
    want = host(ud)
    plan = Plan(3, 7)
    for v in range(plan.tile_variants(stages)):
        for tz in (8, 16, 0):
            plan.set_tile(0, stages, v, tz)
            ud = u0.clone()
            plan.vcycle(ud, f)
            assert np.array_equal(host(ud), want), (stages, v, tz)


# ------------------------------------------------------------------ profiling


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_profile_counts_only_launches_that_ran(precision):
    """The solve loop enqueues cycles ahead of its stop test; the launches of
    cycles after the stopping one exit at once and must not enter the
    profile (their near-zero durations would deflate per-launch averages).
    FP64: the pre-pass runs once per cycle plus once for the final norm; the
    post-pass and restriction once per cycle.  Mixed: one refinement step
    per cycle plus the final one."""
    from paper_1208_4247_amd import capi

    f = dev(wl.rhs_uniform(3, 127, seed=21))
    plan = Plan(3, 7, precision=precision, flags=capi.GMG_PROFILE)
    u = torch.zeros_like(f)
    st, it, rel = plan.solve(u, f, rtol=1e-10)
    prof = plan.profile()
    assert st == 0 and it >= 3
    if precision == "fp64":
        # passes per smoothing step: nu = 2 sweeps in passes of stages / 2 sweeps
        npre = 2 // (plan.get_tile(0, 0)[0] // 2)
        npost = 2 // (plan.get_tile(0, 1)[0] // 2)
        assert prof["smooth_pre_l0"]["launches"] == npre * (it + 1)
        assert prof["smooth_post_l0"]["launches"] == npost * it
        # the restriction runs inside the last pre-pass (then a separate stop
        # test follows every pre-smoothing) or as its own kernel
        nres = prof["resid_restrict_l0"]["launches"]
        assert nres in (0, it)
        if nres == 0:
            assert prof["finalize"]["launches"] == it + 1
        assert prof["bottom"]["launches"] == it
    else:
        assert prof["ir_step"]["launches"] == it + 1
        assert prof["bottom"]["launches"] == it * plan.cfg.inner_cycles
    # a second solve accumulates the same counts again
    u.zero_()
    plan.solve(u, f, rtol=1e-10)
    prof2 = plan.profile()
    key = "smooth_pre_l0" if precision == "fp64" else "ir_step"
    assert prof2[key]["launches"] == 2 * prof[key]["launches"]


# ------------------------------------------------------------------ FMG


@pytest.mark.parametrize("dim,m,nu,smoother", [
    (2, 127, (1, 1), "rbgs"), (2, 255, (2, 2), "rbgs"), (3, 63, (1, 1), "rbgs"),
    (3, 127, (2, 2), "rbgs"), (3, 31, (2, 1), "rbgs"), (2, 63, (2, 2), "wj"),
    (3, 63, (1, 1), "wj"), (2, 7, (1, 1), "rbgs"), (3, 3, (1, 1), "rbgs"), (3, 1, (1, 1), "rbgs")])
def test_fmg_matches_oracle(dim, m, nu, smoother):
    """Full multigrid (Algorithm 2) on the GPU equals the oracle's FMG."""
    fh = wl.rhs_sine(dim, m) + 0.1 * wl.rhs_uniform(dim, m, seed=81)
    f = dev(fh)
    plan = Plan(dim, levels_of(m), nu1=nu[0], nu2=nu[1], smoother=smoother)
    u = torch.full_like(f, float("nan"))  # output only
    plan.fmg(u, f)
    omega = 2 * dim / (2 * dim + 1)
    want = oracle.fmg(fh, nu[0], nu[1], smoother=oracle.WJ if smoother == "wj" else oracle.RBGS,
                      omega=omega)
    assert maxrel(host(u), want) <= 1e-12


def test_fmg_reaches_discretisation_accuracy():
    """FMG for the model problem lands within a small factor of the
    discretisation error of the exact discrete solution, as the FMG columns
    of Tables 12 and 14 do (the oracle's pin uses the same bounds: 2D
    FMG(2,2) within 1.5x, 3D FMG(3,3) within 3x)."""
    for dim, m, nu, bound in ((2, 255, 2, 1.5), (3, 127, 3, 3.0)):
        fh = wl.rhs_sine(dim, m)
        plan = Plan(dim, levels_of(m), nu1=nu, nu2=nu)
        u = torch.zeros_like(dev(fh))
        plan.fmg(u, dev(fh))
        exact = wl.sine_product(dim, m)
        h = 1.0 / (m + 1)
        err = float(np.sqrt(h ** dim * np.sum((host(u) - exact) ** 2)))
        ud, *_ = oracle.solve(fh, rtol=1e-12)
        disc = float(np.sqrt(h ** dim * np.sum((ud - exact) ** 2)))
        assert err <= bound * disc, (dim, m, err, disc)
