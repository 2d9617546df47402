"""GPU checks of plan modes the other files leave out: mixed precision with
weighted Jacobi, with uneven sweep counts and with the flags that change the
schedule (each must reach the FP64 residual by the oracle's own residual);
FP64 solves without temporal blocking, which must give the bits of the
fused-sweep passes (every half-sweep is the same per-point expression); the
captured coarse part against eager launches for every schedule; batches with
the schedule flags against single-problem plans.
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=torch.float64)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def levels_of(m):
    return int(np.log2(m + 1))


MIXED_MODES = [("wj", 2, 2, None), ("rbgs", 1, 2, None), ("rbgs", 2, 1, None),
               ("rbgs", 1, 1, "GMG_POST_FORWARD"), ("rbgs", 2, 2, "GMG_NO_TEMPORAL_BLOCKING"),
               ("rbgs", 1, 1, "GMG_NO_CROSS_CYCLE")]


@pytest.mark.parametrize("dim,m", [(2, 255), (3, 63)])
@pytest.mark.parametrize("smoother,nu1,nu2,flag", MIXED_MODES)
def test_mixed_modes_reach_fp64_residual(dim, m, smoother, nu1, nu2, flag):
    from paper_1208_4247_amd import capi
    from paper_1208_4247_amd.solver import Plan

    flags = getattr(capi, flag) if flag else 0
    f = wl.rhs_uniform(dim, m, seed=200 + m)
    plan = Plan(dim, levels_of(m), smoother=smoother, nu1=nu1, nu2=nu2, precision="mixed",
                flags=flags)
    ud = torch.zeros((m,) * dim, dtype=torch.float64, device="cuda")
    st, it, rel = plan.solve(ud, dev(f), rtol=1e-10, maxit=60)
    r = oracle.norm2(oracle.residual(host(ud), f)) / oracle.norm2(f)
    print("%s V(%d,%d) %s %dD %d: %d steps, relres %.3e (oracle %.3e)" % (
        smoother, nu1, nu2, flag, dim, m, it, rel, r), flush=True)
    assert st == 0
    assert r <= 1e-10
    assert abs(r - rel) <= 1e-3 * max(r, rel)
    plan.close()


@pytest.mark.parametrize("dim,m", [(2, 511), (3, 127)])
@pytest.mark.parametrize("smoother,nu", [("rbgs", 2), ("rbgs", 3), ("wj", 2)])
def test_no_temporal_blocking_same_bits(dim, m, smoother, nu):
    from paper_1208_4247_amd import capi
    from paper_1208_4247_amd.solver import Plan

    fd = dev(wl.rhs_uniform(dim, m, seed=300 + m))
    out = []
    for flags in (0, capi.GMG_NO_TEMPORAL_BLOCKING):
        plan = Plan(dim, levels_of(m), smoother=smoother, nu1=nu, nu2=nu, flags=flags)
        ud = torch.zeros_like(fd)
        st, it, rel = plan.solve(ud, fd, rtol=1e-10)
        out.append((st, it, host(ud)))
        plan.close()
    assert out[0][:2] == out[1][:2] and out[0][0] == 0
    assert np.array_equal(out[0][2], out[1][2])


@pytest.mark.parametrize("kw", [dict(precision="mixed"), dict(smoother="wj"),
                                dict(nu1=1, nu2=1), dict(nu1=1, nu2=1, precision="mixed"),
                                dict(nu1=3, nu2=1)])
def test_graph_replay_equals_eager(kw):
    """The captured coarse part of a cycle (GMG_USE_GRAPH) gives the bits of
    eager launches for every schedule, on the first solve and on replays
    with other work in between."""
    from paper_1208_4247_amd import capi
    from paper_1208_4247_amd.solver import Plan

    fd = dev(wl.rhs_uniform(3, 63, seed=401))
    eager = Plan(3, 6, **kw)
    ue = torch.zeros_like(fd)
    st_e, it_e, _ = eager.solve(ue, fd, rtol=1e-10)
    graph = Plan(3, 6, flags=capi.GMG_USE_GRAPH, **kw)
    for rep in range(3):
        ug = torch.zeros_like(fd)
        _ = torch.ones(1000, device="cuda").sum().item()
        st_g, it_g, _ = graph.solve(ug, fd, rtol=1e-10)
        assert (st_g, it_g) == (st_e, it_e) == (0, it_e)
        assert np.array_equal(host(ug), host(ue)), rep
    eager.close()
    graph.close()


@pytest.mark.parametrize("flag", ["GMG_NO_TEMPORAL_BLOCKING", "GMG_NO_FUSED_RESTRICT",
                                  "GMG_NO_FUSED_COARSE"])
def test_batch_schedule_flags_equal_single_plans(flag):
    """The batch honours the flags that change a plan's schedule: each
    problem gives the bits and cycle count of its own plan with the flag."""
    from paper_1208_4247_amd import capi
    from paper_1208_4247_amd.solver import BatchPlan, Plan

    flags = getattr(capi, flag)
    probs = [(3, 63), (2, 255), (3, 31), (2, 511)]
    fs = [dev(wl.batch_rhs(29, q, d, m)) for q, (d, m) in enumerate(probs)]
    plan = BatchPlan([(d, levels_of(m)) for d, m in probs], flags=flags | capi.GMG_USE_GRAPH)
    us = [torch.zeros_like(f) for f in fs]
    s, its, rels, sts = plan.solve(us, fs, rtol=1e-10)
    for q, (d, m) in enumerate(probs):
        single = Plan(d, levels_of(m), flags=flags)
        ud = torch.zeros_like(fs[q])
        st, it, _ = single.solve(ud, fs[q], rtol=1e-10)
        assert (sts[q], its[q]) == (st, it) == (0, it), (q, d, m)
        assert np.array_equal(host(us[q]), host(ud)), (q, d, m)
        single.close()


@pytest.mark.parametrize("dim,L", [(2, 7), (3, 5)])
def test_paper_variant_graph_and_profile_flags_same_bits(dim, L):
    """The paper's smoother and transfers (multicolour GS, finite-element
    transfers) under GMG_USE_GRAPH and GMG_PROFILE: the bits and cycle count
    of the plain plan."""
    from paper_1208_4247_amd import capi
    from paper_1208_4247_amd.solver import Plan

    m = (1 << L) - 1
    fd = dev(wl.rhs_uniform(dim, m, seed=500 + m))
    out = []
    for extra in (0, capi.GMG_USE_GRAPH, capi.GMG_PROFILE):
        plan = Plan(dim, L, smoother="mcgs", nu1=1, nu2=1, flags=capi.GMG_FE_TRANSFER | extra)
        for _ in range(2):
            ud = torch.zeros_like(fd)
            st, it, rel = plan.solve(ud, fd, rtol=1e-8)
            out.append((st, it, host(ud)))
        plan.close()
    for st, it, u in out[1:]:
        assert (st, it) == out[0][:2] and out[0][0] == 0
        assert np.array_equal(u, out[0][2])


def test_batch_profile_mode_same_bits():
    """A profiled batch (every launch timed on the plan's stream, one branch)
    gives the bits and cycle counts of the unprofiled, two-branch batch."""
    from paper_1208_4247_amd import capi
    from paper_1208_4247_amd.solver import BatchPlan

    probs = [(3, 63), (2, 255), (3, 31), (2, 127)]
    fs = [dev(wl.batch_rhs(31, q, d, m)) for q, (d, m) in enumerate(probs)]
    out = []
    for flags in (capi.GMG_USE_GRAPH, capi.GMG_PROFILE):
        plan = BatchPlan([(d, levels_of(m)) for d, m in probs], flags=flags)
        us = [torch.zeros_like(f) for f in fs]
        s, its, rels, sts = plan.solve(us, fs, rtol=1e-10)
        out.append((list(its), list(sts), [host(u) for u in us]))
        plan.close()
    assert out[0][0] == out[1][0] and out[0][1] == out[1][1] == [0] * len(probs)
    for a, b in zip(out[0][2], out[1][2]):
        assert np.array_equal(a, b)


SWEEP_CASES = [(2, 7), (2, 127), (2, 1023), (3, 3), (3, 31), (3, 127)]


@pytest.mark.parametrize("dim,m", SWEEP_CASES)
@pytest.mark.parametrize("nsweeps,backward", [(1, False), (2, True), (3, False)])
def test_fp64_sweeps_give_the_oracles_bits(dim, m, nsweeps, backward):
    """Every FP64 pointwise solve is (h^2 f + nb) / (2d) rounded as written,
    with the oracle's neighbour order (x-1, x+1, y-1, y+1, z-1, z+1): a
    red-black or weighted-Jacobi pass over any tile gives the oracle's sweep
    bit for bit."""
    from paper_1208_4247_amd.solver import Plan

    f = wl.rhs_uniform(dim, m, seed=600 + m)
    u0 = wl.rhs_uniform(dim, m, seed=700 + m) * 1e-3
    out = torch.empty((m,) * dim, dtype=torch.float64, device="cuda")
    plan = Plan(dim, levels_of(m), nu1=3, nu2=3)
    plan.op_smooth(0, nsweeps, backward, dev(u0), dev(f), None, out)
    assert np.array_equal(host(out), oracle.rbgs(u0, f, nsweeps, backward=backward))
    plan.close()
    omega = 2 * dim / (2 * dim + 1)
    plan = Plan(dim, levels_of(m), smoother="wj", omega=omega, nu1=3, nu2=3)
    plan.op_smooth(0, nsweeps, False, dev(u0), dev(f), None, out)
    assert np.array_equal(host(out), oracle.wj(u0, f, omega, nsweeps))
    plan.close()


@pytest.mark.parametrize("dim,m", [(2, 127), (3, 31), (3, 127)])
@pytest.mark.parametrize("scale", [2.0 ** -900, 1e-250, 1e250, 2.0 ** 1000])
def test_fp64_sweeps_give_the_oracles_bits_at_extreme_scales(dim, m, scale):
    """The same bitwise equality with the data scaled far from 1, so that
    the quotients by 6 (and by 4) of the pointwise solve run over operands
    near both ends of the exponent range (|h^2 f + nb| down to about 2^-910
    and up to about 2^1000)."""
    from paper_1208_4247_amd.solver import Plan

    f = wl.rhs_uniform(dim, m, seed=800 + m) * scale
    u0 = wl.rhs_uniform(dim, m, seed=900 + m) * (scale / 16.0)
    assert np.all(np.isfinite(f)) and np.all(np.isfinite(u0))
    out = torch.empty((m,) * dim, dtype=torch.float64, device="cuda")
    plan = Plan(dim, levels_of(m), nu1=2, nu2=2)
    plan.op_smooth(0, 2, True, dev(u0), dev(f), None, out)
    want = oracle.rbgs(u0, f, 2, backward=True)
    assert np.all(np.isfinite(want))
    assert np.array_equal(host(out), want)
    plan.close()
    omega = 2 * dim / (2 * dim + 1)
    plan = Plan(dim, levels_of(m), smoother="wj", omega=omega, nu1=2, nu2=2)
    plan.op_smooth(0, 2, False, dev(u0), dev(f), None, out)
    assert np.array_equal(host(out), oracle.wj(u0, f, omega, 2))
    plan.close()
