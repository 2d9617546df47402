"""GPU checks of the cross-cycle schedule of FP64 red-black V(1,1) solves.

Between two cycles the level-0 post-smoothing sweep of cycle k (black, red:
Algorithm 1's backward sweep) and the forward pre-smoothing sweep of cycle
k+1 (red, black) run as one pass.  The second red half-sweep recomputes the
red values just formed from the same black neighbours, so it is left out
and the pass has three stages; it also emits the residual norm of the
cycle's iterate u_k for Algorithm 3's stop test, and u_k is formed only
once, after the last cycle.  Every per-point expression is the one of the
two-pass schedule, so iterates are bitwise those of GMG_NO_CROSS_CYCLE
plans (the norms are summed in another order); the solves also equal the
FP64 oracle's (same cycle count, iterates within 1e-12).
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


def capi():
    from paper_1208_4247_amd import capi as c

    return c


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def levels_of(m):
    return int(np.log2(m + 1))


def solve(plan, f, **kw):
    u = torch.zeros_like(f)
    st, it, rel = plan.solve(u, f, **kw)
    return st, it, rel, host(u)


@pytest.mark.parametrize("dim,m", [(2, 7), (2, 127), (2, 1023), (3, 7), (3, 31), (3, 63),
                                   (3, 127)])
def test_cross_solve_matches_oracle_and_two_pass_schedule(dim, m):
    f = wl.rhs_uniform(dim, m, seed=201)
    u_ref, it_ref, rel_ref, st_ref, _ = oracle.solve(f, nu1=1, nu2=1, rtol=1e-10, maxit=80)
    fd = dev(f)
    plan = Plan(dim, levels_of(m), nu1=1, nu2=1)
    st, it, rel, u = solve(plan, fd, rtol=1e-10, maxit=80)
    assert (st, it) == (st_ref, it_ref)
    assert rel2(u, u_ref) <= 1e-12
    assert abs(rel - rel_ref) <= 1e-3 * rel_ref  # the residual amplifies last-bit differences
    two = Plan(dim, levels_of(m), nu1=1, nu2=1, flags=capi().GMG_NO_CROSS_CYCLE)
    st2, it2, rel2_, u2 = solve(two, fd, rtol=1e-10, maxit=80)
    assert (st2, it2) == (st, it)
    assert np.array_equal(u, u2)
    assert abs(rel - rel2_) <= 1e-12 * rel2_


@pytest.mark.parametrize("dim,m", [(3, 63), (3, 127), (2, 255)])
def test_cross_every_tile_and_chunk_bitwise(dim, m):
    """Every three-stage tile, with and without the folded restriction,
    at several z-chunks: the same iterate bit for bit."""
    c = capi()
    f = dev(wl.rhs_uniform(dim, m, seed=202))
    ref = solve(Plan(dim, levels_of(m), nu1=1, nu2=1, flags=c.GMG_NO_CROSS_CYCLE), f,
                rtol=1e-10)
    nv = c.lib().gmg_tile_variant_count(dim, 0, 3)
    assert nv >= 2
    for flags in (0, c.GMG_NO_FUSED_RESTRICT):
        for v in range(nv):
            for tz in (0, 5, 16):
                plan = Plan(dim, levels_of(m), nu1=1, nu2=1, flags=flags)
                try:
                    plan.set_tile(0, 3, v, tz)
                except c.GmgError:
                    continue  # more workgroups than the partial-sum buffer holds
                assert plan.get_tile(0, 2)[:2] == (3, v)
                st, it, rel, u = solve(plan, f, rtol=1e-10)
                assert (st, it) == ref[:2], (flags, v, tz)
                assert np.array_equal(u, ref[3]), (flags, v, tz)


def test_cross_maxit_resume_zero_and_profile():
    c = capi()
    f = wl.rhs_uniform(3, 31, seed=203)
    fd = dev(f)
    plan = Plan(3, 5, nu1=1, nu2=1, flags=c.GMG_PROFILE)
    st, it, rel, u_full = solve(plan, fd, rtol=1e-10)
    prof = plan.profile()
    assert st == 0 and it >= 5
    # one pre-pass (cycle 1), one cross pass per later cycle boundary, the
    # closing post-pass; the stop test after each of them
    assert prof["smooth_pre_l0"]["launches"] == 1
    assert prof["smooth_cross_l0"]["launches"] == it
    assert prof["smooth_post_l0"]["launches"] == 1
    # maxit: the iterate after exactly maxit cycles lands in u
    for maxit in (1, 2, 3):
        ud = torch.zeros_like(fd)
        st3, it3, rel3 = plan.solve(ud, fd, rtol=1e-10, maxit=maxit)
        assert (st3, it3) == (1, maxit)
        want = np.zeros_like(f)
        for _ in range(maxit):
            want = oracle.vcycle(want, f, 1, 1)
        assert rel2(host(ud), want) <= 1e-12
    # resume from the 3-cycle iterate with the original reference norm
    ud = torch.zeros_like(fd)
    plan.solve(ud, fd, rtol=1e-10, maxit=3)
    st4, it4, rel4 = plan.solve(ud, fd, rtol=1e-10, res0=oracle.norm2(f))
    assert st4 == 0 and it4 == it - 3
    assert np.array_equal(host(ud), u_full)
    # zero right-hand side: converged before any cycle, u untouched
    z = torch.zeros_like(fd)
    u0 = torch.full_like(fd, 0.0)
    assert plan.solve(u0, z, rtol=1e-10)[:2] == (0, 0)


def test_cross_nonfinite_and_diverged():
    import ctypes

    c = capi()
    from paper_1208_4247_amd.solver import _ptr

    f = wl.rhs_uniform(3, 31, seed=204)
    f[5, 6, 7] = np.inf
    plan = Plan(3, 5, nu1=1, nu2=1)
    with pytest.raises(c.GmgError) as ei:
        plan.solve(torch.zeros((31,) * 3, dtype=torch.float64, device="cuda"), dev(f))
    assert ei.value.status == c.GMG_ERR_NONFINITE
    g = dev(wl.rhs_uniform(3, 31, seed=205))
    ud = torch.zeros_like(g)
    it, rel = ctypes.c_int(-1), ctypes.c_double(-1.0)
    r0 = ctypes.c_double(1e-30)
    s = c.lib().gmg_solve(plan.handle, _ptr(ud), _ptr(g), 1e-10, 50, ctypes.byref(r0),
                          ctypes.byref(it), ctypes.byref(rel))
    torch.cuda.synchronize()
    assert s == c.GMG_ERR_DIVERGED and it.value == 1


@pytest.mark.parametrize("dim,m,inner", [(3, 63, 1), (3, 63, 2), (3, 127, 4), (2, 255, 3)])
def test_mixed_inner_cycles_cross_bitwise(dim, m, inner):
    """Mixed precision, V(1,1): the FP32 cycles of a refinement step run the
    cross-cycle schedule among themselves (no norm between them); the
    iterates equal those of separate cycles bit for bit, and the solve
    reaches 1e-10 by the oracle's FP64 residual."""
    c = capi()
    f = wl.rhs_uniform(dim, m, seed=206)
    fd = dev(f)
    kw = dict(nu1=1, nu2=1, precision="mixed", inner_cycles=inner)
    a = solve(Plan(dim, levels_of(m), **kw), fd, rtol=1e-10)
    b = solve(Plan(dim, levels_of(m), flags=c.GMG_NO_CROSS_CYCLE, **kw), fd, rtol=1e-10)
    assert a[:2] == b[:2] and a[0] == 0
    assert np.array_equal(a[3], b[3])
    rr = oracle.norm2(oracle.residual(a[3], f)) / oracle.norm2(f)
    assert rr <= 1e-10
