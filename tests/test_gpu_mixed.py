"""GPU checks of the mixed-precision form: FP32 kernels against the FP64
oracle (FP32 tolerance), and FP32 V-cycles inside FP64 iterative refinement
reaching the same 1e-10 relative residual as the FP64 solver.

Parity bar for the mixed form: the returned FP64 iterate's residual,
evaluated by the oracle's own FP64 residual routine, is <= 1e-10 relative;
its distance to the FP64 oracle solution is reported (not bounded at 1e-12,
since refinement reaches a different point inside the same residual ball).
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
    return float(np.max(np.abs(a - b))) / max(float(np.max(np.abs(b))), 1e-300)


def levels_of(m):
    return int(np.log2(m + 1))


@pytest.mark.parametrize("dim,m", [(2, 127), (2, 1023), (3, 31), (3, 127)])
@pytest.mark.parametrize("nsweeps", [1, 2])
def test_fp32_smooth_vs_fp64_oracle(dim, m, nsweeps):
    """FP32 red-black sweeps agree with the FP64 oracle to FP32 accuracy."""
    plan = Plan(dim, levels_of(m), precision="mixed")
    f = wl.rhs_uniform(dim, m, seed=91)
    u0 = wl.rhs_uniform(dim, m, seed=92) * 1e-3
    # the oracle runs on the FP32-rounded inputs so only arithmetic differs
    f32, u32 = f.astype(np.float32).astype(np.float64), u0.astype(np.float32).astype(np.float64)
    out = torch.empty((m,) * dim, dtype=torch.float32, device="cuda")
    plan.op_smooth(0, nsweeps, False, dev(u32, torch.float32), dev(f32, torch.float32), None, out)
    assert maxrel(host(out), oracle.rbgs(u32, f32, nsweeps)) <= 5e-6


@pytest.mark.parametrize("dim,m", [(2, 255), (3, 63)])
def test_fp32_restriction_and_residual(dim, m):
    plan = Plan(dim, levels_of(m), precision="mixed")
    mc = (m - 1) // 2
    f = wl.rhs_uniform(dim, m, seed=93).astype(np.float32).astype(np.float64)
    u = (wl.rhs_uniform(dim, m, seed=94) * 1e-4).astype(np.float32).astype(np.float64)
    fc = torch.empty((mc,) * dim, dtype=torch.float32, device="cuda")
    plan.op_restrict_residual(0, dev(u, torch.float32), dev(f, torch.float32), fc)
    want = oracle.restrict_fw(oracle.residual(u, f))
    # FP32 residual of a 1e-4-scaled u: cancellation limits the relative
    # accuracy to ~eps32 * |A u| / |r|
    assert maxrel(host(fc), want) <= 2e-5


@pytest.mark.parametrize("dim,m", [(2, 255), (2, 1023), (3, 63), (3, 127), (3, 255)])
def test_mixed_solve_reaches_fp64_residual(dim, m):
    L = levels_of(m)
    f = wl.rhs_uniform(dim, m, seed=95)
    plan = Plan(dim, L, precision="mixed")
    ud = torch.zeros((m,) * dim, dtype=torch.float64, device="cuda")
    st, it, rel = plan.solve(ud, dev(f), rtol=1e-10, maxit=60)
    assert st == 0
    u = host(ud)
    r_orc = oracle.norm2(oracle.residual(u, f)) / oracle.norm2(f)
    assert r_orc <= 1e-10, r_orc
    assert abs(r_orc - rel) <= 1e-3 * max(r_orc, rel)
    u_ref, it_ref, rel_ref, st_ref, _ = oracle.solve(f, rtol=1e-10)
    diff = float(np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref))
    print("mixed dim=%d m=%d: %d IR steps (FP64: %d cycles), relres %.2e, |u-u_fp64|/|u_fp64| %.2e"
          % (dim, m, it, it_ref, r_orc, diff))
    # both sit inside the 1e-10 residual ball; their distance is bounded by
    # roughly cond-scaled residuals, far below the discretisation error
    assert diff <= 1e-7
    assert it <= it_ref + 3


def test_mixed_solve_odd_and_even_step_counts_land_in_u():
    """The refinement ping-pongs between the caller's u and a workspace copy;
    whatever the parity of the step count the result must be in u."""
    f = wl.rhs_sine(2, 127)
    plan = Plan(2, 7, precision="mixed")
    fd = dev(f)
    for maxit in (1, 2, 3, 4):
        ud = torch.zeros_like(fd)
        st, it, rel = plan.solve(ud, fd, rtol=1e-30, maxit=maxit)
        assert it == maxit and st == 1
        r = oracle.norm2(oracle.residual(host(ud), f)) / oracle.norm2(f)
        assert abs(r - rel) <= 1e-6 * rel


@pytest.mark.parametrize("dim,m", [(2, 1), (2, 3), (2, 7), (2, 255), (2, 511),
                                   (3, 1), (3, 3), (3, 7), (3, 15), (3, 127)])
def test_refinement_step_residual_at_grid_edges(dim, m):
    """The refinement step moves x-pairs: the lone element at the end of
    every row of an odd side, the tile edges and the one-point grid must give
    the iterate and residual norm that the oracle computes from the returned
    iterate (one and two refinement steps from zero)."""
    f = wl.rhs_uniform(dim, m, seed=100 + m)
    plan = Plan(dim, levels_of(m), precision="mixed")
    fd = dev(f)
    for maxit in (1, 2) if m > 7 else (1,):
        ud = torch.zeros_like(fd)
        st, it, rel = plan.solve(ud, fd, rtol=1e-30, maxit=maxit)
        u = host(ud)
        assert it == maxit and np.all(np.isfinite(u))
        r = oracle.norm2(oracle.residual(u, f)) / oracle.norm2(f)
        assert abs(r - rel) <= 1e-6 * rel, (dim, m, maxit, r, rel)


@pytest.mark.parametrize("inner", [1, 2])
def test_mixed_vcycle_is_one_refinement_step(inner):
    """gmg_vcycle on a mixed plan: one refinement step x <- x + e with e
    from `inner` FP32 cycles on A e = f - A x started at zero; the cycle is
    affine, so this equals `inner` FP64 oracle cycles from the same x (to
    FP32 accuracy of the correction)."""
    f = wl.rhs_uniform(3, 31, seed=96)
    x = wl.rhs_uniform(3, 31, seed=97) * 1e-3
    plan = Plan(3, 5, precision="mixed", inner_cycles=inner)
    xd = dev(x)
    plan.vcycle(xd, dev(f))
    got = host(xd)
    want = x
    for _ in range(inner):
        want = oracle.vcycle(want, f)
    corr = want - x
    assert float(np.max(np.abs(got - want))) <= 1e-5 * float(np.max(np.abs(corr)))


def test_mixed_nonzero_initial_guess_and_inner_cycles():
    f = wl.rhs_uniform(3, 63, seed=98)
    u0 = wl.rhs_uniform(3, 63, seed=99) * 1e-2
    for inner in (1, 2):
        plan = Plan(3, 6, precision="mixed", inner_cycles=inner)
        ud = dev(u0)
        st, it, rel = plan.solve(ud, dev(f), rtol=1e-10)
        assert st == 0
        r = oracle.norm2(oracle.residual(host(ud), f)) / oracle.norm2(oracle.residual(u0, f))
        assert r <= 1e-10
