"""GPU check of gmg_solve_scratch, the solve entry point for callers that
cannot allocate: its workspace is the library's own device array, and it
must give exactly what gmg_setup + gmg_solve give on a caller workspace
(same kernels, same arithmetic: iterates bit for bit, same cycle count and
relative residual).  Two calls in a row, the second on a smaller problem,
then a cross-cycle V(1,1) solve; a problem whose workspace exceeds the
array is refused before any launch."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1208_4247_amd import workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1208_4247_amd import capi

    capi.lib()


def scratch_solve(dim, L, f, nu=2, flags=0, maxit=100):
    from paper_1208_4247_amd import capi
    from paper_1208_4247_amd.solver import _ptr, _stream

    cfg = capi.config_default(dim, L)
    cfg.nu1 = cfg.nu2 = nu
    cfg.flags = flags
    u = torch.zeros_like(f)
    it, rel = ctypes.c_int(-1), ctypes.c_double(-1.0)
    s = capi.lib().gmg_solve_scratch(ctypes.byref(cfg), _ptr(u), _ptr(f), 1e-10, maxit, None,
                                     ctypes.byref(it), ctypes.byref(rel), _stream())
    torch.cuda.synchronize()
    return s, it.value, rel.value, u.cpu().numpy()


def plan_solve(dim, L, f, nu=2):
    from paper_1208_4247_amd.solver import Plan

    plan = Plan(dim, L, nu1=nu, nu2=nu)
    u = torch.zeros_like(f)
    s, it, rel = plan.solve(u, f, rtol=1e-10)
    torch.cuda.synchronize()
    return s, it, rel, u.cpu().numpy()


@pytest.mark.parametrize("dim,L,nu", [(3, 6, 2), (2, 7, 2), (3, 7, 1)])
def test_scratch_solve_equals_plan_solve(dim, L, nu):
    m = (1 << L) - 1
    f = torch.from_numpy(wl.rhs_uniform(dim, m, seed=300 + L)).cuda()
    got = scratch_solve(dim, L, f, nu)
    want = plan_solve(dim, L, f, nu)
    assert got[0] == want[0] == 0
    assert got[1] == want[1]
    assert got[2] == want[2]
    assert np.array_equal(got[3], want[3])


def test_scratch_two_calls_second_smaller():
    f1 = torch.from_numpy(wl.rhs_uniform(3, 63, seed=310)).cuda()
    f2 = torch.from_numpy(wl.rhs_uniform(3, 31, seed=311)).cuda()
    a1 = scratch_solve(3, 6, f1)
    a2 = scratch_solve(3, 5, f2)
    b1 = plan_solve(3, 6, f1)
    b2 = plan_solve(3, 5, f2)
    for a, b in ((a1, b1), (a2, b2)):
        assert a[:3] == b[:3]
        assert np.array_equal(a[3], b[3])


def test_scratch_refuses_without_launching():
    from paper_1208_4247_amd import capi

    f = torch.zeros((255, 255, 255), dtype=torch.float64, device="cuda")
    s, it, rel, _ = scratch_solve(3, 8, f)  # workspace of 255^3 exceeds the array
    assert s == capi.GMG_ERR_WORKSPACE and it == -1
    g = torch.from_numpy(wl.rhs_uniform(3, 31, seed=312)).cuda()
    s, it, rel, _ = scratch_solve(3, 5, g, flags=capi.GMG_AUTOTUNE)
    assert s == capi.GMG_ERR_UNSUPPORTED
    s, it, rel, u = scratch_solve(3, 5, g)
    assert s == 0
