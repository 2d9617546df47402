"""GPU checks of plan modes the other files leave out: mixed precision with
weighted Jacobi, with uneven sweep counts and with the flags that change the
schedule (each must reach the FP64 residual by the oracle's own residual);
FP64 solves without temporal blocking, which must give the bits of the
fused-sweep passes (every half-sweep is the same per-point expression).
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
