"""GPU sine-transform solver (gmg_dst_*) through the C ABI: parity with the
oracle's exact solve, the closed form on sine modes at 1023^3, the paper's
FFT error columns (Tables 12 and 14) from the GPU's own result, and the
ABI's argument checks."""
import json
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1208_4247_amd import workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1208_4247_amd import capi

    capi.lib()


def Dst(d, L):
    from paper_1208_4247_amd.solver import DstSolver

    return DstSolver(d, L)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=torch.float64)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("d,L", [(2, 1), (2, 3), (2, 7), (2, 10), (3, 1), (3, 3), (3, 5), (3, 7)])
def test_dst_matches_oracle(d, L):
    print("dst", d, L, flush=True)
    m = (1 << L) - 1
    f = wl.rhs_uniform(d, m, seed=50 + L)
    s = Dst(d, L)
    u = torch.empty((m,) * d, dtype=torch.float64, device="cuda")
    fd = dev(f)
    s.solve(u, fd)
    want = oracle.dst_solve(f)
    got = host(u)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    assert np.array_equal(host(fd), f)  # f is only read


def test_dst_1023_sine_modes_closed_form():
    """1023^3, f = sum of 8 sine modes (the 1023^3 workload's recipe): the
    exact solution at 4096 sampled points from the closed form."""
    d, L = 3, 10
    m = (1 << L) - 1
    h = 1.0 / (m + 1)
    f = wl.rhs_sine_modes_device(d, m, 5, "cuda")
    s = Dst(d, L)
    u = torch.empty_like(f)
    s.solve(u, f)
    torch.cuda.synchronize()
    amps, ks_all = wl.sine_modes(5)  # amplitudes; frequencies (kx, ky, kz) per mode
    modes = [(float(a), tuple(int(k) for k in ks)) for a, ks in zip(amps, ks_all)]
    rng = np.random.default_rng(51)
    idx = rng.integers(0, m, size=(4096, 3))  # (z, y, x) storage indices
    got = u[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy()
    want = np.zeros(len(idx))
    for a, ks in modes:
        lam = sum(4.0 / h ** 2 * math.sin(k * math.pi * h / 2) ** 2 for k in ks)
        kx, ky, kz = ks
        want += a / lam * (np.sin(kx * np.pi * (idx[:, 2] + 1) * h) *
                           np.sin(ky * np.pi * (idx[:, 1] + 1) * h) *
                           np.sin(kz * np.pi * (idx[:, 0] + 1) * h))
    scale = sum(abs(a) / sum(4.0 / h ** 2 * math.sin(k * math.pi * h / 2) ** 2 for k in ks)
                for a, ks in modes)
    assert np.max(np.abs(got - want)) <= 1e-12 * scale


@pytest.mark.parametrize("d", [2, 3])
def test_dst_reproduces_paper_fft_column(d):
    with open(os.path.join(GOLDEN, "paper_fft_error.json")) as fh:
        g = json.load(fh)
    for L, p in g["%dd" % d].items():
        L = int(L)
        m = (1 << L) - 1
        h = 1.0 / (m + 1)
        phi = wl.sine_product_device(d, m, "cuda")
        s = Dst(d, L)
        u = torch.empty_like(phi)
        s.solve(u, (d * math.pi ** 2) * phi)
        e = math.sqrt(h ** d * float(torch.sum((u - phi) ** 2)))
        q = 10.0 ** (math.floor(math.log10(p)) - 3)
        tol = q * (1 + 1e-9) if d == 3 else 5e-3 * p
        assert abs(e - p) <= tol, (d, L, e, p)


def test_dst_argument_checks():
    from paper_1208_4247_amd import capi
    import ctypes

    L = capi.lib()
    n = ctypes.c_size_t(0)
    assert L.gmg_dst_setup(4, 5, None, ctypes.byref(n), None, None) == capi.GMG_ERR_INVALID_ARG
    assert L.gmg_dst_setup(3, 11, None, ctypes.byref(n), None, None) == capi.GMG_ERR_INVALID_ARG
    assert L.gmg_dst_setup(3, 4, None, ctypes.byref(n), None, None) == capi.GMG_OK and n.value > 0
    small = torch.empty(n.value // 2, dtype=torch.uint8, device="cuda")
    h = ctypes.c_void_p()
    half = ctypes.c_size_t(n.value // 2)
    assert L.gmg_dst_setup(3, 4, ctypes.c_void_p(small.data_ptr()), ctypes.byref(half), None,
                           ctypes.byref(h)) == capi.GMG_ERR_WORKSPACE
    s = Dst(3, 4)
    u = torch.zeros((15,) * 3, dtype=torch.float64, device="cuda")
    assert L.gmg_dst_solve(s._h, ctypes.c_void_p(u.data_ptr()),
                           ctypes.c_void_p(u.data_ptr())) == capi.GMG_ERR_INVALID_ARG
