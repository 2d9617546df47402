"""The seeded input generator (shared by the oracle's and the GPU's tests)."""
import pytest
import numpy as np

from paper_1208_4247_amd import workloads as wl


def test_splitmix64_reference_vector():
    """SplitMix64's output function on the first counter state of seed 0
    (state = golden gamma) gives the published first output 0xE220A8397B1DCDAF."""
    z = wl._mix64(np.array([wl.GOLDEN], dtype=np.uint64))
    assert int(z[0]) == 0xE220A8397B1DCDAF
    assert wl._mix64_int(0x9E3779B97F4A7C15) == 0xE220A8397B1DCDAF


def test_uniform_counter_based_and_chunk_invariant():
    a = wl.uniform_pm1(3, 0, 1000)
    b = wl.uniform_pm1(3, 0, 1000, chunk=7)
    assert np.array_equal(a, b)
    assert np.array_equal(wl.uniform_pm1(3, 0, 10, start=990), a[990:])
    assert a.min() >= -1.0 and a.max() < 1.0
    assert abs(a.mean()) < 0.1
    assert not np.array_equal(a, wl.uniform_pm1(3, 1, 1000))


def test_batch_recipe():
    probs = wl.batch_problems(4)
    assert len(probs) == 256
    assert all(d == 2 and m in (63, 127, 255, 511, 1023) for d, m in probs[:128])
    assert all(d == 3 and m in (31, 63, 127) for d, m in probs[128:])


def test_normals():
    z = wl.normal(5, 1, 20000)
    assert abs(z.mean()) < 0.05 and abs(z.std() - 1) < 0.05


def test_device_sine_modes_equal_host_recipe():
    """The torch-built sum of sine modes (used for the 1023^3 workload) is
    bitwise the host recipe."""
    torch = pytest.importorskip("torch")
    for d, m in ((3, 31), (2, 63), (3, 15)):
        a = wl.rhs_sine_modes(d, m, 5)
        b = wl.rhs_sine_modes_device(d, m, 5, "cpu").numpy()
        assert np.array_equal(a, b)
