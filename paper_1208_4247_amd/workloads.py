"""Seeded synthetic inputs for the multigrid Poisson solver.

This module holds only input generation: a counter-based random generator and
the right-hand-side recipes of the benchmark workloads.  It contains none of
the solver's arithmetic, and both the HIP path's tests/bench and the CPU
oracle's tests draw their inputs from here, so the two sides see bit-identical
data.

Generator: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), used counter-style: the value for linear
index i of stream s under seed k is mix64(key(k, s) + (i + 1) * GOLDEN), where
mix64 is SplitMix64's output function and key(k, s) = mix64(k * GOLDEN ^ s).
Uniforms take the top 53 bits: u = (z >> 11) * 2^-53 in [0, 1), mapped to
[-1, 1) as 2u - 1 (exact in FP64).

Grids are dense interior arrays of side m = 2^L - 1 (numpy shape (m,)*d, last
axis = x fastest); interior node i (0-based) sits at x = (i + 1) / (m + 1).
"""
from __future__ import annotations

import math

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK64 = (1 << 64) - 1


def _mix64_int(z: int) -> int:
    z &= _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def _mix64(z: np.ndarray) -> np.ndarray:
    z = z ^ (z >> np.uint64(30))
    z = z * _M1
    z = z ^ (z >> np.uint64(27))
    z = z * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int, stream: int) -> int:
    return _mix64_int((seed * 0x9E3779B97F4A7C15) ^ stream)


def uniform_pm1(seed: int, stream: int, n: int, start: int = 0,
                chunk: int = 1 << 24) -> np.ndarray:
    """n values of U[-1, 1) for linear indices start .. start+n-1."""
    key = np.uint64(stream_key(seed, stream))
    out = np.empty(n, dtype=np.float64)
    with np.errstate(over="ignore"):
        for a in range(0, n, chunk):
            b = min(n, a + chunk)
            idx = np.arange(start + a + 1, start + b + 1, dtype=np.uint64)
            z = _mix64(key + idx * GOLDEN)
            u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
            out[a:b] = 2.0 * u - 1.0
    return out


def uniform_int(seed: int, stream: int, n: int, lo: int, hi: int) -> np.ndarray:
    """n integers uniform in [lo, hi] (inclusive) via the top 53-bit uniform."""
    u = (uniform_pm1(seed, stream, n) + 1.0) * 0.5
    return lo + np.minimum((u * (hi - lo + 1)).astype(np.int64), hi - lo)


def normal(seed: int, stream: int, n: int) -> np.ndarray:
    """n standard normals by Box-Muller from 2n uniforms of the stream."""
    u = (uniform_pm1(seed, stream, 2 * n) + 1.0) * 0.5
    u1 = 1.0 - u[0::2]  # (0, 1]
    u2 = u[1::2]
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


def nodes(m: int) -> np.ndarray:
    """Interior node coordinates (i + 1) h, h = 1/(m + 1)."""
    return np.arange(1, m + 1, dtype=np.float64) / float(m + 1)


def sine_product(d: int, m: int, freqs=None) -> np.ndarray:
    """prod_i sin(k_i pi x_i) on the interior nodes (k defaults to 1)."""
    freqs = (1,) * d if freqs is None else tuple(freqs)
    x = nodes(m)
    fac = [np.sin(k * math.pi * x) for k in freqs]  # fac[axis] for axis x, y, z
    if d == 2:
        return fac[1][:, None] * fac[0][None, :]
    return fac[2][:, None, None] * fac[1][None, :, None] * fac[0][None, None, :]


def rhs_sine(d: int, m: int) -> np.ndarray:
    """f = d pi^2 prod sin(pi x_i): the model problem whose exact solution is
    u = prod sin(pi x_i)."""
    return (d * math.pi ** 2) * sine_product(d, m)


def rhs_uniform(d: int, m: int, seed: int, stream: int = 0) -> np.ndarray:
    return uniform_pm1(seed, stream, m ** d).reshape((m,) * d)


def rhs_sine_plus_noise(d: int, m: int, seed: int, eps: float = 1e-3) -> np.ndarray:
    """d pi^2 prod sin(pi x_i) + eps * U[-1, 1) noise (3D 255^3 workload)."""
    return rhs_sine(d, m) + eps * rhs_uniform(d, m, seed, stream=0)


def sine_modes(seed: int, d: int = 3, nmodes: int = 8, kmax: int = 32):
    """Amplitudes a_m ~ N(0, 1) and integer frequencies k_{m,i} ~ U{1..kmax}."""
    amps = normal(seed, 1, nmodes)
    ks = uniform_int(seed, 2, nmodes * d, 1, kmax).reshape(nmodes, d)
    return amps, ks


def rhs_sine_modes(d: int, m: int, seed: int, nmodes: int = 8, kmax: int = 32) -> np.ndarray:
    """f = sum_m a_m prod_i sin(k_{m,i} pi x_i) (1023^3 workload recipe)."""
    amps, ks = sine_modes(seed, d, nmodes, kmax)
    f = np.zeros((m,) * d)
    for a, k in zip(amps, ks):
        f += a * sine_product(d, m, k)
    return f


def rhs_sine_modes_device(d: int, m: int, seed: int, device, nmodes: int = 8,
                          kmax: int = 32):
    """The same array as rhs_sine_modes, built on a torch device: the per-axis
    sine vectors come from the host in FP64 and each mode is the same chain of
    IEEE products and one addition, so the result is bitwise the host one.
    For grids too large to build on the host comfortably (1023^3)."""
    import torch

    amps, ks = sine_modes(seed, d, nmodes, kmax)
    x = nodes(m)
    f = torch.zeros((m,) * d, dtype=torch.float64, device=device)
    for a, k in zip(amps, ks):
        fac = [torch.from_numpy(np.sin(int(kk) * math.pi * x)).to(device) for kk in k]
        if d == 2:
            prod = fac[1][:, None] * fac[0][None, :]
        else:
            prod = (fac[2][:, None, None] * fac[1][None, :, None]) * fac[0][None, None, :]
        prod.mul_(float(a))
        f.add_(prod)
        del prod
    return f


def sine_product_device(d: int, m: int, device):
    """prod_i sin(pi x_i) on a torch device, the same chain of products as
    sine_product (bitwise equal)."""
    import torch

    s = torch.from_numpy(np.sin(math.pi * nodes(m))).to(device)
    if d == 2:
        return s[:, None] * s[None, :]
    return (s[:, None, None] * s[None, :, None]) * s[None, None, :]


def batch_problems(seed: int = 4, n2d: int = 128, n3d: int = 128,
                   k2d=(6, 10), k3d=(5, 7)):
    """The uneven batch: (dim, side) per problem.  Problem p < n2d is 2D with
    side 2^k - 1, k ~ U{k2d}; the rest are 3D with k ~ U{k3d} (stream 0)."""
    ks2 = uniform_int(seed, 0, n2d + n3d, k2d[0], k2d[1])[:n2d]
    ks3 = uniform_int(seed, 0, n2d + n3d, k3d[0], k3d[1])[n2d:]
    probs = [(2, (1 << int(k)) - 1) for k in ks2] + [(3, (1 << int(k)) - 1) for k in ks3]
    return probs


def batch_rhs(seed: int, p: int, d: int, m: int) -> np.ndarray:
    """RHS of batch problem p: U[-1, 1) from stream 1 + p."""
    return rhs_uniform(d, m, seed, stream=1 + p)


# Named workloads of the benchmark.  Each entry: dim, side, generator.
WORKLOADS = {
    "poisson2d_127_sine": dict(dim=2, m=127, rhs=lambda: rhs_sine(2, 127)),
    "poisson3d_255_sine_noise": dict(dim=3, m=255, rhs=lambda: rhs_sine_plus_noise(3, 255, 2)),
    "poisson3d_511_uniform": dict(dim=3, m=511, rhs=lambda: rhs_uniform(3, 511, 3)),
    "poisson3d_1023_sine_modes": dict(dim=3, m=1023, rhs=lambda: rhs_sine_modes(3, 1023, 5)),
}
