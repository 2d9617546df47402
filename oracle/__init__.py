"""FP64 CPU oracle for the multigrid Poisson solver (test infrastructure only).

This package is the reference that the HIP library is checked against.  Only
the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it; the product package never does, and it imports
nothing from the product package.

The arithmetic lives in ``gmg_oracle.c`` (plain loops, FP64, no fused
multiply-add); this module only builds and loads that file and marshals numpy
arrays.  Every function follows a passage of Feng, Shu, Xu, Zhang,
arXiv:1208.4247, cited in the C source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gmg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

RBGS = 0
WJ = 1
MCGS = 2  # multicolour Gauss-Seidel: 4 colours in 2D, 8 in 3D

# variant bits of the cycle functions
FE_TRANSFER = 1   # the paper's linear finite-element restriction / interpolation
COARSE_RELAX = 2  # coarsest level relaxed by nu1 smoother sweeps instead of solved exactly


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2 -ffp-contract=off -fopenmp)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-std=c99", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i, d = ctypes.c_int, ctypes.c_double
        L.orc_levels.argtypes = [i]
        L.orc_levels.restype = i
        L.orc_num_threads.restype = i
        L.orc_set_threads.argtypes = [i]
        L.orc_norm2.argtypes = [i, i, dp]
        L.orc_norm2.restype = d
        L.orc_apply_A.argtypes = [i, i, dp, dp]
        L.orc_residual.argtypes = [i, i, dp, dp, dp]
        L.orc_rbgs_color.argtypes = [i, i, dp, dp, i]
        L.orc_rbgs.argtypes = [i, i, dp, dp, i, i]
        L.orc_mcgs_color.argtypes = [i, i, dp, dp, i]
        L.orc_mcgs.argtypes = [i, i, dp, dp, i, i]
        L.orc_wj.argtypes = [i, i, dp, dp, d, i, dp]
        L.orc_restrict_fw.argtypes = [i, i, dp, dp]
        L.orc_prolong_add.argtypes = [i, i, dp, dp]
        L.orc_restrict_fe.argtypes = [i, i, dp, dp]
        L.orc_prolong_add_fe.argtypes = [i, i, dp, dp]
        L.orc_vcycle.argtypes = [i, i, dp, dp, i, i, i, d, i]
        L.orc_vcycle.restype = i
        L.orc_solve.argtypes = [i, i, dp, dp, i, i, i, d, d, i, d,
                                ctypes.POINTER(ctypes.c_int), dp, dp, i]
        L.orc_solve.restype = i
        L.orc_fmg.argtypes = [i, i, dp, dp, i, i, i, d, i]
        L.orc_fmg.restype = i
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _grid(a, d, m):
    a = np.ascontiguousarray(a, dtype=np.float64)
    assert a.size == m ** d, (a.shape, d, m)
    return a


def side(a: np.ndarray) -> int:
    return a.shape[0]


def levels(m0: int) -> int:
    return lib().orc_levels(m0)


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def num_threads() -> int:
    return lib().orc_num_threads()


def norm2(r: np.ndarray) -> float:
    d, m = r.ndim, r.shape[0]
    return lib().orc_norm2(d, m, _p(_grid(r, d, m)))


def apply_A(v: np.ndarray) -> np.ndarray:
    d, m = v.ndim, v.shape[0]
    v = _grid(v, d, m)
    out = np.empty_like(v)
    lib().orc_apply_A(d, m, _p(v), _p(out))
    return out


def residual(u: np.ndarray, f: np.ndarray) -> np.ndarray:
    d, m = u.ndim, u.shape[0]
    u, f = _grid(u, d, m), _grid(f, d, m)
    r = np.empty_like(u)
    lib().orc_residual(d, m, _p(u), _p(f), _p(r))
    return r


def rbgs_color(u: np.ndarray, f: np.ndarray, color: int) -> np.ndarray:
    d, m = u.ndim, u.shape[0]
    u = _grid(u, d, m).copy()
    lib().orc_rbgs_color(d, m, _p(u), _p(_grid(f, d, m)), int(color))
    return u


def rbgs(u: np.ndarray, f: np.ndarray, nsweeps: int, backward: bool = False) -> np.ndarray:
    d, m = u.ndim, u.shape[0]
    u = _grid(u, d, m).copy()
    lib().orc_rbgs(d, m, _p(u), _p(_grid(f, d, m)), int(nsweeps), int(bool(backward)))
    return u


def mcgs_color(u: np.ndarray, f: np.ndarray, color: int) -> np.ndarray:
    d, m = u.ndim, u.shape[0]
    u = _grid(u, d, m).copy()
    lib().orc_mcgs_color(d, m, _p(u), _p(_grid(f, d, m)), int(color))
    return u


def mcgs(u: np.ndarray, f: np.ndarray, nsweeps: int, backward: bool = False) -> np.ndarray:
    d, m = u.ndim, u.shape[0]
    u = _grid(u, d, m).copy()
    lib().orc_mcgs(d, m, _p(u), _p(_grid(f, d, m)), int(nsweeps), int(bool(backward)))
    return u


def wj(u: np.ndarray, f: np.ndarray, omega: float, nsweeps: int) -> np.ndarray:
    d, m = u.ndim, u.shape[0]
    u = _grid(u, d, m).copy()
    tmp = np.empty_like(u)
    lib().orc_wj(d, m, _p(u), _p(_grid(f, d, m)), float(omega), int(nsweeps), _p(tmp))
    return u


def restrict_fw(r: np.ndarray) -> np.ndarray:
    d, mf = r.ndim, r.shape[0]
    mc = (mf - 1) // 2
    out = np.empty((mc,) * d)
    lib().orc_restrict_fw(d, mc, _p(_grid(r, d, mf)), _p(out))
    return out


def prolong_add(e: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Return u + P e (u is the fine grid, side 2 mc + 1)."""
    d, mc = e.ndim, e.shape[0]
    u = _grid(u, d, 2 * mc + 1).copy()
    lib().orc_prolong_add(d, mc, _p(_grid(e, d, mc)), _p(u))
    return u


def restrict_fe(r: np.ndarray) -> np.ndarray:
    d, mf = r.ndim, r.shape[0]
    mc = (mf - 1) // 2
    out = np.empty((mc,) * d)
    lib().orc_restrict_fe(d, mc, _p(_grid(r, d, mf)), _p(out))
    return out


def prolong_add_fe(e: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Return u + P e with the linear finite-element interpolation."""
    d, mc = e.ndim, e.shape[0]
    u = _grid(u, d, 2 * mc + 1).copy()
    lib().orc_prolong_add_fe(d, mc, _p(_grid(e, d, mc)), _p(u))
    return u


def vcycle(u, f, nu1=2, nu2=2, smoother=RBGS, omega=0.8, variant=0) -> np.ndarray:
    d, m = u.ndim, u.shape[0]
    u = _grid(u, d, m).copy()
    rc = lib().orc_vcycle(d, m, _p(u), _p(_grid(f, d, m)), nu1, nu2, smoother, float(omega),
                          int(variant))
    if rc:
        raise ValueError("bad grid for the V-cycle")
    return u


def fmg(f, nu1=1, nu2=1, smoother=RBGS, omega=0.8, variant=0) -> np.ndarray:
    d, m = f.ndim, f.shape[0]
    u = np.zeros((m,) * d)
    rc = lib().orc_fmg(d, m, _p(u), _p(_grid(f, d, m)), nu1, nu2, smoother, float(omega),
                       int(variant))
    if rc:
        raise ValueError("bad grid for FMG")
    return u


def dst_solve(f: np.ndarray) -> np.ndarray:
    """Exact solution of A u = f (Sec. 2.2 scheme, zero Dirichlet data) by the
    discrete sine transform: the sine modes prod_i sin(k_i pi x_i) are the
    eigenvectors of A with eigenvalues sum_i (4/h^2) sin^2(k_i pi h/2), so
    u = S^-1 (S f / lambda) with S the DST-I along every axis (scipy's
    transform as a library step).  The direct method of the paper's FFT
    comparison (Sec. 5.4, Tables 12-15)."""
    import scipy.fft

    d, m = f.ndim, f.shape[0]
    h = 1.0 / (m + 1)
    lam1 = 4.0 / h ** 2 * np.sin(np.arange(1, m + 1) * np.pi * h / 2) ** 2
    lam = lam1[:, None] + lam1[None, :]
    if d == 3:
        lam = lam[:, :, None] + lam1[None, None, :]
    fh = scipy.fft.dstn(np.asarray(f, dtype=np.float64), type=1)
    return scipy.fft.idstn(fh / lam, type=1)


def solve(f, u0=None, nu1=2, nu2=2, smoother=RBGS, omega=0.8, rtol=1e-10, maxit=100,
          res0=0.0, variant=0):
    """Returns (u, iters, relres, status, res_hist)."""
    d, m = f.ndim, f.shape[0]
    f = _grid(f, d, m)
    u = np.zeros_like(f) if u0 is None else _grid(u0, d, m).copy()
    it = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    hist = np.zeros(maxit + 1)
    st = lib().orc_solve(d, m, _p(u), _p(f), nu1, nu2, smoother, float(omega), float(rtol),
                         int(maxit), float(res0), ctypes.byref(it), ctypes.byref(rel), _p(hist),
                         int(variant))
    if st == -1:
        raise ValueError("bad grid for the solver")
    return u, it.value, rel.value, st, hist[: it.value + 1].copy()
