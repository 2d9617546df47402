"""Thin torch-facing wrapper of the C ABI: torch supplies device memory (the
workspace and the grids) and the stream; the library does all the work.

    plan = Plan(dim=3, levels=8)                 # 255^3, RB-GS V(2,2), FP64
    status, iters, relres = plan.solve(u, f, rtol=1e-10)

Grids are torch tensors on the current CUDA (HIP) device, contiguous, shape
(m,)*dim with the last axis x (fastest), float64 (float32 for the FP32
primitives).
"""
from __future__ import annotations

import ctypes

import torch

from . import capi


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Plan:
    def __init__(self, dim: int, levels: int, smoother: str = "rbgs", nu1: int = 2, nu2: int = 2,
                 omega: float = 0.0, precision: str = "fp64", inner_cycles: int | None = None,
                 flags: int = 0):
        L = capi.lib()
        cfg = capi.config_default(dim, levels)
        cfg.smoother = {"rbgs": capi.GMG_SMOOTH_RBGS, "wj": capi.GMG_SMOOTH_WJ,
                        "mcgs": capi.GMG_SMOOTH_MCGS}[smoother]
        cfg.nu1, cfg.nu2 = int(nu1), int(nu2)
        cfg.omega = float(omega)
        cfg.precision = {"fp64": capi.GMG_FP64, "mixed": capi.GMG_MIXED_FP32_IR}[precision]
        if inner_cycles is not None:
            cfg.inner_cycles = int(inner_cycles)
        cfg.flags = int(flags)
        self.cfg = cfg
        self.dim, self.levels = dim, levels
        self.m0 = (1 << levels) - 1
        s, nbytes = capi.workspace_bytes(cfg)
        capi.check(s, "gmg_setup(size query)")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        n = ctypes.c_size_t(nbytes)
        plan = ctypes.c_void_p()
        s = L.gmg_setup(ctypes.byref(cfg), 1, None, None, _ptr(self.workspace), ctypes.byref(n),
                        _stream(), ctypes.byref(plan))
        capi.check(s, "gmg_setup")
        self._plan = plan

    # ------------------------------------------------------------------
    def close(self):
        if getattr(self, "_plan", None):
            capi.lib().gmg_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._plan

    def side(self, level: int) -> int:
        return capi.lib().gmg_level_side(self._plan, 0, int(level))

    # ------------------------------------------------------------------
    def vcycle(self, u: torch.Tensor, f: torch.Tensor) -> None:
        capi.check(capi.lib().gmg_vcycle(self._plan, _ptr(u), _ptr(f)), "gmg_vcycle")

    def fmg(self, u: torch.Tensor, f: torch.Tensor) -> None:
        """Full multigrid (Algorithm 2) into u (enqueue only)."""
        capi.check(capi.lib().gmg_fmg(self._plan, _ptr(u), _ptr(f)), "gmg_fmg")

    def solve(self, u: torch.Tensor, f: torch.Tensor, rtol: float = 1e-10, maxit: int = 100,
              res0: float | None = None):
        it = ctypes.c_int(0)
        rel = ctypes.c_double(0.0)
        r0 = ctypes.byref(ctypes.c_double(res0)) if res0 is not None else None
        s = capi.lib().gmg_solve(self._plan, _ptr(u), _ptr(f), float(rtol), int(maxit), r0,
                                 ctypes.byref(it), ctypes.byref(rel))
        capi.check(s, "gmg_solve")
        return s, it.value, rel.value

    def set_tile(self, level: int, stages: int, variant: int, tz: int = 0) -> None:
        capi.check(capi.lib().gmg_plan_set_tile(self._plan, int(level), int(stages), int(variant),
                                                int(tz)), "gmg_plan_set_tile")

    def set_tile_order(self, level: int, stages: int, strip: int) -> None:
        capi.check(capi.lib().gmg_plan_set_tile_order(self._plan, int(level), int(stages),
                                                      int(strip)), "gmg_plan_set_tile_order")

    def get_tile(self, level, role):
        """(stages, variant, tz) of the first pre- (role 0) or post-smoothing
        (role 1) pass on `level` after autotuning."""
        st, v, tz = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        capi.check(capi.lib().gmg_plan_get_tile(self._plan, int(level), int(role), ctypes.byref(st),
                                                ctypes.byref(v), ctypes.byref(tz)),
                   "gmg_plan_get_tile")
        return st.value, v.value, tz.value

    def tile_variants(self, stages: int) -> int:
        return capi.lib().gmg_tile_variant_count(self.dim, self.cfg.smoother, int(stages))

    # ---------------------------------------------------------- primitives
    def op_smooth(self, level, nsweeps, backward, u_in, f, e_coarse, u_out, want_norm=False):
        dt = capi.GMG_F64 if f.dtype == torch.float64 else capi.GMG_F32
        nrm = ctypes.c_double(0.0)
        s = capi.lib().gmg_op_smooth(self._plan, int(level), dt, int(nsweeps), int(bool(backward)),
                                     _ptr(u_in), _ptr(f), _ptr(e_coarse), _ptr(u_out),
                                     ctypes.byref(nrm) if want_norm else None)
        capi.check(s, "gmg_op_smooth")
        return nrm.value if want_norm else None

    def op_restrict_residual(self, level, u, f, fc):
        dt = capi.GMG_F64 if f.dtype == torch.float64 else capi.GMG_F32
        capi.check(capi.lib().gmg_op_restrict_residual(self._plan, int(level), dt, _ptr(u), _ptr(f),
                                                       _ptr(fc)), "gmg_op_restrict_residual")

    def op_prolong_add(self, level, u_in, e_coarse, u_out):
        dt = capi.GMG_F64 if e_coarse.dtype == torch.float64 else capi.GMG_F32
        capi.check(capi.lib().gmg_op_prolong_add(self._plan, int(level), dt, _ptr(u_in),
                                                 _ptr(e_coarse), _ptr(u_out)),
                   "gmg_op_prolong_add")

    def op_residual(self, level, u, f, r=None, want_norm=True):
        dt = capi.GMG_F64 if f.dtype == torch.float64 else capi.GMG_F32
        nrm = ctypes.c_double(0.0)
        capi.check(capi.lib().gmg_op_residual(self._plan, int(level), dt, _ptr(u), _ptr(f), _ptr(r),
                                              ctypes.byref(nrm) if want_norm else None),
                   "gmg_op_residual")
        return nrm.value if want_norm else None

    # ------------------------------------------------------------ profile
    def profile(self):
        L = capi.lib()
        out = {}
        for i in range(L.gmg_profile_count(self._plan)):
            st = capi.GmgKernelStat()
            capi.check(L.gmg_profile_get(self._plan, i, ctypes.byref(st)), "gmg_profile_get")
            out[st.name.decode()] = dict(launches=st.launches, ms=st.total_ms, bytes=st.alg_bytes)
        return out

    PROFILE_CLASSES = ["smooth_pre_l0", "smooth_post_l0", "resid_restrict_l0", "smooth_pre_coarse",
                       "smooth_post_coarse", "resid_restrict_coarse", "bottom", "finalize",
                       "ir_step", "misc", "smooth_cross_l0"]

    def profile_only(self, names):
        mask = 0
        for n in names:
            mask |= 1 << self.PROFILE_CLASSES.index(n)
        capi.check(capi.lib().gmg_profile_set_mask(self._plan, mask), "gmg_profile_set_mask")

    def profile_reset(self):
        capi.check(capi.lib().gmg_profile_reset(self._plan), "gmg_profile_reset")


class BatchPlan:
    """Many independent problems of uneven sizes solved together: every
    kernel launch covers all problems with a level of that size."""

    def __init__(self, problems, smoother: str = "rbgs", nu1: int = 2, nu2: int = 2,
                 omega: float = 0.0, flags: int = 0):
        L = capi.lib()
        dims = [int(d) for d, _ in problems]
        levels = [int(lv) for _, lv in problems]
        cfg = capi.config_default(dims[0], levels[0])
        cfg.smoother = {"rbgs": capi.GMG_SMOOTH_RBGS, "wj": capi.GMG_SMOOTH_WJ,
                        "mcgs": capi.GMG_SMOOTH_MCGS}[smoother]
        cfg.nu1, cfg.nu2 = int(nu1), int(nu2)
        cfg.omega = float(omega)
        cfg.flags = int(flags)
        self.cfg = cfg
        self.n = len(problems)
        self.problems = list(zip(dims, levels))
        s, nbytes = capi.workspace_bytes(cfg, self.n, dims, levels)
        capi.check(s, "gmg_setup(batch size query)")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        da = (ctypes.c_int * self.n)(*dims)
        la = (ctypes.c_int * self.n)(*levels)
        n = ctypes.c_size_t(nbytes)
        plan = ctypes.c_void_p()
        s = L.gmg_setup(ctypes.byref(cfg), self.n, da, la, _ptr(self.workspace), ctypes.byref(n),
                        _stream(), ctypes.byref(plan))
        capi.check(s, "gmg_setup(batch)")
        self._plan = plan

    def close(self):
        if getattr(self, "_plan", None):
            capi.lib().gmg_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, us, fs, rtol: float = 1e-10, maxit: int = 100):
        n = self.n
        ua = (ctypes.c_void_p * n)(*[t.data_ptr() for t in us])
        fa = (ctypes.c_void_p * n)(*[t.data_ptr() for t in fs])
        for t in list(us) + list(fs):
            if not t.is_cuda or not t.is_contiguous() or t.dtype != torch.float64:
                raise ValueError("expected contiguous float64 device tensors")
        it = (ctypes.c_int * n)()
        rel = (ctypes.c_double * n)()
        st = (ctypes.c_int * n)()
        s = capi.lib().gmg_batch_solve(self._plan, ua, fa, float(rtol), int(maxit), it, rel, st)
        capi.check(s, "gmg_batch_solve")
        return s, list(it), list(rel), list(st)

    def profile(self):
        return Plan.profile(self)

    def profile_reset(self):
        capi.check(capi.lib().gmg_profile_reset(self._plan), "gmg_profile_reset")


class DstSolver:
    """Exact discrete solve u = A^-1 f by the sine transform (gmg_dst_*):
    the fast direct method of the paper's FMG-vs-FFT comparison."""

    def __init__(self, dim: int, levels: int):
        L = capi.lib()
        self.dim, self.levels = dim, levels
        self.m0 = (1 << levels) - 1
        n = ctypes.c_size_t(0)
        capi.check(L.gmg_dst_setup(dim, levels, None, ctypes.byref(n), _stream(), None),
                   "gmg_dst_setup(size query)")
        self.workspace = torch.empty(n.value, dtype=torch.uint8, device="cuda")
        h = ctypes.c_void_p()
        capi.check(L.gmg_dst_setup(dim, levels, _ptr(self.workspace), ctypes.byref(n), _stream(),
                                   ctypes.byref(h)), "gmg_dst_setup")
        self._h = h

    def solve(self, u: torch.Tensor, f: torch.Tensor) -> None:
        capi.check(capi.lib().gmg_dst_solve(self._h, _ptr(u), _ptr(f)), "gmg_dst_solve")

    def close(self):
        if getattr(self, "_h", None):
            capi.lib().gmg_dst_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
