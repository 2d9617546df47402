"""Host-only checks of the C ABI: the library loads, exports every entry
point the public header declares, and rejects invalid arguments before any
HIP call (so these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def capi():
    from paper_1208_4247_amd import capi as c

    if not os.path.exists(c.LIB_PATH):
        from paper_1208_4247_amd import build

        build.build()
    c.lib()
    return c


def declared_symbols():
    hdr = open(os.path.join(ROOT, "include", "gmg.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(gmg_[a-z_0-9]+)\s*\(", hdr)))


def test_every_declared_symbol_is_exported(capi):
    syms = declared_symbols()
    assert len(syms) >= 10
    lib = capi.lib()
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(capi.EXPORTED)


def test_constants_match_the_header(capi):
    """The binding's constants are the header's: every GMG_* flag
    #define has a constant of the same value, and the flags are distinct
    bits."""
    hdr = open(os.path.join(ROOT, "include", "gmg.h")).read()
    flags = dict(re.findall(r"#define (GMG_[A-Z0-9_]+) (0x[0-9a-fA-F]+)u", hdr))
    assert len(flags) >= 11
    seen = 0
    for name, val in flags.items():
        v = int(val, 16)
        assert getattr(capi, name) == v, name
        assert v & (v - 1) == 0 and not (seen & v), name  # one bit, not reused
        seen |= v
    m = re.search(r"#define GMG_SCRATCH_BYTES \((\d+)u << (\d+)\)", hdr)
    assert capi.GMG_SCRATCH_BYTES == int(m.group(1)) << int(m.group(2))
    # enumerators (status codes, smoothers, precisions, element types)
    body = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    enums = re.findall(r"\b(GMG_[A-Z0-9_]+)\s*=\s*(-?\d+)", body)
    assert len(enums) >= 12
    for name, val in enums:
        assert getattr(capi, name) == int(val), name


def test_status_strings(capi):
    for s, name in [(0, "GMG_OK"), (1, "GMG_NOT_CONVERGED"), (-1, "GMG_ERR_INVALID_ARG"),
                    (-2, "GMG_ERR_WORKSPACE"), (-5, "GMG_ERR_HIP"), (-6, "GMG_ERR_UNSUPPORTED")]:
        assert capi.status_string(s) == name


def test_config_default(capi):
    c = capi.config_default(3, 8)
    assert (c.dim, c.levels, c.nu1, c.nu2, c.smoother, c.precision, c.inner_cycles) == (3, 8, 2, 2, 0, 0, 4)


@pytest.mark.parametrize("field,value", [("dim", 1), ("dim", 4), ("levels", 0), ("levels", 11),
                                         ("nu1", -1), ("nu2", 9), ("inner_cycles", 0),
                                         ("precision", 7), ("smoother", 3)])
def test_invalid_config_rejected_without_gpu(capi, field, value):
    c = capi.config_default(3, 5)
    setattr(c, field, value)
    s, n = capi.workspace_bytes(c)
    assert s == capi.GMG_ERR_INVALID_ARG


def test_zero_sweeps_rejected(capi):
    c = capi.config_default(2, 5)
    c.nu1 = c.nu2 = 0
    assert capi.workspace_bytes(c)[0] == capi.GMG_ERR_INVALID_ARG


def test_wj_omega_range(capi):
    c = capi.config_default(2, 5)
    c.smoother = capi.GMG_SMOOTH_WJ
    c.omega = 1.5
    assert capi.workspace_bytes(c)[0] == capi.GMG_ERR_INVALID_ARG
    c.omega = 0.8
    assert capi.workspace_bytes(c)[0] == capi.GMG_OK


def test_workspace_size_model(capi):
    """Workspace against the paper's memory model (Sec. 4, remark on the space
    complexity of the V-cycle: u_l, f_l on every level and r_l below the
    coarsest): here the caller's u, f are level 0, the residual is never
    stored, and the workspace holds the coarse u, w (pre-smoothed), f
    (3 * N0 / (2^d - 1)) plus the level-0 pre-smoothed copy w0 (N0); with
    nu >= 2 every level also carries one scratch array for chained passes
    (+N0 + N0 / (2^d - 1)).  FP64 V(1,1) plans run the cross-cycle schedule,
    whose pre-smoothed iterates alternate between two level-0 arrays (+N0);
    with GMG_NO_CROSS_CYCLE they keep one."""
    for d, L in [(2, 10), (3, 8)]:
        for nu, flags, arrays0, arrays_c in [(1, capi.GMG_NO_CROSS_CYCLE, 1, 3), (1, 0, 2, 3),
                                              (2, 0, 2, 4)]:
            c = capi.config_default(d, L)
            c.nu1 = c.nu2 = nu
            c.flags = flags
            s, n = capi.workspace_bytes(c)
            assert s == 0
            N0 = ((1 << L) - 1) ** d
            model = 8 * (arrays0 * N0 + arrays_c * N0 / (2 ** d - 1))
            assert 0.9 * model < n < 1.05 * model + (1 << 20), (d, nu, n, model)


def test_setup_null_checks(capi):
    lib = capi.lib()
    c = capi.config_default(3, 5)
    n = ctypes.c_size_t(0)
    assert lib.gmg_setup(ctypes.byref(c), 1, None, None, None, None, None, None) == capi.GMG_ERR_INVALID_ARG
    assert lib.gmg_setup(ctypes.byref(c), 0, None, None, None, ctypes.byref(n), None, None) == capi.GMG_ERR_INVALID_ARG
    # a workspace that is too small is refused before any device access
    n.value = 16
    plan = ctypes.c_void_p()
    assert lib.gmg_setup(ctypes.byref(c), 1, None, None, ctypes.c_void_p(4096), ctypes.byref(n), None,
                         ctypes.byref(plan)) == capi.GMG_ERR_WORKSPACE
    assert lib.gmg_solve(None, None, None, 1e-10, 10, None, None, None) == capi.GMG_ERR_INVALID_ARG
    assert lib.gmg_vcycle(None, None, None) == capi.GMG_ERR_INVALID_ARG
    assert lib.gmg_destroy(None) == capi.GMG_ERR_INVALID_ARG
    assert lib.gmg_plan_workspace_bytes(None) == 0
    assert lib.gmg_level_side(None, 0, 0) == -1


def test_paper_variant_rejected_where_unsupported(capi):
    """The paper's smoother and transfers run FP64 single problems only."""
    for smoother, flags in ((capi.GMG_SMOOTH_MCGS, 0), (capi.GMG_SMOOTH_RBGS, capi.GMG_FE_TRANSFER),
                            (capi.GMG_SMOOTH_WJ, capi.GMG_COARSE_RELAX)):
        cfg = capi.config_default(3, 5)
        cfg.smoother = smoother
        cfg.flags = flags
        s, n = capi.workspace_bytes(cfg)
        assert s == capi.GMG_OK and n > 0
        cfg.precision = capi.GMG_MIXED_FP32_IR
        assert capi.workspace_bytes(cfg)[0] == capi.GMG_ERR_UNSUPPORTED
        cfg.precision = capi.GMG_FP64
        s, _ = capi.workspace_bytes(cfg, nproblems=2, dims=[3, 2], levels=[5, 6])
        assert s == capi.GMG_ERR_UNSUPPORTED
    cfg = capi.config_default(2, 5)
    cfg.smoother = 3
    assert capi.workspace_bytes(cfg)[0] == capi.GMG_ERR_INVALID_ARG


def _tile_table_hash():
    """FNV-1a over the tile tables of smooth.hip, in the library's order
    (red-black tables, a -1 separator, Jacobi tables), as the tuner keys its
    cache."""
    src = open(os.path.join(ROOT, "paper_1208_4247_amd", "csrc", "smooth.hip")).read()

    def rows(name):
        body = re.search(r"#define %s\(X\)(.*?)\n(?!\s)" % name, src, flags=re.S).group(1)
        return [tuple(int(v) for v in r.split(",")) for r in re.findall(r"X\(([^)]*)\)", body)]

    h = 2166136261

    def mix(v):
        nonlocal h
        for b in range(4):
            h ^= (v >> (8 * b)) & 0xFF
            h = (h * 16777619) & 0xFFFFFFFF

    for name in ("GMG_RB3_S2", "GMG_RB3_S4", "GMG_RB2_S2", "GMG_RB2_S4", "GMG_RB3_S3", "GMG_RB2_S3"):
        for r in rows(name):
            for v in r:
                mix(v)
    mix(-1 & 0xFFFFFFFF)
    for name in ("GMG_WJ3_S1", "GMG_WJ3_S2", "GMG_WJ2_S1", "GMG_WJ2_S2"):
        for r in rows(name):
            for v in r:
                mix(v)
    return h


def _cache_line(m, smax, stages, var, tz, th, dim=3, cap=2):
    key = "gfx950|d%d|m%d|f64|rbgs|nu2|r0|cap%d|fr1|z4|t%08x" % (dim, m, cap, th)
    return ('{"key": "%s", "smax": %d, "stages": %d, "var": %d, "tz": %d, "fuse": 1, '
            '"us": 1.0}\n' % (key, smax, stages, var, tz))


def test_tune_cache_check_rejects_unusable_lines(capi, tmp_path):
    th = _tile_table_hash()
    good = _cache_line(255, 2, 4, 3, 64, th)
    bad = [
        _cache_line(255, 2, 4, 3, 64, th ^ 1),   # another build's tile tables
        _cache_line(255, 2, 4, 9, 64, th),       # tile index beyond the table
        _cache_line(255, 5, 4, 3, 64, th),       # sweeps per pass above the cap
        _cache_line(255, 2, 4, 3, -8, th),       # negative z-chunk
        _cache_line(1023, 1, 2, 1, 4, th),       # 262144 workgroups > partials buffer
        good.replace("|z4|t%08x" % th, "|z4"),   # key without the table hash
        "not a cache line\n",
    ]
    p = tmp_path / "tune.jsonl"
    p.write_text(good + "\n" + "".join(bad))
    assert capi.tune_cache_check(str(p)) == (1, len(bad))
    p.write_text(good + _cache_line(1023, 2, 2, 0, 0, th))
    assert capi.tune_cache_check(str(p)) == (2, 0)
    with pytest.raises(capi.GmgError):
        capi.tune_cache_check(str(tmp_path / "missing.jsonl"))
