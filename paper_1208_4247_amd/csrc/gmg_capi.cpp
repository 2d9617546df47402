// gmg_capi.cpp -- host orchestration behind the C ABI declared in gmg.h.
//
// A plan holds the level table of Algorithm 3's set-up and the carving of the
// caller's workspace.  One V-cycle (Algorithm 1, with every level on the GPU)
// is enqueued as
//
//   level 0   PRE   w0 = S^nu1(u)            [+ partial sums of |f - A u|^2]
//             FIN   norm, stop test (device state; no host round trip)
//             RES   f1 = FW(f - A w0)
//   l=1..B-1  PRE   w_l = S^nu1(0)    RES  f_{l+1} = FW(f_l - A w_l)
//   bottom    one workgroup runs levels B..L-1 (down to the one-node level)
//   l=B-1..1  POST  u_l = S^nu2(w_l + P u_{l+1})
//   level 0   POST  u   = S^nu2(w0 + P u_1)
//
// where S is a fused multi-sweep pass (temporal blocking).  Every launch reads
// a device "active" flag that the FIN step clears once the relative residual
// reaches rtol (or maxit is hit), so the host can enqueue several cycles
// ahead and only reads the 48-byte state once per batch of cycles.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/gmg.h"
#include "gmg_internal.h"

using namespace gmg;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxLevels = 13;      // side <= 8191: int32 indices in every kernel
constexpr int kMaxPartials = 65536;  // per-workgroup norm partial sums

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

size_t npts(int dim, int m) { return dim == 3 ? (size_t)m * m * m : (size_t)m * m; }

// largest side the one-workgroup bottom kernel holds in LDS
int bottom_side_max(int dim, int smoother, size_t elem) {
  for (int k = 7; k >= 1; --k) {
    const int L = k;
    if (bottom_lds_bytes(dim, L, smoother, elem) <= 150 * 1024) {
      const int m = (1 << L) - 1;
      return dim == 3 ? std::min(m, 15) : std::min(m, 63);
    }
  }
  return 1;
}

struct Prof {
  std::string name;
  long long launches = 0;
  double ms = 0.0;
  double bytes = 0.0;
};

struct PendingEv {
  int cls;
  hipEvent_t a, b;
  double bytes;
};

template <typename T>
struct LevelSet {
  // per level: f (RHS), w (after pre-smoothing), u (after post-smoothing),
  // t (scratch for chained passes).  Level 0's f/u are supplied per call.
  std::vector<T *> f, w, u, t;
};

}  // namespace

struct gmg_plan {
  gmg_config cfg;
  int nproblems = 1;
  hipStream_t stream = nullptr;
  char *ws = nullptr;
  size_t ws_bytes = 0;

  int dim = 3, L = 1, B = 1;  // B: first level handled by the bottom kernel
  std::vector<int> m;         // sides
  int smax = 2;               // sweeps fused per pass
  bool need_tmp = false;

  SolveState *state = nullptr;
  double *partials = nullptr;
  double *scalar = nullptr;  // device scratch for primitive norms

  LevelSet<double> d;  // FP64 levels
  LevelSet<float> s;   // FP32 levels (mixed precision)
  double *x2 = nullptr;  // FP64 ping-pong partner of the caller's u (mixed)

  // per level tile variant for each fused-stage count (index: stages)
  std::vector<std::array<int, 5>> var;
  std::vector<std::array<int, 5>> tz;

  // profiling
  bool profile = false;
  std::vector<Prof> prof;
  std::vector<PendingEv> pending;
  std::vector<hipEvent_t> evpool;

  SolveState *hstate = nullptr;  // pinned host copy
  double *hscalar = nullptr;
};

namespace {

// ------------------------------------------------------------------ errors
#define HIPCHK(x)                         \
  do {                                    \
    hipError_t e_ = (x);                  \
    if (e_ != hipSuccess) return GMG_ERR_HIP; \
  } while (0)

// ------------------------------------------------------------------ profiling
enum ProfClass {
  PC_PRE0 = 0,
  PC_POST0,
  PC_RES0,
  PC_PRE_C,
  PC_POST_C,
  PC_RES_C,
  PC_BOTTOM,
  PC_FIN,
  PC_IR,
  PC_MISC,
  PC_COUNT
};
const char *kProfNames[PC_COUNT] = {"smooth_pre_l0", "smooth_post_l0", "resid_restrict_l0",
                                    "smooth_pre_coarse", "smooth_post_coarse",
                                    "resid_restrict_coarse", "bottom", "finalize", "ir_step",
                                    "misc"};

hipEvent_t get_event(gmg_plan *p) {
  if (!p->evpool.empty()) {
    hipEvent_t e = p->evpool.back();
    p->evpool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

struct ProfScope {
  gmg_plan *p;
  int cls;
  double bytes;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(gmg_plan *p_, int cls_, double bytes_) : p(p_), cls(cls_), bytes(bytes_) {
    if (!p->profile) return;
    a = get_event(p);
    b = get_event(p);
    if (a) (void)hipEventRecord(a, p->stream);
  }
  ~ProfScope() {
    if (!p->profile || !a || !b) return;
    (void)hipEventRecord(b, p->stream);
    p->pending.push_back({cls, a, b, bytes});
  }
};

gmg_status harvest(gmg_plan *p) {
  if (p->pending.empty()) return GMG_OK;
  HIPCHK(hipStreamSynchronize(p->stream));
  for (auto &e : p->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
      p->prof[e.cls].launches += 1;
      p->prof[e.cls].ms += ms;
      p->prof[e.cls].bytes += e.bytes;
    }
    p->evpool.push_back(e.a);
    p->evpool.push_back(e.b);
  }
  p->pending.clear();
  return GMG_OK;
}

// ------------------------------------------------------------------ passes
int stages_of(const gmg_plan *p, int sweeps) {
  return p->cfg.smoother == GMG_SMOOTH_RBGS ? 2 * sweeps : sweeps;
}

template <typename T>
hipError_t one_pass(gmg_plan *p, int level, int sweeps, int flags, const T *src, const T *ec,
                    const T *f, T *dst, double *partials, const int *active, int cls) {
  const int dim = p->dim, m = p->m[level];
  const int st = stages_of(p, sweeps);
  const bool wj = p->cfg.smoother == GMG_SMOOTH_WJ;
  const int v = p->var[level][st];
  const PassTile t = pass_variant(dim, st, wj ? 1 : 0, v);
  const PassGeom g = pass_geometry(dim, m, st, t, p->tz[level][st]);
  PassArgs<T> a;
  a.u_in = src;
  a.f = f;
  a.u_out = dst;
  a.e_c = ec;
  a.partials = partials;
  a.active = active;
  a.m = m;
  a.mc = level + 1 < p->L ? p->m[level + 1] : 0;
  a.ntx = g.ntx;
  a.nty = g.nty;
  a.tz = g.tz;
  a.nblocks = g.nblocks;
  const double h = 1.0 / double(m + 1);
  a.h2 = h * h;
  a.inv_h2 = 1.0 / (h * h);
  a.omega = p->cfg.omega;
  double bytes = (double)npts(dim, m) * sizeof(T) * ((flags & F_ZERO_IN) ? 2 : 3);
  if (flags & F_PROLONG) bytes += (double)npts(dim, a.mc) * sizeof(T);
  ProfScope ps(p, cls, bytes);
  return wj ? launch_wj_pass<T>(dim, st, flags, v, a, p->stream)
            : launch_rb_pass<T>(dim, st, flags, v, a, p->stream);
}

int pass_blocks(const gmg_plan *p, int level, int sweeps) {
  const int st = stages_of(p, sweeps);
  const bool wj = p->cfg.smoother == GMG_SMOOTH_WJ;
  const PassTile t = pass_variant(p->dim, st, wj ? 1 : 0, p->var[level][st]);
  return pass_geometry(p->dim, p->m[level], st, t, p->tz[level][st]).nblocks;
}

// nsweeps of the plan's smoother from (src [+ P ec]) to dst through fused
// passes of at most smax sweeps; intermediate passes alternate between tmp
// and dst so the last one lands in dst and no pass reads what it writes.
// partials != NULL: the first pass emits |f - A src|^2 partial sums.
template <typename T>
hipError_t smooth_chain(gmg_plan *p, int level, int nsweeps, bool backward, const T *src,
                        const T *ec, const T *f, T *dst, T *tmp, double *partials,
                        const int *active, int cls, int *nparts) {
  const int dim = p->dim;
  const int m = p->m[level];
  const int mc = level + 1 < p->L ? p->m[level + 1] : 0;
  if (nparts) *nparts = 0;
  if (nsweeps == 0) {
    hipError_t e = hipSuccess;
    if (partials) {
      ResidArgs<T> r;
      r.u = src;
      r.f = f;
      r.r = nullptr;
      r.partials = partials;
      r.active = active;
      r.m = m;
      r.nblocks = residual_blocks(dim, m);
      const double h = 1.0 / double(m + 1);
      r.inv_h2 = 1.0 / (h * h);
      if (nparts) *nparts = r.nblocks;
      ProfScope ps(p, PC_MISC, (double)npts(dim, m) * sizeof(T) * 2);
      e = launch_residual<T>(dim, r, p->stream);
      if (e != hipSuccess) return e;
    }
    if (ec) {
      ProfScope ps(p, PC_MISC, (double)npts(dim, m) * sizeof(T) * 2);
      return launch_prolong_add<T>(dim, m, mc, src, ec, dst, active, p->stream);
    }
    if (src == dst) return hipSuccess;
    if (!src) return launch_fill_zero(dst, npts(dim, m) * sizeof(T), p->stream);
    return launch_copy(src, dst, npts(dim, m) * sizeof(T), active, p->stream);
  }
  const int K = (nsweeps + p->smax - 1) / p->smax;
  int left = nsweeps;
  const T *in = src;
  for (int k = 1; k <= K; ++k) {
    const int sw = std::min(p->smax, left - (K - k));  // keep later passes non-empty
    const int swk = std::min(sw, p->smax);
    T *out = ((K - k) % 2 == 1) ? tmp : dst;
    int flags = backward ? F_BLACK_FIRST : 0;
    if (k == 1) {
      if (!in) flags |= F_ZERO_IN;
      if (ec) flags |= F_PROLONG;
      if (partials) {
        flags |= F_NORM_IN;
        if (nparts) *nparts = pass_blocks(p, level, swk);
      }
    }
    hipError_t e = one_pass<T>(p, level, swk, flags, in, k == 1 ? ec : nullptr, f, out,
                               k == 1 ? partials : nullptr, active, cls);
    if (e != hipSuccess) return e;
    in = out;
    left -= swk;
  }
  return hipSuccess;
}

template <typename T>
hipError_t restrict_level(gmg_plan *p, int level, const T *u, const T *f, T *fc,
                          const int *active, int cls) {
  const int m = p->m[level];
  if (!u) {  // zero iterate: the residual is f itself
    u = nullptr;
  }
  RestrictArgs<T> a;
  a.u = u;
  a.f = f;
  a.fc = fc;
  a.active = active;
  a.m = m;
  a.mc = p->m[level + 1];
  const double h = 1.0 / double(m + 1);
  a.inv_h2 = 1.0 / (h * h);
  ProfScope ps(p, cls, (double)npts(p->dim, m) * sizeof(T) * 2 + (double)npts(p->dim, a.mc) * sizeof(T));
  return launch_restrict<T>(p->dim, a, p->stream);
}

template <typename T>
LevelSet<T> &levels_of(gmg_plan *p);
template <>
LevelSet<double> &levels_of<double>(gmg_plan *p) {
  return p->d;
}
template <>
LevelSet<float> &levels_of<float>(gmg_plan *p) {
  return p->s;
}

// One V-cycle on the plan's hierarchy in precision T.  Level 0: start value
// u0_in (NULL = zero), result u0_out (must not alias u0_in), RHS f0.
// norm_partials != NULL: the level-0 pre-pass emits the residual norm of
// u0_in, and a finalize step updates the solve state right after it.
template <typename T>
hipError_t enqueue_vcycle(gmg_plan *p, const T *u0_in, const T *f0, T *u0_out,
                          double *norm_partials, const int *active) {
  LevelSet<T> &S = levels_of<T>(p);
  const int L = p->L, B = p->B;
  const bool bwd = !(p->cfg.flags & GMG_POST_FORWARD);
  const int nu1 = p->cfg.nu1, nu2 = p->cfg.nu2;
  hipError_t e;
  int nparts = 0;
  BottomArgs<T> ba;
  ba.active = active;
  ba.dim = p->dim;
  ba.nu1 = nu1;
  ba.nu2 = nu2;
  ba.smoother = p->cfg.smoother == GMG_SMOOTH_WJ ? 1 : 0;
  ba.post_forward = bwd ? 0 : 1;
  ba.omega = p->cfg.omega;
  if (L == 1) {
    // the one-node grid: Algorithm 1 reduces to the exact coarsest solve
    if (norm_partials) {
      e = smooth_chain<T>(p, 0, nu1, false, u0_in, nullptr, f0, S.w[0], S.t[0], norm_partials,
                          active, PC_PRE0, &nparts);
      if (e != hipSuccess) return e;
      {
        ProfScope ps(p, PC_FIN, 0.0);
        e = launch_finalize(norm_partials, nparts, p->state, p->stream);
      }
      if (e != hipSuccess) return e;
    }
    ba.f = f0;
    ba.u = u0_out;
    ba.L = 1;
    ProfScope ps(p, PC_BOTTOM, 2.0 * sizeof(T));
    return launch_bottom<T>(1, ba, nullptr, nullptr, p->stream);
  }
  // ---- descent
  e = smooth_chain<T>(p, 0, nu1, false, u0_in, nullptr, f0, S.w[0], S.t[0], norm_partials, active,
                      PC_PRE0, &nparts);
  if (e != hipSuccess) return e;
  if (norm_partials) {
    ProfScope ps(p, PC_FIN, 0.0);
    e = launch_finalize(norm_partials, nparts, p->state, p->stream);
    if (e != hipSuccess) return e;
  }
  // (nu1 == 0: the chain copied the start value into w0, so the post-pass
  // below never reads the array it writes)
  const T *w0 = S.w[0];
  e = restrict_level<T>(p, 0, w0, f0, S.f[1], active, PC_RES0);
  if (e != hipSuccess) return e;
  for (int l = 1; l < B; ++l) {
    e = smooth_chain<T>(p, l, nu1, false, nullptr, nullptr, S.f[l], S.w[l], S.t[l], nullptr,
                        active, PC_PRE_C, nullptr);
    if (e != hipSuccess) return e;
    e = restrict_level<T>(p, l, S.w[l], S.f[l], S.f[l + 1], active, PC_RES_C);
    if (e != hipSuccess) return e;
  }
  // ---- bottom (levels B..L-1 in one workgroup)
  {
    ba.f = S.f[B];
    ba.u = S.u[B];
    ba.L = L - B;
    ProfScope ps(p, PC_BOTTOM, (double)npts(p->dim, p->m[B]) * sizeof(T) * 2);
    e = launch_bottom<T>(1, ba, nullptr, nullptr, p->stream);
    if (e != hipSuccess) return e;
  }
  // ---- ascent
  for (int l = B - 1; l >= 1; --l) {
    e = smooth_chain<T>(p, l, nu2, bwd, S.w[l], S.u[l + 1], S.f[l], S.u[l], S.t[l], nullptr,
                        active, PC_POST_C, nullptr);
    if (e != hipSuccess) return e;
  }
  return smooth_chain<T>(p, 0, nu2, bwd, w0, S.u[1], f0, u0_out, S.t[0], nullptr, active,
                         PC_POST0, nullptr);
}

// ------------------------------------------------------------------ layout
struct Layout {
  size_t total = 0;
  size_t off_state = 0, off_partials = 0, off_scalar = 0, off_x2 = 0;
  std::vector<size_t> f, w, u, t;      // FP64 levels
  std::vector<size_t> fs, ws, us, ts;  // FP32 levels
};

size_t take(size_t &cur, size_t bytes) {
  const size_t o = cur;
  cur = align_up(cur + bytes);
  return o;
}

Layout make_layout(const gmg_plan &p) {
  Layout Y;
  size_t cur = 0;
  const int L = p.L, B = p.B, dim = p.dim;
  const size_t none = (size_t)-1;
  Y.off_state = take(cur, 4096);
  Y.off_partials = take(cur, sizeof(double) * kMaxPartials);
  Y.off_scalar = take(cur, 256);
  const bool mixed = p.cfg.precision == GMG_MIXED_FP32_IR;
  auto carve = [&](std::vector<size_t> &F, std::vector<size_t> &W, std::vector<size_t> &U,
                   std::vector<size_t> &Tt, size_t elem) {
    F.assign(L, none);
    W.assign(L, none);
    U.assign(L, none);
    Tt.assign(L, none);
    for (int l = 0; l < L; ++l) {
      const size_t n = npts(dim, p.m[l]) * elem;
      if (l == 0) {
        W[0] = take(cur, n);
        if (p.need_tmp) Tt[0] = take(cur, n);
        if (elem == sizeof(float)) {  // mixed: the FP32 cycle's own RHS and result
          F[0] = take(cur, n);
          U[0] = take(cur, n);
        }
        continue;
      }
      if (l < B) {
        F[l] = take(cur, n);
        W[l] = take(cur, n);
        U[l] = take(cur, n);
        if (p.need_tmp) Tt[l] = take(cur, n);
      } else if (l == B) {
        F[l] = take(cur, n);
        U[l] = take(cur, n);
      }
    }
  };
  if (!mixed) {
    carve(Y.f, Y.w, Y.u, Y.t, sizeof(double));
  } else {
    Y.off_x2 = take(cur, npts(dim, p.m[0]) * sizeof(double));
    carve(Y.fs, Y.ws, Y.us, Y.ts, sizeof(float));
    Y.f.assign(L, none);
    Y.w.assign(L, none);
    Y.u.assign(L, none);
    Y.t.assign(L, none);
  }
  Y.total = cur;
  return Y;
}

template <typename T>
void bind(LevelSet<T> &S, char *ws, const std::vector<size_t> &F, const std::vector<size_t> &W,
          const std::vector<size_t> &U, const std::vector<size_t> &Tt) {
  const size_t none = (size_t)-1;
  auto ptr = [&](size_t o) -> T * { return o == none ? nullptr : reinterpret_cast<T *>(ws + o); };
  const size_t L = F.size();
  S.f.resize(L);
  S.w.resize(L);
  S.u.resize(L);
  S.t.resize(L);
  for (size_t l = 0; l < L; ++l) {
    S.f[l] = ptr(F[l]);
    S.w[l] = ptr(W[l]);
    S.u[l] = ptr(U[l]);
    S.t[l] = ptr(Tt[l]);
  }
}

// default tile variant and z-chunk for a level and stage count
void default_tiles(gmg_plan &p) {
  p.var.assign(p.L, {0, 0, 0, 0, 0});
  p.tz.assign(p.L, {0, 0, 0, 0, 0});
  const bool wj = p.cfg.smoother == GMG_SMOOTH_WJ;
  for (int l = 0; l < p.L; ++l) {
    for (int st = 1; st <= 4; ++st) {
      const int nv = pass_variant_count(p.dim, st, wj ? 1 : 0);
      if (nv == 0) continue;
      // prefer the large tile on big levels, the small one otherwise
      const int v = (p.m[l] >= 255 || nv == 1) ? 0 : 1;
      p.var[l][st] = v;
      const PassTile t = pass_variant(p.dim, st, wj ? 1 : 0, v);
      const PassGeom g0 = pass_geometry(p.dim, p.m[l], st, t, p.m[l]);
      // enough workgroups to cover the 256 CUs a few times, z-chunks >= 16
      const int xy = g0.ntx * g0.nty;
      int ntz = std::max(1, (3 * 256 + xy - 1) / xy);
      int tzv = (p.m[l] + ntz - 1) / ntz;
      tzv = std::max(tzv, std::min(p.m[l], 16));
      p.tz[l][st] = tzv;
    }
  }
}

gmg_status validate_cfg(const gmg_config *c) {
  if (!c) return GMG_ERR_INVALID_ARG;
  if (c->dim != 2 && c->dim != 3) return GMG_ERR_INVALID_ARG;
  if (c->levels < 1 || c->levels > kMaxLevels) return GMG_ERR_INVALID_ARG;
  if (c->dim == 3 && c->levels > 10) return GMG_ERR_INVALID_ARG;  // 1023^3 max (int32 index)
  if (c->nu1 < 0 || c->nu2 < 0 || c->nu1 + c->nu2 < 1 || c->nu1 > 8 || c->nu2 > 8)
    return GMG_ERR_INVALID_ARG;
  if (c->smoother != GMG_SMOOTH_RBGS && c->smoother != GMG_SMOOTH_WJ) return GMG_ERR_INVALID_ARG;
  if (c->smoother == GMG_SMOOTH_WJ && !(c->omega >= 0.0 && c->omega <= 1.0))
    return GMG_ERR_INVALID_ARG;
  if (c->precision != GMG_FP64 && c->precision != GMG_MIXED_FP32_IR) return GMG_ERR_INVALID_ARG;
  if (c->inner_cycles < 1 || c->inner_cycles > 16) return GMG_ERR_INVALID_ARG;
  return GMG_OK;
}

gmg_status init_plan_shape(gmg_plan &p, const gmg_config *cfg) {
  p.cfg = *cfg;
  if (p.cfg.smoother == GMG_SMOOTH_WJ && p.cfg.omega == 0.0)
    p.cfg.omega = cfg->dim == 3 ? 6.0 / 7.0 : 0.8;
  p.dim = cfg->dim;
  p.L = cfg->levels;
  p.m.resize(p.L);
  for (int l = 0; l < p.L; ++l) p.m[l] = (1 << (p.L - l)) - 1;
  const size_t elem = cfg->precision == GMG_MIXED_FP32_IR ? sizeof(float) : sizeof(double);
  const int mb = bottom_side_max(p.dim, cfg->smoother == GMG_SMOOTH_WJ ? 1 : 0, elem);
  p.B = p.L;  // first level with side <= mb, but never level 0
  for (int l = 1; l < p.L; ++l)
    if (p.m[l] <= mb) {
      p.B = l;
      break;
    }
  if (p.L == 1) p.B = 1;
  p.smax = (cfg->flags & GMG_NO_TEMPORAL_BLOCKING) ? 1 : 2;
  p.need_tmp = std::max(cfg->nu1, cfg->nu2) > p.smax;
  p.profile = (cfg->flags & GMG_PROFILE) != 0;
  return GMG_OK;
}

gmg_status map_status(int s) {
  switch (s) {
    case 0: return GMG_OK;
    case 1: return GMG_NOT_CONVERGED;
    case -3: return GMG_ERR_NONFINITE;
    case -4: return GMG_ERR_DIVERGED;
    default: return GMG_ERR_HIP;
  }
}

// Cycle bodies still needed judging from the contraction seen so far: the
// state holds res_k after k = done cycles and cycle k+1 already ran.
int estimate_cycles(const SolveState &st, int done) {
  if (st.res0 <= 0.0 || st.res <= 0.0 || done <= 0) return 2;
  const double rel = st.res / st.res0;
  const double rho = std::pow(rel, 1.0 / done);
  if (!(rho > 0.0) || rho >= 0.95) return 4;
  const double need = std::log(st.rtol / rel) / std::log(rho);
  int k = (int)std::ceil(need);
  return std::max(1, std::min(k, 64));
}

}  // namespace

// =================================================================== C ABI
extern "C" {

const char *gmg_status_string(gmg_status s) {
  switch (s) {
    case GMG_OK: return "GMG_OK";
    case GMG_NOT_CONVERGED: return "GMG_NOT_CONVERGED";
    case GMG_ERR_INVALID_ARG: return "GMG_ERR_INVALID_ARG";
    case GMG_ERR_WORKSPACE: return "GMG_ERR_WORKSPACE";
    case GMG_ERR_NONFINITE: return "GMG_ERR_NONFINITE";
    case GMG_ERR_DIVERGED: return "GMG_ERR_DIVERGED";
    case GMG_ERR_HIP: return "GMG_ERR_HIP";
    case GMG_ERR_UNSUPPORTED: return "GMG_ERR_UNSUPPORTED";
  }
  return "GMG_UNKNOWN_STATUS";
}

gmg_status gmg_config_default(gmg_config *cfg, int dim, int levels) {
  if (!cfg) return GMG_ERR_INVALID_ARG;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->dim = dim;
  cfg->levels = levels;
  cfg->smoother = GMG_SMOOTH_RBGS;
  cfg->nu1 = 2;
  cfg->nu2 = 2;
  cfg->omega = 0.0;
  cfg->precision = GMG_FP64;
  cfg->inner_cycles = 1;
  cfg->flags = 0;
  return validate_cfg(cfg);
}

gmg_status gmg_setup(const gmg_config *cfg, int nproblems, const int *dims, const int *levels,
                     void *workspace, size_t *ws_bytes, void *stream, gmg_plan **out) {
  if (!ws_bytes) return GMG_ERR_INVALID_ARG;
  if (nproblems < 1) return GMG_ERR_INVALID_ARG;
  if (nproblems > 1) return GMG_ERR_UNSUPPORTED;  // batch plans: not in this build yet
  gmg_config c = cfg ? *cfg : gmg_config{};
  if (!cfg) return GMG_ERR_INVALID_ARG;
  if (dims) c.dim = dims[0];
  if (levels) c.levels = levels[0];
  gmg_status st = validate_cfg(&c);
  if (st != GMG_OK) return st;
  gmg_plan tmp;
  init_plan_shape(tmp, &c);
  const Layout Y = make_layout(tmp);
  if (!workspace) {
    *ws_bytes = Y.total;
    return GMG_OK;
  }
  if (!out) return GMG_ERR_INVALID_ARG;
  if (*ws_bytes < Y.total) return GMG_ERR_WORKSPACE;
  if (((uintptr_t)workspace) % kAlign) return GMG_ERR_WORKSPACE;
  gmg_plan *p = new gmg_plan();
  init_plan_shape(*p, &c);
  p->nproblems = 1;
  p->stream = (hipStream_t)stream;
  p->ws = (char *)workspace;
  p->ws_bytes = Y.total;
  p->state = reinterpret_cast<SolveState *>(p->ws + Y.off_state);
  p->partials = reinterpret_cast<double *>(p->ws + Y.off_partials);
  p->scalar = reinterpret_cast<double *>(p->ws + Y.off_scalar);
  if (c.precision == GMG_MIXED_FP32_IR) {
    p->x2 = reinterpret_cast<double *>(p->ws + Y.off_x2);
    bind<float>(p->s, p->ws, Y.fs, Y.ws, Y.us, Y.ts);
    bind<double>(p->d, p->ws, Y.f, Y.w, Y.u, Y.t);
  } else {
    bind<double>(p->d, p->ws, Y.f, Y.w, Y.u, Y.t);
    std::vector<size_t> none(p->L, (size_t)-1);
    bind<float>(p->s, p->ws, none, none, none, none);
  }
  default_tiles(*p);
  p->prof.resize(PC_COUNT);
  for (int i = 0; i < PC_COUNT; ++i) p->prof[i].name = kProfNames[i];
  if (hipHostMalloc((void **)&p->hstate, sizeof(SolveState) + 64, hipHostMallocDefault) !=
      hipSuccess) {
    delete p;
    return GMG_ERR_HIP;
  }
  p->hscalar = reinterpret_cast<double *>(reinterpret_cast<char *>(p->hstate) + sizeof(SolveState));
  *out = p;
  return GMG_OK;
}

gmg_status gmg_destroy(gmg_plan *p) {
  if (!p) return GMG_ERR_INVALID_ARG;
  for (auto &e : p->pending) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  for (auto e : p->evpool) (void)hipEventDestroy(e);
  if (p->hstate) (void)hipHostFree(p->hstate);
  delete p;
  return GMG_OK;
}

size_t gmg_plan_workspace_bytes(const gmg_plan *p) { return p ? p->ws_bytes : 0; }

int gmg_level_side(const gmg_plan *p, int problem, int level) {
  if (!p || problem != 0 || level < 0 || level >= p->L) return -1;
  return p->m[level];
}

gmg_status gmg_vcycle(gmg_plan *p, double *u, const double *f) {
  if (!p || !u || !f) return GMG_ERR_INVALID_ARG;
  if (p->cfg.precision == GMG_FP64) {
    // u -> w0 (pre) ... w0 + P u1 -> u (post): u is never read and written by one pass
    HIPCHK(enqueue_vcycle<double>(p, u, f, u, nullptr, nullptr));
    return GMG_OK;
  }
  // mixed: one refinement step, x <- x + V32(f - A x)
  IrArgs a;
  a.x = u;
  a.e = nullptr;
  a.f = f;
  a.x_out = nullptr;
  a.r32 = p->s.f[0];
  a.partials = p->partials;
  a.active = nullptr;
  a.m = p->m[0];
  a.nblocks = ir_blocks(p->dim, p->m[0]);
  const double h = 1.0 / double(p->m[0] + 1);
  a.inv_h2 = 1.0 / (h * h);
  {
    ProfScope ps(p, PC_IR, (double)npts(p->dim, p->m[0]) * 20.0);
    HIPCHK(launch_ir_step(p->dim, a, p->stream));
  }
  for (int c = 0; c < p->cfg.inner_cycles; ++c)
    HIPCHK(enqueue_vcycle<float>(p, c == 0 ? nullptr : p->s.u[0], p->s.f[0], p->s.u[0], nullptr,
                                 nullptr));
  HIPCHK(launch_axpy_f32(u, p->s.u[0], npts(p->dim, p->m[0]), nullptr, p->stream));
  return GMG_OK;
}

static gmg_status read_state(gmg_plan *p) {
  HIPCHK(hipMemcpyAsync(p->hstate, p->state, sizeof(SolveState), hipMemcpyDeviceToHost,
                        p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return GMG_OK;
}

gmg_status gmg_solve(gmg_plan *p, double *u, const double *f, double rtol, int maxit,
                     const double *res0_opt, int *iters, double *relres) {
  if (!p || !u || !f) return GMG_ERR_INVALID_ARG;
  if (!(rtol > 0.0) || maxit < 1) return GMG_ERR_INVALID_ARG;
  if (res0_opt && !(*res0_opt >= 0.0)) return GMG_ERR_INVALID_ARG;
  const double r0 = res0_opt ? *res0_opt : -1.0;
  HIPCHK(launch_state_init(p->state, maxit, rtol, r0, p->stream));
  const int *act = &p->state->active;
  const bool mixed = p->cfg.precision == GMG_MIXED_FP32_IR;
  const int m0 = p->m[0];
  const size_t N0 = npts(p->dim, m0);
  const double h = 1.0 / double(m0 + 1);
  int enq = 0;  // cycle bodies enqueued (body k checks the residual after k cycles)
  int batch = 2;
  for (;;) {
    for (int b = 0; b < batch; ++b, ++enq) {
      if (!mixed) {
        HIPCHK(enqueue_vcycle<double>(p, u, f, u, p->partials, act));
      } else {
        // body k: x_k = x_{k-1} + e (k >= 1), r32 = f - A x_k, norm, stop
        // test, then the FP32 cycle(s) for the next correction.  Iterates
        // alternate between u (even k) and the workspace copy (odd k).
        IrArgs a;
        a.x = (enq == 0 || (enq - 1) % 2 == 0) ? u : p->x2;  // x_{k-1}
        a.e = enq == 0 ? nullptr : p->s.u[0];
        a.x_out = (enq % 2 == 0) ? u : p->x2;                // x_k
        a.f = f;
        a.r32 = p->s.f[0];
        a.partials = p->partials;
        a.active = act;
        a.m = m0;
        a.nblocks = ir_blocks(p->dim, m0);
        a.inv_h2 = 1.0 / (h * h);
        {
          ProfScope ps(p, PC_IR, (double)N0 * (enq == 0 ? 20.0 : 32.0));
          HIPCHK(launch_ir_step(p->dim, a, p->stream));
        }
        {
          ProfScope ps(p, PC_FIN, 0.0);
          HIPCHK(launch_finalize(p->partials, a.nblocks, p->state, p->stream));
        }
        for (int c = 0; c < p->cfg.inner_cycles; ++c)
          HIPCHK(enqueue_vcycle<float>(p, c == 0 ? nullptr : p->s.u[0], p->s.f[0], p->s.u[0],
                                       nullptr, act));
      }
    }
    gmg_status rs = read_state(p);
    if (rs != GMG_OK) return rs;
    if (!p->hstate->active) break;
    // body k checks x_k and (if it continues) computes x_{k+1}; the state
    // machine stops at the latest in body maxit
    if (enq >= maxit + 1) break;
    batch = std::min(estimate_cycles(*p->hstate, p->hstate->iter - 1), maxit + 1 - enq);
    if (batch < 1) batch = 1;
  }
  const SolveState st = *p->hstate;
  if (mixed && (st.iter % 2 == 1)) {
    // the final iterate x_iter sits in the workspace copy
    HIPCHK(launch_copy(p->x2, u, N0 * sizeof(double), nullptr, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
  }
  if (iters) *iters = st.iter;
  if (relres) *relres = st.res0 > 0.0 ? st.res / st.res0 : 0.0;
  if (p->profile) {
    gmg_status hs = harvest(p);
    if (hs != GMG_OK) return hs;
  }
  return map_status(st.status);
}

gmg_status gmg_batch_solve(gmg_plan *p, double *const *u, const double *const *f, double rtol,
                           int maxit, int *iters, double *relres, gmg_status *st) {
  (void)u;
  (void)f;
  (void)rtol;
  (void)maxit;
  (void)iters;
  (void)relres;
  (void)st;
  if (!p) return GMG_ERR_INVALID_ARG;
  return GMG_ERR_UNSUPPORTED;
}

int gmg_tile_variant_count(int dim, gmg_smoother smoother, int stages) {
  if ((dim != 2 && dim != 3) || stages < 1 || stages > 4) return 0;
  return pass_variant_count(dim, stages, smoother == GMG_SMOOTH_WJ ? 1 : 0);
}

gmg_status gmg_plan_set_tile(gmg_plan *p, int level, int stages, int variant, int tz) {
  if (!p || level < 0 || level >= p->L || stages < 1 || stages > 4 || tz < 0)
    return GMG_ERR_INVALID_ARG;
  const int wj = p->cfg.smoother == GMG_SMOOTH_WJ ? 1 : 0;
  const int nv = pass_variant_count(p->dim, stages, wj);
  if (variant < 0 || variant >= nv) return GMG_ERR_INVALID_ARG;
  p->var[level][stages] = variant;
  if (tz > 0) {
    p->tz[level][stages] = std::min(tz, p->m[level]);
  } else {
    const PassTile t = pass_variant(p->dim, stages, wj, variant);
    const PassGeom g0 = pass_geometry(p->dim, p->m[level], stages, t, p->m[level]);
    const int xy = g0.ntx * g0.nty;
    const int ntz = std::max(1, (3 * 256 + xy - 1) / xy);
    p->tz[level][stages] = std::max((p->m[level] + ntz - 1) / ntz, std::min(p->m[level], 16));
  }
  const PassGeom g = pass_geometry(p->dim, p->m[level], stages,
                                   pass_variant(p->dim, stages, wj, variant), p->tz[level][stages]);
  if (g.nblocks > kMaxPartials) return GMG_ERR_INVALID_ARG;
  return GMG_OK;
}

// ------------------------------------------------------------------ primitives
static gmg_status check_level(gmg_plan *p, int level, gmg_dtype dt) {
  if (!p || level < 0 || level >= p->L) return GMG_ERR_INVALID_ARG;
  if (dt != GMG_F64 && dt != GMG_F32) return GMG_ERR_INVALID_ARG;
  return GMG_OK;
}

}  // extern "C"

template <typename T>
static gmg_status op_smooth_t(gmg_plan *p, int level, int nsweeps, int backward, const T *u_in,
                              const T *f, const T *ec, T *u_out, double *res_in_norm) {
  LevelSet<T> &S = levels_of<T>(p);
  T *tmp = level < (int)S.t.size() ? S.t[level] : nullptr;
  const int K = nsweeps == 0 ? 0 : (nsweeps + p->smax - 1) / p->smax;
  if (K >= 2 && !tmp) return GMG_ERR_UNSUPPORTED;  // plan made without chained-pass scratch
  int nparts = 0;
  HIPCHK(smooth_chain<T>(p, level, nsweeps, backward != 0, u_in, ec, f, u_out, tmp,
                         res_in_norm ? p->partials : nullptr, nullptr, PC_MISC, &nparts));
  if (res_in_norm) {
    HIPCHK(launch_reduce_norm(p->partials, nparts, p->scalar, p->stream));
    HIPCHK(hipMemcpyAsync(p->hscalar, p->scalar, sizeof(double), hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    *res_in_norm = *p->hscalar;
  }
  return GMG_OK;
}

extern "C" {

gmg_status gmg_op_smooth(gmg_plan *p, int level, gmg_dtype dt, int nsweeps, int backward,
                         const void *u_in, const void *f, const void *e_coarse, void *u_out,
                         double *res_in_norm) {
  gmg_status s = check_level(p, level, dt);
  if (s != GMG_OK) return s;
  if (!f || !u_out || nsweeps < 0 || nsweeps > 16) return GMG_ERR_INVALID_ARG;
  if (u_out == u_in || u_out == f || u_out == e_coarse) return GMG_ERR_INVALID_ARG;
  if (e_coarse && level + 1 >= p->L) return GMG_ERR_INVALID_ARG;
  if (e_coarse && res_in_norm) return GMG_ERR_INVALID_ARG;
  if (dt == GMG_F64)
    return op_smooth_t<double>(p, level, nsweeps, backward, (const double *)u_in,
                               (const double *)f, (const double *)e_coarse, (double *)u_out,
                               res_in_norm);
  return op_smooth_t<float>(p, level, nsweeps, backward, (const float *)u_in, (const float *)f,
                            (const float *)e_coarse, (float *)u_out, res_in_norm);
}

gmg_status gmg_op_restrict_residual(gmg_plan *p, int level, gmg_dtype dt, const void *u,
                                    const void *f, void *f_coarse) {
  gmg_status s = check_level(p, level, dt);
  if (s != GMG_OK) return s;
  if (level + 1 >= p->L || !u || !f || !f_coarse) return GMG_ERR_INVALID_ARG;
  if (dt == GMG_F64)
    HIPCHK(restrict_level<double>(p, level, (const double *)u, (const double *)f,
                                  (double *)f_coarse, nullptr, PC_MISC));
  else
    HIPCHK(restrict_level<float>(p, level, (const float *)u, (const float *)f, (float *)f_coarse,
                                 nullptr, PC_MISC));
  return GMG_OK;
}

gmg_status gmg_op_residual(gmg_plan *p, int level, gmg_dtype dt, const void *u, const void *f,
                           void *r, double *norm) {
  gmg_status s = check_level(p, level, dt);
  if (s != GMG_OK) return s;
  if (!u || !f) return GMG_ERR_INVALID_ARG;
  const int m = p->m[level];
  const double h = 1.0 / double(m + 1);
  const int nb = residual_blocks(p->dim, m);
  if (dt == GMG_F64) {
    ResidArgs<double> a{(const double *)u, (const double *)f, (double *)r,
                        norm ? p->partials : nullptr, nullptr, m, nb, 1.0 / (h * h)};
    HIPCHK(launch_residual<double>(p->dim, a, p->stream));
  } else {
    ResidArgs<float> a{(const float *)u, (const float *)f, (float *)r,
                       norm ? p->partials : nullptr, nullptr, m, nb, 1.0 / (h * h)};
    HIPCHK(launch_residual<float>(p->dim, a, p->stream));
  }
  if (norm) {
    HIPCHK(launch_reduce_norm(p->partials, nb, p->scalar, p->stream));
    HIPCHK(hipMemcpyAsync(p->hscalar, p->scalar, sizeof(double), hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    *norm = *p->hscalar;
  }
  return GMG_OK;
}

// ------------------------------------------------------------------ profiling
int gmg_profile_count(const gmg_plan *p) { return p ? PC_COUNT : 0; }

gmg_status gmg_profile_get(gmg_plan *p, int idx, gmg_kernel_stat *out) {
  if (!p || !out || idx < 0 || idx >= PC_COUNT) return GMG_ERR_INVALID_ARG;
  gmg_status s = harvest(p);
  if (s != GMG_OK) return s;
  std::memset(out, 0, sizeof(*out));
  std::snprintf(out->name, sizeof(out->name), "%s", p->prof[idx].name.c_str());
  out->launches = p->prof[idx].launches;
  out->total_ms = p->prof[idx].ms;
  out->alg_bytes = p->prof[idx].bytes;
  return GMG_OK;
}

gmg_status gmg_profile_reset(gmg_plan *p) {
  if (!p) return GMG_ERR_INVALID_ARG;
  gmg_status s = harvest(p);
  for (auto &q : p->prof) {
    q.launches = 0;
    q.ms = 0.0;
    q.bytes = 0.0;
  }
  return s;
}

}  // extern "C"
