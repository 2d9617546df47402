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
#include <map>
#include <mutex>
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
  int tag;  // solve-loop body that enqueued the launch (-1: outside a solve)
};

struct PassChoice {
  int smax = 2;
  std::array<int, 5> var{{0, 0, 0, 0, 0}};
  std::array<int, 5> tz{{0, 0, 0, 0, 0}};
  std::array<int, 5> sw{{0, 0, 0, 0, 0}};  // tile order: strip width in tiles (0: rows)
  int fuse = 1;  // pre-smoothing: fold the residual + restriction into the last pass
};

template <typename T>
struct LevelSet {
  // per level: f (RHS), w (after pre-smoothing), u (after post-smoothing),
  // t (scratch for chained passes).  Level 0's f/u are supplied per call.
  std::vector<T *> f, w, u, t;
};

}  // namespace

// ---------------------------------------------------------------- batch plans
// One problem of a batch: its level table and workspace arrays.
struct BProblem {
  int dim = 3, L = 2, B = 1;
  std::vector<int> m;
  std::vector<double *> f, w, u, t;  // per level (level 0: w, t only)
  double *partials = nullptr;        // slice for its level-0 norm pass
  int npart = 0;
  SolveState *st = nullptr;
};

// One launch of the batched cycle; its argument entries live in a device
// table (byte offset tbl_off in the table region).
enum BOpKind { BO_PASS = 0, BO_RESTRICT = 1, BO_FIN = 2, BO_BOTTOM = 3 };
struct BOp {
  int kind = BO_PASS;
  int dim = 3, stages = 0, flags = 0, variant = 0, wj = 0, nent = 0;
  size_t tbl_off = 0;
  int cls = 0;
  double bytes = 0.0;
  size_t lds = 0;      // bottom: LDS bytes for the largest entry
  int bottom_L = 0;    // bottom: largest sub-hierarchy
  int bottom_dim = 3;
  int branch = 0;      // 0: the plan's stream; 1: the side stream (2D problems)
};

struct Batch {
  std::vector<BProblem> pb;
  std::vector<BOp> ops;
  std::vector<char> host_tbl;  // host image of the table region
  char *dev_tbl = nullptr;     // the table region inside the workspace
  char *pinned = nullptr;      // pinned staging copy for uploads
  struct Patch {
    size_t off;  // byte offset of a pointer field in the table image
    int prob;
    int which;   // 0: caller's u, 1: caller's f
  };
  std::vector<Patch> patches;
  SolveState *states = nullptr;
  SolveState *hstates = nullptr;  // pinned
  hipGraphExec_t graph = nullptr;
  // tile choice per (dim, level side, role) after autotuning (else defaults)
  std::map<std::array<int, 3>, PassChoice> choice;
  // problems with a smoothed level of each (dim, side): the workgroups of
  // one launch of that level are this many times a single problem's
  std::map<std::array<int, 2>, int> shape_count;
  bool worst = false;      // sizing: one sweep per pass everywhere (most launches)
  size_t tbl_reserve = 0;  // table region reserved for any choice
  // 2D and 3D problems share no launch and no data, so a batch holding both
  // runs them as two concurrent branches: the 3D launches on the plan's
  // stream, the 2D ones on a side stream forked from it at the start of a
  // cycle and joined back at its end (the same launches as one stream, so
  // the same bits)
  bool two = false;
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

struct gmg_plan {
  gmg_config cfg;
  int nproblems = 1;
  hipStream_t stream = nullptr;
  char *ws = nullptr;
  size_t ws_bytes = 0;

  int dim = 3, L = 1, B = 1;  // B: first level handled by the bottom kernel
  std::vector<int> m;         // sides
  int smax_cap = 2;           // most sweeps fused into one pass
  bool need_tmp = false;
  bool tuned = false;
  double omega_user = 0.0;  // WJ weight as the caller gave it (0: the default of each dimension)

  SolveState *state = nullptr;
  double *partials = nullptr;
  double *scalar = nullptr;  // device scratch for primitive norms

  LevelSet<double> d;  // FP64 levels
  LevelSet<float> s;   // FP32 levels (mixed precision)
  double *x2 = nullptr;  // FP64 ping-pong partner of the caller's u (mixed)

  // per level and role (0: descent / pre-smoothing, 1: ascent / post-smoothing
  // with the fused prolongation): sweeps per pass and the tile shape and
  // z-chunk for each stage count
  std::vector<std::array<PassChoice, 3>> ch;  // role 2: the cross-cycle pass (level 0)
  // FP64 red-black V(1,1) with Algorithm 1's backward post-smoothing: the
  // solve loop runs the cross-cycle schedule (one level-0 pass per cycle that
  // ends the cycle's post-smoothing and starts the next cycle's
  // pre-smoothing)
  bool cross = false;
  // mixed V(1,1) with the same sweep orders: the FP32 cycles of a refinement
  // step run that schedule among themselves
  bool cross32 = false;

  // profiling
  bool profile = false;
  unsigned prof_mask = ~0u;
  std::vector<Prof> prof;
  std::vector<PendingEv> pending;
  int prof_tag = -1;  // body index of the solve loop being enqueued
  std::vector<hipEvent_t> evpool;

  SolveState *hstate = nullptr;  // pinned host copy
  double *hscalar = nullptr;

  // hipGraph of the coarse part of one cycle (levels >= 1 and the bottom),
  // per precision and per "gated by the solve state or not"
  hipGraphExec_t coarse_graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  hipStream_t capture_stream = nullptr;

  struct Batch *batch = nullptr;  // batch plans (nproblems > 1)
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
  PC_CROSS0,
  PC_COUNT
};
const char *kProfNames[PC_COUNT] = {"smooth_pre_l0", "smooth_post_l0", "resid_restrict_l0",
                                    "smooth_pre_coarse", "smooth_post_coarse",
                                    "resid_restrict_coarse", "bottom", "finalize", "ir_step",
                                    "misc", "smooth_cross_l0"};

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

}  // namespace

DispatchEvents &gmg::next_dispatch_events() {
  static thread_local DispatchEvents ev{nullptr, nullptr};
  return ev;
}

namespace {

// Times the one kernel launch inside its scope: the dispatch itself records
// the start and end events (no marker packets around it).
struct ProfScope {
  gmg_plan *p;
  int cls;
  double bytes;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(gmg_plan *p_, int cls_, double bytes_) : p(p_), cls(cls_), bytes(bytes_) {
    if (!p->profile || !((p->prof_mask >> cls) & 1u)) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(p->stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
      return;
    a = get_event(p);
    b = get_event(p);
    if (a && b) next_dispatch_events() = {a, b};
  }
  ~ProfScope() {
    if (!a || !b) return;
    DispatchEvents &ev = next_dispatch_events();
    if (ev.start == a) {  // nothing was launched
      ev.start = ev.stop = nullptr;
      p->evpool.push_back(a);
      p->evpool.push_back(b);
      return;
    }
    p->pending.push_back({cls, a, b, bytes, p->prof_tag});
  }
};

// The solve loop enqueues bodies ahead of its stop test; the kernels of a
// body after the one that stopped the loop return at once.  Drop their
// timings (and, in the stopping body, everything after the step that ran
// the test), so profiles average over launches that did their work.
void prune_profile(gmg_plan *p, int last_body, unsigned keep_mask) {
  std::vector<PendingEv> kept;
  kept.reserve(p->pending.size());
  for (auto &e : p->pending) {
    const bool drop =
        e.tag >= 0 && (e.tag > last_body || (e.tag == last_body && !((keep_mask >> e.cls) & 1u)));
    if (drop) {
      p->evpool.push_back(e.a);
      p->evpool.push_back(e.b);
    } else {
      kept.push_back(e);
    }
  }
  p->pending.swap(kept);
}

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

// Plans that run the paper's own smoother or transfers (multicolour GS, the
// finite-element transfers, the relaxed coarsest level) go through the
// per-step kernels of variant.hip.
bool cfg_variant(const gmg_config &c) {
  return c.smoother == GMG_SMOOTH_MCGS || (c.flags & (GMG_FE_TRANSFER | GMG_COARSE_RELAX));
}
bool is_variant(const gmg_plan *p) { return cfg_variant(p->cfg); }

// ------------------------------------------------------------------ passes
int stages_of(const gmg_plan *p, int sweeps) {
  return p->cfg.smoother == GMG_SMOOTH_RBGS ? 2 * sweeps : sweeps;
}

template <typename T>
hipError_t one_pass_st(gmg_plan *p, int level, int role, int st, int flags, const T *src,
                       const T *ec, const T *f, T *dst, double *partials, const int *active,
                       int cls, T *fc = nullptr) {
  const int dim = p->dim, m = p->m[level];
  const bool wj = p->cfg.smoother == GMG_SMOOTH_WJ;
  const PassChoice &c = p->ch[level][role];
  const int v = c.var[st];
  const PassTile t = pass_variant(dim, st, wj ? 1 : 0, v);
  const PassGeom g = pass_geometry(dim, m, st, t, c.tz[st], (flags & F_RESTRICT) != 0);
  PassArgs<T> a;
  a.u_in = src;
  a.f = f;
  a.u_out = dst;
  a.e_c = ec;
  a.f_c = fc;
  a.partials = partials;
  a.active = active;
  a.m = m;
  a.mc = level + 1 < p->L ? p->m[level + 1] : 0;
  a.ntx = g.ntx;
  a.nty = g.nty;
  a.tz = g.tz;
  a.nblocks = g.nblocks;
  a.sw = c.sw[st];
  const double h = 1.0 / double(m + 1);
  a.h2 = h * h;
  a.inv_h2 = 1.0 / (h * h);
  a.omega = p->cfg.omega;
  double bytes = (double)npts(dim, m) * sizeof(T) * ((flags & F_ZERO_IN) ? 2 : 3);
  if (flags & F_PROLONG) bytes += (double)npts(dim, a.mc) * sizeof(T);
  if (flags & F_RESTRICT) bytes += (double)npts(dim, a.mc) * sizeof(T);
  ProfScope ps(p, cls, bytes);
  return wj ? launch_wj_pass<T>(dim, st, flags, v, a, p->stream)
            : launch_rb_pass<T>(dim, st, flags, v, a, p->stream);
}

template <typename T>
hipError_t one_pass(gmg_plan *p, int level, int role, int sweeps, int flags, const T *src,
                    const T *ec, const T *f, T *dst, double *partials, const int *active,
                    int cls, T *fc = nullptr) {
  return one_pass_st<T>(p, level, role, stages_of(p, sweeps), flags, src, ec, f, dst, partials,
                        active, cls, fc);
}

int pass_blocks(const gmg_plan *p, int level, int role, int sweeps, bool rst = false) {
  const int st = stages_of(p, sweeps);
  const bool wj = p->cfg.smoother == GMG_SMOOTH_WJ;
  const PassChoice &c = p->ch[level][role];
  const PassTile t = pass_variant(p->dim, st, wj ? 1 : 0, c.var[st]);
  return pass_geometry(p->dim, p->m[level], st, t, c.tz[st], rst).nblocks;
}

// Sweeps of the last pass of a chain of nu sweeps in passes of at most smax
// (the split build_chain and smooth_chain make), and the pass count.
int last_pass_sweeps(int nu, int smax, int *npasses) {
  const int K = (nu + smax - 1) / smax;
  int left = nu, last = 0;
  for (int k = 1; k <= K; ++k) {
    last = std::min(smax, left - (K - k));
    left -= last;
  }
  if (npasses) *npasses = K;
  return last;
}

// Whether the pre-smoothing of `level` (nsweeps sweeps in passes of the
// level's pre choice) can end in a pass that also restricts: red-black, a
// coarser level exists, the choice asks for it, and the last pass's tile
// fits in LDS with the restriction's planes.
bool can_fuse_restrict(const gmg_plan *p, int level, int nsweeps, size_t elem) {
  if (p->cfg.smoother != GMG_SMOOTH_RBGS || (p->cfg.flags & GMG_NO_FUSED_RESTRICT)) return false;
  if (nsweeps < 1 || level + 1 >= p->L) return false;
  const PassChoice &c = p->ch[level][0];
  if (!c.fuse) return false;
  const int st = stages_of(p, last_pass_sweeps(nsweeps, c.smax, nullptr));
  if (pass_geometry(p->dim, p->m[level], st, pass_variant(p->dim, st, 0, c.var[st]), c.tz[st], true)
          .nblocks > kMaxPartials)
    return false;
  return rb_pass_fits(p->dim, st, c.var[st], F_RESTRICT | F_NORM_IN, elem);
}

// nsweeps of the plan's smoother from (src [+ P ec]) to dst through fused
// passes of at most smax sweeps; intermediate passes alternate between tmp
// and dst so the last one lands in dst and no pass reads what it writes.
// partials != NULL: the first pass emits |f - A src|^2 partial sums.
// fc_out != NULL (pre-smoothing only): when the level allows it, the last
// pass also writes the restricted residual f_c = R (f - A dst) to fc_out and
// *fused is set; otherwise the caller restricts separately.
template <typename T>
hipError_t smooth_chain(gmg_plan *p, int level, int nsweeps, bool backward, const T *src,
                        const T *ec, const T *f, T *dst, T *tmp, double *partials,
                        const int *active, int cls, int *nparts, T *fc_out = nullptr,
                        bool *fused = nullptr) {
  const int role = ec ? 1 : 0;
  const bool fuse = fc_out && !ec && !backward && can_fuse_restrict(p, level, nsweeps, sizeof(T));
  if (fused) *fused = fuse;
  const int smax = p->ch[level][role].smax;
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
  const int K = (nsweeps + smax - 1) / smax;
  int left = nsweeps;
  const T *in = src;
  for (int k = 1; k <= K; ++k) {
    const int sw = std::min(smax, left - (K - k));  // keep later passes non-empty
    const int swk = std::min(sw, smax);
    T *out = ((K - k) % 2 == 1) ? tmp : dst;
    int flags = backward ? F_BLACK_FIRST : 0;
    const bool rst = fuse && k == K;
    if (rst) flags |= F_RESTRICT;
    if (k == 1) {
      if (!in) flags |= F_ZERO_IN;
      if (ec) flags |= F_PROLONG;
      if (partials) {
        flags |= F_NORM_IN;
        if (nparts) *nparts = pass_blocks(p, level, role, swk, rst);
      }
    }
    hipError_t e = one_pass<T>(p, level, role, swk, flags, in, k == 1 ? ec : nullptr, f, out,
                               k == 1 ? partials : nullptr, active, cls, rst ? fc_out : nullptr);
    if (e != hipSuccess) return e;
    in = out;
    left -= swk;
  }
  return hipSuccess;
}

template <typename T>
hipError_t restrict_level(gmg_plan *p, int level, const T *u, const T *f, T *fc,
                          const int *active, int cls, const double *fin_partials = nullptr,
                          int fin_n = 0) {
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
  a.fin_partials = fin_partials;
  a.fin_n = fin_n;
  a.fin_state = fin_partials ? p->state : nullptr;
  ProfScope ps(p, cls, (double)npts(p->dim, m) * sizeof(T) * 2 + (double)npts(p->dim, a.mc) * sizeof(T));
  return launch_restrict<T>(p->dim, a, p->stream);
}

// ------------------------------------------------------------------ cross-cycle pass
// The level-0 pass between two V(1,1) cycles of an FP64 red-black solve
// (Algorithm 1's cycle with its backward post-smoothing, repeated by
// Algorithm 3's loop).  From w_k + P e_k -- cycle k's pre-smoothed iterate
// and the interpolated coarse correction -- it runs the post-smoothing sweep
// (black, then red), which gives u_k and the partial sums of its residual
// norm for the stop test, and then cycle k+1's forward pre-smoothing sweep.
// That sweep's red half-sweep would recompute the red values just formed,
// from the same black neighbours, so it is left out: its black half-sweep is
// the third and last stage, and the pass writes w_{k+1}.  The residual of
// w_{k+1} and its full weighting (the next cycle's coarse right-hand side)
// are folded in when the tile allows it; otherwise the caller restricts.
// u_k itself is never stored: the solve forms it once, after its last cycle,
// with an ordinary post-smoothing pass from w_k + P e_k.
bool can_fuse_cross(const gmg_plan *p, size_t elem) {
  const PassChoice &c = p->ch[0][2];
  if (!c.fuse || (p->cfg.flags & GMG_NO_FUSED_RESTRICT)) return false;
  const PassTile t = pass_variant(p->dim, 3, 0, c.var[3]);
  if (pass_geometry(p->dim, p->m[0], 3, t, c.tz[3], true).nblocks > kMaxPartials) return false;
  return rb_pass_fits(p->dim, 3, c.var[3], F_PROLONG | F_RESTRICT, elem);
}

// partials != NULL (FP64 solves): the pass emits the norm of u_k's residual.
// The FP32 cycles of a refinement step run it without (no stop test between
// them).
template <typename T>
hipError_t cross_pass(gmg_plan *p, const T *w, const T *ec, const T *f, T *w_next,
                      double *partials, const int *active, T *fc, bool *fused, int *nparts) {
  const bool fz = can_fuse_cross(p, sizeof(T));
  *fused = fz;
  PassChoice &c = p->ch[0][2];
  // a tile made for the folded form (odd row count) cannot run the plain
  // one: the plain form then takes the first tile of the table
  if (!fz && !rb_pass_fits(p->dim, 3, c.var[3], F_PROLONG, sizeof(T))) c.var[3] = 0;
  *nparts = pass_geometry(p->dim, p->m[0], 3, pass_variant(p->dim, 3, 0, c.var[3]), c.tz[3], fz)
                .nblocks;
  const int flags =
      F_PROLONG | F_BLACK_FIRST | (partials ? F_NORM_MID : 0) | (fz ? F_RESTRICT : 0);
  return one_pass_st<T>(p, 0, 2, 3, flags, w, ec, f, w_next, partials, active, PC_CROSS0,
                        fz ? fc : nullptr);
}

// Level-0 buffers of the cross-cycle schedule: w_k (the pre-smoothed
// iterate of cycle k) lives in buffer k & 1 (FP64 solves; the FP32 cycles
// of a refinement step have their own pair).
template <typename T>
T *cross_buf(gmg_plan *p, int k);
template <>
double *cross_buf<double>(gmg_plan *p, int k) { return (k & 1) ? p->d.t[0] : p->d.w[0]; }
template <>
float *cross_buf<float>(gmg_plan *p, int k) { return (k & 1) ? p->s.t[0] : p->s.w[0]; }

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

// The descent on small coarse levels of a single problem goes through the
// fused LDS-tile kernel (red-black only; batches use the passes).
bool use_small(const gmg_plan *p, int dim, int m, int nu, size_t elem) {
  return p->cfg.smoother == GMG_SMOOTH_RBGS && !(p->cfg.flags & GMG_NO_FUSED_COARSE) && nu >= 1 &&
         small_level_ok(dim, m, nu, elem);
}

// Levels 1..B-1 of the descent, the bottom kernel and levels B-1..1 of the
// ascent: everything of a cycle that touches only workspace arrays.
template <typename T>
hipError_t enqueue_coarse(gmg_plan *p, const int *active, int first = 1) {
  LevelSet<T> &S = levels_of<T>(p);
  const int L = p->L, B = p->B;
  const bool bwd = !(p->cfg.flags & GMG_POST_FORWARD);
  const int nu1 = p->cfg.nu1, nu2 = p->cfg.nu2;
  hipError_t e;
  for (int l = first; l < B; ++l) {
    const int m = p->m[l];
    const double h = 1.0 / double(m + 1);
    if (use_small(p, p->dim, m, nu1, sizeof(T))) {
      SmallArgs<T> a{};
      a.f = S.f[l];
      a.w = S.w[l];
      a.fc = S.f[l + 1];
      a.active = active;
      a.m = m;
      a.mc = p->m[l + 1];
      a.nsweeps = nu1;
      a.h2 = h * h;
      a.inv_h2 = 1.0 / (h * h);
      ProfScope ps(p, PC_PRE_C, (double)npts(p->dim, m) * sizeof(T) * 2);
      e = launch_small<T>(p->dim, a, p->stream);
      if (e != hipSuccess) return e;
      continue;
    }
    bool fused = false;
    e = smooth_chain<T>(p, l, nu1, false, nullptr, nullptr, S.f[l], S.w[l], S.t[l], nullptr,
                        active, PC_PRE_C, nullptr, S.f[l + 1], &fused);
    if (e != hipSuccess) return e;
    if (!fused) {
      e = restrict_level<T>(p, l, S.w[l], S.f[l], S.f[l + 1], active, PC_RES_C);
      if (e != hipSuccess) return e;
    }
  }
  {
    BottomArgs<T> ba{};
    ba.active = active;
    ba.dim = p->dim;
    ba.nu1 = nu1;
    ba.nu2 = nu2;
    ba.smoother = p->cfg.smoother == GMG_SMOOTH_WJ ? 1 : 0;
    ba.post_forward = bwd ? 0 : 1;
    ba.omega = p->cfg.omega;
    ba.f = S.f[B];
    ba.u = S.u[B];
    ba.L = L - B;
    ProfScope ps(p, PC_BOTTOM, (double)npts(p->dim, p->m[B]) * sizeof(T) * 2);
    e = launch_bottom<T>(1, ba, nullptr, p->stream);
    if (e != hipSuccess) return e;
  }
  // The ascent of a single problem always takes the plane-marching pass: on
  // every level it beat the LDS-tile kernel (3D 255^3 cycle: 63^3 ascent 15
  // against 24 us, 31^3 14 against 18 us; 2D 4095^2 FMG pass 1.11 against
  // 1.15 ms); batches take it too (their 256-problem solve 77 -> 61 ms).
  for (int l = B - 1; l >= first; --l) {
    e = smooth_chain<T>(p, l, nu2, bwd, S.w[l], S.u[l + 1], S.f[l], S.u[l], S.t[l], nullptr,
                        active, PC_POST_C, nullptr);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The coarse part, eagerly or as a replay of a hipGraph captured on first
// use (GMG_USE_GRAPH; not while events are being recorded for these kernels).
template <typename T>
hipError_t run_coarse(gmg_plan *p, const int *active) {
  const unsigned coarse_cls = (1u << PC_PRE_C) | (1u << PC_RES_C) | (1u << PC_POST_C) |
                              (1u << PC_BOTTOM) | (1u << PC_MISC);
  const bool events = p->profile && (p->prof_mask & coarse_cls);
  if (!(p->cfg.flags & GMG_USE_GRAPH) || events) return enqueue_coarse<T>(p, active);
  const int ti = sizeof(T) == 8 ? 0 : 1, ai = active ? 1 : 0;
  if (!p->coarse_graph[ti][ai]) {
    hipError_t e;
    if (!p->capture_stream) {
      e = hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking);
      if (e != hipSuccess) return e;
    }
    hipStream_t keep = p->stream;
    p->stream = p->capture_stream;
    e = hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
      p->stream = keep;
      return e;
    }
    hipError_t ee = enqueue_coarse<T>(p, active);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(p->capture_stream, &g);
    p->stream = keep;
    if (ee != hipSuccess) return ee;
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&p->coarse_graph[ti][ai], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return e;
  }
  return hipGraphLaunch(p->coarse_graph[ti][ai], p->stream);
}

// One V-cycle on the plan's hierarchy in precision T.  Level 0: start value
// u0_in (NULL = zero), result u0_out (must not alias u0_in), RHS f0.
// norm_partials != NULL: the level-0 pre-pass emits the residual norm of
// u0_in, and a finalize step updates the solve state right after it.
template <typename T>
hipError_t enqueue_vcycle(gmg_plan *p, const T *u0_in, const T *f0, T *u0_out,
                          double *norm_partials, const int *active) {
  LevelSet<T> &S = levels_of<T>(p);
  const int L = p->L;
  const bool bwd = !(p->cfg.flags & GMG_POST_FORWARD);
  const int nu1 = p->cfg.nu1, nu2 = p->cfg.nu2;
  hipError_t e;
  int nparts = 0;
  BottomArgs<T> ba{};
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
    return launch_bottom<T>(1, ba, nullptr, p->stream);
  }
  // ---- descent
  bool fused = false;
  e = smooth_chain<T>(p, 0, nu1, false, u0_in, nullptr, f0, S.w[0], S.t[0], norm_partials, active,
                      PC_PRE0, &nparts, S.f[1], &fused);
  if (e != hipSuccess) return e;
  // (nu1 == 0: the chain copied the start value into w0, so the post-pass
  // below never reads the array it writes)
  const T *w0 = S.w[0];
  if (fused) {
    if (norm_partials) {  // the stop test, before any coarse work
      ProfScope ps(p, PC_FIN, 0.0);
      e = launch_finalize(norm_partials, nparts, p->state, p->stream);
      if (e != hipSuccess) return e;
    }
  } else {
    // the stop test runs in workgroup 0 of the level-0 restriction
    e = restrict_level<T>(p, 0, w0, f0, S.f[1], active, PC_RES0, norm_partials, nparts);
    if (e != hipSuccess) return e;
  }
  e = run_coarse<T>(p, active);
  if (e != hipSuccess) return e;
  return smooth_chain<T>(p, 0, nu2, bwd, w0, S.u[1], f0, u0_out, S.t[0], nullptr, active,
                         PC_POST0, nullptr);
}

// Body k of the cross-cycle solve loop (Algorithm 3 with V(1,1) cycles).
// Body 0: cycle 1's pre-smoothing of u into w_1 with the norm of u's
// residual, the stop test, cycle 1's coarse part.  Body k >= 1: the
// cross-cycle pass (u_k's norm, w_{k+1}, f_1 for cycle k+1), the stop test
// on u_k, cycle k+1's coarse part.  After the loop the solve forms u_K.
hipError_t enqueue_cross_body(gmg_plan *p, int k, const double *u, const double *f,
                              const int *active) {
  LevelSet<double> &S = p->d;
  bool fused = false;
  int nparts = 0;
  double *wn = cross_buf<double>(p, k + 1);
  hipError_t e;
  if (k == 0)
    e = smooth_chain<double>(p, 0, 1, false, u, nullptr, f, wn, nullptr, p->partials, active,
                             PC_PRE0, &nparts, S.f[1], &fused);
  else
    e = cross_pass<double>(p, cross_buf<double>(p, k), S.u[1], f, wn, p->partials, active,
                           S.f[1], &fused, &nparts);
  if (e != hipSuccess) return e;
  if (fused) {
    ProfScope ps(p, PC_FIN, 0.0);
    e = launch_finalize(p->partials, nparts, p->state, p->stream);
  } else {
    e = restrict_level<double>(p, 0, wn, f, S.f[1], active, PC_RES0, p->partials, nparts);
  }
  if (e != hipSuccess) return e;
  return run_coarse<double>(p, active);
}

// The FP32 cycles of one refinement step (mixed plans): inner_cycles V-cycles
// on A e = r32 (level-0 right-hand side s.f[0]) from e = 0, result in s.u[0].
// Plans that run the cross-cycle schedule (V(1,1), Algorithm 1's sweep
// orders) do it among these cycles: cycle 1's pre-smoothing from zero into
// w_1, the three-stage pass between consecutive cycles (no norm: the stop
// test belongs to the refinement step), cycle K's post-smoothing into e, and
// every cycle's coarse part in between -- the same iterates as K separate
// cycles.
hipError_t enqueue_inner(gmg_plan *p, const int *active) {
  LevelSet<float> &S = p->s;
  const int K = p->cfg.inner_cycles;
  if (!p->cross32) {
    for (int c = 0; c < K; ++c) {
      hipError_t e = enqueue_vcycle<float>(p, c == 0 ? nullptr : S.u[0], S.f[0], S.u[0], nullptr,
                                           active);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  for (int c = 1; c <= K; ++c) {
    float *wn = cross_buf<float>(p, c);
    bool fused = false;
    int nparts = 0;
    hipError_t e =
        c == 1 ? smooth_chain<float>(p, 0, 1, false, nullptr, nullptr, S.f[0], wn, nullptr,
                                     nullptr, active, PC_PRE0, &nparts, S.f[1], &fused)
               : cross_pass<float>(p, cross_buf<float>(p, c - 1), S.u[1], S.f[0], wn, nullptr,
                                   active, S.f[1], &fused, &nparts);
    if (e != hipSuccess) return e;
    if (!fused) {
      e = restrict_level<float>(p, 0, wn, S.f[0], S.f[1], active, PC_RES0);
      if (e != hipSuccess) return e;
    }
    e = run_coarse<float>(p, active);
    if (e != hipSuccess) return e;
  }
  return smooth_chain<float>(p, 0, 1, true, cross_buf<float>(p, K), S.u[1], S.f[0], S.u[0],
                             nullptr, nullptr, active, PC_POST0, nullptr);
}

// ------------------------------------------------------------------ FMG
// One V-cycle on the levels s .. L-1 (1 <= s < B) from the start value in the
// workspace u of level s, right-hand side f of level s, result back in u of
// level s: the general passes on level s (non-zero start), then the usual
// coarse part from level s+1.
hipError_t enqueue_vcycle_level(gmg_plan *p, int s) {
  LevelSet<double> &S = p->d;
  const bool bwd = !(p->cfg.flags & GMG_POST_FORWARD);
  bool fused = false;
  hipError_t e = smooth_chain<double>(p, s, p->cfg.nu1, false, S.u[s], nullptr, S.f[s], S.w[s],
                                      S.t[s], nullptr, nullptr, PC_PRE_C, nullptr, S.f[s + 1],
                                      &fused);
  if (e != hipSuccess) return e;
  if (!fused) {
    e = restrict_level<double>(p, s, S.w[s], S.f[s], S.f[s + 1], nullptr, PC_RES_C);
    if (e != hipSuccess) return e;
  }
  e = enqueue_coarse<double>(p, nullptr, s + 1);
  if (e != hipSuccess) return e;
  return smooth_chain<double>(p, s, p->cfg.nu2, bwd, S.w[s], S.u[s + 1], S.f[s], S.u[s], S.t[s],
                              nullptr, nullptr, PC_POST_C, nullptr);
}

// Full multigrid (Algorithm 2) into u: f restricted to every level (full
// weighting), the bottom levels by the bottom kernel's own full multigrid,
// then for each finer level the interpolated coarser solution and one
// V-cycle, ending with the finest level.
hipError_t enqueue_fmg(gmg_plan *p, double *u, const double *f) {
  LevelSet<double> &S = p->d;
  const int L = p->L, B = p->B;
  BottomArgs<double> ba{};
  ba.dim = p->dim;
  ba.nu1 = p->cfg.nu1;
  ba.nu2 = p->cfg.nu2;
  ba.smoother = p->cfg.smoother == GMG_SMOOTH_WJ ? 1 : 0;
  ba.post_forward = (p->cfg.flags & GMG_POST_FORWARD) ? 1 : 0;
  ba.omega = p->cfg.omega;
  ba.fmg = 1;
  hipError_t e;
  if (L == 1) {
    ba.f = f;
    ba.u = u;
    ba.L = 1;
    return launch_bottom<double>(1, ba, nullptr, p->stream);
  }
  for (int l = 0; l < B; ++l) {
    e = restrict_level<double>(p, l, nullptr, l == 0 ? f : S.f[l], S.f[l + 1], nullptr, PC_MISC);
    if (e != hipSuccess) return e;
  }
  ba.f = S.f[B];
  ba.u = S.u[B];
  ba.L = L - B;
  {
    ProfScope ps(p, PC_BOTTOM, (double)npts(p->dim, p->m[B]) * sizeof(double) * 2);
    e = launch_bottom<double>(1, ba, nullptr, p->stream);
    if (e != hipSuccess) return e;
  }
  for (int l = B - 1; l >= 1; --l) {
    e = launch_prolong_add<double>(p->dim, p->m[l], p->m[l + 1], nullptr, S.u[l + 1], S.u[l],
                                   nullptr, p->stream);
    if (e != hipSuccess) return e;
    e = enqueue_vcycle_level(p, l);
    if (e != hipSuccess) return e;
  }
  e = launch_prolong_add<double>(p->dim, p->m[0], p->m[1], nullptr, S.u[1], u, nullptr, p->stream);
  if (e != hipSuccess) return e;
  return enqueue_vcycle<double>(p, u, f, u, nullptr, nullptr);
}

// ------------------------------------------------------------------ paper variant
// nsweeps of the plan's smoother on level l from src (NULL = zero) into dst,
// alternating with tmp so that the last sweep lands in dst and no launch
// reads what it writes.  Red-black and Jacobi reuse the plain passes.
hipError_t var_smooth(gmg_plan *p, int l, int nsweeps, bool backward, const double *src,
                      const double *f, double *dst, double *tmp, const int *active, int cls) {
  if (p->cfg.smoother != GMG_SMOOTH_MCGS)
    return smooth_chain<double>(p, l, nsweeps, backward, src, nullptr, f, dst, tmp, nullptr,
                                active, cls, nullptr);
  const int m = p->m[l];
  const size_t bytes = npts(p->dim, m) * sizeof(double);
  if (nsweeps == 0) {
    if (src == dst) return hipSuccess;
    if (!src) return launch_fill_zero(dst, bytes, p->stream);
    return launch_copy(src, dst, bytes, active, p->stream);
  }
  if (nsweeps >= 2 && !tmp) return hipErrorInvalidValue;
  const double h = 1.0 / double(m + 1);
  const double *in = src;
  const int parts = p->dim == 3 ? 2 : 1;
  for (int k = 1; k <= nsweeps; ++k) {
    double *out = ((nsweeps - k) % 2 == 1) ? tmp : dst;
    for (int part = 0; part < parts; ++part) {
      // algorithmic bytes of a sweep: old values and f read, result written
      // once (3D: half of them in each part)
      ProfScope ps(p, cls, (double)bytes * 3.0 / parts);
      hipError_t e = launch_mc_sweep(p->dim, m, in, f, out, backward ? 1 : 0, h * h, active,
                                     p->stream, part);
      if (e != hipSuccess) return e;
    }
    in = out;
  }
  return hipSuccess;
}

hipError_t var_restrict(gmg_plan *p, int l, const double *u, const double *f, double *fc,
                        const int *active, int cls) {
  if (!(p->cfg.flags & GMG_FE_TRANSFER)) return restrict_level<double>(p, l, u, f, fc, active, cls);
  const int m = p->m[l];
  const double h = 1.0 / double(m + 1);
  ProfScope ps(p, cls, (double)npts(p->dim, m) * sizeof(double) * (u ? 2 : 1) +
                           (double)npts(p->dim, p->m[l + 1]) * sizeof(double));
  return launch_restrict_fe(p->dim, m, p->m[l + 1], u, f, fc, 1.0 / (h * h), active, p->stream);
}

hipError_t var_prolong(gmg_plan *p, int l, const double *in, const double *ec, double *out,
                       const int *active) {
  const int m = p->m[l];
  ProfScope ps(p, PC_MISC, (double)npts(p->dim, m) * sizeof(double) * (in ? 2 : 1) +
                               (double)npts(p->dim, p->m[l + 1]) * sizeof(double));
  if (p->cfg.flags & GMG_FE_TRANSFER)
    return launch_prolong_fe(p->dim, m, p->m[l + 1], in, ec, out, active, p->stream);
  return launch_prolong_add<double>(p->dim, m, p->m[l + 1], in, ec, out, active, p->stream);
}

hipError_t var_coarsest(gmg_plan *p, const double *f, double *u, const int *active) {
  ProfScope ps(p, PC_BOTTOM, 2.0 * sizeof(double));
  return launch_coarsest(p->dim, f, u, (p->cfg.flags & GMG_COARSE_RELAX) ? 1 : 0,
                         p->cfg.smoother == GMG_SMOOTH_WJ ? 1 : 0, p->cfg.nu1, p->cfg.omega,
                         active, p->stream);
}

// One V-cycle (Algorithm 1) on levels s .. L-1 of a variant plan: start value
// u_in (NULL = zero), right-hand side f_s, result u_out (may equal u_in).
// norm_partials (s = 0 only): residual norm of u_in and the stop test first.
hipError_t var_cycle(gmg_plan *p, int s, const double *u_in, const double *f_s, double *u_out,
                     double *norm_partials, const int *active) {
  LevelSet<double> &S = p->d;
  const int L = p->L;
  const bool bwd = !(p->cfg.flags & GMG_POST_FORWARD);
  const int nu1 = p->cfg.nu1, nu2 = p->cfg.nu2;
  hipError_t e;
  if (norm_partials) {
    const int m = p->m[s];
    ResidArgs<double> r{};
    r.u = u_in;
    r.f = f_s;
    r.partials = norm_partials;
    r.active = active;
    r.m = m;
    r.nblocks = residual_blocks(p->dim, m);
    const double h = 1.0 / double(m + 1);
    r.inv_h2 = 1.0 / (h * h);
    {
      // the stop test's residual norm is timed with the stop test
      ProfScope ps(p, PC_FIN, (double)npts(p->dim, m) * sizeof(double) * 2);
      e = launch_residual<double>(p->dim, r, p->stream);
      if (e != hipSuccess) return e;
    }
    ProfScope ps(p, PC_FIN, 0.0);
    e = launch_finalize(norm_partials, r.nblocks, p->state, p->stream);
    if (e != hipSuccess) return e;
  }
  if (s == L - 1) return var_coarsest(p, f_s, u_out, active);
  for (int l = s; l <= L - 2; ++l) {
    const double *f = l == s ? f_s : S.f[l];
    e = var_smooth(p, l, nu1, false, l == s ? u_in : nullptr, f, S.w[l], S.t[l], active,
                   l == 0 ? PC_PRE0 : PC_PRE_C);
    if (e != hipSuccess) return e;
    e = var_restrict(p, l, S.w[l], f, S.f[l + 1], active, l == 0 ? PC_RES0 : PC_RES_C);
    if (e != hipSuccess) return e;
  }
  e = var_coarsest(p, S.f[L - 1], S.u[L - 1], active);
  if (e != hipSuccess) return e;
  for (int l = L - 2; l >= s; --l) {
    const double *f = l == s ? f_s : S.f[l];
    e = var_prolong(p, l, S.w[l], S.u[l + 1], S.w[l], active);
    if (e != hipSuccess) return e;
    e = var_smooth(p, l, nu2, bwd, S.w[l], f, l == s ? u_out : S.u[l], S.t[l], active,
                   l == 0 ? PC_POST0 : PC_POST_C);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Full multigrid (Algorithm 2) of a variant plan.
hipError_t var_fmg(gmg_plan *p, double *u, const double *f) {
  LevelSet<double> &S = p->d;
  const int L = p->L;
  hipError_t e;
  if (L == 1) return var_coarsest(p, f, u, nullptr);
  for (int l = 0; l <= L - 2; ++l) {
    e = var_restrict(p, l, nullptr, l == 0 ? f : S.f[l], S.f[l + 1], nullptr, PC_MISC);
    if (e != hipSuccess) return e;
  }
  e = var_coarsest(p, S.f[L - 1], S.u[L - 1], nullptr);
  if (e != hipSuccess) return e;
  for (int l = L - 2; l >= 0; --l) {
    double *ul = l == 0 ? u : S.u[l];
    e = var_prolong(p, l, nullptr, S.u[l + 1], ul, nullptr);
    if (e != hipSuccess) return e;
    e = var_cycle(p, l, ul, l == 0 ? f : S.f[l], ul, nullptr, nullptr);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
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
        if (p.need_tmp || p.cross || p.cross32) Tt[0] = take(cur, n);
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

// z-chunk giving a few workgroups per compute unit for a tile shape
int auto_tz(int dim, int m, int st, const PassTile &t) {
  const PassGeom g0 = pass_geometry(dim, m, st, t, m);
  const int xy = g0.ntx * g0.nty;
  const int ntz = std::max(1, (3 * 256 + xy - 1) / xy);
  int tzv = (m + ntz - 1) / ntz;
  return std::max(tzv, std::min(m, 8));
}

// Default pass choice for a level and role, from measurements on MI355X
// (single-sweep passes win on small grids and for the prolongation pass;
// two fused sweeps win for plain smoothing of large grids).
PassChoice choice_for(const gmg_config &cfg, int dim, int m, int role, int smax_cap) {
  PassChoice c;
  const bool wj = cfg.smoother == GMG_SMOOTH_WJ;
  const bool big = dim == 3 ? m >= 255 : m >= 2047;
  c.smax = std::min(smax_cap, (big && role == 0) ? 2 : 1);
  if (dim == 2) c.smax = std::min(smax_cap, 2);
  for (int st = 1; st <= 4; ++st) {
    const int nv = pass_variant_count(dim, st, wj ? 1 : 0);
    if (nv == 0) continue;
    int v = 0, tz = 0;
    if (dim == 3 && !wj) {
      if (m <= 127) {
        v = st == 2 ? 2 : 1;  // (66,14,512) / (36,24,256)
        tz = m <= 63 ? 2 : 4;
      } else if (m <= 255) {
        v = 1;
        tz = 32;
      } else {
        v = 0;
        tz = st == 4 ? 0 : 32;
      }
    } else {
      v = (m >= 255 || nv == 1) ? 0 : 1;
    }
    // the three-stage pass: a tile that runs the form with the restriction
    // folded in (odd row count)
    if (st == 3 && dim == 3 && !wj) v = 5;
    v = std::min(v, nv - 1);
    c.var[st] = v;
    const PassTile t = pass_variant(dim, st, wj ? 1 : 0, v);
    c.tz[st] = tz > 0 ? std::min(tz, m) : auto_tz(dim, m, st, t);
  }
  return c;
}

PassChoice default_choice(const gmg_plan &p, int l, int role) {
  return choice_for(p.cfg, p.dim, p.m[l], role, p.smax_cap);
}

void default_tiles(gmg_plan &p) {
  p.ch.resize(p.L);
  for (int l = 0; l < p.L; ++l)
    for (int role = 0; role < 3; ++role) p.ch[l][role] = default_choice(p, l, role);
}

gmg_status validate_cfg(const gmg_config *c) {
  if (!c) return GMG_ERR_INVALID_ARG;
  if (c->dim != 2 && c->dim != 3) return GMG_ERR_INVALID_ARG;
  if (c->levels < 1 || c->levels > kMaxLevels) return GMG_ERR_INVALID_ARG;
  if (c->dim == 3 && c->levels > 10) return GMG_ERR_INVALID_ARG;  // 1023^3 max (int32 index)
  if (c->nu1 < 0 || c->nu2 < 0 || c->nu1 + c->nu2 < 1 || c->nu1 > 8 || c->nu2 > 8)
    return GMG_ERR_INVALID_ARG;
  if (c->smoother != GMG_SMOOTH_RBGS && c->smoother != GMG_SMOOTH_WJ &&
      c->smoother != GMG_SMOOTH_MCGS)
    return GMG_ERR_INVALID_ARG;
  if (c->smoother == GMG_SMOOTH_WJ && !(c->omega >= 0.0 && c->omega <= 1.0))
    return GMG_ERR_INVALID_ARG;
  if (c->precision != GMG_FP64 && c->precision != GMG_MIXED_FP32_IR) return GMG_ERR_INVALID_ARG;
  if (c->inner_cycles < 1 || c->inner_cycles > 16) return GMG_ERR_INVALID_ARG;
  return GMG_OK;
}

// Weighted-Jacobi weight for a problem of dimension dim: the caller's, or
// 2d / (2d + 1) when the caller left it 0 (Remark 1's choice per dimension;
// a batch can hold both dimensions)
double wj_omega(const gmg_plan *p, int dim) {
  return p->omega_user == 0.0 ? (dim == 3 ? 6.0 / 7.0 : 0.8) : p->omega_user;
}

gmg_status init_plan_shape(gmg_plan &p, const gmg_config *cfg) {
  p.cfg = *cfg;
  p.omega_user = cfg->omega;
  if (p.cfg.smoother == GMG_SMOOTH_WJ) p.cfg.omega = wj_omega(&p, cfg->dim);
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
  // the paper's variant has no bottom kernel: only the one-node level is
  // handled separately
  if (cfg_variant(p.cfg)) p.B = std::max(1, p.L - 1);
  p.smax_cap = (cfg->flags & GMG_NO_TEMPORAL_BLOCKING) ? 1 : 2;
  // chained passes need a scratch array whenever a level may run more than
  // one pass (any choice of sweeps per pass, so tuning never changes layout)
  p.need_tmp = std::max(cfg->nu1, cfg->nu2) >= 2;
  const bool cross_ok = cfg->smoother == GMG_SMOOTH_RBGS && !cfg_variant(p.cfg) &&
                        cfg->nu1 == 1 && cfg->nu2 == 1 && p.L >= 2 &&
                        !(cfg->flags & (GMG_POST_FORWARD | GMG_NO_CROSS_CYCLE));
  p.cross = cross_ok && cfg->precision == GMG_FP64;
  p.cross32 = cross_ok && cfg->precision == GMG_MIXED_FP32_IR;
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

// ------------------------------------------------------------------ autotuner
// Times every candidate pass choice (sweeps per pass x tile shape x z-chunk)
// of every level and role on the plan's own buffers with hipEvents and keeps
// the fastest.  Results are bitwise independent of the choice, so tuning only
// changes speed.  A process-wide cache (and, when GMG_TUNE_CACHE names a
// file, an on-disk one) is keyed by device architecture and problem shape.
std::map<std::string, PassChoice> &tune_cache() {
  static std::map<std::string, PassChoice> c;
  return c;
}

std::string arch_name() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return "unknown";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

// z-chunks the tuner tries for a tile on a level of side m: powers of two,
// the chunks that split the planes into 2, 3, 5, 6 or 12 nearly equal runs,
// and the automatic choice; duplicates dropped.  The counter table of the
// microbench (--traffic-table) uses the same rule.
std::vector<int> tune_z_chunks(int dim, int m, int stages, const PassTile &t) {
  std::vector<int> v;
  for (int c : {4, 8, 16, 32, 64}) v.push_back(std::min(c, m));
  for (int k : {2, 3, 5, 6, 12}) v.push_back(std::max(1, (m + k - 1) / k));
  v.push_back(auto_tz(dim, m, stages, t));
  std::sort(v.begin(), v.end());
  v.erase(std::unique(v.begin(), v.end()), v.end());
  return v;
}

// The key names the device, the level's shape and role, the options that
// change which passes run, and a hash of the tile tables, so an entry written
// for another build's tables is never applied.
std::string tune_key(const gmg_plan &p, int l, int role, size_t elem) {
  char buf[192];
  std::snprintf(buf, sizeof(buf), "%s|d%d|m%d|f%d|%s|nu%d|r%d|cap%d|fr%d|z4|t%08x",
                arch_name().c_str(), p.dim, p.m[l], (int)(elem * 8),
                p.cfg.smoother == GMG_SMOOTH_WJ ? "wj" : "rbgs", role == 0 ? p.cfg.nu1 : p.cfg.nu2,
                role, p.smax_cap, (p.cfg.flags & GMG_NO_FUSED_RESTRICT) ? 0 : 1,
                (unsigned)tile_table_hash());
  return buf;
}

// Whether a pass choice can be launched on a level of side m: sweeps per
// pass within the plan's cap, every stage count's tile index inside the tile
// table, a non-negative z-chunk, and no pass with more workgroups than the
// norm-partials buffer holds.  (The folded restriction re-checks its own,
// larger geometry and LDS before every use.)
bool choice_ok(int dim, int m, int smax_cap, bool wj, const PassChoice &c) {
  if (c.smax < 1 || c.smax > smax_cap || (c.fuse != 0 && c.fuse != 1)) return false;
  for (int st = 1; st <= 4; ++st) {
    const int nv = pass_variant_count(dim, st, wj ? 1 : 0);
    if (nv == 0) continue;
    if (c.var[st] < 0 || c.var[st] >= nv || c.tz[st] < 0 || c.sw[st] < 0) return false;
    const PassTile t = pass_variant(dim, st, wj ? 1 : 0, c.var[st]);
    if (pass_geometry(dim, m, st, t, c.tz[st]).nblocks > kMaxPartials) return false;
  }
  return true;
}

// One line of the on-disk cache: key, sweeps per pass, stage count, tile
// index, z-chunk, fold flag.  False for a line that does not parse.
bool parse_cache_line(const char *line, std::string &key, PassChoice &c, int &st) {
  char kb[256];
  int v = 0, tz = 0, fz = 1, sw = 0;
  st = 0;
  if (std::sscanf(line,
                  "{\"key\": \"%255[^\"]\", \"smax\": %d, \"stages\": %d, \"var\": %d, \"tz\": %d, "
                  "\"fuse\": %d, \"sw\": %d",
                  kb, &c.smax, &st, &v, &tz, &fz, &sw) < 6 || st < 1 || st > 4)
    return false;
  key = kb;
  c.var[st] = v;
  c.tz[st] = tz;
  c.sw[st] = sw;
  c.fuse = fz;
  return true;
}

// The level shape a key describes (dimension, side, Jacobi or not, sweep cap)
// and whether the key carries the tile-table hash compiled into this library.
bool key_shape(const std::string &key, int &dim, int &m, bool &wj, int &cap) {
  const size_t bar = key.find('|');
  if (bar == std::string::npos) return false;
  char smooth[16] = {0};
  int f = 0, nu = 0, r = 0, fr = 0, z = 0;
  unsigned th = 0;
  if (std::sscanf(key.c_str() + bar, "|d%d|m%d|f%d|%15[a-z]|nu%d|r%d|cap%d|fr%d|z%d|t%x", &dim, &m,
                  &f, smooth, &nu, &r, &cap, &fr, &z, &th) != 10)
    return false;
  wj = std::strcmp(smooth, "wj") == 0;
  return th == tile_table_hash() && (dim == 2 || dim == 3) && m >= 1 && cap >= 1;
}

// Loads GMG_TUNE_CACHE once per process.  Lines that do not parse, name
// another build's tile tables or a choice that cannot run are skipped (that
// level is tuned again).
void tune_cache_load() {
  static bool loaded = false;
  if (loaded) return;
  loaded = true;
  const char *path = std::getenv("GMG_TUNE_CACHE");
  if (!path || !*path) return;
  FILE *fh = std::fopen(path, "r");
  if (!fh) return;
  char line[512];
  while (std::fgets(line, sizeof(line), fh)) {
    std::string key;
    PassChoice c;
    int st = 0, dim = 0, m = 0, cap = 0;
    bool wj = false;
    if (!parse_cache_line(line, key, c, st) || !key_shape(key, dim, m, wj, cap)) continue;
    auto it = tune_cache().find(key);
    PassChoice &d = it == tune_cache().end() ? (tune_cache()[key] = c) : it->second;
    d.smax = c.smax;
    d.var[st] = c.var[st];
    d.tz[st] = c.tz[st];
    d.sw[st] = c.sw[st];
    d.fuse = c.fuse;
  }
  std::fclose(fh);
}

void tune_cache_store(const std::string &key, const PassChoice &c, int st, double us) {
  tune_cache()[key] = c;
  const char *path = std::getenv("GMG_TUNE_CACHE");
  if (!path || !*path) return;
  FILE *fh = std::fopen(path, "a");
  if (!fh) return;
  std::fprintf(fh,
               "{\"key\": \"%s\", \"smax\": %d, \"stages\": %d, \"var\": %d, \"tz\": %d, "
               "\"fuse\": %d, \"sw\": %d, \"us\": %.2f}\n",
               key.c_str(), c.smax, st, c.var[st], c.tz[st], c.fuse, c.sw[st], us);
  std::fclose(fh);
}

// Mean time in microseconds of reps launches of run() after one warm-up.
template <typename F>
hipError_t time_runs(gmg_plan *p, hipEvent_t e0, hipEvent_t e1, int reps, F &&run, double &us) {
  hipError_t err = run();
  if (err == hipSuccess) err = hipEventRecord(e0, p->stream);
  for (int r = 0; r < reps && err == hipSuccess; ++r) err = run();
  if (err == hipSuccess) err = hipEventRecord(e1, p->stream);
  if (err == hipSuccess) err = hipEventSynchronize(e1);
  float ms = 0.f;
  if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
  us = 1e3 * ms / reps;
  return err;
}

// One timed candidate of the autotuner.
struct Cand {
  PassChoice c;
  int st = 0;
  double us = 1e30;
};

// Sweeps time each candidate over a few launches only; the fastest few of a
// sweep are timed again over three times as many launches (in the same
// order), so timing noise does not decide between near-equal candidates.
// Returns the fastest of them; run() launches with p->ch[l][role].
template <typename F>
hipError_t refine_best(gmg_plan *p, int l, int role, std::vector<Cand> &cands, hipEvent_t e0,
                       hipEvent_t e1, int reps, F &&run, Cand &best) {
  std::sort(cands.begin(), cands.end(), [](const Cand &a, const Cand &b) { return a.us < b.us; });
  if (cands.size() > 4) cands.resize(4);
  best = Cand();
  for (Cand &c : cands) {
    p->ch[l][role] = c.c;
    double us = 0.0;
    hipError_t err = time_runs(p, e0, e1, 3 * reps, run, us);
    if (err != hipSuccess) return err;
    c.us = us;
    if (us < best.us) best = c;
  }
  return hipSuccess;
}

// fc (pre-smoothing): the next coarser level's right-hand side.  Each
// candidate is timed together with the restriction, fused into the last
// pass where the tile allows it and as a kernel of its own, and the faster
// form is kept.
template <typename T>
hipError_t tune_role(gmg_plan *p, int l, int role, const T *src, const T *ec, const T *f, T *dst,
                     T *tmp, double *partials, size_t elem, T *fc = nullptr) {
  const int nu = role == 0 ? p->cfg.nu1 : p->cfg.nu2;
  if (nu == 0) return hipSuccess;
  const std::string key = tune_key(*p, l, role, elem);
  const bool wj = p->cfg.smoother == GMG_SMOOTH_WJ;
  auto it = tune_cache().find(key);
  if (it != tune_cache().end()) {
    if (choice_ok(p->dim, p->m[l], p->smax_cap, wj, it->second)) {
      p->ch[l][role] = it->second;
      return hipSuccess;
    }
    tune_cache().erase(it);  // unusable cached choice: tune this level again
  }
  const int m = p->m[l];
  hipEvent_t e0, e1;
  hipError_t err = hipEventCreate(&e0);
  if (err != hipSuccess) return err;
  err = hipEventCreate(&e1);
  if (err != hipSuccess) return err;
  const size_t N = npts(p->dim, m);
  const int reps = N > (1u << 24) ? 2 : (N > (1u << 20) ? 4 : 10);
  const PassChoice base = p->ch[l][role];
  // exactly the cycle's launches for this step (with p->ch[l][role]): with a
  // folded restriction the solve's stop test follows as a kernel of its own,
  // otherwise it runs in workgroup 0 of the restriction
  auto run = [&]() -> hipError_t {
    bool fused = false;
    int nparts = 0;
    hipError_t e2 = smooth_chain<T>(p, l, nu, role == 1, src, ec, f, dst, tmp, partials, nullptr,
                                    PC_MISC, &nparts, fc, &fused);
    if (e2 != hipSuccess || !fc) return e2;
    if (fused)
      return partials ? launch_finalize(partials, nparts, p->state, p->stream) : hipSuccess;
    return restrict_level<T>(p, l, dst, f, fc, nullptr, PC_MISC, partials, nparts);
  };
  // candidates with and without the folded restriction
  std::vector<Cand> cands[2];
  for (int sm = 1; sm <= std::min(p->smax_cap, nu); ++sm) {
    const int st = stages_of(p, sm);
    const int nv = pass_variant_count(p->dim, st, wj ? 1 : 0);
    for (int v = 0; v < nv; ++v) {
      const PassTile t = pass_variant(p->dim, st, wj ? 1 : 0, v);
      const std::vector<int> tzs = tune_z_chunks(p->dim, m, st, t);
      for (const int tzv : tzs) {
        if (pass_geometry(p->dim, m, st, t, tzv).nblocks > kMaxPartials) continue;
        for (int fz = (fc ? 1 : 0); fz >= 0; --fz) {
          PassChoice c = base;
          c.smax = sm;
          c.var[st] = v;
          c.tz[st] = tzv;
          c.fuse = fz;
          p->ch[l][role] = c;
          if (fz && !can_fuse_restrict(p, l, nu, elem)) continue;
          double us = 0.0;
          err = time_runs(p, e0, e1, reps, run, us);
          if (err != hipSuccess) break;
          cands[fz].push_back(Cand{c, st, us});
        }
        if (err != hipSuccess) break;
      }
      if (err != hipSuccess) break;
    }
    if (err != hipSuccess) break;
  }
  PassChoice best[2] = {base, base};
  double best_us[2] = {1e30, 1e30};
  int best_st[2] = {stages_of(p, std::min(base.smax, nu)), stages_of(p, std::min(base.smax, nu))};
  for (int fz = 0; fz < 2 && err == hipSuccess; ++fz) {
    Cand b;
    err = refine_best(p, l, role, cands[fz], e0, e1, reps, run, b);
    if (b.us < 1e30) {
      best[fz] = b.c;
      best_us[fz] = b.us;
      best_st[fz] = b.st;
    }
  }
  // the folded restriction enlarges the pass's halo and LDS: keep the plain
  // pass and the separate restriction unless folding is clearly faster
  // (timing noise of a few percent would otherwise flip the choice)
  const int pick = best_us[1] < 0.97 * best_us[0] ? 1 : 0;
  p->ch[l][role] = best[pick];
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err == hipSuccess) tune_cache_store(key, best[pick], best_st[pick], best_us[pick]);
  return err;
}

// The cross-cycle pass (role 2 of level 0) is tuned like the other roles:
// every three-stage tile and z-chunk, with the restriction folded in where
// the tile allows it and as a kernel of its own, each timed together with
// the step that follows it in the solve (the stop test as a kernel of its
// own, or the restriction whose workgroup 0 runs it).
template <typename T>
hipError_t tune_cross(gmg_plan *p, const T *w, const T *ec, const T *f, T *wn, T *fc) {
  const std::string key = tune_key(*p, 0, 2, sizeof(T));
  // FP64 solves: with the norm and the stop test after it; FP32 inner
  // cycles: neither
  double *parts = sizeof(T) == 8 ? p->partials : nullptr;
  auto it = tune_cache().find(key);
  if (it != tune_cache().end()) {
    if (choice_ok(p->dim, p->m[0], p->smax_cap, false, it->second)) {
      p->ch[0][2] = it->second;
      return hipSuccess;
    }
    tune_cache().erase(it);
  }
  const int m = p->m[0];
  hipEvent_t e0, e1;
  hipError_t err = hipEventCreate(&e0);
  if (err != hipSuccess) return err;
  err = hipEventCreate(&e1);
  if (err != hipSuccess) return err;
  const size_t N = npts(p->dim, m);
  const int reps = N > (1u << 24) ? 2 : (N > (1u << 20) ? 4 : 10);
  const PassChoice base = p->ch[0][2];
  // the pass and the step after it in the solve, with p->ch[0][2]
  auto run = [&]() -> hipError_t {
    bool fused = false;
    int nparts = 0;
    hipError_t e2 = cross_pass<T>(p, w, ec, f, wn, parts, nullptr, fc, &fused, &nparts);
    if (e2 != hipSuccess) return e2;
    if (fused) return parts ? launch_finalize(parts, nparts, p->state, p->stream) : hipSuccess;
    return restrict_level<T>(p, 0, wn, f, fc, nullptr, PC_MISC, parts, parts ? nparts : 0);
  };
  std::vector<Cand> cands[2];
  const int nv = pass_variant_count(p->dim, 3, 0);
  for (int v = 0; v < nv && err == hipSuccess; ++v) {
    const PassTile t = pass_variant(p->dim, 3, 0, v);
    for (const int tzv : tune_z_chunks(p->dim, m, 3, t)) {
      if (pass_geometry(p->dim, m, 3, t, tzv).nblocks > kMaxPartials) continue;
      for (int fz = 1; fz >= 0 && err == hipSuccess; --fz) {
        PassChoice c = base;
        c.var[3] = v;
        c.tz[3] = tzv;
        c.fuse = fz;
        p->ch[0][2] = c;
        // each tile runs one form or both (folded: odd row count)
        if (fz ? !can_fuse_cross(p, sizeof(T))
               : !rb_pass_fits(p->dim, 3, v, F_PROLONG, sizeof(T)))
          continue;
        double us = 0.0;
        err = time_runs(p, e0, e1, reps, run, us);
        if (err != hipSuccess) break;
        cands[fz].push_back(Cand{c, 3, us});
      }
      if (err != hipSuccess) break;
    }
  }
  PassChoice best[2] = {base, base};
  double best_us[2] = {1e30, 1e30};
  for (int fz = 0; fz < 2 && err == hipSuccess; ++fz) {
    Cand b;
    err = refine_best(p, 0, 2, cands[fz], e0, e1, reps, run, b);
    if (b.us < 1e30) {
      best[fz] = b.c;
      best_us[fz] = b.us;
    }
  }
  const int pick = best_us[1] < 0.97 * best_us[0] ? 1 : 0;
  p->ch[0][2] = best[pick];
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err == hipSuccess && best_us[pick] < 1e30)
    tune_cache_store(key, best[pick], 3, best_us[pick]);
  return err;
}

// Tune every pass-kernel level of the plan in precision T.  src0/f0: level-0
// start value and right-hand side (read only); the workspace arrays are used
// as outputs and scratch.
template <typename T>
hipError_t tune_plan(gmg_plan *p, const T *src0, const T *f0, double *partials0) {
  tune_cache_load();
  LevelSet<T> &S = levels_of<T>(p);
  const bool prof = p->profile;
  p->profile = false;
  // the timed level-0 steps update the solve state like a solve does; give
  // it defined contents (the solve initialises it again afterwards)
  hipError_t e = (partials0 || p->cross) ? launch_state_init(p->state, 1, 1.0, -1.0, p->stream)
                                         : hipSuccess;
  if (e != hipSuccess) {
    p->profile = prof;
    return e;
  }
  for (int l = 0; l < p->B && l + 1 < p->L && e == hipSuccess; ++l) {
    const T *f = l == 0 ? f0 : S.f[l];
    // descent: level 0 reads the start value (and reports its residual norm)
    e = tune_role<T>(p, l, 0, l == 0 ? src0 : nullptr, nullptr, f, S.w[l], S.t[l],
                     l == 0 ? partials0 : nullptr, sizeof(T), S.f[l + 1]);
    if (e != hipSuccess) break;
    // ascent with the fused prolongation from level l+1
    const T *src = l == 0 ? (src0 ? src0 : S.w[0]) : S.w[l];
    T *dst = l == 0 ? (src0 ? S.w[0] : S.u[0]) : S.u[l];
    e = tune_role<T>(p, l, 1, src, S.u[l + 1], f, dst, S.t[l], nullptr, sizeof(T));
    if (e == hipSuccess && l == 0 && (sizeof(T) == 8 ? p->cross : p->cross32))
      e = tune_cross<T>(p, S.w[0], S.u[1], f, S.t[0], S.f[1]);
  }
  p->profile = prof;
  p->tuned = true;
  return e;
}

// ------------------------------------------------------------------ batch
// Problems are grouped by dimension and level size: every kernel launch of a
// batched cycle covers all problems that have a level of that size (the
// table entry of a problem is its blockIdx.y), the bottom levels of all
// problems run in one launch with one workgroup per problem, and each
// problem keeps its own solve state, so converged problems drop out (their
// workgroups return at once) while the others continue.
struct BatchBuilder {
  gmg_plan *p;
  Batch *b;
  char *ws;  // workspace base (nullptr while sizing)
  size_t cur = 0;
  size_t take_bytes(size_t n) { return take(cur, n); }
  template <typename E>
  size_t push(const E &e) {
    const size_t off = b->host_tbl.size();
    b->host_tbl.resize(off + sizeof(E));
    std::memcpy(b->host_tbl.data() + off, &e, sizeof(E));
    return off;
  }
  void align_tbl() { b->host_tbl.resize(align_up(b->host_tbl.size())); }
};

int bottom_first_level(int dim, int L, int smoother) {
  const int mb = bottom_side_max(dim, smoother, sizeof(double));
  for (int l = 1; l < L; ++l)
    if ((1 << (L - l)) - 1 <= mb) return l;
  return L - 1;
}

// One chain of passes (nu sweeps) for a set of entries that share a level
// size.  Per entry: src/ec/f/dst/tmp pointers, which of them are the
// caller's arrays (patched per call), partial-sum slice and state.
struct ChainEnt {
  int q, level;
  double *src, *ec, *f, *dst, *tmp;
  bool src_user, f_user, dst_user;
  double *partials;
  double *fc = nullptr;  // the coarse right-hand side, when the last pass restricts
};

PassChoice batch_choice(const gmg_plan *p, const Batch *b, int dim, int m, int role);

// Whether the pre-smoothing chains of the level size (dim, m) whose first
// pass has first_flags end in a pass that also restricts, as single
// problems do: red-black, the choice asks for it, the tile runs that form
// and its workgroups fit a problem's partial-sum slice.
bool batch_fold(const gmg_plan *p, const Batch *b, int dim, int m, int nu, int first_flags) {
  if (p->cfg.smoother != GMG_SMOOTH_RBGS || (p->cfg.flags & GMG_NO_FUSED_RESTRICT) || nu < 1)
    return false;
  // the sizing build keeps every restriction entry: folding only removes
  // entries, so its table bounds that of any choice
  if (b->worst) return false;
  const PassChoice c = batch_choice(p, b, dim, m, 0);
  if (!c.fuse) return false;
  int K = 0;
  const int st = 2 * last_pass_sweeps(nu, c.smax, &K);
  const PassTile t = pass_variant(dim, st, 0, c.var[st]);
  if (pass_geometry(dim, m, st, t, c.tz[st], true).nblocks > kMaxPartials) return false;
  return rb_pass_fits(dim, st, c.var[st], F_RESTRICT | (K == 1 ? first_flags : 0), sizeof(double));
}

void build_chain(BatchBuilder &bb, int dim, int m, int role, int nu, int first_flags, bool backward,
                 const std::vector<ChainEnt> &ents, int cls, bool fold = false) {
  gmg_plan *p = bb.p;
  Batch *b = bb.b;
  if (ents.empty() || nu == 0) return;
  const bool wj = p->cfg.smoother == GMG_SMOOTH_WJ;
  const PassChoice c = batch_choice(p, b, dim, m, role);
  const int K = (nu + c.smax - 1) / c.smax;
  int left = nu;
  const double h = 1.0 / double(m + 1);
  const int mc = (m - 1) / 2;
  for (int k = 1; k <= K; ++k) {
    const int sw = std::min(c.smax, left - (K - k));
    const int st = wj ? sw : 2 * sw;
    const int v = c.var[st];
    const PassTile t = pass_variant(dim, st, wj ? 1 : 0, v);
    const bool rst = fold && k == K;  // the last pass restricts onto f_c
    const PassGeom g = pass_geometry(dim, m, st, t, c.tz[st], rst);
    int flags = backward ? F_BLACK_FIRST : 0;
    if (k == 1) flags |= first_flags;
    if (rst) flags |= F_RESTRICT;
    BOp op;
    op.kind = BO_PASS;
    op.dim = dim;
    op.stages = st;
    op.flags = flags;
    op.variant = v;
    op.wj = wj ? 1 : 0;
    op.nent = (int)ents.size();
    op.cls = cls;
    bb.align_tbl();
    op.tbl_off = b->host_tbl.size();
    for (const ChainEnt &e : ents) {
      // pass k reads buf_{k-1} and writes buf_k; intermediates alternate
      // between tmp and dst so the last pass lands in dst
      auto out_of = [&](int j) -> double * { return ((K - j) % 2 == 1) ? e.tmp : e.dst; };
      auto out_user = [&](int j) -> bool { return ((K - j) % 2 == 1) ? false : e.dst_user; };
      PassArgs<double> a{};
      a.u_in = k == 1 ? e.src : out_of(k - 1);
      a.f = e.f;
      a.u_out = out_of(k);
      a.e_c = k == 1 ? e.ec : nullptr;
      a.f_c = rst ? e.fc : nullptr;
      a.partials = (k == 1 && (first_flags & F_NORM_IN)) ? e.partials : nullptr;
      a.active = &b->pb[e.q].st->active;
      a.m = m;
      a.mc = mc;
      a.ntx = g.ntx;
      a.nty = g.nty;
      a.tz = g.tz;
      a.nblocks = g.nblocks;
      a.h2 = h * h;
      a.inv_h2 = 1.0 / (h * h);
      a.omega = wj_omega(p, dim);
      const size_t off = bb.push(a);
      const bool in_user = k == 1 ? e.src_user : out_user(k - 1);
      if (in_user) b->patches.push_back({off + offsetof(PassArgs<double>, u_in), e.q, 0});
      if (e.f_user) b->patches.push_back({off + offsetof(PassArgs<double>, f), e.q, 1});
      if (out_user(k)) b->patches.push_back({off + offsetof(PassArgs<double>, u_out), e.q, 0});
      op.bytes += (double)npts(dim, m) * 8.0 * ((k == 1 && (first_flags & F_ZERO_IN)) ? 2 : 3);
      if (rst) op.bytes += (double)npts(dim, mc) * 8.0;
    }
    b->ops.push_back(op);
    left -= sw;
  }
}

// In a batch, the problems that have a level of one size share each launch
// of that level, so the workgroups come from the problem count as well as
// from the chunks.  A z-chunk chosen for one problem alone (short chunks keep
// 256 compute units busy on a small grid) is widened to the longest tuner
// candidate that still gives the launch kBatchMinBlocks workgroups: longer
// chunks recompute fewer halo planes.  Results do not depend on the chunk.
// (256-problem batch: 52.9 ms unwidened; 45.2, 39.9, 37.6, 39.4 and 44.5 ms
// with 256, 512, 1024, 1536 and 4096 as the floor.)
constexpr int kBatchMinBlocks = 1024;

void batch_widen_tz(const gmg_plan *p, PassChoice &c, int dim, int m, int count) {
  const int wj = p->cfg.smoother == GMG_SMOOTH_WJ ? 1 : 0;
  for (int st = 1; st <= 4; ++st) {
    const int nv = pass_variant_count(dim, st, wj);
    if (nv == 0 || c.var[st] < 0 || c.var[st] >= nv) continue;
    const PassTile t = pass_variant(dim, st, wj, c.var[st]);
    int best = c.tz[st] > 0 ? std::min(c.tz[st], m) : auto_tz(dim, m, st, t);
    std::vector<int> cand = tune_z_chunks(dim, m, st, t);
    cand.push_back(m);
    for (int tz : cand)
      if (tz > best && (long long)count * pass_geometry(dim, m, st, t, tz).nblocks >= kBatchMinBlocks)
        best = tz;
    c.tz[st] = best;
  }
}

PassChoice batch_choice(const gmg_plan *p, const Batch *b, int dim, int m, int role) {
  auto it = b->choice.find({dim, m, role});
  PassChoice c = it != b->choice.end() ? it->second : choice_for(p->cfg, dim, m, role, p->smax_cap);
  if (b->worst) c.smax = 1;
  auto n = b->shape_count.find({dim, m});
  if (n != b->shape_count.end() && n->second > 1) batch_widen_tz(p, c, dim, m, n->second);
  return c;
}

// Largest block count any first pass of this level size can have (the
// partial-sum slice of a problem is sized for it, so tuning keeps layouts).
int max_first_pass_blocks(const gmg_plan *p, int dim, int m) {
  const bool wj = p->cfg.smoother == GMG_SMOOTH_WJ;
  int mx = 1;
  for (int st = 1; st <= 4; ++st) {
    const int nv = pass_variant_count(dim, st, wj ? 1 : 0);
    for (int v = 0; v < nv; ++v) {
      const PassTile t = pass_variant(dim, st, wj ? 1 : 0, v);
      for (int tz : {1, 2, 4, 8, 16, 32, 64, 0}) {  // every z-chunk a choice may hold
        const int tzv = tz > 0 ? std::min(tz, m) : auto_tz(dim, m, st, t);
        for (bool rst : {false, true})  // (with the restriction folded in: larger halo)
          mx = std::max(mx, pass_geometry(dim, m, st, t, tzv, rst).nblocks);
      }
    }
  }
  return mx;
}

int first_pass_blocks(const gmg_plan *p, const Batch *b, int dim, int m, int nu) {
  const bool wj = p->cfg.smoother == GMG_SMOOTH_WJ;
  const PassChoice c = batch_choice(p, b, dim, m, 0);
  const int K = (nu + c.smax - 1) / c.smax;
  const int sw = std::min(c.smax, nu - (K - 1));
  const int st = wj ? sw : 2 * sw;
  const bool rst = K == 1 && batch_fold(p, b, dim, m, nu, F_NORM_IN);
  return pass_geometry(dim, m, st, pass_variant(dim, st, wj ? 1 : 0, c.var[st]), c.tz[st], rst)
      .nblocks;
}

// Lay out the workspace and build the launch list.  ws == nullptr: sizing
// only (the pointers recorded are offsets and never dereferenced).
size_t batch_build(gmg_plan *p, Batch *b, int n, const int *dims, const int *levels, char *ws) {
  BatchBuilder bb{p, b, ws};
  const int sm = p->cfg.smoother == GMG_SMOOTH_WJ ? 1 : 0;
  b->shape_count.clear();
  for (int q = 0; q < n; ++q) {
    const int B = bottom_first_level(dims[q], levels[q], sm);
    for (int l = 0; l < B; ++l) ++b->shape_count[{dims[q], (1 << (levels[q] - l)) - 1}];
  }
  b->pb.assign(n, BProblem());
  auto P = [&](size_t off) { return reinterpret_cast<double *>(ws + off); };
  const size_t st_off = bb.take_bytes(sizeof(SolveState) * (size_t)n);
  b->states = reinterpret_cast<SolveState *>(ws + st_off);
  for (int q = 0; q < n; ++q) {
    BProblem &pr = b->pb[q];
    pr.dim = dims[q];
    pr.L = levels[q];
    pr.B = bottom_first_level(pr.dim, pr.L, sm);
    pr.m.resize(pr.L);
    for (int l = 0; l < pr.L; ++l) pr.m[l] = (1 << (pr.L - l)) - 1;
    pr.st = b->states + q;
    pr.npart = first_pass_blocks(p, b, pr.dim, pr.m[0], p->cfg.nu1);
    pr.partials = P(bb.take_bytes(
        sizeof(double) * std::max(pr.npart, max_first_pass_blocks(p, pr.dim, pr.m[0]))));
    pr.f.assign(pr.L, nullptr);
    pr.w.assign(pr.L, nullptr);
    pr.u.assign(pr.L, nullptr);
    pr.t.assign(pr.L, nullptr);
    for (int l = 0; l <= pr.B; ++l) {
      const size_t nb = npts(pr.dim, pr.m[l]) * sizeof(double);
      if (l == 0) {
        pr.w[0] = P(bb.take_bytes(nb));
        if (p->need_tmp) pr.t[0] = P(bb.take_bytes(nb));
      } else if (l < pr.B) {
        pr.f[l] = P(bb.take_bytes(nb));
        pr.w[l] = P(bb.take_bytes(nb));
        pr.u[l] = P(bb.take_bytes(nb));
        if (p->need_tmp) pr.t[l] = P(bb.take_bytes(nb));
      } else {
        pr.f[l] = P(bb.take_bytes(nb));
        pr.u[l] = P(bb.take_bytes(nb));
      }
    }
  }
  const bool bwd = !(p->cfg.flags & GMG_POST_FORWARD);
  const int nu1 = p->cfg.nu1, nu2 = p->cfg.nu2;
  b->host_tbl.clear();
  b->ops.clear();
  b->patches.clear();
  for (int dim = 3; dim >= 2; --dim) {
    int Emax = 0;
    for (auto &pr : b->pb)
      if (pr.dim == dim) Emax = std::max(Emax, pr.L);
    for (int e = Emax; e >= 2; --e) {
      const int m = (1 << e) - 1;
      std::vector<ChainEnt> top, coarse;
      std::vector<int> tops;
      for (int q = 0; q < n; ++q) {
        BProblem &pr = b->pb[q];
        if (pr.dim != dim) continue;
        const int l = pr.L - e;
        if (l < 0 || l >= pr.B) continue;
        if (l == 0) {
          top.push_back({q, 0, nullptr, nullptr, nullptr, pr.w[0], pr.t[0], true, true, false,
                         pr.partials, pr.f[1]});
          tops.push_back(q);
        } else {
          coarse.push_back({q, l, nullptr, nullptr, pr.f[l], pr.w[l], pr.t[l], false, false,
                            false, nullptr, pr.f[l + 1]});
        }
      }
      const bool fold_top = batch_fold(p, b, dim, m, nu1, F_NORM_IN);
      const bool fold_coarse = batch_fold(p, b, dim, m, nu1, F_ZERO_IN);
      build_chain(bb, dim, m, 0, nu1, F_NORM_IN, false, top, PC_PRE0, fold_top);
      if (!tops.empty()) {
        BOp op;
        op.kind = BO_FIN;
        op.dim = dim;
        op.nent = (int)tops.size();
        op.cls = PC_FIN;
        bb.align_tbl();
        op.tbl_off = b->host_tbl.size();
        for (int q : tops) bb.push(FinEntry{b->pb[q].partials, b->pb[q].npart, b->pb[q].st});
        b->ops.push_back(op);
      }
      // the coarse descent takes the plane-marching passes as well: in a
      // batch the LDS-tile descent kernel is slower (256-problem batch 61
      // against 52 ms)
      build_chain(bb, dim, m, 0, nu1, F_ZERO_IN, false, coarse, PC_PRE_C, fold_coarse);
      // residual + restriction for every entry of this size whose last
      // pre-smoothing pass did not restrict
      std::vector<ChainEnt> all;
      if (!fold_top) all = top;
      if (!fold_coarse) all.insert(all.end(), coarse.begin(), coarse.end());
      if (!all.empty()) {
        BOp op;
        op.kind = BO_RESTRICT;
        op.dim = dim;
        op.nent = (int)all.size();
        op.cls = PC_RES_C;
        bb.align_tbl();
        op.tbl_off = b->host_tbl.size();
        const double h = 1.0 / double(m + 1);
        for (const ChainEnt &ce : all) {
          BProblem &pr = b->pb[ce.q];
          RestrictArgs<double> a{};
          a.u = pr.w[ce.level];
          a.f = ce.level == 0 ? nullptr : pr.f[ce.level];
          a.fc = pr.f[ce.level + 1];
          a.active = &pr.st->active;
          a.m = m;
          a.mc = (m - 1) / 2;
          a.inv_h2 = 1.0 / (h * h);
          const size_t off = bb.push(a);
          if (ce.level == 0) b->patches.push_back({off + offsetof(RestrictArgs<double>, f), ce.q, 1});
          op.bytes += (double)npts(dim, m) * 16.0 + (double)npts(dim, (m - 1) / 2) * 8.0;
        }
        b->ops.push_back(op);
      }
    }
  }
  for (int dim = 3; dim >= 2; --dim) {  // bottom levels, one workgroup per problem
    BOp op;
    op.kind = BO_BOTTOM;
    op.dim = dim;
    op.nent = 0;
    op.cls = PC_BOTTOM;
    bb.align_tbl();
    op.tbl_off = b->host_tbl.size();
    for (int q = 0; q < n; ++q) {
      BProblem &pr = b->pb[q];
      if (pr.dim != dim) continue;
      ++op.nent;
      BottomArgs<double> a{};
      a.f = pr.f[pr.B];
      a.u = pr.u[pr.B];
      a.active = &pr.st->active;
      a.dim = pr.dim;
      a.L = pr.L - pr.B;
      a.nu1 = nu1;
      a.nu2 = nu2;
      a.smoother = sm;
      a.post_forward = bwd ? 0 : 1;
      a.omega = wj_omega(p, pr.dim);
      bb.push(a);
      const size_t lds = bottom_lds_bytes(pr.dim, a.L, sm, sizeof(double));
      if (lds > op.lds) {
        op.lds = lds;
        op.bottom_L = a.L;
        op.bottom_dim = pr.dim;
      }
    }
    if (op.nent > 0) b->ops.push_back(op);
  }
  for (int dim = 3; dim >= 2; --dim) {
    int Emax = 0;
    for (auto &pr : b->pb)
      if (pr.dim == dim) Emax = std::max(Emax, pr.L);
    for (int e = 2; e <= Emax; ++e) {
      const int m = (1 << e) - 1;
      std::vector<ChainEnt> ents;
      for (int q = 0; q < n; ++q) {
        BProblem &pr = b->pb[q];
        if (pr.dim != dim) continue;
        const int l = pr.L - e;
        if (l < 0 || l >= pr.B) continue;
        ents.push_back({q, l, pr.w[l], pr.u[l + 1], l == 0 ? nullptr : pr.f[l],
                        l == 0 ? nullptr : pr.u[l], pr.t[l], false, l == 0, l == 0, nullptr});
      }
      // the ascent always takes the plane-marching pass, as for single
      // problems (faster than the LDS-tile kernel on every level)
      build_chain(bb, dim, m, 1, nu2, F_PROLONG, bwd, ents, PC_POST_C);
    }
  }
  bool has2 = false, has3 = false;
  for (const auto &pr : b->pb) (pr.dim == 2 ? has2 : has3) = true;
  b->two = has2 && has3 && !(p->cfg.flags & GMG_BATCH_ONE_STREAM);
  for (BOp &op : b->ops) op.branch = b->two && op.dim == 2 ? 1 : 0;
  bb.align_tbl();
  const size_t tbl_off = bb.take_bytes(std::max(b->host_tbl.size(), b->tbl_reserve));
  b->dev_tbl = ws + tbl_off;
  return bb.cur;
}

hipError_t batch_enqueue_cycle(gmg_plan *p) {
  Batch *b = p->batch;
  // profiled cycles time every launch on the plan's stream: one branch
  const bool fork = b->two && !p->profile;
  if (fork) {
    hipError_t e = hipSuccess;
    if (!b->side) e = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking);
    if (e == hipSuccess && !b->ev_fork)
      e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess && !b->ev_join)
      e = hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(b->ev_fork, p->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->side, b->ev_fork, 0);
    if (e != hipSuccess) return e;
  }
  for (const BOp &op : b->ops) {
    const char *tbl = b->dev_tbl + op.tbl_off;
    const char *host = b->host_tbl.data() + op.tbl_off;
    const hipStream_t s = fork && op.branch ? b->side : p->stream;
    hipError_t e = hipSuccess;
    ProfScope ps(p, op.cls, op.bytes);
    switch (op.kind) {
      case BO_PASS: {
        PassArgs<double> a;
        std::memcpy(&a, host, sizeof(a));
        e = op.wj ? launch_wj_pass<double>(op.dim, op.stages, op.flags, op.variant, a, s,
                                           (const PassArgs<double> *)tbl, op.nent)
                  : launch_rb_pass<double>(op.dim, op.stages, op.flags, op.variant, a, s,
                                           (const PassArgs<double> *)tbl, op.nent);
        break;
      }
      case BO_RESTRICT: {
        RestrictArgs<double> a{};
        std::memcpy(&a, host, sizeof(a));
        e = launch_restrict<double>(op.dim, a, s, (const RestrictArgs<double> *)tbl,
                                    op.nent);
        break;
      }
      case BO_FIN:
        e = launch_finalize_batch((const FinEntry *)tbl, op.nent, s);
        break;
      case BO_BOTTOM: {
        BottomArgs<double> a{};
        a.dim = op.bottom_dim;
        a.L = op.bottom_L;
        a.smoother = p->cfg.smoother == GMG_SMOOTH_WJ ? 1 : 0;
        e = launch_bottom<double>(op.nent, a, (const BottomArgs<double> *)tbl, s, op.lds);
        break;
      }
    }
    if (e != hipSuccess) return e;
  }
  if (fork) {
    hipError_t e = hipEventRecord(b->ev_join, b->side);
    if (e == hipSuccess) e = hipStreamWaitEvent(p->stream, b->ev_join, 0);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t batch_run_cycle(gmg_plan *p) {
  Batch *b = p->batch;
  if (!(p->cfg.flags & GMG_USE_GRAPH) || p->profile) return batch_enqueue_cycle(p);
  if (!b->graph) {
    hipError_t e;
    if (!p->capture_stream) {
      e = hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking);
      if (e != hipSuccess) return e;
    }
    hipStream_t keep = p->stream;
    p->stream = p->capture_stream;
    e = hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
      p->stream = keep;
      return e;
    }
    hipError_t ee = batch_enqueue_cycle(p);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(p->capture_stream, &g);
    p->stream = keep;
    if (ee != hipSuccess) return ee;
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return e;
  }
  return hipGraphLaunch(b->graph, p->stream);
}

gmg_status batch_setup(const gmg_config *cfg, int n, const int *dims, const int *levels,
                       void *workspace, size_t *ws_bytes, void *stream, gmg_plan **out) {
  if (!dims || !levels) return GMG_ERR_INVALID_ARG;
  gmg_config c = *cfg;
  c.dim = dims[0];
  c.levels = levels[0];
  gmg_status st = validate_cfg(&c);
  if (st != GMG_OK) return st;
  if (c.precision != GMG_FP64) return GMG_ERR_UNSUPPORTED;  // batch: FP64 cycles
  if (cfg_variant(c)) return GMG_ERR_UNSUPPORTED;
  if (c.nu1 < 1 || c.nu2 < 1) return GMG_ERR_UNSUPPORTED;
  for (int q = 0; q < n; ++q) {
    if (dims[q] != 2 && dims[q] != 3) return GMG_ERR_INVALID_ARG;
    if (levels[q] < 2 || levels[q] > (dims[q] == 3 ? 10 : kMaxLevels)) return GMG_ERR_INVALID_ARG;
  }
  gmg_plan tmp;
  init_plan_shape(tmp, &c);
  tmp.cross = false;
  Batch tw;  // the most launches any tile choice can give sizes the table region
  tw.worst = true;
  batch_build(&tmp, &tw, n, dims, levels, nullptr);
  const size_t reserve = align_up(tw.host_tbl.size());
  Batch tb;
  tb.tbl_reserve = reserve;
  const size_t total = batch_build(&tmp, &tb, n, dims, levels, nullptr);
  if (!workspace) {
    *ws_bytes = total;
    return GMG_OK;
  }
  if (!out) return GMG_ERR_INVALID_ARG;
  if (*ws_bytes < total) return GMG_ERR_WORKSPACE;
  if (((uintptr_t)workspace) % kAlign) return GMG_ERR_WORKSPACE;
  gmg_plan *p = new gmg_plan();
  init_plan_shape(*p, &c);
  p->cross = false;  // batches run the two-pass schedule on every problem
  p->nproblems = n;
  p->stream = (hipStream_t)stream;
  p->ws = (char *)workspace;
  p->ws_bytes = total;
  p->batch = new Batch();
  p->batch->tbl_reserve = reserve;
  batch_build(p, p->batch, n, dims, levels, p->ws);
  p->prof.resize(PC_COUNT);
  for (int i = 0; i < PC_COUNT; ++i) p->prof[i].name = kProfNames[i];
  Batch *b = p->batch;
  if (hipHostMalloc((void **)&b->pinned, reserve + 64, hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc((void **)&b->hstates, sizeof(SolveState) * n, hipHostMallocDefault) !=
          hipSuccess) {
    if (b->pinned) (void)hipHostFree(b->pinned);
    delete b;
    delete p;
    return GMG_ERR_HIP;
  }
  *out = p;
  return GMG_OK;
}

// Autotuning of a batch plan (first gmg_batch_solve): one problem of every
// distinct (dim, levels) shape is tuned with the single-problem tuner on its
// own slice of the workspace (the caller's u and f are only read), the
// choices are kept per (dim, level side, role), and the launch tables are
// rebuilt.  Batch launches keep the restriction a kernel of its own, so the
// candidates are timed that way.
hipError_t batch_tune(gmg_plan *p, double *const *u, const double *const *f) {
  Batch *b = p->batch;
  const int n = p->nproblems;
  std::vector<int> dims(n), levels(n);
  std::map<std::pair<int, int>, int> shapes;
  for (int q = 0; q < n; ++q) {
    dims[q] = b->pb[q].dim;
    levels[q] = b->pb[q].L;
    shapes.emplace(std::make_pair(dims[q], levels[q]), q);
  }
  for (const auto &sh : shapes) {
    const int q = sh.second;
    const BProblem &pr = b->pb[q];
    gmg_config c = p->cfg;
    c.dim = pr.dim;
    c.levels = pr.L;
    c.omega = p->omega_user;
    c.flags = c.flags & ~(unsigned)GMG_PROFILE;
    gmg_plan v;
    init_plan_shape(v, &c);
    v.cross = false;
    if (v.B != pr.B) continue;
    v.stream = p->stream;
    v.profile = false;
    v.ch.resize(v.L);
    for (int l = 0; l < v.L; ++l)
      for (int r = 0; r < 2; ++r) v.ch[l][r] = batch_choice(p, b, pr.dim, pr.m[l], r);
    v.d.f = pr.f;
    v.d.w = pr.w;
    v.d.u = pr.u;
    v.d.t = pr.t;
    v.d.f[0] = const_cast<double *>(f[q]);
    hipError_t e = tune_plan<double>(&v, u[q], f[q], nullptr);
    if (e != hipSuccess) return e;
    for (int l = 0; l < v.B && l + 1 < v.L; ++l)
      for (int r = 0; r < 2; ++r) {
        b->choice.emplace(std::array<int, 3>{pr.dim, pr.m[l], r}, v.ch[l][r]);
      }
  }
  batch_build(p, b, n, dims.data(), levels.data(), p->ws);
  if (b->graph) {
    (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
  }
  return hipSuccess;
}

}  // namespace

namespace {
// Binds a single-problem plan to its workspace: the solve state, norm
// partials and level arrays carved as the layout says, default tile choices,
// and the host copy of the solve state (hstate: room for the state and one
// double after it).
void bind_single(gmg_plan &p, const gmg_config &c, const Layout &Y, void *workspace,
                 hipStream_t stream, SolveState *hstate) {
  init_plan_shape(p, &c);
  p.nproblems = 1;
  p.stream = stream;
  p.ws = (char *)workspace;
  p.ws_bytes = Y.total;
  p.state = reinterpret_cast<SolveState *>(p.ws + Y.off_state);
  p.partials = reinterpret_cast<double *>(p.ws + Y.off_partials);
  p.scalar = reinterpret_cast<double *>(p.ws + Y.off_scalar);
  if (c.precision == GMG_MIXED_FP32_IR) {
    p.x2 = reinterpret_cast<double *>(p.ws + Y.off_x2);
    bind<float>(p.s, p.ws, Y.fs, Y.ws, Y.us, Y.ts);
    bind<double>(p.d, p.ws, Y.f, Y.w, Y.u, Y.t);
  } else {
    bind<double>(p.d, p.ws, Y.f, Y.w, Y.u, Y.t);
    std::vector<size_t> none(p.L, (size_t)-1);
    bind<float>(p.s, p.ws, none, none, none, none);
  }
  default_tiles(p);
  p.prof.resize(PC_COUNT);
  for (int i = 0; i < PC_COUNT; ++i) p.prof[i].name = kProfNames[i];
  p.hstate = hstate;
  p.hscalar = reinterpret_cast<double *>(reinterpret_cast<char *>(hstate) + sizeof(SolveState));
}
}  // namespace

// ------------------------------------------------------------------ static scratch
// The workspace of gmg_solve_scratch: a file-scope device array (each GPU the
// library runs on holds its own copy until the process ends).  On the host
// the name `scratch` is only a stand-in, never a device address: the address
// of a device's copy comes from hipGetSymbolAddress, called once per device
// with that device current and kept in scratch_addr, and only that address is
// handed to kernels.
constexpr size_t kScratchBytes = (size_t)GMG_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_addr[kMaxDevices] = {};

// Address of the current device's scratch array (looked up on its first use).
gmg_status scratch_base(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GMG_ERR_HIP;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_addr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return GMG_ERR_HIP;
    scratch_addr[dev] = ptr;
  }
  *out = scratch_addr[dev];
  return GMG_OK;
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
  cfg->inner_cycles = 4;
  cfg->flags = 0;
  return validate_cfg(cfg);
}

gmg_status gmg_setup(const gmg_config *cfg, int nproblems, const int *dims, const int *levels,
                     void *workspace, size_t *ws_bytes, void *stream, gmg_plan **out) {
  if (!ws_bytes) return GMG_ERR_INVALID_ARG;
  if (nproblems < 1) return GMG_ERR_INVALID_ARG;
  if (!cfg) return GMG_ERR_INVALID_ARG;
  if (nproblems > 1) return batch_setup(cfg, nproblems, dims, levels, workspace, ws_bytes, stream, out);
  gmg_config c = *cfg;
  if (dims) c.dim = dims[0];
  if (levels) c.levels = levels[0];
  gmg_status st = validate_cfg(&c);
  if (st != GMG_OK) return st;
  if (cfg_variant(c) && c.precision != GMG_FP64) return GMG_ERR_UNSUPPORTED;
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
  SolveState *hs = nullptr;
  if (hipHostMalloc((void **)&hs, sizeof(SolveState) + 64, hipHostMallocDefault) != hipSuccess) {
    delete p;
    return GMG_ERR_HIP;
  }
  bind_single(*p, c, Y, workspace, (hipStream_t)stream, hs);
  *out = p;
  return GMG_OK;
}

gmg_status gmg_solve_scratch(const gmg_config *cfg, double *u, const double *f, double rtol,
                             int maxit, const double *res0_opt, int *iters, double *relres,
                             void *stream) {
  if (!cfg || !u || !f) return GMG_ERR_INVALID_ARG;
  if (!(rtol > 0.0) || maxit < 1) return GMG_ERR_INVALID_ARG;
  if (res0_opt && !(*res0_opt >= 0.0)) return GMG_ERR_INVALID_ARG;
  gmg_config c = *cfg;
  gmg_status st = validate_cfg(&c);
  if (st != GMG_OK) return st;
  if (cfg_variant(c) && c.precision != GMG_FP64) return GMG_ERR_UNSUPPORTED;
  // tuning and profiling create events, graphs instantiate device objects
  if (c.flags & (GMG_AUTOTUNE | GMG_PROFILE | GMG_USE_GRAPH)) return GMG_ERR_UNSUPPORTED;
  gmg_plan tmp;
  init_plan_shape(tmp, &c);
  const Layout Y = make_layout(tmp);
  if (Y.total > kScratchBytes) return GMG_ERR_WORKSPACE;
  void *ws = nullptr;
  st = scratch_base(&ws);
  if (st != GMG_OK) return st;
  // the host copy of the solve state: pageable, on this stack frame
  alignas(64) unsigned char hbuf[sizeof(SolveState) + 64];
  gmg_plan p;
  bind_single(p, c, Y, ws, (hipStream_t)stream, reinterpret_cast<SolveState *>(hbuf));
  return gmg_solve(&p, u, f, rtol, maxit, res0_opt, iters, relres);
}

gmg_status gmg_destroy(gmg_plan *p) {
  if (!p) return GMG_ERR_INVALID_ARG;
  for (auto &e : p->pending) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  for (auto e : p->evpool) (void)hipEventDestroy(e);
  if (p->hstate) (void)hipHostFree(p->hstate);
  for (auto &row : p->coarse_graph)
    for (auto &g : row)
      if (g) (void)hipGraphExecDestroy(g);
  if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
  if (p->batch) {
    if (p->batch->graph) (void)hipGraphExecDestroy(p->batch->graph);
    if (p->batch->ev_fork) (void)hipEventDestroy(p->batch->ev_fork);
    if (p->batch->ev_join) (void)hipEventDestroy(p->batch->ev_join);
    if (p->batch->side) (void)hipStreamDestroy(p->batch->side);
    if (p->batch->pinned) (void)hipHostFree(p->batch->pinned);
    if (p->batch->hstates) (void)hipHostFree(p->batch->hstates);
    delete p->batch;
  }
  delete p;
  return GMG_OK;
}

size_t gmg_plan_workspace_bytes(const gmg_plan *p) { return p ? p->ws_bytes : 0; }

int gmg_level_side(const gmg_plan *p, int problem, int level) {
  if (p && p->batch) {
    if (problem < 0 || problem >= p->nproblems) return -1;
    const BProblem &pr = p->batch->pb[problem];
    if (level < 0 || level >= pr.L) return -1;
    return pr.m[level];
  }
  if (!p || problem != 0 || level < 0 || level >= p->L) return -1;
  return p->m[level];
}

gmg_status gmg_fmg(gmg_plan *p, double *u, const double *f) {
  if (!p || !u || !f || p->batch) return GMG_ERR_INVALID_ARG;
  if (p->cfg.precision != GMG_FP64) return GMG_ERR_UNSUPPORTED;
  if (is_variant(p)) {
    HIPCHK(var_fmg(p, u, f));
    return GMG_OK;
  }
  if ((p->cfg.flags & GMG_AUTOTUNE) && !p->tuned) HIPCHK(tune_plan<double>(p, u, f, nullptr));
  HIPCHK(enqueue_fmg(p, u, f));
  return GMG_OK;
}

gmg_status gmg_vcycle(gmg_plan *p, double *u, const double *f) {
  if (!p || !u || !f || p->batch) return GMG_ERR_INVALID_ARG;
  if (is_variant(p)) {
    HIPCHK(var_cycle(p, 0, u, f, u, nullptr, nullptr));
    return GMG_OK;
  }
  if ((p->cfg.flags & GMG_AUTOTUNE) && !p->tuned) {
    if (p->cfg.precision == GMG_FP64)
      HIPCHK(tune_plan<double>(p, u, f, nullptr));
    else
      HIPCHK(tune_plan<float>(p, nullptr, p->s.f[0], nullptr));
  }
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
  HIPCHK(enqueue_inner(p, nullptr));
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
  if (!p || !u || !f || p->batch) return GMG_ERR_INVALID_ARG;
  if (!(rtol > 0.0) || maxit < 1) return GMG_ERR_INVALID_ARG;
  if (res0_opt && !(*res0_opt >= 0.0)) return GMG_ERR_INVALID_ARG;
  struct TagReset {
    gmg_plan *p;
    ~TagReset() { p->prof_tag = -1; }
  } tag_reset{p};
  if ((p->cfg.flags & GMG_AUTOTUNE) && !p->tuned && !is_variant(p)) {
    if (p->cfg.precision == GMG_FP64)
      HIPCHK(tune_plan<double>(p, u, f, p->partials));
    else
      HIPCHK(tune_plan<float>(p, nullptr, p->s.f[0], nullptr));
  }
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
      p->prof_tag = enq;
      if (is_variant(p)) {
        HIPCHK(var_cycle(p, 0, u, f, u, p->partials, act));
      } else if (p->cross) {
        HIPCHK(enqueue_cross_body(p, enq, u, f, act));
      } else if (!mixed) {
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
        HIPCHK(enqueue_inner(p, act));
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
  p->prof_tag = -1;
  const SolveState st = *p->hstate;
  // the stopping body ran its first step and the stop test
  if (p->profile)
    prune_profile(p, st.iter,
                  is_variant(p) ? (1u << PC_FIN)
                                : (1u << PC_FIN) | (1u << (mixed ? PC_IR : PC_PRE0)) |
                                      (1u << PC_CROSS0));
  if (p->cross && st.iter >= 1) {
    // u = u_K, the iterate the loop stopped at, from w_K + P e_K (both left
    // in place: every launch after the stop test returned at once)
    const int K = st.iter;
    HIPCHK(smooth_chain<double>(p, 0, 1, true, cross_buf<double>(p, K), p->d.u[1], f, u, nullptr,
                                nullptr, nullptr, PC_POST0, nullptr));
    HIPCHK(hipStreamSynchronize(p->stream));
  }
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
  if (!p || !u || !f) return GMG_ERR_INVALID_ARG;
  if (!p->batch) return GMG_ERR_INVALID_ARG;
  if (!(rtol > 0.0) || maxit < 1) return GMG_ERR_INVALID_ARG;
  Batch *b = p->batch;
  const int n = p->nproblems;
  for (int q = 0; q < n; ++q)
    if (!u[q] || !f[q]) return GMG_ERR_INVALID_ARG;
  if ((p->cfg.flags & GMG_AUTOTUNE) && !p->tuned) {
    HIPCHK(batch_tune(p, u, f));
    p->tuned = true;
  }
  // the caller's arrays go into the level-0 entries of the launch tables
  for (const auto &pt : b->patches) {
    void *v = pt.which == 0 ? (void *)u[pt.prob] : (void *)f[pt.prob];
    std::memcpy(b->host_tbl.data() + pt.off, &v, sizeof(void *));
  }
  std::memcpy(b->pinned, b->host_tbl.data(), b->host_tbl.size());
  HIPCHK(hipMemcpyAsync(b->dev_tbl, b->pinned, b->host_tbl.size(), hipMemcpyHostToDevice,
                        p->stream));
  HIPCHK(launch_state_init_batch(b->states, n, maxit, rtol, p->stream));
  int enq = 0, batch = 2;
  for (;;) {
    for (int k = 0; k < batch; ++k, ++enq) HIPCHK(batch_run_cycle(p));
    HIPCHK(hipMemcpyAsync(b->hstates, b->states, sizeof(SolveState) * n, hipMemcpyDeviceToHost,
                          p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    int need = 0, active = 0;
    for (int q = 0; q < n; ++q) {
      const SolveState &s = b->hstates[q];
      if (!s.active) continue;
      ++active;
      need = std::max(need, estimate_cycles(s, s.iter - 1));
    }
    if (!active || enq >= maxit + 1) break;
    batch = std::max(1, std::min(need, maxit + 1 - enq));
  }
  gmg_status worst = GMG_OK;
  for (int q = 0; q < n; ++q) {
    const SolveState &s = b->hstates[q];
    const gmg_status sq = map_status(s.status);
    if (iters) iters[q] = s.iter;
    if (relres) relres[q] = s.res0 > 0.0 ? s.res / s.res0 : 0.0;
    if (st) st[q] = sq;
    if (sq < 0 && (worst >= 0 || sq < worst)) worst = sq;
    if (sq == GMG_NOT_CONVERGED && worst == GMG_OK) worst = sq;
  }
  if (p->profile) {
    gmg_status hs = harvest(p);
    if (hs != GMG_OK) return hs;
  }
  return worst;
}

int gmg_tile_variant_count(int dim, gmg_smoother smoother, int stages) {
  if ((dim != 2 && dim != 3) || stages < 1 || stages > 4) return 0;
  return pass_variant_count(dim, stages, smoother == GMG_SMOOTH_WJ ? 1 : 0);
}

gmg_status gmg_plan_set_tile(gmg_plan *p, int level, int stages, int variant, int tz) {
  if (!p || p->batch || level < 0 || level >= p->L || stages < 1 || stages > 4 || tz < 0)
    return GMG_ERR_INVALID_ARG;
  const int wj = p->cfg.smoother == GMG_SMOOTH_WJ ? 1 : 0;
  const int nv = pass_variant_count(p->dim, stages, wj);
  if (variant < 0 || variant >= nv) return GMG_ERR_INVALID_ARG;
  const PassTile t = pass_variant(p->dim, stages, wj, variant);
  const int tzv = tz > 0 ? std::min(tz, p->m[level]) : auto_tz(p->dim, p->m[level], stages, t);
  if (pass_geometry(p->dim, p->m[level], stages, t, tzv).nblocks > kMaxPartials)
    return GMG_ERR_INVALID_ARG;
  if (!wj && stages == 3) {  // the cross-cycle pass of level 0
    if (level != 0) return GMG_ERR_INVALID_ARG;
    // the tile must run the form the plan will use: the restriction folded
    // in when the plan allows it and the tile fits, the plain form otherwise
    const size_t elem = p->cfg.precision == GMG_MIXED_FP32_IR ? sizeof(float) : sizeof(double);
    const bool fold = !(p->cfg.flags & GMG_NO_FUSED_RESTRICT) &&
                      pass_geometry(p->dim, p->m[0], 3, t, tzv, true).nblocks <= kMaxPartials &&
                      rb_pass_fits(p->dim, 3, variant, F_PROLONG | F_RESTRICT, elem);
    if (!fold && !rb_pass_fits(p->dim, 3, variant, F_PROLONG, elem)) return GMG_ERR_INVALID_ARG;
    PassChoice &c = p->ch[0][2];
    c.var[3] = variant;
    c.tz[3] = tzv;
    return GMG_OK;
  }
  const int sweeps = wj ? stages : stages / 2;
  if (sweeps < 1 || sweeps > p->smax_cap) return GMG_ERR_INVALID_ARG;
  for (int role = 0; role < 2; ++role) {
    PassChoice &c = p->ch[level][role];
    c.var[stages] = variant;
    c.tz[stages] = tzv;
    c.smax = sweeps;
  }
  return GMG_OK;
}

gmg_status gmg_plan_set_tile_order(gmg_plan *p, int level, int stages, int strip) {
  if (!p || p->batch || level < 0 || level >= p->L || stages < 1 || stages > 4 || strip < 0)
    return GMG_ERR_INVALID_ARG;
  const int wj = p->cfg.smoother == GMG_SMOOTH_WJ ? 1 : 0;
  if (pass_variant_count(p->dim, stages, wj) == 0) return GMG_ERR_INVALID_ARG;
  if (!wj && stages == 3) {
    if (level != 0) return GMG_ERR_INVALID_ARG;
    p->ch[0][2].sw[3] = strip;
    return GMG_OK;
  }
  for (int role = 0; role < 2; ++role) p->ch[level][role].sw[stages] = strip;
  return GMG_OK;
}

gmg_status gmg_plan_get_tile(const gmg_plan *p, int level, int role, int *stages, int *variant,
                             int *tz) {
  if (!p || p->batch || level < 0 || level >= p->L || role < 0 || role > 2)
    return GMG_ERR_INVALID_ARG;
  const int wj = p->cfg.smoother == GMG_SMOOTH_WJ ? 1 : 0;
  int st;
  if (role == 2) {
    if (level != 0 || !(p->cross || p->cross32)) return GMG_ERR_INVALID_ARG;
    st = 3;
  } else {
    const int nu = role == 0 ? p->cfg.nu1 : p->cfg.nu2;
    if (nu < 1) return GMG_ERR_INVALID_ARG;
    st = stages_of(p, std::min(p->ch[level][role].smax, nu));
  }
  const PassChoice &c = p->ch[level][role];
  const PassTile t = pass_variant(p->dim, st, wj, c.var[st]);
  if (stages) *stages = st;
  if (variant) *variant = c.var[st];
  if (tz) *tz = c.tz[st] > 0 ? std::min(c.tz[st], p->m[level])
                             : auto_tz(p->dim, p->m[level], st, t);
  return GMG_OK;
}

gmg_status gmg_tune_cache_check(const char *path, int *n_valid, int *n_invalid) {
  if (!path || !n_valid || !n_invalid) return GMG_ERR_INVALID_ARG;
  FILE *fh = std::fopen(path, "r");
  if (!fh) return GMG_ERR_INVALID_ARG;
  *n_valid = *n_invalid = 0;
  char line[512];
  while (std::fgets(line, sizeof(line), fh)) {
    bool blank = true;
    for (const char *c = line; *c; ++c) blank = blank && (*c == ' ' || *c == '\n' || *c == '\r');
    if (blank) continue;
    std::string key;
    PassChoice c;
    int st = 0, dim = 0, m = 0, cap = 0;
    bool wj = false;
    const bool ok = parse_cache_line(line, key, c, st) && key_shape(key, dim, m, wj, cap) &&
                    cap <= 2 && choice_ok(dim, m, cap, wj, c);
    ++(ok ? *n_valid : *n_invalid);
  }
  std::fclose(fh);
  return GMG_OK;
}

// ------------------------------------------------------------------ primitives
static gmg_status check_level(gmg_plan *p, int level, gmg_dtype dt) {
  if (!p || p->batch || level < 0 || level >= p->L) return GMG_ERR_INVALID_ARG;
  if (dt != GMG_F64 && dt != GMG_F32) return GMG_ERR_INVALID_ARG;
  return GMG_OK;
}

}  // extern "C"

template <typename T>
static gmg_status op_smooth_t(gmg_plan *p, int level, int nsweeps, int backward, const T *u_in,
                              const T *f, const T *ec, T *u_out, double *res_in_norm) {
  LevelSet<T> &S = levels_of<T>(p);
  if (is_variant(p) && p->cfg.smoother == GMG_SMOOTH_MCGS) {
    if constexpr (sizeof(T) != 8) {
      return GMG_ERR_UNSUPPORTED;
    } else {
      if (ec) return GMG_ERR_UNSUPPORTED;
      double *tmp = level < (int)S.t.size() ? S.t[level] : nullptr;
      if (nsweeps >= 2 && !tmp) return GMG_ERR_UNSUPPORTED;
      const int m = p->m[level];
      const int nb = residual_blocks(p->dim, m);
      if (res_in_norm) {
        const double h = 1.0 / double(m + 1);
        ResidArgs<double> r{u_in, f, nullptr, p->partials, nullptr, m, nb, 1.0 / (h * h)};
        HIPCHK(launch_residual<double>(p->dim, r, p->stream));
      }
      HIPCHK(var_smooth(p, level, nsweeps, backward != 0, u_in, f, u_out, tmp, nullptr, PC_MISC));
      if (res_in_norm) {
        HIPCHK(launch_reduce_norm(p->partials, nb, p->scalar, p->stream));
        HIPCHK(hipMemcpyAsync(p->hscalar, p->scalar, sizeof(double), hipMemcpyDeviceToHost,
                              p->stream));
        HIPCHK(hipStreamSynchronize(p->stream));
        *res_in_norm = *p->hscalar;
      }
      return GMG_OK;
    }
  }
  if (is_variant(p) && ec) return GMG_ERR_UNSUPPORTED;
  T *tmp = level < (int)S.t.size() ? S.t[level] : nullptr;
  const int smax = p->ch[level][ec ? 1 : 0].smax;
  const int K = nsweeps == 0 ? 0 : (nsweeps + smax - 1) / smax;
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
  if (p->cfg.flags & GMG_FE_TRANSFER) {
    if (dt != GMG_F64) return GMG_ERR_UNSUPPORTED;
    HIPCHK(var_restrict(p, level, (const double *)u, (const double *)f, (double *)f_coarse,
                        nullptr, PC_MISC));
    return GMG_OK;
  }
  if (dt == GMG_F64)
    HIPCHK(restrict_level<double>(p, level, (const double *)u, (const double *)f,
                                  (double *)f_coarse, nullptr, PC_MISC));
  else
    HIPCHK(restrict_level<float>(p, level, (const float *)u, (const float *)f, (float *)f_coarse,
                                 nullptr, PC_MISC));
  return GMG_OK;
}

gmg_status gmg_op_prolong_add(gmg_plan *p, int level, gmg_dtype dt, const void *u_in,
                              const void *e_coarse, void *u_out) {
  gmg_status s = check_level(p, level, dt);
  if (s != GMG_OK) return s;
  if (level + 1 >= p->L || !e_coarse || !u_out || e_coarse == u_out) return GMG_ERR_INVALID_ARG;
  if (dt == GMG_F64) {
    HIPCHK(var_prolong(p, level, (const double *)u_in, (const double *)e_coarse, (double *)u_out,
                       nullptr));
    return GMG_OK;
  }
  if (p->cfg.flags & GMG_FE_TRANSFER) return GMG_ERR_UNSUPPORTED;
  HIPCHK(launch_prolong_add<float>(p->dim, p->m[level], p->m[level + 1], (const float *)u_in,
                                   (const float *)e_coarse, (float *)u_out, nullptr, p->stream));
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

gmg_status gmg_profile_set_mask(gmg_plan *p, unsigned mask) {
  if (!p) return GMG_ERR_INVALID_ARG;
  p->prof_mask = mask;
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
