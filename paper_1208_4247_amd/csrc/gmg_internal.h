// gmg_internal.h -- declarations shared by the HIP kernels and the host
// orchestration of the multigrid library (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stddef.h>
#include <stdint.h>

namespace gmg {

// Global-memory views of device pointers.  Accesses through them compile to
// global_* instructions; accesses through generic pointers compile to flat_*
// ones, which also count on the LDS wait counter, so every LDS wait would
// also wait for the HBM loads in flight.
#define GMG_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GMG_GLOBAL T *gbl(T *p) {
  return (GMG_GLOBAL T *)p;
}
template <typename T>
__device__ __forceinline__ const GMG_GLOBAL T *gbl(const T *p) {
  return (const GMG_GLOBAL T *)p;
}

// Event pair that the library's profiler wants the next kernel dispatch of
// this host thread to record (start and end of that dispatch, the same
// timestamps a kernel-trace profiler reports), or {NULL, NULL}.
struct DispatchEvents {
  hipEvent_t start, stop;
};
DispatchEvents &next_dispatch_events();

// Every kernel launch of the library goes through here.
template <typename F, typename... Args>
inline void gmg_launch(F k, dim3 grid, dim3 block, size_t lds, hipStream_t s, Args... args) {
  DispatchEvents &ev = next_dispatch_events();
  if (ev.start) {
    hipEvent_t a = ev.start, b = ev.stop;
    ev.start = ev.stop = nullptr;
    hipExtLaunchKernelGGL(k, grid, block, (uint32_t)lds, s, a, b, 0u, args...);
  } else {
    hipLaunchKernelGGL(k, grid, block, lds, s, args...);
  }
}

// ---- buffer-resource access used by the plane-marching kernels.  A raw
// buffer over one plane (no records for a plane outside the grid) with a
// per-element byte offset that is out of range outside the grid: such loads
// return 0 and such stores are dropped, so the zero Dirichlet boundary costs
// no branches.
constexpr int kOOB = 0x7ffffff0;  // byte offset beyond any plane resource

template <int V>
struct IntC {
  static constexpr int value = V;
};

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const T *base, int z, int m,
                                                             int plane) {
  // raw buffer over plane z (no records when z is outside 0..m-1)
  const bool in = z >= 0 && z < m;
  const T *p = base + (in ? (size_t)z * plane : 0);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(p), (short)0,
                                           in ? plane * (int)sizeof(T) : 0, 0x00020000);
}

// raw buffer over plane z when `on`, else one with no records (its loads
// return 0 and its stores are dropped).  Lets a store that applies to some
// steps only be issued on every step, with no branch around it, so the
// compiler's count of outstanding memory operations stays exact and a wait
// for an older load never has to include younger loads.
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc_if(const T *base, int z, bool on,
                                                                int plane) {
  const T *p = base + (on ? (size_t)z * plane : 0);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(p), (short)0,
                                           on ? plane * (int)sizeof(T) : 0, 0x00020000);
}

template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, int off) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

typedef unsigned int gmg_u32x2 __attribute__((ext_vector_type(2)));

template <typename T>
struct PairOf {
  T lo, hi;
};

// two adjacent elements in one load (16 bytes for FP64, 8 for FP32)
template <typename T>
__device__ __forceinline__ PairOf<T> bload2(__amdgpu_buffer_rsrc_t r, int off) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(PairOf<T>, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
  else
    return __builtin_bit_cast(PairOf<T>, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

template <typename T>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, int off, T v) {
  if constexpr (sizeof(T) == 8)
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(gmg_u32x2, v), r, off, 0, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, 0);
}


// two adjacent elements in one store (the counterpart of bload2)
template <typename T>
__device__ __forceinline__ void bstore2(__amdgpu_buffer_rsrc_t r, int off, T lo, T hi) {
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  const PairOf<T> v{lo, hi};
  if constexpr (sizeof(T) == 8)
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, off, 0, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(gmg_u32x2, v), r, off, 0, 0);
}

// The pointwise solve (h^2 f + nb) / (2d) of a Gauss-Seidel or Jacobi update
// (the relaxation of Sec. 3.2).  FP64: rounded as written -- the product
// h^2 f, the sum and the quotient each rounded to nearest, so the iterates are
// those of the formula evaluated literally.  The quotient by 4 is exact.  The
// quotient by 6 is y * (C_hi + C_lo) with C_hi = RN(1/6), C_lo = RN(1/6 - C_hi),
// formed as one FMA over the small product: fma(y, C_hi, RN(y C_lo)).  That is
// the correctly rounded y/6 for every y whose y C_lo stays normal
// (|y| > 2^-965): y/3 has a 53-bit integer numerator over 3, so it lies at
// least 1/6 ulp from any rounding midpoint, while the value the FMA rounds
// differs from y/6 by at most 2^-108 |y|.  Two dependent operations where the
// reciprocal-and-correction form (Markstein) takes three.  FP32 (the inner
// cycles of the mixed form, whose corrections the FP64 refinement checks): one
// FMA and the rounded reciprocal.
template <typename T, int DIM>
__device__ __forceinline__ T point_solve(T h2, T f, T nb) {
  if constexpr (sizeof(T) == 4) {
    return fma(h2, f, nb) * (DIM == 3 ? T(1.0 / 6.0) : T(0.25));
  } else {
    const T y = h2 * f + nb;
    if constexpr (DIM == 2) {
      return y * T(0.25);
    } else {
      return fma(y, T(0x1.5555555555555p-3), y * T(0x1.5555555555555p-57));
    }
  }
}

// Flags of a fused smoothing pass.
enum PassFlags : int {
  F_ZERO_IN = 1,     // start value is zero: u_in is not read
  F_PROLONG = 2,     // start value is u_in + P e_coarse (linear interpolation)
  F_NORM_IN = 4,     // emit per-workgroup partial sums of |f - A u_in|^2
  F_BLACK_FIRST = 8, // red-black order black -> red (backward sweep)
  F_RESTRICT = 16,   // red-black: also form f_c = R (f - A u_out), the residual's
                     // full weighting onto the next coarser grid
  F_NORM_MID = 32,   // red-black, S = 2q - 1 stages: emit per-workgroup partial
                     // sums of |f - A u_q|^2, u_q the iterate after stage q
};

// Device-resident state of one solve (one per problem in batch mode).
struct SolveState {
  int active;   // 1 while further cycles should run
  int iter;     // cycles started (the finalize step counts the cycle it admits)
  int maxit;
  int status;   // 0 converged/running, 1 maxit, -3 non-finite, -4 diverged
  double rtol;
  double res0;  // < 0: take from the first norm
  double res;   // last residual norm
  double pad;
};

template <typename T>
struct PassArgs {
  const T *u_in;        // start value (ignored with F_ZERO_IN)
  const T *f;           // right-hand side of this level
  T *u_out;             // result (never aliases u_in / f / e_c)
  const T *e_c;         // coarse correction (F_PROLONG)
  T *f_c;               // coarse right-hand side out (F_RESTRICT)
  double *partials;     // F_NORM_IN: one double per workgroup
  const int *active;    // skip the launch when *active == 0 (NULL: always run)
  int m, mc;            // fine / coarse interior side
  int ntx, nty, tz;     // tiles along x, y; output planes per z-chunk
  int nblocks;          // grid size (for the XCD remap)
  int sw;               // tile order: strips of sw tiles along x (0: whole rows)
  double h2;            // h^2 of the fine level
  double inv_h2;
  double omega;         // weighted Jacobi
};

template <typename T>
struct RestrictArgs {
  const T *u;
  const T *f;
  T *fc;
  const int *active;
  int m, mc;
  double inv_h2;
  // optional stop test of the solve loop, done by workgroup 0 before its
  // share of the restriction (fin_state NULL: none).  The other workgroups
  // may still restrict in the cycle that converges; nothing reads that.
  const double *fin_partials;
  int fin_n;
  SolveState *fin_state;
};

template <typename T>
struct ResidArgs {
  const T *u;
  const T *f;
  T *r;                 // may be NULL (norm only)
  double *partials;     // may be NULL
  const int *active;
  int m;
  int nblocks;
  double inv_h2;
};

// Bottom of the V-cycle for the small levels, one workgroup per problem.
template <typename T>
struct BottomArgs {
  const T *f;           // right-hand side of the first bottom level (global)
  T *u;                 // result on that level (global)
  const int *active;
  int dim, L;           // levels in the bottom sub-hierarchy (finest side 2^L-1)
  int nu1, nu2;
  int smoother;         // 0 RBGS, 1 WJ
  int post_forward;     // post-smoothing in forward order
  int fmg;              // 1: full multigrid over the bottom levels (Algorithm 2)
                        // instead of one V-cycle from zero
  double omega;
};

// Fused LDS-tile kernel for the descent on small coarse levels of a single
// problem: zero start, nsweeps forward sweeps, w = result, fc = FW(f - A w).
// ntile/nblocks are filled by the launcher.
template <typename T>
struct SmallArgs {
  const T *f;
  T *w;
  T *fc;
  const int *active;
  int m, mc, nsweeps, ntile, nblocks;
  double h2, inv_h2;
};

// Outer step of iterative refinement (FP64 residual around FP32 cycles).
struct IrArgs {
  const double *x;      // current iterate
  const float *e;       // correction from the FP32 cycle (NULL: none)
  const double *f;
  double *x_out;        // x + e (never aliases x)
  float *r32;           // (float)(f - A (x + e))
  double *partials;
  const int *active;
  int m, nblocks;       // nblocks must equal ir_blocks(dim, m)
  int cz;               // set by the launcher: planes per workgroup
  double inv_h2;
};

// ---------------------------------------------------------------- launchers
// Tile shape of a fused smoothing pass; the host picks one per level.
struct PassTile {
  int exp_;  // pairs per extended row (= output pairs + halo pairs)
  int ey;    // extended rows (3D) / 1 (2D)
  int nt;    // threads per workgroup
};

// Geometry of a pass launch (computed by pass_geometry).
struct PassGeom {
  int ntx, nty, ntz, tz, nblocks;
};

int pass_variant_count(int dim, int stages, int wj);
PassTile pass_variant(int dim, int stages, int wj, int v);
PassGeom pass_geometry(int dim, int m, int stages, const PassTile &t, int tz,
                       bool restrict_ = false);
// Halo of a red-black pass with S stages, in pairs (x) and rows (3D) on the
// low and high side of the output tile.  Plain passes: S points rounded up to
// a pair, and as many rows as points.  With the folded restriction the final
// values must be exact one point past the tile on the low side and two past
// it on the high side; low-side rows are rounded up to an even count so that
// the tile origin stays on an even row (coarse rows are the odd ones).
struct RbHalo {
  int pl, ph, yl, yh;
};
constexpr RbHalo rb_halo(int S, bool rst) {
  return rst ? RbHalo{(S + 2) / 2, (S + 3) / 2, (S + 2) & ~1, S + 2}
             : RbHalo{(S + 1) / 2, (S + 1) / 2, 2 * ((S + 1) / 2), 2 * ((S + 1) / 2)};
}
// LDS of a red-black pass and whether it fits the per-workgroup limit and
// leaves a valid output tile (an even, positive row count in 3D)
constexpr size_t kMaxPassLds = 160 * 1024;
size_t rb_pass_lds_bytes(int dim, int stages, int exp_, int ey, int flags, size_t elem);
bool rb_pass_fits(int dim, int stages, int variant, int flags, size_t elem);
// FNV-1a hash of the tile tables (shape of every variant index): part of the
// autotuner's cache key, so a cached variant index never names another shape
uint32_t tile_table_hash();

// Launchers.  Batch mode: tbl != NULL points to nent device-resident argument
// entries (one problem each, all with the same level size); the grid gets a
// y-dimension of nent and every workgroup reads its entry.
template <typename T>
hipError_t launch_rb_pass(int dim, int stages, int flags, int variant, PassArgs<T> a,
                          hipStream_t s, const PassArgs<T> *tbl = nullptr, int nent = 1);
template <typename T>
hipError_t launch_wj_pass(int dim, int sweeps, int flags, int variant, PassArgs<T> a,
                          hipStream_t s, const PassArgs<T> *tbl = nullptr, int nent = 1);
template <typename T>
hipError_t launch_restrict(int dim, RestrictArgs<T> a, hipStream_t s,
                           const RestrictArgs<T> *tbl = nullptr, int nent = 1);
template <typename T>
hipError_t launch_residual(int dim, ResidArgs<T> a, hipStream_t s);
int residual_blocks(int dim, int m);
// bottom: tbl != NULL gives one entry (problem) per workgroup; a.L must then
// be the largest entry's level count (it sizes the LDS)
template <typename T>
hipError_t launch_bottom(int nproblems, BottomArgs<T> a, const BottomArgs<T> *tbl, hipStream_t s,
                         size_t lds_bytes = 0);
size_t bottom_lds_bytes(int dim, int L, int smoother, size_t elem);
hipError_t launch_ir_step(int dim, IrArgs a, hipStream_t s);
bool small_level_ok(int dim, int m, int nsweeps, size_t elem);
size_t small_lds_bytes(int dim, int nsweeps, size_t elem);
template <typename T>
hipError_t launch_small(int dim, SmallArgs<T> a, hipStream_t s);
int ir_blocks(int dim, int m);

template <typename T>
hipError_t launch_prolong_add(int dim, int m, int mc, const T *in, const T *ec, T *out,
                              const int *active, hipStream_t s);
hipError_t launch_axpy_f32(double *x, const float *e, size_t n, const int *active, hipStream_t s);

hipError_t launch_finalize(const double *partials, int n, SolveState *st, hipStream_t s);

struct FinEntry {
  const double *partials;
  int n;
  SolveState *st;
};
hipError_t launch_finalize_batch(const FinEntry *tbl, int n, hipStream_t s);
hipError_t launch_state_init_batch(SolveState *st, int n, int maxit, double rtol, hipStream_t s);
hipError_t launch_state_init(SolveState *st, int maxit, double rtol, double res0, hipStream_t s);
hipError_t launch_reduce_norm(const double *partials, int n, double *out, hipStream_t s);
hipError_t launch_copy(const void *src, void *dst, size_t bytes, const int *active, hipStream_t s);

// The paper's smoother and transfers (FP64): one multicolour Gauss-Seidel
// sweep src -> dst (src NULL = zero start; dst must differ from src and f;
// in 3D a sweep is two launches, part 0 then part 1, each relaxing the
// planes of one node-index parity; part is ignored in 2D),
// the fused residual + finite-element restriction (u NULL = zero iterate),
// the finite-element interpolation out = in + P ec (in NULL = zero; in may
// equal out), and the one-node coarsest level.
hipError_t launch_mc_sweep(int dim, int m, const double *src, const double *f, double *dst,
                           int backward, double h2, const int *active, hipStream_t s, int part);
hipError_t launch_restrict_fe(int dim, int m, int mc, const double *u, const double *f, double *fc,
                              double inv_h2, const int *active, hipStream_t s);
hipError_t launch_prolong_fe(int dim, int m, int mc, const double *in, const double *ec,
                             double *out, const int *active, hipStream_t s);
hipError_t launch_coarsest(int dim, const double *f, double *u, int relax, int wj, int nsweeps,
                           double omega, const int *active, hipStream_t s);
hipError_t launch_fill_zero(void *dst, size_t bytes, hipStream_t s);

}  // namespace gmg
