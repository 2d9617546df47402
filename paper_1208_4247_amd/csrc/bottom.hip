// bottom.hip -- the bottom of the V-cycle in one workgroup.
//
// The paper identifies the coarse levels as the hard part of multigrid on a
// GPU: a launch per level and colour leaves almost every compute unit idle
// (Sec. 5.3, the per-level profile of Table 10).  Here every level whose grid
// fits in LDS (side <= 15 in 3D, <= 63 in 2D) is handled by ONE workgroup in
// ONE launch: the whole sub-V-cycle (Algorithm 1 restricted to those levels,
// down to the exactly solved one-node level, see the remark on the
// coarsest-level solver) runs out of LDS with workgroup barriers between the
// colours.  In batch mode the grid has one workgroup per problem.
//
// LDS layout: a level with n = m + 1 = 2^k intervals is stored with pitch n
// in x and y plus zero pad planes, element (x, y, z) at ((z+1) n + y) n + x
// (2D: (y+1) n + x).  Column x = m, row y = m and planes 0 and n are never
// written, so every neighbour is at a fixed offset (+-1, +-n, +-n^2) and the
// Dirichlet zeros come for free.  In-place red-black Gauss-Seidel is
// race-free because a colour's updates only read the other colour and every
// colour ends with a barrier.
//
// Every step of a level is a pass over its points followed by a barrier, and
// on the smallest levels the barrier is most of the cost: a step of a level
// with a handful of points takes as long as one of a level with a thousand.
// The levels whose every step fits one wavefront (one point per lane: side
// <= 7 in 2D, <= 3 in 3D) therefore run in wavefront 0 alone, synchronised
// by waiting for its own LDS operations, while the other wavefronts wait at
// one barrier for the whole sub-cycle.  Each point is computed by the same
// expression either way.
#include "gmg_internal.h"

namespace gmg {

namespace {

struct BL {
  int m, k, n;  // side, log2(n), n = m + 1
  int size;     // padded elements
};

__device__ __forceinline__ BL bl_make(int dim, int L, int l) {
  BL b;
  b.k = L - l;
  b.n = 1 << b.k;
  b.m = b.n - 1;
  b.size = dim == 3 ? (b.n + 1) * b.n * b.n : (b.n + 1) * b.n;
  return b;
}

// The threads that run a step and how a step ends.  W = false: the whole
// workgroup, ending with a barrier.  W = true: wavefront 0 alone (lane =
// threadIdx.x < 64), ending when its LDS operations have completed; the
// "memory" clobber keeps the compiler from moving LDS accesses across it.
template <bool W>
struct Team {
  static __device__ __forceinline__ int stride() { return W ? 64 : (int)blockDim.x; }
  static __device__ __forceinline__ void sync() {
    if (W)
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    else
      __syncthreads();
  }
};

// one colour of red-black Gauss-Seidel on an LDS level
template <typename T, int DIM, bool W>
__device__ void b_rb_colour(const BL &b, T *u, const T *f, int colour, T h2) {
  const int half = b.n >> 1;
  const int rows = DIM == 3 ? b.n * b.m : b.m;  // (y incl. pad row) x z, or y
  const int total = half * rows;
  const int sy = b.n, sz = b.n * b.n;
  for (int h = threadIdx.x; h < total; h += Team<W>::stride()) {
    const int j = h & (half - 1);
    const int row = h >> (b.k - 1);
    int y, z;
    if (DIM == 3) {
      y = row & (b.n - 1);
      z = row >> b.k;
      if (y == b.m) continue;
    } else {
      y = row;
      z = 0;
    }
    const int x = 2 * j + ((y + z + DIM + colour) & 1);
    if (x >= b.m) continue;
    const int i = DIM == 3 ? ((z + 1) * b.n + y) * b.n + x : (y + 1) * b.n + x;
    T nb = u[i - 1] + u[i + 1];
    nb += u[i - sy];
    nb += u[i + sy];
    if (DIM == 3) {
      nb += u[i - sz];
      nb += u[i + sz];
    }
    u[i] = point_solve<T, DIM>(h2, f[i], nb);
  }
  Team<W>::sync();
}

// visit every interior point of a level: fn(i, x, y, z)
template <int DIM, bool W = false, typename F>
__device__ __forceinline__ void b_for_all(const BL &b, F fn) {
  const int total = DIM == 3 ? b.m * b.n * b.n : b.m * b.n;
  for (int h = threadIdx.x; h < total; h += Team<W>::stride()) {
    const int x = h & (b.n - 1);
    const int y = DIM == 3 ? (h >> b.k) & (b.n - 1) : h >> b.k;
    const int z = DIM == 3 ? h >> (2 * b.k) : 0;
    if (x == b.m || (DIM == 3 && y == b.m)) continue;
    const int i = h + (DIM == 3 ? b.n * b.n : b.n);  // skip the leading pad plane/row
    fn(i, x, y, z);
  }
}

template <typename T, int DIM, bool W>
__device__ void b_wj(const BL &b, T *u, const T *f, T *tmp, T h2, T omega) {
  const int sy = b.n, sz = b.n * b.n;
  b_for_all<DIM, W>(b, [&](int i, int, int, int) {
    T nb = u[i - 1] + u[i + 1];
    nb += u[i - sy];
    nb += u[i + sy];
    if (DIM == 3) {
      nb += u[i - sz];
      nb += u[i + sz];
    }
    tmp[i] = (T(1) - omega) * u[i] + omega * point_solve<T, DIM>(h2, f[i], nb);
  });
  Team<W>::sync();
  b_for_all<DIM, W>(b, [&](int i, int, int, int) { u[i] = tmp[i]; });
  Team<W>::sync();
}

template <typename T, int DIM, bool W>
__device__ void b_smooth(const BL &b, T *u, const T *f, T *tmp, int nsw, bool black_first,
                         int smoother, T omega) {
  // h = 1/n with n = 2^k: h and h^2 are exact powers of two
  const T h = ldexp(T(1), -b.k);
  const T h2 = h * h;
  for (int s = 0; s < nsw; ++s) {
    if (smoother == 0) {
      b_rb_colour<T, DIM, W>(b, u, f, black_first ? 1 : 0, h2);
      b_rb_colour<T, DIM, W>(b, u, f, black_first ? 0 : 1, h2);
    } else {
      b_wj<T, DIM, W>(b, u, f, tmp, h2, omega);
    }
  }
}

// fc = FW(f - A u): the residual goes to r (LDS scratch) first
template <typename T, int DIM, bool W = false>
__device__ void b_restrict(const BL &F, const T *u, const T *f, T *r, const BL &C, T *fc) {
  const T inv_h2 = T(F.n) * T(F.n);
  const int sy = F.n, sz = F.n * F.n;
  b_for_all<DIM, W>(F, [&](int i, int, int, int) {
    T nb = u[i - 1] + u[i + 1];
    nb += u[i - sy];
    nb += u[i + sy];
    if (DIM == 3) {
      nb += u[i - sz];
      nb += u[i + sz];
    }
    r[i] = f[i] - (T(2 * DIM) * u[i] - nb) * inv_h2;
  });
  Team<W>::sync();
  b_for_all<DIM, W>(C, [&](int ic, int a, int bb, int c) {
    // fine centre (2a+1, 2b+1, 2c+1)
    const int i = DIM == 3 ? ((2 * c + 2) * F.n + 2 * bb + 1) * F.n + 2 * a + 1
                           : (2 * bb + 2) * F.n + 2 * a + 1;
    auto rowsum = [&](int j) { return T(0.25) * r[j - 1] + T(0.5) * r[j] + T(0.25) * r[j + 1]; };
    auto plane = [&](int j) {
      return T(0.25) * rowsum(j - sy) + T(0.5) * rowsum(j) + T(0.25) * rowsum(j + sy);
    };
    fc[ic] = DIM == 3 ? T(0.25) * plane(i - sz) + T(0.5) * plane(i) + T(0.25) * plane(i + sz)
                      : plane(i);
  });
  Team<W>::sync();
}

// u_F += P u_C (linear interpolation; coarse pads supply the boundary zeros)
template <typename T, int DIM, bool W = false>
__device__ void b_prolong(const BL &F, T *u, const BL &C, const T *uc) {
  const int sy = C.n, sz = C.n * C.n;
  b_for_all<DIM, W>(F, [&](int i, int x, int y, int z) {
    // per axis: fine storage x odd -> coarse storage (x-1)/2; even -> x/2-1 and x/2
    const int cx = (x - 1) >> 1, cy = (y - 1) >> 1, cz = (z - 1) >> 1;
    const bool ox = x & 1, oy = y & 1, oz = z & 1;
    // coarse index of (cx, cy, cz); the pad row/plane at index -1 reads as 0
    const int ci = DIM == 3 ? ((cz + 1) * C.n + cy) * C.n + cx : (cy + 1) * C.n + cx;
    auto xs = [&](int j) { return ox ? uc[j] : T(0.5) * (uc[j] + uc[j + 1]); };
    auto ys = [&](int j) { return oy ? xs(j) : T(0.5) * (xs(j) + xs(j + sy)); };
    T s;
    if (DIM == 3)
      s = oz ? ys(ci) : T(0.5) * (ys(ci) + ys(ci + sz));
    else
      s = ys(ci);
    u[i] += s;
  });
  Team<W>::sync();
}

// element offset of level l's u array (f follows it); levels are packed
// finest first, each as u then f, and the scratch follows the last level
__device__ __forceinline__ int bl_offset(int dim, int L, int l) {
  int off = 0;
  for (int j = 0; j < l; ++j) off += 2 * bl_make(dim, L, j).size;
  return off;
}

// Levels of the bottom hierarchy run by wavefront 0 alone: those whose side
// is at most 7 (2D) or 3 (3D), so that every step has at most one point per
// lane (a colour of a 7 x 7 level has 28 points, the level with its pad
// column 56; a 3^3 level with pads 48).
__device__ __forceinline__ int bl_first_small(int dim, int L) {
  return max(0, L - (dim == 3 ? 2 : 3));
}

// Descent on the levels lo .. hi-1 (smooth from the start value in u, then
// restrict onto level l+1), run by team W.
template <typename T, int DIM, bool W>
__device__ void b_descend(const BottomArgs<T> &a, T *sm, T *R, int L, int lo, int hi, int top,
                          bool clear) {
  const T omega = T(a.omega);
  for (int l = lo; l < hi; ++l) {
    const BL b = bl_make(DIM, L, l), c = bl_make(DIM, L, l + 1);
    T *U = sm + bl_offset(DIM, L, l);
    T *F = U + b.size;
    T *Fc = sm + bl_offset(DIM, L, l + 1) + c.size;
    if (clear && l > top) {
      b_for_all<DIM, W>(b, [&](int i, int, int, int) { U[i] = T(0); });
      Team<W>::sync();
    }
    b_smooth<T, DIM, W>(b, U, F, R, a.nu1, false, a.smoother, omega);
    b_restrict<T, DIM, W>(b, U, F, R, c, Fc);
  }
}

// Ascent on the levels hi-1 down to lo (interpolate and add the correction
// from level l+1, then smooth), run by team W.
template <typename T, int DIM, bool W>
__device__ void b_ascend(const BottomArgs<T> &a, T *sm, T *R, int L, int lo, int hi) {
  const T omega = T(a.omega);
  for (int l = hi - 1; l >= lo; --l) {
    const BL b = bl_make(DIM, L, l), c = bl_make(DIM, L, l + 1);
    T *U = sm + bl_offset(DIM, L, l);
    T *F = U + b.size;
    const T *Uc = sm + bl_offset(DIM, L, l + 1);
    b_prolong<T, DIM, W>(b, U, c, Uc);
    b_smooth<T, DIM, W>(b, U, F, R, a.nu2, !a.post_forward, a.smoother, omega);
  }
}

// one-node level: 2d u / h^2 = f, in FP64 (one lane)
template <typename T, int DIM>
__device__ __forceinline__ void b_coarsest(T *sm, int L) {
  const BL c = bl_make(DIM, L, L - 1);
  T *U = sm + bl_offset(DIM, L, L - 1);
  const int i = DIM == 3 ? c.n * c.n : c.n;  // element (0,0[,0])
  const double h = 1.0 / double(c.n);
  U[i] = T((h * h * double(U[c.size + i])) / double(2 * DIM));
}

// ---- The smallest levels in registers (red-black smoothing) ---------------
// A level with n = 2^k (side m = n - 1, n^DIM <= 64) maps one point to each
// lane of wavefront 0: lane = (z n + y) n + x, x, y (, z) in [0, n), the
// indices equal to m being the zero pads.  Neighbours come from other lanes
// (__shfl), so a step is a few cross-lane reads and the point's arithmetic,
// with no LDS round trip and no wait between steps.  Every expression is the
// one the LDS steps above evaluate, in the same order, with zeros wherever
// they read a pad.  Every lane takes part in every shuffle (a lane that sits
// one out does not supply its value to the others); the results are
// selected afterwards.
template <int DIM>
struct RLev {
  int n, m, x, y, z;
  bool in;  // an interior point of this level
};

template <int DIM>
__device__ __forceinline__ RLev<DIM> rl_make(int k) {
  RLev<DIM> g;
  const int lane = threadIdx.x;
  g.n = 1 << k;
  g.m = g.n - 1;
  g.x = lane & (g.n - 1);
  g.y = (lane >> k) & (g.n - 1);
  g.z = DIM == 3 ? lane >> (2 * k) : 0;
  const bool own = lane < (DIM == 3 ? g.n * g.n * g.n : g.n * g.n);
  g.in = own && g.x < g.m && g.y < g.m && (DIM == 2 || g.z < g.m);
  return g;
}

// the value of v in lane src, or zero when `ok` is false
template <typename T>
__device__ __forceinline__ T lane_val(T v, int src, bool ok) {
  const T r = __shfl(v, src & 63);
  return ok ? r : T(0);
}

// neighbour sum in the order of the LDS steps: x-1 + x+1, then y-1, y+1,
// then z-1, z+1 (pads and indices below zero read as zero)
template <typename T, int DIM>
__device__ __forceinline__ T r_nbsum(const RLev<DIM> &g, T u) {
  const int lane = threadIdx.x, sy = g.n, sz = g.n * g.n;
  const T xm = lane_val(u, lane - 1, g.x > 0), xp = lane_val(u, lane + 1, g.x + 1 < g.m);
  const T ym = lane_val(u, lane - sy, g.y > 0), yp = lane_val(u, lane + sy, g.y + 1 < g.m);
  T nb = xm + xp;
  nb += ym;
  nb += yp;
  if (DIM == 3) {
    const T zm = lane_val(u, lane - sz, g.z > 0), zp = lane_val(u, lane + sz, g.z + 1 < g.m);
    nb += zm;
    nb += zp;
  }
  return nb;
}

template <typename T, int DIM>
__device__ __forceinline__ T r_colour(const RLev<DIM> &g, T u, T f, int colour, T h2) {
  const T nb = r_nbsum<T, DIM>(g, u);
  const bool upd = g.in && ((g.x + g.y + g.z + DIM + colour) & 1) == 0;
  return upd ? point_solve<T, DIM>(h2, f, nb) : u;
}

// full weighting of the fine level's residual onto the coarse lane's point
template <typename T, int DIM>
__device__ __forceinline__ T r_restrict(const RLev<DIM> &F, T u, T f, const RLev<DIM> &C) {
  const T inv_h2 = T(F.n) * T(F.n);
  const T nb = r_nbsum<T, DIM>(F, u);
  const T r = F.in ? f - (T(2 * DIM) * u - nb) * inv_h2 : T(0);
  const int sy = F.n, sz = F.n * F.n;
  const int i = ((DIM == 3 ? (2 * C.z + 1) * F.n : 0) + 2 * C.y + 1) * F.n + 2 * C.x + 1;
  auto R = [&](int j) { return __shfl(r, j & 63); };
  auto rowsum = [&](int j) { return T(0.25) * R(j - 1) + T(0.5) * R(j) + T(0.25) * R(j + 1); };
  auto plane = [&](int j) {
    return T(0.25) * rowsum(j - sy) + T(0.5) * rowsum(j) + T(0.25) * rowsum(j + sy);
  };
  const T fc = DIM == 3 ? T(0.25) * plane(i - sz) + T(0.5) * plane(i) + T(0.25) * plane(i + sz)
                        : plane(i);
  return C.in ? fc : T(0);
}

// u + P uc (linear interpolation from the coarse lanes)
template <typename T, int DIM>
__device__ __forceinline__ T r_prolong(const RLev<DIM> &F, T u, const RLev<DIM> &C, T uc) {
  const int cx = (F.x - 1) >> 1, cy = (F.y - 1) >> 1, cz = (F.z - 1) >> 1;
  const bool ox = F.x & 1, oy = F.y & 1, oz = F.z & 1;
  T v[2][2][2];  // coarse values at (cx + dx, cy + dy, cz + dz), zero outside
#pragma unroll
  for (int dz = 0; dz < (DIM == 3 ? 2 : 1); ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) {
        const int X = cx + dx, Y = cy + dy, Z = cz + dz;
        const bool ok = X >= 0 && X < C.m && Y >= 0 && Y < C.m && (DIM == 2 || (Z >= 0 && Z < C.m));
        v[dz][dy][dx] = lane_val(uc, ((DIM == 3 ? Z * C.n : 0) + Y) * C.n + X, ok);
      }
  auto xs = [&](int dz, int dy) {
    return ox ? v[dz][dy][0] : T(0.5) * (v[dz][dy][0] + v[dz][dy][1]);
  };
  auto ys = [&](int dz) { return oy ? xs(dz, 0) : T(0.5) * (xs(dz, 0) + xs(dz, 1)); };
  T s;
  if (DIM == 3)
    s = oz ? ys(0) : T(0.5) * (ys(0) + ys(1));
  else
    s = ys(0);
  return F.in ? u + s : u;
}

// One V-cycle on D register levels from level side 2^k - 1 (start value u,
// right-hand side f of this lane's point); D = 1 is the one-node level.
template <typename T, int DIM, int D>
__device__ __forceinline__ T r_vcycle(const BottomArgs<T> &a, int k, T u, T f) {
  if constexpr (D == 1) {
    const double h = 1.0 / double(1 << k);  // one-node level: 2d u / h^2 = f, in FP64
    return threadIdx.x == 0 ? T((h * h * double(f)) / double(2 * DIM)) : T(0);
  } else {
    const RLev<DIM> F = rl_make<DIM>(k), C = rl_make<DIM>(k - 1);
    const T h = ldexp(T(1), -k);
    const T h2 = h * h;
    for (int s = 0; s < a.nu1; ++s) {
      u = r_colour<T, DIM>(F, u, f, 0, h2);
      u = r_colour<T, DIM>(F, u, f, 1, h2);
    }
    const T fc = r_restrict<T, DIM>(F, u, f, C);
    const T uc = r_vcycle<T, DIM, D - 1>(a, k - 1, T(0), fc);
    u = r_prolong<T, DIM>(F, u, C, uc);
    const int c0 = a.post_forward ? 0 : 1;
    for (int s = 0; s < a.nu2; ++s) {
      u = r_colour<T, DIM>(F, u, f, c0, h2);
      u = r_colour<T, DIM>(F, u, f, 1 - c0, h2);
    }
    return u;
  }
}

// The levels ls .. L-1 in registers (wavefront 0): start value and
// right-hand side of level ls from LDS, the result back into its u.
template <typename T, int DIM>
__device__ __forceinline__ void b_regs_cycle(const BottomArgs<T> &a, T *sm, int L, int ls, bool from_lds) {
  const BL b = bl_make(DIM, L, ls);
  const RLev<DIM> g = rl_make<DIM>(b.k);
  T *U = sm + bl_offset(DIM, L, ls);
  const T *F = U + b.size;
  const int i = DIM == 3 ? ((g.z + 1) * b.n + g.y) * b.n + g.x : (g.y + 1) * b.n + g.x;
  const T f = g.in ? F[i] : T(0);
  T u = (g.in && from_lds) ? U[i] : T(0);
  switch (L - ls) {
    case 1: u = r_vcycle<T, DIM, 1>(a, b.k, u, f); break;
    case 2: u = r_vcycle<T, DIM, 2>(a, b.k, u, f); break;
    default:
      if constexpr (DIM == 2) u = r_vcycle<T, DIM, 3>(a, b.k, u, f);
      break;
  }
  if (g.in) U[i] = u;
}

// One V-cycle (Algorithm 1) on the levels top .. L-1 of the LDS hierarchy,
// from the start value held in level top's u; the coarser levels start from
// zero (cleared here when `clear`, otherwise already zero).  The levels from
// bl_first_small down, and the one-node level, run in wavefront 0: in
// registers with red-black smoothing, in LDS with weighted Jacobi.
template <typename T, int DIM>
__device__ __forceinline__ void b_vcycle(const BottomArgs<T> &a, T *sm, T *R, int L, int top, bool clear) {
  const int ls = max(top, bl_first_small(DIM, L));
  b_descend<T, DIM, false>(a, sm, R, L, top, ls, top, clear);
  if (threadIdx.x < 64) {
    if (a.smoother == 0) {
      // the start value of level ls: the caller's at the top, else zero
      b_regs_cycle<T, DIM>(a, sm, L, ls, ls == top);
    } else {
      b_descend<T, DIM, true>(a, sm, R, L, ls, L - 1, top, clear);
      if (threadIdx.x == 0) b_coarsest<T, DIM>(sm, L);
      Team<true>::sync();
      b_ascend<T, DIM, true>(a, sm, R, L, ls, L - 1);
    }
  }
  __syncthreads();
  b_ascend<T, DIM, false>(a, sm, R, L, top, ls);
}

template <typename T, int DIM>
__device__ __forceinline__ void bottom_body(const BottomArgs<T> &a, const GMG_GLOBAL T *fin, GMG_GLOBAL T *uout, T *sm) {
  const int L = a.L;
  const int total = bl_offset(DIM, L, L) + bl_make(DIM, L, 0).size;
  T *R = sm + bl_offset(DIM, L, L);  // residual / Jacobi scratch, size of level 0
  for (int i = threadIdx.x; i < total; i += blockDim.x) sm[i] = T(0);
  __syncthreads();
  const BL b0 = bl_make(DIM, L, 0);
  {
    T *F0 = sm + b0.size;
    b_for_all<DIM>(b0, [&](int i, int x, int y, int z) {
      const int m = b0.m;
      F0[i] = fin[DIM == 3 ? (z * m + y) * m + x : y * m + x];
    });
  }
  __syncthreads();
  if (!a.fmg) {
    b_vcycle<T, DIM>(a, sm, R, L, 0, false);
  } else {
    // Algorithm 2: f to every level by full weighting (the residual of the
    // zero iterate), the coarsest level exactly, then per level from the
    // coarse end: interpolate the coarser solution and run one V-cycle
    for (int l = 0; l + 1 < L; ++l) {
      const BL b = bl_make(DIM, L, l), c = bl_make(DIM, L, l + 1);
      T *U = sm + bl_offset(DIM, L, l);
      b_restrict<T, DIM>(b, U, U + b.size, R, c, sm + bl_offset(DIM, L, l + 1) + c.size);
    }
    if (threadIdx.x == 0) b_coarsest<T, DIM>(sm, L);
    __syncthreads();
    for (int l = L - 2; l >= 0; --l) {
      const BL b = bl_make(DIM, L, l), c = bl_make(DIM, L, l + 1);
      b_prolong<T, DIM>(b, sm + bl_offset(DIM, L, l), c, sm + bl_offset(DIM, L, l + 1));
      b_vcycle<T, DIM>(a, sm, R, L, l, true);
    }
  }
  b_for_all<DIM>(b0, [&](int i, int x, int y, int z) {
    const int m = b0.m;
    uout[DIM == 3 ? (z * m + y) * m + x : y * m + x] = sm[i];
  });
}

}  // namespace

template <typename T>
__global__ void __launch_bounds__(1024) k_bottom(BottomArgs<T> arg, const BottomArgs<T> *tbl) {
  const BottomArgs<T> a = tbl ? tbl[blockIdx.x] : arg;  // batch: one problem per workgroup
  if (a.active && *gbl(a.active) == 0) return;
  const GMG_GLOBAL T *fin = gbl(a.f);
  GMG_GLOBAL T *uout = gbl(a.u);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *sm = reinterpret_cast<T *>(smem_raw);
  if (a.dim == 3)
    bottom_body<T, 3>(a, fin, uout, sm);
  else
    bottom_body<T, 2>(a, fin, uout, sm);
}

size_t bottom_lds_bytes(int dim, int L, int smoother, size_t elem) {
  (void)smoother;  // weighted Jacobi reuses the residual scratch
  size_t n_el = 0;
  for (int l = 0; l < L; ++l) {
    const size_t n = (size_t)1 << (L - l);
    n_el += 2 * (dim == 3 ? (n + 1) * n * n : (n + 1) * n);
  }
  const size_t n0 = (size_t)1 << L;
  n_el += dim == 3 ? (n0 + 1) * n0 * n0 : (n0 + 1) * n0;
  return n_el * elem;
}

template <typename T>
hipError_t launch_bottom(int nproblems, BottomArgs<T> a, const BottomArgs<T> *tbl, hipStream_t s,
                         size_t lds_bytes) {
  const size_t lds = lds_bytes ? lds_bytes : bottom_lds_bytes(a.dim, a.L, a.smoother, sizeof(T));
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void *)k_bottom<T>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int nt = (a.dim == 3 && a.L <= 3) || (a.dim == 2 && a.L <= 4) ? 256 : 1024;
  gmg_launch(k_bottom<T>, dim3(nproblems), dim3(nt), lds, s, a, tbl);
  return hipGetLastError();
}

template hipError_t launch_bottom<double>(int, BottomArgs<double>, const BottomArgs<double> *,
                                          hipStream_t, size_t);
template hipError_t launch_bottom<float>(int, BottomArgs<float>, const BottomArgs<float> *,
                                         hipStream_t, size_t);

}  // namespace gmg
