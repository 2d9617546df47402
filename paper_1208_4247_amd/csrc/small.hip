// small.hip -- fused LDS-tile kernel for the descent on small coarse levels.
//
// On a coarse level of side <= 63 (3D) / <= 511 (2D) a z-marching pass is
// latency bound: every plane step waits on L2 loads and barriers.  Here one
// workgroup owns a small cube (3D) or square (2D) of fine points, loads it
// once with a halo wide enough for every fused step, and runs the level's
// whole descent in LDS: u = 0; S = 2 nu1 red-black half-sweeps (Algorithm
// 1's Relax_forward from the zero coarse start value); write w on the core;
// r = f - A w on the core and a one-point ring; full weighting of r to the
// coarse points of the tile.  (The ascent always takes the plane-marching
// pass: an LDS-tile version of it measured slower on every level.)
//
// Halo values are recomputed by neighbouring workgroups (the redundancy is
// cheap at these sizes: everything lives in L2).  Stage s is evaluated on
// local coordinates [s, E-s), which is exact given exact stage s-1 values on
// [s-1, E-s+1), so after S stages the box [S, E-S) is exact.  The box
// starts S+1 points before the core and ends S+2 after it: full weighting
// of the tile's last coarse point needs the residual one point past the
// core, which needs u one point further.  Results are the same bits as the
// z-marching passes: every half-sweep evaluates the same per-point
// expression on the same inputs.
#include "gmg_internal.h"

namespace gmg {

namespace {

__device__ __forceinline__ int xcd_remap_s(int bid, int n) {
  const int xcd = bid & 7, loc = bid >> 3;
  const int per = n >> 3, rem = n & 7;
  return xcd * per + min(xcd, rem) + loc;
}

template <int DIM>
struct Box {
  int E;            // edge of the tile in points
  int o[3];         // global coordinate of local 0 per axis (x, y, z)
  __device__ int size() const { return DIM == 3 ? E * E * E : E * E; }
};

// visit local points with coordinates in [lo, hi) on every axis:
// fn(i, lx, ly, lz)
template <int DIM, typename F>
__device__ __forceinline__ void box_for(int E, int lo, int hi, F fn) {
  const int w = hi - lo;
  if (w <= 0) return;
  const int n = DIM == 3 ? w * w * w : w * w;
  for (int h = threadIdx.x; h < n; h += blockDim.x) {
    const int lx = lo + h % w;
    const int ly = lo + (h / w) % w;
    const int lz = DIM == 3 ? lo + h / (w * w) : 0;
    const int i = DIM == 3 ? (lz * E + ly) * E + lx : ly * E + lx;
    fn(i, lx, ly, lz);
  }
}

template <typename T, int DIM>
__device__ __forceinline__ T nb_sum(const T *u, int i, int E) {
  T nb = u[i - 1] + u[i + 1];
  nb += u[i - E];
  nb += u[i + E];
  if (DIM == 3) {
    nb += u[i - E * E];
    nb += u[i + E * E];
  }
  return nb;
}

template <int DIM>
__device__ __forceinline__ bool in_dom(const Box<DIM> &b, int lx, int ly, int lz, int m) {
  const int gx = b.o[0] + lx, gy = b.o[1] + ly;
  if (gx < 0 || gx >= m || gy < 0 || gy >= m) return false;
  if (DIM == 3) {
    const int gz = b.o[2] + lz;
    if (gz < 0 || gz >= m) return false;
  }
  return true;
}

template <int DIM>
__device__ __forceinline__ size_t gidx(const Box<DIM> &b, int lx, int ly, int lz, int m) {
  const size_t gx = b.o[0] + lx, gy = b.o[1] + ly;
  if (DIM == 3) return ((size_t)(b.o[2] + lz) * m + gy) * m + gx;
  return gy * m + gx;
}

// S red-black half-sweeps in LDS, stage s on local coordinates [s, E-s)
template <typename T, int DIM>
__device__ void lds_sweeps(const Box<DIM> &b, T *u, const T *f, int S, int c1, int m, T h2) {
  const int E = b.E;
  for (int s = 1; s <= S; ++s) {
    const int cs = (c1 + s - 1) & 1;
    box_for<DIM>(E, s, E - s, [&](int i, int lx, int ly, int lz) {
      const int gx = b.o[0] + lx, gy = b.o[1] + ly, gz = DIM == 3 ? b.o[2] + lz : 0;
      if (((gx + gy + gz + DIM) & 1) != cs) return;
      if (!in_dom<DIM>(b, lx, ly, lz, m)) return;
      u[i] = point_solve<T, DIM>(h2, f[i], nb_sum<T, DIM>(u, i, E));
    });
    __syncthreads();
  }
}

}  // namespace

// local coordinates of local index i in a box of edge E (compile-time E)
template <int DIM, int E>
__device__ __forceinline__ void box_coord(int i, int &lx, int &ly, int &lz) {
  lx = i % E;
  ly = (i / E) % E;
  lz = DIM == 3 ? i / (E * E) : 0;
}

// ------------------------------------------------------------------ descent
template <typename T, int DIM, int CT, int NSW, int NT>
__global__ void __launch_bounds__(NT) k_small_down(SmallArgs<T> a) {
  if (a.active && *gbl(a.active) == 0) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int S = 2 * NSW;
  constexpr int H = S + 1;  // local index of the first core point
  constexpr int E = 2 * CT + 2 * S + 3;
  constexpr int N = DIM == 3 ? E * E * E : E * E;
  constexpr int NPT = (N + NT - 1) / NT;
  const int m = a.m, mc = a.mc;
  Box<DIM> b;
  b.E = E;
  const int nt = a.ntile;
  const int bid = xcd_remap_s(blockIdx.x, a.nblocks);
  const int tx = bid % nt, ty = (bid / nt) % nt, tz = DIM == 3 ? bid / (nt * nt) : 0;
  const int A0[3] = {tx * CT, ty * CT, tz * CT};  // first coarse point of the tile
  for (int k = 0; k < 3; ++k) b.o[k] = 2 * A0[k] - H;
  T *u = reinterpret_cast<T *>(smem_raw);
  T *f = u + N;
  const T h2 = T(a.h2);
  const T inv_h2 = T(a.inv_h2);
  {  // all loads of a thread in flight before any store
    T fv[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const int i = threadIdx.x + NT * k;
      int lx, ly, lz;
      box_coord<DIM, E>(i, lx, ly, lz);
      fv[k] = (i < N && in_dom<DIM>(b, lx, ly, lz, m)) ? gbl(a.f)[gidx<DIM>(b, lx, ly, lz, m)] : T(0);
    }
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
      const int i = threadIdx.x + NT * k;
      if (i < N) {
        u[i] = T(0);
        f[i] = fv[k];
      }
    }
  }
  __syncthreads();
  lds_sweeps<T, DIM>(b, u, f, S, 0, m, h2);
  // pre-smoothed values on the core (fine points 2*A0 .. 2*A0 + 2CT - 1)
  box_for<DIM>(E, H, H + 2 * CT, [&](int i, int lx, int ly, int lz) {
    if (in_dom<DIM>(b, lx, ly, lz, m)) gbl(a.w)[gidx<DIM>(b, lx, ly, lz, m)] = u[i];
  });
  // residual on the core and one point past it (f is overwritten in place:
  // each point reads only its own f and the neighbours' u)
  box_for<DIM>(E, H, H + 2 * CT + 1, [&](int i, int, int, int) {
    f[i] = f[i] - (T(2 * DIM) * u[i] - nb_sum<T, DIM>(u, i, E)) * inv_h2;
  });
  __syncthreads();
  // full weighting to the tile's coarse points
  constexpr int NC = DIM == 3 ? CT * CT * CT : CT * CT;
  for (int h = threadIdx.x; h < NC; h += NT) {
    const int ax = h % CT, ay = (h / CT) % CT, az = DIM == 3 ? h / (CT * CT) : 0;
    const int cx = A0[0] + ax, cy = A0[1] + ay, cz = A0[2] + az;
    if (cx >= mc || cy >= mc || (DIM == 3 && cz >= mc)) continue;
    // fine centre 2a+1 -> local 2*ax + 1 + H
    const int lx = 2 * ax + 1 + H, ly = 2 * ay + 1 + H, lz = DIM == 3 ? 2 * az + 1 + H : 0;
    const int i = DIM == 3 ? (lz * E + ly) * E + lx : ly * E + lx;
    auto row = [&](int j) { return T(0.25) * f[j - 1] + T(0.5) * f[j] + T(0.25) * f[j + 1]; };
    auto pl = [&](int j) { return T(0.25) * row(j - E) + T(0.5) * row(j) + T(0.25) * row(j + E); };
    const T v = DIM == 3 ? T(0.25) * pl(i - E * E) + T(0.5) * pl(i) + T(0.25) * pl(i + E * E)
                         : pl(i);
    const size_t o = DIM == 3 ? ((size_t)cz * mc + cy) * mc + cx : (size_t)cy * mc + cx;
    gbl(a.fc)[o] = v;
  }
}

// ------------------------------------------------------------------ launchers
namespace {
constexpr int kCT3 = 4, kCT2 = 16;
constexpr int kNT3 = 1024, kNT2 = 512;

template <typename T, int DIM, int NSW>
hipError_t run_small(SmallArgs<T> a, hipStream_t s, size_t lds) {
  constexpr int CT = DIM == 3 ? kCT3 : kCT2;
  constexpr int NT = DIM == 3 ? kNT3 : kNT2;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void *)k_small_down<T, DIM, CT, NSW, NT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 120 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  gmg_launch((k_small_down<T, DIM, CT, NSW, NT>), dim3(a.nblocks), dim3(NT), lds, s, a);
  return hipGetLastError();
}
}  // namespace


size_t small_lds_bytes(int dim, int nsweeps, size_t elem) {
  const int S = 2 * nsweeps;
  const int ct = dim == 3 ? kCT3 : kCT2;
  const size_t E = 2 * ct + 2 * S + 3;
  const size_t N = dim == 3 ? E * E * E : E * E;
  return 2 * N * elem;
}

bool small_level_ok(int dim, int m, int nsweeps, size_t elem) {
  if (nsweeps < 1 || nsweeps > 3) return false;
  if (dim == 3 ? m > 63 : m > 511) return false;
  return small_lds_bytes(dim, nsweeps, elem) <= 120 * 1024;
}

template <typename T>
hipError_t launch_small(int dim, SmallArgs<T> a, hipStream_t s) {
  const int ct = dim == 3 ? kCT3 : kCT2;
  // tiles of ct coarse points; their fine cores (2 ct points) cover all
  // m = 2 mc + 1 fine points
  a.ntile = (a.m + 2 * ct - 1) / (2 * ct);
  a.nblocks = dim == 3 ? a.ntile * a.ntile * a.ntile : a.ntile * a.ntile;
  const size_t lds = small_lds_bytes(dim, a.nsweeps, sizeof(T));
  if (dim == 3) {
    switch (a.nsweeps) {
      case 1: return run_small<T, 3, 1>(a, s, lds);
      case 2: return run_small<T, 3, 2>(a, s, lds);
      default: return hipErrorInvalidValue;
    }
  }
  switch (a.nsweeps) {
    case 1: return run_small<T, 2, 1>(a, s, lds);
    case 2: return run_small<T, 2, 2>(a, s, lds);
    case 3: return run_small<T, 2, 3>(a, s, lds);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_small<double>(int, SmallArgs<double>, hipStream_t);
template hipError_t launch_small<float>(int, SmallArgs<float>, hipStream_t);

}  // namespace gmg
