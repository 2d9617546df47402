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
// In-place red-black Gauss-Seidel is race-free here because a colour's
// updates only read the other colour and every colour ends with a barrier.
#include "gmg_internal.h"

namespace gmg {

template <typename T>
struct BLevel {
  int m;
  T *u, *f;
};

template <typename T>
__device__ __forceinline__ T at(const T *v, int m, int dim, int x, int y, int z) {
  if (x < 0 || y < 0 || x >= m || y >= m) return T(0);
  if (dim == 3) {
    if (z < 0 || z >= m) return T(0);
    return v[(z * m + y) * m + x];
  }
  return v[y * m + x];
}

template <typename T>
__device__ __forceinline__ T nbsum(const T *v, int m, int dim, int x, int y, int z) {
  T nb = at(v, m, dim, x - 1, y, z) + at(v, m, dim, x + 1, y, z);
  nb += at(v, m, dim, x, y - 1, z);
  nb += at(v, m, dim, x, y + 1, z);
  if (dim == 3) {
    nb += at(v, m, dim, x, y, z - 1);
    nb += at(v, m, dim, x, y, z + 1);
  }
  return nb;
}

template <typename T>
__device__ void b_rb_colour(BLevel<T> L, int dim, int colour) {
  const int N = dim == 3 ? L.m * L.m * L.m : L.m * L.m;
  const T h = T(1) / T(L.m + 1);
  const T h2 = h * h;
  const T inv2d = dim == 3 ? T(1.0 / 6.0) : T(0.25);
  for (int p = threadIdx.x; p < N; p += blockDim.x) {
    const int x = p % L.m, y = (p / L.m) % L.m, z = dim == 3 ? p / (L.m * L.m) : 0;
    if (((x + y + z + dim) & 1) != colour) continue;
    const T nb = nbsum(L.u, L.m, dim, x, y, z);
    L.u[p] = fma(h2, L.f[p], nb) * inv2d;
  }
  __syncthreads();
}

template <typename T>
__device__ void b_wj(BLevel<T> L, int dim, T *tmp, T omega) {
  const int N = dim == 3 ? L.m * L.m * L.m : L.m * L.m;
  const T h = T(1) / T(L.m + 1);
  const T h2 = h * h;
  const T inv2d = dim == 3 ? T(1.0 / 6.0) : T(0.25);
  for (int p = threadIdx.x; p < N; p += blockDim.x) {
    const int x = p % L.m, y = (p / L.m) % L.m, z = dim == 3 ? p / (L.m * L.m) : 0;
    const T nb = nbsum(L.u, L.m, dim, x, y, z);
    tmp[p] = (T(1) - omega) * L.u[p] + omega * (fma(h2, L.f[p], nb) * inv2d);
  }
  __syncthreads();
  for (int p = threadIdx.x; p < N; p += blockDim.x) L.u[p] = tmp[p];
  __syncthreads();
}

template <typename T>
__device__ void b_smooth(BLevel<T> L, int dim, int nsw, bool black_first, int smoother, T *tmp,
                         T omega) {
  for (int s = 0; s < nsw; ++s) {
    if (smoother == 0) {
      b_rb_colour(L, dim, black_first ? 1 : 0);
      b_rb_colour(L, dim, black_first ? 0 : 1);
    } else {
      b_wj(L, dim, tmp, omega);
    }
  }
}

// f_c = FW(f - A u) with the residual formed on the fly (27 / 9 points).
template <typename T>
__device__ void b_restrict(BLevel<T> F, BLevel<T> C, int dim) {
  const int Nc = dim == 3 ? C.m * C.m * C.m : C.m * C.m;
  const T h = T(1) / T(F.m + 1);
  const T inv_h2 = T(1) / (h * h);
  const T w[3] = {T(0.25), T(0.5), T(0.25)};
  for (int p = threadIdx.x; p < Nc; p += blockDim.x) {
    const int a = p % C.m, b = (p / C.m) % C.m, c = dim == 3 ? p / (C.m * C.m) : 0;
    T s = T(0);
    const int nz = dim == 3 ? 3 : 1;
    for (int oz = 0; oz < nz; ++oz)
      for (int oy = 0; oy < 3; ++oy)
        for (int ox = 0; ox < 3; ++ox) {
          const int x = 2 * a + ox, y = 2 * b + oy, z = dim == 3 ? 2 * c + oz : 0;
          const int q = dim == 3 ? (z * F.m + y) * F.m + x : y * F.m + x;
          const T r = F.f[q] - (T(2 * dim) * F.u[q] - nbsum(F.u, F.m, dim, x, y, z)) * inv_h2;
          const T wt = dim == 3 ? w[ox] * w[oy] * w[oz] : w[ox] * w[oy];
          s += wt * r;
        }
    C.f[p] = s;
  }
  __syncthreads();
}

// F.u += P C.u (linear interpolation, zero coarse boundary).
template <typename T>
__device__ void b_prolong(BLevel<T> F, BLevel<T> C, int dim) {
  const int N = dim == 3 ? F.m * F.m * F.m : F.m * F.m;
  for (int p = threadIdx.x; p < N; p += blockDim.x) {
    const int x = p % F.m, y = (p / F.m) % F.m, z = dim == 3 ? p / (F.m * F.m) : 0;
    int cx[2], cy[2], cz[2];
    T wx[2], wy[2], wz[2];
    auto axis = [](int v, int *c, T *wt) -> int {
      if (v & 1) {
        c[0] = (v - 1) >> 1;
        wt[0] = T(1);
        return 1;
      }
      c[0] = (v >> 1) - 1;
      c[1] = v >> 1;
      wt[0] = wt[1] = T(0.5);
      return 2;
    };
    const int nx = axis(x, cx, wx), ny = axis(y, cy, wy);
    const int nz = dim == 3 ? axis(z, cz, wz) : 1;
    if (dim == 2) {
      cz[0] = 0;
      wz[0] = T(1);
    }
    T s = T(0);
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          const T v = at(C.u, C.m, dim, cx[i], cy[j], cz[k]);
          s += (dim == 3 ? wx[i] * wy[j] * wz[k] : wx[i] * wy[j]) * v;
        }
    F.u[p] += s;
  }
  __syncthreads();
}

template <typename T>
__global__ void __launch_bounds__(1024) k_bottom(BottomArgs<T> a, const T *const *f_list,
                                                 T *const *u_list, int active_stride) {
  const int prob = blockIdx.x;
  if (a.active && a.active[(size_t)prob * active_stride] == 0) return;
  const T *fin = f_list ? f_list[prob] : a.f;
  T *uout = u_list ? u_list[prob] : a.u;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *sm = reinterpret_cast<T *>(smem_raw);
  const int dim = a.dim, L = a.L;
  BLevel<T> lv[12];
  size_t off = 0;
  for (int l = 0; l < L; ++l) {
    lv[l].m = (1 << (L - l)) - 1;
    const int N = dim == 3 ? lv[l].m * lv[l].m * lv[l].m : lv[l].m * lv[l].m;
    lv[l].u = sm + off;
    off += N;
    lv[l].f = sm + off;
    off += N;
  }
  T *tmp = sm + off;
  const T omega = T(a.omega);
  const int N0 = dim == 3 ? lv[0].m * lv[0].m * lv[0].m : lv[0].m * lv[0].m;
  for (int p = threadIdx.x; p < N0; p += blockDim.x) {
    lv[0].f[p] = fin[p];
    lv[0].u[p] = T(0);
  }
  __syncthreads();
  for (int l = 0; l + 1 < L; ++l) {
    if (l > 0) {
      const int N = dim == 3 ? lv[l].m * lv[l].m * lv[l].m : lv[l].m * lv[l].m;
      for (int p = threadIdx.x; p < N; p += blockDim.x) lv[l].u[p] = T(0);
      __syncthreads();
    }
    b_smooth(lv[l], dim, a.nu1, false, a.smoother, tmp, omega);
    b_restrict(lv[l], lv[l + 1], dim);
  }
  // one-node level: exact solve 2d u / h^2 = f, evaluated in FP64
  if (threadIdx.x == 0) {
    const double h = 1.0 / double(lv[L - 1].m + 1);
    lv[L - 1].u[0] = T((h * h * double(lv[L - 1].f[0])) / double(2 * dim));
  }
  __syncthreads();
  for (int l = L - 2; l >= 0; --l) {
    b_prolong(lv[l], lv[l + 1], dim);
    b_smooth(lv[l], dim, a.nu2, !a.post_forward, a.smoother, tmp, omega);
  }
  for (int p = threadIdx.x; p < N0; p += blockDim.x) uout[p] = lv[0].u[p];
}

size_t bottom_lds_bytes(int dim, int L, int smoother, size_t elem) {
  size_t n = 0;
  for (int l = 0; l < L; ++l) {
    const size_t m = ((size_t)1 << (L - l)) - 1;
    n += 2 * (dim == 3 ? m * m * m : m * m);
  }
  const size_t m0 = ((size_t)1 << L) - 1;
  if (smoother == 1) n += dim == 3 ? m0 * m0 * m0 : m0 * m0;
  return n * elem;
}

template <typename T>
hipError_t launch_bottom(int nproblems, BottomArgs<T> a, const T *const *f_list, T *const *u_list,
                         hipStream_t s) {
  const size_t lds = bottom_lds_bytes(a.dim, a.L, a.smoother, sizeof(T));
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void *)k_bottom<T>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int stride = (int)(sizeof(SolveState) / sizeof(int));
  hipLaunchKernelGGL(k_bottom<T>, dim3(nproblems), dim3(1024), lds, s, a, f_list, u_list, stride);
  return hipGetLastError();
}

template hipError_t launch_bottom<double>(int, BottomArgs<double>, const double *const *,
                                          double *const *, hipStream_t);
template hipError_t launch_bottom<float>(int, BottomArgs<float>, const float *const *,
                                         float *const *, hipStream_t);

}  // namespace gmg
