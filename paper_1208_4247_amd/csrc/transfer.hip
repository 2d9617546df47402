// transfer.hip -- residual, full-weighting restriction, norm reduction and the
// solve-state update for the multigrid library (gfx950).
//
// Residual: r = f - A u with (A u)_p = (2d u_p - sum of neighbours) / h^2
// (Sec. 4, eq. residual_2D and its 3D count).  Restriction: full weighting,
// the tensor product of [1/4, 1/2, 1/4] (Algorithm 1's f_{l+1} = R r_l with
// the standard weights).  Norm: Euclidean norm of the residual (Sec. 4, eq.
// Inner_product2D, with the square root), summed in a fixed order so that the
// stop decision is reproducible.
#include "gmg_internal.h"

namespace gmg {

__device__ __forceinline__ int xcd_remap_t(int bid, int n) {
  const int xcd = bid & 7, loc = bid >> 3;
  const int per = n >> 3, rem = n & 7;
  return xcd * per + min(xcd, rem) + loc;
}

// ------------------------------------------------------------------------
// Fixed-order reduction of per-block partial sums (the first 64 threads) and
// the stop test of the solve loop (Algorithm 3's while condition).
// ------------------------------------------------------------------------
__device__ __forceinline__ double sum_partials(const double *p, int n) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 64) s += p[i];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off);
  return s;
}

__device__ __forceinline__ void update_state(SolveState *st, double tot) {
  const double res = sqrt(tot);
  if (st->res0 < 0.0) st->res0 = res;
  st->res = res;
  const double res0 = st->res0;
  if (!isfinite(res)) {
    st->status = -3;
    st->active = 0;
  } else if (!(res > st->rtol * res0)) {
    st->status = 0;
    st->active = 0;
  } else if (res > 1e3 * res0 && st->iter > 0) {
    st->status = -4;
    st->active = 0;
  } else if (st->iter >= st->maxit) {
    st->status = 1;
    st->active = 0;
  } else {
    st->iter += 1;  // admit one more cycle
  }
}

// ------------------------------------------------------------------------
// Residual + full weighting: the residual is formed in LDS one fine plane at
// a time and reduced to coarse points without ever being stored.
// Workgroup: a CX x CY block of coarse columns (3D; CX x 1 in 2D) marching
// over a chunk of coarse planes (rows in 2D).  Fine u planes sit in a
// three-plane LDS ring; the next u plane and the next f plane are loaded into
// registers one step ahead, so global latency overlaps the LDS work.
// ------------------------------------------------------------------------
// Argument block of this workgroup: the kernel argument, or (batch mode) table
// entry e, read through the scalar cache so that the plane resources built
// from it stay in scalar registers.
template <typename A>
__device__ __forceinline__ A uniform_entry(const A &arg, const A *tbl, unsigned e) {
  if (!tbl) return arg;
  A r;
  __builtin_memcpy(&r, (const __attribute__((address_space(4))) A *)tbl + e, sizeof(A));
  return r;
}

template <typename T, int DIM, int CX, int CY, int NT>
__global__ void __launch_bounds__(NT) k_restrict(RestrictArgs<T> arg, const RestrictArgs<T> *tbl,
                                                 int ncx, int ncy, int czc, int nblocks) {
  const RestrictArgs<T> a = uniform_entry(arg, tbl, blockIdx.y);  // batch: one entry per blockIdx.y
  if (a.active && *a.active == 0) return;
  if (a.fin_state && blockIdx.x == 0 && threadIdx.x < 64) {
    const double tot = sum_partials(a.fin_partials, a.fin_n);
    if (threadIdx.x == 0) update_state(a.fin_state, tot);
  }
  const int m = a.m, mc = a.mc;
  const int bid = xcd_remap_t(blockIdx.x, nblocks);
  const int bx = bid % ncx;
  const int rest = bid / ncx;
  const int by = DIM == 3 ? rest % ncy : 0;
  const int bz = DIM == 3 ? rest / ncy : rest;
  const int A0 = bx * CX;
  const int B0 = DIM == 3 ? by * CY : 0;
  const int C0 = bz * czc;
  const int C1 = min(C0 + czc, mc);
  constexpr int RX = 2 * CX + 1;
  constexpr int RY = DIM == 3 ? 2 * CY + 1 : 1;
  constexpr int UX = RX + 2;
  constexpr int UY = DIM == 3 ? RY + 2 : 1;
  constexpr int NU = (UX * UY + NT - 1) / NT;
  constexpr int NR = (RX * RY + NT - 1) / NT;
  __shared__ T su[3][UY * UX];  // fine u planes, ring indexed by (z + 3) % 3
  __shared__ T sr[RY * RX];     // fine residual of the current plane
  const T inv_h2 = T(a.inv_h2);
  const T two_d = T(2 * DIM);
  const int planeS = DIM == 3 ? m * m : m;
  GMG_GLOBAL T *__restrict__ fcg = gbl(a.fc);

  // u-tile element q -> byte offset in its plane, out of range (kOOB) outside
  // the domain: loads go through one-plane buffer resources, so the zero
  // boundary and a missing u (zero start) cost no branches and the next
  // plane's loads stay in flight across the current plane's work
  int uo[NU];
#pragma unroll
  for (int k = 0; k < NU; ++k) {
    const int q = threadIdx.x + NT * k;
    const int ux = q % UX, uy = q / UX;
    const int x = 2 * A0 - 1 + ux, y = DIM == 3 ? 2 * B0 - 1 + uy : 0;
    const bool in = q < UX * UY && x >= 0 && x < m && y >= 0 && y < m;
    uo[k] = in ? (DIM == 3 ? y * m + x : x) * (int)sizeof(T) : kOOB;
  }
  int ro[NR];
  bool rin[NR];
#pragma unroll
  for (int k = 0; k < NR; ++k) {
    const int q = threadIdx.x + NT * k;
    const int rx = q % RX, ry = q / RX;
    const int x = 2 * A0 + rx, y = DIM == 3 ? 2 * B0 + ry : 0;
    rin[k] = q < RX * RY && x < m && y < m;
    ro[k] = rin[k] ? (DIM == 3 ? y * m + x : x) * (int)sizeof(T) : kOOB;
  }
  auto load_u = [&](int z, T *v) {
    // no u: a plane index outside the grid gives a resource with no records
    const __amdgpu_buffer_rsrc_t r = plane_rsrc(a.u ? a.u : a.f, a.u ? z : -1, m, planeS);
#pragma unroll
    for (int k = 0; k < NU; ++k) v[k] = bload<T>(r, uo[k]);
  };
  auto load_f = [&](int z, T *v) {
    const __amdgpu_buffer_rsrc_t r = plane_rsrc(a.f, z, m, planeS);
#pragma unroll
    for (int k = 0; k < NR; ++k) v[k] = bload<T>(r, ro[k]);
  };
  auto store_u = [&](int z, const T *v) {
    T *dst = su[(z + 3) % 3];
#pragma unroll
    for (int k = 0; k < NU; ++k) {
      const int q = threadIdx.x + NT * k;
      if (q < UX * UY) dst[q] = v[k];
    }
  };

  const int cxl = threadIdx.x % CX;
  const int cyl = DIM == 3 ? (threadIdx.x / CX) % CY : 0;
  const bool cown = threadIdx.x < CX * (DIM == 3 ? CY : 1);
  const int cx = A0 + cxl, cy = B0 + cyl;
  const bool cvalid = cown && cx < mc && (DIM == 2 || cy < mc);
  T acc = T(0);

  const int zf0 = 2 * C0, zf1 = 2 * C1;  // fine residual planes zf0 .. zf1
  {
    T v[NU];
    load_u(zf0 - 1, v);
    store_u(zf0 - 1, v);
    load_u(zf0, v);
    store_u(zf0, v);
    load_u(zf0 + 1, v);
    store_u(zf0 + 1, v);
  }
  T pf[NR];
  load_f(zf0, pf);
  __syncthreads();
  for (int zf = zf0; zf <= zf1; ++zf) {
    T nu[NU], nf[NR];
    load_u(zf + 2, nu);
    load_f(zf + 1, nf);
    const T *um = su[(zf - 1 + 3) % 3];
    const T *u0 = su[(zf + 3) % 3];
    const T *up = su[(zf + 1 + 3) % 3];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const int q = threadIdx.x + NT * k;
      if (q >= RX * RY) continue;
      const int rx = q % RX, ry = q / RX;
      T r = T(0);
      if (rin[k] && zf < m) {
        const int c = (ry + (DIM == 3 ? 1 : 0)) * UX + rx + 1;  // centre in the u tile
        T nb = u0[c - 1] + u0[c + 1];
        if (DIM == 3) {
          nb += u0[c - UX];
          nb += u0[c + UX];
        }
        nb += um[c];
        nb += up[c];
        r = pf[k] - (two_d * u0[c] - nb) * inv_h2;
      }
      sr[q] = r;
    }
    __syncthreads();
    // fine plane zf = 2c+1 weighs 1/2 for coarse plane c; zf = 2c+2 weighs
    // 1/4 for coarse planes c and c+1
    if (cvalid) {
      const int lx = 2 * cxl + 1;
      T sxy;
      if (DIM == 3) {
        const int ly = 2 * cyl + 1;
        const T *r0 = sr + (ly - 1) * RX, *r1 = sr + ly * RX, *r2 = sr + (ly + 1) * RX;
        const T a0 = T(0.25) * r0[lx - 1] + T(0.5) * r0[lx] + T(0.25) * r0[lx + 1];
        const T a1 = T(0.25) * r1[lx - 1] + T(0.5) * r1[lx] + T(0.25) * r1[lx + 1];
        const T a2 = T(0.25) * r2[lx - 1] + T(0.5) * r2[lx] + T(0.25) * r2[lx + 1];
        sxy = T(0.25) * a0 + T(0.5) * a1 + T(0.25) * a2;
      } else {
        sxy = T(0.25) * sr[lx - 1] + T(0.5) * sr[lx] + T(0.25) * sr[lx + 1];
      }
      if (zf & 1) {
        acc += T(0.5) * sxy;
      } else {
        const int c = zf / 2 - 1;
        if (c >= C0) {
          acc += T(0.25) * sxy;
          const size_t o = DIM == 3 ? ((size_t)c * mc + cy) * mc + cx : (size_t)c * mc + cx;
          fcg[o] = acc;
        }
        acc = T(0.25) * sxy;
      }
    }
    store_u(zf + 2, nu);  // the ring slot of plane zf-1, read before the barrier
#pragma unroll
    for (int k = 0; k < NR; ++k) pf[k] = nf[k];
    __syncthreads();
  }
}

// ------------------------------------------------------------------------
// Residual r = f - A u (and/or per-workgroup sums of its square), marching
// over planes like the refinement step: a workgroup owns a TX x TY tile
// (TX x 1 rows in 2D) and a chunk of planes; u planes sit in a four-slot LDS
// ring with a one-point halo, and the next u plane and the current f plane
// come in through buffer loads that stay in flight across the plane's work.
// Neighbours are summed in the order x-1, x+1, y-1, y+1, z-1, z+1.
// ------------------------------------------------------------------------
template <typename T, int DIM, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT) k_residual(ResidArgs<T> a, int cz) {
  if (a.active && *gbl(a.active) == 0) return;
  constexpr int HX = TX + 2, HY = DIM == 3 ? TY + 2 : 1, HP = HX * HY;
  constexpr int NL = (HP + NT - 1) / NT;
  __shared__ T ring[4][HP];
  const int m = a.m;
  const int planeS = DIM == 3 ? m * m : m;
  const int ntx = (m + TX - 1) / TX, nty = DIM == 3 ? (m + TY - 1) / TY : 1;
  const int bid = xcd_remap_t(blockIdx.x, gridDim.x);
  const int tx = bid % ntx;
  const int rest = bid / ntx;
  const int ty = DIM == 3 ? rest % nty : 0;
  const int tzc = DIM == 3 ? rest / nty : rest;
  const int X0 = tx * TX, Y0 = ty * TY;
  const int Z0 = tzc * cz, Z1 = min(Z0 + cz, m);
  // halo-tile elements this thread loads (byte offsets in a plane)
  int hoff[NL];
  int hj[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int j = threadIdx.x + NT * k;
    hj[k] = j < HP ? j : -1;
    const int hx = j % HX, hy = j / HX;
    const int x = X0 - 1 + hx, y = DIM == 3 ? Y0 - 1 + hy : 0;
    const bool in = j < HP && x >= 0 && x < m && (DIM == 2 || (y >= 0 && y < m));
    hoff[k] = in ? ((DIM == 3 ? y * m : 0) + x) * (int)sizeof(T) : kOOB;
  }
  T uv[NL];
  auto load_plane = [&](int z, T *v) {
    // no u (zero iterate): a plane index outside the grid gives no records
    const __amdgpu_buffer_rsrc_t ru = plane_rsrc(a.u ? a.u : a.f, a.u ? z : -1, m, planeS);
#pragma unroll
    for (int k = 0; k < NL; ++k) v[k] = bload<T>(ru, hoff[k]);
  };
  auto store_plane = [&](int z, const T *v) {
    T *dst = ring[z & 3];
#pragma unroll
    for (int k = 0; k < NL; ++k)
      if (hj[k] >= 0) dst[hj[k]] = v[k];
  };
  // this thread's point
  const int cx = threadIdx.x % TX, cy = threadIdx.x / TX;
  const int gx = X0 + cx, gy = DIM == 3 ? Y0 + cy : 0;
  const bool mine = threadIdx.x < TX * TY && gx < m && (DIM == 2 || gy < m);
  const int ci = (DIM == 3 ? (cy + 1) * HX : 0) + cx + 1;
  const int coff = (DIM == 3 ? gy * m : 0) + gx;
  // prologue: planes Z0 - 1, Z0, Z0 + 1 in the ring
  load_plane(Z0 - 1, uv);
  store_plane(Z0 - 1, uv);
  load_plane(Z0, uv);
  store_plane(Z0, uv);
  load_plane(Z0 + 1, uv);
  store_plane(Z0 + 1, uv);
  __syncthreads();
  const T inv_h2 = T(a.inv_h2);
  double acc = 0.0;
  for (int z = Z0; z < Z1; ++z) {
    // f first: the load counter is in order, so waiting for f then leaves
    // the next plane's loads in flight during this plane's residual
    const __amdgpu_buffer_rsrc_t rf = plane_rsrc(a.f, z, m, planeS);
    const T fv = bload<T>(rf, mine ? coff * (int)sizeof(T) : kOOB);
    load_plane(z + 2, uv);
    if (mine) {
      const T *P = ring[z & 3];
      const T c = P[ci];
      T nb = P[ci - 1] + P[ci + 1];
      if (DIM == 3) {
        nb += P[ci - HX];
        nb += P[ci + HX];
      }
      nb += ring[(z - 1) & 3][ci];
      nb += ring[(z + 1) & 3][ci];
      const T r = fv - (T(2 * DIM) * c - nb) * inv_h2;
      if (a.r) gbl(a.r)[(size_t)z * planeS + coff] = r;
      acc += double(r) * double(r);
    }
    // slot (z + 2) & 3 last held plane z - 2, read by nobody in this step
    store_plane(z + 2, uv);
    __syncthreads();
  }
  if (a.partials) {
    __shared__ double red[NT / 64];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double sum = 0.0;
      for (int w = 0; w < NT / 64; ++w) sum += red[w];
      gbl(a.partials)[blockIdx.x] = sum;
    }
  }
}


// ------------------------------------------------------------------------
// Refinement step: x_out = x + e (FP64), r32 = float(f - A x_out), norm
// partials of |f - A x_out|^2.  Both x and e are read at the neighbours, so
// x_out never aliases x (the caller ping-pongs).
//
// A workgroup owns a TX x TY column tile (3D; TX x 1 in 2D) and marches along
// the outermost axis over a chunk of planes.  x + e of a plane, with a
// one-point halo, is formed once per plane into a four-plane LDS ring; the
// next plane's loads are in flight while the current plane's residual is
// computed.  Loads use plane buffer resources (zero outside the grid).
// ------------------------------------------------------------------------
template <int DIM, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT) k_ir_step(IrArgs a) {
  if (a.active && *gbl(a.active) == 0) return;
  constexpr int HX = TX + 2, HY = DIM == 3 ? TY + 2 : 1, HP = HX * HY;
  constexpr int NL = (HP + NT - 1) / NT;
  __shared__ double ring[4][HP];
  const int m = a.m;
  const int planeS = DIM == 3 ? m * m : m;
  const int ntx = (m + TX - 1) / TX, nty = DIM == 3 ? (m + TY - 1) / TY : 1;
  const int bid = xcd_remap_t(blockIdx.x, gridDim.x);
  const int tx = bid % ntx;
  const int rest = bid / ntx;
  const int ty = DIM == 3 ? rest % nty : 0;
  const int tzc = DIM == 3 ? rest / nty : rest;
  const int X0 = tx * TX, Y0 = ty * TY;
  const int Z0 = tzc * a.cz, Z1 = min(Z0 + a.cz, m);
  // halo-tile elements this thread loads (byte offsets in a plane)
  int hoff[NL];
  int hj[NL];
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    const int j = threadIdx.x + NT * k;
    hj[k] = j < HP ? j : -1;
    const int hx = j % HX, hy = j / HX;
    const int x = X0 - 1 + hx, y = DIM == 3 ? Y0 - 1 + hy : 0;
    const bool in = j < HP && x >= 0 && x < m && (DIM == 2 || (y >= 0 && y < m));
    hoff[k] = in ? ((DIM == 3 ? y * m : 0) + x) : -1;
  }
  const bool use_e = a.e != nullptr;
  // x and e of a plane stay separate in registers until the plane is stored
  // (x + e is formed then), so their loads stay in flight meanwhile
  double xv[NL];
  float ev[NL];
  auto load_plane = [&](int z, double *v, float *w) {
    const __amdgpu_buffer_rsrc_t rx = plane_rsrc(a.x, z, m, planeS);
    const __amdgpu_buffer_rsrc_t re = plane_rsrc(a.e, use_e ? z : -1, m, planeS);
#pragma unroll
    for (int k = 0; k < NL; ++k) {
      const int o = hoff[k];
      v[k] = bload<double>(rx, o >= 0 ? o * 8 : kOOB);
      w[k] = use_e ? bload<float>(re, o >= 0 ? o * 4 : kOOB) : 0.0f;
    }
  };
  auto store_plane = [&](int z, const double *v, const float *w) {
    double *dst = ring[z & 3];
#pragma unroll
    for (int k = 0; k < NL; ++k)
      if (hj[k] >= 0) dst[hj[k]] = use_e ? v[k] + double(w[k]) : v[k];
  };
  // this thread's point
  const int cx = threadIdx.x % TX, cy = threadIdx.x / TX;
  const int gx = X0 + cx, gy = DIM == 3 ? Y0 + cy : 0;
  const bool mine = threadIdx.x < TX * TY && gx < m && (DIM == 2 || gy < m);
  const int ci = (DIM == 3 ? (cy + 1) * HX : 0) + cx + 1;
  const int coff = (DIM == 3 ? gy * m : 0) + gx;
  // prologue: planes Z0 - 1, Z0, Z0 + 1 in the ring
  load_plane(Z0 - 1, xv, ev);
  store_plane(Z0 - 1, xv, ev);
  load_plane(Z0, xv, ev);
  store_plane(Z0, xv, ev);
  load_plane(Z0 + 1, xv, ev);
  store_plane(Z0 + 1, xv, ev);
  __syncthreads();
  const double inv_h2 = a.inv_h2;
  double acc = 0.0;
  for (int z = Z0; z < Z1; ++z) {
    // f first: the load counter is in order, so waiting for f then leaves
    // the next plane's loads in flight during this plane's residual
    const __amdgpu_buffer_rsrc_t rf = plane_rsrc(a.f, z, m, planeS);
    const double fv = bload<double>(rf, mine ? coff * 8 : kOOB);
    load_plane(z + 2, xv, ev);
    if (mine) {
      const double *P = ring[z & 3];
      const double c = P[ci];
      double nb = P[ci - 1] + P[ci + 1];
      if (DIM == 3) {
        nb += P[ci - HX];
        nb += P[ci + HX];
      }
      nb += ring[(z - 1) & 3][ci];
      nb += ring[(z + 1) & 3][ci];
      const double r = fv - (double(2 * DIM) * c - nb) * inv_h2;
      const size_t o = (size_t)z * planeS + coff;
      if (use_e) gbl(a.x_out)[o] = c;
      gbl(a.r32)[o] = float(r);
      acc += r * r;
    }
    // slot (z + 2) & 3 last held plane z - 2, read by nobody in this step
    store_plane(z + 2, xv, ev);
    __syncthreads();
  }
  __shared__ double red[NT / 64];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < NT / 64; ++w) s += red[w];
    gbl(a.partials)[blockIdx.x] = s;
  }
}

namespace {
constexpr int kIrTX3 = 64, kIrTY3 = 8, kIrTX2 = 256;
// planes per workgroup: enough workgroups to fill the chip, at most 65536
// (one norm partial each)
int ir_chunk(int dim, int m) {
  const long tiles = dim == 3 ? (long)((m + kIrTX3 - 1) / kIrTX3) * ((m + kIrTY3 - 1) / kIrTY3)
                              : (long)((m + kIrTX2 - 1) / kIrTX2);
  long cz = dim == 3 ? 16 : 8;
  while (tiles * ((m + cz - 1) / cz) > 65536) cz *= 2;
  if (cz > m) cz = m;
  return (int)cz;
}
}  // namespace

int ir_blocks(int dim, int m) {
  const int cz = ir_chunk(dim, m);
  const long tiles = dim == 3 ? (long)((m + kIrTX3 - 1) / kIrTX3) * ((m + kIrTY3 - 1) / kIrTY3)
                              : (long)((m + kIrTX2 - 1) / kIrTX2);
  return (int)(tiles * ((m + cz - 1) / cz));
}

// the residual kernel uses the refinement step's tiling and plane chunks
int residual_blocks(int dim, int m) { return ir_blocks(dim, m); }

// The stop test after a kernel that left n partial sums: 1024 threads,
// fixed order (strided per-thread sums, then a halving tree).
__global__ void __launch_bounds__(1024) k_finalize(const double *partials, int n, SolveState *st) {
  if (st->active == 0) return;
  __shared__ double red[1024];
  const GMG_GLOBAL double *pg = gbl(partials);
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) s += pg[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) update_state(st, red[0]);
}

// batch: one workgroup per table entry
__global__ void __launch_bounds__(64) k_finalize_batch(const FinEntry *tbl) {
  const FinEntry e = tbl[blockIdx.x];
  SolveState *st = e.st;
  if (st->active == 0) return;
  const double tot = sum_partials(e.partials, e.n);
  if (threadIdx.x == 0) update_state(st, tot);
}

__global__ void k_state_init_batch(SolveState *st, int n, int maxit, double rtol) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    st[i].active = 1;
    st[i].iter = 0;
    st[i].maxit = maxit;
    st[i].status = 0;
    st[i].rtol = rtol;
    st[i].res0 = -1.0;
    st[i].res = 0.0;
    st[i].pad = 0.0;
  }
}

__global__ void k_reduce_norm(const double *partials, int n, double *out) {
  const double tot = sum_partials(partials, n);
  if (threadIdx.x == 0) *out = sqrt(tot);
}

__global__ void k_state_init(SolveState *st, int maxit, double rtol, double res0) {
  if (threadIdx.x == 0) {
    st->active = 1;
    st->iter = 0;
    st->maxit = maxit;
    st->status = 0;
    st->rtol = rtol;
    st->res0 = res0;
    st->res = 0.0;
    st->pad = 0.0;
  }
}

__global__ void k_copy(const double2 *__restrict__ src, double2 *__restrict__ dst, size_t n2,
                       const unsigned char *__restrict__ src_tail,
                       unsigned char *__restrict__ dst_tail, size_t tail, const int *active) {
  if (active && *active == 0) return;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
  if (blockIdx.x == 0 && threadIdx.x < tail) dst_tail[threadIdx.x] = src_tail[threadIdx.x];
}

__global__ void k_fill_zero(unsigned char *dst, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    dst[i] = 0;
}

// ------------------------------------------------------------------------
// out = in + P e (in NULL = zero), one thread per fine point: x from the
// block and thread index, the row y and plane z from the grid's y and z, so
// no wide integer division.  Used when a level has no post-smoothing sweep
// (nu2 = 0) and for the interpolation of full multigrid; in may alias out.
// ------------------------------------------------------------------------
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_prolong_add(const T *in, const T *__restrict__ ec, T *out,
                                                     int m, int mc, const int *active) {
  if (active && *active == 0) return;
  const int x = blockIdx.x * 256 + threadIdx.x;
  const int y = blockIdx.y;
  const int z = DIM == 3 ? (int)blockIdx.z : 0;
  if (x < m) {
    const size_t p = ((size_t)z * m + y) * m + x;
    // canonical order: average along x, then y, then z (zero coarse boundary).
    // Per axis the two coarse neighbours i0 = (x-1)/2 rounded down and
    // i1 = x/2 coincide for odd x; all of them are loaded unconditionally
    // through a buffer resource with out-of-range offsets for the boundary,
    // and the parity only selects, so the loads issue together.
    const size_t nc = DIM == 3 ? (size_t)mc * mc * mc : (size_t)mc * mc;
    const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<T *>(ec), (short)0, (int)(nc * sizeof(T)), 0x00020000);
    auto cv = [&](int a, int b, int c) -> T {
      const bool ok = a >= 0 && b >= 0 && a < mc && b < mc && (DIM == 2 || (c >= 0 && c < mc));
      const int off = DIM == 3 ? (c * mc + b) * mc + a : b * mc + a;
      return bload<T>(rc, ok ? off * (int)sizeof(T) : kOOB);
    };
    const int x0 = (x - 1) >> 1, x1 = x >> 1;
    const int y0 = (y - 1) >> 1, y1 = y >> 1;
    auto xs = [&](int b, int c) {
      const T l = cv(x0, b, c), r = cv(x1, b, c);
      return (x & 1) ? l : T(0.5) * (l + r);
    };
    auto ys = [&](int c) {
      const T l = xs(y0, c), r = xs(y1, c);
      return (y & 1) ? l : T(0.5) * (l + r);
    };
    T s;
    if (DIM == 3) {
      const T l = ys((z - 1) >> 1), r = ys(z >> 1);
      s = (z & 1) ? l : T(0.5) * (l + r);
    } else {
      s = ys(0);
    }
    out[p] = (in ? in[p] : T(0)) + s;
  }
}

// x += e (FP64 += FP32), in place.
__global__ void __launch_bounds__(256) k_axpy_f32(double *x, const float *__restrict__ e, size_t n,
                                                  const int *active) {
  if (active && *active == 0) return;
  for (size_t p = (size_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (size_t)gridDim.x * 256)
    x[p] += double(e[p]);
}

// ------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------
template <typename T>
hipError_t launch_restrict(int dim, RestrictArgs<T> a, hipStream_t s, const RestrictArgs<T> *tbl,
                           int nent) {
  // tile and chunk by size: small coarse grids get small tiles and short
  // chunks (many short-lived workgroups), large ones long chunks
  const int mc = a.mc;
  if (dim == 3) {
    if (mc >= 64) {
      const int ncx = (mc + 31) / 32, ncy = (mc + 7) / 8;
      const int czc = mc >= 256 ? 8 : 4;
      const int ncz = (mc + czc - 1) / czc;
      const int nb = ncx * ncy * ncz;
      gmg_launch((k_restrict<T, 3, 32, 8, 256>), dim3(nb, nent), dim3(256), 0, s, a, tbl, ncx,
                         ncy, czc, nb);
    } else {
      const int ncx = (mc + 15) / 16, ncy = (mc + 7) / 8;
      const int czc = mc >= 16 ? 2 : 1;
      const int ncz = (mc + czc - 1) / czc;
      const int nb = ncx * ncy * ncz;
      gmg_launch((k_restrict<T, 3, 16, 8, 128>), dim3(nb, nent), dim3(128), 0, s, a, tbl, ncx,
                         ncy, czc, nb);
    }
  } else {
    const int ncx = (mc + 63) / 64;
    const int czc = mc >= 512 ? 16 : (mc >= 128 ? 8 : 2);
    const int ncz = (mc + czc - 1) / czc;
    const int nb = ncx * ncz;
    gmg_launch((k_restrict<T, 2, 64, 1, 128>), dim3(nb, nent), dim3(128), 0, s, a, tbl, ncx, 1,
                       czc, nb);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_residual(int dim, ResidArgs<T> a, hipStream_t s) {
  // the grid must be exactly the tiling the partial sums are counted for
  const int nb = residual_blocks(dim, a.m);
  if (a.nblocks > 0 && a.nblocks != nb) return hipErrorInvalidValue;
  const int cz = ir_chunk(dim, a.m);
  if (dim == 3)
    gmg_launch((k_residual<T, 3, kIrTX3, kIrTY3, kIrTX3 * kIrTY3>), dim3(nb),
               dim3(kIrTX3 * kIrTY3), 0, s, a, cz);
  else
    gmg_launch((k_residual<T, 2, kIrTX2, 1, kIrTX2>), dim3(nb), dim3(kIrTX2), 0, s, a, cz);
  return hipGetLastError();
}

hipError_t launch_ir_step(int dim, IrArgs a, hipStream_t s) {
  // the grid must be exactly the tiling the partial sums are counted for
  a.cz = ir_chunk(dim, a.m);
  const int nb = ir_blocks(dim, a.m);
  if (a.nblocks != nb) return hipErrorInvalidValue;
  if (dim == 3)
    gmg_launch((k_ir_step<3, kIrTX3, kIrTY3, kIrTX3 * kIrTY3>), dim3(nb), dim3(kIrTX3 * kIrTY3), 0,
               s, a);
  else
    gmg_launch((k_ir_step<2, kIrTX2, 1, kIrTX2>), dim3(nb), dim3(kIrTX2), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_finalize(const double *partials, int n, SolveState *st, hipStream_t s) {
  gmg_launch(k_finalize, dim3(1), dim3(1024), 0, s, partials, n, st);
  return hipGetLastError();
}

hipError_t launch_finalize_batch(const FinEntry *tbl, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  gmg_launch(k_finalize_batch, dim3(n), dim3(64), 0, s, tbl);
  return hipGetLastError();
}

hipError_t launch_state_init_batch(SolveState *st, int n, int maxit, double rtol, hipStream_t s) {
  gmg_launch(k_state_init_batch, dim3((n + 255) / 256), dim3(256), 0, s, st, n, maxit, rtol);
  return hipGetLastError();
}

hipError_t launch_reduce_norm(const double *partials, int n, double *out, hipStream_t s) {
  gmg_launch(k_reduce_norm, dim3(1), dim3(64), 0, s, partials, n, out);
  return hipGetLastError();
}

hipError_t launch_state_init(SolveState *st, int maxit, double rtol, double res0, hipStream_t s) {
  gmg_launch(k_state_init, dim3(1), dim3(64), 0, s, st, maxit, rtol, res0);
  return hipGetLastError();
}

hipError_t launch_copy(const void *src, void *dst, size_t bytes, const int *active,
                       hipStream_t s) {
  const size_t n2 = bytes / 16, tail = bytes % 16;
  size_t nb = (n2 + 255) / 256;
  if (nb > 8192) nb = 8192;
  if (nb < 1) nb = 1;
  gmg_launch(k_copy, dim3((unsigned)nb), dim3(256), 0, s, (const double2 *)src,
                     (double2 *)dst, n2, (const unsigned char *)src + n2 * 16,
                     (unsigned char *)dst + n2 * 16, tail, active);
  return hipGetLastError();
}

hipError_t launch_fill_zero(void *dst, size_t bytes, hipStream_t s) {
  size_t nb = (bytes + 255) / 256;
  if (nb > 8192) nb = 8192;
  if (nb < 1) nb = 1;
  gmg_launch(k_fill_zero, dim3((unsigned)nb), dim3(256), 0, s, (unsigned char *)dst,
                     bytes);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong_add(int dim, int m, int mc, const T *in, const T *ec, T *out,
                              const int *active, hipStream_t s) {
  const dim3 grid((m + 255) / 256, m, dim == 3 ? m : 1);
  if (dim == 3)
    gmg_launch((k_prolong_add<T, 3>), grid, dim3(256), 0, s, in, ec, out, m, mc, active);
  else
    gmg_launch((k_prolong_add<T, 2>), grid, dim3(256), 0, s, in, ec, out, m, mc, active);
  return hipGetLastError();
}

hipError_t launch_axpy_f32(double *x, const float *e, size_t n, const int *active, hipStream_t s) {
  size_t nb = (n + 255) / 256;
  if (nb > 8192) nb = 8192;
  if (nb < 1) nb = 1;
  gmg_launch(k_axpy_f32, dim3((unsigned)nb), dim3(256), 0, s, x, e, n, active);
  return hipGetLastError();
}

template hipError_t launch_prolong_add<double>(int, int, int, const double *, const double *,
                                               double *, const int *, hipStream_t);
template hipError_t launch_prolong_add<float>(int, int, int, const float *, const float *, float *,
                                              const int *, hipStream_t);
template hipError_t launch_restrict<double>(int, RestrictArgs<double>, hipStream_t,
                                            const RestrictArgs<double> *, int);
template hipError_t launch_restrict<float>(int, RestrictArgs<float>, hipStream_t,
                                           const RestrictArgs<float> *, int);
template hipError_t launch_residual<double>(int, ResidArgs<double>, hipStream_t);
template hipError_t launch_residual<float>(int, ResidArgs<float>, hipStream_t);

}  // namespace gmg
