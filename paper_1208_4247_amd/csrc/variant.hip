// variant.hip -- the paper's own smoother and grid transfers, as an
// alternative to red-black Gauss-Seidel with full weighting / (bi/tri)linear
// interpolation:
//   * multicolour Gauss-Seidel (Remark 1): 4 colours in 2D, 8 in 3D.  Node
//     (i, j[, k]) has colour (i&1) + 2(j&1) [+ 4(k&1)]; the forward sweep
//     visits colours in increasing order, the backward sweep in decreasing
//     order.  Each update is the pointwise solve of eq. relax_2D (and its 3D
//     analogue).
//   * linear finite-element restriction (eq. Restriction2d; 15 points in 3D)
//     fused with the residual (eq. residual_2D), and the matching linear
//     interpolation (eq. Prolongation2d and its 3D analogue).  The
//     triangulation's edges are the directions with components in {0, 1}.
//   * the one-node coarsest level, solved exactly or relaxed by the smoother
//     (Algorithm 1 as printed; they differ only for weighted Jacobi).
// FP64 only.
#include <algorithm>

#include "gmg_internal.h"

namespace gmg {

// ------------------------------------------------------------------------
// Multicolour Gauss-Seidel.
//
// 3D: the colours with k even are exactly the points of the planes with an
// even node index k, and their z-neighbours all lie in planes of the other
// parity.  A forward sweep is therefore two launches: first every plane of
// one parity gets an in-plane 4-colour sweep with its z-neighbours fixed,
// then every plane of the other parity, whose z-neighbours are the planes
// just updated.  2D is one launch: the in-plane sweep of the single plane.
//
// In-plane sweep of a TX x TY tile: the tile and a halo of two points sit in
// LDS (D2).  The four colour steps update every point of their colour in the
// tile plus a halo of one point (D1); after them the tile's own points are
// exact, because the last colour reads the third and second colours one
// point away, those read the first colour one point away, and the first
// colour reads old values one point away.  Only the tile is written back.
//
// Work is organised by 2x2 quads (one point of each colour) aligned to even
// storage indices; thread t owns quads t, t + NT, ...  Every launch reads src
// (and, in 3D, zsrc) and writes dst; no launch reads what it writes.
// ------------------------------------------------------------------------
struct McArgs {
  const double *src;   // old values of the planes being updated (NULL: zero)
  const double *zsrc;  // 3D: values of the other planes (NULL: zero)
  const double *f;
  double *dst;
  const int *active;
  int m;
  int pz;        // 3D: node-index parity of the planes this launch updates
  int backward;  // colour order reversed
  int ntx, nty;  // tiles along x, y
  int czp;       // 3D: own planes per workgroup
  double h2;
};

// Raw buffer over the part of an array a tile reads: in 3D one plane (no
// records for a plane outside the grid), in 2D the rows y0 .. y0+rows-1
// clipped to the grid.  Offsets are relative to the returned first row.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t mc_rsrc(const double *base, int dim, int z,
                                                         int m, int y0, int rows, int *ybase) {
  if (dim == 3) {
    *ybase = 0;
    return plane_rsrc(base, z, m, m * m);
  }
  const int a = max(y0, 0), b = min(y0 + rows, m);
  *ybase = a;
  const int n = b > a ? (b - a) * m : 0;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(base + (size_t)a * m), (short)0,
                                           n * (int)sizeof(double), 0x00020000);
}

template <int DIM, int QX, int QY, int NT>
__global__ void __launch_bounds__(NT) k_mc_sweep(McArgs a) {
  if (a.active && *a.active == 0) return;
  constexpr int W = 2 * QX, H = 2 * QY;  // D2 extent
  constexpr int TX = W - 4, TY = H - 4;  // tile
  constexpr int NQ = QX * QY;
  static_assert(NQ % NT == 0, "whole quads per thread");
  constexpr int QPT = NQ / NT;  // quads per thread
  __shared__ double U[H * W];   // current values on D2
  const int m = a.m;
  const int t = threadIdx.x;
  const int tile = blockIdx.x;
  const int x0 = (tile % a.ntx) * TX, y0 = (tile / a.ntx) * TY;
  const int xb = x0 - 2, yb = y0 - 2;  // storage index of D2's corner (even)
  const double diag = 2.0 * DIM;

  // own planes of this workgroup (3D): storage z with node parity pz
  int z_first = 0, nown = 1;
  if (DIM == 3) {
    const int zs = 1 - a.pz;  // first storage plane of that parity
    const int tot = (m - zs + 1) / 2;
    const int o0 = blockIdx.y * a.czp;
    nown = min(a.czp, tot - o0);
    z_first = zs + 2 * o0;
    if (nown <= 0) return;
  }

  // this thread's quads: D2-local corner and the byte offset of each of its
  // four points (row r, column c) relative to the resource's first row, or
  // kOOB outside the grid
  int lx0[QPT], ly0[QPT];
  int off[QPT][4];
  int ybase = 0;
  (void)mc_rsrc(a.f, DIM, 0, m, yb, H, &ybase);
#pragma unroll
  for (int i = 0; i < QPT; ++i) {
    const int q = t + i * NT;
    lx0[i] = 2 * (q % QX);
    ly0[i] = 2 * (q / QX);
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int x = xb + lx0[i] + c, y = yb + ly0[i] + r;
        const bool in = x >= 0 && x < m && y >= 0 && y < m;
        off[i][2 * r + c] = in ? ((y - ybase) * m + x) * (int)sizeof(double) : kOOB;
      }
  }

  double R[QPT][4];    // h^2 f + z-neighbours of the quad's points
  double zlo[QPT][4];  // 3D: the plane below, carried from one own plane to the next
  if (DIM == 3) {
    const __amdgpu_buffer_rsrc_t rz = a.zsrc ? plane_rsrc(a.zsrc, z_first - 1, m, m * m)
                                             : plane_rsrc(a.f, -1, m, m * m);
#pragma unroll
    for (int i = 0; i < QPT; ++i)
#pragma unroll
      for (int k = 0; k < 4; ++k) zlo[i][k] = bload<double>(rz, off[i][k]);
  }

  // loads of one own plane: old values, f and (3D) the plane above; issued
  // for plane o + 1 before the colour steps of plane o so that they overlap
  double pu[QPT][4], pf[QPT][4], pz[QPT][4];
  auto load_plane = [&](int z) {
    int yb2 = 0;
    const __amdgpu_buffer_rsrc_t rf = mc_rsrc(a.f, DIM, z, m, yb, H, &yb2);
    const __amdgpu_buffer_rsrc_t ru = a.src ? mc_rsrc(a.src, DIM, z, m, yb, H, &yb2)
                                            : plane_rsrc(a.f, -1, m, m * m);  // no records: zero
    __amdgpu_buffer_rsrc_t rzh = plane_rsrc(a.f, -1, m, m * m);
    if (DIM == 3 && a.zsrc) rzh = plane_rsrc(a.zsrc, z + 1, m, m * m);
#pragma unroll
    for (int i = 0; i < QPT; ++i)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        pu[i][k] = bload<double>(ru, off[i][k]);
        pf[i][k] = bload<double>(rf, off[i][k]);
        if (DIM == 3) pz[i][k] = bload<double>(rzh, off[i][k]);
      }
  };
  load_plane(z_first);

  for (int o = 0; o < nown; ++o) {
    const int z = z_first + 2 * o;
#pragma unroll
    for (int i = 0; i < QPT; ++i)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        double r = a.h2 * pf[i][k];
        if (DIM == 3) {
          r = r + (zlo[i][k] + pz[i][k]);
          zlo[i][k] = pz[i][k];  // the plane above is the next own plane's plane below
        }
        R[i][k] = r;
        U[(ly0[i] + (k >> 1)) * W + lx0[i] + (k & 1)] = pu[i][k];
      }
    if (o + 1 < nown) load_plane(z + 2);
    __syncthreads();
    // four colour steps on D1 (the tile plus a halo of one point)
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int c = a.backward ? 3 - s : s;
      const int ax = c & 1, by = c >> 1;  // node-index parities of this colour
      const int k = 2 * (1 - by) + (1 - ax);  // that point's index in the quad
#pragma unroll
      for (int i = 0; i < QPT; ++i) {
        const int lx = lx0[i] + (1 - ax), ly = ly0[i] + (1 - by);
        if (lx < 1 || lx >= W - 1 || ly < 1 || ly >= H - 1) continue;  // D1 only
        if (off[i][k] == kOOB) continue;                                // boundary stays 0
        const int p = ly * W + lx;
        U[p] = (R[i][k] + ((U[p - 1] + U[p + 1]) + (U[p - W] + U[p + W]))) / diag;
      }
      __syncthreads();
    }
    // the tile's own points: quads lie wholly inside or outside the tile
    int yb2 = 0;
    const __amdgpu_buffer_rsrc_t rd = mc_rsrc(a.dst, DIM, z, m, yb, H, &yb2);
#pragma unroll
    for (int i = 0; i < QPT; ++i) {
      if (lx0[i] < 2 || lx0[i] >= W - 2 || ly0[i] < 2 || ly0[i] >= H - 2) continue;
#pragma unroll
      for (int k = 0; k < 4; ++k)
        bstore<double>(rd, off[i][k], U[(ly0[i] + (k >> 1)) * W + lx0[i] + (k & 1)]);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------------
// Residual + linear finite-element restriction.  Coarse node I receives
// (2 r(2I) + sum over the edge directions e of r(2I + e) + r(2I - e)) /
// 2^(d+1), r = f - A u (u NULL: the zero iterate, r = f).  A workgroup owns
// a CX x CY tile of coarse points and, in 3D, a run of coarse planes; it
// marches over the fine planes 2c-1 .. 2c+1 of each (storage 2c .. 2c+2),
// keeping three fine u planes of its fine footprint (plus a halo of one) in
// an LDS ring.  Each fine plane's residual is formed once in LDS and added
// to the coarse planes it belongs to: the plane through the coarse nodes
// with the in-plane 7-point pattern (centre weight 2), the plane above with
// the four directions of positive z (centre, +x, +y, +x+y), the plane below
// with their negatives.
// ------------------------------------------------------------------------
struct FeRestrictArgs {
  const double *u;  // NULL: zero iterate
  const double *f;
  double *fc;
  const int *active;
  int m, mc, ntx, nty, czc;  // czc: coarse planes per workgroup (3D)
  double inv_h2;
};

template <int DIM, int CX, int CY>
__global__ void __launch_bounds__(CX *CY) k_restrict_fe(FeRestrictArgs a) {
  if (a.active && *a.active == 0) return;
  constexpr int NT = CX * CY;
  constexpr int RW = 2 * CX + 1, RH = 2 * CY + 1;  // fine footprint
  constexpr int UW = RW + 2, UH = RH + 2;          // with the residual's halo
  constexpr int NU = UW * UH, NR = RW * RH;
  constexpr int NRING = DIM == 3 ? 3 : 1;
  __shared__ double Us[NRING][NU];
  __shared__ double Rs[NR];
  const int m = a.m, mc = a.mc;
  const int t = threadIdx.x;
  const int tile = blockIdx.x;
  const int a0 = (tile % a.ntx) * CX, b0 = (tile / a.ntx) * CY;
  const int fx0 = 2 * a0, fy0 = 2 * b0;  // fine storage index of the footprint's corner
  const double diag = 2.0 * DIM;
  const int ta = t % CX, tb = t / CX;
  const int ca = a0 + ta, cb = b0 + tb;
  // this thread's coarse point in local footprint coordinates
  const int lx = 2 * ta + 1, ly = 2 * tb + 1;

  // Byte offsets of this thread's u-footprint and residual elements inside a
  // plane (the whole grid in 2D), out of range (kOOB) outside the grid.
  // Loads go through buffer resources, so they need no branches and stay in
  // flight across the work that does not use them.
  constexpr int UPT = (NU + NT - 1) / NT;
  constexpr int RPT = (NR + NT - 1) / NT;
  int uo[UPT], ro[RPT];
  bool rin[RPT];
#pragma unroll
  for (int q = 0; q < UPT; ++q) {
    const int p = t + q * NT;
    const int x = fx0 - 1 + p % UW, y = fy0 - 1 + p / UW;
    uo[q] = (p < NU && x >= 0 && x < m && y >= 0 && y < m) ? (y * m + x) * 8 : kOOB;
  }
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int p = t + k * NT;
    const int x = fx0 + p % RW, y = fy0 + p / RW;
    rin[k] = p < NR && x < m && y < m;
    ro[k] = rin[k] ? (y * m + x) * 8 : kOOB;
  }
  const int mm = m * m;
  double pre[UPT], fcur[RPT], fnext[RPT];
  auto fetch_u = [&](int z) {
    // no u: a plane index outside the grid gives a resource with no records
    const __amdgpu_buffer_rsrc_t r =
        plane_rsrc(a.u ? a.u : a.f, a.u ? z : -1, DIM == 3 ? m : 1, mm);
#pragma unroll
    for (int q = 0; q < UPT; ++q) pre[q] = bload<double>(r, uo[q]);
  };
  auto fetch_f = [&](int z, double *v) {
    const __amdgpu_buffer_rsrc_t r = plane_rsrc(a.f, z, DIM == 3 ? m : 1, mm);
#pragma unroll
    for (int k = 0; k < RPT; ++k) v[k] = bload<double>(r, ro[k]);
  };
  auto store_u = [&](int slot) {
#pragma unroll
    for (int q = 0; q < UPT; ++q) {
      const int p = t + q * NT;
      if (p < NU) Us[slot][p] = pre[q];
    }
  };
  // residual of fine plane z into Rs (ring slots of planes z-1, z, z+1; f
  // of plane z in fcur)
  auto residual = [&](int z, int sm, int s0, int sp) {
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int p = t + k * NT;
      if (p >= NR) continue;
      double r = 0.0;
      if (rin[k] && (DIM == 2 || (z >= 0 && z < m))) {
        if (a.u) {
          const int q = (p / RW + 1) * UW + (p % RW + 1);
          double nb = Us[s0][q - 1] + Us[s0][q + 1] + Us[s0][q - UW] + Us[s0][q + UW];
          if (DIM == 3) nb = nb + Us[sm][q] + Us[sp][q];
          r = fcur[k] - (diag * Us[s0][q] - nb) * a.inv_h2;
        } else {
          r = fcur[k];
        }
      }
      Rs[p] = r;
    }
  };
  auto R = [&](int dx, int dy) { return Rs[(ly + dy) * RW + (lx + dx)]; };
  const bool mine = ca < mc && cb < mc;

  if (DIM == 2) {
    fetch_u(0);
    fetch_f(0, fcur);
    store_u(0);
    __syncthreads();
    residual(0, 0, 0, 0);
    __syncthreads();
    if (mine) {
      const double s = 2.0 * R(0, 0) + (R(1, 0) + R(-1, 0)) + (R(0, 1) + R(0, -1)) +
                       (R(1, 1) + R(-1, -1));
      gbl(a.fc)[(size_t)cb * mc + ca] = s * 0.125;
    }
    return;
  }

  const int c0 = blockIdx.y * a.czc;
  const int c1 = min(mc, c0 + a.czc);
  if (c0 >= c1) return;
  const size_t cplane = (size_t)mc * mc;
  // Fine planes 2c0 .. 2c1 (storage); ring slot of plane z is (z + 3) % 3.
  // The u plane two ahead and the f plane one ahead are loaded into
  // registers while the residual of plane z is formed; the u plane is stored
  // into the slot plane z - 1 frees.
  for (int zz = 2 * c0 - 1; zz <= 2 * c0 + 1; ++zz) {
    fetch_u(zz);
    store_u((zz + 3) % 3);
  }
  fetch_f(2 * c0, fcur);
  __syncthreads();
  double acc = 0.0;
  for (int z = 2 * c0; z <= 2 * c1; ++z) {
    const bool more = z + 2 <= 2 * c1 + 1;
    if (more) fetch_u(z + 2);
    if (z < 2 * c1) fetch_f(z + 1, fnext);
    residual(z, (z - 1 + 3) % 3, (z + 3) % 3, (z + 1 + 3) % 3);
    __syncthreads();
    if (z & 1) {
      // the plane through coarse plane c = (z - 1) / 2
      acc = acc + (2.0 * R(0, 0) + (R(1, 0) + R(-1, 0)) + (R(0, 1) + R(0, -1)) +
                   (R(1, 1) + R(-1, -1)));
    } else {
      if (z > 2 * c0) {
        // the plane above coarse plane c = z / 2 - 1: directions with z = +1
        acc = acc + (R(0, 0) + R(1, 0) + R(0, 1) + R(1, 1));
        if (mine) gbl(a.fc)[(size_t)(z / 2 - 1) * cplane + (size_t)cb * mc + ca] = acc * 0.0625;
      }
      // the plane below coarse plane z / 2: directions with z = -1
      acc = R(0, 0) + R(-1, 0) + R(0, -1) + R(-1, -1);
    }
    // plane z + 2 into the slot of plane z - 1 (no longer read)
    if (more) store_u((z + 2) % 3);
    if (z < 2 * c1) {
#pragma unroll
      for (int k = 0; k < RPT; ++k) fcur[k] = fnext[k];
    }
    __syncthreads();  // Rs and the ring are reused
  }
}

// ------------------------------------------------------------------------
// out = in + P e with the linear finite-element interpolation (in NULL:
// zero; in may alias out): fine node 2I takes coarse node I, fine node
// 2I + o (o != 0 with components in {0, 1}) the mean of coarse nodes I and
// I + o.  One thread per fine point.
// ------------------------------------------------------------------------
template <int DIM>
__global__ void __launch_bounds__(256) k_prolong_fe(const double *in, const double *__restrict__ ec,
                                                    double *out, int m, int mc,
                                                    const int *active) {
  if (active && *active == 0) return;
  const int xs = blockIdx.x * 256 + threadIdx.x;  // storage indices: x, row, plane
  const int ys = blockIdx.y;
  const int zs = DIM == 3 ? (int)blockIdx.z : 0;
  if (xs < m) {
    const size_t p = ((size_t)zs * m + ys) * m + xs;
    // node indices of the fine point
    const int i = xs + 1;
    const int j = ys + 1;
    const int k = DIM == 3 ? zs + 1 : 0;
    const int oi = i & 1, oj = j & 1, ok = k & 1;
    const int I = (i - oi) >> 1, J = (j - oj) >> 1, K = (k - ok) >> 1;
    // coarse node value, 0 on the boundary: both loads issue unconditionally
    // through a buffer resource over the coarse grid (out-of-range offsets
    // read 0); the parity only selects
    const int nc = DIM == 3 ? mc * mc * mc : mc * mc;
    const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<double *>(ec), (short)0, nc * 8, 0x00020000);
    auto cv = [&](int ci, int cj, int ck) -> double {
      const bool in = ci >= 1 && cj >= 1 && ci <= mc && cj <= mc &&
                      (DIM == 2 || (ck >= 1 && ck <= mc));
      const int o = DIM == 3 ? ((ck - 1) * mc + (cj - 1)) * mc + (ci - 1) : (cj - 1) * mc + (ci - 1);
      return bload<double>(rc, in ? o * 8 : kOOB);
    };
    const double c0 = cv(I, J, K);
    const double c1 = cv(I + oi, J + oj, K + ok);
    const double s = (oi | oj | ok) ? 0.5 * (c0 + c1) : c0;
    out[p] = (in ? in[p] : 0.0) + s;
  }
}

// ------------------------------------------------------------------------
// The one-node coarsest level: exact (u = h^2 f / (2d)), or nsweeps sweeps
// of the smoother from zero (weighted Jacobi: u <- (1 - w) u + w h^2 f/(2d);
// a Gauss-Seidel sweep is already exact).
// ------------------------------------------------------------------------
__global__ void k_coarsest(const double *f, double *u, int dim, int relax, int wj, int nsweeps,
                           double omega, const int *active) {
  if (active && *active == 0) return;
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double h2 = 0.25;  // h = 1/2 on the one-node grid
  const double ex = (h2 * f[0]) / (2.0 * dim);
  double v = ex;
  if (relax) {
    v = 0.0;
    for (int s = 0; s < nsweeps; ++s) v = wj ? (1.0 - omega) * v + omega * ex : ex;
  }
  u[0] = v;
}

// ------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------
namespace {
template <int DIM, int QX, int QY, int NT>
hipError_t mc_launch(McArgs a, hipStream_t s) {
  constexpr int TX = 2 * QX - 4, TY = 2 * QY - 4;
  const int m = a.m;
  a.ntx = (m + TX - 1) / TX;
  a.nty = (m + TY - 1) / TY;
  const int tiles = a.ntx * a.nty;
  int nz = 1;
  if (DIM == 3) {
    const int own = (m + 1) / 2;  // most planes of one parity
    // a few planes per workgroup (the next plane's loads overlap this
    // plane's colour steps, and the plane below comes from the previous
    // plane's plane above) while keeping a few thousand workgroups
    a.czp = std::max(2, std::min(16, own * tiles / 2048));
    nz = (own + a.czp - 1) / a.czp;
  }
  gmg_launch((k_mc_sweep<DIM, QX, QY, NT>), dim3(tiles, nz), dim3(NT), 0, s, a);
  return hipGetLastError();
}

template <int DIM>
hipError_t mc_sweep_dim(McArgs a, hipStream_t s) {
  if (a.m >= (DIM == 3 ? 127 : 255))
    return DIM == 3 ? mc_launch<DIM, 64, 16, 512>(a, s) : mc_launch<DIM, 64, 16, 256>(a, s);
  return mc_launch<DIM, 16, 8, 128>(a, s);
}
}  // namespace

hipError_t launch_mc_sweep(int dim, int m, const double *src, const double *f, double *dst,
                           int backward, double h2, const int *active, hipStream_t s, int part) {
  if (m < 1 || !f || !dst || dst == src || dst == f) return hipErrorInvalidValue;
  McArgs a{};
  a.src = src;
  a.f = f;
  a.dst = dst;
  a.active = active;
  a.m = m;
  a.backward = backward;
  a.h2 = h2;
  if (dim == 2) return mc_sweep_dim<2>(a, s);
  // forward: planes of even node index, then odd; backward: odd, then even
  const int first = backward ? 1 : 0;
  if (part == 0) {
    a.pz = first;
    a.zsrc = src;  // the other planes still hold their old values
  } else {
    a.pz = 1 - first;
    a.zsrc = dst;  // the planes the first part updated
  }
  return mc_sweep_dim<3>(a, s);
}

hipError_t launch_restrict_fe(int dim, int m, int mc, const double *u, const double *f, double *fc,
                              double inv_h2, const int *active, hipStream_t s) {
  if (mc < 1 || m != 2 * mc + 1 || !f || !fc) return hipErrorInvalidValue;
  FeRestrictArgs a{};
  a.u = u;
  a.f = f;
  a.fc = fc;
  a.active = active;
  a.m = m;
  a.mc = mc;
  a.inv_h2 = inv_h2;
  if (dim == 2) {
    constexpr int CX = 32, CY = 8;
    a.ntx = (mc + CX - 1) / CX;
    a.nty = (mc + CY - 1) / CY;
    gmg_launch((k_restrict_fe<2, CX, CY>), dim3(a.ntx * a.nty, 1), dim3(CX * CY), 0, s, a);
    return hipGetLastError();
  }
  constexpr int CX = 32, CY = 8;
  a.ntx = (mc + CX - 1) / CX;
  a.nty = (mc + CY - 1) / CY;
  const int tiles = a.ntx * a.nty;
  a.czc = std::max(1, std::min(8, mc * tiles / 1024));
  const int nz = (mc + a.czc - 1) / a.czc;
  gmg_launch((k_restrict_fe<3, CX, CY>), dim3(tiles, nz), dim3(CX * CY), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_prolong_fe(int dim, int m, int mc, const double *in, const double *ec,
                             double *out, const int *active, hipStream_t s) {
  if (mc < 1 || m != 2 * mc + 1 || !ec || !out) return hipErrorInvalidValue;
  const dim3 grid((m + 255) / 256, m, dim == 3 ? m : 1);
  if (dim == 2)
    gmg_launch((k_prolong_fe<2>), grid, dim3(256), 0, s, in, ec, out, m, mc, active);
  else
    gmg_launch((k_prolong_fe<3>), grid, dim3(256), 0, s, in, ec, out, m, mc, active);
  return hipGetLastError();
}

hipError_t launch_coarsest(int dim, const double *f, double *u, int relax, int wj, int nsweeps,
                           double omega, const int *active, hipStream_t s) {
  gmg_launch(k_coarsest, dim3(1), dim3(64), 0, s, f, u, dim, relax, wj, nsweeps, omega, active);
  return hipGetLastError();
}

}  // namespace gmg
