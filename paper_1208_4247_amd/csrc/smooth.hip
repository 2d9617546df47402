// smooth.hip -- fused smoothing passes for gfx950 (red-black Gauss-Seidel and
// weighted Jacobi) on the 5-/7-point Poisson stencil.
//
// Smoother: Sec. 3.2 Remark 1 and the relaxation formula of Sec. 4 (eq.
// relax_2D, u = (h^2 f + sum of neighbours) / (2d)); red-black colouring by
// parity of the node-index sum (red even); a forward sweep relaxes red then
// black, a backward sweep black then red (Algorithm 1's Relax_forward /
// Relax_backward).  Weighted Jacobi: Remark 1 and Table 5.
//
// One launch = one pass over HBM that applies S stages (S half-sweeps for
// red-black, S full sweeps for Jacobi) -- temporal blocking:
//
//  * A workgroup owns an output tile of TX x TY columns (3D; TX x 1 in 2D) and
//    marches along the outermost axis (z in 3D, y in 2D) over a chunk of
//    planes.  Stage s lags the input by s planes; every stage keeps a
//    three-plane window of its values in registers (the marching-axis
//    neighbours) and publishes its newest plane in LDS for the in-plane
//    neighbours.  The tile carries a halo of S points on each in-plane side so
//    that the last stage is exact on the output tile; halo values are
//    recomputed redundantly by neighbouring tiles (cheap: the kernel is HBM
//    bound at ~0.3 flop/byte).
//  * Each lane owns a PAIR of adjacent x columns.  In any row and plane
//    exactly one element of the pair has a given colour, and which one is the
//    same for all lanes of the row, so a red-black half-sweep does exactly one
//    update per lane with no divergence, and one of the two x-neighbours of
//    that element is the other element of the lane's own pair.
//  * Optional fusions: the start value may be zero (coarse levels of the
//    correction scheme), or the previous iterate plus the (bi/tri)linearly
//    interpolated coarse correction (the prolongation of Algorithm 1's ascent);
//    the pass may emit per-workgroup sums of |f - A u_in|^2 (the convergence
//    test of Algorithm 3 evaluated on the pass's input, which the pass reads
//    anyway).
//  * Workgroup -> tile mapping is XCD-aware: the 8 XCDs receive contiguous
//    ranges of tiles, so halo re-reads of neighbouring tiles hit the same L2.
#include "gmg_internal.h"

namespace gmg {

// Compiler-only fences for the load pipelines of the passes (no instruction
// is emitted).  pin_value: v is computed here, not sunk below this point,
// and no memory access moves across; compiler_fence: only the latter.  A
// load issued after the fence into registers whose previous contents were
// consumed before it can reuse those registers, so a value loaded for a
// later step is carried around the loop without a copy, and nothing waits
// on it until it is used.
template <typename T>
__device__ __forceinline__ void pin_value(T &v) {
  asm volatile("" : "+v"(v) : : "memory");
}
__device__ __forceinline__ void compiler_fence() { asm volatile("" : : : "memory"); }

__device__ __forceinline__ int xcd_remap(int bid, int n) {
  const int xcd = bid & 7, loc = bid >> 3;
  const int per = n >> 3, rem = n & 7;
  return xcd * per + min(xcd, rem) + loc;
}

// Tile (tx, ty) and z-chunk tz of tile index j.  Chunks are outermost; a
// chunk's tiles run down vertical strips sw tiles wide (row by row inside a
// strip; sw = 0 or >= ntx: whole rows).  With the XCD remap each XCD takes
// a contiguous run of indices, so the workgroups one XCD runs at a time
// cover a compact block of neighbouring tiles rather than a thin band of
// rows, and more of their halos are shared in that XCD's L2.
template <int DIM>
__device__ __forceinline__ void tile_coords(int j, int ntx, int nty, int sw, int &tx, int &ty,
                                            int &tz) {
  if (DIM == 2) {
    tx = j % ntx;
    ty = 0;
    tz = j / ntx;
    return;
  }
  const int per = ntx * nty;
  tz = j / per;
  const int r = j - tz * per;
  const int bw = (sw > 0 && sw < ntx) ? sw : ntx;
  const int s = r / (bw * nty);
  const int q = r - s * bw * nty;
  const int w = min(bw, ntx - s * bw);  // the last strip may be narrower
  ty = q / w;
  tx = s * bw + (q - ty * w);
}

template <int NT>
__device__ __forceinline__ void block_sum_store(double acc, GMG_GLOBAL double *out) {
  __shared__ double red[NT / 64];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < NT / 64; ++w) s += red[w];
    out[blockIdx.x] = s;
  }
}

// ------------------------------------------------------------------------
// Per-slot geometry shared by the passes.  A slot is a pair of adjacent x
// columns (xb, xb+1), xb even, in row y of the extended tile.
// ------------------------------------------------------------------------
struct SlotGeo {
  int off;       // y*m + xb (3D) / xb (2D): offset inside a plane
  int q;         // slot index inside the tile (LDS position)
  int par;       // (y + DIM) & 1: element e has colour (e + par + z) & 1
  int ok;        // bit0 / bit1: element 0 / 1 inside the domain (x and y); bit2 live
  int outp;      // slot belongs to the output tile
  int y;         // row (3D) or 0
  int xb;
};

template <int DIM, int S_HALO, int EXP, int EY, int NT, int NS>
__device__ __forceinline__ void slot_setup(SlotGeo (&g)[NS], int X0, int Y0, int m) {
  constexpr int PL = EXP * EY;
  constexpr int HP = (S_HALO + 1) / 2;
  constexpr int H = 2 * HP;
  constexpr int TXP = EXP - 2 * HP;
  constexpr int TY = DIM == 3 ? EY - 2 * H : 1;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const int q = threadIdx.x + NT * i;
    const bool live = q < PL;
    const int p = q % EXP, r = q / EXP;
    const int xb = X0 - H + 2 * p;
    const int y = DIM == 3 ? Y0 - H + r : 0;
    const bool yin = DIM == 2 || (y >= 0 && y < m);
    g[i].q = live ? q : PL - 1;
    g[i].xb = xb;
    g[i].y = y;
    g[i].off = (DIM == 3 ? y * m : 0) + xb;
    g[i].par = (y + DIM) & 1;
    g[i].ok = ((live && yin && xb >= 0 && xb < m) ? 1 : 0) |
              ((live && yin && xb + 1 >= 0 && xb + 1 < m) ? 2 : 0) | (live ? 4 : 0);
    g[i].outp = live && yin && p >= HP && p < HP + TXP &&
                (DIM == 2 || (r >= H && r < H + TY)) && xb < m;
  }
}

// ------------------------------------------------------------------------
// Red-black Gauss-Seidel pass: S half-sweeps, colour of stage s is
// (C1 + s - 1) mod 2 with C1 = 0 (red first) or 1 (black first).
//
// Step t: stage 0 holds the start value of plane t (prefetched during step
// t-1), stage s computes plane t-s of colour c_s from stage s-1's planes
// t-s-1 .. t-s+1 (registers) and its in-plane neighbours (LDS, published at
// step t-1).  Plane t-S leaves the pipeline: colour c_S from stage S, the
// other colour from stage S-1.
//
// Memory access: every HBM access goes through a buffer resource of one
// plane (zero records for a plane outside the grid) and a per-element byte
// offset that is out of range for elements outside the grid or (stores)
// outside the output tile, so loads of the zero boundary return 0 and
// stores outside the tile are dropped, without branches.  Steps come in
// pairs (t even, t odd), which makes every colour and parity decision a
// compile-time choice between the two elements of a pair, and the LDS planes
// are double-buffered by step parity, so one barrier per step suffices.
// ------------------------------------------------------------------------
// Argument block of this workgroup: the kernel argument, or (batch mode) the
// table entry of problem blockIdx.y, read through the scalar cache.
template <typename A>
__device__ __forceinline__ A entry_of(const A &arg, const A *tbl) {
  if (!tbl) return arg;
  A r;
  __builtin_memcpy(&r, (const __attribute__((address_space(4))) A *)tbl + blockIdx.y, sizeof(A));
  return r;
}

template <typename T, int DIM, int S, int EXP, int EY, int NT, int FL>
__global__ void __launch_bounds__(NT) k_rb_pass(PassArgs<T> arg, const PassArgs<T> *tbl) {
  const PassArgs<T> a = entry_of(arg, tbl);
  if (a.active && *gbl(a.active) == 0) return;
  constexpr int PL = EXP * EY;
  constexpr int NS = (PL + NT - 1) / NT;        // slots per thread
  constexpr bool TAIL = NS * NT > PL;           // the last slot index has dead lanes
  constexpr bool ZERO = (FL & F_ZERO_IN) != 0;
  constexpr bool PRO = (FL & F_PROLONG) != 0;
  constexpr bool NORM = (FL & F_NORM_IN) != 0;
  constexpr bool RST = (FL & F_RESTRICT) != 0;
  // NMID: the norm of the residual of the iterate after stage QN = (S+1)/2
  // (a pass that ends one sweep -- Algorithm 1's backward post-smoothing --
  // and starts the next cycle's forward sweep, whose first half-sweep would
  // repeat the red one just done and is left out)
  constexpr bool NMID = (FL & F_NORM_MID) != 0;
  constexpr int QN = (S + 1) / 2;
  static_assert(!NMID || (S % 2 == 1 && S >= 3 && !NORM), "mid-pass norm: odd S >= 3");
  // halo (rb_halo): S points for the stages; RST needs the final values one
  // point past the output tile on the low side (the residual at its first
  // point) and two on the high side (the residual one point past it, for the
  // full weighting of the edge coarse points)
  constexpr RbHalo HA = rb_halo(S, RST);
  constexpr int HPL = HA.pl, HPH = HA.ph;       // halo in pairs, low / high side
  constexpr int HYL = HA.yl, HYH = HA.yh;       // halo in rows (3D), low / high side
  constexpr int TXP = EXP - HPL - HPH;          // output pairs per row
  constexpr int TY = DIM == 3 ? EY - HYL - HYH : 1;
  static_assert(TXP > 0 && TY > 0 && (DIM == 2 || TY % 2 == 0), "tile too small");
  constexpr int C1 = (FL & F_BLACK_FIRST) ? 1 : 0;
  constexpr int C0 = 1 - C1;  // colour the first stage reads
  constexpr int NB = S + (NORM ? 1 : 0);  // LDS planes per buffer
  // PRO: the coarse correction's footprint under the tile, one coarse plane
  // at a time, staged in LDS (two planes in a ring).  Column j <-> coarse x
  // index CX0 + j, row k <-> coarse y index CY0 + k; zero outside the grid.
  constexpr int NCX = EXP + 1;
  constexpr int NCY = DIM == 3 ? (EY + 1) / 2 + 1 : 1;
  constexpr int CPL = NCX * NCY;
  constexpr int NCP = PRO ? (CPL + NT - 1) / NT : 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // [2 (step parity)][NB][PL]; RST: final plane and residual plane, each
  // [2 (step parity)][2 (element)][PL]; PRO: [2][CPL]
  T *lds = reinterpret_cast<T *>(smem_raw);
  T *fwl = lds + 2 * NB * PL;
  T *rl = fwl + 4 * PL;
  T *cring = lds + 2 * NB * PL + (RST ? 8 * PL : 0);

  const int m = a.m;
  int tx, ty, tzc;
  tile_coords<DIM>(xcd_remap(blockIdx.x, a.nblocks), a.ntx, a.nty, a.sw, tx, ty, tzc);
  const int X0 = tx * 2 * TXP;
  const bool xend = (m & 1) && X0 + 2 * TXP >= m;  // the output tile holds x = m - 1
  const int Y0 = ty * TY;
  const int Z0 = tzc * a.tz;
  const int Z1 = min(Z0 + a.tz, m);
  const int planeS = DIM == 3 ? m * m : m;
  const T h2 = T(a.h2);

  // ---- per-slot geometry.  "P" is the element whose index equals the row
  // parity par = (y + DIM) & 1, "Q" the other one; an element e of plane z
  // has colour (e + par + z) & 1.
  // Loads take both elements of a pair at once from byte offset o2 (kOOB
  // when neither is inside the grid); the pair at the end of a row (xb =
  // m - 1, m odd) loads elements (xb - 1, xb) instead, so element 0 is then
  // the high half.  hP / hQ: element P / Q is the high half of the load.
  int o2[NS];
  bool hP[NS], hQ[NS];
  // stores: a pair of the output tile with both elements in the grid takes
  // one 16-byte store at w2; the lone element of a row-end pair (m odd) an
  // 8-byte store at w1 (kOOB elsewhere)
  int w2[NS], w1[NS];
  bool nP[NS], nQ[NS];   // NORM: element inside the grid and the output tile
  bool kP[NS], kQ[NS];   // element inside the grid
  int lq[NS], lP[NS], lQ[NS], lu[NS], ld[NS];  // LDS: self, x-side of P / Q, y-1, y+1
  bool live[NS];
  int cb[PRO ? NS : 1];
  bool c2[PRO ? NS : 1];
  bool pone[NS];  // element P is element 1 of the pair
  bool k0[RST ? NS : 1], k1[RST ? NS : 1];  // element 0 / 1 inside the grid
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const int q = threadIdx.x + NT * i;
    live[i] = q < PL;
    const int qc = live[i] ? q : PL - 1;
    const int p = qc % EXP, r = qc / EXP;
    const int xb = X0 - 2 * HPL + 2 * p;
    const int y = DIM == 3 ? Y0 - HYL + r : 0;
    const bool yin = DIM == 2 || (y >= 0 && y < m);
    const int par = (y + DIM) & 1;
    const int off = (DIM == 3 ? y * m : 0) + xb;
    const bool in0 = live[i] && yin && xb >= 0 && xb < m;
    const bool in1 = live[i] && yin && xb + 1 >= 0 && xb + 1 < m;
    const bool outp = live[i] && yin && p >= HPL && p < HPL + TXP &&
                      (DIM == 2 || (r >= HYL && r < HYL + TY)) && xb < m;
    const int o0 = in0 ? off * (int)sizeof(T) : kOOB;
    const int o1 = in1 ? (off + 1) * (int)sizeof(T) : kOOB;
    const bool half = in0 && !in1;
    o2[i] = in0 ? (off - (half ? 1 : 0)) * (int)sizeof(T) : kOOB;
    hP[i] = par ? true : half;
    hQ[i] = par ? half : true;
    kP[i] = par ? in1 : in0;
    kQ[i] = par ? in0 : in1;
    w2[i] = (outp && in1) ? o0 : kOOB;
    w1[i] = (outp && half) ? o0 : kOOB;
    nP[i] = outp && kP[i];
    nQ[i] = outp && kQ[i];
    lq[i] = qc;
    const int left = max(qc - 1, 0), right = min(qc + 1, PL - 1);
    lP[i] = par ? right : left;  // element 1 updates from the pair to its right
    lQ[i] = par ? left : right;
    lu[i] = max(qc - EXP, 0);
    ld[i] = min(qc + EXP, PL - 1);
    pone[i] = par != 0;
    if (RST) {
      k0[i] = in0;
      k1[i] = in1;
    }
    if (PRO) {
      const int rr = DIM == 3 ? r : 0;
      c2[i] = DIM == 3 && !(rr & 1);
      cb[i] = (DIM == 3 ? ((rr & 1) ? (rr + 1) >> 1 : rr >> 1) * NCX : 0) + p;
    }
  }

  T W[S][NS][3];  // stage windows: [0] newest plane, [1] previous, [2] two back
  T WB[NORM ? NS : 1][3];
  T pu0[NS], pu1[NS];  // start value of the plane being entered (elements P, Q)
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int i = 0; i < NS; ++i) W[s][i][0] = W[s][i][1] = W[s][i][2] = T(0);
#pragma unroll
  for (int i = 0; i < (NORM ? NS : 1); ++i) WB[i][0] = WB[i][1] = WB[i][2] = T(0);
  double acc = 0.0;

  // RST: coarse planes c with fine centre 2c+1 in [Z0, Z1) belong to this
  // chunk; their residual planes are 2*CZ0 .. 2*CZ1
  const int mc = a.mc;
  const int CZ0 = Z0 >> 1, CZ1 = min(Z1 >> 1, mc);
  // steps in pairs from an even start; the extra leading or trailing step
  // only touches planes outside the exact region
  const int t0 = (Z0 - S - (RST ? 2 : 0)) & ~1;
  const int t1 = RST ? 2 * CZ1 + S + 3 : Z1 + S;

  // Loads run two steps ahead of their use: plane t + 2's start value and
  // right-hand side are issued during step t, right after plane t's raw
  // loads have been consumed, into the same registers (uR / fR, indexed by
  // plane parity, which is a compile-time index in the pair of steps).  Two
  // planes of loads are then in flight per workgroup while one is computed;
  // one plane's worth does not cover the memory latency.  The raw pairs are
  // only unpacked (element choice, zero boundary) when their plane is used,
  // so nothing waits on a load early.
  PairOf<T> uR[2][ZERO ? 1 : NS], fR[2][NS];
  auto issue_u = [&](int t, PairOf<T> *v) {
    if (ZERO) return;
    const __amdgpu_buffer_rsrc_t r = plane_rsrc(a.u_in, t, m, planeS);
#pragma unroll
    for (int i = 0; i < NS; ++i) v[i] = bload2<T>(r, o2[i]);
  };
  auto take_u = [&](const PairOf<T> *v, T *v0, T *v1) {
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      if (ZERO) {
        v0[i] = v1[i] = T(0);
      } else {
        v0[i] = kP[i] ? (hP[i] ? v[i].hi : v[i].lo) : T(0);
        v1[i] = kQ[i] ? (hQ[i] ? v[i].hi : v[i].lo) : T(0);
      }
    }
  };
  auto issue_f = [&](int z, PairOf<T> *v) {
    const __amdgpu_buffer_rsrc_t r = plane_rsrc(a.f, z, m, planeS);
#pragma unroll
    for (int i = 0; i < NS; ++i) v[i] = bload2<T>(r, o2[i]);
  };
  auto take_f = [&](const PairOf<T> *v, T *vP, T *vQ) {
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      vP[i] = hP[i] ? v[i].hi : v[i].lo;
      vQ[i] = hQ[i] ? v[i].hi : v[i].lo;
    }
  };
  issue_u(t0, uR[0]);
  issue_f(t0, fR[0]);
  issue_u(t0 + 1, uR[1]);
  issue_f(t0 + 1, fR[1]);

  // PRO geometry: tile origin (X0 - S, Y0 - S) is even in both axes, so pair
  // p reads coarse columns p (left) and p + 1 (right); an odd row r of the
  // extended tile lies on coarse row (r + 1) / 2, an even one halfway between
  // rows r / 2 and r / 2 + 1.
  const int CX0 = ((X0 - 2 * HPL) >> 1) - 1;
  const int CY0 = DIM == 3 ? ((Y0 - HYL) >> 1) - 1 : 0;
  const int cplane = DIM == 3 ? mc * mc : mc;
  int coff[NCP];
  if (PRO) {
#pragma unroll
    for (int k = 0; k < NCP; ++k) {
      const int j = threadIdx.x + NT * k;
      const int cx = CX0 + j % NCX, cy = CY0 + j / NCX;
      const bool ok = j < CPL && cx >= 0 && cx < mc && (DIM == 2 || (cy >= 0 && cy < mc));
      coff[k] = ok ? ((DIM == 3 ? cy * mc : 0) + cx) * (int)sizeof(T) : kOOB;
    }
  }
  auto load_c = [&](int cz, T *v) {
    const __amdgpu_buffer_rsrc_t r = plane_rsrc(a.e_c, cz, mc, cplane);
#pragma unroll
    for (int k = 0; k < NCP; ++k) v[k] = bload<T>(r, coff[k]);
  };
  auto store_c = [&](int cz, const T *v) {
    T *dst = cring + (cz & 1) * CPL;
#pragma unroll
    for (int k = 0; k < NCP; ++k) {
      const int j = threadIdx.x + NT * k;
      if (NCP * NT == CPL || j < CPL) dst[j] = v[k];
    }
  };
  // xy-interpolated correction of the two elements of slot i (element 0 /
  // element 1 of the pair) from one staged coarse plane, canonical order
  auto cxy = [&](int cz, int i, T &v0, T &v1) {
    const T *P = cring + (cz & 1) * CPL + cb[i];
    const T el = P[0], er = P[1];
    v0 = T(0.5) * (el + er);
    v1 = er;
    if (c2[i]) {
      const T fl = P[NCX], fr = P[NCX + 1];
      v0 = T(0.5) * (v0 + T(0.5) * (fl + fr));
      v1 = T(0.5) * (v1 + fr);
    }
  };
  if (PRO) {
    // coarse planes t0 / 2 - 1 and t0 / 2 (t0 is even)
    T cv[NCP];
    load_c((t0 >> 1) - 1, cv);
    store_c((t0 >> 1) - 1, cv);
    load_c(t0 >> 1, cv);
    store_c(t0 >> 1, cv);
    __syncthreads();
  }

  // right-hand side window: fP[j] / fQ[j] hold elements P / Q of f on plane
  // t - j (j = 0 .. NF - 1) during step t; stage s reads plane t - s.  Plane
  // t enters the window at the top of step t from its raw loads.
  constexpr int NF = S + 1 + (RST ? 1 : 0);  // RST: plane t-S-1 for the residual
  T fP[NF][NS], fQ[NF][NS];
#pragma unroll
  for (int j = 1; j < NF; ++j) {
    PairOf<T> v[NS];
    issue_f(t0 - j, v);
    take_f(v, fP[j], fQ[j]);
  }
  // RST: final values (elements 0 / 1) of planes t-S, t-S-1, t-S-2, and the
  // full-weighting accumulator of this thread's coarse point
  T fw0[RST ? NS : 1][3], fw1[RST ? NS : 1][3];
#pragma unroll
  for (int i = 0; i < (RST ? NS : 1); ++i)
    fw0[i][0] = fw0[i][1] = fw0[i][2] = fw1[i][0] = fw1[i][1] = fw1[i][2] = T(0);
  constexpr int NCC = DIM == 3 ? TXP * (TY / 2) : TXP;  // coarse points of the tile
  const int ccx = threadIdx.x % TXP, ccy = DIM == 3 ? threadIdx.x / TXP : 0;
  const int cgx = (X0 >> 1) + ccx, cgy = DIM == 3 ? (Y0 >> 1) + ccy : 0;
  const bool cown = RST && (int)threadIdx.x < NCC && cgx < mc && (DIM == 2 || cgy < mc);
  const int cq = (DIM == 3 ? (HYL + 2 * ccy + 1) * EXP : 0) + HPL + ccx;  // slot of the centre
  T cacc = T(0);
  static_assert(!RST || NCC <= NT, "one thread per coarse point");
  // PRO: coarse plane (t + 1) / 2 for the odd step t, loaded at the odd step
  // before it (right after that step staged its own plane in LDS)
  T cnext[NCP];
  if (PRO) load_c((t0 + 2) >> 1, cnext);

  auto step = [&](int t, auto tp_tag) {
    constexpr int TP = decltype(tp_tag)::value;  // t & 1
    auto isP = [](int s) { return (((C1 + s - 1) + TP - s) & 1) == 0; };
    constexpr bool B0P = ((C0 + TP - 1) & 1) == 0;  // colour-C0 element of plane t-1 is P
    const int zr = t - 1;
    const bool rin = NORM && zr >= Z0 && zr < Z1;
    // plane t: start value and right-hand side from the raw loads of step
    // t - 2, then plane t + 2's loads into the same registers
    take_u(uR[TP], pu0, pu1);
#pragma unroll
    for (int j = NF - 1; j >= 1; --j)
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        fP[j][i] = fP[j - 1][i];
        fQ[j][i] = fQ[j - 1][i];
      }
    take_f(fR[TP], fP[0], fQ[0]);
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      pin_value(pu0[i]);
      pin_value(pu1[i]);
      pin_value(fP[0][i]);
      pin_value(fQ[0][i]);
    }
    issue_u(t + 2, uR[TP]);
    issue_f(t + 2, fR[TP]);
    const T *Lprev = lds + (1 - TP) * NB * PL;  // planes published at step t-1

    // ---- RST: full weighting of the residual plane t-S-2 (published at step
    // t-1) onto this thread's coarse point: in-plane x, then y, then the
    // three fine planes of a coarse plane (1/4, 1/2, 1/4)
    if (RST) {
      const int zf = t - S - 2;  // zf & 1 == (TP + S) & 1: a compile-time choice
      const bool use = cown && zf >= 2 * CZ0 && zf <= 2 * CZ1;
      T sxy = T(0);
      if (use) {
        const T *R0 = rl + (1 - TP) * 2 * PL, *R1 = R0 + PL;
        auto row = [&](int q) {
          return T(0.25) * R0[q] + T(0.5) * R1[q] + T(0.25) * R0[q + 1];
        };
        if (DIM == 3)
          sxy = T(0.25) * row(cq - EXP) + T(0.5) * row(cq) + T(0.25) * row(cq + EXP);
        else
          sxy = row(cq);
      }
      if constexpr (((TP + S) & 1) != 0) {
        if (use) cacc += T(0.5) * sxy;
      } else {
        // a coarse plane is complete: store it (every lane issues the store;
        // it lands only for coarse points of this tile and chunk)
        const int c = zf / 2 - 1;
        const bool cin = zf >= 2 * CZ0 && zf <= 2 * CZ1 && c >= CZ0 && c < CZ1;
        const __amdgpu_buffer_rsrc_t rc = plane_rsrc_if(a.f_c, c, cin, cplane);
        bstore<T>(rc, use ? (cgy * mc + cgx) * (int)sizeof(T) : kOOB, cacc + T(0.25) * sxy);
        if (use) cacc = T(0.25) * sxy;
      }
    }

    // ---- stage 0: start value on plane t (colour C0 into the window)
    constexpr bool S0P = ((C0 + TP) & 1) == 0;  // colour-C0 element of plane t is P
    const bool tin = t >= 0 && t < m;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      T vP = pu0[i], vQ = pu1[i];
      if (PRO) {
        T c0, c1;
        if (TP == 1) {  // fine node t+1 even: on coarse plane (t-1)/2
          cxy((t - 1) >> 1, i, c0, c1);
        } else {        // between coarse planes t/2-1 and t/2
          T l0, l1, h0, h1;
          cxy((t >> 1) - 1, i, l0, l1);
          cxy(t >> 1, i, h0, h1);
          c0 = T(0.5) * (l0 + h0);
          c1 = T(0.5) * (l1 + h1);
        }
        const T cP = pone[i] ? c1 : c0, cQ = pone[i] ? c0 : c1;
        vP = (tin && kP[i]) ? vP + cP : vP;
        vQ = (tin && kQ[i]) ? vQ + cQ : vQ;
      }
      W[0][i][2] = W[0][i][1];
      W[0][i][1] = W[0][i][0];
      W[0][i][0] = S0P ? vP : vQ;
      if (NORM) {
        WB[i][2] = WB[i][1];
        WB[i][1] = WB[i][0];
        WB[i][0] = S0P ? vQ : vP;
      }
    }
    // ---- residual of the start value on plane t-1 (convergence test)
    if (NORM && rin) {
      const T *L0 = Lprev;           // colour C0 values of plane t-1
      const T *LB = Lprev + S * PL;  // colour C1 values of plane t-1
#pragma unroll
      for (int i = 0; i < NS; ++i) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {  // 0: the colour-C0 element, 1: the other
          const bool eP = (c == 0) == B0P;
          const T self = c == 0 ? W[0][i][1] : WB[i][1];
          const T own = c == 0 ? WB[i][1] : W[0][i][1];
          const T *Ln = c == 0 ? LB : L0;
          T nb = own + Ln[eP ? lP[i] : lQ[i]];
          if (DIM == 3) {
            nb += Ln[lu[i]];
            nb += Ln[ld[i]];
          }
          nb += c == 0 ? WB[i][2] : W[0][i][2];
          nb += c == 0 ? WB[i][0] : W[0][i][0];
          const T fv = eP ? fP[1][i] : fQ[1][i];
          const double r = double(fv) - (double(T(2 * DIM) * self) - double(nb)) * a.inv_h2;
          const bool use = eP ? nP[i] : nQ[i];
          acc += use ? r * r : 0.0;
        }
      }
    }
    // ---- stages 1..S
    T newS[NS];
#pragma unroll
    for (int s = 1; s <= S; ++s) {
      const int zs = t - s;
      const bool zin = zs >= 0 && zs < m;
      const T *L = Lprev + (s - 1) * PL;
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        T nb = W[s - 1][i][1] + L[isP(s) ? lP[i] : lQ[i]];  // x-1 and x+1 (one is the own pair)
        if (DIM == 3) {
          nb += L[lu[i]];  // y - 1
          nb += L[ld[i]];  // y + 1
        }
        nb += W[s - 1][i][2];  // marching axis - 1
        nb += W[s - 1][i][0];  // marching axis + 1
        const bool in = zin && (isP(s) ? kP[i] : kQ[i]);
        const T fv = isP(s) ? fP[s][i] : fQ[s][i];
        const T v = in ? point_solve<T, DIM>(h2, fv, nb) : T(0);
        if (NMID && s == QN) {
          // the updated colour's residual after stage QN, from the same
          // neighbour sum: plane t - QN
          const double r = double(fv) - (double(T(2 * DIM) * v) - double(nb)) * a.inv_h2;
          const bool use = zs >= Z0 && zs < Z1 && (isP(s) ? nP[i] : nQ[i]);
          acc += use ? r * r : 0.0;
        }
        if (s < S) {
          W[s][i][2] = W[s][i][1];
          W[s][i][1] = W[s][i][0];
          W[s][i][0] = v;
        } else {
          newS[i] = v;
        }
      }
    }
    // ---- NMID: the other colour's residual after stage QN on plane
    // t - QN - 1: its value from stage QN - 1, its neighbours (all of the
    // colour stage QN updated) from stage QN's window and published plane;
    // neighbour order x-1, x+1, y-1, y+1, z-1, z+1 as in the stages
    if (NMID) {
      const int zb = t - QN - 1;
      const bool bin = zb >= Z0 && zb < Z1;
      const T *Lq = Lprev + QN * PL;  // stage QN's plane zb (published at step t-1)
      constexpr bool EP = isP(QN - 1);     // the colour of stage QN - 1 is element P
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        T nb = W[QN][i][1] + Lq[EP ? lP[i] : lQ[i]];
        if (DIM == 3) {
          nb += Lq[lu[i]];
          nb += Lq[ld[i]];
        }
        nb += W[QN][i][2];
        nb += W[QN][i][0];
        const T fv = EP ? fP[QN + 1][i] : fQ[QN + 1][i];
        const double r =
            double(fv) - (double(T(2 * DIM) * W[QN - 1][i][2]) - double(nb)) * a.inv_h2;
        const bool use = bin && (EP ? nP[i] : nQ[i]);
        acc += use ? r * r : 0.0;
      }
    }
    // ---- output plane t-S: last stage's colour from newS, the other from
    // S-1; both elements in one store (the tile at the high x end of a grid
    // of odd side adds the 8-byte store of its row-end elements)
    const int zo = t - S;
    {
      const __amdgpu_buffer_rsrc_t r = plane_rsrc_if(a.u_out, zo, zo >= Z0 && zo < Z1, planeS);
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        const T vP = isP(S) ? newS[i] : W[S - 1][i][1];
        const T vQ = isP(S) ? W[S - 1][i][1] : newS[i];
        const T e0 = pone[i] ? vQ : vP, e1 = pone[i] ? vP : vQ;
        bstore2<T>(r, w2[i], e0, e1);
        if (xend) bstore<T>(r, w1[i], e0);
      }
    }
    // ---- RST: final values of plane t-S into the window; residual of plane
    // t-S-1 (same expression as the separate restriction kernel: neighbours
    // x-1, x+1, y-1, y+1, z-1, z+1 in that order)
    T *FWnow = fwl + TP * 2 * PL;
    T *Rnow = rl + TP * 2 * PL;
    if (RST) {
      const T *F0 = fwl + (1 - TP) * 2 * PL, *F1 = F0 + PL;  // plane t-S-1
      const int zw = t - S - 1;
      const bool win = zw >= 0 && zw < m;
      const T inv_h2 = T(a.inv_h2);
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        const T vP = isP(S) ? newS[i] : W[S - 1][i][1];
        const T vQ = isP(S) ? W[S - 1][i][1] : newS[i];
        fw0[i][2] = fw0[i][1];
        fw0[i][1] = fw0[i][0];
        fw0[i][0] = pone[i] ? vQ : vP;
        fw1[i][2] = fw1[i][1];
        fw1[i][1] = fw1[i][0];
        fw1[i][0] = pone[i] ? vP : vQ;
        const int q = lq[i];
        const int left = max(q - 1, 0), right = min(q + 1, PL - 1);
        const T f0 = pone[i] ? fQ[S + 1][i] : fP[S + 1][i];
        const T f1 = pone[i] ? fP[S + 1][i] : fQ[S + 1][i];
        T nb0 = F1[left] + fw1[i][1];
        T nb1 = fw0[i][1] + F0[right];
        if (DIM == 3) {
          nb0 += F0[lu[i]];
          nb0 += F0[ld[i]];
          nb1 += F1[lu[i]];
          nb1 += F1[ld[i]];
        }
        nb0 += fw0[i][2];
        nb0 += fw0[i][0];
        nb1 += fw1[i][2];
        nb1 += fw1[i][0];
        const T r0 = f0 - (T(2 * DIM) * fw0[i][1] - nb0) * inv_h2;
        const T r1 = f1 - (T(2 * DIM) * fw1[i][1] - nb1) * inv_h2;
        if (TAIL && i == NS - 1 && !live[i]) continue;
        Rnow[q] = (win && k0[i]) ? r0 : T(0);
        Rnow[PL + q] = (win && k1[i]) ? r1 : T(0);
        FWnow[q] = fw0[i][0];
        FWnow[PL + q] = fw1[i][0];
      }
    }
    // ---- publish the newest plane of every stage for step t+1
    T *Lnow = lds + TP * NB * PL;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      if (TAIL && i == NS - 1 && !live[i]) continue;
#pragma unroll
      for (int s = 0; s < S; ++s) Lnow[s * PL + lq[i]] = W[s][i][0];
      if (NORM) Lnow[S * PL + lq[i]] = WB[i][0];
    }
    if (PRO && TP == 1) {
      store_c((t + 1) >> 1, cnext);
      compiler_fence();
      load_c((t + 3) >> 1, cnext);
    }
    __syncthreads();
  };
  for (int t = t0; t < t1; t += 2) {
    step(t, IntC<0>());
    step(t + 1, IntC<1>());
  }
  if (NORM || NMID) block_sum_store<NT>(acc, gbl(a.partials));
}

// ------------------------------------------------------------------------
// Weighted-Jacobi pass: S full sweeps, every stage updates both elements of
// every pair from the previous stage's values.  Same pipeline, memory access
// and fusions as the red-black pass (buffer loads with zero-boundary range
// checks, pair loads, right-hand-side window, step-parity LDS buffers, the
// coarse correction staged in LDS); a stage publishes both elements.
// ------------------------------------------------------------------------
template <typename T, int DIM, int S, int EXP, int EY, int NT, int FL>
__global__ void __launch_bounds__(NT) k_wj_pass(PassArgs<T> arg, const PassArgs<T> *tbl) {
  const PassArgs<T> a = entry_of(arg, tbl);
  if (a.active && *gbl(a.active) == 0) return;
  constexpr int PL = EXP * EY;
  constexpr int NS = (PL + NT - 1) / NT;
  constexpr bool TAIL = NS * NT > PL;
  constexpr int HP = (S + 1) / 2;  // halo in pairs (>= S points)
  constexpr int H = 2 * HP;        // halo in rows (3D)
  constexpr int TXP = EXP - 2 * HP;
  constexpr int TY = DIM == 3 ? EY - 2 * H : 1;
  constexpr bool ZERO = (FL & F_ZERO_IN) != 0;
  constexpr bool PRO = (FL & F_PROLONG) != 0;
  constexpr bool NORM = (FL & F_NORM_IN) != 0;
  constexpr int NCX = EXP + 1;
  constexpr int NCY = DIM == 3 ? EY / 2 + 1 : 1;
  constexpr int CPL = NCX * NCY;
  constexpr int NCP = PRO ? (CPL + NT - 1) / NT : 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // [2 (step parity)][S][2 (element)][PL], then PRO: [2][CPL]
  T *lds = reinterpret_cast<T *>(smem_raw);
  T *cring = lds + 4 * S * PL;

  const int m = a.m;
  int tx, ty, tzc;
  tile_coords<DIM>(xcd_remap(blockIdx.x, a.nblocks), a.ntx, a.nty, a.sw, tx, ty, tzc);
  const int X0 = tx * 2 * TXP;
  const bool xend = (m & 1) && X0 + 2 * TXP >= m;  // the output tile holds x = m - 1
  const int Y0 = ty * TY;
  const int Z0 = tzc * a.tz;
  const int Z1 = min(Z0 + a.tz, m);
  const int planeS = DIM == 3 ? m * m : m;
  const T h2 = T(a.h2);
  const T om = T(a.omega);
  const T om1 = T(1.0 - a.omega);

  // per-slot geometry (see the red-black pass; here elements keep their
  // index: k0 / k1 element inside the grid, h0 element 0 is the high half of
  // the pair load)
  // stores as in the red-black pass: w2 a whole pair, w1 a row-end element
  int o2[NS], w2[NS], w1[NS], lq[NS], lft[NS], rgt[NS], lu[NS], ld[NS];
  bool h0[NS], k0[NS], k1[NS], n0[NS], n1[NS], live[NS];
  int cb[PRO ? NS : 1];
  bool c2[PRO ? NS : 1];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const int q = threadIdx.x + NT * i;
    live[i] = q < PL;
    const int qc = live[i] ? q : PL - 1;
    const int p = qc % EXP, r = qc / EXP;
    const int xb = X0 - H + 2 * p;
    const int y = DIM == 3 ? Y0 - H + r : 0;
    const bool yin = DIM == 2 || (y >= 0 && y < m);
    const int off = (DIM == 3 ? y * m : 0) + xb;
    const bool in0 = live[i] && yin && xb >= 0 && xb < m;
    const bool in1 = live[i] && yin && xb + 1 >= 0 && xb + 1 < m;
    const bool outp = live[i] && yin && p >= HP && p < HP + TXP &&
                      (DIM == 2 || (r >= H && r < H + TY)) && xb < m;
    const bool half = in0 && !in1;
    o2[i] = in0 ? (off - (half ? 1 : 0)) * (int)sizeof(T) : kOOB;
    h0[i] = half;
    k0[i] = in0;
    k1[i] = in1;
    w2[i] = (outp && in1) ? off * (int)sizeof(T) : kOOB;
    w1[i] = (outp && half) ? off * (int)sizeof(T) : kOOB;
    n0[i] = outp && in0;
    n1[i] = outp && in1;
    lq[i] = qc;
    lft[i] = max(qc - 1, 0);
    rgt[i] = min(qc + 1, PL - 1);
    lu[i] = max(qc - EXP, 0);
    ld[i] = min(qc + EXP, PL - 1);
    if (PRO) {
      const int rr = DIM == 3 ? r : 0;
      c2[i] = DIM == 3 && !(rr & 1);
      cb[i] = (DIM == 3 ? ((rr & 1) ? (rr + 1) >> 1 : rr >> 1) * NCX : 0) + p;
    }
  }

  T W[S][NS][2][3];  // stage windows per element: [0] newest plane
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int i = 0; i < NS; ++i)
#pragma unroll
      for (int e = 0; e < 2; ++e) W[s][i][e][0] = W[s][i][e][1] = W[s][i][e][2] = T(0);
  double acc = 0.0;

  const int t0 = (Z0 - S) & ~1, t1 = Z1 + S;
  auto load_pair = [&](const T *base, int z, T *v0, T *v1, bool mask) {
    const __amdgpu_buffer_rsrc_t rs = plane_rsrc(base, z, m, planeS);
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const PairOf<T> v = bload2<T>(rs, o2[i]);
      const T e0 = h0[i] ? v.hi : v.lo, e1 = v.hi;
      v0[i] = (!mask || k0[i]) ? e0 : T(0);
      v1[i] = (!mask || k1[i]) ? e1 : T(0);
    }
  };
  T pu0[NS], pu1[NS];
  if (ZERO) {
#pragma unroll
    for (int i = 0; i < NS; ++i) pu0[i] = pu1[i] = T(0);
  } else {
    load_pair(a.u_in, t0, pu0, pu1, true);
  }
  T fe0[S + 1][NS], fe1[S + 1][NS];  // f of plane t - j, elements 0 / 1
#pragma unroll
  for (int j = 0; j <= S; ++j) load_pair(a.f, t0 - j, fe0[j], fe1[j], false);

  const int CX0 = ((X0 - H) >> 1) - 1;
  const int CY0 = DIM == 3 ? ((Y0 - H) >> 1) - 1 : 0;
  const int mc = a.mc;
  const int cplane = DIM == 3 ? mc * mc : mc;
  int coff[NCP];
  if (PRO) {
#pragma unroll
    for (int k = 0; k < NCP; ++k) {
      const int j = threadIdx.x + NT * k;
      const int cx = CX0 + j % NCX, cy = CY0 + j / NCX;
      const bool ok = j < CPL && cx >= 0 && cx < mc && (DIM == 2 || (cy >= 0 && cy < mc));
      coff[k] = ok ? ((DIM == 3 ? cy * mc : 0) + cx) * (int)sizeof(T) : kOOB;
    }
  }
  auto load_c = [&](int cz, T *v) {
    const __amdgpu_buffer_rsrc_t rs = plane_rsrc(a.e_c, cz, mc, cplane);
#pragma unroll
    for (int k = 0; k < NCP; ++k) v[k] = bload<T>(rs, coff[k]);
  };
  auto store_c = [&](int cz, const T *v) {
    T *dst = cring + (cz & 1) * CPL;
#pragma unroll
    for (int k = 0; k < NCP; ++k) {
      const int j = threadIdx.x + NT * k;
      if (NCP * NT == CPL || j < CPL) dst[j] = v[k];
    }
  };
  auto cxy = [&](int cz, int i, T &v0, T &v1) {
    const T *P = cring + (cz & 1) * CPL + cb[i];
    const T el = P[0], er = P[1];
    v0 = T(0.5) * (el + er);
    v1 = er;
    if (c2[i]) {
      const T fl = P[NCX], fr = P[NCX + 1];
      v0 = T(0.5) * (v0 + T(0.5) * (fl + fr));
      v1 = T(0.5) * (v1 + fr);
    }
  };
  T cnext[NCP];
  if (PRO) {
    T cv[NCP];
    load_c((t0 >> 1) - 1, cv);
    store_c((t0 >> 1) - 1, cv);
    load_c(t0 >> 1, cv);
    store_c(t0 >> 1, cv);
    load_c((t0 + 2) >> 1, cnext);
    __syncthreads();
  }

  // the stencil sum of element e around the previous stage's plane: x-1,
  // x+1, y-1, y+1, z-1, z+1 in that order
  auto nbsum = [&](const T *L, const T (&Wp)[NS][2][3], int i, int e) {
    const T *Ln = L + (1 - e) * PL;  // the other element of neighbouring pairs
    const T *Ls = L + e * PL;        // same element (y neighbours)
    const T own = Wp[i][1 - e][1];
    const T side = e ? Ln[rgt[i]] : Ln[lft[i]];
    T nb = e ? own : side;
    nb += e ? side : own;
    if (DIM == 3) {
      nb += Ls[lu[i]];
      nb += Ls[ld[i]];
    }
    nb += Wp[i][e][2];
    nb += Wp[i][e][0];
    return nb;
  };

  auto step = [&](int t, auto tp_tag) {
    constexpr int TP = decltype(tp_tag)::value;
    T nu0[NS], nu1[NS];
    if (!ZERO) load_pair(a.u_in, t + 1, nu0, nu1, true);
    T fn0[NS], fn1[NS];
    load_pair(a.f, t + 1, fn0, fn1, false);
    T cnn[NCP];
    if (PRO && TP == 1) load_c((t + 3) >> 1, cnn);
    const T *Lprev = lds + (1 - TP) * 2 * S * PL;
    // ---- stage 0: start value of plane t
    const bool tin = t >= 0 && t < m;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      T v0 = pu0[i], v1 = pu1[i];
      if (PRO) {
        T c0, c1;
        if (TP == 1) {
          cxy((t - 1) >> 1, i, c0, c1);
        } else {
          T l0, l1, g0, g1;
          cxy((t >> 1) - 1, i, l0, l1);
          cxy(t >> 1, i, g0, g1);
          c0 = T(0.5) * (l0 + g0);
          c1 = T(0.5) * (l1 + g1);
        }
        v0 = (tin && k0[i]) ? v0 + c0 : v0;
        v1 = (tin && k1[i]) ? v1 + c1 : v1;
      }
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        W[0][i][e][2] = W[0][i][e][1];
        W[0][i][e][1] = W[0][i][e][0];
      }
      W[0][i][0][0] = v0;
      W[0][i][1][0] = v1;
    }
    // ---- residual of the start value on plane t-1 (convergence test)
    if (NORM) {
      const int zr = t - 1;
      if (zr >= Z0 && zr < Z1) {
#pragma unroll
        for (int i = 0; i < NS; ++i) {
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            const T nb = nbsum(Lprev, W[0], i, e);
            const T fv = e ? fe1[1][i] : fe0[1][i];
            const double r =
                double(fv) - (double(T(2 * DIM) * W[0][i][e][1]) - double(nb)) * a.inv_h2;
            acc += (e ? n1[i] : n0[i]) ? r * r : 0.0;
          }
        }
      }
    }
    // ---- stages 1..S
    T newS[NS][2];
#pragma unroll
    for (int s = 1; s <= S; ++s) {
      const int zs = t - s;
      const bool zin = zs >= 0 && zs < m;
      const T *L = Lprev + (s - 1) * 2 * PL;
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        T nv[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const T nb = nbsum(L, W[s - 1], i, e);
          const T fv = e ? fe1[s][i] : fe0[s][i];
          const bool in = zin && (e ? k1[i] : k0[i]);
          nv[e] = in ? om1 * W[s - 1][i][e][1] + om * point_solve<T, DIM>(h2, fv, nb) : T(0);
        }
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          if (s < S) {
            W[s][i][e][2] = W[s][i][e][1];
            W[s][i][e][1] = W[s][i][e][0];
            W[s][i][e][0] = nv[e];
          } else {
            newS[i][e] = nv[e];
          }
        }
      }
    }
    // ---- output plane t-S
    const int zo = t - S;
    if (zo >= Z0 && zo < Z1) {
      const __amdgpu_buffer_rsrc_t rs = plane_rsrc(a.u_out, zo, m, planeS);
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        bstore2<T>(rs, w2[i], newS[i][0], newS[i][1]);
        if (xend) bstore<T>(rs, w1[i], newS[i][0]);
      }
    }
    // ---- publish the newest plane of every stage (both elements)
    T *Lnow = lds + TP * 2 * S * PL;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      if (TAIL && i == NS - 1 && !live[i]) continue;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        Lnow[(2 * s) * PL + lq[i]] = W[s][i][0][0];
        Lnow[(2 * s + 1) * PL + lq[i]] = W[s][i][1][0];
      }
    }
    if (PRO && TP == 1) store_c((t + 1) >> 1, cnext);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      if (!ZERO) {
        pu0[i] = nu0[i];
        pu1[i] = nu1[i];
      }
#pragma unroll
      for (int j = S; j >= 1; --j) {
        fe0[j][i] = fe0[j - 1][i];
        fe1[j][i] = fe1[j - 1][i];
      }
      fe0[0][i] = fn0[i];
      fe1[0][i] = fn1[i];
    }
    if (PRO && TP == 1) {
#pragma unroll
      for (int k = 0; k < NCP; ++k) cnext[k] = cnn[k];
    }
  };
  for (int t = t0; t < t1; t += 2) {
    step(t, IntC<0>());
    step(t + 1, IntC<1>());
  }
  if (NORM) block_sum_store<NT>(acc, gbl(a.partials));
}

// ------------------------------------------------------------------------
// Tile tables and dispatch.
// ------------------------------------------------------------------------
// Each entry: pairs per extended row, extended rows, threads.  Output tile:
// TX = 2*(EXP - 2*halo_pairs), TY = EY - 2*halo (3D).
#define GMG_RB3_S2(X) \
  X(3, 2, 66, 30, 1024) X(3, 2, 34, 20, 256) X(3, 2, 66, 14, 512) X(3, 2, 34, 30, 1024)
#define GMG_RB3_S4(X) X(3, 4, 36, 28, 1024) X(3, 4, 36, 24, 256) X(3, 4, 68, 22, 512) X(3, 4, 36, 24, 896)
// Three stages (black, red, black): the pass that ends one cycle's backward
// V(1,1) post-smoothing and starts the next cycle's forward sweep.
// (Tiles with an even row count run the plain form, odd ones the form with
// the restriction folded in: its halo is one row taller on the high side.)
#define GMG_RB3_S3(X) \
  X(3, 3, 34, 30, 1024) X(3, 3, 36, 28, 1024) X(3, 3, 66, 30, 1024) X(3, 3, 34, 30, 512) \
  X(3, 3, 66, 14, 512) X(3, 3, 34, 29, 1024) X(3, 3, 36, 27, 1024) X(3, 3, 33, 31, 1024)
#define GMG_RB2_S3(X) X(2, 3, 64, 1, 64) X(2, 3, 128, 1, 128)
#define GMG_RB2_S2(X) X(2, 2, 64, 1, 64) X(2, 2, 128, 1, 128)
#define GMG_RB2_S4(X) X(2, 4, 64, 1, 64) X(2, 4, 128, 1, 128)
#define GMG_WJ3_S1(X) X(3, 1, 34, 30, 1024) X(3, 1, 66, 14, 1024) X(3, 1, 34, 14, 512)
#define GMG_WJ3_S2(X) X(3, 2, 34, 30, 1024) X(3, 2, 66, 14, 1024) X(3, 2, 34, 14, 512)
#define GMG_WJ2_S1(X) X(2, 1, 64, 1, 64) X(2, 1, 128, 1, 128)
#define GMG_WJ2_S2(X) X(2, 2, 64, 1, 64) X(2, 2, 128, 1, 128)

namespace {
struct TileRow {
  int dim, s, exp_, ey, nt;
};
#define GMG_ROW(D, S, E, Y, N) {D, S, E, Y, N},
const TileRow kRbTiles[] = {GMG_RB3_S2(GMG_ROW) GMG_RB3_S4(GMG_ROW) GMG_RB2_S2(GMG_ROW)
                                GMG_RB2_S4(GMG_ROW) GMG_RB3_S3(GMG_ROW) GMG_RB2_S3(GMG_ROW)};
const TileRow kWjTiles[] = {GMG_WJ3_S1(GMG_ROW) GMG_WJ3_S2(GMG_ROW) GMG_WJ2_S1(GMG_ROW)
                                GMG_WJ2_S2(GMG_ROW)};
#undef GMG_ROW

template <int N>
int find_rows(const TileRow (&tab)[N], int dim, int s, int *idx) {
  int n = 0;
  for (int i = 0; i < N; ++i)
    if (tab[i].dim == dim && tab[i].s == s) idx[n++] = i;
  return n;
}
}  // namespace

int pass_variant_count(int dim, int stages, int wj) {
  int idx[16];
  return wj ? find_rows(kWjTiles, dim, stages, idx) : find_rows(kRbTiles, dim, stages, idx);
}

PassTile pass_variant(int dim, int stages, int wj, int v) {
  int idx[16];
  int n = wj ? find_rows(kWjTiles, dim, stages, idx) : find_rows(kRbTiles, dim, stages, idx);
  PassTile t{0, 0, 0};
  if (n == 0) return t;
  if (v < 0 || v >= n) v = 0;
  const TileRow &r = wj ? kWjTiles[idx[v]] : kRbTiles[idx[v]];
  t.exp_ = r.exp_;
  t.ey = r.ey;
  t.nt = r.nt;
  return t;
}

uint32_t tile_table_hash() {
  uint32_t h = 2166136261u;
  auto mix = [&](int v) {
    for (int b = 0; b < 4; ++b) {
      h ^= (uint32_t)(v >> (8 * b)) & 0xffu;
      h *= 16777619u;
    }
  };
  for (const TileRow &r : kRbTiles) {
    mix(r.dim); mix(r.s); mix(r.exp_); mix(r.ey); mix(r.nt);
  }
  mix(-1);
  for (const TileRow &r : kWjTiles) {
    mix(r.dim); mix(r.s); mix(r.exp_); mix(r.ey); mix(r.nt);
  }
  return h;
}

size_t rb_pass_lds_bytes(int dim, int stages, int exp_, int ey, int flags, size_t elem) {
  const size_t pl = (size_t)exp_ * ey;
  size_t n = 2 * pl * (size_t)(stages + ((flags & F_NORM_IN) ? 1 : 0));
  if (flags & F_RESTRICT) n += 8 * pl;
  if (flags & F_PROLONG) n += 2 * (size_t)(exp_ + 1) * (dim == 3 ? (ey + 1) / 2 + 1 : 1);
  return n * elem;
}

bool rb_pass_fits(int dim, int stages, int variant, int flags, size_t elem) {
  const PassTile t = pass_variant(dim, stages, 0, variant);
  if (t.nt == 0) return false;
  const RbHalo h = rb_halo(stages, (flags & F_RESTRICT) != 0);
  const int txp = t.exp_ - h.pl - h.ph, ty = dim == 3 ? t.ey - h.yl - h.yh : 2;
  return txp > 0 && ty > 0 && ty % 2 == 0 &&
         rb_pass_lds_bytes(dim, stages, t.exp_, t.ey, flags, elem) <= kMaxPassLds;
}

PassGeom pass_geometry(int dim, int m, int stages, const PassTile &t, int tz, bool restrict_) {
  // the red-black halo (rb_halo); Jacobi passes use the plain one (S points
  // rounded up to a pair on each side)
  const RbHalo h = rb_halo(stages, restrict_);
  const int tx = 2 * (t.exp_ - h.pl - h.ph);
  PassGeom g;
  g.ntx = (m + tx - 1) / tx;
  if (dim == 3) {
    const int ty = t.ey - h.yl - h.yh;
    g.nty = (m + ty - 1) / ty;
  } else {
    g.nty = 1;
  }
  g.tz = tz > 0 ? tz : m;
  if (g.tz > m) g.tz = m;
  g.ntz = (m + g.tz - 1) / g.tz;
  g.nblocks = g.ntx * g.nty * g.ntz;
  return g;
}

namespace {
template <typename T, int DIM, int S, int EXP, int EY, int NT, int FL>
hipError_t run_rb(PassArgs<T> a, hipStream_t st, const PassArgs<T> *tbl, int nent) {
  constexpr RbHalo h = rb_halo(S, (FL & F_RESTRICT) != 0);
  constexpr int txp = EXP - h.pl - h.ph, ty = DIM == 3 ? EY - h.yl - h.yh : 2;
  if constexpr (txp <= 0 || ty <= 0 || ty % 2 != 0) {
    return hipErrorInvalidValue;  // this tile does not run this form
  } else {
  const size_t lds = rb_pass_lds_bytes(DIM, S, EXP, EY, FL, sizeof(T));
  if (lds > kMaxPassLds) return hipErrorInvalidConfiguration;
  auto k = k_rb_pass<T, DIM, S, EXP, EY, NT, FL>;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  gmg_launch(k, dim3(a.nblocks, nent), dim3(NT), lds, st, a, tbl);
  return hipGetLastError();
  }
}

template <typename T, int DIM, int S, int EXP, int EY, int NT, int FL>
hipError_t run_wj(PassArgs<T> a, hipStream_t st, const PassArgs<T> *tbl, int nent) {
  // two step-parity buffers of S planes of both elements, then the coarse ring
  const size_t cpl = (FL & F_PROLONG) ? 2 * (size_t)(EXP + 1) * (DIM == 3 ? EY / 2 + 1 : 1) : 0;
  const size_t lds = sizeof(T) * (4 * (size_t)S * EXP * EY + cpl);
  auto k = k_wj_pass<T, DIM, S, EXP, EY, NT, FL>;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  gmg_launch(k, dim3(a.nblocks, nent), dim3(NT), lds, st, a, tbl);
  return hipGetLastError();
}

// The fused-flag combinations a cycle uses (restriction: red-black only).
#define GMG_RST_CASES_run_rb(RUN, T, D, S, E, Y, N)                                          \
  case F_RESTRICT: return RUN<T, D, S, E, Y, N, F_RESTRICT>(a, st, tbl, nent);              \
  case F_RESTRICT | F_ZERO_IN: return RUN<T, D, S, E, Y, N, F_RESTRICT | F_ZERO_IN>(a, st, tbl, nent); \
  case F_RESTRICT | F_NORM_IN: return RUN<T, D, S, E, Y, N, F_RESTRICT | F_NORM_IN>(a, st, tbl, nent);
#define GMG_RST_CASES_run_wj(RUN, T, D, S, E, Y, N)
#define GMG_RST_CASES(RUN, T, D, S, E, Y, N) GMG_RST_CASES_##RUN(RUN, T, D, S, E, Y, N)
#define GMG_FLAG_SWITCH(RUN, T, D, S, E, Y, N)                                            \
  switch (flags) {                                                                     \
    case 0: return RUN<T, D, S, E, Y, N, 0>(a, st, tbl, nent);                                    \
    case F_ZERO_IN: return RUN<T, D, S, E, Y, N, F_ZERO_IN>(a, st, tbl, nent);                    \
    case F_PROLONG: return RUN<T, D, S, E, Y, N, F_PROLONG>(a, st, tbl, nent);                    \
    case F_NORM_IN: return RUN<T, D, S, E, Y, N, F_NORM_IN>(a, st, tbl, nent);                    \
    case F_BLACK_FIRST: return RUN<T, D, S, E, Y, N, F_BLACK_FIRST>(a, st, tbl, nent);            \
    case F_ZERO_IN | F_BLACK_FIRST: return RUN<T, D, S, E, Y, N, F_ZERO_IN | F_BLACK_FIRST>(a, st, tbl, nent); \
    case F_PROLONG | F_BLACK_FIRST: return RUN<T, D, S, E, Y, N, F_PROLONG | F_BLACK_FIRST>(a, st, tbl, nent); \
    case F_NORM_IN | F_BLACK_FIRST: return RUN<T, D, S, E, Y, N, F_NORM_IN | F_BLACK_FIRST>(a, st, tbl, nent); \
    GMG_RST_CASES(RUN, T, D, S, E, Y, N)                                               \
    default: return hipErrorInvalidValue;                                              \
  }
}  // namespace

// The three-stage pass runs in two forms only: interpolated correction in,
// mid-pass norm (FP64 solves) or none (the FP32 cycles of a refinement step),
// with or without the folded restriction.
#define GMG_CROSS_SWITCH(RUN, T, D, S, E, Y, N)                                        \
  switch (flags) {                                                                  \
    case F_PROLONG | F_BLACK_FIRST | F_NORM_MID:                                    \
      return RUN<T, D, S, E, Y, N, F_PROLONG | F_BLACK_FIRST | F_NORM_MID>(a, st, tbl, nent); \
    case F_PROLONG | F_BLACK_FIRST | F_NORM_MID | F_RESTRICT:                       \
      return RUN<T, D, S, E, Y, N, F_PROLONG | F_BLACK_FIRST | F_NORM_MID | F_RESTRICT>(   \
          a, st, tbl, nent);                                                        \
    default: return hipErrorInvalidValue;                                           \
  }

#define GMG_CROSS32_SWITCH(RUN, T, D, S, E, Y, N)                                      \
  switch (flags) {                                                                  \
    case F_PROLONG | F_BLACK_FIRST:                                                 \
      return RUN<T, D, S, E, Y, N, F_PROLONG | F_BLACK_FIRST>(a, st, tbl, nent);    \
    case F_PROLONG | F_BLACK_FIRST | F_RESTRICT:                                    \
      return RUN<T, D, S, E, Y, N, F_PROLONG | F_BLACK_FIRST | F_RESTRICT>(a, st, tbl, nent); \
    default: return hipErrorInvalidValue;                                           \
  }

template <typename T>
hipError_t launch_rb_pass(int dim, int stages, int flags, int variant, PassArgs<T> a,
                          hipStream_t st, const PassArgs<T> *tbl, int nent) {
  const PassTile t = pass_variant(dim, stages, 0, variant);
  if (t.nt == 0) return hipErrorInvalidValue;
#define GMG_TRY(D, S, E, Y, N)                                       \
  if (dim == D && stages == S && t.exp_ == E && t.ey == Y && t.nt == N) { \
    GMG_FLAG_SWITCH(run_rb, T, D, S, E, Y, N)                         \
  }
  GMG_RB3_S2(GMG_TRY) GMG_RB3_S4(GMG_TRY) GMG_RB2_S2(GMG_TRY) GMG_RB2_S4(GMG_TRY)
#undef GMG_TRY
  if constexpr (sizeof(T) == 8) {
#define GMG_TRY(D, S, E, Y, N)                                       \
  if (dim == D && stages == S && t.exp_ == E && t.ey == Y && t.nt == N) { \
    GMG_CROSS_SWITCH(run_rb, T, D, S, E, Y, N)                        \
  }
    GMG_RB3_S3(GMG_TRY) GMG_RB2_S3(GMG_TRY)
#undef GMG_TRY
  } else {
    // FP32 (the inner cycles of the mixed form): no norm between them
#define GMG_TRY(D, S, E, Y, N)                                       \
  if (dim == D && stages == S && t.exp_ == E && t.ey == Y && t.nt == N) { \
    GMG_CROSS32_SWITCH(run_rb, T, D, S, E, Y, N)                      \
  }
    GMG_RB3_S3(GMG_TRY) GMG_RB2_S3(GMG_TRY)
#undef GMG_TRY
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_wj_pass(int dim, int sweeps, int flags, int variant, PassArgs<T> a,
                          hipStream_t st, const PassArgs<T> *tbl, int nent) {
  const PassTile t = pass_variant(dim, sweeps, 1, variant);
  if (t.nt == 0) return hipErrorInvalidValue;
  flags &= ~F_BLACK_FIRST;
#define GMG_TRY(D, S, E, Y, N)                                       \
  if (dim == D && sweeps == S && t.exp_ == E && t.ey == Y && t.nt == N) { \
    GMG_FLAG_SWITCH(run_wj, T, D, S, E, Y, N)                         \
  }
  GMG_WJ3_S1(GMG_TRY) GMG_WJ3_S2(GMG_TRY) GMG_WJ2_S1(GMG_TRY) GMG_WJ2_S2(GMG_TRY)
#undef GMG_TRY
  return hipErrorInvalidValue;
}

template hipError_t launch_rb_pass<double>(int, int, int, int, PassArgs<double>, hipStream_t,
                                           const PassArgs<double> *, int);
template hipError_t launch_rb_pass<float>(int, int, int, int, PassArgs<float>, hipStream_t,
                                          const PassArgs<float> *, int);
template hipError_t launch_wj_pass<double>(int, int, int, int, PassArgs<double>, hipStream_t,
                                           const PassArgs<double> *, int);
template hipError_t launch_wj_pass<float>(int, int, int, int, PassArgs<float>, hipStream_t,
                                          const PassArgs<float> *, int);

}  // namespace gmg
