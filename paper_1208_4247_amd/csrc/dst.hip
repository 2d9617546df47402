// dst.hip -- exact solve of the discrete Poisson problem (the 5-/7-point
// scheme with zero Dirichlet data, Sec. 2.2) by the discrete sine transform
// (DST-I), the fast direct method the paper compares full multigrid with
// (Sec. 5.4, Tables 12-15).  The sine modes prod_i sin(k_i pi x_i) are the
// eigenvectors of A with eigenvalues sum_i (4/h^2) sin^2(k_i pi h / 2), so
//   u = S^-1 diag(lambda)^-1 S f,   S = DST-I along every axis.
//
// One DST-I of length m along the contiguous axis of an array: the odd
// extension (0, x_1 .. x_m, 0, -x_m .. -x_1) of a line, length N = 2(m+1),
// is real and odd, so its DFT is purely imaginary with coefficient k equal
// to -2i sum_j x_j sin(pi j k/(m+1)).  Two lines a, b therefore share one
// complex FFT of z = ext_a + i ext_b: Z_k = -2i S_a(k) + 2 S_b(k), so
// S_a(k) = -Im Z_k / 2 and S_b(k) = Re Z_k / 2, with no post-processing.
//   pack    the odd extensions of f's lines as complex lines (pairing below)
//   FFT     a batched complex FFT of length N (rocFFT, used as a library)
//   unpack  S(k) for every line, written with the transformed axis moved to
//           the slowest position (an LDS tile transpose)
// Pairing: a pass's m^(d-1) lines are numbered l = a o + s with o = m in 3D
// (a, s the two untransformed axes, a the slower) and o = 1 in 2D (s = 0);
// lines a and a+1 (a even) with the same s form complex line (a/2) o + s,
// line a in the real part (an odd count of a leaves the last imaginary parts
// zero).  The unpack moves mode k to the slow axis, so modes k and k+1 of a
// line land in one complex line of the next pass: every pack and unpack
// thread reads and writes whole complex values.
// so d passes visit every axis and return the array to its own axis order.
// Only f is packed by a kernel of its own: every unpack but the last writes
// its result directly as the next pass's complex lines, into the buffer the
// FFT has just consumed.
// The last forward pass divides by the eigenvalues and applies the inverse's
// scale (2/(m+1))^d (DST-I is its own inverse up to (m+1)/2 per axis); d
// more passes invert the transform.  FP64 throughout.
#include <rocfft/rocfft.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "../../include/gmg.h"
#include "gmg_internal.h"

namespace gmg {

// Pack f: thread t of complex line c = (a/2) o + s reads element t of lines
// a o + s and (a+1) o + s (zero past the last a) and writes both halves of
// the odd extension; the thread of t = m writes the two zeros.  blockIdx.x
// covers t, blockIdx.y strides over the complex lines.
__global__ void __launch_bounds__(256) k_dst_pack(const double *__restrict__ src,
                                                  double2 *__restrict__ z, int m, int o) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t > m) return;
  const size_t N = 2 * (size_t)(m + 1);
  const size_t ncl = (size_t)((m + 1) / 2) * o;
  for (size_t c = blockIdx.y; c < ncl; c += gridDim.y) {
    double2 *zl = z + c * N;
    if (t == m) {
      zl[0] = make_double2(0.0, 0.0);
      zl[m + 1] = make_double2(0.0, 0.0);
      continue;
    }
    const int a = 2 * (int)(c / o), sx = (int)(c % o);
    const double va = src[((size_t)a * o + sx) * m + t];
    const double vb = a + 1 < m ? src[((size_t)(a + 1) * o + sx) * m + t] : 0.0;
    zl[t + 1] = make_double2(va, vb);
    zl[N - 1 - t] = make_double2(-va, -vb);
  }
}

// 1/lambda times `scale` for mode k along the axis just transformed; the
// line's index holds the (0-based) modes of the other axes
template <int DIM>
__device__ __forceinline__ double dst_eig(int m, size_t line, int k, double scale,
                                          double inv_h2) {
  const double t = M_PI / (2.0 * (m + 1));
  auto s2 = [&](long q) {
    const double sv = sin(t * (double)q);
    return sv * sv;
  };
  double lam = s2(k);
  if (DIM == 2) {
    lam += s2((long)line + 1);
  } else {
    lam += s2((long)(line / m) + 1) + s2((long)(line % m) + 1);
  }
  return scale / (4.0 * inv_h2 * lam);
}

// Unpack with transpose.  A workgroup takes 32 complex lines (3D: a pair
// (a, a+1) = 2 blockIdx.z + {0, 1} and s = 32 blockIdx.y + r; 2D: a = 64
// blockIdx.y + 2 r + {0, 1}) times 32 modes k = 1 + 32 blockIdx.x + kk,
// reads them as whole complex values into LDS, then writes modes k, k+1 (k
// odd) of each line l = a o + s as one complex value of the next pass: line
// (k-1) o + l / m, element l % m, i.e. complex line ((k-1)/2) o + l / m
// (EXT); or, for the last pass, into out[(k-1) m^(d-1) + l].  eig != 0 (the
// last forward pass): divide by the eigenvalue and multiply by `scale`.
template <int DIM, bool EXT>
__global__ void __launch_bounds__(256) k_dst_unpack(const double2 *__restrict__ Z,
                                                    void *__restrict__ out, int m, int eig,
                                                    double scale, double inv_h2) {
  __shared__ double tile[2][32][33];  // [line of the pair][row r][mode kk]
  const int o = DIM == 3 ? m : 1;
  const size_t lines = (size_t)m * o;
  const size_t N = 2 * (size_t)(m + 1);
  const size_t ncl = (size_t)((m + 1) / 2) * o;
  const int k0 = 1 + blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    size_t c;
    bool ok;
    if (DIM == 3) {
      const int sx = blockIdx.y * 32 + r;
      c = (size_t)blockIdx.z * o + sx;
      ok = sx < o;
    } else {
      c = (size_t)blockIdx.y * 32 + r;
      ok = c < ncl;
    }
    const int k = k0 + tx;
    const double2 v = (ok && k <= m) ? Z[c * N + k] : make_double2(0.0, 0.0);
    tile[0][r][tx] = -0.5 * v.y;  // line a: real part of its extension
    tile[1][r][tx] = 0.5 * v.x;   // line a+1: imaginary part
  }
  __syncthreads();
  const int r = tx;
  for (int j = ty; j < 32; j += 8) {
    const int ai = j & 1, kk = 2 * (j >> 1);
    const int a = DIM == 3 ? 2 * (int)blockIdx.z + ai : (int)blockIdx.y * 64 + 2 * r + ai;
    const int sx = DIM == 3 ? (int)blockIdx.y * 32 + r : 0;
    const int k = k0 + kk;
    if (a >= m || sx >= o || k > m) continue;
    const size_t line = (size_t)a * o + sx;
    const bool has1 = k + 1 <= m;
    double v0 = tile[ai][r][kk];
    double v1 = has1 ? tile[ai][r][kk + 1] : 0.0;
    if (eig) {
      v0 *= dst_eig<DIM>(m, line, k, scale, inv_h2);
      if (has1) v1 *= dst_eig<DIM>(m, line, k + 1, scale, inv_h2);
    }
    if (EXT) {
      // next pass: line (k-1) o + a (3D) / k-1 (2D), element s (3D) / a (2D)
      const int te = DIM == 3 ? sx : a;
      double2 *zl = (double2 *)out + ((size_t)((k - 1) >> 1) * o + (DIM == 3 ? a : 0)) * N;
      zl[te + 1] = make_double2(v0, v1);
      zl[N - 1 - te] = make_double2(-v0, -v1);
      if (te == 0) {
        zl[0] = make_double2(0.0, 0.0);
        zl[m + 1] = make_double2(0.0, 0.0);
      }
    } else {
      double *d = (double *)out;
      d[(size_t)(k - 1) * lines + line] = v0;
      if (has1) d[(size_t)k * lines + line] = v1;
    }
  }
}

}  // namespace gmg

using namespace gmg;

struct gmg_dst {
  int dim = 3, m = 1;
  size_t lines = 1;
  hipStream_t stream = nullptr;
  double *E = nullptr;    // odd extensions, two real lines per complex line
  double2 *C = nullptr;   // their FFT coefficients
  void *work = nullptr;   // rocFFT work buffer
  size_t work_bytes = 0;
  rocfft_plan plan = nullptr;
  rocfft_execution_info info = nullptr;
};

namespace {

constexpr size_t kAlignDst = 256;
size_t up(size_t x) { return (x + kAlignDst - 1) / kAlignDst * kAlignDst; }

bool rocfft_ready() {
  static bool ok = rocfft_setup() == rocfft_status_success;
  return ok;
}

struct DstSizes {
  size_t E, C;
};
size_t dst_pairs(int dim, int m) {
  // complex lines: lines a, a+1 of the same s share one
  return (size_t)((m + 1) / 2) * (dim == 3 ? (size_t)m : 1);
}

DstSizes dst_sizes(int dim, int m) {
  const size_t bytes = dst_pairs(dim, m) * 2 * (size_t)(m + 1) * sizeof(double2);
  DstSizes s;
  s.E = up(bytes);
  s.C = up(bytes);
  return s;
}

rocfft_status make_plan(int dim, int m, rocfft_plan *plan) {
  const size_t len = 2 * (size_t)(m + 1);
  return rocfft_plan_create(plan, rocfft_placement_notinplace,
                            rocfft_transform_type_complex_forward, rocfft_precision_double, 1,
                            &len, dst_pairs(dim, m), nullptr);
}

// FFT of the complex lines in E into C, then the unpack: into the next
// pass's complex lines in E (out == NULL) or, for the last pass, into out.
hipError_t dst_pass(gmg_dst *p, double *out, int eig, double scale) {
  const int m = p->m;
  void *in[1] = {p->E};
  void *o[1] = {p->C};
  if (rocfft_execute(p->plan, in, o, p->info) != rocfft_status_success) return hipErrorUnknown;
  const double h = 1.0 / double(m + 1);
  const unsigned kt = (m + 31) / 32;
  const dim3 grid = p->dim == 3 ? dim3(kt, kt, (m + 1) / 2)
                                : dim3(kt, (unsigned)((dst_pairs(2, m) + 31) / 32), 1);
  const double2 *Z = (const double2 *)p->C;
  void *dst = out ? (void *)out : (void *)p->E;
  const double ih2 = 1.0 / (h * h);
  if (p->dim == 2) {
    if (out)
      gmg_launch((k_dst_unpack<2, false>), grid, dim3(256), 0, p->stream, Z, dst, m, eig, scale,
                 ih2);
    else
      gmg_launch((k_dst_unpack<2, true>), grid, dim3(256), 0, p->stream, Z, dst, m, eig, scale,
                 ih2);
  } else {
    if (out)
      gmg_launch((k_dst_unpack<3, false>), grid, dim3(256), 0, p->stream, Z, dst, m, eig, scale,
                 ih2);
    else
      gmg_launch((k_dst_unpack<3, true>), grid, dim3(256), 0, p->stream, Z, dst, m, eig, scale,
                 ih2);
  }
  return hipGetLastError();
}

}  // namespace

extern "C" {

gmg_status gmg_dst_setup(int dim, int levels, void *workspace, size_t *ws_bytes, void *stream,
                         gmg_dst **out) {
  if (!ws_bytes || (dim != 2 && dim != 3) || levels < 1) return GMG_ERR_INVALID_ARG;
  if (levels > (dim == 3 ? 10 : 14)) return GMG_ERR_INVALID_ARG;
  const int m = (1 << levels) - 1;
  if (!rocfft_ready()) return GMG_ERR_HIP;
  rocfft_plan plan = nullptr;
  if (make_plan(dim, m, &plan) != rocfft_status_success) return GMG_ERR_HIP;
  size_t wb = 0;
  if (rocfft_plan_get_work_buffer_size(plan, &wb) != rocfft_status_success) {
    rocfft_plan_destroy(plan);
    return GMG_ERR_HIP;
  }
  const DstSizes s = dst_sizes(dim, m);
  const size_t total = s.E + s.C + up(wb);
  if (!workspace) {
    rocfft_plan_destroy(plan);
    *ws_bytes = total;
    return GMG_OK;
  }
  if (!out) {
    rocfft_plan_destroy(plan);
    return GMG_ERR_INVALID_ARG;
  }
  if (*ws_bytes < total || ((uintptr_t)workspace) % kAlignDst) {
    rocfft_plan_destroy(plan);
    return GMG_ERR_WORKSPACE;
  }
  gmg_dst *p = new gmg_dst();
  p->dim = dim;
  p->m = m;
  p->lines = dim == 3 ? (size_t)m * m : (size_t)m;
  p->stream = (hipStream_t)stream;
  char *w = (char *)workspace;
  p->E = (double *)w;
  p->C = (double2 *)(w + s.E);
  p->work = wb ? (void *)(w + s.E + s.C) : nullptr;
  p->work_bytes = wb;
  p->plan = plan;
  if (rocfft_execution_info_create(&p->info) != rocfft_status_success ||
      rocfft_execution_info_set_stream(p->info, p->stream) != rocfft_status_success ||
      (wb && rocfft_execution_info_set_work_buffer(p->info, p->work, wb) !=
                 rocfft_status_success)) {
    if (p->info) rocfft_execution_info_destroy(p->info);
    rocfft_plan_destroy(plan);
    delete p;
    return GMG_ERR_HIP;
  }
  *out = p;
  return GMG_OK;
}

gmg_status gmg_dst_solve(gmg_dst *p, double *u, const double *f) {
  if (!p || !u || !f || (const double *)u == f) return GMG_ERR_INVALID_ARG;
  const double scale = std::pow(2.0 / double(p->m + 1), p->dim);
  const int m = p->m;
  const dim3 pgrid((m + 1 + 255) / 256, (unsigned)std::min<size_t>(dst_pairs(p->dim, m), 65535));
  gmg_launch(k_dst_pack, pgrid, dim3(256), 0, p->stream, f, (double2 *)p->E, m,
             p->dim == 3 ? m : 1);
  if (hipGetLastError() != hipSuccess) return GMG_ERR_HIP;
  // d forward passes (the last divides by lambda), d inverse passes; only the
  // last one writes u
  for (int a = 0; a < 2 * p->dim; ++a) {
    const int eig = a == p->dim - 1;
    if (dst_pass(p, a == 2 * p->dim - 1 ? u : nullptr, eig, eig ? scale : 1.0) != hipSuccess)
      return GMG_ERR_HIP;
  }
  return GMG_OK;
}

gmg_status gmg_dst_destroy(gmg_dst *p) {
  if (!p) return GMG_ERR_INVALID_ARG;
  if (p->info) rocfft_execution_info_destroy(p->info);
  if (p->plan) rocfft_plan_destroy(p->plan);
  delete p;
  return GMG_OK;
}

}  // extern "C"
