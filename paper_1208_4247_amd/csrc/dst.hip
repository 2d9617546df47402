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
//   pack    the odd extensions of lines 2p, 2p+1 as complex line p (a zero
//           line pads an odd line count)
//   FFT     a batched complex FFT of length N (rocFFT, used as a library)
//   unpack  S(k) for every line, written with the transformed axis moved to
//           the slowest position (an LDS tile transpose)
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

// Store value v of element t (0-based, t < m) of line `line` into the
// complex lines z (N = 2(m+1) per line): +v at t+1, -v at N-(t+1), in the
// real part for an even line and the imaginary part for an odd one.  The
// thread of t = 0 also writes the zeros at 0 and m+1; for the last of an odd
// number of lines the partner (padding) line is written as zeros too.
__device__ __forceinline__ void dst_put(double *z, int m, size_t lines, size_t line, int t,
                                        double v) {
  const size_t N = 2 * (size_t)(m + 1);
  const int c = (int)(line & 1);
  double *zl = z + (line >> 1) * 2 * N;  // complex line, interleaved
  zl[2 * (t + 1) + c] = v;
  zl[2 * (N - (t + 1)) + c] = -v;
  if (t == 0) {
    zl[c] = 0.0;
    zl[2 * (m + 1) + c] = 0.0;
  }
  if (c == 0 && line + 1 == lines) {  // odd count: the padding line is zero
    zl[2 * (t + 1) + 1] = 0.0;
    zl[2 * (N - (t + 1)) + 1] = 0.0;
    if (t == 0) {
      zl[1] = 0.0;
      zl[2 * (m + 1) + 1] = 0.0;
    }
  }
}

// one thread per element of src (lines x m): the complex lines of f
__global__ void __launch_bounds__(256) k_dst_pack(const double *__restrict__ src,
                                                  double *__restrict__ z, int m, size_t lines) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < lines * (size_t)m;
       i += (size_t)gridDim.x * 256)
    dst_put(z, m, lines, i / (size_t)m, (int)(i % (size_t)m), src[i]);
}

// S(k) of line `line` from the FFT of its complex line
__device__ __forceinline__ double dst_get(const double2 *__restrict__ Z, int m, size_t line,
                                          int k) {
  const size_t N = 2 * (size_t)(m + 1);
  const double2 c = Z[(line >> 1) * N + k];
  return (line & 1) ? 0.5 * c.x : -0.5 * c.y;
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

// Unpack with transpose, a 32 x 32 tile (lines x modes) per workgroup.
// EXT: write mode k of line (s, t) (t the fastest index of the line number)
// as element t of line (k-1) * (lines/m) + s of the next pass's complex
// lines; else to dst[(k-1) * lines + line].  eig != 0 (the last forward
// pass): divide by the eigenvalue and multiply by `scale`.
template <int DIM, bool EXT>
__global__ void __launch_bounds__(256) k_dst_unpack(const double2 *__restrict__ Z,
                                                    double *__restrict__ dst, int m, size_t lines,
                                                    int eig, double scale, double inv_h2) {
  __shared__ double tile[32][33];
  const size_t l0 = (size_t)blockIdx.y * 32;
  const int k0 = 1 + blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const size_t line = l0 + r;
    const int k = k0 + tx;
    tile[r][tx] = (line < lines && k <= m) ? dst_get(Z, m, line, k) : 0.0;
  }
  __syncthreads();
  const size_t outer = lines / (size_t)m;  // lines of the next pass per mode
  for (int r = ty; r < 32; r += 8) {
    const int k = k0 + r;
    const size_t line = l0 + tx;
    if (k > m || line >= lines) continue;
    double v = tile[tx][r];
    if (eig) v = v * dst_eig<DIM>(m, line, k, scale, inv_h2);
    if (EXT)
      dst_put(dst, m, lines, (size_t)(k - 1) * outer + line / (size_t)m,
              (int)(line % (size_t)m), v);
    else
      dst[(size_t)(k - 1) * lines + line] = v;
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
  const size_t lines = dim == 3 ? (size_t)m * m : (size_t)m;
  return (lines + 1) / 2;  // complex lines: two real lines each
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
  const dim3 grid((m + 31) / 32, (unsigned)((p->lines + 31) / 32));
  const double2 *Z = (const double2 *)p->C;
  double *dst = out ? out : p->E;
  const double ih2 = 1.0 / (h * h);
  if (p->dim == 2) {
    if (out)
      gmg_launch((k_dst_unpack<2, false>), grid, dim3(256), 0, p->stream, Z, dst, m, p->lines, eig,
                 scale, ih2);
    else
      gmg_launch((k_dst_unpack<2, true>), grid, dim3(256), 0, p->stream, Z, dst, m, p->lines, eig,
                 scale, ih2);
  } else {
    if (out)
      gmg_launch((k_dst_unpack<3, false>), grid, dim3(256), 0, p->stream, Z, dst, m, p->lines, eig,
                 scale, ih2);
    else
      gmg_launch((k_dst_unpack<3, true>), grid, dim3(256), 0, p->stream, Z, dst, m, p->lines, eig,
                 scale, ih2);
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
  const size_t n = p->lines * (size_t)m;
  const int nb = (int)std::min<size_t>((n + 255) / 256, 1 << 20);
  gmg_launch(k_dst_pack, dim3(nb), dim3(256), 0, p->stream, f, p->E, m, p->lines);
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
