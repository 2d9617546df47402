// dst.hip -- exact solve of the discrete Poisson problem (the 5-/7-point
// scheme with zero Dirichlet data, Sec. 2.2) by the discrete sine transform
// (DST-I), the fast direct method the paper compares full multigrid with
// (Sec. 5.4, Tables 12-15).  The sine modes prod_i sin(k_i pi x_i) are the
// eigenvectors of A with eigenvalues sum_i (4/h^2) sin^2(k_i pi h / 2), so
//   u = S^-1 diag(lambda)^-1 S f,   S = DST-I along every axis.
//
// One DST-I of length m along the contiguous axis of an array is done as
//   pack    the odd extension (0, x_1 .. x_m, 0, -x_m .. -x_1) of every line,
//           length 2(m+1)
//   FFT     a batched real-to-complex FFT of that length (rocFFT, used as a
//           library), whose coefficient k is -2i sum_j x_j sin(pi j k/(m+1))
//   unpack  y_k = -Im(X_k) / 2, written with the transformed axis moved to
//           the slowest position (an LDS tile transpose)
// so d passes visit every axis and return the array to its own axis order.
// Only f is packed by a kernel of its own: every unpack but the last writes
// its result directly as the odd extensions of the next pass's lines, into
// the buffer the FFT has just consumed.
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

// lines x (m+2) threads: ext[line][0 .. 2m+1] from src[line][0 .. m-1]
__global__ void __launch_bounds__(256) k_dst_pack(const double *__restrict__ src,
                                                  double *__restrict__ ext, int m, size_t lines) {
  const size_t L2 = 2 * (size_t)(m + 1);
  const size_t per = (size_t)m + 2;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < lines * per;
       i += (size_t)gridDim.x * 256) {
    const size_t line = i / per;
    const int n = (int)(i % per);  // 0 .. m+1
    double *e = ext + line * L2;
    if (n == 0 || n == m + 1) {
      e[n] = 0.0;
    } else {
      const double v = src[line * m + (n - 1)];
      e[n] = v;
      e[L2 - n] = -v;
    }
  }
}

// Unpack with transpose: dst[(k-1) * lines + line] = scale(k, line) *
// (-Im C[line][k] / 2), k = 1..m.  A 32 x 32 tile (lines x modes) per
// workgroup.  With eig != 0 (the last forward pass) the value is divided by
// the eigenvalue of mode (k, line's modes) and multiplied by `scale`.
template <int DIM>
__global__ void __launch_bounds__(256) k_dst_unpack(const double2 *__restrict__ C,
                                                    double *__restrict__ dst, int m, size_t lines,
                                                    int eig, double scale, double inv_h2) {
  __shared__ double tile[32][33];
  const size_t per = (size_t)m + 2;  // complex coefficients per line
  const size_t l0 = (size_t)blockIdx.y * 32;
  const int k0 = 1 + blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const size_t line = l0 + r;
    const int k = k0 + tx;
    double v = 0.0;
    if (line < lines && k <= m) v = -0.5 * C[line * per + k].y;
    tile[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int k = k0 + r;
    const size_t line = l0 + tx;
    if (k > m || line >= lines) continue;
    double v = tile[tx][r];
    if (eig) {
      // modes: k along the axis just transformed, the line's index holds the
      // modes of the other axes (1-based)
      const double t = M_PI / (2.0 * (m + 1));
      auto s2 = [&](long q) {
        const double s = sin(t * (double)q);
        return s * s;
      };
      double lam = s2(k);
      if (DIM == 2) {
        lam += s2((long)line + 1);
      } else {
        lam += s2((long)(line / m) + 1) + s2((long)(line % m) + 1);
      }
      v = v * scale / (4.0 * inv_h2 * lam);
    }
    dst[(size_t)(k - 1) * lines + line] = v;
  }
}

// Unpack straight into the next pass's odd extensions: the value for mode k
// of line (s, t) (t the fastest index of the line number) belongs to line
// (k-1) * (lines/m) + s, element t, of the next pass, so it is written to
// ext[line'][t+1] and, negated, to ext[line'][2(m+1)-(t+1)]; the thread of
// t = 0 also writes the two zeros of that line.  eig / scale as above.
template <int DIM>
__global__ void __launch_bounds__(256) k_dst_unpack_ext(const double2 *__restrict__ C,
                                                        double *__restrict__ ext, int m,
                                                        size_t lines, int eig, double scale,
                                                        double inv_h2) {
  __shared__ double tile[32][33];
  const size_t per = (size_t)m + 2;
  const size_t L2 = 2 * (size_t)(m + 1);
  const size_t l0 = (size_t)blockIdx.y * 32;
  const int k0 = 1 + blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const size_t line = l0 + r;
    const int k = k0 + tx;
    double v = 0.0;
    if (line < lines && k <= m) v = -0.5 * C[line * per + k].y;
    tile[r][tx] = v;
  }
  __syncthreads();
  const size_t outer = lines / (size_t)m;  // lines of the next pass per mode
  for (int r = ty; r < 32; r += 8) {
    const int k = k0 + r;
    const size_t line = l0 + tx;
    if (k > m || line >= lines) continue;
    double v = tile[tx][r];
    if (eig) {
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
      v = v * scale / (4.0 * inv_h2 * lam);
    }
    const size_t s_ = line / (size_t)m;
    const int t_ = (int)(line % (size_t)m);
    double *e = ext + ((size_t)(k - 1) * outer + s_) * L2;
    e[t_ + 1] = v;
    e[L2 - (t_ + 1)] = -v;
    if (t_ == 0) {
      e[0] = 0.0;
      e[m + 1] = 0.0;
    }
  }
}

}  // namespace gmg

using namespace gmg;

struct gmg_dst {
  int dim = 3, m = 1;
  size_t lines = 1;
  hipStream_t stream = nullptr;
  double *E = nullptr;    // odd extensions
  double2 *C = nullptr;   // FFT coefficients
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
DstSizes dst_sizes(int dim, int m) {
  const size_t lines = dim == 3 ? (size_t)m * m : (size_t)m;
  DstSizes s;
  s.E = up(lines * 2 * (size_t)(m + 1) * sizeof(double));
  s.C = up(lines * (size_t)(m + 2) * sizeof(double2));
  return s;
}

rocfft_status make_plan(int dim, int m, rocfft_plan *plan) {
  const size_t lines = dim == 3 ? (size_t)m * m : (size_t)m;
  const size_t len = 2 * (size_t)(m + 1);
  return rocfft_plan_create(plan, rocfft_placement_notinplace, rocfft_transform_type_real_forward,
                            rocfft_precision_double, 1, &len, lines, nullptr);
}

// FFT of the extensions in E into C, then the unpack: into the next pass's
// extensions in E (out == NULL) or, for the last pass, into out.
hipError_t dst_pass(gmg_dst *p, double *out, int eig, double scale) {
  const int m = p->m;
  void *in[1] = {p->E};
  void *o[1] = {p->C};
  if (rocfft_execute(p->plan, in, o, p->info) != rocfft_status_success) return hipErrorUnknown;
  const double h = 1.0 / double(m + 1);
  const dim3 grid((m + 31) / 32, (unsigned)((p->lines + 31) / 32));
  const double2 *C = (const double2 *)p->C;
  if (out) {
    if (p->dim == 2)
      gmg_launch((k_dst_unpack<2>), grid, dim3(256), 0, p->stream, C, out, m, p->lines, eig, scale,
                 1.0 / (h * h));
    else
      gmg_launch((k_dst_unpack<3>), grid, dim3(256), 0, p->stream, C, out, m, p->lines, eig, scale,
                 1.0 / (h * h));
  } else {
    if (p->dim == 2)
      gmg_launch((k_dst_unpack_ext<2>), grid, dim3(256), 0, p->stream, C, p->E, m, p->lines, eig,
                 scale, 1.0 / (h * h));
    else
      gmg_launch((k_dst_unpack_ext<3>), grid, dim3(256), 0, p->stream, C, p->E, m, p->lines, eig,
                 scale, 1.0 / (h * h));
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
  const size_t n = p->lines * (size_t)(m + 2);
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
