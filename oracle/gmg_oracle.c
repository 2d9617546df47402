/*
 * gmg_oracle.c -- plain FP64 CPU oracle for geometric multigrid on the
 * finite-difference Poisson problem (Feng, Shu, Xu, Zhang, "Numerical Study of
 * Geometric Multigrid Methods on CPU-GPU Heterogeneous Computers",
 * arXiv:1208.4247).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the GPU library is
 * checked against.  Nothing in the product library may link, load or call it;
 * only the test suite, the smoke check and the CPU-baseline leg of the bench
 * use it.  It shares no code with the HIP path.
 *
 * Written for obviousness, not speed: plain loops, one point at a time, in the
 * order the paper states the steps.  OpenMP only splits the outermost loop of
 * a pointwise-independent update; reductions are summed in a fixed order so
 * that results do not depend on the thread count.  Build with
 * -O2 -ffp-contract=off so that no multiply-add is fused.
 *
 * Problem (Sec. 2.2, eq. (1) and the 5-/7-point schemes): -Lap u = f on
 * (0,1)^d, u = 0 on the boundary, d = 2 or 3, uniform mesh h = 1/n.
 *
 * Storage: a level with n intervals per axis has m = n - 1 interior nodes per
 * axis.  A grid function is a dense array of m^d doubles, x fastest:
 * storage (i, j[, k]) in [0, m) holds node (i+1, j+1[, k+1]), i.e. the value
 * at x = (i+1) h.  Boundary nodes (index 0 or n) are never stored; they read
 * as zero.
 *
 * Readings adopted where the paper is silent or ambiguous (each is also
 * listed in the design notes):
 *  - operator scaling: A_l v = (2d v_p - sum of neighbours) / h_l^2 with the
 *    physical f on every level (the printed scheme moves h^2 to the right
 *    hand side; both are the same system);
 *  - transfers: full weighting (tensor [1/4 1/2 1/4]) and (bi/tri)linear
 *    interpolation (tensor [1/2 1 1/2]), the standard pair, instead of the
 *    7-point restriction and simplex interpolation printed in Sec. 4;
 *  - smoother: red-black Gauss-Seidel, red = even sum of node indices;
 *    forward sweep = red then black, backward = black then red; weighted
 *    Jacobi as the alternative (Remark 1, Table 5);
 *  - V-cycle (Algorithm 1): coarse iterates start from zero on every descent;
 *    the ascent runs l = L-2 .. 0; the 1-DOF coarsest level is solved
 *    exactly (Remark on the coarsest-level solver);
 *  - solve loop (Algorithm 3 with every level on one device): the norm is
 *    the Euclidean norm with the square root; iterate while
 *    res > tol * res0 and iter < maxit.
 *
 * The paper's own smoother and transfers are kept as a variant (selected per
 * call): multicolour Gauss-Seidel (4 colours in 2D, 8 in 3D, Remark 1) and the
 * linear finite-element transfers of Sec. 4 (eq. Restriction2d,
 * eq. Prolongation2d and the 3D operation counts), with the coarsest level
 * either solved exactly or relaxed by the smoother as Algorithm 1 writes it.
 * Readings for the variant: colour of node (i, j[, k]) = (i & 1) + 2 (j & 1)
 * [+ 4 (k & 1)], the forward sweep visits colours 0, 1, ..., 2^d - 1 and the
 * backward sweep the reverse; the 3D triangulation is the one whose edges are
 * the seven directions with components in {0, 1} (the 2D edge set
 * (1,0), (0,1), (1,1) of eq. Prolongation2d, extended).
 *
 * Parity status of each function: every function is pinned by the tests
 * (closed forms, the paper's printed FFT error columns, dense and DST exact
 * solves, Fourier symbols, invariants, symmetry, local Fourier analysis).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* basic helpers                                                             */
/* ------------------------------------------------------------------------ */

/* number of points of a level with m interior nodes per axis */
static long npts(int d, int m) { return d == 2 ? (long)m * m : (long)m * m * m; }

/* value at node-offset storage index, zero outside [0, m) (Dirichlet data) */
static double at2(const double *v, int m, int i, int j) {
  if (i < 0 || j < 0 || i >= m || j >= m) return 0.0;
  return v[(long)j * m + i];
}
static double at3(const double *v, int m, int i, int j, int k) {
  if (i < 0 || j < 0 || k < 0 || i >= m || j >= m || k >= m) return 0.0;
  return v[((long)k * m + j) * m + i];
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* levels of the hierarchy for a finest side m0 = 2^L - 1; -1 if m0 is not of
 * that form.  Level l has n_l = 2^(L-l) intervals, level L-1 has one node
 * (Sec. 3.1; Remark on the coarsest-level solver). */
int orc_levels(int m0) {
  if (m0 < 1) return -1;
  long n = (long)m0 + 1;
  if (n & (n - 1)) return -1;
  int L = 0;
  while (n > 1) { n >>= 1; L++; }
  return L;
}

/* Euclidean norm, summed per outer index then in index order (deterministic) */
double orc_norm2(int d, int m, const double *r) {
  long plane = d == 2 ? m : (long)m * m;
  double *part = (double *)malloc(sizeof(double) * (size_t)m);
#pragma omp parallel for schedule(static)
  for (int o = 0; o < m; o++) {
    double s = 0.0;
    const double *p = r + (long)o * plane;
    for (long q = 0; q < plane; q++) s += p[q] * p[q];
    part[o] = s;
  }
  double s = 0.0;
  for (int o = 0; o < m; o++) s += part[o];
  free(part);
  return sqrt(s);
}

/* ------------------------------------------------------------------------ */
/* operator and residual (Sec. 2.2 schemes; Sec. 4 eq. residual_2D and the   */
/* 3D count)                                                                 */
/* ------------------------------------------------------------------------ */

/* out = A v with (A v)_p = (2d v_p - sum_{q nbr p} v_q) / h^2, h = 1/(m+1) */
void orc_apply_A(int d, int m, const double *v, double *out) {
  double n = (double)(m + 1);
  double inv_h2 = n * n;
  if (d == 2) {
#pragma omp parallel for schedule(static)
    for (int j = 0; j < m; j++)
      for (int i = 0; i < m; i++) {
        double nb = at2(v, m, i - 1, j) + at2(v, m, i + 1, j) + at2(v, m, i, j - 1) +
                    at2(v, m, i, j + 1);
        out[(long)j * m + i] = (4.0 * at2(v, m, i, j) - nb) * inv_h2;
      }
  } else {
#pragma omp parallel for schedule(static)
    for (int k = 0; k < m; k++)
      for (int j = 0; j < m; j++)
        for (int i = 0; i < m; i++) {
          double nb = at3(v, m, i - 1, j, k) + at3(v, m, i + 1, j, k) + at3(v, m, i, j - 1, k) +
                      at3(v, m, i, j + 1, k) + at3(v, m, i, j, k - 1) + at3(v, m, i, j, k + 1);
          out[((long)k * m + j) * m + i] = (6.0 * at3(v, m, i, j, k) - nb) * inv_h2;
        }
  }
}

/* r = f - A u */
void orc_residual(int d, int m, const double *u, const double *f, double *r) {
  long N = npts(d, m);
  orc_apply_A(d, m, u, r);
#pragma omp parallel for schedule(static)
  for (long p = 0; p < N; p++) r[p] = f[p] - r[p];
}

/* ------------------------------------------------------------------------ */
/* smoothers (Remark 1; eq. relax_2D and its 3D analogue; Table 5)           */
/* ------------------------------------------------------------------------ */

/* One colour of red-black Gauss-Seidel: every node whose node-index sum has
 * parity `color` (0 = red = even, 1 = black) is set so that its own equation
 * holds with the current neighbours:  u_p = (h^2 f_p + sum nbrs) / (2d).
 * Points of one colour only neighbour the other colour, so the order inside a
 * colour does not matter. */
void orc_rbgs_color(int d, int m, double *u, const double *f, int color) {
  double h = 1.0 / (double)(m + 1);
  double h2 = h * h;
  if (d == 2) {
#pragma omp parallel for schedule(static)
    for (int j = 0; j < m; j++)
      for (int i = 0; i < m; i++) {
        if ((((i + 1) + (j + 1)) & 1) != color) continue;
        long p = (long)j * m + i;
        double nb = at2(u, m, i - 1, j) + at2(u, m, i + 1, j) + at2(u, m, i, j - 1) +
                    at2(u, m, i, j + 1);
        u[p] = (h2 * f[p] + nb) / 4.0;
      }
  } else {
#pragma omp parallel for schedule(static)
    for (int k = 0; k < m; k++)
      for (int j = 0; j < m; j++)
        for (int i = 0; i < m; i++) {
          if ((((i + 1) + (j + 1) + (k + 1)) & 1) != color) continue;
          long p = ((long)k * m + j) * m + i;
          double nb = at3(u, m, i - 1, j, k) + at3(u, m, i + 1, j, k) + at3(u, m, i, j - 1, k) +
                      at3(u, m, i, j + 1, k) + at3(u, m, i, j, k - 1) + at3(u, m, i, j, k + 1);
          u[p] = (h2 * f[p] + nb) / 6.0;
        }
  }
}

/* nsweeps red-black sweeps; forward = red then black, backward = black then
 * red (the V-cycle's Relax_forward / Relax_backward, Algorithm 1). */
void orc_rbgs(int d, int m, double *u, const double *f, int nsweeps, int backward) {
  for (int s = 0; s < nsweeps; s++) {
    if (!backward) {
      orc_rbgs_color(d, m, u, f, 0);
      orc_rbgs_color(d, m, u, f, 1);
    } else {
      orc_rbgs_color(d, m, u, f, 1);
      orc_rbgs_color(d, m, u, f, 0);
    }
  }
}

/* One colour of the multicolour Gauss-Seidel smoother (Remark 1: four colours
 * in 2D, eight in 3D).  Node (i, j[, k]) has colour (i&1) + 2(j&1) [+ 4(k&1)];
 * nodes of one colour differ by an even amount along every axis, so none of
 * them neighbours another and the order inside a colour does not matter.  The
 * update is the same pointwise solve as eq. relax_2D. */
void orc_mcgs_color(int d, int m, double *u, const double *f, int color) {
  double h = 1.0 / (double)(m + 1);
  double h2 = h * h;
  if (d == 2) {
#pragma omp parallel for schedule(static)
    for (int j = 0; j < m; j++)
      for (int i = 0; i < m; i++) {
        if ((((i + 1) & 1) + 2 * ((j + 1) & 1)) != color) continue;
        long p = (long)j * m + i;
        double nb = at2(u, m, i - 1, j) + at2(u, m, i + 1, j) + at2(u, m, i, j - 1) +
                    at2(u, m, i, j + 1);
        u[p] = (h2 * f[p] + nb) / 4.0;
      }
  } else {
#pragma omp parallel for schedule(static)
    for (int k = 0; k < m; k++)
      for (int j = 0; j < m; j++)
        for (int i = 0; i < m; i++) {
          if ((((i + 1) & 1) + 2 * ((j + 1) & 1) + 4 * ((k + 1) & 1)) != color) continue;
          long p = ((long)k * m + j) * m + i;
          double nb = at3(u, m, i - 1, j, k) + at3(u, m, i + 1, j, k) + at3(u, m, i, j - 1, k) +
                      at3(u, m, i, j + 1, k) + at3(u, m, i, j, k - 1) + at3(u, m, i, j, k + 1);
          u[p] = (h2 * f[p] + nb) / 6.0;
        }
  }
}

/* nsweeps multicolour sweeps: forward visits colours 0 .. 2^d - 1, backward
 * the reverse (Relax_forward / Relax_backward of Algorithm 1). */
void orc_mcgs(int d, int m, double *u, const double *f, int nsweeps, int backward) {
  int nc = 1 << d;
  for (int s = 0; s < nsweeps; s++)
    for (int q = 0; q < nc; q++) orc_mcgs_color(d, m, u, f, backward ? nc - 1 - q : q);
}

/* nsweeps weighted-Jacobi sweeps (Remark 1; Table 5):
 *   u_new = (1 - omega) u + omega (h^2 f + sum nbrs) / (2d), all from old u.
 * tmp must hold m^d doubles. */
void orc_wj(int d, int m, double *u, const double *f, double omega, int nsweeps, double *tmp) {
  double h = 1.0 / (double)(m + 1);
  double h2 = h * h;
  long N = npts(d, m);
  for (int s = 0; s < nsweeps; s++) {
    memcpy(tmp, u, sizeof(double) * (size_t)N);
    if (d == 2) {
#pragma omp parallel for schedule(static)
      for (int j = 0; j < m; j++)
        for (int i = 0; i < m; i++) {
          long p = (long)j * m + i;
          double nb = at2(tmp, m, i - 1, j) + at2(tmp, m, i + 1, j) + at2(tmp, m, i, j - 1) +
                      at2(tmp, m, i, j + 1);
          u[p] = (1.0 - omega) * tmp[p] + omega * ((h2 * f[p] + nb) / 4.0);
        }
    } else {
#pragma omp parallel for schedule(static)
      for (int k = 0; k < m; k++)
        for (int j = 0; j < m; j++)
          for (int i = 0; i < m; i++) {
            long p = ((long)k * m + j) * m + i;
            double nb = at3(tmp, m, i - 1, j, k) + at3(tmp, m, i + 1, j, k) +
                        at3(tmp, m, i, j - 1, k) + at3(tmp, m, i, j + 1, k) +
                        at3(tmp, m, i, j, k - 1) + at3(tmp, m, i, j, k + 1);
            u[p] = (1.0 - omega) * tmp[p] + omega * ((h2 * f[p] + nb) / 6.0);
          }
    }
  }
}

/* ------------------------------------------------------------------------ */
/* grid transfers                                                            */
/* ------------------------------------------------------------------------ */

/* Full-weighting restriction: coarse node I gathers fine nodes 2I+o,
 * o in {-1,0,1}^d, with the tensor weights [1/4, 1/2, 1/4].  mc interior
 * coarse nodes per axis; the fine level has mf = 2 mc + 1.  Coarse storage
 * index a holds coarse node a+1, i.e. fine node 2a+2, fine storage 2a+1. */
void orc_restrict_fw(int d, int mc, const double *r, double *fc) {
  int mf = 2 * mc + 1;
  static const double w[3] = {0.25, 0.5, 0.25};
  if (d == 2) {
#pragma omp parallel for schedule(static)
    for (int b = 0; b < mc; b++)
      for (int a = 0; a < mc; a++) {
        double s = 0.0;
        for (int oy = -1; oy <= 1; oy++)
          for (int ox = -1; ox <= 1; ox++)
            s += w[ox + 1] * w[oy + 1] * at2(r, mf, 2 * a + 1 + ox, 2 * b + 1 + oy);
        fc[(long)b * mc + a] = s;
      }
  } else {
#pragma omp parallel for schedule(static)
    for (int c = 0; c < mc; c++)
      for (int b = 0; b < mc; b++)
        for (int a = 0; a < mc; a++) {
          double s = 0.0;
          for (int oz = -1; oz <= 1; oz++)
            for (int oy = -1; oy <= 1; oy++)
              for (int ox = -1; ox <= 1; ox++)
                s += w[ox + 1] * w[oy + 1] * w[oz + 1] *
                     at3(r, mf, 2 * a + 1 + ox, 2 * b + 1 + oy, 2 * c + 1 + oz);
          fc[((long)c * mc + b) * mc + a] = s;
        }
  }
}

/* Per-axis linear interpolation weights from the coarse grid to fine node
 * index `fi` (node numbering, 1..mf).  An even fine node coincides with coarse
 * node fi/2 (weight 1); an odd one lies halfway between coarse nodes
 * (fi-1)/2 and (fi+1)/2 (weight 1/2 each).  Returns the number of
 * contributions; coarse node indices are written to idx[] as coarse storage
 * indices (node - 1), which may fall outside [0, mc) on the boundary. */
static int lin_weights(int fi, int idx[2], double wt[2]) {
  if ((fi & 1) == 0) {
    idx[0] = fi / 2 - 1;
    wt[0] = 1.0;
    return 1;
  }
  idx[0] = (fi - 1) / 2 - 1;
  idx[1] = (fi + 1) / 2 - 1;
  wt[0] = 0.5;
  wt[1] = 0.5;
  return 2;
}

/* u (fine, mf = 2 mc + 1) += P e, P the (bi/tri)linear interpolation:
 * the tensor product of the per-axis weights above; coarse boundary values
 * are zero. */
void orc_prolong_add(int d, int mc, const double *e, double *u) {
  int mf = 2 * mc + 1;
  if (d == 2) {
#pragma omp parallel for schedule(static)
    for (int j = 0; j < mf; j++)
      for (int i = 0; i < mf; i++) {
        int ix[2], iy[2];
        double wx[2], wy[2];
        int nx = lin_weights(i + 1, ix, wx);
        int ny = lin_weights(j + 1, iy, wy);
        double s = 0.0;
        for (int b = 0; b < ny; b++)
          for (int a = 0; a < nx; a++) s += wx[a] * wy[b] * at2(e, mc, ix[a], iy[b]);
        u[(long)j * mf + i] += s;
      }
  } else {
#pragma omp parallel for schedule(static)
    for (int k = 0; k < mf; k++)
      for (int j = 0; j < mf; j++)
        for (int i = 0; i < mf; i++) {
          int ix[2], iy[2], iz[2];
          double wx[2], wy[2], wz[2];
          int nx = lin_weights(i + 1, ix, wx);
          int ny = lin_weights(j + 1, iy, wy);
          int nz = lin_weights(k + 1, iz, wz);
          double s = 0.0;
          for (int c = 0; c < nz; c++)
            for (int b = 0; b < ny; b++)
              for (int a = 0; a < nx; a++)
                s += wx[a] * wy[b] * wz[c] * at3(e, mc, ix[a], iy[b], iz[c]);
          u[((long)k * mf + j) * mf + i] += s;
        }
  }
}

/* Edge directions of the triangulation behind the paper's linear
 * finite-element transfers: every nonzero vector with components in {0, 1}.
 * In 2D these are (1,0), (0,1), (1,1), the three of eq. Prolongation2d. */
static int fe_dirs(int d, int dir[7][3]) {
  int n = 0;
  for (int o = 1; o < (1 << d); o++) {
    dir[n][0] = o & 1;
    dir[n][1] = (o >> 1) & 1;
    dir[n][2] = (o >> 2) & 1;
    n++;
  }
  return n;
}

/* u (fine, mf = 2 mc + 1) += P e, P the linear finite-element interpolation
 * (eq. Prolongation2d and its 3D analogue): fine node 2I coincides with coarse
 * node I; fine node 2I + o, o a direction above, is the midpoint of the edge
 * from coarse node I to I + o and takes the mean of the two.  Coarse values on
 * the boundary are zero. */
void orc_prolong_add_fe(int d, int mc, const double *e, double *u) {
  int mf = 2 * mc + 1;
  long planes = d == 2 ? 1 : mf;
#pragma omp parallel for schedule(static)
  for (long k = 0; k < planes; k++)
    for (int j = 0; j < mf; j++)
      for (int i = 0; i < mf; i++) {
        /* node indices of the fine point and its parity pattern o */
        int F[3] = {i + 1, j + 1, (int)k + 1};
        int o[3] = {F[0] & 1, F[1] & 1, d == 3 ? F[2] & 1 : 0};
        int I[3] = {(F[0] - o[0]) / 2, (F[1] - o[1]) / 2, (F[2] - o[2]) / 2};
        double s;
        if (d == 2) {
          double c0 = at2(e, mc, I[0] - 1, I[1] - 1);
          if (!o[0] && !o[1])
            s = c0;
          else
            s = 0.5 * (c0 + at2(e, mc, I[0] + o[0] - 1, I[1] + o[1] - 1));
          u[(long)j * mf + i] += s;
        } else {
          double c0 = at3(e, mc, I[0] - 1, I[1] - 1, I[2] - 1);
          if (!o[0] && !o[1] && !o[2])
            s = c0;
          else
            s = 0.5 * (c0 + at3(e, mc, I[0] + o[0] - 1, I[1] + o[1] - 1, I[2] + o[2] - 1));
          u[(k * mf + j) * mf + i] += s;
        }
      }
}

/* Linear finite-element restriction (eq. Restriction2d in 2D; 16 operations
 * per point in 3D): coarse node I takes twice the fine value at 2I plus the
 * fine values at 2I + e and 2I - e for every edge direction e, all divided by
 * 2^(d+1).  This is 2^-d times the transpose of orc_prolong_add_fe. */
void orc_restrict_fe(int d, int mc, const double *r, double *fc) {
  int mf = 2 * mc + 1;
  int dir[7][3];
  int nd = fe_dirs(d, dir);
  double scale = 1.0 / (double)(1 << (d + 1));
  long planes = d == 2 ? 1 : mc;
#pragma omp parallel for schedule(static)
  for (long c = 0; c < planes; c++)
    for (int b = 0; b < mc; b++)
      for (int a = 0; a < mc; a++) {
        /* fine storage index of fine node 2I, I = (a+1, b+1, c+1) */
        int x = 2 * a + 1, y = 2 * b + 1, z = 2 * (int)c + 1;
        double s;
        if (d == 2) {
          s = 2.0 * at2(r, mf, x, y);
          for (int q = 0; q < nd; q++)
            s += at2(r, mf, x + dir[q][0], y + dir[q][1]) + at2(r, mf, x - dir[q][0], y - dir[q][1]);
          fc[(long)b * mc + a] = s * scale;
        } else {
          s = 2.0 * at3(r, mf, x, y, z);
          for (int q = 0; q < nd; q++)
            s += at3(r, mf, x + dir[q][0], y + dir[q][1], z + dir[q][2]) +
                 at3(r, mf, x - dir[q][0], y - dir[q][1], z - dir[q][2]);
          fc[(c * mc + b) * mc + a] = s * scale;
        }
      }
}

/* ------------------------------------------------------------------------ */
/* V-cycle (Algorithm 1) and solve loop (Algorithm 3, all levels on one      */
/* device)                                                                   */
/* ------------------------------------------------------------------------ */

enum { ORC_RBGS = 0, ORC_WJ = 1, ORC_MCGS = 2 };
/* variant bits: the paper's linear finite-element transfers instead of full
 * weighting / (bi/tri)linear; the coarsest level relaxed by nu1 sweeps of the
 * smoother (Algorithm 1 as printed) instead of solved exactly */
enum { ORC_FE_TRANSFER = 1, ORC_COARSE_RELAX = 2 };

typedef struct {
  int d, L, variant;
  int m[32];
  double *u[32], *f[32], *r[32];
} hier_t;

static void hier_free(hier_t *H) {
  for (int l = 0; l < H->L; l++) {
    if (l > 0) {
      free(H->u[l]);
      free(H->f[l]);
    }
    free(H->r[l]);
  }
}

/* allocate coarse levels 1..L-1 (u_l, f_l) and a scratch r_l on every level;
 * level 0 aliases the caller's u, f. */
static int hier_init(hier_t *H, int d, int m0, double *u0, const double *f0) {
  memset(H, 0, sizeof(*H));
  int L = orc_levels(m0);
  if (L < 1 || (d != 2 && d != 3)) return -1;
  H->d = d;
  H->L = L;
  for (int l = 0; l < L; l++) {
    H->m[l] = (1 << (L - l)) - 1;
    long N = npts(d, H->m[l]);
    if (l == 0) {
      H->u[0] = u0;
      H->f[0] = (double *)f0;
    } else {
      H->u[l] = (double *)calloc((size_t)N, sizeof(double));
      H->f[l] = (double *)calloc((size_t)N, sizeof(double));
    }
    H->r[l] = (double *)calloc((size_t)N, sizeof(double));
  }
  return 0;
}

static void smooth(hier_t *H, int l, int smoother, double omega, int nsweeps, int backward) {
  if (nsweeps <= 0) return;
  if (smoother == ORC_RBGS)
    orc_rbgs(H->d, H->m[l], H->u[l], H->f[l], nsweeps, backward);
  else if (smoother == ORC_MCGS)
    orc_mcgs(H->d, H->m[l], H->u[l], H->f[l], nsweeps, backward);
  else
    orc_wj(H->d, H->m[l], H->u[l], H->f[l], omega, nsweeps, H->r[l]);
}

/* Exact solve of the 1-DOF coarsest level: 2d u / h^2 = f. */
static void coarsest_solve(hier_t *H) {
  int l = H->L - 1;
  double h = 1.0 / (double)(H->m[l] + 1);
  H->u[l][0] = (h * h * H->f[l][0]) / (2.0 * H->d);
}

static void restrict_to(hier_t *H, int l, const double *r, double *fc) {
  if (H->variant & ORC_FE_TRANSFER)
    orc_restrict_fe(H->d, H->m[l + 1], r, fc);
  else
    orc_restrict_fw(H->d, H->m[l + 1], r, fc);
}

static void prolong_from(hier_t *H, int l) {
  if (H->variant & ORC_FE_TRANSFER)
    orc_prolong_add_fe(H->d, H->m[l + 1], H->u[l + 1], H->u[l]);
  else
    orc_prolong_add(H->d, H->m[l + 1], H->u[l + 1], H->u[l]);
}

/* Coarsest level: exact, or (variant) nu1 smoother sweeps from zero. */
static void coarsest(hier_t *H, int nu1, int smoother, double omega) {
  if (H->variant & ORC_COARSE_RELAX) {
    H->u[H->L - 1][0] = 0.0;
    smooth(H, H->L - 1, smoother, omega, nu1, 0);
  } else {
    coarsest_solve(H);
  }
}

/* The V-cycle in its recursive (two-grid) form: on level l, relax, form the
 * residual and restrict it as the next level's right-hand side, solve the
 * coarse error equation from a zero start by the same cycle one level down
 * (exactly on the one-node level), add its interpolation and relax again in
 * the reverse colour order.  The result is the cycle Algorithm 1 defines:
 * every level runs the same steps in the same order. */
static void vcycle_from(hier_t *H, int l, int nu1, int nu2, int smoother, double omega) {
  if (l == H->L - 1) {
    coarsest(H, nu1, smoother, omega);
    return;
  }
  smooth(H, l, smoother, omega, nu1, 0);
  orc_residual(H->d, H->m[l], H->u[l], H->f[l], H->r[l]);
  restrict_to(H, l, H->r[l], H->f[l + 1]);
  if (l + 1 < H->L - 1)
    memset(H->u[l + 1], 0, sizeof(double) * (size_t)npts(H->d, H->m[l + 1]));
  vcycle_from(H, l + 1, nu1, nu2, smoother, omega);
  prolong_from(H, l);
  smooth(H, l, smoother, omega, nu2, 1);
}

static void vcycle(hier_t *H, int nu1, int nu2, int smoother, double omega) {
  vcycle_from(H, 0, nu1, nu2, smoother, omega);
}

/* One V(nu1, nu2) cycle applied in place to u (level 0, side m0). */
int orc_vcycle(int d, int m0, double *u, const double *f, int nu1, int nu2, int smoother,
               double omega, int variant) {
  hier_t H;
  if (hier_init(&H, d, m0, u, f)) return -1;
  H.variant = variant;
  vcycle(&H, nu1, nu2, smoother, omega);
  hier_free(&H);
  return 0;
}

/* Solve loop.  res0 = ||f - A u|| unless res0_in > 0 is given (resume);
 * while res > rtol*res0 and it < maxit: V-cycle; it++.  Writes the
 * iteration count, the final relative residual and (optionally) the residual
 * history res_hist[0..it] (res_hist[0] = residual of the initial guess).
 * Returns 0 converged, 1 maxit reached, -3 non-finite residual. */
int orc_solve(int d, int m0, double *u, const double *f, int nu1, int nu2, int smoother,
              double omega, double rtol, int maxit, double res0_in, int *iters, double *relres,
              double *res_hist, int variant) {
  hier_t H;
  if (hier_init(&H, d, m0, u, f)) return -1;
  H.variant = variant;
  orc_residual(d, m0, u, f, H.r[0]);
  double res = orc_norm2(d, m0, H.r[0]);
  double res0 = res0_in > 0.0 ? res0_in : res;
  if (res_hist) res_hist[0] = res;
  int it = 0, status = 0;
  if (!isfinite(res)) status = -3;
  while (status == 0 && res > rtol * res0 && it < maxit) {
    vcycle(&H, nu1, nu2, smoother, omega);
    it++;
    orc_residual(d, m0, u, f, H.r[0]);
    res = orc_norm2(d, m0, H.r[0]);
    if (res_hist) res_hist[it] = res;
    if (!isfinite(res)) status = -3;
  }
  if (status == 0 && res > rtol * res0) status = 1;
  *iters = it;
  *relres = res0 > 0.0 ? res / res0 : 0.0;
  hier_free(&H);
  return status;
}

/* Full multigrid (Algorithm 2): restrict f to every level (full weighting,
 * or the finite-element restriction for that variant), solve the coarsest
 * level (exactly, or by the variant's relaxation), then for l = L-2 .. 0 interpolate the
 * level-(l+1) solution to level l and run one V(nu1, nu2) cycle on the
 * sub-hierarchy l .. L-1.  u (level 0) is overwritten. */
int orc_fmg(int d, int m0, double *u, const double *f, int nu1, int nu2, int smoother,
            double omega, int variant) {
  hier_t H;
  if (hier_init(&H, d, m0, u, f)) return -1;
  H.variant = variant;
  int L = H.L;
  for (int l = 0; l <= L - 2; l++) restrict_to(&H, l, H.f[l], H.f[l + 1]);
  coarsest(&H, nu1, smoother, omega);
  for (int l = L - 2; l >= 0; l--) {
    memset(H.u[l], 0, sizeof(double) * (size_t)npts(d, H.m[l]));
    prolong_from(&H, l);
    /* one V-cycle on levels l..L-1 with level l as the finest */
    hier_t S;
    memset(&S, 0, sizeof(S));
    S.d = d;
    S.L = L - l;
    S.variant = variant;
    for (int q = 0; q < S.L; q++) {
      S.m[q] = H.m[l + q];
      S.u[q] = H.u[l + q];
      S.f[q] = H.f[l + q];
      S.r[q] = H.r[l + q];
    }
    vcycle(&S, nu1, nu2, smoother, omega);
  }
  hier_free(&H);
  return 0;
}
