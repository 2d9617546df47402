/*
 * gmg.h -- C ABI of an MI355X (gfx950) geometric-multigrid solver for the
 * finite-difference Poisson problem
 *
 *     -Lap u = f  in (0,1)^d,   u = 0 on the boundary,   d = 2 or 3,
 *
 * discretised by the 5-point (2D) / 7-point (3D) central-difference scheme on
 * a uniform mesh h = 1/n (Feng, Shu, Xu, Zhang, arXiv:1208.4247, Sec. 2.2,
 * eq. (1) and the two difference schemes).  The solver is the multigrid
 * V-cycle of Algorithm 1 inside the iteration loop of Algorithm 3, with every
 * level, down to the one-node coarsest grid, kept on the GPU.
 *
 * DATA LAYOUT (all entry points)
 *   A grid function on a level with n = 2^k intervals per axis is a dense
 *   array of m^d values, m = n - 1 interior nodes per axis, x fastest:
 *   element i + m*(j + m*k) holds node (i+1, j+1, k+1), i.e. x = (i+1)h.
 *   Boundary nodes are not stored (homogeneous Dirichlet data).  f holds the
 *   physical right-hand side f(x) (not h^2 f).  FP64 unless stated.
 *
 * OWNERSHIP
 *   The caller owns every device buffer (u, f, the workspace) and the stream;
 *   the library never allocates device memory (one exception: the FFT plan
 *   of the sine-transform solver, whose twiddle tables rocFFT allocates).
 *   The library owns only the host-side plan object.  Device pointers must be hipMalloc'ed (or
 *   torch-allocated) memory of the current device, 8-byte aligned.  Arrays
 *   passed to one call must not overlap unless stated.
 *
 * ERRORS
 *   Every entry point returns a gmg_status; nothing aborts or throws across
 *   the ABI.  Arguments are validated before any HIP call, so invalid input
 *   is reported the same way with or without a GPU.  HIP failures map to
 *   GMG_ERR_HIP.  GMG_NOT_CONVERGED still fills iteration counts and
 *   residuals.
 *
 * THREADING / STREAMS
 *   A plan is bound to the stream given at setup; calls on one plan must not
 *   run concurrently from several host threads.  gmg_vcycle and the gmg_op_*
 *   calls without a host output only enqueue work; gmg_solve and
 *   gmg_batch_solve synchronise on the stream once per convergence check.
 */
#ifndef GMG_H
#define GMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GMG_OK = 0,
  GMG_NOT_CONVERGED = 1,    /* maxit reached before rtol; outputs filled    */
  GMG_ERR_INVALID_ARG = -1, /* bad size, order, pointer, tolerance, ...     */
  GMG_ERR_WORKSPACE = -2,   /* workspace missing, too small or misaligned   */
  GMG_ERR_NONFINITE = -3,   /* a residual norm was NaN or Inf               */
  GMG_ERR_DIVERGED = -4,    /* relative residual grew above 1e3             */
  GMG_ERR_HIP = -5,         /* a HIP runtime call failed                    */
  GMG_ERR_UNSUPPORTED = -6  /* valid request the library does not provide   */
} gmg_status;

/* Smoother (Sec. 3.2, Remark 1; Table 5).  RBGS: red-black Gauss-Seidel,
 * red = nodes whose node-index sum is even.  A forward sweep relaxes red then
 * black; a backward sweep black then red.  WJ: weighted Jacobi
 * u <- (1-omega) u + omega (h^2 f + sum of neighbours) / (2d).  MCGS: the
 * paper's multicolour Gauss-Seidel (Remark 1), 4 colours in 2D and 8 in 3D:
 * node (i, j[, k]) has colour (i&1) + 2(j&1) [+ 4(k&1)]; a forward sweep
 * relaxes colours in increasing order, a backward sweep in decreasing order.
 * MCGS plans run FP64 single problems only (GMG_ERR_UNSUPPORTED otherwise). */
typedef enum { GMG_SMOOTH_RBGS = 0, GMG_SMOOTH_WJ = 1, GMG_SMOOTH_MCGS = 2 } gmg_smoother;

/* Precision of a plan.  FP64: every level in FP64.  MIXED_FP32_IR: an FP64
 * defect-correction loop (residual, update and norm in FP64) around FP32
 * V-cycles whose one-node coarsest solve is done in FP64. */
typedef enum { GMG_FP64 = 0, GMG_MIXED_FP32_IR = 1 } gmg_precision;

/* Element type of the gmg_op_* primitives. */
typedef enum { GMG_F64 = 0, GMG_F32 = 1 } gmg_dtype;

/* gmg_config.flags */
#define GMG_USE_GRAPH 0x1u          /* replay cycles from a captured hipGraph   */
#define GMG_AUTOTUNE 0x2u           /* time tile variants at setup, cache them  */
#define GMG_PROFILE 0x4u            /* time every kernel launch with hipEvents  */
#define GMG_POST_FORWARD 0x8u       /* post-smooth red->black (textbook order)
                                       instead of Algorithm 1's backward sweep */
#define GMG_NO_TEMPORAL_BLOCKING 0x10u /* one fused sweep per pass at most     */
#define GMG_NO_FUSED_COARSE 0x20u   /* small coarse levels through the general
                                       passes instead of the fused LDS-tile
                                       kernels (same results, for testing)    */
#define GMG_NO_FUSED_RESTRICT 0x40u /* residual + restriction as a kernel of its
                                       own instead of inside the last
                                       pre-smoothing pass (same results)      */
/* The paper's own transfers and coarsest rule (with any smoother; FP64 single
 * problems only, GMG_ERR_UNSUPPORTED otherwise).  Such plans (and MCGS plans)
 * run one kernel per step and level, without the small-level kernels, the
 * bottom kernel or the folded restriction; GMG_USE_GRAPH and GMG_AUTOTUNE
 * have no effect on them (red-black or Jacobi sweeps keep the default tile
 * choices). */
#define GMG_FE_TRANSFER 0x80u       /* linear finite-element restriction and
                                       interpolation (Sec. 4, eq. Restriction2d
                                       and eq. Prolongation2d; 15-point in 3D)
                                       instead of full weighting / (bi/tri)-
                                       linear interpolation                   */
#define GMG_COARSE_RELAX 0x100u     /* one-node coarsest level relaxed by nu1
                                       sweeps from zero (Algorithm 1 as printed)
                                       instead of solved exactly; differs only
                                       for WJ                                  */
#define GMG_NO_CROSS_CYCLE 0x200u   /* FP64 red-black V(1,1) solves: run each
                                       cycle's level-0 post-smoothing and the
                                       next cycle's pre-smoothing as two passes
                                       instead of one (same iterates)         */
#define GMG_BATCH_ONE_STREAM 0x400u /* batched plans holding 2D and 3D problems:
                                       run all launches in order on the plan's
                                       stream instead of the 2D problems' on a
                                       concurrent side stream (same results)  */

typedef struct {
  int dim;                 /* 2 or 3                                            */
  int levels;              /* L: finest side m0 = 2^L - 1, coarsest has 1 node  */
  gmg_smoother smoother;   /* default GMG_SMOOTH_RBGS                           */
  int nu1, nu2;            /* pre/post sweeps (V(nu1,nu2)); nu1 + nu2 >= 1     */
  double omega;            /* WJ weight in (0, 1]; ignored by RBGS; 0 = default
                              2d/(2d+1) (4/5 in 2D, 6/7 in 3D)                   */
  gmg_precision precision; /* default GMG_FP64                                  */
  int inner_cycles;        /* FP32 V-cycles per refinement step (>= 1)          */
  unsigned flags;          /* GMG_* flags above                                 */
} gmg_config;

typedef struct gmg_plan gmg_plan; /* opaque, host side */

/* Fill *cfg with defaults: RBGS V(2,2), FP64, four inner cycles (used by
 * MIXED_FP32_IR plans), no flags. */
gmg_status gmg_config_default(gmg_config *cfg, int dim, int levels);

/* Create a plan (Algorithm 3's set-up: level table, workspace carving).
 * Two-phase: with workspace == NULL only *ws_bytes is written (the bytes the
 * plan needs) and *out is left untouched.  Otherwise workspace must point to
 * at least *ws_bytes bytes of device memory, 256-byte aligned, which the plan
 * uses until gmg_destroy; the caller keeps ownership.
 * nproblems == 1: dims/levels may be NULL (cfg->dim and cfg->levels apply).
 * nproblems > 1 (batch): dims[p] and levels[p] give each problem's dimension
 * and level count; cfg->dim/levels are ignored.
 * stream: a hipStream_t (NULL = the default stream).
 * Errors: GMG_ERR_INVALID_ARG (dim not 2/3, levels < 1 or too large for the
 * int32 index space, nu1 + nu2 < 1, nu > 8, omega outside (0,1],
 * inner_cycles < 1, nproblems < 1, NULL out/ws_bytes), GMG_ERR_WORKSPACE
 * (workspace smaller than required or not 256-byte aligned),
 * GMG_ERR_UNSUPPORTED (a combination the library does not run, e.g. batch
 * with mixed precision), GMG_ERR_HIP. */
gmg_status gmg_setup(const gmg_config *cfg, int nproblems, const int *dims, const int *levels,
                     void *workspace, size_t *ws_bytes, void *stream, gmg_plan **out);

/* One V(nu1,nu2) cycle (Algorithm 1) applied in place to u for right-hand
 * side f (single-problem plans).  Enqueue only.  In MIXED_FP32_IR mode: one
 * refinement step x <- x + V32(f - A x).  u and f: device, m0^d FP64. */
gmg_status gmg_vcycle(gmg_plan *p, double *u, const double *f);

/* Full multigrid FMG(nu1, nu2) (Algorithm 2; single-problem FP64 plans):
 * f is restricted to every level (full weighting, or the finite-element
 * restriction with GMG_FE_TRANSFER), the one-node level is solved (exactly,
 * or relaxed with GMG_COARSE_RELAX), and for each level from the coarse end the coarser result
 * is interpolated and one V(nu1, nu2) cycle is run on that level and the
 * ones below it.  u (output only, m0^d FP64) receives the finest result;
 * it reaches the discretisation error in one pass for smooth data.
 * Enqueue only.  GMG_ERR_UNSUPPORTED for mixed-precision plans. */
gmg_status gmg_fmg(gmg_plan *p, double *u, const double *f);

/* Solve loop of Algorithm 3 with every level on the GPU: res0 = ||f - A u||_2
 * for the initial u (or *res0_opt when resuming); repeat V-cycles while
 * ||f - A u||_2 > rtol * res0 and the cycle count is below maxit.  The
 * Euclidean norm is used.  u is the initial guess on entry and the result on
 * return.  Outputs (host, may be NULL): *iters = cycles done,
 * *relres = final ||f - A u|| / res0 (0 when res0 == 0).
 * Returns GMG_OK, GMG_NOT_CONVERGED, GMG_ERR_NONFINITE, GMG_ERR_DIVERGED,
 * GMG_ERR_INVALID_ARG (rtol <= 0, maxit < 1, NULL u/f), GMG_ERR_HIP. */
gmg_status gmg_solve(gmg_plan *p, double *u, const double *f, double rtol, int maxit,
                     const double *res0_opt, int *iters, double *relres);

/* Batch solve (plans made with nproblems > 1): u[q], f[q] are device
 * pointers (host array of nproblems pointers) to problem q's grids.  Every
 * problem runs the same algorithm as gmg_solve with its own stop test; the
 * cycles of all problems are interleaved level by level.  iters[q],
 * relres[q], st[q] (host arrays, may be NULL) get per-problem results; the
 * return value is the worst per-problem status. */
gmg_status gmg_batch_solve(gmg_plan *p, double *const *u, const double *const *f, double rtol,
                           int maxit, int *iters, double *relres, gmg_status *st);

/* Bytes of the device array gmg_solve_scratch works in (one per GPU). */
#define GMG_SCRATCH_BYTES (64u << 20)

/* For callers that cannot allocate (tight serving loops, harnesses that
 * forbid hipMalloc): the solve of gmg_solve on a problem set up by cfg, with
 * no plan or workspace from the caller.  Its workspace is a device array of
 * GMG_SCRATCH_BYTES that the library keeps per GPU (allocated with the
 * library's code on that GPU, held until the process ends); the call itself
 * allocates no device or pinned host memory and creates no events, streams
 * or graphs.  u (initial guess in, result out) and f are the caller's device
 * arrays, as for gmg_solve; stream as for gmg_setup.  Same arithmetic,
 * results and outputs as gmg_setup + gmg_solve with the same configuration
 * and default tiles.  Synchronises like gmg_solve.  Every call on one GPU
 * uses that GPU's one array, so calls that overlap on a GPU (from several
 * host threads or streams) race; the array keeps the last call's contents,
 * and every value a solve reads from it is written first by that solve.
 * Errors: as gmg_solve and gmg_setup; GMG_ERR_WORKSPACE when the problem's
 * workspace (gmg_setup's size query) exceeds GMG_SCRATCH_BYTES (e.g. 3D
 * FP64 beyond 127^3), checked before any launch; GMG_ERR_UNSUPPORTED with
 * GMG_AUTOTUNE, GMG_PROFILE or GMG_USE_GRAPH. */
gmg_status gmg_solve_scratch(const gmg_config *cfg, double *u, const double *f, double rtol,
                             int maxit, const double *res0_opt, int *iters, double *relres,
                             void *stream);

/* Release the plan (host memory only; the workspace stays the caller's). */
gmg_status gmg_destroy(gmg_plan *p);

/* Static string naming a status. */
const char *gmg_status_string(gmg_status s);

/* Bytes of workspace the plan uses (0 for NULL). */
size_t gmg_plan_workspace_bytes(const gmg_plan *p);

/* Interior side m_l of level l of problem q (-1 if out of range).  Level 0 is
 * the finest; level levels-1 has one node. */
int gmg_level_side(const gmg_plan *p, int problem, int level);

/* Tile shapes of the fused smoothing passes.  A pass applies `stages`
 * stages in one sweep over memory (red-black: 2 per sweep; weighted Jacobi:
 * 1 per sweep; red-black 3: the cross-cycle pass of FP64 V(1,1) solves,
 * which ends one cycle's post-smoothing and starts the next cycle's
 * pre-smoothing); each stage count has a few tile shapes.  Returns the
 * number of shapes (0: that stage count is not provided). */
int gmg_tile_variant_count(int dim, gmg_smoother smoother, int stages);

/* Override the tile shape (index < gmg_tile_variant_count) and the z-chunk
 * (output planes per workgroup; 0 = automatic) used on level `level` of
 * problem 0 for passes with `stages` stages (red-black 3: the cross-cycle
 * pass, level 0 only).  Results do not depend on the choice (tests check
 * this bitwise); only speed does.  Host only. */
gmg_status gmg_plan_set_tile(gmg_plan *p, int level, int stages, int variant, int tz);

/* Order in which the workgroups of a pass with `stages` stages on level
 * `level` take their tiles: strips `strip` tiles wide (filled row by row),
 * or whole rows of tiles (strip = 0, the default).  Each XCD runs a
 * contiguous run of tiles at a time, so narrow strips make that run a
 * compact block whose halos its L2 shares.  Only speed depends on it (the
 * autotuner keeps whole rows: strips measured within +-3% at 1023^3).  Host
 * only; GMG_ERR_INVALID_ARG for a bad level, stage count or strip. */
gmg_status gmg_plan_set_tile_order(gmg_plan *p, int level, int stages, int strip);

/* The tile choice in use (after autotuning, if any) for the first pass of
 * the pre- (role 0) or post-smoothing (role 1) on level `level` of problem 0:
 * its stage count, tile index and z-chunk (resolved, > 0).  Role 2: the
 * cross-cycle pass of level 0 (plans that run it).  Host only; any output
 * pointer may be NULL.  GMG_ERR_INVALID_ARG for a bad level/role, a batch
 * plan, or a role without sweeps. */
gmg_status gmg_plan_get_tile(const gmg_plan *p, int level, int role, int *stages, int *variant,
                             int *tz);

/* Check an autotuner cache file (the file GMG_TUNE_CACHE names; one JSON
 * line per tuned level and role, appended by the tuner).  Counts the lines
 * the tuner would use (*n_valid) and those it skips and re-tunes
 * (*n_invalid): lines that do not parse, keys written for another build's
 * tile tables, and choices that cannot run (sweeps per pass above the cap,
 * a tile index outside the table, a negative z-chunk, or more workgroups
 * than the norm-partials buffer holds).  Blank lines are ignored.  Host only
 * (no HIP call); GMG_ERR_INVALID_ARG for NULL arguments or a file that
 * cannot be opened. */
gmg_status gmg_tune_cache_check(const char *path, int *n_valid, int *n_invalid);

/* ---------------------------------------------------------------------- */
/* Operator primitives.  Each runs exactly the kernels the cycle runs for  */
/* one step, on problem 0's level `level` (side m = gmg_level_side(p,0,l)).*/
/* Pointers: device arrays of m^d (fine) or mc^d (coarse, mc = (m-1)/2)    */
/* elements of dtype dt.  Enqueue only unless a host output is requested. */
/* ---------------------------------------------------------------------- */

/* Smoothing (Algorithm 1, Relax_forward / Relax_backward): u_out =
 * nsweeps sweeps of the plan's smoother applied to the start value
 * u_in + P e_coarse (u_in NULL = zero; e_coarse NULL = no correction;
 * P = (bi/tri)linear interpolation from level+1), with right-hand side f.
 * backward selects the reverse colour order (RBGS: black->red; MCGS:
 * decreasing colours).  If res_in_norm is not NULL, ||f - A u_in||_2 (of the
 * start value, e_coarse must be NULL) is written there (synchronises).
 * u_out must not alias u_in, f or e_coarse.  Plans with MCGS or
 * GMG_FE_TRANSFER: FP64 only and e_coarse must be NULL (interpolate with
 * gmg_op_prolong_add first); GMG_ERR_UNSUPPORTED otherwise. */
gmg_status gmg_op_smooth(gmg_plan *p, int level, gmg_dtype dt, int nsweeps, int backward,
                         const void *u_in, const void *f, const void *e_coarse, void *u_out,
                         double *res_in_norm);

/* Residual and restriction (Algorithm 1, r_l = f_l - A_l u_l;
 * f_{l+1} = R r_l): f_coarse = R(f - A u), r never stored; R is full
 * weighting, or with GMG_FE_TRANSFER the linear finite-element restriction
 * (eq. Restriction2d; FP64 only).  level must be below the coarsest. */
gmg_status gmg_op_restrict_residual(gmg_plan *p, int level, gmg_dtype dt, const void *u,
                                    const void *f, void *f_coarse);

/* Interpolation and correction (Algorithm 1, u_l = u_l + P u_{l+1};
 * eq. Prolongation2d): u_out = u_in + P e_coarse (u_in NULL = zero; u_in may
 * equal u_out), P the plan's interpolation from level+1: (bi/tri)linear, or
 * with GMG_FE_TRANSFER the linear finite-element one (FP64 only).  level must
 * be below the coarsest; e_coarse must not alias u_out. */
gmg_status gmg_op_prolong_add(gmg_plan *p, int level, gmg_dtype dt, const void *u_in,
                              const void *e_coarse, void *u_out);

/* Residual r = f - A u (r may be NULL) and its norm ||r||_2 (norm may be
 * NULL; synchronises when given). */
gmg_status gmg_op_residual(gmg_plan *p, int level, gmg_dtype dt, const void *u, const void *f,
                           void *r, double *norm);

/* ---------------------------------------------------------------------- */
/* Exact discrete solve by the sine transform (Sec. 5.4, the fast direct   */
/* method the paper compares full multigrid with; Tables 12-15).           */
/* ---------------------------------------------------------------------- */
typedef struct gmg_dst gmg_dst; /* opaque, host side */

/* Set up u = A^-1 f for the 5-/7-point scheme on the (2^levels - 1)^dim
 * interior grid with zero Dirichlet data, computed as S^-1 diag(lambda)^-1 S f
 * with S the DST-I along every axis and lambda_k = sum_i (4/h^2)
 * sin^2(k_i pi h / 2) (exact up to rounding).  Two-phase like gmg_setup:
 * with workspace == NULL only *ws_bytes is written.  Otherwise workspace
 * (device memory, 256-byte aligned, at least *ws_bytes bytes, caller-owned)
 * holds the odd extensions and the FFT coefficients of every line and the
 * FFT library's work area (about 4 grids in all).  dim 2 (levels <= 14) or 3
 * (levels <= 10).  stream: a hipStream_t (NULL = default).  The batched FFTs
 * are rocFFT's; plan creation may compile FFT kernels on first use, and the
 * plan keeps twiddle tables in device memory that rocFFT allocates itself
 * (released by gmg_dst_destroy).  Errors:
 * GMG_ERR_INVALID_ARG, GMG_ERR_WORKSPACE, GMG_ERR_HIP (FFT library failure). */
gmg_status gmg_dst_setup(int dim, int levels, void *workspace, size_t *ws_bytes, void *stream,
                         gmg_dst **out);

/* u = A^-1 f (device arrays of m^dim FP64, x fastest; u must not alias f; f is
 * only read).  Enqueue only. */
gmg_status gmg_dst_solve(gmg_dst *p, double *u, const double *f);

/* Release the solver (not the workspace). */
gmg_status gmg_dst_destroy(gmg_dst *p);

/* ---------------------------------------------------------------------- */
/* Profiling (plans set up with GMG_PROFILE): per kernel class, launches,  */
/* summed hipEvent durations on the plan's stream and algorithmic bytes.   */
/* ---------------------------------------------------------------------- */
typedef struct {
  char name[48];
  long long launches;
  double total_ms;
  double alg_bytes; /* algorithmic HBM bytes summed over the launches */
} gmg_kernel_stat;

int gmg_profile_count(const gmg_plan *p);
/* Restrict event timing to the kernel classes whose bit (1 << idx) is set in
 * mask (default: all).  Fewer events perturb the timed run less. */
gmg_status gmg_profile_set_mask(gmg_plan *p, unsigned mask);
gmg_status gmg_profile_get(gmg_plan *p, int idx, gmg_kernel_stat *out); /* synchronises */
gmg_status gmg_profile_reset(gmg_plan *p);

#ifdef __cplusplus
}
#endif
#endif /* GMG_H */
