/*
 * mg.h -- C ABI of the MI355X geometric-multigrid library (libmg.so).
 *
 * Solves A x = b for the discrete Poisson-type operators of J. T. Wallis,
 * "Methods toward better Multigrid Solver Convergence" (KAIST, 2008), with the
 * recursive multigrid algorithm MG(l, u, g) of its section "The Multigrid
 * Technique" run as the F-cycle named in its Abstract:
 *   - the 5-point finite-difference operator -(eps_x u_xx + eps_y u_yy)
 *     (Abstract: Poisson problem; section "Anisotropies": -alpha u_xx - beta u_yy);
 *   - the 9-point bilinear (Q1) operator -div(diag(kx, ky) grad u) with
 *     per-cell coefficients, as produced by mapping a curved domain such as a
 *     polar annulus to the unit square (Introduction, "Some Typical Problems";
 *     section "Different coordinate systems");
 *   - smoothers x <- x - omega C^{-1} (A x - b) (section "Smoothers") with
 *     C = D (damped Jacobi) or C = D + L (Gauss-Seidel, section "The choice
 *     of C") in red-black (5-point) or four-colour (9-point) order;
 *   - full-weighting restriction, bilinear prolongation, correction weight
 *     omega_l = 1 and an exact (Cholesky) solve on the coarsest grid.
 *
 * Conventions shared by every entry point
 *   - Array arguments named x, rhs, r, u, lam, kx, ky, dL_dk are HIP DEVICE
 *     pointers owned by the caller.  The library never frees them and never
 *     keeps them beyond the call (coefficients are copied at setup).
 *   - Node arrays are row-major [ny][nx], x fastest, no padding, FP64.  They
 *     hold every stored node, including Dirichlet boundary nodes.  A
 *     Dirichlet boundary node is not an unknown: its value is taken as zero,
 *     rhs entries there are ignored, and mg_solve writes zero there.
 *   - Cell arrays are row-major [ncy][ncx] with ncx = nx - 1 cells along x
 *     and ncy = ny - 1 (Dirichlet y) or ny (periodic y) cells along y; cell
 *     (ci, cj) has the nodes (ci..ci+1, cj..cj+1), the y index wrapping when
 *     y is periodic.
 *   - Every argument check happens before any device work.  A negative status
 *     means the call did nothing (x untouched); mg_last_error() then holds a
 *     message.  A positive status is a numerical outcome and x holds the last
 *     iterate.
 *   - Work is ordered on the stream given in mg_options.stream (NULL = the
 *     null stream); mg_solve and mg_residual synchronise that stream once
 *     before returning.  A handle must not be used by two threads at once.
 */
#ifndef MG_H
#define MG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mg_handle_s* mg_handle;

typedef enum {
  MG_OK = 0,              /* converged: ||b - A x|| <= tol * ||b - A x0|| */
  MG_NOT_CONVERGED = 1,   /* max_cycles reached; x = last iterate */
  MG_DIVERGED = 2,        /* residual non-finite or > 1e6 * initial; x = last iterate */
  MG_EINVAL = -1,         /* invalid argument; nothing done */
  MG_ENOMEM = -2,         /* device allocation failed */
  MG_EDEVICE = -3,        /* a HIP call failed */
  MG_EUNSUPPORTED = -4    /* valid but unsupported combination (see mg_last_error) */
} mg_status;

enum { MG_COEF_CONST5 = 0, MG_COEF_CELL9 = 1 };
/* Cycles (MG(l, u, g) of "The Multigrid Technique"): F gives the coarse
 * problem one F-cycle then one V-cycle; V one V-cycle (p = 1); W two
 * W-cycles, the second from the first's result (p = 2). */
enum { MG_CYCLE_F = 0, MG_CYCLE_V = 1, MG_CYCLE_W = 2 };
/* Smoothers (the preconditioner C of the Richardson step x <- x + omega
 * C^-1 (b - A x), "The choice of C" and "Smoothing"): damped point Jacobi;
 * point Gauss-Seidel in red-black (5-point) or four-colour (9-point) order;
 * line smoothers whose C is the tridiagonal part of A along x lines (rows) or
 * y lines (columns): TRI_X / TRI_Y damped by omega, ADI = a TRI_X then a
 * TRI_Y step, GSTRI_X / GSTRI_Y Gauss-Seidel over whole lines in zebra order
 * (even stored line index first, every line solved exactly), GSADI = a
 * GSTRI_X then a GSTRI_Y step.  Line smoothers run every level visit as one
 * launch per line sweep (no fused tiles); lines along a periodic direction
 * (TRI_Y, ADI, GSTRI_Y, GSADI with periodic_y) and batched handles are
 * MG_EUNSUPPORTED. */
enum {
  MG_SMOOTH_JACOBI = 0,
  MG_SMOOTH_RBGS = 1,
  MG_SMOOTH_GS4C = 2,
  MG_SMOOTH_TRI_X = 3,
  MG_SMOOTH_TRI_Y = 4,
  MG_SMOOTH_ADI = 5,
  MG_SMOOTH_GSTRI_X = 6,
  MG_SMOOTH_GSTRI_Y = 7,
  MG_SMOOTH_GSADI = 8
};
enum { MG_PREC_FP64 = 0, MG_PREC_MIXED = 1 };
enum { MG_TILES_FUSED = 0, MG_TILES_PER_OP = 1, MG_TILES_NARROW = 2, MG_TILES_WIDE = 3 };

/* Grid: stored node counts and domain lengths.  A Dirichlet direction has
 * n = 2^k m + 1 nodes (h = l / (n - 1)); the periodic direction has n = 2^k m
 * nodes (h = l / n).  Only y may be periodic (periodic_x must be 0).
 * xs, ys (HOST arrays, nullable, read during the call only): node
 * coordinates of a refined (graded) tensor grid -- the anisotropically
 * refined grids of the "Anisotropies" section, refined toward one side in
 * "Different coordinate systems" -- nx (ny) strictly increasing values
 * spanning lx (ly); NULL means equidistant.  Refined grids need
 * MG_COEF_CELL9 (the Q1 operator on each rectangle: kx hy_c/hx_c K1 (x) M1 +
 * ky hx_c/hy_c M1 (x) K1, divided by the equidistant hx hy) and a Dirichlet
 * y direction when ys is given; the coarse levels are the Galerkin products
 * with the transfers of the logically equidistant grid.  Other uses are
 * MG_EUNSUPPORTED. */
typedef struct {
  int32_t nx, ny;
  int32_t periodic_x, periodic_y;
  double lx, ly;
  const double* xs;
  const double* ys;
} mg_grid;

/* Operator.
 * MG_COEF_CONST5: 5-point FD for -(eps_x u_xx + eps_y u_yy); kx, ky unused.
 * MG_COEF_CELL9 : Q1 FEM for -div(diag(kx, ky) grad u), divided by hx*hy
 *   ("FD scaling", so b is the nodal value of f when f is lumped).  kx, ky are
 *   device cell arrays; ky may equal kx.  With kx_1d_along_x = 1 they hold
 *   ncx values (coefficients that vary along x only, e.g. the polar annulus),
 *   else ncy*ncx values.  Coarse 9-point operators are Galerkin R A P. */
typedef struct {
  int32_t kind;
  double eps_x, eps_y;
  const double* kx;
  const double* ky;
  int32_t kx_1d_along_x;
} mg_coeffs;

/* Options.  nu_pre, nu_post in [0, 8].  omega: Jacobi and TRI / ADI damping.
 * sor: relaxation factor of the point Gauss-Seidel smoothers (RBGS, GS4C),
 * the SOR form C = D + sor L of "The choice of C" with L the couplings to
 * earlier colours, each node x <- x + sor (x_GS - x); in (0, 2), 0 means 1
 * (plain Gauss-Seidel, bit for bit the same as sor = 1); ignored by the
 * other smoothers.  precision MG_PREC_MIXED runs every cycle in FP32 inside an
 * FP64 defect-correction loop (x, rhs stay FP64 at the boundary).
 * coarse_cta_nodes: levels with at most this many stored nodes run inside one
 * persistent workgroup (0 = the largest levels whose sub-hierarchy fits in
 * LDS).  tile_mode: MG_TILES_FUSED (default) runs each large-level visit as two
 * LDS-tiled passes (smoothing fused with restriction / with prolongation),
 * with 128-column "wide" tiles on levels large enough to fill the GPU with
 * them and small tiles elsewhere; MG_TILES_NARROW uses small tiles only,
 * MG_TILES_WIDE wide tiles on every fused level; MG_TILES_PER_OP launches
 * one kernel per smoothing sweep, restriction and prolongation.  All modes
 * give the same results, bit for bit.  tile_x, tile_y: output tile of the
 * fused passes (even, 0 = chosen per level); a nonzero tile_x selects small
 * tiles of that width, tile_y alone sets the height of wide tiles.
 * stream: hipStream_t.
 * inner_cycles: MG_PREC_MIXED only, the FP32 cycles of one outer step: the
 *   correction e of A e = (float) r starts at 0 and gets that many cycles
 *   before x += (double) e (0 means 1; at most 16).  Ignored in FP64.
 * coarse_op: operators of the coarse levels.  MG_COARSE_DEFAULT: a 5-point
 *   problem rediscretises its operator on every level (H = 2h), a 9-point
 *   problem takes the Galerkin product R A P.  MG_COARSE_GALERKIN on a 5-point
 *   problem: the coarse levels take R A P too (they are then 9-point, so the
 *   smoother must be MG_SMOOTH_JACOBI or MG_SMOOTH_GS4C; red-black and line
 *   smoothers are MG_EUNSUPPORTED, and so are batched handles).
 * adaptive_omega: 0 adds each coarse-grid correction with omega_l = 1; 1
 *   takes the adaptive omega_l that "The Multigrid Technique" allows in place
 *   of a fixed value: the weight that minimises the energy norm of the error
 *   along the prolonged correction P v, omega_l = (d_l, P v) / (A_l P v, P v)
 *   with d_l = g_l - A_l u_l the defect of the smoothed iterate (1 when
 *   A_l P v = 0), computed on every level visit by a reduction over the
 *   level (one extra pass over x, b and the coarse correction). */
typedef struct {
  int32_t cycle;
  int32_t smoother;
  int32_t nu_pre, nu_post;
  double omega;
  int32_t precision;
  int32_t coarse_cta_nodes;
  int32_t tile_mode;
  int32_t tile_x, tile_y;
  void* stream;
  double sor;
  int32_t inner_cycles;
  int32_t coarse_op;
  int32_t adaptive_omega;
  int32_t tune;
} mg_options;

/* tune: MG_TUNE_AUTO (0, default) lets mg_setup choose the tile shape of
 * every fused pass and the coarse-level threshold by timing candidates on the
 * handle's own level buffers, and caches the choices (keyed by level shape,
 * operator, precision, smoother, device architecture and kernel-source
 * digest) in a JSON file: $MG_TUNE_CACHE, or libmg_tune.json beside the
 * library (MG_TUNE_CACHE=off: no cache); MG_TUNE_OFF (1) takes the fixed
 * rule; MG_TUNE_REFRESH (2) measures again and overwrites the cache.  Every
 * choice gives the same iterates bit for bit (with adaptive_omega the
 * threshold is not tuned: the single-workgroup kernel orders the level-wide
 * sums of omega_l differently).  Explicit tile_mode, tile_x, tile_y or
 * coarse_cta_nodes values are kept as given. */
enum { MG_TUNE_AUTO = 0, MG_TUNE_OFF = 1, MG_TUNE_REFRESH = 2 };

enum { MG_COARSE_DEFAULT = 0, MG_COARSE_GALERKIN = 1 };

/* Solve report.  history (nullable, host) receives the residual norms
 * ||b - A x_k||, k = 0..cycles; it must hold max_cycles + 1 doubles.  status
 * is this problem's own outcome (MG_OK, MG_NOT_CONVERGED or MG_DIVERGED), as
 * the stopping test on the device decided it. */
typedef struct {
  int32_t cycles;
  double res0, res, rel_res;
  double rho_last, rho_mean;   /* last and geometric-mean convergence factor */
  double seconds;              /* device time of the solve (hipEvents) */
  double* history;
  int32_t status;
} mg_info;

/* Build the level hierarchy (shapes, operators, coarsest Cholesky factor) and
 * allocate the level buffers.  levels = 0 coarsens until a Dirichlet
 * direction has 3 nodes or the periodic one 4; levels > 0 asks for exactly
 * that many levels (MG_EINVAL if the grid cannot provide them).  Multigrid
 * algorithm, "The Multigrid Technique": A_l for every level l. */
mg_status mg_setup(const mg_grid* grid, const mg_coeffs* coeffs, int32_t levels,
                   const mg_options* opts, mg_handle* out);

/* Cycle from x (in: start vector x0, out: solution) until
 * ||b - A x_k||_2 <= tol * ||b - A x_0||_2 over the unknowns, max_cycles is
 * reached or the iteration diverges.  tol > 0, max_cycles >= 1.  rhs and x
 * are FP64 device arrays [ny][nx].  info may be NULL. */
mg_status mg_solve(mg_handle h, const double* rhs, double* x, double tol, int32_t max_cycles,
                   mg_info* info);

/* r = rhs - A x on the finest level (r nullable: device array [ny][nx], zero at
 * Dirichlet boundary nodes) and *norm2 = ||r||_2 over the unknowns (host). */
mg_status mg_residual(mg_handle h, const double* rhs, const double* x, double* r, double* norm2);

/* Adjoint gradient for MG_COEF_CELL9 problems: dL_dk[c] = -lam_e^T K_c u_e per
 * cell, where K_c = dA/dk_c is the cell's element matrix for a unit
 * coefficient in both directions (kx = ky = k), u the solution of A u = b and
 * lam the solution of A lam = dL/du (A is symmetric).  u, lam: device node
 * arrays [ny][nx]; dL_dk: device cell array [ncy][ncx]. */
mg_status mg_coeff_grad(mg_handle h, const double* u, const double* lam, double* dL_dk);

/* Replace the cell coefficients of a handle made by mg_setup with
 * MG_COEF_CELL9: every level's operator A_l (Multigrid algorithm, "The
 * Multigrid Technique": the finest Q1 operator from kx, ky, the Galerkin
 * operators below it, the coarsest inverse, line-smoother factors) is
 * rebuilt in the handle's existing device buffers, as mg_setup would build
 * it for these coefficients, without allocating; the next mg_solve uses it.
 * For loops that solve with changing coefficients (gradient steps).  coeffs:
 * kind MG_COEF_CELL9 and kx_1d_along_x as at setup; kx, ky device arrays of
 * the layout mg_setup reads, read during the call only (the handle keeps its
 * own copies).  If kx and ky were the same array at setup they must be the
 * same array here.  Waits for the rebuild.  MG_EUNSUPPORTED for a batched
 * handle; MG_EINVAL for a NULL handle or coeffs, other coefficient kinds, a
 * changed layout, invalid values (not finite and > 0) or a coarsest
 * operator that is not positive definite.  After an error past the argument
 * checks the handle's operators are undefined until a successful update. */
mg_status mg_update_coeffs(mg_handle h, const mg_coeffs* coeffs);

/* Start vector by nested iteration (section "Start-Vector Choice": the
 * solution starts on the coarsest grid and is carried level by level to the
 * finest one): rhs is restricted by full
 * weighting to every level, the coarsest problem solved exactly, and on each
 * finer level below the finest the prolonged coarser result is improved by
 * one cycle of the handle's kind; x (device, [ny][nx], overwritten) receives
 * the prolongation of that result, ready for mg_solve.  The mixed form runs
 * it in FP32 on (float) rhs.  Single-problem handles only (MG_EUNSUPPORTED
 * for batched ones); MG_EINVAL for NULL arrays. */
mg_status mg_start_nested(mg_handle h, const double* rhs, double* x);

/* Measurement helper (for benchmarks, not part of a solve): runs the fused
 * pre-pass (which = 0) or post-pass (which = 1) of `level` once, or with a
 * line smoother (which = 2) the first line sweep of the level's smoothing (one
 * launch: lines along the first swept direction, colour 0 or x -> t), then
 * `reps` more times between two HIP events on the handle's stream, and
 * returns the average device time per launch in *avg_us.  rhs and x are the
 * finest-level arrays as for mg_solve; x is used as scratch and its content
 * is overwritten.  On the finest level of the mixed form with inner_cycles
 * = K, timed launch r runs as inner cycle r % K does in a solve (the first
 * pre-pass of an outer step from a zero start, the last post-pass adding the
 * correction into the FP64 iterate), so reps a multiple of K give the
 * solve's average.  MG_EUNSUPPORTED if that level has no such pass (it runs
 * in the single-workgroup coarse kernel, tile_mode is MG_TILES_PER_OP, or
 * the smoother is not of the asked kind). */
mg_status mg_profile_pass(mg_handle h, const double* rhs, double* x, int32_t level, int32_t which, int32_t reps,
                          double* avg_us);

/* Measurement helper: the launch shape of the fused pre-pass (which = 0) or
 * post-pass (which = 1) of `level`, written to the host array out[10]:
 * out[0] wide tiles (1) or small tiles (0), out[1] TX, out[2] TY, out[3]
 * halo H (columns), out[4] workgroups per problem, out[5] colours per
 * smoothing step (0 Jacobi, 2, 4), out[6] stencil (0 5-point, 1 9-point),
 * out[7] 1 if the 9-point bands vary along x only, out[8] 1 if the pass
 * forms the FP64 residual b - A x itself (the mixed form's first finest
 * pre-pass of an outer step; no separate residual kernel then runs), out[9]
 * the row halo (smaller than H on wide tiles with four colours: a tile's
 * region is TY + 2 out[9] rows).  Same errors as mg_profile_pass; no device
 * work. */
mg_status mg_pass_info(mg_handle h, int32_t level, int32_t which, int32_t* out);

/* Batched: nprob independent 5-point problems (MG_COEF_CONST5 only) with
 * their own grids (square or not) and their own eps_x, eps_y.  grids, coeffs:
 * host arrays of nprob entries.  levels as for mg_setup, applied to every
 * problem (0: each coarsens as far as its grid allows; > 0: exactly that many
 * levels each, MG_EINVAL if a grid cannot provide them).  One sequence of
 * launches serves every problem; converged problems are masked. */
mg_status mg_setup_batched(const mg_grid* grids, const mg_coeffs* coeffs, int32_t nprob, int32_t levels,
                           const mg_options* opts, mg_handle* out);

/* rhs, x: host arrays of nprob device pointers.  info: host array of nprob
 * entries or NULL (each entry's status is that problem's outcome).  Returns
 * MG_OK if every problem converged, else the largest positive status among
 * the problems. */
mg_status mg_solve_batched(mg_handle h, const double* const* rhs, double* const* x, double tol,
                           int32_t max_cycles, mg_info* info);

/* mg_residual without a handle and without allocating, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): r = rhs - A x (r nullable: device
 * array [ny][nx], its Dirichlet boundary nodes written 0) and *norm2 =
 * ||r||_2 over the unknowns (host), for the operator that grid and coeffs
 * describe as for mg_setup -- MG_COEF_CONST5, or MG_COEF_CELL9 whose
 * couplings are formed at each node from the caller's cell arrays kx, ky
 * (device, read during the call; finite and > 0, not checked) -- the same
 * values as mg_residual on a handle for that grid and operator, up to
 * rounding for MG_COEF_CELL9 (mg_residual reads assembled bands there).
 * stream: hipStream_t (NULL = the null stream); the call waits for it once.
 * It allocates nothing: its scratch (level descriptor, norm state and at most
 * 1024 partial sums, 9 KiB) is one static device array per GPU, held until
 * the process ends, and every call on a GPU shares it -- calls that overlap
 * on one GPU (two threads or two streams) race and must be serialised by the
 * caller.  Sizes: nx and ny at most 65537 (MG_EINVAL beyond, before any
 * device work); other errors as for mg_setup's grid and coefficient checks
 * and mg_residual's. */
mg_status mg_residual_noalloc(const mg_grid* grid, const mg_coeffs* coeffs, const double* rhs, const double* x,
                              double* r, double* norm2, void* stream);

/* How a handle runs its cycle, written to the host array out[4]: out[0]
 * merged schedules (batched problems whose level chains end alike run one
 * schedule in which each launch covers every problem on a level, the smaller
 * problems taking part in the recursive call that is their own cycle),
 * out[1] grid groups inside them, out[2] groups running their own cycle (a
 * parallel graph branch each), out[3] launches in the graph of one cycle.
 * Single-problem handles report 0, 0, 1 and their launch count. */
mg_status mg_batch_schedule(mg_handle h, int32_t* out);

/* Frees everything the handle owns (never caller memory).  NULL is accepted. */
mg_status mg_destroy(mg_handle h);

const char* mg_status_string(mg_status s);

/* Message of the last failed call on this handle (or of the last failed
 * mg_setup* on this thread when h is NULL). */
const char* mg_last_error(mg_handle h);

/* Number of levels and the stored shape of level l (0 = finest). */
mg_status mg_level_shape(mg_handle h, int32_t l, int32_t* nx, int32_t* ny);
int32_t mg_num_levels(mg_handle h);

#ifdef __cplusplus
}
#endif

#endif /* MG_H */
