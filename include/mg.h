/*
 * mg.h -- C ABI of the MI355X (gfx950) tensor-product multigrid solver for the
 * anisotropic Helmholtz-type pressure equation on a latitude-longitude shell.
 *
 * The problem (paper, Section 2): the linear system H u = b of one
 * semi-implicit pressure update. The operator is assembled here as the
 * cell-centred 7-point finite-volume discretisation of
 *     -div(K grad u) + alpha u
 * on a spherical shell, each row integrated over its cell, with periodic
 * longitude, zero flux across the poles and homogeneous Neumann top and
 * bottom; it is symmetric positive definite with seven entries per row.
 *
 * The method (paper, Sections 2.1-2.3): split H = H_z + dH (H_z: diagonal
 * and in-column couplings, dH: horizontal couplings); smooth with damped
 * vertical-line block-Jacobi (Eq. 1, one tridiagonal solve per column);
 * coarsen only horizontally, longitude always and latitude only where the
 * horizontal anisotropy of a row is small (conditional semi-coarsening);
 * run V-cycles with a few smoother sweeps on the coarsest level. The V-cycle
 * runs in FP32 inside an FP64 iterative-refinement loop (residual and update
 * in FP64), entirely in FP64, or entirely in FP32.
 *
 * Conventions for every entry point:
 *  - Field arguments are caller-owned DEVICE pointers holding N =
 *    nlon*nlat*nlev contiguous FP64 values in [k][j][i] order (longitude i
 *    fastest, latitude row j from the south pole, layer k from the surface).
 *    The library never keeps a caller pointer past the call.
 *  - The handle owns all hierarchy and workspace memory (freed by
 *    mg_destroy). All work is ordered on the stream given in mg_options
 *    (a hipStream_t; NULL = the default stream). Solves return after the
 *    result is complete on that stream. A handle is not thread-safe.
 *  - Every call returns an mg_status; no exception crosses the ABI.
 *    MG_ERR_* values < 0 leave outputs unspecified; MG_ERR_NOT_CONVERGED > 0
 *    is a warning (the last iterate is returned). mg_last_error() gives a
 *    human-readable detail of the last failure on a handle.
 *  - With the environment variable MG_LOG set (and not "0") when a handle is
 *    set up, its solves print one line per outer iteration to stderr
 *    (relative residual and contraction factor).
 */
#ifndef MG_H
#define MG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MG_MAX_LEVELS 32
#define MG_MAX_NLEV 128      /* largest supported number of vertical layers */
#define MG_HIST 128          /* residual-history entries kept in mg_stats */

typedef enum {
    MG_OK = 0,
    MG_ERR_NOT_CONVERGED = 1, /* max_iters reached; u holds the last iterate */
    MG_ERR_ARG = -1,          /* invalid argument (message in mg_last_error) */
    MG_ERR_HIP = -2,          /* a HIP runtime call failed */
    MG_ERR_OOM = -3,          /* device allocation failed */
    MG_ERR_BREAKDOWN = -4     /* non-finite residual norm */
} mg_status;

typedef enum {
    MG_PREC_MIXED = 0,        /* FP32 V-cycle inside FP64 refinement */
    MG_PREC_FP64 = 1,         /* everything in FP64 */
    MG_PREC_FP32 = 2          /* everything in FP32: b and u are cast to FP32
                                 on entry (u back on exit), the residual is
                                 FP32 (its norm summed in FP64). Contracts
                                 like MG_PREC_MIXED until the residual meets
                                 the floor set by rounding u to FP32,
                                 ||H (u - fl32(u))|| / ||b|| (1e-4 to 4e-4
                                 on the synthetic shells), then stays there;
                                 tighter tolerances end in
                                 MG_ERR_NOT_CONVERGED */
} mg_precision;

/* Grid of the shell.
 * nlon, nlat : cells in longitude and latitude; both even, nlon >= 2.
 * nlev       : vertical layers, 1..MG_MAX_NLEV.
 *              nlon * nlat * nlev < 2^29 (an FP64 field below 4 GiB).
 * radius     : inner radius R > 0 (the surface).
 * thickness  : shell depth D > 0.
 * stretch    : q > 0; layer depths dz_k = dz_0 q^k upward from the surface,
 *              dz_0 = D (q-1)/(q^nlev - 1) (D/nlev for q = 1).
 * K          : scalar diffusion coefficient > 0. */
typedef struct {
    int32_t nlon, nlat, nlev;
    double radius, thickness, stretch;
    double K;
} mg_grid;

/* alpha: device pointer to N FP64 values, every one finite and > 0. */
typedef struct {
    const double* alpha;
} mg_coeffs;

/* Solver options (fill with mg_options_default, then override).
 * levels        : 0 = automatic (coarsen until every row of the coarsest
 *                 level has anisotropy <= semi_threshold, until the number
 *                 of longitudes is odd, or until a coarser level would have
 *                 fewer than 4 longitudes); n > 0 = at most n levels (the
 *                 paper's shallow hierarchy uses 4).
 * nu_pre/nu_post: smoother sweeps before/after the coarse correction
 *                 (nu_pre >= 1; the first pre-sweep starts from zero).
 * coarse_sweeps : smoother sweeps from zero on the coarsest level (>= 1).
 * max_iters     : cap on outer iterations (<= MG_HIST - 1).
 * omega         : smoother damping (0 < omega < 2); default 0.8.
 * semi_threshold: rows merge in latitude only if both have anisotropy
 *                 a = (dtheta/(cos(theta) dlambda))^2 <= this; default 2.
 * precision     : mg_precision.
 * stream        : hipStream_t used for all work (NULL = default stream).
 * profile       : 0 = off; 1 = time every finest-level kernel launch with
 *                 HIP events and report per-kernel totals in mg_stats;
 *                 2 = time every launch on every level (adds small gaps);
 *                 3 = time only the post-smoothing sweeps of each forward
 *                 V-cycle on the finest level, as one group of nu_post
 *                 launches (two events per cycle: the fewest, for timing
 *                 a solve and its dominant kernel together).
 * smooth_lo, smooth_hi: smoothing interval. smooth_lo > 0 (default 1/3,
 *                 2): the nu sweeps of one smoothing step use damping
 *                 factors omega_k = 1/lambda_k, k = 0..nu-1, with lambda_k
 *                 the nu Chebyshev nodes of [smooth_lo, smooth_hi] (the
 *                 eigenvalues of H_z^{-1} H the smoother must damp), in
 *                 decreasing order of lambda; 0 < smooth_lo < smooth_hi.
 *                 For V(2,2) on [1/3, 2] these are 0.570 and 1.732.
 *                 smooth_lo = 0: every pre- and post-smoothing sweep uses
 *                 omega. A smoothing step of one sweep (nu = 1) and the
 *                 coarsest-level sweeps always use omega.
 * staged_columns: levels with fewer columns (nlon * nlat) than this run
 *                 their sweeps (in the forward and the transposed cycle)
 *                 with the staged kernel: eight wavefronts load a
 *                 64-column segment into LDS in one round trip, two solve
 *                 its columns from there (default 65536; 0 = never). The
 *                 same operations either way, equal up to rounding; the
 *                 speed differs.
 * stall_factor, stall_iters: stagnation guard of MG_PREC_MIXED. When
 *                 stall_iters consecutive outer iterations each leave the
 *                 residual norm above stall_factor times the previous one
 *                 (the FP32 cycle no longer contracts), the solve continues
 *                 from its current iterate with FP64 V-cycles and reports
 *                 fell_back_fp64 = 1. Defaults 0.9 and 3; stall_iters = 0
 *                 turns the guard off.
 * graphs        : 1 (default): the forward V-cycle below the finest level
 *                 is captured once as a HIP graph (at setup, again when
 *                 an option it depends on changes: nu_pre, nu_post,
 *                 coarse_sweeps, omega, precision, smooth_lo, smooth_hi,
 *                 staged_columns, graphs) and replayed in every cycle; 0:
 *                 every kernel is launched directly. Same kernels and
 *                 results.
 * zero_guess    : 0 (default): u holds the initial guess on entry to a
 *                 solve. 1: solves start from u = 0 whatever u holds (u is
 *                 only written), so the first residual is b itself and the
 *                 first update reads no old iterate. The iterates are those
 *                 of passing u = 0 with zero_guess = 0 (only the norms of b
 *                 and of the first residual are summed in another order).
 * poison        : 1: every floating-point array the library allocates from
 *                 then on is filled with quiet NaN first (a check that no
 *                 result depends on memory the library never wrote; costs a
 *                 fill per allocation). Default 0. */
typedef struct {
    int32_t levels;
    int32_t nu_pre, nu_post, coarse_sweeps, max_iters;
    double omega, semi_threshold;
    int32_t precision;
    void* stream;
    int32_t profile;
    double smooth_lo, smooth_hi;
    int32_t staged_columns;
    double stall_factor;
    int32_t stall_iters;
    int32_t graphs;
    int32_t zero_guess;
    int32_t poison;
} mg_options;

/* Kernel classes reported by mg_stats when profiling. */
enum {
    MG_K_RESIDUAL64 = 0,  /* FP64 update + residual + norm partials (fine)  */
    MG_K_SMOOTH,          /* block-Jacobi sweep from an iterate, all levels  */
    MG_K_RESTRICT,        /* fused residual + restriction                     */
    MG_K_PROLONG,         /* bilinear prolongation (add)                      */
    MG_K_COARSE,          /* coarsest-level solve                             */
    MG_K_ADJOINT,         /* unused: the transposed cycle's kernels are     */
                          /* counted in the classes of their forward kinds  */
    MG_K_OTHER,           /* reductions, copies                               */
    MG_K_SMOOTH0,         /* first sweep of a level, from zero                */
    MG_NK
};

/* Statistics of one solve.
 * iters       : outer iterations performed.
 * relres      : final ||b - H u||_2 / ||b||_2 (unweighted 2-norm; the
 *               residual in FP64, in FP32 for MG_PREC_FP32; sums in FP64).
 * res_hist    : ||r_m||_2 for m = 0..iters.
 * ms_total    : wall time of the solve on the host clock (ms).
 * levels_used : levels in the hierarchy.
 * alg_bytes   : algorithmic bytes moved by the solve (each vector read or
 *               written once per pass), for bandwidth figures.
 * kern_ms[c], kern_launches[c], kern_bytes[c]: with options.profile, total
 *               event-timed milliseconds, launches and algorithmic bytes per
 *               kernel class; kern_fine_* the same restricted to the finest
 *               level.
 * ms_vcycle   : with options.profile 1 or 2, device time of the V-cycles
 *               (HIP events around each one); 0 otherwise.
 * ms_residual : the same for the refinement steps (update, residual and
 *               its norm).
 * fell_back_fp64: 1 if the stagnation guard switched a MG_PREC_MIXED solve
 *               to FP64 V-cycles (see mg_options.stall_factor). */
typedef struct {
    int32_t iters;
    double relres;
    double res_hist[MG_HIST];
    double ms_total;
    int32_t levels_used;
    double alg_bytes;
    double kern_ms[MG_NK];
    int64_t kern_launches[MG_NK];
    double kern_bytes[MG_NK];
    double kern_fine_ms[MG_NK];
    int64_t kern_fine_launches[MG_NK];
    double kern_fine_bytes[MG_NK];
    double ms_vcycle, ms_residual;
    int32_t fell_back_fp64;
} mg_stats;

typedef struct mg_handle mg_handle;

/* Fill *opts with defaults: levels 0 (auto), V(2,2), 40 coarse sweeps,
 * max_iters 100, omega 0.8, semi_threshold 2, MG_PREC_MIXED, default stream,
 * no profiling, smoothing interval [1/3, 2] (the eigenvalues of H_z^{-1} H
 * on the modes the smoother must damp when merged latitude rows carry
 * anisotropy up to semi_threshold = 2: from 1/(1 + 2) to 2), stagnation
 * guard 0.9 over 3 iterations, graphs on. */
void mg_options_default(mg_options* opts);

/* Build the hierarchy for grid and coefficients (Sections 2.1-2.3):
 * geometry tables and the conditional semi-coarsening map on the host in
 * FP64, then on the device the aggregated mass sum(alpha V) per level and
 * the column pivots. *out receives a new handle (NULL on failure).
 * Errors: MG_ERR_ARG for an invalid grid/options/NULL pointer (alpha values
 * are checked on the device: non-positive or non-finite -> MG_ERR_ARG),
 * MG_ERR_OOM, MG_ERR_HIP. */
mg_status mg_setup(const mg_grid* grid, const mg_coeffs* coeffs,
                   const mg_options* opts, mg_handle** out);

/* Replace alpha (same grid, no reallocation): recomputes masses, pivots and
 * the coarsest level's solve matrix. alpha is checked first: a value that
 * is not finite and > 0 gives MG_ERR_ARG and leaves the handle as it was. */
mg_status mg_update_coeffs(mg_handle* h, const mg_coeffs* coeffs);

/* Change the options of an existing handle; the hierarchy shape options
 * (levels, semi_threshold) must be unchanged. */
mg_status mg_set_options(mg_handle* h, const mg_options* opts);

/* Solve H u = rhs (Section 2) to ||rhs - H u||_2 <= tol ||rhs||_2.
 * u is in/out: the initial guess on entry, the solution on exit.
 * stats may be NULL. tol > 0. Returns MG_ERR_NOT_CONVERGED after max_iters
 * outer iterations, MG_ERR_BREAKDOWN on a non-finite residual. */
mg_status mg_solve(mg_handle* h, const double* rhs, double* u, double tol,
                   mg_stats* stats);

/* Adjoint solve H^T lambda = w with the transposed V-cycle inside the same
 * refinement loop (lambda in/out like u). For L = <w, u>, dL/drhs = lambda. */
mg_status mg_solve_adjoint(mg_handle* h, const double* w, double* lambda,
                           double tol, mg_stats* stats);

/* mg_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same solve, same arguments and results, but it allocates nothing.
 * It records no HIP events (stats->kern_* and ms_vcycle/ms_residual stay
 * 0; profiling options are ignored for the call), its norm partials go to
 * a device array of the library's own (one per GPU, kept until the process
 * ends; grids whose finest level has more than 8.4M columns are rejected
 * with MG_ERR_ARG), and it needs the work buffers of the handle's
 * precision, which mg_setup and mg_set_options allocate (MG_ERR_ARG if they
 * are missing). The stagnation guard switches to FP64 only if the FP64
 * buffers exist (after an FP64 solve on the handle). Calls that overlap on
 * one GPU race on that array: serialise them. */
mg_status mg_solve_noalloc(mg_handle* h, const double* rhs, double* u, double tol,
                           mg_stats* stats);

/* grad = -lambda * V * u elementwise (dL/dalpha for L = <w, u>). */
mg_status mg_grad_alpha(mg_handle* h, const double* lambda, const double* u,
                        double* grad);

/* y = H x in FP64 on the finest level (difference form). */
mg_status mg_apply(mg_handle* h, const double* x, double* y);

/* V[c] = volume of every fine cell (N values). */
mg_status mg_cell_volumes(mg_handle* h, double* V);

/* x = one V-cycle applied to f from zero (transposed = 1: the transposed
 * V-cycle), on the finest level, in the handle's precision (FP32 cycles
 * read and write FP64 here with a cast at the boundary). */
mg_status mg_vcycle(mg_handle* h, const double* f, double* x, int32_t transposed);

/* Per-level operations in the handle's precision, for inspection and tests.
 * Field arguments hold the level's nlon*nlat*nlev FP64 values.
 *   mg_level_shape : shape[3] = {nlon, nlat, nlev} of level l.
 *   mg_level_sweep : x_out = x_in + omega H_z^{-1}(f - H x_in) on level l
 *                    (x_in NULL: the sweep from zero, omega H_z^{-1} f).
 *   mg_level_residual_restrict : fc = R(f - H x), level l -> l+1.
 *   mg_level_prolong_add       : x += P xc, level l+1 -> l. */
mg_status mg_level_shape(const mg_handle* h, int32_t l, int32_t shape[3]);
mg_status mg_level_sweep(mg_handle* h, int32_t l, const double* f,
                         const double* x_in, double* x_out);
mg_status mg_level_residual_restrict(mg_handle* h, int32_t l, const double* f,
                                     const double* x, double* fc);
mg_status mg_level_prolong_add(mg_handle* h, int32_t l, const double* xc,
                               double* x);

/* Host-only planning (no GPU needed): the hierarchy the given grid and
 * options would produce.
 * levels_out       : number of levels;
 * nlon_out/nlat_out: per level (capacity MG_MAX_LEVELS);
 * child_first/child_count: for levels 1..levels-1, concatenated, the first
 *                    fine row and the number (1 or 2) of fine rows of every
 *                    coarse row; cap = capacity of each array (entries
 *                    needed: sum of nlat over levels 1..levels-1). */
mg_status mg_plan(const mg_grid* grid, const mg_options* opts,
                  int32_t* levels_out, int32_t* nlon_out, int32_t* nlat_out,
                  int32_t* child_first, int32_t* child_count, int32_t cap);

/* Host-only: the FP64 geometry tables of level l of that hierarchy.
 * V, Tlam: nlev*nlat_l values [k][J]; Tth: nlev*(nlat_l+1) [k][F], face F
 * south of row F; Tr: (nlev+1)*nlat_l [F][J], face F below layer F. */
mg_status mg_plan_tables(const mg_grid* grid, const mg_options* opts,
                         int32_t l, double* V, double* Tlam, double* Tth,
                         double* Tr);

void mg_destroy(mg_handle* h);
const char* mg_status_string(mg_status s);
const char* mg_last_error(const mg_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* MG_H */
