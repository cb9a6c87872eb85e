/*
 * stk.h — C ABI of the MI355X (gfx950) matrix-free velocity smoother library
 * for the 2D staggered-grid variable-viscosity Stokes equations.
 *
 * Source of the mathematics: Ferrari, Puentener, Sotoudeh, Viebig, "3D Blocking
 * for Matrix-free Smoothers in 2D Variable-Viscosity Stokes Equations"
 * (arXiv:2509.19061):
 *   Sec. 2.1  Cauchy-form Stokes equations and the staggered grid (Fig. 1),
 *   Sec. 3.1  saddle-point system, velocity subsystem M v + G p = f,
 *   Sec. 3.2  inexact Uzawa with a matrix-free geometric multigrid velocity
 *             solve whose smoothing dominates the cost,
 *   Sec. 4    loop fusion, spatial blocking, RAS-type temporal blocking (Alg. 2),
 *   Sec. 5    the five smoothers,
 *   Sec. 6.4  the energy residual norms.
 *
 * ---------------------------------------------------------------------------
 * Conventions shared by every call
 * ---------------------------------------------------------------------------
 * Grid: nx x ny cells of size dx x dy.  Cell (i,j), 0<=i<nx, 0<=j<ny, carries
 * eta_c (the paper's eta_P) and the pressure p; node (i,j), 0<=i<=nx,
 * 0<=j<=ny, carries eta_n (eta_B).  vx(i,j) sits on the left face of cell
 * (i,j) and vy(i,j) on its bottom face; fx lives with vx and fy with vy.
 *
 * Memory layout: every field is a row-major array with x fastest and ONE
 * common row stride `ld` (elements, >= nx+1); element (i,j) is at
 * base[j*ld + i].  Used extents (rows x columns):
 *     vx, fx : ny     x (nx+1)        vy, fy : (ny+1) x nx
 *     eta_c, p : ny   x nx            eta_n  : (ny+1) x (nx+1)
 * Nothing outside the used extents is read or written.  dtype STK_F64 means
 * every field is double, STK_F32 float.  All field pointers are DEVICE
 * pointers owned by the caller; the library never frees or retains them
 * beyond the call (an stk_mg copies what it keeps).
 *
 * Boundary conditions: free-slip walls.  The wall velocities vx(0,.),
 * vx(nx,.), vy(.,0), vy(.,ny) are Dirichlet 0: they are read as 0 whatever
 * they hold, and every call that writes a velocity writes 0 there.  The shear
 * stress vanishes at boundary nodes.
 *
 * Operator (A = -M is symmetric positive definite):
 *   txx = 2 eta_c (vx(i+1,j)-vx(i,j))/dx,  tyy = 2 eta_c (vy(i,j+1)-vy(i,j))/dy,
 *   txy = eta_n ((vx(i,j)-vx(i,j-1))/dy + (vy(i,j)-vy(i-1,j))/dx) at interior nodes,
 *   (Mv)_x = d(txx)/dx + d(txy)/dy,  (Mv)_y = d(txy)/dx + d(tyy)/dy (centred).
 *   Right-hand side for fixed pressure: b = f - G p, (Gp)_x = -(p(i,j)-p(i-1,j))/dx,
 *   (Gp)_y = -(p(i,j)-p(i,j-1))/dy; p == NULL means p = 0.
 *
 * Asynchrony: calls enqueue work on the context's HIP stream and return
 * without waiting, except where a host result is produced (noted per call).
 * Errors: every call returns an stk status; on error nothing has been
 * enqueued and no caller array has been modified; stk_last_error() gives a
 * thread-local message.  No exception crosses the ABI.
 */
#ifndef STK_H
#define STK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    STK_OK = 0,
    STK_EINVAL = -1,        /* invalid argument (message names it)                       */
    STK_ENOMEM = -2,        /* device allocation failed                                  */
    STK_EHIP = -3,          /* a HIP runtime call failed (message has the HIP error)     */
    STK_ENOTCONV = -4,      /* solve hit max_iters; results and the achieved residual are written */
    STK_ENONFINITE = -5,    /* a norm came out NaN/Inf (outputs are still written)       */
    STK_EUNSUPPORTED = -6   /* valid but not supported here (e.g. tile+halo beyond LDS)  */
};

typedef enum { STK_F64 = 0, STK_F32 = 1 } stk_dtype;

/* The smoothers of Sec. 5 (list (i)-(v)).  Blocked fused Jacobi is
 * STK_RAS_JACOBI with k = 1, halo = 0. */
typedef enum {
    STK_JACOBI = 0,        /* damped Jacobi, separate vx and vy passes (Sec. 5 (ii))            */
    STK_JACOBI_FUSED = 1,  /* damped Jacobi, vx and vy in one pass (Sec. 4.1, Sec. 5 (iii))     */
    STK_RAS_JACOBI = 2,    /* Jacobi with RAS-type temporal blocking (Sec. 4.3, Alg. 2, Sec. 5 (v)) */
    STK_RBGS = 3           /* red-black Gauss-Seidel (Sec. 5 (i))                                */
} stk_variant;

typedef struct {
    int nx, ny;     /* cells, each >= 2                                   */
    int64_t ld;     /* common row stride in elements, >= nx + 1           */
    double dx, dy;  /* cell size, > 0                                     */
} stk_grid;

/* Options of stk_smooth.  Fill with stk_smooth_opts_default(); a NULL
 * options pointer means the defaults. */
typedef struct {
    double omega;          /* damping, in (0, 2); 0 = variant default (0.7 Jacobi forms, 1.0 RBGS) */
    int tile_x, tile_y;    /* RAS owned tile in cells (default 64 x 64)                            */
    int halo;              /* RAS overlap h in cells, >= 0; -1 (default) = k                        */
    int k;                 /* RAS inner sweeps per outer iteration (T_inner of Alg. 2), default 4   */
    const int32_t* shifts; /* HOST array, 2 ints (sx, sy) per outer iteration, reduced mod the tile;
                              NULL (default) = drawn from `seed` (stk_ras_shifts)                    */
    uint64_t seed;         /* seed of the shift stream when shifts == NULL (default 0)              */
    int last_partial;      /* 1 (default): the last outer iteration runs only the remaining sweeps,
                              so exactly `sweeps` sweeps happen; 0: ceil(sweeps/k) full outer
                              iterations as Alg. 2 writes it                                         */
} stk_smooth_opts;

typedef struct stk_ctx stk_ctx;
typedef struct stk_mg stk_mg;

/* ------------------------------------------------------------ context -- */

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  The context owns scratch
 * (ping-pong velocity buffers, folded right-hand sides, reduction partials),
 * grown on demand and freed by stk_ctx_destroy.  Not thread-safe: one host
 * thread per context at a time. */
int stk_ctx_create(stk_ctx** out, int device, void* hip_stream);
int stk_ctx_destroy(stk_ctx* ctx);
int stk_ctx_set_stream(stk_ctx* ctx, void* hip_stream);
/* Block until the context's stream has drained. */
int stk_ctx_sync(stk_ctx* ctx);
/* Bytes of device scratch the context currently holds. */
int stk_ctx_scratch_bytes(const stk_ctx* ctx, size_t* bytes);
/* Thread-local message of the last failing call on this thread. */
const char* stk_last_error(void);

void stk_smooth_opts_default(stk_smooth_opts* o);

/* -------------------------------------------------------------- smooth -- */

/* `sweeps` smoothing sweeps of `variant` on M v = f - G p (Sec. 3.1), in
 * place on (vx, vy).  Jacobi forms: v <- v + omega (b - M v)/diag(M) from the
 * old iterate (split and fused give the same values).  RBGS: the sets vx-red,
 * vx-black, vy-red, vy-black (colour (i+j) mod 2, red = 0) relaxed in that
 * order.  RAS (Alg. 2 with snapshot semantics): per outer iteration the tile
 * grid is cut at positions congruent to the shift modulo the tile size (edge
 * tiles partial); every tile copies the current field on its tile grown by
 * `halo` cells (clipped to the domain) plus a one-cell frozen ring, runs k
 * Jacobi sweeps there, and writes back its owned cells only; all tiles read
 * the same snapshot, so the result is deterministic.  With halo >= k-1 this
 * equals k Jacobi sweeps exactly.  sweeps = 0 is a no-op.  Asynchronous.
 * Errors: STK_EINVAL (bad sizes/pointers/options), STK_EUNSUPPORTED (RAS
 * tile plus halo exceeding the LDS budget), STK_ENOMEM, STK_EHIP. */
int stk_smooth(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, void* vx, void* vy, const void* p,
               const void* eta_c, const void* eta_n, const void* fx, const void* fy, int sweeps,
               stk_variant variant, const stk_smooth_opts* opts);

/* Shift stream of RAS outer iterations: for t = 0..n_outer-1, sx = (z >> 32)
 * mod tile_x and sy = (z' >> 32) mod tile_y where z, z' are consecutive
 * SplitMix64 outputs from `seed` (Steele, Lea & Flood 2014).  Alg. 2 draws a
 * random shift per outer iteration.  `out` is a host array of 2*n_outer. */
int stk_ras_shifts(uint64_t seed, int n_outer, int tile_x, int tile_y, int32_t* out);

/* One RAS outer iteration (Alg. 2, snapshot form) out of place, with an
 * explicit shift: (ox, oy) <- kt Jacobi sweeps per tile as in stk_smooth,
 * with b = (bx, by) the already-folded right-hand side (b = f - G p, 0 on
 * walls; pass fx, fy when p = 0).  Every velocity entry of (ox, oy) in the
 * used extents is written (walls 0); (vx, vy) are not modified.  Outputs
 * must not alias inputs.  kt = 0 copies.  For callers that manage their own
 * ping-pong buffers.  Asynchronous; errors as stk_smooth. */
int stk_ras_outer(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const void* vx, const void* vy, const void* eta_c,
                  const void* eta_n, const void* bx, const void* by, void* ox, void* oy, double omega, int tile_x,
                  int tile_y, int halo, int kt, int sx, int sy);

/* ------------------------------------------------------------ residual -- */

/* rx, ry <- r_v = b - M v on the unknowns (0 on walls); rp (nullable) <-
 * r_p = -D v per cell, (Dv) = (vx(i+1,j)-vx(i,j))/dx + (vy(i,j+1)-vy(i,j))/dy
 * (Sec. 6.4).  With fx = fy = 0 and p = NULL this is -M v.  Output arrays use
 * the same layout and dtype as the inputs and must not alias them.
 * Asynchronous. */
int stk_residual(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const void* vx, const void* vy, const void* p,
                 const void* eta_c, const void* eta_n, const void* fx, const void* fy, void* rx, void* ry,
                 void* rp);

/* Energy residual norms of Sec. 6.4, accumulated in FP64 for both dtypes:
 *   out[0] N_v = sum over unknowns r_v^2 / diag(-M)
 *   out[1] N_p = sum over cells r_p^2 eta_c / (2/dx^2 + 2/dy^2)
 *   out[2] N_f = sum over unknowns f^2 / diag(-M)
 *   out[3] E   = sqrt((N_v + N_p) / N_f)     (global relative energy residual)
 *   out[4] E_v = sqrt(N_v / N_f)             (velocity part)
 * `out` is a HOST array of 5 doubles.  The reduction order is fixed (bitwise
 * reproducible run to run).  Synchronises the context's stream.
 * STK_ENONFINITE if any value is NaN/Inf (e.g. N_f = 0); out is still written. */
int stk_energy_norm(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const void* vx, const void* vy,
                    const void* p, const void* eta_c, const void* eta_n, const void* fx, const void* fy,
                    double out[5]);

/* The energy norms of stk_energy_norm for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): `out` is a DEVICE array of 5 doubles that receives
 * {N_v, N_p, N_f, E, E_v} (E and E_v computed on the device); the call
 * enqueues the work and returns without waiting.  The per-wave partial sums
 * live in a fixed 8 MiB array of the library on each GPU (held until the
 * process ends), not in the context's scratch: nothing is allocated and the
 * context's scratch is not touched.  N_v, N_p, N_f are bitwise those of
 * stk_energy_norm.  Every call on one GPU shares that array, so calls that
 * may overlap on one GPU (other streams, other host threads) race: order them
 * on one stream.  Nothing needs to start at zero (every partial is written
 * before it is read).  Grids needing more than 349525 partial triples
 * (ceil((nx+1)/62) * ceil((ny+1)/64); about 37000 x 37000 cells) return
 * STK_EUNSUPPORTED.  Non-finite results are not reported (there is no host
 * result to check).  Other errors as stk_energy_norm. */
int stk_energy_norm_noalloc(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const void* vx, const void* vy,
                            const void* p, const void* eta_c, const void* eta_n, const void* fx, const void* fy,
                            double* out);

/* ---------------------------------------------------------- measurement -- */

/* A plain streaming pass with the traffic of one RAS outer iteration (Sec.
 * 4.3: six planes read, two written), the practical HBM ceiling the smoother
 * kernels are measured against and the calibration kernel of the HBM byte
 * counters: o0 = a0 + a2 * a4 and o1 = a1 + a3 * a5 elementwise over all
 * (ny + 1) * ld elements of each plane (DEVICE arrays of that many elements,
 * dtype dt; outputs must not alias inputs).  Bytes moved: 8 (ny + 1) ld w.
 * Asynchronous. */
int stk_stream_probe(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const void* a0, const void* a1, const void* a2,
                     const void* a3, const void* a4, const void* a5, void* o0, void* o1);

/* ----------------------------------------------------------- multigrid -- */

/* Geometric multigrid for the velocity block (Sec. 3.2: the velocity update
 * of the inexact Uzawa scheme is solved approximately with a matrix-free
 * geometric multigrid whose smoothing dominates the cost; Sec. 6.2 runs one
 * V-cycle per Uzawa cycle).  The paper gives no transfer operators; this
 * library coarsens by 2 in x and y while min(nx, ny) > coarsest and both are
 * even, prolongs bilinearly per component (linear across faces, 3/4-1/4 along
 * them, mirrored at the free-slip walls), restricts with R = P^T / 4, uses
 * Galerkin coarse operators M_c = R M P (a row has 31 couplings; M_c is
 * symmetric and each coupling is stored once, 32 * (ny_c+1) * ld_c words per
 * coarse level; the finest level is matrix-free), smooths with damped Jacobi
 * (on the finest level each smoothing stage is one RAS-Jacobi outer
 * iteration with 64 x 64 tiles and halo = k = the sweep count, bit-identical
 * to that many Jacobi sweeps) and solves the coarsest level exactly in FP64
 * (dense inverse of -M_c built at setup). */
typedef struct {
    int nu1, nu2;      /* pre / post smoothing sweeps per level (default 2, 2)                 */
    double omega;      /* Jacobi damping (default 0.7)                                          */
    int coarsest;      /* stop coarsening at min(nx, ny) <= coarsest (default 8).  The coarsest
                          level is solved exactly, and at high viscosity contrast a larger one
                          converges in far fewer iterations (2048^2, contrast 1e8: 925 FCG
                          iterations at 8, 286 at 32) for a larger inverse: 32 gives 1984
                          unknowns, 31 MB and about 0.1 s of host setup (host threads: the
                          affinity mask, at most OMP_NUM_THREADS)                            */
    /* Smoother variants of the paper's solver (Sec. 6.2, 6.3).  The defaults
     * give the cycle described above. */
    int fine_k;        /* finest level: RAS inner sweeps per outer iteration (64 x 64 tiles, shift
                          0); a smoothing stage of nu sweeps is ceil(nu / fine_k) outer
                          iterations, the last one partial; 0 (default) = nu (one outer iteration) */
    int fine_halo;     /* finest-level RAS overlap in cells; -1 (default) = the outer iteration's
                          sweep count, which makes it exactly that many Jacobi sweeps; 0 is the
                          paper's thin overlap                                                   */
    int coarse_smoother; /* 0 (default): damped Jacobi on the coarse (Galerkin) levels; 1: RAS on
                          them, the paper's mixed smoother (Jacobi finest, RAS coarse)           */
    int coarse_tile;   /* coarse RAS tile in cells (default 32, the paper's)                       */
    int coarse_k;      /* coarse RAS inner sweeps per outer iteration (default 4, the paper's)     */
    int coarse_halo;   /* coarse RAS overlap in cells (default 0, the paper's thin overlap)        */
    double sweep_growth; /* level l takes floor(nu * sweep_growth^l + 1/2) pre- and post-sweeps
                          (default 1; the paper grows them by 2.5 per level)                     */
    int max_levels;    /* 0 (default): coarsen down to `coarsest` and solve there exactly; L >= 2:
                          at most L levels, and when that stops the coarsening early the last
                          level is relaxed by its pre- plus post-sweeps instead of solved (the
                          paper runs four levels)                                                 */
    int stall_checks;  /* 0 (default): a solve runs to tol or max_iters.  N >= 1: a solve also
                          stops, not converged, after N consecutive true-residual checks that
                          each fail to halve N_v against the check before (the recurrence
                          residual reached tol, the true one did not, and restarts no longer
                          gain): E_v is then at its FP64 floor, set by the rounding of the
                          solution itself                                                        */
} stk_mg_opts;

/* Both modes run the same FP64 outer iteration: flexible conjugate gradients
 * with FP64 residual, operator, dot products and energy norms; each iteration
 * refines the FP64 iterate by a preconditioned correction.  They differ in the
 * precision of the preconditioner, one V-cycle per iteration: */
typedef enum {
    STK_SOLVE_F64 = 0,         /* FP64 V-cycle                                                          */
    STK_SOLVE_F32_REFINED = 1  /* FP32 V-cycle (smoothing, transfers, coarse stencils in FP32; the
                                  coarsest solve accumulates in FP64), applied to the FP64 residual
                                  rounded to FP32; the FP64 Krylov steps read its FP32 result       */
} stk_solve_mode;

typedef struct {
    int iterations;        /* Krylov iterations (= V-cycles applied) of this instance              */
    int converged;         /* final true E_v <= tol                                                 */
    double ev;             /* final E_v = sqrt(N_v / N_f) from a freshly computed FP64 residual     */
    double nf;             /* N_f = sum f^2 / diag(-M)                                              */
    double seconds;        /* host wall time of the call                                            */
} stk_report;

void stk_mg_opts_default(stk_mg_opts* o);

/* Build the hierarchy for grid g from DEVICE FP64 viscosities in g's layout.
 * The handle copies what it keeps and owns every level buffer until
 * stk_mg_destroy.  STK_EUNSUPPORTED if the coarsest level would exceed 4096
 * unknowns (choose nx, ny divisible by a power of two).  Synchronises. */
int stk_mg_create(stk_ctx* ctx, stk_mg** out, const stk_grid* g, const double* eta_c, const double* eta_n,
                  const stk_mg_opts* opts);
int stk_mg_destroy(stk_mg* mg);
/* Move a hierarchy to another context on the same device, e.g. one built by
 * a setup thread on its own stream and then solved in a batch on the serving
 * stream: the device buffers that solves in `mode` need are created first
 * (on the old context's stream), that stream is drained, and from then on
 * the handle enqueues on `ctx`.  STK_EINVAL if the handle is in a batch or
 * the devices differ.  Synchronises the old context's stream. */
int stk_mg_bind(stk_mg* mg, stk_ctx* ctx, int mode);
/* Levels, coarsest-grid unknowns and device bytes currently held. */
int stk_mg_info(const stk_mg* mg, int* levels, int* coarse_unknowns, size_t* bytes);
/* Device bytes a hierarchy for g needs when solving in `mode` (0 F64, 1 F32_REFINED),
 * including the solver's vectors: the admission figure of a serving loop. */
int stk_mg_footprint(const stk_grid* g, const stk_mg_opts* opts, int mode, size_t* bytes);

/* One V(nu1, nu2)-cycle for M v = b on the finest level, in place on (vx, vy);
 * device arrays in the layout of the grid given at creation, dtype dt (FP32
 * uses FP32 copies of the viscosities and coarse stencils; the coarsest solve
 * is FP64).
 * Asynchronous. */
int stk_mg_vcycle(stk_mg* mg, stk_dtype dt, void* vx, void* vy, const void* bx, const void* by);

/* Solve M v = f - G p to the velocity energy residual E_v = sqrt(N_v / N_f)
 * <= tol (Sec. 6.4), starting from (vx, vy) (device FP64, in/out).  p may be
 * NULL.  At most max_iters Krylov iterations.  When the recurrence residual
 * reaches tol the true FP64 residual is recomputed, and the iteration restarts
 * from the current iterate if it is still above tol.  STK_ENOTCONV if the
 * final E_v > tol (the iterate and the report are still written).
 * Synchronises. */
int stk_mg_solve(stk_mg* mg, stk_solve_mode mode, double* vx, double* vy, const double* p, const double* fx,
                 const double* fy, double tol, int max_iters, stk_report* rep);

/* The same for n independent instances (distinct handles on one context,
 * equal nu1, nu2, omega): every level kernel is ONE launch across all
 * instances (work-list of (instance, block)); instances stop individually;
 * one host synchronisation per iteration reads all convergence flags.  Arrays
 * of n pointers; p may be NULL or hold NULL entries; reps may be NULL.  Each
 * instance's arithmetic is independent of the others: its result is the same
 * bit for bit alone and in any mix. */
int stk_mg_solve_batch(stk_ctx* ctx, int n, stk_mg* const* mgs, stk_solve_mode mode, double* const* vx,
                       double* const* vy, const double* const* p, const double* const* fx, const double* const* fy,
                       double tol, int max_iters, stk_report* reps);

/* ------------------------------------------------ continuous batching -- */

/* A batch of in-flight solves that instances join and leave at any time
 * (the engine of stk_mg_solve_batch and of a serving loop).  Each step
 * advances every in-flight solve together, one launch per (level, kernel)
 * across all of them, and hands back the solves that finished.  Results are
 * those of stk_mg_solve, bit for bit, whatever else shares the batch.  A batch
 * is used from one host thread; its handles must not be destroyed while they
 * are in it. */
typedef struct stk_batch stk_batch;

int stk_batch_create(stk_ctx* ctx, stk_solve_mode mode, int max_slots, stk_batch** out);
/* Abandons solves still in flight (their handles become free again). */
int stk_batch_destroy(stk_batch* b);
/* Admit a solve of M v = f - G p (arguments as for stk_mg_solve, device FP64,
 * caller-owned; vx, vy are read now and written when the solve finishes, p,
 * fx, fy are read now).  *slot receives its slot id.  STK_EINVAL if no slot is
 * free, the handle is already in a batch, or its nu1, nu2, omega differ from
 * the batch's.  Asynchronous except for pressure staging. */
int stk_batch_add(stk_batch* b, stk_mg* mg, double* vx, double* vy, const double* p, const double* fx,
                  const double* fy, double tol, int max_iters, int* slot);
/* Advance every in-flight solve by up to `iters` Krylov iterations.  On
 * return done[0..*ndone) are the slots whose solves finished during the step
 * (converged, or out of iterations: see reps[k].converged; seconds = time
 * since admission), their solutions already in the caller's arrays, and those
 * slots are free again.  done and reps need room for max_slots entries. */
int stk_batch_step(stk_batch* b, int iters, int* done, stk_report* reps, int* ndone);
/* Number of solves in flight. */
int stk_batch_count(const stk_batch* b, int* in_flight);

/* --------------------------------------------------- inexact Uzawa -- */

/* The full Stokes system M v + G p = f, D v = 0 (Sec. 3.1) by the inexact
 * Uzawa iteration (Sec. 3.2): each cycle updates the velocity for the current
 * pressure approximately with V-cycles, then takes a Richardson step on the
 * pressure Schur complement with the cell viscosity as its approximate inverse,
 *   p <- p + omega_p eta_c r_p,   r_p = -D v,
 * and removes the pressure's domain mean (Sec. 6.2: the pressure is defined up
 * to a constant).  With this library's G (b = f - G p, G p = -grad p) the
 * Schur complement of -M is positive and this is the convergent sign; the
 * paper prints the same step with the sign carried by its D.  All arrays are
 * DEVICE FP64 in the grid's layout (p: ny rows of nx cells, stride ld). */
typedef struct {
    double omega_p;   /* pressure relaxation, > 0 (default 0.6, Sec. 6.3)                      */
    int vcycles;      /* V-cycles of the velocity update per Uzawa cycle, >= 1 (default 1, Sec. 6.2) */
    double tol;       /* stop when the global energy residual E (Sec. 6.4, with N_p) <= tol
                         (default 1e-8)                                                           */
    int max_cycles;   /* at most this many Uzawa cycles, continuation stages included (default 1000) */
    int stages;       /* viscosity continuation (Sec. 6.2): stages s = 0 .. stages-1 run on
                         (1 - theta) eta_min + theta eta with theta = s / stages (cell and nodal
                         fields, eta_min = the smallest cell viscosity), each with a hierarchy of
                         its own built for the call, before the true system (theta = 1, `mg`);
                         0 (default) = none; the paper runs 4                                   */
    int stage_cycles; /* Uzawa cycles per stage with theta < 1 (default 25, Sec. 6.2)             */
    int mode;         /* velocity update precision (stk_solve_mode; default STK_SOLVE_F64): with
                         STK_SOLVE_F32_REFINED each V-cycle runs in FP32 on the FP64 residual
                         f - G p - M v rounded to FP32, from zero, and its result is added to
                         the FP64 velocity (the V-cycle is consistent, so this is the FP64 cycle
                         up to FP32 rounding); pressure step and norms stay FP64           */
} stk_uzawa_opts;

typedef struct {
    int cycles;       /* Uzawa cycles run                                                          */
    int converged;    /* final E <= tol                                                            */
    double e;         /* final E = sqrt((N_v + N_p) / N_f)                                         */
    double ev;        /* final E_v = sqrt(N_v / N_f)                                               */
    double seconds;   /* host wall time of the call                                                */
} stk_uzawa_report;

void stk_uzawa_opts_default(stk_uzawa_opts* o);

/* Lithostatic pressure (Sec. 6.2's initial pressure): p balances the vertical
 * body force on every interior vy face, (p(i,j-1) - p(i,j)) / dy = fy(i,j),
 * integrated from the top row down, then shifted to zero mean.  fy has the vy
 * layout (ny + 1 rows).  Asynchronous. */
int stk_litho_pressure(stk_ctx* ctx, const stk_grid* g, const double* fy, double* p);

/* One pressure update of the Uzawa cycle, in place on p:
 * p <- p + omega_p eta_c r_p(v), then p <- p - mean(p).  omega_p > 0.
 * The mean is reduced in a fixed order (bitwise reproducible).  Asynchronous. */
int stk_uzawa_pressure(stk_ctx* ctx, const stk_grid* g, const double* vx, const double* vy, const double* eta_c,
                       double omega_p, double* p);

/* Uzawa cycles from (vx, vy, p), all in/out, until E <= tol or max_cycles:
 *   b = f - G p;  `vcycles` FP64 V(nu1, nu2)-cycles of `mg` on M v = b from v;
 *   stk_uzawa_pressure;  E from a fresh FP64 residual (both blocks).
 * With opts->stages > 0 the continuation stages come first (their cycles use
 * the stage's hierarchy and its eta_c in the pressure step; E and the history
 * always measure the true system, and only the last stage tests tol).
 * g must be the grid `mg` was created for (same nx, ny, ld) and eta_c, eta_n
 * the viscosities it was built from.  hist (nullable, HOST, max_cycles + 1
 * doubles) receives E of the start and after every cycle; rep (nullable) the
 * summary.  opts NULL means the defaults.  STK_ENOTCONV if E > tol at the end
 * (arrays, hist and rep are still written); the handle must not be in a
 * batch.  With continuation it allocates, for the call's duration, the stage
 * viscosities and hierarchies (stk_mg_footprint(g, .., 0) bytes each).  With
 * mode STK_SOLVE_F32_REFINED the V-cycles run in FP32 on the FP64 residual
 * rounded to FP32 (in the handle's FP32 vectors, no further device memory)
 * and their results are added to the FP64 velocity.
 * Synchronises once per cycle (the stopping test). */
int stk_uzawa_solve(stk_mg* mg, const stk_grid* g, double* vx, double* vy, double* p, const double* eta_c,
                    const double* eta_n, const double* fx, const double* fy, const stk_uzawa_opts* opts,
                    double* hist, stk_uzawa_report* rep);

/* Anderson acceleration of the Uzawa cycles (Sec. 3.3, Alg. 1) on
 * x = [v, p], from (vx, vy, p), all in/out.  F(x) is one Uzawa cycle as in
 * stk_uzawa_solve (fold, opts->vcycles V-cycles of `mg`, pressure step).
 * x_1 = F(x_0); then, with m_k = min(depth, k) and r_i = F(x_i) - x_i,
 *   x_{k+1} = sum_t alpha_t F(x_{k-m_k+t}),
 *   alpha = argmin || sum_t alpha_t r_{k-m_k+t} ||_2  with  sum_t alpha_t = 1,
 * the l2 norm running over every velocity unknown and pressure cell.  The
 * weights solve the bordered Gram system of that constrained least-squares
 * problem on the host (a singular system takes the plain step alpha =
 * (0, .., 0, 1)); depth 0 is the plain iteration.  Stops when E of x_{k+1}
 * (Sec. 6.4) <= opts->tol or after opts->max_cycles evaluations of F.
 * depth in [0, 8].  opts->mode selects FP64 or FP32 V-cycles and
 * opts->stages the viscosity continuation, as in stk_uzawa_solve: each stage
 * runs its own Anderson steps (the history restarts with the stage, whose
 * map F differs), and max_cycles bounds the steps of all stages together.
 * hist (nullable, HOST, max_cycles + 1 doubles): E of x_0, x_1, ..;
 * rep->cycles counts F evaluations.  Allocates 6 (depth + 1) planes of
 * (ny + 1) * ld doubles and 9 doubles per 256 plane elements (the products'
 * partial sums) for the call's duration.  The l2 norm and the combination
 * take no wall value: walls are read as 0 and written as 0.  Synchronises once per
 * step.  STK_ENOTCONV as stk_uzawa_solve. */
int stk_uzawa_anderson(stk_mg* mg, const stk_grid* g, double* vx, double* vy, double* p, const double* eta_c,
                       const double* eta_n, const double* fx, const double* fy, int depth,
                       const stk_uzawa_opts* opts, double* hist, stk_uzawa_report* rep);

/* ----------------------------------------------------------------- 3D -- */

/* The 3D extension (the paper's future work, Sec. 9): the staggered
 * variable-viscosity operator in three dimensions, smoothed by damped Jacobi
 * or by RAS-type temporal blocking of 3D tiles (Alg. 2 with snapshot
 * semantics on T x T x T tiles: three space dimensions and the inner
 * sweeps).  The paper gives only the 2D formulas; these follow them axis by
 * axis:
 *   cells (i,j,k) carry eta_c; vx(i,j,k) is the x-face at (i dx, (j+1/2) dy,
 *   (k+1/2) dz), an unknown iff 1 <= i <= nx-1; vy, vz likewise along y, z;
 *   the wall values are 0.  eta_xy lives on the z-parallel edges
 *   (i dx, j dy, (k+1/2) dz), eta_xz on the y-parallel edges (i dx, (j+1/2) dy,
 *   k dz), eta_yz on the x-parallel edges ((i+1/2) dx, j dy, k dz); shear
 *   stresses vanish on boundary edges (free slip).
 *   t_xx = 2 eta_c dvx/dx per cell (yy, zz alike); t_xy = eta_xy (dvx/dy +
 *   dvy/dx) per interior z-parallel edge (xz, yz alike); (Mv)_x = dt_xx/dx +
 *   dt_xy/dy + dt_xz/dz at the x-faces (y, z alike).
 * Layout: every field is plane-major with one row stride ld and one plane
 * stride lp (elements): element (i,j,k) at base[k*lp + j*ld + i].  Used
 * extents (planes x rows x columns): vx nz x ny x (nx+1), vy nz x (ny+1) x nx,
 * vz (nz+1) x ny x nx, eta_c nz x ny x nx, eta_xy nz x (ny+1) x (nx+1),
 * eta_xz (nz+1) x ny x (nx+1), eta_yz (nz+1) x (ny+1) x nx.  All arrays are
 * caller-owned DEVICE arrays of (nz+1) * lp elements of dtype dt.  The
 * right-hand side b = (bx, by, bz) has the velocity layout (0 on walls). */
typedef struct {
    int nx, ny, nz;     /* cells, each >= 2 (nz + 1 <= 65535)                 */
    int64_t ld, lp;     /* row stride >= nx + 1; plane stride >= (ny + 1) ld  */
    double dx, dy, dz;  /* cell size, > 0                                     */
} stk_grid3;

typedef struct {
    double omega;          /* damping in (0, 2) (default 0.7)                                    */
    int tile;              /* RAS tile edge T in cells (default 8)                               */
    int halo;              /* RAS overlap h >= 0; -1 (default) = k, which is Jacobi^k exactly    */
    int k;                 /* RAS inner sweeps per outer iteration (default 2)                   */
    const int32_t* shifts; /* HOST, 3 ints (x, y, z) per outer iteration; NULL: SplitMix64(seed),
                              (z >> 32) mod T drawn x, y, z per outer iteration                  */
    uint64_t seed;
} stk_smooth3d_opts;

void stk_smooth3d_opts_default(stk_smooth3d_opts* o);

/* `sweeps` sweeps of damped Jacobi (STK_JACOBI_FUSED) or RAS-Jacobi
 * (STK_RAS_JACOBI, the last outer iteration partial) on M v = b, in place.
 * The RAS workgroup stages its tile grown by h plus a one-cell frozen ring in
 * LDS (3 components, 2 buffers: 6 (T + 2h + 2)^3 words): STK_EUNSUPPORTED
 * when that exceeds a workgroup's LDS.  Uses 6 fields of context scratch.
 * Asynchronous. */
int stk_smooth3d(stk_ctx* ctx, stk_dtype dt, const stk_grid3* g, void* vx, void* vy, void* vz, const void* eta_c,
                 const void* eta_xy, const void* eta_xz, const void* eta_yz, const void* bx, const void* by,
                 const void* bz, int sweeps, stk_variant variant, const stk_smooth3d_opts* opts);
/* One 3D RAS outer iteration out of place with explicit shifts (outputs must
 * not alias inputs; every velocity entry of the used extents is written, 0 on
 * walls).  Asynchronous. */
int stk_ras_outer3d(stk_ctx* ctx, stk_dtype dt, const stk_grid3* g, const void* vx, const void* vy, const void* vz,
                    const void* eta_c, const void* eta_xy, const void* eta_xz, const void* eta_yz, const void* bx,
                    const void* by, const void* bz, void* ox, void* oy, void* oz, double omega, int tile, int halo,
                    int kt, int sx, int sy, int sz);
/* r = b - M v on the unknowns, 0 on the walls.  Asynchronous. */
int stk_residual3d(stk_ctx* ctx, stk_dtype dt, const stk_grid3* g, const void* vx, const void* vy, const void* vz,
                   const void* eta_c, const void* eta_xy, const void* eta_xz, const void* eta_yz, const void* bx,
                   const void* by, const void* bz, void* rx, void* ry, void* rz);
/* Velocity energy norms (Sec. 6.4) with b = f: out = {N_v = sum r^2/d,
 * N_f = sum f^2/d, E_v = sqrt(N_v/N_f)}, FP64 sums in a fixed order.  HOST
 * out; synchronises. */
int stk_energy_norm3d(stk_ctx* ctx, stk_dtype dt, const stk_grid3* g, const void* vx, const void* vy, const void* vz,
                      const void* eta_c, const void* eta_xy, const void* eta_xz, const void* eta_yz, const void* fx,
                      const void* fy, const void* fz, double out[3]);

#ifdef __cplusplus
}
#endif

#endif /* STK_H */
