// Internal types of the multigrid / Krylov layer (host and device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "stk_internal.hpp"

namespace stk {

// One instance at one level of its hierarchy, everything a level kernel
// touches.  The transfer kernels also read the next-coarser level (c*).
template <typename T>
struct LevelJob {
    int nx, ny;
    int64_t ld;
    T idx, idy;
    gptr<const T> ec;
    gptr<const T> en;
    gptr<T> vx, vy;  // level iterate
    gptr<T> wx, wy;  // ping-pong partner of the smoother
    gptr<T> bx, by;  // right-hand side
    gptr<T> rx, ry;  // residual scratch
    int cnx, cny;
    int64_t cld;
    gptr<T> cbx, cby;  // coarse right-hand side
    gptr<T> cvx, cvy;  // coarse iterate
    gptr<const T> st;  // stored Galerkin stencil (coarse levels), nullptr on the finest
    int64_t plane;     // elements per stencil plane
    // the restriction also takes the coarse level's first smoothing sweep from 0
    // (damped Jacobi, written to cw*) when `first`; cst / cplane: its stencil
    int first;
    gptr<const T> cst;
    int64_t cplane;
    gptr<T> cwx, cwy;
};

// Coarsest level of one instance: n unknowns, map[q] = (component << 30) |
// (j * ld + i), dense row-major inverse of -M.
template <typename T>
struct CoarseJob {
    int n;
    gptr<const int> map;
    gptr<const double> ainv;
    gptr<const T> bx, by;
    gptr<T> vx, vy;
};

// Krylov vectors of one instance on its finest level (FP64): X, R, Z, P, Q =
// iterate / residual b - M x / preconditioned residual / direction / A p;
// F = force (for N_f), B = folded right-hand side f - G p.  The FP32 V-cycle
// of the mixed-precision mode uses FP32 R and Z slots of its own.
enum { VS_X = 0, VS_R, VS_Z, VS_P, VS_Q, VS_F, VS_B, VS_N };
struct VecJob {
    int nx, ny;
    int64_t ld;
    double idx, idy;
    gptr<const double> ec;  // FP64 viscosities for the diag(-M) energy weights
    gptr<const double> en;
    gptr<void> v[VS_N][2];  // slot -> (x component, y component)
};

// Per-instance scalars of flexible CG (device resident).
struct FcgState {
    double gamma;   // rho . z of the last preconditioned residual
    double alpha;   // step
    double beta;    // direction update
    double pq;      // p . A p
    double rz;      // rho . z
    double zq;      // z . q
    double nv;      // sum r^2 / d  (current residual, velocity energy)
    double nf;      // sum f^2 / d
    double thr;     // stop when nv <= thr
    double tol2;    // tol^2 of this instance (thr = tol2 * nf)
    int active;     // 1 while this instance iterates
    int left;       // iterations left in its budget (PH_NV stops the instance at 0)
};

// ---- launchers (mg_kernels.hip) ----------------------------------------------
struct Batch {       // a job array resident on the device plus its block prefix
    const void* jobs = nullptr;
    const int* pre = nullptr;
    int n = 0;       // instances
    int blocks = 0;  // total blocks
    // reductions over the blocks (vector batches only): per-instance chunks of
    // at most SUM_CHUNK block partials, chunk prefix cpre[0..n]
    const int* cpre = nullptr;
    // finest (matrix-free) level: workgroup prefix of the row-streaming kernels
    // (rowstream.hpp); when set, smoothing and residual use them
    const int* rpre = nullptr;
    int rblocks = 0;
};
constexpr int SUM_CHUNK = 4096;

template <typename T> int mg_jacobi(stk_ctx* ctx, const Batch& b, double omega, int dir);
template <typename T> int mg_residual(stk_ctx* ctx, const Batch& b);
// coarse right-hand side = R r, and the coarse iterate set to 0, or, for jobs
// with `first`, the coarse level's first Jacobi sweep from 0 (damping omega)
// written to its w
template <typename T> int mg_restrict(stk_ctx* ctx, const Batch& b_coarse_blocks, double omega);
template <typename T> int mg_prolong(stk_ctx* ctx, const Batch& b);
// Stored-stencil levels: v + P e_c, then one Jacobi sweep of it into w, in one
// pass (v itself is left as it was)
template <typename T> int mg_jacobi_prolonged(stk_ctx* ctx, const Batch& b, double omega);
template <typename T> int mg_coarse(stk_ctx* ctx, const void* jobs, int n, int max_unknowns);

// Galerkin setup of one coarse level from the next finer one (galerkin.hip).
// fst == nullptr: the finer level is the finest and its rows come from the
// viscosities ec, en; otherwise from its stored stencil fst.
struct GalerkinArgs {
    int nx, ny;          // finer level
    int64_t ld;
    double idx, idy;
    const double* ec;
    const double* en;
    const double* fst;
    int64_t fplane;
    int NX, NY;          // coarse level
    int64_t cld;
    double* cst;
    int64_t cplane;
};
int mg_galerkin(stk_ctx* ctx, const GalerkinArgs& g);

// (q = A p and p.q are one fused pass: fcg_apply_pq)
enum VecOp {
    OP_UPDATE = 0,  // x += alpha p; r += alpha q; acc0 += r^2/d; z = 0 (an FP64 Z slot)
    OP_RZ_ZQ,       // acc0 += r.z ; acc1 += z.q  (rho = -r: gamma = -acc0)
    OP_XPBY,        // p = z + beta p
    OP_FNORM,       // acc0 += f^2/d
    OP_INIT_P,      // p = z; acc0 += r.z
    OP_ZERO_Z       // z = 0
};
// phases of the scalar update: PH_NF sets N_f and the stop threshold
// tol2 * N_f, PH_NV ends a CG iteration (stop below the threshold or when the
// budget runs out), PH_TRUE takes a recomputed true residual (stop below the
// threshold only)
enum { PH_NF = 0, PH_NV, PH_INIT, PH_ALPHA, PH_BETA, PH_TRUE };
// Slot dtype T for the slots touched (R, Z, P, Q, X); partial sums land in
// `part` (2 per block), summed per instance by fcg_reduce.  z32: the batch's Z
// slot holds FP32 vectors (the FP32 V-cycle's output, read in place by the
// FP64 Krylov operations).
template <typename T>
int vec_op(stk_ctx* ctx, const Batch& b, int op, const FcgState* st, double* part, bool z32 = false);
// R = B - M X in FP64, block partials of sum R^2 / d in `part`
int vec_residual64_st(stk_ctx* ctx, const Batch& b, const FcgState* st, double* part);
// Per-instance sums of the block partials over the reduction chunks of `red`
// (fixed order) into sums (2 per instance) and the scalar update of `phase`,
// in one launch; out != nullptr (device-visible pinned host memory): the
// updated states are also copied there.
int fcg_reduce(stk_ctx* ctx, const Batch& red, const double* part, double* sums, FcgState* st, int phase,
               FcgState* out = nullptr);

// Entry of the FP32 V-cycle preconditioner (active instances): r32 = (float)
// r64 and z32 = 0 (its initial guess) in one pass.  Its output z32 is read in
// place by the FP64 Krylov operations.
struct XCastJob {
    int nx, ny;
    int64_t ld;
    gptr<const double> r64[2];
    gptr<float> r32[2];
    gptr<float> z32[2];
};
int prec_cast(stk_ctx* ctx, const Batch& b, const FcgState* st);
// FP64 FCG, finest level: Q = A P and the block partials of P . Q (apply: the
// operator batch with its row-streaming prefix; summed over its reduction
// chunks by fcg_reduce)
int fcg_apply_pq(stk_ctx* ctx, const Batch& apply, const FcgState* st, double* part);
template <typename T> int mg_copy_wv(stk_ctx* ctx, const Batch& b);
// Coarse-level RAS outer iteration (mg_ras.hip): kt sweeps per tile of the
// stored stencil, tiles `tile` cells cut at multiples of it, overlap h; b's
// prefix counts tiles (mg_ras_tiles per instance); dir 0 v -> w, 1 w -> v.
template <typename T> int mg_ras(stk_ctx* ctx, const Batch& b, int tile, int h, int kt, double omega, int dir);
size_t mg_ras_lds_bytes(int tile, int h, size_t es);
int mg_ras_tiles(int nx, int ny, int tile);
// Sweeps of level l: floor(nu * growth^l + 1/2).
int level_sweeps(int nu, double growth, int l);
// Two handles smooth alike (may share a batch).
bool same_smoothing(const stk_mg_opts& a, const stk_mg_opts& b);

}  // namespace stk
