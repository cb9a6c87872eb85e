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
    const T* ec;
    const T* en;
    T *vx, *vy;  // level iterate
    T *wx, *wy;  // ping-pong partner of the smoother
    T *bx, *by;  // right-hand side
    T *rx, *ry;  // residual scratch
    int cnx, cny;
    int64_t cld;
    T *cbx, *cby;  // coarse right-hand side
    T *cvx, *cvy;  // coarse iterate
    const T* st;    // stored Galerkin stencil (coarse levels), nullptr on the finest
    int64_t plane;  // elements per stencil plane
};

// Coarsest level of one instance: n unknowns, map[q] = (component << 30) |
// (j * ld + i), dense row-major inverse of -M.
template <typename T>
struct CoarseJob {
    int n;
    const int* map;
    const double* ainv;
    const T *bx, *by;
    T *vx, *vy;
};

// Krylov vectors of one instance on its finest level.
// X, R, Z, P, Q: Krylov iterate / residual / preconditioned residual /
// direction / A p, in the Krylov dtype.  F, B64, X64, R64: FP64 force, folded
// right-hand side, solution and true residual (refinement).
enum { VS_X = 0, VS_R, VS_Z, VS_P, VS_Q, VS_F, VS_B64, VS_X64, VS_R64, VS_N };
struct VecJob {
    int nx, ny;
    int64_t ld;
    double idx, idy;
    const double* ec;  // FP64 viscosities for the diag(-M) energy weights
    const double* en;
    void* v[VS_N][2];  // slot -> (x component, y component)
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
    double nv0;     // nv at the start of the current (inner) solve
    double nf;      // sum f^2 / d
    double thr;     // stop when nv <= thr
    int active;     // 1 while this instance iterates
    int pad;
};

// ---- launchers (mg_kernels.hip) ----------------------------------------------
struct Batch {       // a job array resident on the device plus its block prefix
    const void* jobs = nullptr;
    const int* pre = nullptr;
    int n = 0;       // instances
    int blocks = 0;  // total blocks
};

template <typename T> int mg_jacobi(stk_ctx* ctx, const Batch& b, double omega, int dir);
template <typename T> int mg_residual(stk_ctx* ctx, const Batch& b);
template <typename T> int mg_restrict(stk_ctx* ctx, const Batch& b_coarse_blocks);
template <typename T> int mg_zero_coarse(stk_ctx* ctx, const Batch& b_coarse_blocks);
template <typename T> int mg_prolong(stk_ctx* ctx, const Batch& b);
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

enum VecOp {
    OP_PQ = 0,      // acc0 += p.q
    OP_UPDATE,      // x += alpha p; r += alpha q; acc0 += r^2/d
    OP_RZ_ZQ,       // acc0 += r.z ; acc1 += z.q  (rho = -r: gamma = -acc0)
    OP_XPBY,        // p = z + beta p
    OP_RNORM,       // acc0 += r^2/d
    OP_FNORM,       // acc0 += f^2/d
    OP_INIT_P,      // p = z; acc0 += r.z
    OP_ZERO_Z,      // z = 0
    OP_ZERO_X       // x = 0
};
// phases of fcg_scalars
enum { PH_NF = 0, PH_NV, PH_NV0, PH_INIT, PH_ALPHA, PH_BETA, PH_THR };
// Slot dtype T for the Krylov vectors (R, Z, P, Q, X); partial sums land in
// `part` (2 per block), then per-instance sums in `sums` (2 per instance).
template <typename T>
int vec_op(stk_ctx* ctx, const Batch& b, int op, const FcgState* st, double* part, double* sums);
// cast slot src -> dst (to_f32: FP64 -> float, else float -> FP64), active instances only
int vec_cast_st(stk_ctx* ctx, const Batch& b, const FcgState* st, int src, int dst, int to_f32);
int vec_add_x64_st(stk_ctx* ctx, const Batch& b, const FcgState* st);  // X64 += (double) X (float)
// R64 = B64 - M X64 (FP64); sums[2i] = sum R64^2 / d
int vec_residual64_st(stk_ctx* ctx, const Batch& b, const FcgState* st, double* part, double* sums);
// Per-instance scalar update from the reduced sums (one thread per instance);
// `factor` scales the stop threshold (tol^2 for PH_NF, inner_tol^2 for PH_NV0).
int fcg_scalars(stk_ctx* ctx, FcgState* st, const double* sums, int n, int phase, double factor);
int inst_sums(stk_ctx* ctx, const Batch& b, const double* part, double* sums);
template <typename T> int mg_copy_wv(stk_ctx* ctx, const Batch& b);

}  // namespace stk
