// Multigrid and Krylov kernels for gfx950, batched over independent
// instances (one launch per (level, kernel) serves every instance).
//
// Geometric multigrid for the velocity block (paper Sec. 3.2, Sec. 6.2); the
// paper does not print the transfers, so these follow the stated reading:
// coarsening by 2, bilinear prolongation per velocity component (linear
// between coarse faces along the face normal, weights 3/4 and 1/4 between
// neighbouring coarse rows tangentially, mirrored at the free-slip walls),
// restriction R = P^T / 4, Galerkin coarse operators stored as 31-point
// stencils (coarse_stencil.hpp); the finest level is matrix-free.
//
// Launch shape: a flat grid of 256-thread blocks; block b belongs to the
// instance i with pre[i] <= b < pre[i+1] and covers a 64 x 4 patch of that
// instance's (nx+1) x (ny+1) index box.
#include <type_traits>

#include "coarse_stencil.hpp"
#include "mg_internal.hpp"
#include "rowstream.hpp"
#include "stencil.hpp"

namespace stk {
namespace {

constexpr int BX = 64, BY = 4, NT = BX * BY;

__device__ __forceinline__ int find_inst(const int* __restrict__ pre, int n, int b) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// (instance, i, j) of this thread for a box of (nx+1) x (ny+1) indices, block
// B of the flat grid
#define STK_BATCH_INDEX_B(JOBS, PRE, N, NXF, NYF, B)                                \
    const int inst = find_inst(PRE, N, (B));                                         \
    const auto& J = JOBS[inst];                                                      \
    const int lb = (B) - PRE[inst];                                                  \
    const int gxb = (NXF(J) + 1 + BX - 1) / BX;                                      \
    const int i = (lb % gxb) * BX + (int)(threadIdx.x % BX);                         \
    const int j = (lb / gxb) * BY + (int)(threadIdx.x / BX);
#define STK_BATCH_INDEX(JOBS, PRE, N, NXF, NYF) STK_BATCH_INDEX_B(JOBS, PRE, N, NXF, NYF, (int)blockIdx.x)
// The same with the blocks renumbered by XCD (xcd_tile): the block above a
// block (gxb further on) then runs on the same XCD at about the same time, and
// the rows both read (the stencil's reach, the transfers' windows) come from
// that XCD's L2.  In row order the level-1 Jacobi sweep of the 2048^2 solve
// read 1.4 times its algorithmic bytes.  For the kernels without block
// partials (their order would change the sums).
#define STK_BATCH_INDEX_XCD(JOBS, PRE, N, NXF, NYF) \
    STK_BATCH_INDEX_B(JOBS, PRE, N, NXF, NYF, xcd_tile((int)blockIdx.x, (int)gridDim.x))

#define FINE_NX(J) (J).nx
#define FINE_NY(J) (J).ny
#define COARSE_NX(J) (J).cnx
#define COARSE_NY(J) (J).cny

template <typename T>
__device__ __forceinline__ Grid<T> job_grid(const LevelJob<T>& J, const T* bx, const T* by, T omega) {
    Grid<T> g;
    g.ec = J.ec;
    g.en = J.en;
    g.bx = bx;
    g.by = by;
    g.ld = J.ld;
    g.nx = J.nx;
    g.ny = J.ny;
    g.idx = J.idx;
    g.idy = J.idy;
    g.omega = omega;
    return g;
}

// ---------------------------------------------------------------- smoother --
// Stored-stencil levels in FP64: the velocity of a workgroup's 64 x 4 patch,
// grown by the stencil's reach of two cells, is staged in LDS (0 outside the
// grid and on the walls, the operands of the global loaders), and the rows
// read it from there; the coefficients come from global memory.  In FP64 this
// cut a thread's registers from 196 to 128 VGPRs (twice the resident waves)
// and the 2048^2 solve iteration from 1.49 to 1.39 ms.  In FP32 the staged
// form (78 VGPRs) was slower than the gather (1.325 against 1.286 s for the
// 2048^2 FP32 V-cycle solve, interleaved runs), so FP32 levels gather.  Same
// row function (stencil_av_l) either way.
constexpr int SWX = BX + 4, SWY = BY + 4;  // staged window
template <typename T>
struct PatchPair {
    const T* win;
    int i0, j0;  // cell of window element (0, 0)
    __device__ __forceinline__ T operator()(int c, int i, int j) const {
        return win[(c * SWY + (j - j0)) * SWX + (i - i0)];
    }
};
template <typename T>
__device__ __forceinline__ PatchPair<T> stage_patch(T* win, const T* vx, const T* vy, int64_t ld, int nx, int ny,
                                                    int i, int j) {
    const int i0 = i - (int)(threadIdx.x % BX) - 2, j0 = j - (int)(threadIdx.x / BX) - 2;
    for (int e = threadIdx.x; e < 2 * SWY * SWX; e += NT) {
        const int c = e / (SWY * SWX), r = (e / SWX) % SWY, x = e % SWX;
        win[e] = c == 0 ? ldvx<T>(vx, ld, nx, ny, i0 + x, j0 + r) : ldvy<T>(vy, ld, nx, ny, i0 + x, j0 + r);
    }
    __syncthreads();
    return PatchPair<T>{win, i0, j0};
}

// One damped Jacobi sweep (dir 0: v -> w, dir 1: w -> v), the shared update.
template <typename T>
__global__ __launch_bounds__(NT) void k_mg_jacobi(const LevelJob<T>* __restrict__ jobs, const int* __restrict__ pre,
                                                  int n, T omega, int dir) {
    STK_BATCH_INDEX_XCD(jobs, pre, n, FINE_NX, FINE_NY)
    const T* sx = dir ? J.wx : J.vx;
    const T* sy = dir ? J.wy : J.vy;
    T* dx_ = dir ? J.vx : J.wx;
    T* dy_ = dir ? J.vy : J.wy;
    const int64_t k = (int64_t)j * J.ld + i;
    if (J.st) {  // stored Galerkin stencil: m = M v = -(A v), g = omega / A_ii (the instance is the block's)
        auto sweep = [&](const auto& lv) {
            if (i > J.nx || j > J.ny) return;
            for (int a = 0; a < 2; ++a) {
                if (a == 0 ? j >= J.ny : i >= J.nx) continue;
                T out = T(0);
                if (a == 0 ? is_vx_unknown(J.nx, J.ny, i, j) : is_vy_unknown(J.nx, J.ny, i, j)) {
                    T d;
                    const T av = stencil_av_l<T>(J.st, J.plane, a, lv, J.ld, J.nx, J.ny, i, j, d);
                    out = jac_step<T>(lv(a, i, j), omega / d, (a == 0 ? J.bx : J.by)[k], -av);
                }
                (a == 0 ? dx_ : dy_)[k] = out;
            }
        };
        if constexpr (sizeof(T) == 8) {
            __shared__ T win[2 * SWY * SWX];
            sweep(stage_patch<T>(win, sx, sy, J.ld, J.nx, J.ny, i, j));
        } else {
            if (i > J.nx || j > J.ny) return;
            for (int a = 0; a < 2; ++a) {
                if (a == 0 ? j >= J.ny : i >= J.nx) continue;
                T out = T(0);
                if (a == 0 ? is_vx_unknown(J.nx, J.ny, i, j) : is_vy_unknown(J.nx, J.ny, i, j)) {
                    T d;
                    const T av = stencil_av<T>(J.st, J.plane, a, sx, sy, J.ld, J.nx, J.ny, i, j, d);
                    out = jac_step<T>((a == 0 ? sx : sy)[k], omega / d, (a == 0 ? J.bx : J.by)[k], -av);
                }
                (a == 0 ? dx_ : dy_)[k] = out;
            }
        }
        return;
    }
    if (i > J.nx || j > J.ny) return;
    const Grid<T> g = job_grid<T>(J, J.bx, J.by, omega);
    if (j < J.ny) dx_[k] = is_vx_unknown(J.nx, J.ny, i, j) ? jac_vx_global(g, sx, sy, i, j) : T(0);
    if (i < J.nx) dy_[k] = is_vy_unknown(J.nx, J.ny, i, j) ? jac_vy_global(g, sx, sy, i, j) : T(0);
}

// Finest (matrix-free) level on the row-streaming engine (rowstream.hpp):
// workgroup b (renumbered by XCD) belongs to the instance with
// rpre[i] <= b < rpre[i+1], and its waves cover that instance's strips x
// segments.  Same operands, same stencil functions: the same values as the
// kernels above.
template <typename T>
__device__ __forceinline__ const LevelJob<T>& row_job(const LevelJob<T>* jobs, const int* rpre, int n, int& wv) {
    const int b = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    const int inst = find_inst(rpre, n, b);
    wv = (b - rpre[inst]) * rows::WPB + rows::wave_in_group();
    return jobs[inst];
}

template <typename T>
__global__ __launch_bounds__(64 * rows::WPB) void k_mg_jacobi_rows(const LevelJob<T>* __restrict__ jobs,
                                                                   const int* __restrict__ rpre, int n, T omega,
                                                                   int dir) {
    int wv;
    const LevelJob<T>& J = row_job(jobs, rpre, n, wv);
    const int nx = J.nx, ny = J.ny;
    const rows::Place q = rows::place(wv, nx, ny);
    if (q.y0 >= q.y1) return;  // the whole wave
    const int i = q.i;
    const T* sx = dir ? J.wx : J.vx;
    const T* sy = dir ? J.wy : J.vy;
    T* dx_ = dir ? J.vx : J.wx;
    T* dy_ = dir ? J.vy : J.wy;
    const rows::Loader<T> L = rows::make_loader<T>(sx, sy, J.ec, J.en, J.bx, J.by, nullptr, J.ld, nx, ny, i);
    const bool xcol = i >= 1 && i <= nx - 1, ycol = i >= 0 && i <= nx - 1;
    const unsigned col = (unsigned)i * (unsigned)sizeof(T);
    const unsigned s_x = q.own ? col : OOB, s_y = (q.own && ycol) ? col : OOB;
    rows::walk_rows<T>(L, q.y0, q.y1, [&](const rows::Row<T>& a, const rows::Row<T>& b, const rows::Row<T>& c, int j) {
        T ux, uy;
        rows::jacobi_row<T>(a, b, c, omega, J.idx, J.idy, ux, uy);
        const bool xu = xcol && j <= ny - 1, yu = ycol && j >= 1 && j <= ny - 1;
        rows::store_pair<T>(dx_, dy_, J.ld, nx, ny, j, xu ? ux : T(0), yu ? uy : T(0), s_x, s_y);
    });
}

template <typename T>
__global__ __launch_bounds__(64 * rows::WPB) void k_mg_residual_rows(const LevelJob<T>* __restrict__ jobs,
                                                                     const int* __restrict__ rpre, int n) {
    int wv;
    const LevelJob<T>& J = row_job(jobs, rpre, n, wv);
    const int nx = J.nx, ny = J.ny;
    const rows::Place q = rows::place(wv, nx, ny);
    if (q.y0 >= q.y1) return;  // the whole wave
    const int i = q.i;
    const rows::Loader<T> L = rows::make_loader<T>(J.vx, J.vy, J.ec, J.en, J.bx, J.by, nullptr, J.ld, nx, ny, i);
    const bool xcol = i >= 1 && i <= nx - 1, ycol = i >= 0 && i <= nx - 1;
    const unsigned col = (unsigned)i * (unsigned)sizeof(T);
    const unsigned s_x = q.own ? col : OOB, s_y = (q.own && ycol) ? col : OOB;
    rows::walk_rows<T>(L, q.y0, q.y1, [&](const rows::Row<T>& a, const rows::Row<T>& b, const rows::Row<T>& c, int j) {
        const rows::Res<T> r = rows::residual_row<T, T>(a, b, c, false, J.idx, J.idy);
        const bool xu = xcol && j <= ny - 1, yu = ycol && j >= 1 && j <= ny - 1;
        rows::store_pair<T>(J.rx, J.ry, J.ld, nx, ny, j, xu ? r.rx : T(0), yu ? r.ry : T(0), s_x, s_y);
    });
}

// ---------------------------------------------------------------- residual --
// r = b - M v at (i, j) of the matrix-free level (0 on walls and outside the
// box of each component).
template <typename T>
__device__ __forceinline__ void mf_residual(const LevelJob<T>& J, int i, int j, T& rx, T& ry) {
    const int nx = J.nx, ny = J.ny;
    const int64_t ld = J.ld, k = (int64_t)j * ld + i;
    auto VX = [&](int a, int b) { return ldvx<T>(J.vx, ld, nx, ny, a, b); };
    auto VY = [&](int a, int b) { return ldvy<T>(J.vy, ld, nx, ny, a, b); };
    auto ENH = [&](int a, int b) { return (a >= 1 && a <= nx - 1 && b >= 1 && b <= ny - 1) ? J.en[(int64_t)b * ld + a] : T(0); };
    rx = T(0);
    ry = T(0);
    if (is_vx_unknown(nx, ny, i, j))
        rx = J.bx[k] - mv_x<T>(VX(i, j), VX(i - 1, j), VX(i + 1, j), VX(i, j - 1), VX(i, j + 1), VY(i, j),
                               VY(i - 1, j), VY(i, j + 1), VY(i - 1, j + 1), J.ec[k - 1], J.ec[k], ENH(i, j),
                               ENH(i, j + 1), J.idx, J.idy);
    if (is_vy_unknown(nx, ny, i, j))
        ry = J.by[k] - mv_y<T>(VY(i, j), VY(i - 1, j), VY(i + 1, j), VY(i, j - 1), VY(i, j + 1), VX(i, j),
                               VX(i + 1, j), VX(i, j - 1), VX(i + 1, j - 1), J.ec[k - ld], J.ec[k], ENH(i, j),
                               ENH(i + 1, j), J.idx, J.idy);
}

// r = b - M v on the unknowns (0 on walls).
template <typename T>
__global__ __launch_bounds__(NT) void k_mg_residual(const LevelJob<T>* __restrict__ jobs, const int* __restrict__ pre,
                                                    int n) {
    STK_BATCH_INDEX_XCD(jobs, pre, n, FINE_NX, FINE_NY)
    const int nx = J.nx, ny = J.ny;
    const int64_t ld = J.ld, k = (int64_t)j * ld + i;
    if (J.st) {  // r = b - M v = b + A v (velocity staged in FP64, as in k_mg_jacobi)
        auto resid = [&](const auto& lv) {
            if (i > nx || j > ny) return;
            for (int a = 0; a < 2; ++a) {
                if (a == 0 ? j >= ny : i >= nx) continue;
                T r = T(0);
                if (a == 0 ? is_vx_unknown(nx, ny, i, j) : is_vy_unknown(nx, ny, i, j)) {
                    T d;
                    r = (a == 0 ? J.bx : J.by)[k] + stencil_av_l<T>(J.st, J.plane, a, lv, ld, nx, ny, i, j, d);
                }
                (a == 0 ? J.rx : J.ry)[k] = r;
            }
        };
        if constexpr (sizeof(T) == 8) {
            __shared__ T win[2 * SWY * SWX];
            resid(stage_patch<T>(win, J.vx, J.vy, ld, nx, ny, i, j));
        } else {
            if (i > nx || j > ny) return;
            for (int a = 0; a < 2; ++a) {
                if (a == 0 ? j >= ny : i >= nx) continue;
                T r = T(0);
                if (a == 0 ? is_vx_unknown(nx, ny, i, j) : is_vy_unknown(nx, ny, i, j)) {
                    T d;
                    r = (a == 0 ? J.bx : J.by)[k] + stencil_av<T>(J.st, J.plane, a, J.vx, J.vy, ld, nx, ny, i, j, d);
                }
                (a == 0 ? J.rx : J.ry)[k] = r;
            }
        }
        return;
    }
    if (i > nx || j > ny) return;
    T rx, ry;
    mf_residual<T>(J, i, j, rx, ry);
    if (j < ny) J.rx[k] = rx;
    if (i < nx) J.ry[k] = ry;
}

// --------------------------------------------------------------- transfers --
// Weights of a fine index f on coarse indices along one axis (see header):
// normal axis: f even -> f/2 (1); f odd -> (f-1)/2, (f+1)/2 (1/2 each).
// tangential axis: J = f/2 with 3/4, neighbour J-1 (f even) or J+1 (f odd)
// with 1/4, the neighbour mirrored onto J outside [0, nc).
__device__ __forceinline__ int w_normal(int f, int* c, double* w) {
    if ((f & 1) == 0) { c[0] = f >> 1; w[0] = 1.0; return 1; }
    c[0] = (f - 1) >> 1; w[0] = 0.5;
    c[1] = (f + 1) >> 1; w[1] = 0.5;
    return 2;
}
__device__ __forceinline__ int w_tangent(int f, int nc, int* c, double* w) {
    const int J = f >> 1, nb = (f & 1) ? J + 1 : J - 1;
    if (nb < 0 || nb >= nc) { c[0] = J; w[0] = 1.0; return 1; }
    c[0] = J; w[0] = 0.75;
    c[1] = nb; w[1] = 0.25;
    return 2;
}

// coarse rhs = R r = P^T r / 4, gathered per coarse unknown from the fine
// unknowns that prolongate from it; the coarse iterate is set to 0 in the same
// pass (the coarse problem is solved for the correction from 0).  The fine
// values of a coarse unknown's 3 x 4 window are loaded first, all at once
// (rows or columns outside the grid clamped onto it), and the terms whose
// weights are nonzero are then added in window order, so a thread waits for
// one round trip instead of one per term.
// rf(c, fi, fj): the fine residual of component c (as double); (i, j) inside
// the coarse (cnx+1) x (cny+1) box.
//
// J.first: the coarse level's first smoothing sweep is taken here.  That
// sweep starts from the zero iterate, so A v = 0 and each new value depends
// only on the point's own right-hand side and diagonal: the damped Jacobi
// update jac_step(0, omega / a_ii, b, -0), the same operation with the same
// operands as in k_mg_jacobi (which sums the zero terms to +0).  It is written
// to w, where that sweep writes, and v is not cleared (the next sweep, w -> v,
// or the odd-count copy overwrites it before anything reads it).
template <typename T, typename RF>
__device__ __forceinline__ void restrict_from(const LevelJob<T>& J, int i, int j, const RF& rf, T omega) {
    const int NX = J.cnx, NY = J.cny, nx = J.nx, ny = J.ny;
    const int64_t cld = J.cld, k = (int64_t)j * cld + i;
    if (j < NY) {  // coarse vx(I=i, J=j): fine columns 2i-1..2i+1 (normal), rows 2j-1..2j+2 (tangential)
        double s = 0.0;
        if (i >= 1 && i <= NX - 1) {
            double rv[3][4];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    rv[a][b] = rf(0, 2 * i - 1 + a, min(max(2 * j - 1 + b, 0), ny - 1));
                }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int fi = 2 * i - 1 + a;
                int ci[2];
                double wi[2];
                const int nci = w_normal(fi, ci, wi);
                double wn = 0.0;
                for (int q = 0; q < nci; ++q) wn += ci[q] == i ? wi[q] : 0.0;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int fj = 2 * j - 1 + b;
                    if (fj < 0 || fj >= ny) continue;
                    int cj[2];
                    double wj[2];
                    const int ncj = w_tangent(fj, NY, cj, wj);
                    double wt = 0.0;
                    for (int q = 0; q < ncj; ++q) wt += cj[q] == j ? wj[q] : 0.0;
                    if (wn != 0.0 && wt != 0.0) s += 0.25 * wn * wt * rv[a][b];
                }
            }
        }
        const T bc = T(s);
        J.cbx[k] = bc;
        if (J.first)
            J.cwx[k] = (i >= 1 && i <= NX - 1) ? jac_step<T>(T(0), omega / J.cst[k], bc, -T(0)) : T(0);
        else
            J.cvx[k] = T(0);
    }
    if (i < NX) {  // coarse vy(I=i, J=j): fine rows 2j-1..2j+1 (normal), columns 2i-1..2i+2 (tangential)
        double s = 0.0;
        if (j >= 1 && j <= NY - 1) {
            double rv[3][4];
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    rv[b][a] = rf(1, min(max(2 * i - 1 + a, 0), nx - 1), 2 * j - 1 + b);
                }
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const int fj = 2 * j - 1 + b;
                int cj[2];
                double wj[2];
                const int ncj = w_normal(fj, cj, wj);
                double wn = 0.0;
                for (int q = 0; q < ncj; ++q) wn += cj[q] == j ? wj[q] : 0.0;
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const int fi = 2 * i - 1 + a;
                    if (fi < 0 || fi >= nx) continue;
                    int ci[2];
                    double wi[2];
                    const int nci = w_tangent(fi, NX, ci, wi);
                    double wt = 0.0;
                    for (int q = 0; q < nci; ++q) wt += ci[q] == i ? wi[q] : 0.0;
                    if (wn != 0.0 && wt != 0.0) s += 0.25 * wn * wt * rv[b][a];
                }
            }
        }
        const T bc = T(s);
        J.cby[k] = bc;
        if (J.first)
            J.cwy[k] = (j >= 1 && j <= NY - 1) ? jac_step<T>(T(0), omega / J.cst[PL_VY * J.cplane + k], bc, -T(0))
                                               : T(0);
        else
            J.cvy[k] = T(0);
    }
}
template <typename T>
__global__ __launch_bounds__(NT) void k_mg_restrict(const LevelJob<T>* __restrict__ jobs, const int* __restrict__ pre,
                                                    int n, T omega) {
    STK_BATCH_INDEX_XCD(jobs, pre, n, COARSE_NX, COARSE_NY)
    if (i > J.cnx || j > J.cny) return;
    const int64_t ld = J.ld;
    restrict_from<T>(
        J, i, j, [&](int c, int fi, int fj) { return (double)(c == 0 ? J.rx : J.ry)[(int64_t)fj * ld + fi]; }, omega);
}

// Interpolation terms of one fine unknown: up to 2 x 2 coarse indices with
// weights; absent terms repeat the first index and are masked out.
struct Terms {
    int ci[2], cj[2];
    double wi[2], wj[2];
    int na, nb;
};
__device__ __forceinline__ void pad_terms(Terms& t) {
    if (t.na == 1) { t.ci[1] = t.ci[0]; t.wi[1] = 0.0; }
    if (t.nb == 1) { t.cj[1] = t.cj[0]; t.wj[1] = 0.0; }
}

// (P e_c) at a fine vx / vy unknown (i, j), as double.  The coarse values are
// loaded first, all at once (their indices are inside the coarse arrays
// whether or not the term is used), and the terms added in the order the
// weights list them.
template <typename T>
__device__ __forceinline__ double prolong_sx(const LevelJob<T>& J, int i, int j) {
    Terms t;
    t.na = w_normal(i, t.ci, t.wi);
    t.nb = w_tangent(j, J.cny, t.cj, t.wj);
    pad_terms(t);
    double c[2][2];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) c[p][q] = (double)J.cvx[(int64_t)t.cj[q] * J.cld + t.ci[p]];
    double s = 0.0;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const double cv = (t.ci[p] >= 1 && t.ci[p] <= J.cnx - 1) ? c[p][q] : 0.0;
            if (p < t.na && q < t.nb) s += t.wi[p] * t.wj[q] * cv;
        }
    return s;
}
template <typename T>
__device__ __forceinline__ double prolong_sy(const LevelJob<T>& J, int i, int j) {
    Terms t;
    t.na = w_tangent(i, J.cnx, t.ci, t.wi);
    t.nb = w_normal(j, t.cj, t.wj);
    pad_terms(t);
    double c[2][2];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) c[p][q] = (double)J.cvy[(int64_t)t.cj[q] * J.cld + t.ci[p]];
    double s = 0.0;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const double cv = (t.cj[q] >= 1 && t.cj[q] <= J.cny - 1) ? c[p][q] : 0.0;
            if (p < t.na && q < t.nb) s += t.wi[p] * t.wj[q] * cv;
        }
    return s;
}

// v += P e_c on the fine unknowns.
template <typename T>
__global__ __launch_bounds__(NT) void k_mg_prolong(const LevelJob<T>* __restrict__ jobs, const int* __restrict__ pre,
                                                   int n) {
    STK_BATCH_INDEX_XCD(jobs, pre, n, FINE_NX, FINE_NY)
    const int nx = J.nx, ny = J.ny;
    if (i > nx || j > ny) return;
    const int64_t k = (int64_t)j * J.ld + i;
    if (is_vx_unknown(nx, ny, i, j)) {
        const T v = J.vx[k];
        J.vx[k] = v + T(prolong_sx(J, i, j));
    }
    if (is_vy_unknown(nx, ny, i, j)) {
        const T v = J.vy[k];
        J.vy[k] = v + T(prolong_sy(J, i, j));
    }
}

// Stored-stencil levels: the prolongation and the first post-smoothing sweep
// (v + P e_c -> w) in one pass.  The staged window holds the corrected
// iterate, v + T(P e_c) on the unknowns and 0 elsewhere, which is what
// k_mg_prolong stores and the loaders then read; it is not stored, since the
// next sweep (w -> v) or the odd-count copy overwrites v.  Staged in both
// precisions: the correction is computed where it is staged.
template <typename T>
__global__ __launch_bounds__(NT) void k_mg_jacobi_prolonged(const LevelJob<T>* __restrict__ jobs,
                                                            const int* __restrict__ pre, int n, T omega) {
    STK_BATCH_INDEX_XCD(jobs, pre, n, FINE_NX, FINE_NY)
    const int nx = J.nx, ny = J.ny;
    const int64_t ld = J.ld;
    __shared__ T win[2 * SWY * SWX];
    const int i0 = i - (int)(threadIdx.x % BX) - 2, j0 = j - (int)(threadIdx.x / BX) - 2;
    for (int e = threadIdx.x; e < 2 * SWY * SWX; e += NT) {
        const int c = e / (SWY * SWX), r = (e / SWX) % SWY, x = e % SWX;
        const int ii = i0 + x, jj = j0 + r;
        const int64_t kk = (int64_t)jj * ld + ii;
        T val = T(0);
        if (c == 0 && is_vx_unknown(nx, ny, ii, jj)) {
            const T v = J.vx[kk];
            val = v + T(prolong_sx(J, ii, jj));
        } else if (c == 1 && is_vy_unknown(nx, ny, ii, jj)) {
            const T v = J.vy[kk];
            val = v + T(prolong_sy(J, ii, jj));
        }
        win[e] = val;
    }
    __syncthreads();
    const PatchPair<T> lv{win, i0, j0};
    if (i > nx || j > ny) return;
    const int64_t k = (int64_t)j * ld + i;
    for (int a = 0; a < 2; ++a) {
        if (a == 0 ? j >= ny : i >= nx) continue;
        T out = T(0);
        if (a == 0 ? is_vx_unknown(nx, ny, i, j) : is_vy_unknown(nx, ny, i, j)) {
            T d;
            const T av = stencil_av_l<T>(J.st, J.plane, a, lv, ld, nx, ny, i, j, d);
            out = jac_step<T>(lv(a, i, j), omega / d, (a == 0 ? J.bx : J.by)[k], -av);
        }
        (a == 0 ? J.wx : J.wy)[k] = out;
    }
}

// ------------------------------------------------------------ coarsest grid --
// One workgroup per instance: dense FP64 solve x = A^{-1} (-b) of the coarsest
// problem (A = -M assembled and inverted on the host at setup), gathered from
// and scattered to the level layout through the unknown index map.
// Coarsest solve v = A^-1 (-b).  A workgroup takes 64 rows (grid x) of one
// instance (grid y); its CW waves each sum a contiguous chunk of the columns
// for those rows, and the chunk sums are added in chunk order.  The inverse is
// stored column by column, so a wave's loads of one column are contiguous, and
// a large coarsest level spreads its inverse over many waves and CUs (a single
// chain per row left the 1984-unknown solve of a 32^2 level latency-bound at
// about 200 us; the chunks, each loaded one column at a time, at 63 us).
constexpr int CW = 16;
template <typename T>
__global__ __launch_bounds__(64 * CW) void k_mg_coarse(const CoarseJob<T>* __restrict__ jobs) {
    extern __shared__ double csh[];  // CW x 64 chunk sums, then the right-hand side
    double* part = csh;
    double* rhs = csh + CW * 64;
    const CoarseJob<T>& J = jobs[blockIdx.y];
    const int nu = J.n;
    if ((int)blockIdx.x * 64 >= nu) return;  // the whole workgroup: no rows of this instance
    for (int r = threadIdx.x; r < nu; r += 64 * CW) {
        const int code = J.map[r];  // (component << 30) | (j * ld + i) offset
        const int off = code & 0x3fffffff;
        rhs[r] = -(double)((code >> 30) ? J.by[off] : J.bx[off]);
    }
    __syncthreads();
    const int w = (int)threadIdx.x / 64, lane = (int)threadIdx.x % 64, q = (int)blockIdx.x * 64 + lane;
    const int c0 = (int)((int64_t)nu * w / CW), c1 = (int)((int64_t)nu * (w + 1) / CW);
    double s = 0.0;
    if (q < nu) {
        // eight loads in flight before their products are added, in column order
        const double* col = J.ainv + q;
        int c = c0;
        for (; c + 8 <= c1; c += 8) {
            double a[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] = col[(int64_t)(c + u) * nu];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += a[u] * rhs[c + u];
        }
        for (; c < c1; ++c) s += col[(int64_t)c * nu] * rhs[c];
    }
    part[w * 64 + lane] = s;
    __syncthreads();
    if (w == 0 && q < nu) {
        double t = part[lane];
        for (int u = 1; u < CW; ++u) t += part[u * 64 + lane];
        const int code = J.map[q];
        const int off = code & 0x3fffffff;
        if (code >> 30) J.vy[off] = T(t); else J.vx[off] = T(t);
    }
}

// w -> v copy of the level iterate (after an odd number of sweeps)
template <typename T>
__global__ __launch_bounds__(NT) void k_mg_copy_wv(const LevelJob<T>* __restrict__ jobs, const int* __restrict__ pre,
                                                   int n) {
    STK_BATCH_INDEX(jobs, pre, n, FINE_NX, FINE_NY)
    if (i > J.nx || j > J.ny) return;
    const int64_t k = (int64_t)j * J.ld + i;
    if (j < J.ny) J.vx[k] = J.wx[k];
    if (i < J.nx) J.vy[k] = J.wy[k];
}

// --------------------------------------------------------- Krylov vectors --
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}
__device__ __forceinline__ void block_sum2(double a0, double a1, double* part) {
    __shared__ double red[2][NT / 64];
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][w] = a0;
        red[1][w] = a1;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double s = 0.0;
        for (int q = 0; q < NT / 64; ++q) s += red[threadIdx.x][q];
        part[2 * blockIdx.x + threadIdx.x] = s;
    }
}

// diag(-M) at vx(i,j) / vy(i,j) from the FP64 viscosities (unknowns only)
__device__ __forceinline__ double dgx(const VecJob& J, int i, int j) {
    const int64_t ld = J.ld, k = (int64_t)j * ld + i;
    const double enb = (j >= 1 && j <= J.ny - 1) ? J.en[k] : 0.0;
    const double ent = (j + 1 <= J.ny - 1) ? J.en[k + ld] : 0.0;
    return diag_x<double>(J.ec[k - 1], J.ec[k], enb, ent, J.idx, J.idy);
}
__device__ __forceinline__ double dgy(const VecJob& J, int i, int j) {
    const int64_t ld = J.ld, k = (int64_t)j * ld + i;
    const double enl = (i >= 1 && i <= J.nx - 1) ? J.en[k] : 0.0;
    const double enr = (i + 1 <= J.nx - 1) ? J.en[k + 1] : 0.0;
    return diag_y<double>(J.ec[k - ld], J.ec[k], enl, enr, J.idx, J.idy);
}

template <typename T, typename ZT>
__global__ __launch_bounds__(NT) void k_vec(const VecJob* __restrict__ jobs, const int* __restrict__ pre, int n,
                                            int op, const FcgState* __restrict__ st, double* __restrict__ part) {
    STK_BATCH_INDEX(jobs, pre, n, FINE_NX, FINE_NY)
    double a0 = 0.0, a1 = 0.0;
    if (i <= J.nx && j <= J.ny && st[inst].active) {
        const int64_t k = (int64_t)j * J.ld + i;
        const double al = st[inst].alpha, be = st[inst].beta;
        for (int c = 0; c < 2; ++c) {
            const bool u = c == 0 ? is_vx_unknown(J.nx, J.ny, i, j) : is_vy_unknown(J.nx, J.ny, i, j);
            const bool inbox = c == 0 ? j < J.ny : i < J.nx;
            if (!inbox) continue;
            T* X = (T*)(J.v[VS_X][c]);
            T* R = (T*)(J.v[VS_R][c]);
            ZT* Z = (ZT*)(J.v[VS_Z][c]);
            T* P = (T*)(J.v[VS_P][c]);
            T* Q = (T*)(J.v[VS_Q][c]);
            switch (op) {
                case OP_UPDATE:
                    if (u) {
                        X[k] = T((double)X[k] + al * (double)P[k]);
                        const T r = T((double)R[k] + al * (double)Q[k]);
                        R[k] = r;
                        a0 += (double)r * (double)r / (c == 0 ? dgx(J, i, j) : dgy(J, i, j));
                    }
                    // the next V-cycle's initial guess (OP_ZERO_Z), when Z is this plan's own
                    // FP64 slot; the FP32 one is zeroed by the cast that starts that V-cycle
                    if constexpr (std::is_same<ZT, T>::value) Z[k] = ZT(0);
                    break;
                case OP_XPBY:
                    P[k] = u ? T((double)Z[k] + be * (double)P[k]) : T(0);
                    break;
                case OP_RZ_ZQ:
                    if (u) {
                        a0 += (double)R[k] * (double)Z[k];
                        a1 += (double)Z[k] * (double)Q[k];
                    }
                    break;
                case OP_FNORM: {
                    const double* F = (const double*)(J.v[VS_F][c]);
                    if (u) a0 += F[k] * F[k] / (c == 0 ? dgx(J, i, j) : dgy(J, i, j));
                    break;
                }
                case OP_INIT_P:
                    P[k] = u ? T(Z[k]) : T(0);
                    if (u) a0 += (double)R[k] * (double)Z[k];
                    break;
                default:  // OP_ZERO_Z
                    Z[k] = ZT(0);
                    break;
            }
        }
    }
    block_sum2(a0, a1, part);
}

// FCG operator apply on the finest level fused with its dot product: Q = A P
// = -(M P) and the partial sums of P . Q, one per workgroup in part[2 b]
// (workgroup b in the rpre numbering; part[2 b + 1] = 0), in one
// row-streaming pass.  Jobs: v = P, no right-hand side, r = Q.  P is only
// read (updating it here in place would race with the neighbouring waves'
// halo reads).  Inactive instances are left as they are (zero partials).
__global__ __launch_bounds__(64 * rows::WPB) void k_fcg_apply_rows(const LevelJob<double>* __restrict__ jobs,
                                                                   const int* __restrict__ rpre, int n,
                                                                   const FcgState* __restrict__ st,
                                                                   double* __restrict__ part) {
    const int b = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    const int inst = find_inst(rpre, n, b);
    const LevelJob<double>& J = jobs[inst];
    const int wv = (b - rpre[inst]) * rows::WPB + rows::wave_in_group();
    const int nx = J.nx, ny = J.ny;
    const rows::Place q = rows::place(wv, nx, ny);
    double pq = 0.0;
    if (st[inst].active && q.y0 < q.y1) {
        const int i = q.i;
        const rows::Loader<double> L =
            rows::make_loader<double>(J.vx, J.vy, J.ec, J.en, nullptr, nullptr, nullptr, J.ld, nx, ny, i);
        const bool xcol = i >= 1 && i <= nx - 1, ycol = i >= 0 && i <= nx - 1;
        const unsigned col = (unsigned)i * (unsigned)sizeof(double);
        const unsigned s_x = q.own ? col : OOB, s_y = (q.own && ycol) ? col : OOB;
        rows::walk_rows<double>(L, q.y0, q.y1,
                                [&](const rows::Row<double>& a, const rows::Row<double>& c0, const rows::Row<double>& c,
                                    int j) {
                                    const rows::Res<double> r = rows::residual_row<double, double>(a, c0, c, false,
                                                                                                  J.idx, J.idy);
                                    const bool xu = xcol && j <= ny - 1, yu = ycol && j >= 1 && j <= ny - 1;
                                    rows::store_pair<double>(J.rx, J.ry, J.ld, nx, ny, j, xu ? r.rx : 0.0,
                                                             yu ? r.ry : 0.0, s_x, s_y);
                                    if (q.own && xu) pq += c0.vx * r.rx;
                                    if (q.own && yu) pq += c0.vy * r.ry;
                                });
    }
    __shared__ double red[rows::WPB];
    pq = wave_sum(pq);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = pq;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < rows::WPB; ++w) s += red[w];
        part[2 * b] = s;
        part[2 * b + 1] = 0.0;
    }
}

// r32 = (float) r64 and z32 = 0, walls included
__global__ __launch_bounds__(NT) void k_prec_cast(const XCastJob* __restrict__ jobs, const int* __restrict__ pre,
                                                  int n, const FcgState* __restrict__ st) {
    STK_BATCH_INDEX(jobs, pre, n, FINE_NX, FINE_NY)
    if (i > J.nx || j > J.ny || !st[inst].active) return;
    const int64_t k = (int64_t)j * J.ld + i;
    for (int c = 0; c < 2; ++c) {
        if (c == 0 ? j >= J.ny : i >= J.nx) continue;
        J.r32[c][k] = (float)J.r64[c][k];
        J.z32[c][k] = 0.0f;
    }
}

// R = B - M X in FP64 with sum R^2 / d
__global__ __launch_bounds__(NT) void k_vec_res64(const VecJob* __restrict__ jobs, const int* __restrict__ pre, int n,
                                                  const FcgState* __restrict__ st, double* __restrict__ part) {
    STK_BATCH_INDEX(jobs, pre, n, FINE_NX, FINE_NY)
    double a0 = 0.0;
    if (i <= J.nx && j <= J.ny && st[inst].active) {
        const int nx = J.nx, ny = J.ny;
        const int64_t ld = J.ld, k = (int64_t)j * ld + i;
        const double* vx = (const double*)(J.v[VS_X][0]);
        const double* vy = (const double*)(J.v[VS_X][1]);
        auto VX = [&](int a, int b) { return ldvx<double>(vx, ld, nx, ny, a, b); };
        auto VY = [&](int a, int b) { return ldvy<double>(vy, ld, nx, ny, a, b); };
        auto ENH = [&](int a, int b) { return (a >= 1 && a <= nx - 1 && b >= 1 && b <= ny - 1) ? J.en[(int64_t)b * ld + a] : 0.0; };
        if (j < ny) {
            double r = 0.0;
            if (is_vx_unknown(nx, ny, i, j)) {
                const double m = mv_x<double>(VX(i, j), VX(i - 1, j), VX(i + 1, j), VX(i, j - 1), VX(i, j + 1), VY(i, j),
                                              VY(i - 1, j), VY(i, j + 1), VY(i - 1, j + 1), J.ec[k - 1], J.ec[k],
                                              ENH(i, j), ENH(i, j + 1), J.idx, J.idy);
                r = ((const double*)J.v[VS_B][0])[k] - m;
                a0 += r * r / dgx(J, i, j);
            }
            ((double*)J.v[VS_R][0])[k] = r;
        }
        if (i < nx) {
            double r = 0.0;
            if (is_vy_unknown(nx, ny, i, j)) {
                const double m = mv_y<double>(VY(i, j), VY(i - 1, j), VY(i + 1, j), VY(i, j - 1), VY(i, j + 1), VX(i, j),
                                              VX(i + 1, j), VX(i, j - 1), VX(i + 1, j - 1), J.ec[k - ld], J.ec[k],
                                              ENH(i, j), ENH(i + 1, j), J.idx, J.idy);
                r = ((const double*)J.v[VS_B][1])[k] - m;
                a0 += r * r / dgy(J, i, j);
            }
            ((double*)J.v[VS_R][1])[k] = r;
        }
    }
    block_sum2(a0, 0.0, part);
}

__device__ __forceinline__ void fcg_update(FcgState& s, double s0, double s1, int phase) {
    switch (phase) {
        case PH_NF:  // N_f and the stop threshold
            if (s.active) {
                s.nf = s0;
                s.thr = s.tol2 * s0;
            }
            break;
        case PH_NV:
            if (s.active) {
                s.nv = s0;
                s.left -= 1;
                s.active = s0 > s.thr && s.left > 0;
            }
            break;
        case PH_TRUE:
            if (s.active) {
                s.nv = s0;
                s.active = s0 > s.thr;
            }
            break;
        case PH_INIT:
            if (s.active) s.gamma = -s0;
            break;
        case PH_ALPHA:
            if (s.active) {
                s.pq = s0;
                s.alpha = (s0 != 0.0) ? s.gamma / s0 : 0.0;
            }
            break;
        default: {  // PH_BETA: rho = -r, gamma' = rho.z, beta = -alpha (z.q) / gamma
            if (s.active) {
                const double gnew = -s0;
                s.rz = s0;
                s.zq = s1;
                s.beta = (s.gamma != 0.0) ? -s.alpha * s1 / s.gamma : 0.0;
                s.gamma = gnew;
            }
        }
    }
}

// Per-instance sums of the per-block partials and the scalar update in one
// launch, one workgroup per instance.  The order is fixed and depends only on
// the instance's own block count: its partials come in chunks of SUM_CHUNK
// blocks; in a chunk, thread t sums partials t, t + 256, ... in turn, the
// waves reduce by shuffles, and the four wave sums are added in order; the
// chunk sums are added in chunk order.  Then the scalar update of `phase`,
// and optionally a copy of the updated state to `out` (pinned host memory).
// This replaced three launches per dot product (chunk sums, instance sums,
// scalar update), each about 5 us on the device however small.
__global__ __launch_bounds__(256) void k_fcg_reduce(const int* __restrict__ pre, const int* __restrict__ cpre,
                                                    const double* __restrict__ part, double* __restrict__ sums,
                                                    FcgState* __restrict__ st, int phase, FcgState* out) {
    const int inst = blockIdx.x;
    __shared__ double red[2][256 / 64];
    double t0 = 0.0, t1 = 0.0;
    for (int c = cpre[inst]; c < cpre[inst + 1]; ++c) {
        const int b0 = pre[inst] + (c - cpre[inst]) * SUM_CHUNK;
        const int b1 = min(pre[inst + 1], b0 + SUM_CHUNK);
        // a thread's SUM_CHUNK / 256 partials are loaded before they are added (in
        // the order above): one round trip per chunk instead of one per partial
        double v0[SUM_CHUNK / 256], v1[SUM_CHUNK / 256];
#pragma unroll
        for (int q = 0; q < SUM_CHUNK / 256; ++q) {
            const int b = min(b0 + (int)threadIdx.x + 256 * q, b1 - 1);  // a chunk is never empty
            v0[q] = part[2 * b];
            v1[q] = part[2 * b + 1];
        }
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int q = 0; q < SUM_CHUNK / 256; ++q) {
            if (b0 + (int)threadIdx.x + 256 * q < b1) {
                s0 += v0[q];
                s1 += v1[q];
            }
        }
        s0 = wave_sum(s0);
        s1 = wave_sum(s1);
        if ((threadIdx.x & 63) == 0) {
            red[0][threadIdx.x >> 6] = s0;
            red[1][threadIdx.x >> 6] = s1;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double c0 = 0.0, c1 = 0.0;
            for (int q = 0; q < 256 / 64; ++q) {
                c0 += red[0][q];
                c1 += red[1][q];
            }
            t0 += c0;
            t1 += c1;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sums[2 * inst] = t0;
        sums[2 * inst + 1] = t1;
        fcg_update(st[inst], t0, t1, phase);
        if (out) out[inst] = st[inst];
    }
}

inline dim3 nblk(int blocks) { return dim3((unsigned)blocks); }

}  // namespace
}  // namespace stk

namespace stk {

#define STK_LAUNCH_CHECK() STK_HIP(hipGetLastError())

template <typename T>
int mg_jacobi(stk_ctx* ctx, const Batch& b, double omega, int dir) {
    if (!b.n) return STK_OK;
    if (b.rpre)
        hipLaunchKernelGGL(k_mg_jacobi_rows<T>, dim3(b.rblocks), dim3(64 * rows::WPB), 0, ctx->stream,
                           static_cast<const LevelJob<T>*>(b.jobs), b.rpre, b.n, T(omega), dir);
    else
        hipLaunchKernelGGL(k_mg_jacobi<T>, dim3(b.blocks), dim3(NT), 0, ctx->stream,
                           static_cast<const LevelJob<T>*>(b.jobs), b.pre, b.n, T(omega), dir);
    STK_LAUNCH_CHECK();
    return STK_OK;
}
template <typename T>
int mg_copy_wv(stk_ctx* ctx, const Batch& b) {
    if (!b.n) return STK_OK;
    hipLaunchKernelGGL(k_mg_copy_wv<T>, dim3(b.blocks), dim3(NT), 0, ctx->stream,
                       static_cast<const LevelJob<T>*>(b.jobs), b.pre, b.n);
    STK_LAUNCH_CHECK();
    return STK_OK;
}
template <typename T>
int mg_residual(stk_ctx* ctx, const Batch& b) {
    if (!b.n) return STK_OK;
    if (b.rpre)
        hipLaunchKernelGGL(k_mg_residual_rows<T>, dim3(b.rblocks), dim3(64 * rows::WPB), 0, ctx->stream,
                           static_cast<const LevelJob<T>*>(b.jobs), b.rpre, b.n);
    else
        hipLaunchKernelGGL(k_mg_residual<T>, dim3(b.blocks), dim3(NT), 0, ctx->stream,
                           static_cast<const LevelJob<T>*>(b.jobs), b.pre, b.n);
    STK_LAUNCH_CHECK();
    return STK_OK;
}
template <typename T>
int mg_restrict(stk_ctx* ctx, const Batch& b, double omega) {
    if (!b.n) return STK_OK;
    hipLaunchKernelGGL(k_mg_restrict<T>, dim3(b.blocks), dim3(NT), 0, ctx->stream,
                       static_cast<const LevelJob<T>*>(b.jobs), b.pre, b.n, T(omega));
    STK_LAUNCH_CHECK();
    return STK_OK;
}
template <typename T>
int mg_prolong(stk_ctx* ctx, const Batch& b) {
    if (!b.n) return STK_OK;
    hipLaunchKernelGGL(k_mg_prolong<T>, dim3(b.blocks), dim3(NT), 0, ctx->stream,
                       static_cast<const LevelJob<T>*>(b.jobs), b.pre, b.n);
    STK_LAUNCH_CHECK();
    return STK_OK;
}
template <typename T>
int mg_jacobi_prolonged(stk_ctx* ctx, const Batch& b, double omega) {
    if (!b.n) return STK_OK;
    hipLaunchKernelGGL(k_mg_jacobi_prolonged<T>, dim3(b.blocks), dim3(NT), 0, ctx->stream,
                       static_cast<const LevelJob<T>*>(b.jobs), b.pre, b.n, T(omega));
    STK_LAUNCH_CHECK();
    return STK_OK;
}
template <typename T>
int mg_coarse(stk_ctx* ctx, const void* jobs, int n, int max_unknowns) {
    if (!n) return STK_OK;
    hipLaunchKernelGGL(k_mg_coarse<T>, dim3((unsigned)((max_unknowns + 63) / 64), (unsigned)n), dim3(64 * CW),
                       (size_t)(CW * 64 + max_unknowns) * sizeof(double), ctx->stream,
                       static_cast<const CoarseJob<T>*>(jobs));
    STK_LAUNCH_CHECK();
    return STK_OK;
}
template int mg_jacobi<double>(stk_ctx*, const Batch&, double, int);
template int mg_jacobi<float>(stk_ctx*, const Batch&, double, int);
template int mg_copy_wv<double>(stk_ctx*, const Batch&);
template int mg_copy_wv<float>(stk_ctx*, const Batch&);
template int mg_residual<double>(stk_ctx*, const Batch&);
template int mg_residual<float>(stk_ctx*, const Batch&);
template int mg_restrict<double>(stk_ctx*, const Batch&, double);
template int mg_restrict<float>(stk_ctx*, const Batch&, double);
template int mg_prolong<double>(stk_ctx*, const Batch&);
template int mg_prolong<float>(stk_ctx*, const Batch&);
template int mg_jacobi_prolonged<double>(stk_ctx*, const Batch&, double);
template int mg_jacobi_prolonged<float>(stk_ctx*, const Batch&, double);
template int mg_coarse<double>(stk_ctx*, const void*, int, int);
template int mg_coarse<float>(stk_ctx*, const void*, int, int);

template <typename T>
int vec_op(stk_ctx* ctx, const Batch& b, int op, const FcgState* st, double* part, bool z32) {
    if (!b.n) return STK_OK;
    if (z32)
        hipLaunchKernelGGL((k_vec<T, float>), dim3(b.blocks), dim3(NT), 0, ctx->stream,
                           static_cast<const VecJob*>(b.jobs), b.pre, b.n, op, st, part);
    else
        hipLaunchKernelGGL((k_vec<T, T>), dim3(b.blocks), dim3(NT), 0, ctx->stream, static_cast<const VecJob*>(b.jobs),
                           b.pre, b.n, op, st, part);
    STK_LAUNCH_CHECK();
    return STK_OK;
}
template int vec_op<double>(stk_ctx*, const Batch&, int, const FcgState*, double*, bool);

int fcg_apply_pq(stk_ctx* ctx, const Batch& apply, const FcgState* st, double* part) {
    if (!apply.n) return STK_OK;
    if (!apply.rpre) return set_error(STK_EINVAL, "internal: operator batch without row-streaming prefix");
    hipLaunchKernelGGL(k_fcg_apply_rows, dim3(apply.rblocks), dim3(64 * rows::WPB), 0, ctx->stream,
                       static_cast<const LevelJob<double>*>(apply.jobs), apply.rpre, apply.n, st, part);
    STK_LAUNCH_CHECK();
    return STK_OK;
}

int prec_cast(stk_ctx* ctx, const Batch& b, const FcgState* st) {
    if (!b.n) return STK_OK;
    hipLaunchKernelGGL(k_prec_cast, dim3(b.blocks), dim3(NT), 0, ctx->stream, static_cast<const XCastJob*>(b.jobs),
                       b.pre, b.n, st);
    STK_LAUNCH_CHECK();
    return STK_OK;
}
int vec_residual64_st(stk_ctx* ctx, const Batch& b, const FcgState* st, double* part) {
    if (!b.n) return STK_OK;
    hipLaunchKernelGGL(k_vec_res64, dim3(b.blocks), dim3(NT), 0, ctx->stream, static_cast<const VecJob*>(b.jobs), b.pre,
                       b.n, st, part);
    STK_LAUNCH_CHECK();
    return STK_OK;
}
int fcg_reduce(stk_ctx* ctx, const Batch& red, const double* part, double* sums, FcgState* st, int phase,
               FcgState* out) {
    if (!red.n) return STK_OK;
    if (!red.cpre) return set_error(STK_EINVAL, "internal: batch without reduction chunks");
    hipLaunchKernelGGL(k_fcg_reduce, dim3(red.n), dim3(256), 0, ctx->stream, red.pre, red.cpre, part, sums, st, phase,
                       out);
    STK_LAUNCH_CHECK();
    return STK_OK;
}

}  // namespace stk
