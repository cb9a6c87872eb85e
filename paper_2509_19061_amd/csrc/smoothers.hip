// Smoother kernels for gfx950: fused / split damped Jacobi, red-black
// Gauss-Seidel and RAS-type temporally blocked Jacobi (paper Sec. 4, Sec. 5,
// Alg. 2), plus the right-hand-side fold b = f - G p and a velocity copy.
#include <algorithm>

#include "stencil.hpp"
#include "stk_internal.hpp"

namespace stk {
namespace {

constexpr int BX = 64;  // threads along x (one wave per row segment)
constexpr int BY = 4;

template <typename T>
Grid<T> make_grid(const stk_grid* g, const FieldPtrs& f, double omega) {
    Grid<T> r;
    r.ec = static_cast<const T*>(f.eta_c);
    r.en = static_cast<const T*>(f.eta_n);
    r.bx = static_cast<const T*>(f.bx);
    r.by = static_cast<const T*>(f.by);
    r.ld = g->ld;
    r.nx = g->nx;
    r.ny = g->ny;
    r.idx = T(1.0 / g->dx);
    r.idy = T(1.0 / g->dy);
    r.omega = T(omega);
    return r;
}

inline dim3 cell_grid(const stk_grid* g) {
    return dim3((unsigned)((g->nx + 1 + BX - 1) / BX), (unsigned)((g->ny + 1 + BY - 1) / BY));
}

// ---------------------------------------------------------------- fold ----
// b = f - G p with (Gp)_x = -(p(i,j)-p(i-1,j))/dx, (Gp)_y = -(p(i,j)-p(i,j-1))/dy
// on the unknowns, 0 on the walls (Sec. 3.1, velocity subsystem M v + G p = f).
template <typename T>
__global__ __launch_bounds__(BX* BY) void k_fold_rhs(int nx, int ny, int64_t ld, T idx, T idy, const T* __restrict__ fx,
                                                    const T* __restrict__ fy, const T* __restrict__ p,
                                                    T* __restrict__ bx, T* __restrict__ by) {
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i > nx || j > ny) return;
    const int64_t k = (int64_t)j * ld + i;
    if (j < ny) bx[k] = is_vx_unknown(nx, ny, i, j) ? fx[k] + (p[k] - p[k - 1]) * idx : T(0);
    if (i < nx) by[k] = is_vy_unknown(nx, ny, i, j) ? fy[k] + (p[k] - p[k - ld]) * idy : T(0);
}

// ---------------------------------------------------------- split Jacobi --
// Separate vx and vy passes, both from the old iterate (Sec. 5 (ii)).
template <typename T>
__global__ __launch_bounds__(BX* BY) void k_jacobi_x(Grid<T> g, const T* __restrict__ vx, const T* __restrict__ vy,
                                                    T* __restrict__ ox) {
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i > g.nx || j >= g.ny) return;
    ox[(int64_t)j * g.ld + i] = is_vx_unknown(g.nx, g.ny, i, j) ? jac_vx_global(g, vx, vy, i, j) : T(0);
}
template <typename T>
__global__ __launch_bounds__(BX* BY) void k_jacobi_y(Grid<T> g, const T* __restrict__ vx, const T* __restrict__ vy,
                                                    T* __restrict__ oy) {
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i >= g.nx || j > g.ny) return;
    oy[(int64_t)j * g.ld + i] = is_vy_unknown(g.nx, g.ny, i, j) ? jac_vy_global(g, vx, vy, i, j) : T(0);
}

// ------------------------------------------------------------------ RBGS --
// Half-sweep of one component and one colour, in place.  Thread t of row j
// handles i = 2t + ((colour + j) & 1), so (i + j) mod 2 == colour.  Unknowns
// of one set do not couple, so reading neighbours in place is race-free.
template <typename T, int COMP>
__global__ __launch_bounds__(BX* BY) void k_rbgs(Grid<T> g, T* __restrict__ vx, T* __restrict__ vy, int colour) {
    const int t = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    const int i = 2 * t + ((colour + j) & 1);
    if (COMP == 0) {
        if (!is_vx_unknown(g.nx, g.ny, i, j)) return;
        const T v = jac_vx_global(g, vx, vy, i, j);
        vx[(int64_t)j * g.ld + i] = v;
    } else {
        if (!is_vy_unknown(g.nx, g.ny, i, j)) return;
        const T v = jac_vy_global(g, vx, vy, i, j);
        vy[(int64_t)j * g.ld + i] = v;
    }
}

// ------------------------------------------------------------ copy/zero --
template <typename T>
__global__ __launch_bounds__(BX* BY) void k_copy_velocity(int nx, int ny, int64_t ld, const T* __restrict__ vx,
                                                         const T* __restrict__ vy, T* __restrict__ ox,
                                                         T* __restrict__ oy) {
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i > nx || j > ny) return;
    const int64_t k = (int64_t)j * ld + i;
    if (j < ny) ox[k] = is_vx_unknown(nx, ny, i, j) ? vx[k] : T(0);
    if (i < nx) oy[k] = is_vy_unknown(nx, ny, i, j) ? vy[k] : T(0);
}

// Zero the Dirichlet wall entries of a velocity in place (in-place smoothers
// never touch them otherwise).
template <typename T>
__global__ __launch_bounds__(256) void k_zero_walls(int nx, int ny, int64_t ld, T* __restrict__ vx,
                                                    T* __restrict__ vy) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t < ny) {
        vx[(int64_t)t * ld] = T(0);
        vx[(int64_t)t * ld + nx] = T(0);
    }
    if (t < nx) {
        vy[t] = T(0);
        vy[(int64_t)ny * ld + t] = T(0);
    }
}

// ------------------------------------------------------------------- RAS --
// One outer iteration of RAS-type temporal blocking (Alg. 2), snapshot form.
// Workgroup = one tile.  Tile (tx, ty) owns cells [x0,x1) x [y0,y1), cut at
// positions congruent to the shift modulo the tile size.  Its extended region
// E = owned box grown by h (clipped) is relaxed kt times with everything
// outside E frozen at the snapshot; the owned unknowns are written back.
//
// LDS holds the velocity of the window [X0-1, X1] x [Y0-1, Y1] (E plus a
// one-cell ring; cells outside the domain hold 0), so one HBM read of the
// tile serves all kt sweeps.  Each sweep computes the new values of a
// thread's cells into registers, then (after a barrier) stores them.
constexpr int RAS_NT = 1024;

template <typename T, int MAXC>
__global__ __launch_bounds__(RAS_NT) void k_ras(Grid<T> g, const T* __restrict__ vx, const T* __restrict__ vy,
                                                T* __restrict__ ox, T* __restrict__ oy, int Tx, int Ty, int h, int kt,
                                                int sx, int sy) {
    extern __shared__ unsigned char smem_raw[];
    const int nx = g.nx, ny = g.ny;
    const int64_t ld = g.ld;
    const int x0 = max(0, sx + ((int)blockIdx.x - 1) * Tx), x1 = min(nx, sx + (int)blockIdx.x * Tx);
    const int y0 = max(0, sy + ((int)blockIdx.y - 1) * Ty), y1 = min(ny, sy + (int)blockIdx.y * Ty);
    if (x0 >= x1 || y0 >= y1) return;  // empty tile (whole workgroup leaves)
    const int X0 = max(x0 - h, 0), X1 = min(x1 + h, nx), Y0 = max(y0 - h, 0), Y1 = min(y1 + h, ny);
    const int ox0 = X0 - 1, oy0 = Y0 - 1;  // window origin
    const int W = X1 - X0 + 2, H = Y1 - Y0 + 2;
    T* sxv = reinterpret_cast<T*>(smem_raw);
    T* syv = sxv + W * H;
    const int tid = threadIdx.x;

    for (int c = tid; c < W * H; c += RAS_NT) {
        const int i = ox0 + c % W, j = oy0 + c / W;
        sxv[c] = ldvx(vx, ld, nx, ny, i, j);
        syv[c] = ldvy(vy, ld, nx, ny, i, j);
    }
    __syncthreads();

    const int EW = X1 - X0, ne = EW * (Y1 - Y0);
    for (int s = 0; s < kt; ++s) {
        T nvx[MAXC], nvy[MAXC];
#pragma unroll
        for (int m = 0; m < MAXC; ++m) {
            const int e = tid + m * RAS_NT;
            if (e < ne) {
                const int i = X0 + e % EW, j = Y0 + e / EW;
                const int l = (j - oy0) * W + (i - ox0);
                if (is_vx_unknown(nx, ny, i, j)) {
                    nvx[m] = jac_vx<T>(sxv[l], sxv[l - 1], sxv[l + 1], sxv[l - W], sxv[l + W], syv[l], syv[l - 1],
                                       syv[l + W], syv[l + W - 1], g.ec[(int64_t)j * ld + i - 1],
                                       g.ec[(int64_t)j * ld + i], ldenh(g, i, j), ldenh(g, i, j + 1),
                                       g.bx[(int64_t)j * ld + i], g.omega, g.idx, g.idy);
                }
                if (is_vy_unknown(nx, ny, i, j)) {
                    nvy[m] = jac_vy<T>(syv[l], syv[l - 1], syv[l + 1], syv[l - W], syv[l + W], sxv[l], sxv[l + 1],
                                       sxv[l - W], sxv[l - W + 1], g.ec[(int64_t)(j - 1) * ld + i],
                                       g.ec[(int64_t)j * ld + i], ldenh(g, i, j), ldenh(g, i + 1, j),
                                       g.by[(int64_t)j * ld + i], g.omega, g.idx, g.idy);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < MAXC; ++m) {
            const int e = tid + m * RAS_NT;
            if (e < ne) {
                const int i = X0 + e % EW, j = Y0 + e / EW;
                const int l = (j - oy0) * W + (i - ox0);
                if (is_vx_unknown(nx, ny, i, j)) sxv[l] = nvx[m];
                if (is_vy_unknown(nx, ny, i, j)) syv[l] = nvy[m];
            }
        }
        __syncthreads();
    }

    const int OW = x1 - x0, no = OW * (y1 - y0);
    for (int c = tid; c < no; c += RAS_NT) {
        const int i = x0 + c % OW, j = y0 + c / OW;
        const int l = (j - oy0) * W + (i - ox0);
        const int64_t k = (int64_t)j * ld + i;
        ox[k] = is_vx_unknown(nx, ny, i, j) ? sxv[l] : T(0);
        oy[k] = is_vy_unknown(nx, ny, i, j) ? syv[l] : T(0);
    }
    // walls that belong to no cell: right column of vx, top row of vy
    if (x1 == nx)
        for (int j = y0 + tid; j < y1; j += RAS_NT) ox[(int64_t)j * ld + nx] = T(0);
    if (y1 == ny)
        for (int i = x0 + tid; i < x1; i += RAS_NT) oy[(int64_t)ny * ld + i] = T(0);
}

// LDS of one tile: the window is at most (min(T + 2h, n) + 2) cells wide per axis.
template <typename T>
size_t ras_bytes(const stk_grid* g, int tile_x, int tile_y, int halo) {
    const int64_t w = std::min<int64_t>((int64_t)tile_x + 2 * (int64_t)halo, g->nx) + 2;
    const int64_t hh = std::min<int64_t>((int64_t)tile_y + 2 * (int64_t)halo, g->ny) + 2;
    return (size_t)2 * sizeof(T) * (size_t)w * (size_t)hh;
}

template <typename T, int MAXC>
int launch_ras_t(stk_ctx* ctx, const stk_grid* g, const Grid<T>& gg, int Tx, int Ty, int h, int kt, int sx, int sy,
                 const T* vx, const T* vy, T* ox, T* oy) {
    const size_t lds = ras_bytes<T>(g, Tx, Ty, h);
    static size_t attr_set[64] = {};
    const int dev = ctx->device < 64 ? ctx->device : 63;
    if (lds > attr_set[dev]) {
        STK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_ras<T, MAXC>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr_set[dev] = lds;
    }
    const dim3 grid((unsigned)((g->nx + Tx - 1) / Tx + 1), (unsigned)((g->ny + Ty - 1) / Ty + 1));
    hipLaunchKernelGGL((k_ras<T, MAXC>), grid, dim3(RAS_NT), lds, ctx->stream, gg, vx, vy, ox, oy, Tx, Ty, h, kt, sx,
                       sy);
    STK_HIP(hipGetLastError());
    return STK_OK;
}

template <typename T>
int launch_ras_dispatch(stk_ctx* ctx, const stk_grid* g, const FieldPtrs& f, double omega, int Tx, int Ty, int h,
                        int kt, int sx, int sy, const void* vx, const void* vy, void* ox, void* oy) {
    const Grid<T> gg = make_grid<T>(g, f, omega);
    const long ne = (long)std::min(Tx + 2 * h, g->nx) * (long)std::min(Ty + 2 * h, g->ny);
    const long per = (ne + RAS_NT - 1) / RAS_NT;
    auto a = static_cast<const T*>(vx);
    auto b = static_cast<const T*>(vy);
    auto c = static_cast<T*>(ox);
    auto d = static_cast<T*>(oy);
    if (per <= 2) return launch_ras_t<T, 2>(ctx, g, gg, Tx, Ty, h, kt, sx, sy, a, b, c, d);
    if (per <= 4) return launch_ras_t<T, 4>(ctx, g, gg, Tx, Ty, h, kt, sx, sy, a, b, c, d);
    if (per <= 8) return launch_ras_t<T, 8>(ctx, g, gg, Tx, Ty, h, kt, sx, sy, a, b, c, d);
    if (per <= 16) return launch_ras_t<T, 16>(ctx, g, gg, Tx, Ty, h, kt, sx, sy, a, b, c, d);
    if (per <= 32) return launch_ras_t<T, 32>(ctx, g, gg, Tx, Ty, h, kt, sx, sy, a, b, c, d);
    return set_error(STK_EUNSUPPORTED, "RAS extended tile of %ld cells exceeds the per-workgroup limit", ne);
}

}  // namespace

int ras_lds_bytes(stk_dtype dt, const stk_grid* g, int tile_x, int tile_y, int halo, size_t* bytes) {
    *bytes = dt == STK_F64 ? ras_bytes<double>(g, tile_x, tile_y, halo) : ras_bytes<float>(g, tile_x, tile_y, halo);
    return STK_OK;
}

int launch_fold_rhs(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const void* fx, const void* fy, const void* p,
                    void* bx, void* by) {
    const dim3 grid = cell_grid(g), block(BX, BY);
    if (dt == STK_F64)
        hipLaunchKernelGGL(k_fold_rhs<double>, grid, block, 0, ctx->stream, g->nx, g->ny, g->ld, 1.0 / g->dx,
                           1.0 / g->dy, (const double*)fx, (const double*)fy, (const double*)p, (double*)bx,
                           (double*)by);
    else
        hipLaunchKernelGGL(k_fold_rhs<float>, grid, block, 0, ctx->stream, g->nx, g->ny, g->ld, float(1.0 / g->dx),
                           float(1.0 / g->dy), (const float*)fx, (const float*)fy, (const float*)p, (float*)bx,
                           (float*)by);
    STK_HIP(hipGetLastError());
    return STK_OK;
}

// Fused Jacobi (one pass updates vx and vy of a cell, Sec. 4.1): the
// row-streaming kernel (rowstream.hip).
int launch_jacobi_fused(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const FieldPtrs& f, double omega,
                        const void* vx, const void* vy, void* ox, void* oy) {
    return launch_jacobi_rows(ctx, dt, g, f, omega, vx, vy, ox, oy);
}

int launch_jacobi_split(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const FieldPtrs& f, double omega,
                        const void* vx, const void* vy, void* ox, void* oy) {
    const dim3 grid = cell_grid(g), block(BX, BY);
    if (dt == STK_F64) {
        const Grid<double> gg = make_grid<double>(g, f, omega);
        hipLaunchKernelGGL(k_jacobi_x<double>, grid, block, 0, ctx->stream, gg, (const double*)vx, (const double*)vy,
                           (double*)ox);
        hipLaunchKernelGGL(k_jacobi_y<double>, grid, block, 0, ctx->stream, gg, (const double*)vx, (const double*)vy,
                           (double*)oy);
    } else {
        const Grid<float> gg = make_grid<float>(g, f, omega);
        hipLaunchKernelGGL(k_jacobi_x<float>, grid, block, 0, ctx->stream, gg, (const float*)vx, (const float*)vy,
                           (float*)ox);
        hipLaunchKernelGGL(k_jacobi_y<float>, grid, block, 0, ctx->stream, gg, (const float*)vx, (const float*)vy,
                           (float*)oy);
    }
    STK_HIP(hipGetLastError());
    return STK_OK;
}

int launch_zero_walls(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, void* vx, void* vy) {
    const int n = std::max(g->nx, g->ny);
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (dt == STK_F64)
        hipLaunchKernelGGL(k_zero_walls<double>, grid, block, 0, ctx->stream, g->nx, g->ny, g->ld, (double*)vx,
                           (double*)vy);
    else
        hipLaunchKernelGGL(k_zero_walls<float>, grid, block, 0, ctx->stream, g->nx, g->ny, g->ld, (float*)vx,
                           (float*)vy);
    STK_HIP(hipGetLastError());
    return STK_OK;
}

int launch_rbgs(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const FieldPtrs& f, double omega, void* vx, void* vy) {
    const dim3 grid((unsigned)((g->nx / 2 + 1 + BX - 1) / BX), (unsigned)((g->ny + 1 + BY - 1) / BY)), block(BX, BY);
    for (int comp = 0; comp < 2; ++comp)
        for (int colour = 0; colour < 2; ++colour) {
            if (dt == STK_F64) {
                const Grid<double> gg = make_grid<double>(g, f, omega);
                if (comp == 0)
                    hipLaunchKernelGGL((k_rbgs<double, 0>), grid, block, 0, ctx->stream, gg, (double*)vx, (double*)vy,
                                       colour);
                else
                    hipLaunchKernelGGL((k_rbgs<double, 1>), grid, block, 0, ctx->stream, gg, (double*)vx, (double*)vy,
                                       colour);
            } else {
                const Grid<float> gg = make_grid<float>(g, f, omega);
                if (comp == 0)
                    hipLaunchKernelGGL((k_rbgs<float, 0>), grid, block, 0, ctx->stream, gg, (float*)vx, (float*)vy,
                                       colour);
                else
                    hipLaunchKernelGGL((k_rbgs<float, 1>), grid, block, 0, ctx->stream, gg, (float*)vx, (float*)vy,
                                       colour);
            }
        }
    STK_HIP(hipGetLastError());
    return STK_OK;
}

int launch_ras(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const FieldPtrs& f, double omega, int tile_x, int tile_y,
               int halo, int kt, int sx, int sy, const void* vx, const void* vy, void* ox, void* oy) {
    size_t lds = 0;
    ras_lds_bytes(dt, g, tile_x, tile_y, halo, &lds);
    if (lds > (size_t)ctx->lds_max)
        return set_error(STK_EUNSUPPORTED, "RAS tile %dx%d with halo %d needs %zu bytes of LDS (limit %d)", tile_x,
                         tile_y, halo, lds, ctx->lds_max);
    if (ctx->ras_kernel != 1) {
        bool done = false;
        STK_TRY(launch_ras_stream(ctx, dt, g, f, omega, tile_x, tile_y, halo, kt, sx, sy, vx, vy, ox, oy, &done));
        if (done) return STK_OK;
        if (ctx->ras_kernel == 2)
            return set_error(STK_EUNSUPPORTED, "streaming RAS kernel cannot take tile %dx%d, halo %d, k %d", tile_x,
                             tile_y, halo, kt);
    }
    if (dt == STK_F64) return launch_ras_dispatch<double>(ctx, g, f, omega, tile_x, tile_y, halo, kt, sx, sy, vx, vy, ox, oy);
    return launch_ras_dispatch<float>(ctx, g, f, omega, tile_x, tile_y, halo, kt, sx, sy, vx, vy, ox, oy);
}

int launch_copy_velocity(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const void* vx, const void* vy, void* ox,
                         void* oy) {
    const dim3 grid = cell_grid(g), block(BX, BY);
    if (dt == STK_F64)
        hipLaunchKernelGGL(k_copy_velocity<double>, grid, block, 0, ctx->stream, g->nx, g->ny, g->ld,
                           (const double*)vx, (const double*)vy, (double*)ox, (double*)oy);
    else
        hipLaunchKernelGGL(k_copy_velocity<float>, grid, block, 0, ctx->stream, g->nx, g->ny, g->ld, (const float*)vx,
                           (const float*)vy, (float*)ox, (float*)oy);
    STK_HIP(hipGetLastError());
    return STK_OK;
}

}  // namespace stk
