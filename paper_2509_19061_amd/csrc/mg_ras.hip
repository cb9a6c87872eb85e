// RAS-type temporal blocking (Sec. 4.3, Alg. 2, snapshot semantics) on the
// stored Galerkin stencils of the coarse multigrid levels: the coarse half
// of the paper's mixed smoother (Sec. 6.3: Jacobi on the finest level, RAS
// on all coarser ones).
//
// One workgroup per tile of one instance (work-list over (instance, tile)):
// the tile's owned cells grown by the overlap h (clipped) form the region E;
// its unknowns (the left-face vx and bottom-face vy of each cell) take kt
// damped-Jacobi sweeps in LDS while every value outside E keeps the snapshot;
// the owned unknowns are written to the partner vector.  A Galerkin row
// couples to neighbours at most two cells away, so the LDS window is E grown
// by two cells; values outside the grid and on the walls are 0.  The sweep
// computes each row exactly as the coarse Jacobi kernel does (same slot
// order, same coefficients, same update), so an overlap of at least
// 2 (kt - 1) reproduces kt Jacobi sweeps bit for bit.
#include "coarse_stencil.hpp"
#include "mg_host.hpp"

namespace stk {
namespace {

constexpr int RT = 256;  // threads per workgroup
constexpr int REACH = 2;  // Galerkin stencil reach in cells

__device__ __forceinline__ int find_tile_inst(const int* __restrict__ pre, int n, int b) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// (A w) at the unknown (a, i, j) with w read from the LDS window (origin
// (wx0, wy0), row stride ws; component c of buffer at base + c * plane_w),
// coefficients from the stored planes (stencil_av_l: the slot order of every
// stored-stencil kernel).
template <typename T>
struct WindowPair {
    const T* win;
    int plane_w, ws, wx0, wy0;
    __device__ __forceinline__ T operator()(int c, int i, int j) const {
        return win[c * plane_w + (j - wy0) * ws + (i - wx0)];
    }
};
template <typename T>
__device__ __forceinline__ T stencil_av_window(const T* __restrict__ st, int64_t plane, int a, const T* win,
                                               int plane_w, int ws, int wx0, int wy0, int64_t ld, int nx, int ny,
                                               int i, int j, T& diag) {
    return stencil_av_l<T>(st, plane, a, WindowPair<T>{win, plane_w, ws, wx0, wy0}, ld, nx, ny, i, j, diag);
}

// dir 0: (v) -> (w); dir 1: (w) -> (v).  Tiles T x T cells cut at multiples
// of T; window row stride ws >= T + 2h + 2 REACH + 1.
template <typename T>
__global__ __launch_bounds__(RT) void k_mg_ras(const LevelJob<T>* __restrict__ jobs, const int* __restrict__ pre,
                                               int n, int tile, int h, int kt, T omega, int dir, int ws) {
    extern __shared__ unsigned char smem_raw[];
    T* win = reinterpret_cast<T*>(smem_raw);
    const int inst = find_tile_inst(pre, n, (int)blockIdx.x);
    const LevelJob<T>& J = jobs[inst];
    const int nx = J.nx, ny = J.ny;
    const int64_t ld = J.ld;
    const int tl = (int)blockIdx.x - pre[inst];
    const int ntx = (nx + tile - 1) / tile;
    const int x0 = (tl % ntx) * tile, y0 = (tl / ntx) * tile;
    const int x1 = min(x0 + tile, nx), y1 = min(y0 + tile, ny);
    const int X0 = max(x0 - h, 0), X1 = min(x1 + h, nx), Y0 = max(y0 - h, 0), Y1 = min(y1 + h, ny);
    // window: cells (i, j), i in [X0 - R, X1 + R], j in [Y0 - R, Y1 + R]
    const int wx0 = X0 - REACH, wy0 = Y0 - REACH;
    const int ww = X1 - X0 + 2 * REACH + 1, wh = Y1 - Y0 + 2 * REACH + 1;
    const int plane_w = ws * ws;  // one component
    const T* sx = dir ? J.wx : J.vx;
    const T* sy = dir ? J.wy : J.vy;
    T* ox = dir ? J.vx : J.wx;
    T* oy = dir ? J.vy : J.wy;
    // snapshot into both buffers (frozen values are never rewritten)
    for (int e = threadIdx.x; e < ww * wh; e += RT) {
        const int ci = e % ww, cj = e / ww;
        const int i = wx0 + ci, j = wy0 + cj;
        const T vx = ldvx<T>(sx, ld, nx, ny, i, j), vy = ldvy<T>(sy, ld, nx, ny, i, j);
        const int o = cj * ws + ci;
        win[o] = vx;
        win[plane_w + o] = vy;
        win[2 * plane_w + o] = vx;
        win[3 * plane_w + o] = vy;
    }
    __syncthreads();
    // unknowns of E: vx(i, j) for cells of E with 1 <= i <= nx - 1, vy(i, j) with 1 <= j <= ny - 1
    const int ew = X1 - X0, eh = Y1 - Y0, ne = ew * eh;
    for (int s = 0; s < kt; ++s) {
        const T* cur = win + (s & 1) * 2 * plane_w;
        T* nxt = win + ((s & 1) ^ 1) * 2 * plane_w;
        for (int e = threadIdx.x; e < 2 * ne; e += RT) {
            const int a = e >= ne ? 1 : 0, c = e - a * ne;
            const int i = X0 + c % ew, j = Y0 + c / ew;
            if (a == 0 ? !is_vx_unknown(nx, ny, i, j) : !is_vy_unknown(nx, ny, i, j)) continue;
            const int o = (j - wy0) * ws + (i - wx0);
            T d;
            const T av = stencil_av_window<T>(J.st, J.plane, a, cur, plane_w, ws, wx0, wy0, ld, nx, ny, i, j, d);
            const int64_t k = (int64_t)j * ld + i;
            nxt[a * plane_w + o] = jac_step<T>(cur[a * plane_w + o], omega / d, (a == 0 ? J.bx : J.by)[k], -av);
        }
        __syncthreads();
    }
    // owned unknowns (and the walls of the tiles at the right and top edges) to the partner
    const T* fin = win + (kt & 1) * 2 * plane_w;
    const int ow = x1 - x0 + 1, oh = y1 - y0 + 1;  // one more column / row for the right and top walls
    for (int e = threadIdx.x; e < ow * oh; e += RT) {
        const int i = x0 + e % ow, j = y0 + e / ow;
        const int o = (j - wy0) * ws + (i - wx0);
        const int64_t k = (int64_t)j * ld + i;
        const bool in_x = i < x1 || i == nx, in_y = j < y1 || j == ny;
        if (in_x && j < y1 && j < ny) ox[k] = is_vx_unknown(nx, ny, i, j) ? fin[o] : T(0);
        if (in_y && i < x1 && i < nx) oy[k] = is_vy_unknown(nx, ny, i, j) ? fin[plane_w + o] : T(0);
    }
}

}  // namespace

size_t mg_ras_lds_bytes(int tile, int h, size_t es) {
    const size_t ws = (size_t)tile + 2 * (size_t)h + 2 * REACH + 1;
    return 4 * ws * ws * es;
}

int mg_ras_tiles(int nx, int ny, int tile) { return ((nx + tile - 1) / tile) * ((ny + tile - 1) / tile); }

template <typename T>
int mg_ras(stk_ctx* ctx, const Batch& b, int tile, int h, int kt, double omega, int dir) {
    if (!b.n || kt < 1) return STK_OK;
    const int ws = tile + 2 * h + 2 * REACH + 1;
    const size_t lds = mg_ras_lds_bytes(tile, h, sizeof(T));
    static size_t attr_set[64] = {};
    const int dev = ctx->device < 64 ? ctx->device : 63;
    if (lds > attr_set[dev]) {
        STK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mg_ras<T>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr_set[dev] = lds;
    }
    hipLaunchKernelGGL(k_mg_ras<T>, dim3((unsigned)b.blocks), dim3(RT), lds, ctx->stream,
                       static_cast<const LevelJob<T>*>(b.jobs), b.pre, b.n, tile, h, kt, T(omega), dir, ws);
    STK_HIP(hipGetLastError());
    return STK_OK;
}
template int mg_ras<double>(stk_ctx*, const Batch&, int, int, int, double, int);
template int mg_ras<float>(stk_ctx*, const Batch&, int, int, int, double, int);

}  // namespace stk
