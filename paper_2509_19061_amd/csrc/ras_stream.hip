// RAS-type temporal blocking (paper Sec. 4.3, Alg. 2), streaming kernel for
// gfx950.
//
// Semantics are those of the LDS-window kernel: one outer iteration, tiles cut
// at positions congruent to the shift modulo the tile size, each tile's
// extended region E (owned box grown by h, clipped) relaxed kt times with the
// one-cell ring outside E frozen at the snapshot, owned cells written back.
//
// Execution: one workgroup streams up a column of NT tiles.  The rows of the
// tiles' windows (ring row, E rows, ring row; tile after tile) form one
// "virtual" row stream; ring rows never update, so the stencil of an E row
// never reaches into another tile's rows and the stream need not drain
// between tiles.  Lane (c, s) owns window column c at sweep level s (1..kt);
// at step t level s relaxes virtual row t - 1 - 2s, two rows behind level
// s - 1, so all levels advance together with ONE barrier per step.
//   * level 0 (the snapshot) and the tile's viscosities and right-hand side
//     are read from HBM once, P rows ahead through a per-thread register
//     FIFO, into LDS row rings; every level re-uses them from LDS;
//   * omega / diag(-M) is computed once per cell (not once per sweep);
//   * each lane keeps a 3 x 3 window of level s-1 values in registers and
//     reads only the incoming row from LDS;
//   * level kt writes the owned cells straight to HBM.
// The update calls the same stencil functions as every other smoother, so
// results are bit-identical to fused Jacobi wherever RAS equals Jacobi^kt.
#include <algorithm>

#include "stencil.hpp"
#include "stk_internal.hpp"

namespace stk {
namespace {

constexpr int P = 6;     // prefetch depth in rows (also the unroll factor; multiple of 3)
constexpr int RS0 = 8;   // level-0 ring rows
constexpr int RS = 4;    // level >= 1 ring rows
constexpr int YMASK = (1 << 27) - 1;
constexpr int F_RING = 1 << 29, F_OWNED = 1 << 28, F_TOPWALL = 1 << 27;
enum { CF_EC = 0, CF_EN, CF_BX, CF_BY, CF_GX, CF_GY, CF_N };

struct RasArgs {
    int Tx, Ty, h, kt, sx, sy;
    int NT;    // tiles per workgroup along y
    int Wm;    // window width bound: min(Tx + 2h, nx) + 2
    int Vmax;  // virtual rows bound: NT * (min(Ty + 2h, ny) + 2)
};

// Workgroup barrier that orders LDS only.  __syncthreads() also waits for
// every outstanding global access (vmcnt(0) on gfx9), which would drain the
// load FIFO each row; lanes here communicate through LDS alone.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__host__ __device__ inline size_t align16(size_t b) { return (b + 15) & ~size_t(15); }

constexpr int WS = 96;  // LDS row stride (elements): window width bound, fixed so offsets fold

template <typename T>
size_t stream_lds_bytes(const RasArgs& a) {
    const size_t n = (size_t)RS0 * 2 * WS + (size_t)(a.kt - 1) * RS * 2 * WS + (size_t)(2 * a.kt + 2) * CF_N * WS;
    return align16((size_t)(a.Vmax + 1) * sizeof(int)) + n * sizeof(T);
}

// MMAX = HBM loads per thread per row (6 fields x Wm / threads).
template <typename T, int NTMAX, int MMAX>
__global__ __launch_bounds__(NTMAX) void k_ras_stream(Grid<T> g, const T* __restrict__ vx, const T* __restrict__ vy,
                                                      T* __restrict__ ox, T* __restrict__ oy, RasArgs a) {
    extern __shared__ unsigned char smem_raw[];
    const int nx = g.nx, ny = g.ny;
    const int64_t ld = g.ld;
    const int kt = a.kt, Wm = a.Wm, RC = 2 * a.kt + 2;
    const int NTHR = blockDim.x, tid = threadIdx.x;

    // ---- this workgroup's tile column and window columns
    const int x0 = max(0, a.sx + ((int)blockIdx.x - 1) * a.Tx), x1 = min(nx, a.sx + (int)blockIdx.x * a.Tx);
    if (x0 >= x1) return;  // empty tile column: the whole workgroup leaves
    const int X0 = max(x0 - a.h, 0), X1 = min(x1 + a.h, nx);
    const int W = X1 - X0 + 2;  // window column c <-> cell column i = X0 - 1 + c
    const int ci0 = X0 - 1;

    int* vtab = reinterpret_cast<int*>(smem_raw);
    T* s0 = reinterpret_cast<T*>(smem_raw + align16((size_t)(a.Vmax + 1) * sizeof(int)));
    T* s1 = s0 + RS0 * 2 * WS;
    T* cf = s1 + (kt - 1) * RS * 2 * WS;

    // ---- virtual row table: y + 1 and flags, tile after tile
    if (tid == 0) {
        const int nty = (ny + a.Ty - 1) / a.Ty + 1;
        const int tyb = blockIdx.y * a.NT, tye = min(nty, tyb + a.NT);
        int v = 0;
        for (int ty = tyb; ty < tye; ++ty) {
            const int y0 = max(0, a.sy + (ty - 1) * a.Ty), y1 = min(ny, a.sy + ty * a.Ty);
            if (y0 >= y1) continue;
            const int Y0 = max(y0 - a.h, 0), Y1 = min(y1 + a.h, ny);
            for (int y = Y0 - 1; y <= Y1; ++y) {
                int f = y + 1;
                if (y == Y0 - 1 || y == Y1) f |= F_RING;
                if (y >= y0 && y < y1) f |= F_OWNED;
                if (y == ny && y1 == ny) f |= F_TOPWALL;
                vtab[v++] = f;
            }
        }
        vtab[a.Vmax] = v;
    }
    lds_barrier();
    const int V = vtab[a.Vmax];
    if (V == 0) return;

    // ---- lane roles
    const int c = tid % Wm, s = tid / Wm + 1;  // column, sweep level
    const bool lane_on = (s <= kt) && (c < W);
    const int i = ci0 + c;
    const bool ecol = c >= 1 && c <= W - 2;  // column inside E (else frozen ring)
    // this lane's column in the level s-1 ring, the level s ring and the coefficient ring
    // (idle lanes, s > kt, read as level kt so that every LDS address stays in bounds)
    const int sl = min(s, kt);
    const T* prevc = ((sl == 1) ? s0 : s1 + (sl - 2) * RS * 2 * WS) + c;
    const int prs = (sl == 1) ? RS0 - 1 : RS - 1;
    T* minec = s1 + (sl - 1) * RS * 2 * WS + c;
    const T* cfc = cf + c;
    int sa = RC - 1 - 2 * sl;  // ring slot of row t - 1 - 2s at t = 0
    if (sa < 0) sa += RC;

    // ---- HBM row loads: task m of this thread = (field f, column cq), decoded
    // once into a base pointer, a column predicate, a valid row range and an
    // LDS destination.
    const int nq = 6 * Wm;
    const T* tbase[MMAX];
    T* tdst[MMAX];
    int tylo[MMAX];
    bool tok[MMAX], ts0[MMAX];
#pragma unroll
    for (int m = 0; m < MMAX; ++m) {
        const int q = tid + m * NTHR;
        const int f = q < nq ? q / Wm : 0, cq = q < nq ? q - f * Wm : 0, ii = ci0 + cq;
        // field f: 0 vx, 1 vy, 2 eta_c, 3 eta_n (boundary nodes 0), 4 bx, 5 by
        const T* b = f == 0 ? vx : f == 1 ? vy : f == 2 ? g.ec : f == 3 ? g.en : f == 4 ? g.bx : g.by;
        const bool xface = (f == 0 || f == 4), yface = (f == 1 || f == 5);
        const bool colok = (xface || f == 3) ? (ii >= 1 && ii <= nx - 1) : (ii >= 0 && ii <= nx - 1);
        tok[m] = q < nq && colok;
        tbase[m] = b + (colok ? ii : 0);
        tylo[m] = (yface || f == 3) ? 1 : 0;  // vy, by, eta_n-hat live on rows 1..ny-1
        ts0[m] = f < 2;
        tdst[m] = q >= nq ? nullptr : (f < 2 ? s0 + f * WS + cq : cf + (f - 2) * WS + cq);
    }
    auto load_row = [&](int m, int y, int64_t yoff) -> T {
        return (tok[m] && y >= tylo[m] && y <= ny - 1) ? tbase[m][yoff] : T(0);
    };
    T fifo[P][MMAX];
#pragma unroll
    for (int u = 0; u < P; ++u) {
        const int y = u < V ? (__builtin_amdgcn_readfirstlane(vtab[u]) & YMASK) - 1 : -1;
#pragma unroll
        for (int m = 0; m < MMAX; ++m) fifo[u][m] = load_row(m, y, (int64_t)y * ld);
    }

    // window of level s-1 values at columns c-1, c, c+1: rows a-1, a, a+1
    T wx[3][3], wy[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) wx[r][q] = wy[r][q] = T(0);
    T ec_prev = T(0), en_prev = T(0);  // eta_c(c, a-1), eta_n-hat(c, a)

    // steps past V + 2kt are no-ops (their LDS stores land in ring slots no level
    // reads), so the loop runs whole groups of P steps without per-step guards
    const int nsteps = V + 2 * kt + 1;
    int rA = 0;  // t % RC
    for (int t0 = 0; t0 < nsteps; t0 += P) {
#pragma unroll
        for (int u = 0; u < P; ++u) {
            const int t = t0 + u;
            {
                // (A) row t: FIFO -> LDS; issue the HBM loads of row t + P
                {
                    const int o0 = (t & (RS0 - 1)) * 2 * WS, oc = rA * CF_N * WS;
#pragma unroll
                    for (int m = 0; m < MMAX; ++m)
                        if (tdst[m]) tdst[m][ts0[m] ? o0 : oc] = fifo[u][m];
                }
                {
                    const int y = (t + P < V) ? (__builtin_amdgcn_readfirstlane(vtab[t + P]) & YMASK) - 1 : -1;
                    const int64_t yoff = (int64_t)y * ld;
#pragma unroll
                    for (int m = 0; m < MMAX; ++m) fifo[u][m] = load_row(m, y, yoff);
                }
                // (B) omega / diag for the E cells of row t - 2 (lanes < Wm: vx, next Wm: vy;
                //     diag_y is diag_x with the roles of x and y exchanged)
                {
                    const int r = t - 2;
                    if (r >= 0 && r < V && tid < 2 * Wm) {
                        const int fl = __builtin_amdgcn_readfirstlane(vtab[r]);
                        const bool cy = tid >= Wm;
                        const int cq = cy ? tid - Wm : tid;
                        const int y = (fl & YMASK) - 1, ii = ci0 + cq;
                        const int sr = rA >= 2 ? rA - 2 : rA + RC - 2;
                        const int sm = sr >= 1 ? sr - 1 : RC - 1, sp = sr + 1 == RC ? 0 : sr + 1;
                        const T* row = cf + sr * CF_N * WS + cq;
                        const bool live = !(fl & F_RING) && cq >= 1 && cq <= W - 2 &&
                                          (cy ? is_vy_unknown(nx, ny, ii, y) : is_vx_unknown(nx, ny, ii, y));
                        const T e0 = cy ? cf[sm * CF_N * WS + CF_EC * WS + cq] : row[CF_EC * WS - 1];
                        const T e1 = row[CF_EC * WS];
                        const T n0 = row[CF_EN * WS];
                        const T n1 = cy ? row[CF_EN * WS + 1] : cf[sp * CF_N * WS + CF_EN * WS + cq];
                        const T d = diag_x<T>(e0, e1, n0, n1, cy ? g.idy : g.idx, cy ? g.idx : g.idy);
                        const T gv = live ? g.omega / d : T(0);
                        cf[sr * CF_N * WS + (cy ? CF_GY : CF_GX) * WS + cq] = gv;
                    }
                }
                // (C) level s relaxes row a = t - 1 - 2s
                {
                    const int a2 = t - 1 - 2 * sl;
                    // window rows 0, 1, 2 = a-1, a, a+1: shifted every step so that, unrolled,
                    // the shift is a register renaming
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        wx[0][q] = wx[1][q];
                        wx[1][q] = wx[2][q];
                        wy[0][q] = wy[1][q];
                        wy[1][q] = wy[2][q];
                    }
                    const bool rin = a2 >= -1 && a2 + 1 < V;
                    const T* pr = prevc + ((a2 + 1) & prs) * (2 * WS);
                    wx[2][0] = rin ? pr[-1] : T(0);
                    wx[2][1] = rin ? pr[0] : T(0);
                    wx[2][2] = rin ? pr[1] : T(0);
                    wy[2][0] = rin ? pr[WS - 1] : T(0);
                    wy[2][1] = rin ? pr[WS] : T(0);
                    wy[2][2] = rin ? pr[WS + 1] : T(0);
                    const int sa1 = (sa + 1 == RC) ? 0 : sa + 1;
                    const bool ain = a2 >= 0 && a2 < V;
                    const int fl = vtab[ain ? a2 : 0];
                    const int y = (fl & YMASK) - 1;
                    const T* row = cfc + sa * (CF_N * WS);
                    const T ecA = row[CF_EC * WS];
                    const T ent = (a2 + 1 < V) ? cfc[sa1 * (CF_N * WS) + CF_EN * WS] : T(0);
                    const bool upd = !(fl & F_RING) && ecol;
                    const T mx = mv_x<T>(wx[1][1], wx[1][0], wx[1][2], wx[0][1], wx[2][1], wy[1][1], wy[1][0],
                                         wy[2][1], wy[2][0], row[CF_EC * WS - 1], ecA, en_prev, ent, g.idx, g.idy);
                    const T my = mv_y<T>(wy[1][1], wy[1][0], wy[1][2], wy[0][1], wy[2][1], wx[1][1], wx[1][2],
                                         wx[0][1], wx[0][2], ec_prev, ecA, en_prev, row[CF_EN * WS + 1], g.idx,
                                         g.idy);
                    const T ux = jac_step<T>(wx[1][1], row[CF_GX * WS], row[CF_BX * WS], mx);
                    const T uy = jac_step<T>(wy[1][1], row[CF_GY * WS], row[CF_BY * WS], my);
                    // frozen cells (ring rows/columns, walls) keep the snapshot value
                    const T nvx = (upd && is_vx_unknown(nx, ny, i, y)) ? ux : wx[1][1];
                    const T nvy = (upd && is_vy_unknown(nx, ny, i, y)) ? uy : wy[1][1];
                    ec_prev = ain ? ecA : ec_prev;
                    en_prev = ain ? ent : en_prev;
                    if (lane_on && ain) {
                        if (s < kt) {
                            T* w = minec + (a2 & (RS - 1)) * (2 * WS);
                            w[0] = nvx;
                            w[WS] = nvy;
                        } else {
                            const bool ocol = i >= x0 && i < x1;
                            if ((fl & F_OWNED) && ocol) {
                                const int64_t k = (int64_t)y * ld + i;
                                ox[k] = is_vx_unknown(nx, ny, i, y) ? nvx : T(0);
                                oy[k] = is_vy_unknown(nx, ny, i, y) ? nvy : T(0);
                            }
                            if ((fl & F_OWNED) && i == nx && x1 == nx) ox[(int64_t)y * ld + nx] = T(0);
                            if ((fl & F_TOPWALL) && ocol) oy[(int64_t)ny * ld + i] = T(0);
                        }
                    }
                    sa = sa1;
                }
                rA = (rA + 1 == RC) ? 0 : rA + 1;
                lds_barrier();
            }
        }
    }
}

template <typename T, int NTMAX, int MMAX>
int launch_stream_t(stk_ctx* ctx, const Grid<T>& gg, const RasArgs& a, int nthr, size_t lds, dim3 grid, const T* vx,
                    const T* vy, T* ox, T* oy) {
    static size_t attr_set[64] = {};
    const int dev = ctx->device < 64 ? ctx->device : 63;
    if (lds > attr_set[dev]) {
        STK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_ras_stream<T, NTMAX, MMAX>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr_set[dev] = lds;
    }
    hipLaunchKernelGGL((k_ras_stream<T, NTMAX, MMAX>), grid, dim3(nthr), lds, ctx->stream, gg, vx, vy, ox, oy, a);
    STK_HIP(hipGetLastError());
    return STK_OK;
}

// Resident workgroups per CU for the streaming kernel instance that serves
// `nthr` threads with `mm` loads per thread and `lds` bytes.
template <typename T, int NTM, int MM>
int occ_one(int nthr, size_t lds) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(&k_ras_stream<T, NTM, MM>),
                                                     nthr, lds) != hipSuccess)
        return 0;
    return n;
}
template <typename T>
int stream_occupancy(int nthr, int mm, size_t lds) {
    const int NTM = nthr <= 256 ? 256 : nthr <= 512 ? 512 : 1024;
    if (NTM == 256) return mm == 1 ? occ_one<T, 256, 1>(nthr, lds) : mm == 2 ? occ_one<T, 256, 2>(nthr, lds) : occ_one<T, 256, 3>(nthr, lds);
    if (NTM == 512) return mm == 1 ? occ_one<T, 512, 1>(nthr, lds) : mm == 2 ? occ_one<T, 512, 2>(nthr, lds) : occ_one<T, 512, 3>(nthr, lds);
    return mm == 1 ? occ_one<T, 1024, 1>(nthr, lds) : mm == 2 ? occ_one<T, 1024, 2>(nthr, lds) : occ_one<T, 1024, 3>(nthr, lds);
}

template <typename T>
int try_stream(stk_ctx* ctx, const stk_grid* g, const Grid<T>& gg, int Tx, int Ty, int h, int kt, int sx, int sy,
               const void* vx, const void* vy, void* ox, void* oy, bool* done) {
    *done = false;
    if (kt < 1) return STK_OK;
    RasArgs a{};
    a.Tx = Tx;
    a.Ty = Ty;
    a.h = h;
    a.kt = kt;
    a.sx = sx;
    a.sy = sy;
    a.Wm = (int)std::min<int64_t>((int64_t)Tx + 2 * (int64_t)h, g->nx) + 2;
    const int64_t lanes = (int64_t)a.Wm * kt;
    if (lanes > 1024 || a.Wm > WS) return STK_OK;
    int nthr = (int)std::max<int64_t>(((lanes + 63) / 64) * 64, ((2 * (int64_t)a.Wm + 63) / 64) * 64);
    if (nthr > 1024 || 6 * a.Wm > 3 * nthr) return STK_OK;
    const int mm = (6 * a.Wm + nthr - 1) / nthr;
    const int ntx = (g->nx + Tx - 1) / Tx + 1, nty = (g->ny + Ty - 1) / Ty + 1;
    const int rows_per_tile = (int)std::min<int64_t>((int64_t)Ty + 2 * (int64_t)h, g->ny) + 2;
    // Tiles per workgroup NT: a workgroup streams NT tiles (NT * rows + 2kt + 1 steps);
    // pick the NT that minimises (rounds of resident workgroups) x (steps per workgroup).
    int best_nt = 1;
    double best_cost = 1e300;
    size_t lds = 0;
    for (int NT = 1; NT <= 8; ++NT) {
        RasArgs t = a;
        t.NT = NT;
        t.Vmax = NT * rows_per_tile;
        const size_t l = stream_lds_bytes<T>(t);
        if (l > (size_t)ctx->lds_max) break;
        const int per_cu = stream_occupancy<T>(nthr, (6 * a.Wm + nthr - 1) / nthr, l);
        if (per_cu < 1) break;
        const int64_t nwg = (int64_t)ntx * ((nty + NT - 1) / NT);
        const int64_t slots = (int64_t)per_cu * std::max(ctx->num_cu, 1);
        const double cost = (double)((nwg + slots - 1) / slots) * (NT * rows_per_tile + 2 * kt + 1);
        if (cost < best_cost) {
            best_cost = cost;
            best_nt = NT;
            lds = l;
        }
    }
    if (best_cost >= 1e300) return STK_OK;
    a.NT = best_nt;
    a.Vmax = best_nt * rows_per_tile;
    const dim3 grid((unsigned)ntx, (unsigned)((nty + best_nt - 1) / best_nt));
    auto* a0 = static_cast<const T*>(vx);
    auto* a1 = static_cast<const T*>(vy);
    auto* b0 = static_cast<T*>(ox);
    auto* b1 = static_cast<T*>(oy);
    int rc = STK_OK;
#define STK_STREAM_CASE(NTM, MM)                                                               \
    if (nthr <= NTM && mm == MM) rc = launch_stream_t<T, NTM, MM>(ctx, gg, a, nthr, lds, grid, a0, a1, b0, b1); \
    else
    STK_STREAM_CASE(256, 1) STK_STREAM_CASE(256, 2) STK_STREAM_CASE(256, 3)
    STK_STREAM_CASE(512, 1) STK_STREAM_CASE(512, 2) STK_STREAM_CASE(512, 3)
    STK_STREAM_CASE(1024, 1) STK_STREAM_CASE(1024, 2) STK_STREAM_CASE(1024, 3)
    return STK_OK;
#undef STK_STREAM_CASE
    if (rc == STK_OK) *done = true;
    return rc;
}

}  // namespace

int launch_ras_stream(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const FieldPtrs& f, double omega, int tile_x,
                      int tile_y, int halo, int kt, int sx, int sy, const void* vx, const void* vy, void* ox, void* oy,
                      bool* done) {
    if (dt == STK_F64) {
        Grid<double> gg{static_cast<const double*>(f.eta_c), static_cast<const double*>(f.eta_n),
                        static_cast<const double*>(f.bx), static_cast<const double*>(f.by), g->ld, g->nx, g->ny,
                        1.0 / g->dx, 1.0 / g->dy, omega};
        return try_stream<double>(ctx, g, gg, tile_x, tile_y, halo, kt, sx, sy, vx, vy, ox, oy, done);
    }
    Grid<float> gg{static_cast<const float*>(f.eta_c), static_cast<const float*>(f.eta_n),
                   static_cast<const float*>(f.bx), static_cast<const float*>(f.by), g->ld, g->nx, g->ny,
                   float(1.0 / g->dx), float(1.0 / g->dy), float(omega)};
    return try_stream<float>(ctx, g, gg, tile_x, tile_y, halo, kt, sx, sy, vx, vy, ox, oy, done);
}

}  // namespace stk
