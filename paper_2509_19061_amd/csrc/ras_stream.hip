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
// between tiles.  Sweep level s (1..kt) relaxes virtual row t - 1 - 2s at
// step t, two rows behind level s - 1, so all levels advance together with
// ONE barrier per step.  The waves of a workgroup have fixed roles:
//   * level waves: wave w < kt owns window columns 0..63 of level w + 1, so
//     its level, ring slots and row flags are wave-uniform (scalar); the
//     columns past 64 of every level (window wider than 64) go to the
//     remainder wave(s) after them;
//   * feeder waves (the last NF): stream the snapshot, viscosities and
//     right-hand side from HBM into LDS row rings through a P-row register
//     FIFO, and compute omega / diag(-M) once per cell of each row.
// A level lane keeps a 3 x 3 window of level s-1 values in registers and reads
// one new row per step from LDS; level kt writes the owned cells to HBM.
// The update calls the same stencil functions as every other smoother, so
// results are bit-identical to fused Jacobi wherever RAS equals Jacobi^kt.
#include <algorithm>

#include "stencil.hpp"
#include "stk_internal.hpp"

namespace stk {
namespace {

constexpr int P = 6;     // FIFO depth in rows (also the unroll factor; multiple of 3)
constexpr int NF = 3;    // feeder waves: 64 NF >= 2 Wm for Wm <= WS
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
// feeders' load FIFO each row; waves here communicate through LDS alone.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__host__ __device__ inline size_t align16(size_t b) { return (b + 15) & ~size_t(15); }

constexpr int WS = 96;  // LDS row stride (elements): window width bound, fixed so offsets fold

// level lanes: 64 per level for columns 0..63, then Wm - 64 per level
__host__ __device__ inline int level_lanes(int Wm, int kt) { return 64 * kt + kt * (Wm > 64 ? Wm - 64 : 0); }
__host__ __device__ inline int level_waves(int Wm, int kt) { return (level_lanes(Wm, kt) + 63) / 64; }

template <typename T>
size_t stream_lds_bytes(const RasArgs& a, int nthr) {
    const size_t n = (size_t)RS0 * 2 * WS + (size_t)(a.kt - 1) * RS * 2 * WS + (size_t)(2 * a.kt + 2) * CF_N * WS +
                     (size_t)nthr;  // + one sink element per thread for disabled LDS stores
    return align16((size_t)(a.Vmax + 1) * sizeof(int)) + n * sizeof(T);
}

// Bounds-checked output stores: a buffer resource over the used extent of an
// output array; a lane with nothing to store passes an out-of-range offset and
// the hardware drops its write (no branch).
constexpr unsigned OOB = 0xFFFFFFF0u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t out_rsrc(void* p, size_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(p, (short)0, (int)bytes, 0x00020000);
}
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void store_out(double v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)off, 0, 0);
}
__device__ __forceinline__ void store_out(float v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, 0, 0);
}

// Per-workgroup geometry shared by the roles.
struct Geo {
    int nx, ny;
    int64_t ld;
    int kt, Wm, RC, V, nsteps;
    int x0, x1, W, ci0;
    const int* vtab;
};

// ---------------------------------------------------------------- feeders --
// Feeder lane fid (0 .. 64 NF - 1).  Task m = (field, window column): row t of
// it goes to LDS at step t, row t + P is loaded at step t (unconditionally,
// from a row clamped into the array; the validity of the value is applied when
// it leaves the FIFO, so no load sits under a branch that would wait for it).
// Lanes past the last task repeat it (same value to the same place).  Then
// omega / diag of row t - 2 for every window cell: the value of a cell that is
// not relaxed (ring, wall) is never read, since its update is discarded.
template <typename T, int MM>
__device__ __forceinline__ void feeder(const Grid<T>& g, const T* __restrict__ vx, const T* __restrict__ vy,
                                       const Geo& G, T* s0, T* cf, T* dummy, int fid) {
    const int nx = G.nx, ny = G.ny, Wm = G.Wm, RC = G.RC, V = G.V, ci0 = G.ci0;
    const int64_t ld = G.ld;
    const int* vtab = G.vtab;
    const int nq = 6 * Wm;
    const T* tbase[MM];
    int tdst[MM];  // element offset of the task's column in its ring row
    int tylo[MM];
    bool tok[MM], ts0[MM];
#pragma unroll
    for (int m = 0; m < MM; ++m) {
        const int q = min(fid + m * 64 * NF, nq - 1);
        const int f = q / Wm, cq = q - f * Wm, ii = ci0 + cq;
        // field f: 0 vx, 1 vy, 2 eta_c, 3 eta_n (boundary nodes 0), 4 bx, 5 by
        const T* b = f == 0 ? vx : f == 1 ? vy : f == 2 ? g.ec : f == 3 ? g.en : f == 4 ? g.bx : g.by;
        const bool xface = (f == 0 || f == 4), yface = (f == 1 || f == 5);
        const bool colok = (xface || f == 3) ? (ii >= 1 && ii <= nx - 1) : (ii >= 0 && ii <= nx - 1);
        tok[m] = colok;
        tbase[m] = b + (colok ? ii : 0);
        tylo[m] = (yface || f == 3) ? 1 : 0;  // vy, by, eta_n-hat live on rows 1..ny-1
        ts0[m] = f < 2;
        tdst[m] = f < 2 ? f * WS + cq : (f - 2) * WS + cq;
    }
    auto row_off = [&](int y) -> int64_t { return (int64_t)min(max(y, 0), ny - 1) * ld; };
    T fifo[P][MM];
    int fy[P];  // the row each FIFO slot holds (uniform)
#pragma unroll
    for (int u = 0; u < P; ++u) {
        fy[u] = u < V ? (__builtin_amdgcn_readfirstlane(vtab[u]) & YMASK) - 1 : -1;
        const int64_t yo = row_off(fy[u]);
#pragma unroll
        for (int m = 0; m < MM; ++m) fifo[u][m] = tbase[m][yo];
    }
    int rA = 0;  // t % RC
    for (int t0 = 0; t0 < G.nsteps; t0 += P) {
#pragma unroll
        for (int u = 0; u < P; ++u) {
            const int t = t0 + u;
            {  // (A) row t: FIFO -> LDS rings; loads of row t + P
                T* r0 = s0 + (t & (RS0 - 1)) * 2 * WS;
                T* rc = cf + rA * CF_N * WS;
                const int y = fy[u];
#pragma unroll
                for (int m = 0; m < MM; ++m) {
                    const bool ok = tok[m] && y >= tylo[m] && y <= ny - 1;
                    (ts0[m] ? r0 : rc)[tdst[m]] = ok ? fifo[u][m] : T(0);
                }
                const int yn = (t + P < V) ? (__builtin_amdgcn_readfirstlane(vtab[t + P]) & YMASK) - 1 : -1;
                fy[u] = yn;
                const int64_t yo = row_off(yn);
#pragma unroll
                for (int m = 0; m < MM; ++m) fifo[u][m] = tbase[m][yo];
            }
            {  // (B) omega / diag for the E cells of row t - 2 (values 0..Wm-1: vx, Wm..2Wm-1: vy;
               //     diag_y is diag_x with the roles of x and y exchanged)
                const int r = t - 2;
                if (r >= 0 && r < V) {
                    const int sr = rA >= 2 ? rA - 2 : rA + RC - 2;
                    const int sm = sr >= 1 ? sr - 1 : RC - 1, sp = sr + 1 == RC ? 0 : sr + 1;
                    const int v = fid;  // 64 NF >= 2 Wm: one value per lane
                    const bool bl = v < 2 * Wm;
                    const bool cy = v >= Wm;
                    const int cq = bl ? (cy ? v - Wm : v) : 1;
                    const T* row = cf + sr * CF_N * WS + cq;
                    const T e0 = cy ? cf[sm * CF_N * WS + CF_EC * WS + cq] : row[CF_EC * WS - 1];
                    const T e1 = row[CF_EC * WS];
                    const T n0 = row[CF_EN * WS];
                    const T n1 = cy ? row[CF_EN * WS + 1] : cf[sp * CF_N * WS + CF_EN * WS + cq];
                    const T d = diag_x<T>(e0, e1, n0, n1, cy ? g.idy : g.idx, cy ? g.idx : g.idy);
                    T* dst = bl ? cf + sr * CF_N * WS + (cy ? CF_GY : CF_GX) * WS + cq : dummy;
                    *dst = g.omega / d;
                }
            }
            rA = (rA + 1 == RC) ? 0 : rA + 1;
            lds_barrier();
        }
    }
}

// ------------------------------------------------------------------ levels --
// Lanes of level s (1..kt, or > kt for an idle lane) at window column c.
// UNI: the whole wave has one level (level waves), so the compiler keeps the
// level-dependent quantities scalar.
template <typename T, bool UNI>
__device__ __forceinline__ void levels(const Grid<T>& g, T* __restrict__ ox, T* __restrict__ oy, const Geo& G,
                                       const T* s0, T* s1, const T* cf, T* dummy, int s_in, int c) {
    const int s = UNI ? __builtin_amdgcn_readfirstlane(s_in) : s_in;
    const int nx = G.nx, ny = G.ny, kt = G.kt, RC = G.RC, V = G.V, W = G.W;
    const int64_t ld = G.ld;
    const int* vtab = G.vtab;
    const bool lane_on = (s <= kt) && (c < W);
    const int i = G.ci0 + c;
    const bool ecol = c >= 1 && c <= W - 2;    // column inside E (else frozen ring)
    const bool ocol = i >= G.x0 && i < G.x1;  // owned column
    const bool xcol = i >= 1 && i <= nx - 1;   // vx(i, .) is an unknown column
    const bool ycol = i >= 0 && i <= nx - 1;   // vy(i, .) is an unknown column
    // waves that hold level < kt lanes store to LDS, waves that hold level kt lanes store to HBM
    const bool wave_lds = UNI ? s < kt : __builtin_amdgcn_readfirstlane(__ballot(lane_on && s < kt) != 0);
    const bool wave_out = UNI ? s == kt : __builtin_amdgcn_readfirstlane(__ballot(lane_on && s == kt) != 0);
    const int sl = min(s, kt);
    const T* prevc = ((sl == 1) ? s0 : s1 + (sl - 2) * RS * 2 * WS) + c;
    const int prs = (sl == 1) ? RS0 - 1 : RS - 1;
    T* minec = s1 + (sl - 1) * RS * 2 * WS + c;  // level s ring (unused for s = kt)
    const T* cfc = cf + c;
    int sa = RC - 1 - 2 * sl;  // ring slot of row t - 1 - 2s at t = 0
    if (sa < 0) sa += RC;
    const __amdgpu_buffer_rsrc_t rox = out_rsrc(ox, ((size_t)(ny - 1) * ld + nx + 1) * sizeof(T));
    const __amdgpu_buffer_rsrc_t roy = out_rsrc(oy, ((size_t)ny * ld + nx) * sizeof(T));

    // window of level s-1 values at columns c-1, c, c+1: rows a-1, a, a+1
    T wx[3][3], wy[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) wx[r][q] = wy[r][q] = T(0);
    T ec_prev = T(0), en_prev = T(0);  // eta_c(c, a-1), eta_n-hat(c, a)

    // Values of rows outside [0, V) (before the first and after the last virtual
    // row) are never used by an updated row: rows 0 and V-1 are ring rows, which
    // keep their snapshot value, and ring rows separate the tiles.  Only the
    // HBM stores and the row flags need guarding.  Steps past V + 2kt are
    // no-ops, so the loop runs whole groups of P steps without per-step guards.
    for (int t0 = 0; t0 < G.nsteps; t0 += P) {
#pragma unroll
        for (int u = 0; u < P; ++u) {
            const int t = t0 + u;
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
            const T* pr = prevc + ((a2 + 1) & prs) * (2 * WS);
            wx[2][0] = pr[-1];
            wx[2][1] = pr[0];
            wx[2][2] = pr[1];
            wy[2][0] = pr[WS - 1];
            wy[2][1] = pr[WS];
            wy[2][2] = pr[WS + 1];
            const int sa1 = (sa + 1 == RC) ? 0 : sa + 1;
            const bool ain = a2 >= 0 && a2 < V;
            const int fl_l = vtab[min(max(a2, 0), V - 1)];
            const int fl = UNI ? __builtin_amdgcn_readfirstlane(fl_l) : fl_l;  // one row per level wave
            const int y = (fl & YMASK) - 1;
            const T* row = cfc + sa * (CF_N * WS);
            const T ecA = row[CF_EC * WS];
            const T ent = cfc[sa1 * (CF_N * WS) + CF_EN * WS];
            const bool upd = !(fl & F_RING) && ecol;
            const T mx = mv_x<T>(wx[1][1], wx[1][0], wx[1][2], wx[0][1], wx[2][1], wy[1][1], wy[1][0], wy[2][1],
                                 wy[2][0], row[CF_EC * WS - 1], ecA, en_prev, ent, g.idx, g.idy);
            const T my = mv_y<T>(wy[1][1], wy[1][0], wy[1][2], wy[0][1], wy[2][1], wx[1][1], wx[1][2], wx[0][1],
                                 wx[0][2], ec_prev, ecA, en_prev, row[CF_EN * WS + 1], g.idx, g.idy);
            const T ux = jac_step<T>(wx[1][1], row[CF_GX * WS], row[CF_BX * WS], mx);
            const T uy = jac_step<T>(wy[1][1], row[CF_GY * WS], row[CF_BY * WS], my);
            // frozen cells (ring rows/columns, walls) keep the snapshot value
            const bool xu = xcol && y >= 0 && y < ny, yu = ycol && y >= 1 && y <= ny - 1;
            const T nvx = (upd && xu) ? ux : wx[1][1];
            const T nvy = (upd && yu) ? uy : wy[1][1];
            ec_prev = ecA;
            en_prev = ent;
            if (wave_lds) {  // levels < kt: into the level-s ring (other lanes into their sink)
                const bool w = lane_on && s < kt;
                T* wp = minec + (a2 & (RS - 1)) * (2 * WS);
                (w ? wp : dummy)[0] = nvx;
                (w ? wp + WS : dummy)[0] = nvy;
            }
            if (wave_out) {  // level kt: owned cells to HBM, walls as 0
                const bool own = lane_on && s == kt && ain && (fl & F_OWNED);
                const unsigned k = (unsigned)((int64_t)y * ld + i) * (unsigned)sizeof(T);
                store_out(xu ? nvx : T(0), rox, own && ocol ? k : OOB);
                store_out(yu ? nvy : T(0), roy, own && ocol ? k : OOB);
                // right wall vx(nx, y) and top wall vy(i, ny) of the owning tiles
                const bool rw = own && i == nx && G.x1 == nx;
                store_out(T(0), rox, rw ? (unsigned)((int64_t)y * ld + nx) * (unsigned)sizeof(T) : OOB);
                const bool tw = lane_on && s == kt && ain && (fl & F_TOPWALL) && ocol;
                store_out(T(0), roy, tw ? (unsigned)((int64_t)ny * ld + i) * (unsigned)sizeof(T) : OOB);
            }
            sa = sa1;
            lds_barrier();
        }
    }
}

// MM = HBM loads per feeder lane per row (6 fields x Wm / (64 NF)).
template <typename T, int NTMAX, int MM>
__global__ __launch_bounds__(NTMAX) void k_ras_stream(Grid<T> g, const T* __restrict__ vx, const T* __restrict__ vy,
                                                      T* __restrict__ ox, T* __restrict__ oy, RasArgs a) {
    extern __shared__ unsigned char smem_raw[];
    const int nx = g.nx, ny = g.ny;
    const int kt = a.kt, Wm = a.Wm;
    const int tid = threadIdx.x;

    // ---- this workgroup's tile column and window columns
    const int x0 = max(0, a.sx + ((int)blockIdx.x - 1) * a.Tx), x1 = min(nx, a.sx + (int)blockIdx.x * a.Tx);
    if (x0 >= x1) return;  // empty tile column: the whole workgroup leaves
    const int X0 = max(x0 - a.h, 0), X1 = min(x1 + a.h, nx);

    int* vtab = reinterpret_cast<int*>(smem_raw);
    T* s0 = reinterpret_cast<T*>(smem_raw + align16((size_t)(a.Vmax + 1) * sizeof(int)));
    T* s1 = s0 + RS0 * 2 * WS;
    T* cf = s1 + (kt - 1) * RS * 2 * WS;
    T* dummy = cf + (2 * kt + 2) * CF_N * WS + tid;  // this thread's sink for disabled LDS stores

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
    Geo G;
    G.nx = nx;
    G.ny = ny;
    G.ld = g.ld;
    G.kt = kt;
    G.Wm = Wm;
    G.RC = 2 * kt + 2;
    G.V = vtab[a.Vmax];
    if (G.V == 0) return;
    G.nsteps = G.V + 2 * kt + 1;
    G.x0 = x0;
    G.x1 = x1;
    G.W = X1 - X0 + 2;  // window column c <-> cell column i = X0 - 1 + c
    G.ci0 = X0 - 1;
    G.vtab = vtab;

    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int nlw = level_waves(Wm, kt);
    if (wave >= nlw) {
        feeder<T, MM>(g, vx, vy, G, s0, cf, dummy, (wave - nlw) * 64 + lane);
    } else if (wave < kt) {
        levels<T, true>(g, ox, oy, G, s0, s1, cf, dummy, wave + 1, lane);
    } else {  // remainder: columns 64.. of every level
        const int R = Wm - 64, j = (wave - kt) * 64 + lane;
        const int s = j / R + 1;
        levels<T, false>(g, ox, oy, G, s0, s1, cf, dummy, s, s > kt ? 0 : 64 + j % R);
    }
}

template <typename T, int NTMAX, int MM>
int launch_stream_t(stk_ctx* ctx, const Grid<T>& gg, const RasArgs& a, int nthr, size_t lds, dim3 grid, const T* vx,
                    const T* vy, T* ox, T* oy) {
    static size_t attr_set[64] = {};
    const int dev = ctx->device < 64 ? ctx->device : 63;
    if (lds > attr_set[dev]) {
        STK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_ras_stream<T, NTMAX, MM>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr_set[dev] = lds;
    }
    hipLaunchKernelGGL((k_ras_stream<T, NTMAX, MM>), grid, dim3(nthr), lds, ctx->stream, gg, vx, vy, ox, oy, a);
    STK_HIP(hipGetLastError());
    return STK_OK;
}

// Resident workgroups per CU for the instance that serves `nthr` threads with
// `mm` loads per feeder lane and `lds` bytes.
template <typename T, int NTM, int MM>
int occ_one(int nthr, size_t lds) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(&k_ras_stream<T, NTM, MM>),
                                                     nthr, lds) != hipSuccess)
        return 0;
    return n;
}
template <typename T, int NTM>
int occ_mm(int mm, int nthr, size_t lds) {
    switch (mm) {
        case 1: return occ_one<T, NTM, 1>(nthr, lds);
        case 2: return occ_one<T, NTM, 2>(nthr, lds);
        default: return occ_one<T, NTM, 3>(nthr, lds);
    }
}
template <typename T>
int stream_occupancy(int nthr, int mm, size_t lds) {
    if (nthr <= 256) return occ_mm<T, 256>(mm, nthr, lds);
    if (nthr <= 512) return occ_mm<T, 512>(mm, nthr, lds);
    return occ_mm<T, 1024>(mm, nthr, lds);
}
template <typename T, int NTM>
int launch_mm(stk_ctx* ctx, int mm, const Grid<T>& gg, const RasArgs& a, int nthr, size_t lds, dim3 grid,
              const T* vx, const T* vy, T* ox, T* oy) {
    switch (mm) {
        case 1: return launch_stream_t<T, NTM, 1>(ctx, gg, a, nthr, lds, grid, vx, vy, ox, oy);
        case 2: return launch_stream_t<T, NTM, 2>(ctx, gg, a, nthr, lds, grid, vx, vy, ox, oy);
        default: return launch_stream_t<T, NTM, 3>(ctx, gg, a, nthr, lds, grid, vx, vy, ox, oy);
    }
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
    if (a.Wm > WS || kt > 16) return STK_OK;
    // the output stores address whole arrays through 32-bit buffer offsets
    if (((size_t)g->ny * g->ld + g->nx + 1) * sizeof(T) >= (size_t)OOB) return STK_OK;
    const int nthr = 64 * (level_waves(a.Wm, kt) + NF);
    if (nthr > 1024) return STK_OK;
    const int mm = (6 * a.Wm + 64 * NF - 1) / (64 * NF);  // <= 3 for Wm <= WS
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
        const size_t l = stream_lds_bytes<T>(t, nthr);
        if (l > (size_t)ctx->lds_max) break;
        const int per_cu = stream_occupancy<T>(nthr, mm, l);
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
    int rc;
    if (nthr <= 256) rc = launch_mm<T, 256>(ctx, mm, gg, a, nthr, lds, grid, a0, a1, b0, b1);
    else if (nthr <= 512) rc = launch_mm<T, 512>(ctx, mm, gg, a, nthr, lds, grid, a0, a1, b0, b1);
    else rc = launch_mm<T, 1024>(ctx, mm, gg, a, nthr, lds, grid, a0, a1, b0, b1);
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
