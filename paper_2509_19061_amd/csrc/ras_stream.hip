// RAS-type temporal blocking (paper Sec. 4.3, Alg. 2), streaming kernel for
// gfx950.
//
// Semantics are those of the LDS-window kernel: one outer iteration, tiles cut
// at positions congruent to the shift modulo the tile size, each tile's
// extended region E (owned box grown by h, clipped) relaxed kt times with the
// one-cell ring outside E frozen at the snapshot, owned cells written back.
//
// Execution: one workgroup streams up a column of NT tiles.  The rows of the
// tiles' windows (tile after tile) form one "virtual" row stream.  Sweep level
// s (1..kt) relaxes virtual row t - 1 - 2s at step t, two rows behind level
// s - 1, so all levels advance together with ONE barrier per step.
//
// Level kt is needed on the owned rows only, level kt - 1 one row further out,
// and so on, so level 0 (the snapshot) is needed within min(kt, h + 1) rows of
// the owned rows (h + 1 = the frozen ring).  Rows farther out are read by no
// level and are left out of the stream.  Every row within kt - s of the owned
// rows reads only rows of its own tile; level s relaxes the other rows too (so
// that its LDS reads are unconditional), but their values are never read.
//
// Frozen cells (ring rows and columns, walls, cells outside the grid) get
// omega / diag = 0 from the feeders, so the update v - g (b - Mv) leaves them
// unchanged without a select.  LDS is zeroed first and only finite values are
// written to it, so the products with g = 0 are exact zeros.
//
// The waves of a workgroup have fixed roles:
//   * level waves: wave w < kt relaxes window columns 0..62 of level w + 1
//     (lane 63 carries column 63 as their neighbour), so its level, ring
//     slots and row flags are wave-uniform (scalar) and neighbouring columns
//     come from neighbouring lanes; columns 63.. of every level go to the
//     remainder wave(s) after them;
//   * feeder waves (the last NF): stream the snapshot, viscosities (stored as
//     the scaled coefficients A and N of the stencil) and right-hand side from
//     HBM into LDS row rings through a PF-row register FIFO, and compute
//     omega / diag(-M) once per cell of each row.
// A level lane keeps a 3 x 3 window of level s-1 values in registers and reads
// one new row per step from LDS; level kt writes the owned cells to HBM.
// The update calls the same stencil functions as every other smoother, so
// results are bit-identical to fused Jacobi wherever RAS equals Jacobi^kt.
#include <algorithm>
#include <cstdint>
#include <mutex>
#include <set>
#include <vector>

#include "stencil.hpp"
#include "stk_internal.hpp"
#include "wave.hpp"

namespace stk {
namespace {

constexpr int U = 6;     // steps per unrolled group
constexpr int PF = 3;    // feeder FIFO depth in rows
// rows per level ring (levels 0..kt-1; level 0 = the snapshot): at step t row t - 2s
// of level s - 1 is read while row t + 1 - 2s of it is written, and row t - 1 - 2s is
// read at the next step, so three rows suffice
constexpr int RING = 3;
constexpr int NF = 3;    // feeder waves: 64 NF >= 2 Wm for Wm <= WS_WIDE
// U: a multiple of 3 (the register window shifts by renaming), of RING (ring
// slots are compile-time per unrolled step) and of PF (FIFO slots likewise)
static_assert(U % 3 == 0 && U % RING == 0 && U % PF == 0, "unroll");
// ring slot of row r (r may be negative)
__device__ __forceinline__ int ring_slot(int r) { return ((r % RING) + RING) % RING; }
// virtual row flags: y + 1, owned, frozen ring
constexpr int YMASK = (1 << 20) - 1;
constexpr int F_OWNED = 1 << 28, F_RING = 1 << 29;
// Row element offsets y * ld are 32-bit in the stream (ny * ld < 2^31,
// checked on the host): one scalar multiply per row.
enum { CF_EC = 0, CF_EN, CF_BX, CF_BY, CF_GX, CF_GY, CF_N };

struct RasArgs {
    int Tx, Ty, h, kt, sx, sy;
    int NT;    // tiles per workgroup along y
    int merge; // 1: the NT tiles are streamed as one tile (full overlap: the values do not depend on the cuts)
    int Wm;    // window width bound: min(Tx + 2h, nx) + 2
    int Vmax;  // virtual rows bound: NT * (min(Ty + 2h, ny) + 2)
    int ntx;   // tile columns (the grid is ntx x tile-row groups, flattened)
    int nwg;   // workgroups
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

// LDS row stride WS (elements): a compile-time bound on the window width, so
// that row offsets fold into the instructions.  The narrow stride takes the
// windows of T = 64 with overlap up to 3 (full overlap up to k = 4, whose
// overlap is streamed as k - 1) and keeps such an FP64 workgroup within a
// third of the CU's LDS (three resident workgroups) with room for a row table
// of some 350 rows (one tall tile per workgroup); wider windows take the wide
// one.
constexpr int WS_NARROW = 72, WS_WIDE = 96;
// A third stride for FP64 windows of many sweeps with full overlap (kt >= 6,
// window <= 63 columns, so no remainder wave).  Its instances keep four
// coefficient fields per row (A, N, bx, by).  The level waves compute the
// Jacobi factors from the coefficients they already hold, in the feeders'
// operation order, so the values are the same.  A kt = 8 workgroup then takes
// 62 KB of LDS instead of 123 KB, and two fit in a CU.
constexpr int WS_LG = 64;
constexpr int LG_MIN_K = 6;  // FP64 full-overlap launches with at least this many sweeps use WS_LG
__host__ __device__ constexpr bool level_factors(int WS) { return WS == WS_LG; }
__host__ __device__ constexpr int cf_fields(int WS) { return level_factors(WS) ? 4 : CF_N; }
// element stride of one coefficient row
template <int WS>
__host__ __device__ constexpr int cf_row() { return cf_fields(WS) * WS; }

// level lanes: 64 per level for columns 0..63 (column 63 only as the right
// neighbour of column 62), then a group per level for columns 63..Wm-1.
// Remainder lanes come in groups of GS per level: 16 when the Wm - 63 columns
// fit (a 16-lane group then reads one LDS row, free of bank conflicts with the
// other levels' groups), else Wm - 63.
__host__ __device__ inline int rem_group(int Wm) { return Wm - 63 <= 16 ? 16 : Wm - 63; }
__host__ __device__ inline int level_lanes(int Wm, int kt) { return 64 * kt + kt * (Wm > 63 ? rem_group(Wm) : 0); }
__host__ __device__ inline int level_waves(int Wm, int kt) { return (level_lanes(Wm, kt) + 63) / 64; }

// LDS: row table | kt level rings | 2kt + 2 coefficient rows | sink for
// disabled stores (one element per lane, shared by the waves, + WS for the
// second component of a ring write)
template <int WS>
__host__ __device__ inline size_t stream_lds_elems(int kt) {
    return (size_t)kt * RING * 2 * WS + (size_t)(2 * kt + 2) * cf_fields(WS) * WS + 64 + WS;
}
template <typename T, int WS>
size_t stream_lds_bytes(const RasArgs& a) {
    return align16((size_t)(a.Vmax + 1) * sizeof(int)) + stream_lds_elems<WS>(a.kt) * sizeof(T);
}


// The scaled-stencil constants in scalar registers.
template <typename T>
__device__ __forceinline__ Scale<T> uniform_scale(const Scale<T>& s) {
    return {wave_uniform(s.a), wave_uniform(s.n), wave_uniform(s.kap), wave_uniform(s.ry), wave_uniform(s.rx)};
}

// Per-workgroup geometry shared by the roles.
struct Geo {
    int nx, ny;
    int64_t ld;
    int kt, Wm, RC, V, nsteps;
    int x0, x1, W, ci0;
    const int* vtab;
};

// Owned-row stores of level kt at grid row y (element offset off): vx and vy
// of the owned columns (lane_off), the right wall vx(nx, y) when the tile
// column ends at nx (rw_off), and the top wall vy(., ny) after the last row.
// Offsets are lane-constant; the row is folded into the (scalar) buffer
// resources.
template <typename T>
__device__ __forceinline__ void store_row(T* __restrict__ ox, T* __restrict__ oy, const Geo& G, int y, int off, T ux,
                                          T uy, unsigned lane_off, unsigned rw_off) {
    const __amdgpu_buffer_rsrc_t rox = buf_rsrc(ox + off, (size_t)(G.nx + 1) * sizeof(T));  // off = y * ld
    const __amdgpu_buffer_rsrc_t roy = buf_rsrc(oy + off, (size_t)G.nx * sizeof(T));
    buf_store(ux, rox, lane_off);
    buf_store(uy, roy, lane_off);
    if (G.x1 == G.nx) buf_store(T(0), rox, rw_off);
    if (y == G.ny - 1)
        buf_store(T(0), buf_rsrc(oy + (int64_t)G.ny * G.ld, (size_t)G.nx * sizeof(T)), lane_off);
}

// diag(-M) of the scaled stencil from the coefficients around a cell: e0, e1
// the normal-stress coefficients on either side (scaled by kl: 1 for vx, kap
// for vy), n0, n1 the shear ones (scaled by rr).  The feeders and, in the
// level-factor instances, the level waves evaluate this one expression, so
// they produce the same bits.
template <typename T>
__device__ __forceinline__ T diag_scaled(T e0, T e1, T n0, T n1, T kl, T rr) {
    return fmaT(n0 + n1, rr, e0 * kl + e1 * kl);
}

// ---------------------------------------------------------------- feeders --
// Feeder lane fid (0 .. 64 NF - 1).  Load slot 0 carries the snapshot (vx,
// vy: 2 Wm tasks) into the level-0 ring; slots 1 .. MM-1 carry eta_c, eta_n,
// bx, by (4 Wm tasks) into the coefficient rows, eta_c as A = 2 eta_c idx^2
// and eta_n as N = eta_n idx idy (the scaled stencil coefficients).  Row t of
// a task goes to LDS at step t, row t + PF is loaded at step t
// (unconditionally, from a row clamped into the array; the validity of the
// value is applied when it leaves the FIFO, so no load sits under a branch
// that would wait for it).  Lanes past the last task of a slot repeat it
// (same value to the same place).  Then omega / diag of row t - 2 for every
// window cell, 0 for a cell that is not relaxed (ring row or column, wall,
// outside the grid).
__host__ __device__ inline int feeder_loads(int Wm) { return 1 + (4 * Wm + 64 * NF - 1) / (64 * NF); }

template <typename T, int WS, int MM>
__device__ __forceinline__ void feeder(const Grid<T>& g, const T* __restrict__ vx, const T* __restrict__ vy,
                                       const Geo& G, T* rings, T* cf, T* sink, int fid) {
    const int nx = g.nx, ny = g.ny, Wm = G.Wm, W = G.W, RC = G.RC, V = G.V, ci0 = G.ci0;
    const int* vtab = G.vtab;
    const int ld32 = (int)G.ld;
    const Scale<T> sc = uniform_scale(stencil_scale(g.idx, g.idy));
    const T* tbase[MM];
    int tdst[MM];  // element offset of the task's column in its ring or coefficient row
    int tylo[MM];
    bool tok[MM];
    // slot 1 holds every eta_c and eta_n task (64 NF >= 2 Wm); its scale: 2 idx^2 for
    // eta_c, idx idy for eta_n, 1 for the rest
    const T tsc1 = fid < Wm ? sc.a : fid < 2 * Wm ? sc.n : T(1);
#pragma unroll
    for (int m = 0; m < MM; ++m) {
        const int q = m == 0 ? min(fid, 2 * Wm - 1) : min(fid + (m - 1) * 64 * NF, 4 * Wm - 1);
        const int fl = q / Wm, cq = q - fl * Wm, ii = ci0 + cq;
        // field f: 0 vx, 1 vy, 2 eta_c, 3 eta_n (boundary nodes 0), 4 bx, 5 by
        const int f = (m == 0 ? 0 : 2) + fl;
        const T* b = f == 0 ? vx : f == 1 ? vy : f == 2 ? g.ec : f == 3 ? g.en : f == 4 ? g.bx : g.by;
        const bool xface = (f == 0 || f == 4), yface = (f == 1 || f == 5);
        const bool colok = (xface || f == 3) ? (ii >= 1 && ii <= nx - 1) : (ii >= 0 && ii <= nx - 1);
        tok[m] = colok;
        tylo[m] = (yface || f == 3) ? 1 : 0;  // vy, by, eta_n-hat live on rows 1..ny-1
        tbase[m] = b + (colok ? ii : 0);
        tdst[m] = fl * WS + cq;
    }
    // omega / diag task of this lane: value v (0..Wm-1: vx, Wm..2Wm-1: vy)
    const int v = fid;  // 64 NF >= 2 Wm: one value per lane
    const bool bl = v < 2 * Wm;
    const bool cy = v >= Wm;
    const int cq = bl ? (cy ? v - Wm : v) : 1;
    const int ii = ci0 + cq;
    const bool gcol = bl && cq >= 1 && cq <= W - 2 && (cy ? ii <= nx - 1 : (ii >= 1 && ii <= nx - 1));
    const int gylo = cy ? 1 : 0;
    auto row_off = [&](int y) -> int { return min(max(y, 0), ny - 1) * ld32; };
    // diag reads: e0 = A left (vx) or below (vy), n1 = N above (vx) or right (vy); for vy
    // the normal-stress coefficients are B = A kap and the shear terms carry rx
    const int off_e0 = CF_EC * WS + cq - (cy ? 0 : 1), off_n1 = CF_EN * WS + cq + (cy ? 1 : 0);
    const T kl = cy ? sc.kap : T(1), rr = cy ? sc.rx : sc.ry;
    T fifo[PF][MM];
    int ff[PF];  // flags of the row each FIFO slot holds (uniform; 0 past the last row)
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        ff[u] = u < V ? __builtin_amdgcn_readfirstlane(vtab[u]) : 0;
        const int yo = row_off((ff[u] & YMASK) - 1);
#pragma unroll
        for (int m = 0; m < MM; ++m) fifo[u][m] = tbase[m][yo];
    }
    int fn = PF < V ? vtab[PF] : 0;  // flags of row t + PF, read one step ahead
    int f1 = 0, f2 = 0;              // flags of rows t - 1 and t - 2
    // coefficient-row slots of rows t, t - 1, t - 2, t - 3 (mod RC; RC >= 4): one
    // modular increment per step, the others are the last three values
    int rA = 0, r1 = RC - 1, r2 = RC - 2, r3 = RC - 3;
    for (int t0 = 0; t0 < G.nsteps; t0 += U) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + u, q = u % PF;
            // (B, reads) coefficients around row t - 2, written at steps t - 3 .. t - 1
            const int sr = r2, sm = r3, sp = r1;
            T e0 = T(0), e1 = T(0), n0 = T(0), n1 = T(0);
            if constexpr (!level_factors(WS)) {
                e0 = cf[(cy ? sm : sr) * cf_row<WS>() + off_e0];
                e1 = cf[sr * cf_row<WS>() + CF_EC * WS + cq];
                n0 = cf[sr * cf_row<WS>() + CF_EN * WS + cq];
                n1 = cf[(cy ? sr : sp) * cf_row<WS>() + off_n1];
            }
            __builtin_amdgcn_sched_barrier(0);
            const int ff_t = ff[q];  // flags of row t
            {  // (A) row t: FIFO -> LDS (slot 0 to the level-0 ring, the others to the
               //     coefficient row); loads of row t + PF
                T* r0 = rings + (u % RING) * 2 * WS;
                T* rc = cf + rA * cf_row<WS>();
                const int y = (ff_t & YMASK) - 1;
#pragma unroll
                for (int m = 0; m < MM; ++m) {
                    const bool ok = tok[m] && y >= tylo[m] && y <= ny - 1;
                    const T val = m == 1 ? fifo[q][m] * tsc1 : fifo[q][m];
                    (m == 0 ? r0 : rc)[tdst[m]] = ok ? val : T(0);
                }
                const int fnext = __builtin_amdgcn_readfirstlane(fn);
                ff[q] = fnext;
                const int yo = row_off((fnext & YMASK) - 1);
#pragma unroll
                for (int m = 0; m < MM; ++m) fifo[q][m] = tbase[m][yo];
                fn = t + PF + 1 < V ? vtab[t + PF + 1] : 0;
            }
            if constexpr (!level_factors(WS)) {  // (B) omega / diag for row t - 2; 0 for a cell
                                                   //     that is not relaxed, and for no row
                                                   //     (t < 2 or past the last row)
                const int yr = (f2 & YMASK) - 1;
                const bool upd = gcol && !(f2 & F_RING) && yr >= gylo && yr <= ny - 1;
                const T d = diag_scaled(e0, e1, n0, n1, kl, rr);
                T* dst = bl ? cf + sr * cf_row<WS>() + (cy ? CF_GY : CF_GX) * WS + cq : sink;
                const T gf = jac_factor(g.omega, d);  // not finite where d is 0: not selected
                *dst = upd ? gf : T(0);
            }
            f2 = f1;
            f1 = ff_t;
            r3 = r2;
            r2 = r1;
            r1 = rA;
            rA = (rA + 1 == RC) ? 0 : rA + 1;
            lds_barrier();
        }
    }
}

// ------------------------------------------------------------- level wave --
// Window columns c = 0..62 of level s (the same for the whole wave): level,
// ring slots and row flags are scalar.  Of the new row and of the
// coefficients each lane reads its own column; the neighbouring columns come
// from the neighbouring lanes.  Lane 63 holds column 63 as the right
// neighbour of column 62; its own result (which lacks column 64) goes to the
// sink, and the remainder wave relaxes column 63.  TOP: s == kt, the level
// that stores the owned rows to HBM instead of writing a ring.
template <typename T, int WS, bool TOP>
__device__ __forceinline__ void level_loop(const Grid<T>& g, T* __restrict__ ox, T* __restrict__ oy, const Geo& G,
                                           T* rings, const T* cf, T* sink, int s, int c) {
    const int kt = G.kt, RC = G.RC, V = G.V;
    const int* vtab = G.vtab;
    const int i = G.ci0 + c;
    const Scale<T> sc = uniform_scale(stencil_scale(g.idx, g.idy));
    // step t = t0 + u (t0 % RING == 0) reads level s-1 row t - 2s and writes level s row t - 1 - 2s
    const T* pr[RING];
    T* wr[RING];
#pragma unroll
    for (int k = 0; k < RING; ++k) {
        pr[k] = rings + ((s - 1) * RING + ring_slot(k - 2 * s)) * 2 * WS + c;
        wr[k] = c < 63 ? rings + (min(s, kt - 1) * RING + ring_slot(k - 1 - 2 * s)) * 2 * WS + c : sink;
    }
    const T* cfc = cf + c;
    int sa = RC - 1 - 2 * s;  // coefficient slot of row t - 1 - 2s at t = 0
    const unsigned lane_off = (c < 63 && i >= G.x0 && i < G.x1) ? (unsigned)i * (unsigned)sizeof(T) : OOB;
    const unsigned rw_off = (c < 63 && i == G.nx) ? (unsigned)i * (unsigned)sizeof(T) : OOB;
    // level-factor instances: the lane's column may hold a relaxed vx / vy (the
    // feeders' column test)
    const bool colx = c >= 1 && c <= G.W - 2 && i >= 1 && i <= G.nx - 1;
    const bool coly = c >= 1 && c <= G.W - 2 && i <= G.nx - 1;

    // window of level s-1 values at columns c-1, c, c+1: rows a-1, a, a+1
    T wx[3][3], wy[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) wx[r][q] = wy[r][q] = T(0);
    T b_prev = T(0), n_prev = T(0);  // B(c, a-1), N(c, a)
    T a_prev = T(0);                 // A(c, a-1) (level-factor instances)
    // A, bx, by of row a and N of row a + 1 are read one step ahead, before the barrier:
    // they were written two or more steps earlier, and their reads then stay out of the
    // burst of LDS reads that follows each barrier
    T qa, qbx, qby, qnt;
    {
        const T* row = cfc + sa * cf_row<WS>();
        qa = row[CF_EC * WS];
        qbx = row[CF_BX * WS];
        qby = row[CF_BY * WS];
        qnt = cfc[(sa + 1 == RC ? 0 : sa + 1) * cf_row<WS>() + CF_EN * WS];
    }

    for (int t0 = 0; t0 < G.nsteps; t0 += U) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int a2 = t0 + u - 1 - 2 * s;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                wx[0][q] = wx[1][q];
                wx[1][q] = wx[2][q];
                wy[0][q] = wy[1][q];
                wy[1][q] = wy[2][q];
            }
            const T* p = pr[u % RING];
            const int sa1 = (sa + 1 == RC) ? 0 : sa + 1;
            // row flags: the level that stores the owned rows needs them, and so do the
            // levels that compute their Jacobi factors
            const int fl = (TOP || level_factors(WS)) ? __builtin_amdgcn_readfirstlane(vtab[min(max(a2, 0), V - 1)]) : 0;
            const T* row = cfc + sa * cf_row<WS>();
            const T xc = p[0], yc = p[WS];
            T gx = T(0), gy = T(0);
            if constexpr (!level_factors(WS)) {
                gx = row[CF_GX * WS];  // level 1's are written in the last step
                gy = row[CF_GY * WS];
            }
            const T aA = qa, bx = qbx, by = qby, nt = qnt;
            // every row is relaxed (a row outside the level's cone is never read), and the LDS
            // reads of the step are issued together, ahead of the arithmetic
            __builtin_amdgcn_sched_barrier(0);
            // columns c - 1 and c + 1 from the neighbouring lanes (lane 0 is the frozen ring
            // column and lane 63 is discarded: a 0 neighbour will do for both)
            wx[2][1] = xc;
            wy[2][1] = yc;
            wx[2][0] = wave_shift<DPP_FROM_PREV>(xc);
            wy[2][0] = wave_shift<DPP_FROM_PREV>(yc);
            wx[2][2] = wave_shift<DPP_FROM_NEXT>(xc);
            wy[2][2] = wave_shift<DPP_FROM_NEXT>(yc);
            const T aL = wave_shift<DPP_FROM_PREV>(aA);     // A(c - 1, a)
            const T nR = wave_shift<DPP_FROM_NEXT>(n_prev);  // N(c + 1, a)
            const T bA = coef_b(aA, sc);
            const T mx = mvx_scaled<T>(wx[1][1], wx[1][0], wx[1][2], wx[0][1], wx[2][1], wy[1][1], wy[1][0], wy[2][1],
                                       wy[2][0], aL, aA, n_prev, nt, sc.ry);
            const T my = mvy_scaled<T>(wy[1][1], wy[1][0], wy[1][2], wy[0][1], wy[2][1], wx[1][1], wx[1][2], wx[0][1],
                                       wx[0][2], b_prev, bA, n_prev, nR, sc.rx);
            if constexpr (level_factors(WS)) {  // omega / diag of row a, 0 where the feeders would store 0
                const int fr = (a2 >= 0 && a2 < V) ? fl : 0;
                const int y = (fr & YMASK) - 1;
                const bool rok = !(fr & F_RING);
                const T gfx = jac_factor(g.omega, diag_scaled(aL, aA, n_prev, nt, T(1), sc.ry));
                const T gfy = jac_factor(g.omega, diag_scaled(a_prev, aA, n_prev, nR, sc.kap, sc.rx));
                gx = (colx && rok && y >= 0 && y <= G.ny - 1) ? gfx : T(0);
                gy = (coly && rok && y >= 1 && y <= G.ny - 1) ? gfy : T(0);
            }
            const T ux = jac_step<T>(wx[1][1], gx, bx, mx);
            const T uy = jac_step<T>(wy[1][1], gy, by, my);
            if (!TOP) {
                T* w = wr[u % RING];
                w[0] = ux;
                w[WS] = uy;
            } else if (a2 >= 0 && a2 < V && (fl & F_OWNED)) {
                const int y = (fl & YMASK) - 1;
                store_row<T>(ox, oy, G, y, y * (int)G.ld, ux, uy, lane_off, rw_off);
            }
            b_prev = bA;
            n_prev = nt;
            a_prev = aA;
            sa = sa1;
            {
                const T* nrow = cfc + sa * cf_row<WS>();
                qa = nrow[CF_EC * WS];
                qbx = nrow[CF_BX * WS];
                qby = nrow[CF_BY * WS];
                qnt = cfc[(sa + 1 == RC ? 0 : sa + 1) * cf_row<WS>() + CF_EN * WS];
            }
            lds_barrier();
        }
    }
}
template <typename T, int WS>
__device__ __forceinline__ void level_wave(const Grid<T>& g, T* __restrict__ ox, T* __restrict__ oy, const Geo& G,
                                           T* rings, const T* cf, T* sink, int s_in, int c) {
    const int s = __builtin_amdgcn_readfirstlane(s_in);
    if (s == G.kt) level_loop<T, WS, true>(g, ox, oy, G, rings, cf, sink, s, c);
    else level_loop<T, WS, false>(g, ox, oy, G, rings, cf, sink, s, c);
}

// --------------------------------------------------------- remainder wave --
// Lanes of mixed levels: level s (1..kt) at window column c >= 63, or idle
// (s > kt, or a spare lane of a level's group, which repeats a column of its
// group so that its LDS reads stay in the group's rows).  Every row is
// relaxed (results outside a level's cone are not read).  Ring writes of
// level-kt and idle lanes go to the sink; the level-kt lanes share one row
// per step, whose flags are read once for the stores.
template <typename T, int WS>
__device__ __forceinline__ void remainder_wave(const Grid<T>& g, T* __restrict__ ox, T* __restrict__ oy,
                                               const Geo& G, T* rings, const T* cf, T* sink, int s, int c,
                                               bool idle) {
    const int kt = G.kt, RC = G.RC, V = G.V;
    const int* vtab = G.vtab;
    const int sl = min(s, kt);
    const int i = G.ci0 + c;
    const T* pr[RING];
    T* wr[RING];
#pragma unroll
    for (int k = 0; k < RING; ++k) {
        pr[k] = rings + ((sl - 1) * RING + ring_slot(k - 2 * sl)) * 2 * WS + c;
        wr[k] = sl < kt && !idle ? rings + (sl * RING + ring_slot(k - 1 - 2 * sl)) * 2 * WS + c : sink;
    }
    const T* cfc = cf + c;
    const Scale<T> sc = uniform_scale(stencil_scale(g.idx, g.idy));
    int sa = RC - 1 - 2 * sl;
    const bool top = s == kt && !idle;
    const unsigned lane_off = (top && i >= G.x0 && i < G.x1) ? (unsigned)i * (unsigned)sizeof(T) : OOB;
    const unsigned rw_off = (top && i == G.nx) ? (unsigned)i * (unsigned)sizeof(T) : OOB;

    T wx[3][3], wy[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) wx[r][q] = wy[r][q] = T(0);
    T b_prev = T(0), n_prev = T(0);  // B(c, a-1), N(c, a)

    for (int t0 = 0; t0 < G.nsteps; t0 += U) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                wx[0][q] = wx[1][q];
                wx[1][q] = wx[2][q];
                wy[0][q] = wy[1][q];
                wy[1][q] = wy[2][q];
            }
            const T* p = pr[u % RING];
            wx[2][0] = p[-1];
            wx[2][1] = p[0];
            wx[2][2] = p[1];
            wy[2][0] = p[WS - 1];
            wy[2][1] = p[WS];
            wy[2][2] = p[WS + 1];
            const int sa1 = (sa + 1 == RC) ? 0 : sa + 1;
            const T* row = cfc + sa * cf_row<WS>();
            const T aA = row[CF_EC * WS], aL = row[CF_EC * WS - 1], nR = row[CF_EN * WS + 1];
            const T nt = cfc[sa1 * cf_row<WS>() + CF_EN * WS];
            const int ak = t0 + u - 1 - 2 * kt;  // the row of the level-kt lanes
            const int flk = __builtin_amdgcn_readfirstlane(vtab[min(max(ak, 0), V - 1)]);
            __builtin_amdgcn_sched_barrier(0);
            const T bA = coef_b(aA, sc);
            const T mx = mvx_scaled<T>(wx[1][1], wx[1][0], wx[1][2], wx[0][1], wx[2][1], wy[1][1], wy[1][0], wy[2][1],
                                       wy[2][0], aL, aA, n_prev, nt, sc.ry);
            const T my = mvy_scaled<T>(wy[1][1], wy[1][0], wy[1][2], wy[0][1], wy[2][1], wx[1][1], wx[1][2], wx[0][1],
                                       wx[0][2], b_prev, bA, n_prev, nR, sc.rx);
            // the update's factors are read after the operator values: fewer registers in flight
            __builtin_amdgcn_sched_barrier(0);
            const T gx = row[CF_GX * WS], bx = row[CF_BX * WS], gy = row[CF_GY * WS], by = row[CF_BY * WS];
            const T ux = jac_step<T>(wx[1][1], gx, bx, mx);
            const T uy = jac_step<T>(wy[1][1], gy, by, my);
            T* w = wr[u % RING];
            w[0] = ux;
            w[WS] = uy;
            if (ak >= 0 && ak < V && (flk & F_OWNED)) {
                const int y = (flk & YMASK) - 1;
                store_row<T>(ox, oy, G, y, y * (int)G.ld, ux, uy, lane_off, rw_off);
            }
            b_prev = bA;
            n_prev = nt;
            sa = sa1;
            lds_barrier();
        }
    }
}

// MM = HBM loads per feeder lane per row (feeder_loads).
// One workgroup: tile column bx, tile rows by*NT .. by*NT + NT - 1.
template <typename T, int MM, int WS>
__device__ __forceinline__ void ras_workgroup(const Grid<T>& g, const T* __restrict__ vx, const T* __restrict__ vy,
                                              T* __restrict__ ox, T* __restrict__ oy, const RasArgs& a, int bx,
                                              int by) {
    extern __shared__ unsigned char smem_raw[];
    const int nx = g.nx, ny = g.ny;
    const int kt = a.kt, Wm = a.Wm;
    const int tid = threadIdx.x, nthr = blockDim.x;

    // ---- this workgroup's tile column and window columns
    const int x0 = max(0, a.sx + (bx - 1) * a.Tx), x1 = min(nx, a.sx + bx * a.Tx);
    if (x0 >= x1) return;  // empty tile column: the whole workgroup leaves
    const int X0 = max(x0 - a.h, 0), X1 = min(x1 + a.h, nx);

    int* vtab = reinterpret_cast<int*>(smem_raw);
    T* rings = reinterpret_cast<T*>(smem_raw + align16((size_t)(a.Vmax + 1) * sizeof(int)));
    T* cf = rings + kt * RING * 2 * WS;
    T* sink = cf + (2 * kt + 2) * cf_row<WS>() + (tid & 63);  // this lane's sink for disabled LDS stores

    // ---- virtual row table: y + 1 and flags, tile after tile.
    // Tile ty of this workgroup contributes the rows y of [Y0 - 1, Y1] within D of its owned rows.
    // Merged: the NT tiles as one tile of NT Ty rows.
    const int D = min(kt, a.h + 1);
    const int nty = (ny + a.Ty - 1) / a.Ty + 1;
    const int tyb = by * a.NT;
    const int span = a.merge ? a.NT : 1;  // tiles per streamed tile
    int V = 0;
    for (int q = 0; q < a.NT; q += span) {
        const int ty = tyb + q;
        if (ty >= nty) break;
        const int y0 = max(0, a.sy + (ty - 1) * a.Ty), y1 = min(ny, a.sy + (ty + span - 1) * a.Ty);
        if (y0 >= y1) continue;
        const int Y0 = max(y0 - a.h, 0), Y1 = min(y1 + a.h, ny);
        const int lo = max(Y0 - 1, y0 - D), hi = min(Y1, y1 - 1 + D);
        for (int v = V + tid; v <= V + hi - lo; v += nthr) {
            const int y = lo + v - V;
            int f = y + 1;
            if (y == Y0 - 1 || y == Y1) f |= F_RING;
            if (y >= y0 && y < y1) f |= F_OWNED;
            vtab[v] = f;
        }
        V += hi - lo + 1;
    }
    // ---- LDS rings, coefficient rows and sinks start at 0 (finite everywhere)
    {
        const int n = (int)stream_lds_elems<WS>(kt);
        for (int e = tid; e < n; e += nthr) rings[e] = T(0);
    }
    lds_barrier();
    if (V == 0) return;
    Geo G;
    G.nx = nx;
    G.ny = ny;
    G.ld = g.ld;
    G.kt = kt;
    G.Wm = Wm;
    G.RC = 2 * kt + 2;
    G.V = V;
    G.nsteps = V + 2 * kt + 1;
    G.x0 = x0;
    G.x1 = x1;
    G.W = X1 - X0 + 2;  // window column c <-> cell column i = X0 - 1 + c
    G.ci0 = X0 - 1;
    G.vtab = vtab;

    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int nlw = level_waves(Wm, kt);
    if (wave >= nlw) {
        // the feeders set the pace of a step (every role waits for their rows at the
        // barrier): they issue ahead of the other waves of their SIMD
        __builtin_amdgcn_s_setprio(1);
        feeder<T, WS, MM>(g, vx, vy, G, rings, cf, sink, (wave - nlw) * 64 + lane);
    } else if (wave < kt) {
        level_wave<T, WS>(g, ox, oy, G, rings, cf, sink, wave + 1, lane);
    } else if constexpr (!level_factors(WS)) {  // remainder: columns 63.. of every level (level-factor
                                                // windows have none)
        const int R = Wm - 63, GS = rem_group(Wm), j = (wave - kt) * 64 + lane;
        const int s = j / GS + 1, q = j % GS;
        remainder_wave<T, WS>(g, ox, oy, G, rings, cf, sink, s, s > kt ? 63 : 63 + min(q, R - 1), s > kt || q >= R);
    }
}

// Waves per SIMD the register allocation must leave room for (at most 72
// VGPRs each): an FP64 workgroup of up to 8 waves (k <= 4 with T = 64) is
// resident three or four times per CU, 6 to 7 waves per SIMD, and the waves
// of a workgroup do not always spread evenly over the SIMDs; so is a pair of
// level-factor workgroups of up to 14 waves.  Other sizes are bound by LDS or
// by their own wave count first.
constexpr int ras_waves_per_simd(int nthr, int ws) { return (nthr == 512 || level_factors(ws)) ? 7 : 1; }

template <typename T, int NTMAX, int MM, int WS>
__global__ __launch_bounds__(NTMAX, ras_waves_per_simd(NTMAX, WS)) void k_ras_stream(Grid<T> g, const T* __restrict__ vx, const T* __restrict__ vy,
                                                      T* __restrict__ ox, T* __restrict__ oy, RasArgs a) {
    // tiles row-major, renumbered by XCD: tile columns side by side run on one
    // XCD at the same time and share the halo columns of their windows in L2
    const int tw = xcd_tile((int)blockIdx.x, a.nwg);
    ras_workgroup<T, MM, WS>(g, vx, vy, ox, oy, a, tw % a.ntx, tw / a.ntx);
}

// Batched: workgroup b (renumbered by XCD over the whole batch) belongs to
// the instance with pre[i] <= b < pre[i+1]; the launch shape (tile, halo, k,
// tiles per workgroup, window bound) is shared, the geometry is the
// instance's, shifts are 0.
template <typename T, int NTMAX, int MM, int WS>
__global__ __launch_bounds__(NTMAX, ras_waves_per_simd(NTMAX, WS)) void k_ras_batch(const RasJob<T>* __restrict__ jobs, const int* __restrict__ pre,
                                                     int n, RasArgs a, T omega) {
    const int b = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    const RasJob<T>& J = jobs[lo];
    const Grid<T> g{J.ec, J.en, J.bx, J.by, J.ld, J.nx, J.ny, J.idx, J.idy, omega};
    const int tw = b - pre[lo];
    ras_workgroup<T, MM, WS>(g, J.vx, J.vy, J.ox, J.oy, a, tw % J.ntx, tw / J.ntx);
}

template <typename T, int NTMAX, int MM, int WS>
int launch_stream_t(stk_ctx* ctx, const Grid<T>& gg, const RasArgs& a, int nthr, size_t lds, dim3 grid, const T* vx,
                    const T* vy, T* ox, T* oy) {
    static size_t attr_set[64] = {};
    const int dev = ctx->device < 64 ? ctx->device : 63;
    if (lds > attr_set[dev]) {
        STK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_ras_stream<T, NTMAX, MM, WS>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr_set[dev] = lds;
    }
    hipLaunchKernelGGL((k_ras_stream<T, NTMAX, MM, WS>), grid, dim3(nthr), lds, ctx->stream, gg, vx, vy, ox, oy, a);
    STK_HIP(hipGetLastError());
    return STK_OK;
}

// Resident workgroups per CU for the instance that serves `nthr` threads with
// `mm` loads per feeder lane and `lds` bytes.
template <typename T, int NTM, int MM, int WS>
int occ_one(int nthr, size_t lds) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(&k_ras_stream<T, NTM, MM, WS>),
                                                     nthr, lds) != hipSuccess)
        return 0;
    return n;
}
template <typename T, int NTM, int WS>
int occ_mm(int mm, int nthr, size_t lds) {
    switch (mm) {
        case 2: return occ_one<T, NTM, 2, WS>(nthr, lds);
        default: return occ_one<T, NTM, 3, WS>(nthr, lds);
    }
}
// Cached per (device, block size, loads per lane, LDS bytes): the query is
// slow next to a launch, and every outer iteration asks for up to 8 of them.
template <typename T, int WS>
int stream_occupancy(int dev, int nthr, int mm, size_t lds) {
    struct Entry {
        int dev, nthr, mm;
        size_t lds;
        int n;
    };
    static std::mutex mu;
    static std::vector<Entry> cache;
    {
        std::lock_guard<std::mutex> lk(mu);
        for (const Entry& e : cache)
            if (e.dev == dev && e.nthr == nthr && e.mm == mm && e.lds == lds) return e.n;
    }
    int n;
    if constexpr (level_factors(WS)) n = occ_mm<T, 1024, WS>(mm, nthr, lds);  // kt >= 6: over 512 threads
    else if (nthr <= 256) n = occ_mm<T, 256, WS>(mm, nthr, lds);
    else if (nthr <= 512) n = occ_mm<T, 512, WS>(mm, nthr, lds);
    else n = occ_mm<T, 1024, WS>(mm, nthr, lds);
    std::lock_guard<std::mutex> lk(mu);
    if (cache.size() < 1024) cache.push_back({dev, nthr, mm, lds, n});
    return n;
}
template <typename T, int NTM, int WS>
int launch_mm(stk_ctx* ctx, int mm, const Grid<T>& gg, const RasArgs& a, int nthr, size_t lds, dim3 grid,
              const T* vx, const T* vy, T* ox, T* oy) {
    switch (mm) {
        case 2: return launch_stream_t<T, NTM, 2, WS>(ctx, gg, a, nthr, lds, grid, vx, vy, ox, oy);
        default: return launch_stream_t<T, NTM, 3, WS>(ctx, gg, a, nthr, lds, grid, vx, vy, ox, oy);
    }
}

template <typename T, int WS>
int try_stream_ws(stk_ctx* ctx, const stk_grid* g, const Grid<T>& gg, RasArgs a, const void* vx, const void* vy,
                  void* ox, void* oy, bool* done) {
    const int kt = a.kt, Tx = a.Tx, Ty = a.Ty, h = a.h;
    const int nthr = 64 * (level_waves(a.Wm, kt) + NF);
    if (nthr > 1024) return STK_OK;
    const int mm = feeder_loads(a.Wm);  // 2 or 3 for Wm <= WS_WIDE
    // tiles cut at s + m T: one more tile column (row) for the partial tile before the
    // first cut, none when the cuts fall on multiples of T (s == T)
    const int ntx = (g->nx + Tx - 1) / Tx + (a.sx == Tx ? 0 : 1), nty = (g->ny + Ty - 1) / Ty + (a.sy == Ty ? 0 : 1);
    // rows of a tile of height H in the stream: at most H + 2 min(kt, h + 1), and at most the window's
    const int D = std::min(kt, h + 1);
    auto tile_rows = [&](int64_t H) {
        return (int)std::min<int64_t>(std::min<int64_t>(H + 2 * (int64_t)h, g->ny) + 2, std::min<int64_t>(H, g->ny) + 2 * D);
    };
    // Resident workgroups per CU: the occupancy query, and LDS counted in 2 KiB
    // granules against the CU's LDS (a workgroup just over a third of the LDS is
    // resident only twice per CU, whatever the query says).
    auto slots_for = [&](size_t l, int occ) -> int64_t {
        if (l > (size_t)ctx->lds_max) return 0;
        int per_cu = occ;
        if (ctx->lds_cu > 0) per_cu = std::min<int>(per_cu, ctx->lds_cu / (int)((l + 2047) & ~size_t(2047)));
        return (int64_t)std::max(per_cu, 0) * std::max(ctx->num_cu, 1);
    };
    // Launch time model: (rounds of resident workgroups) x (row steps per workgroup).
    double best_cost = 1e300;
    size_t lds = 0;
    if (h >= kt - 1) {
        // Full overlap: the owned values do not depend on where the tiles are cut, so each
        // workgroup streams one tile of H rows (no overlap rows inside it), cut at multiples
        // of H; H is chosen by the model, so that the workgroups fill whole rounds.
        a.merge = 1;
        a.NT = 1;
        RasArgs t0 = a;
        t0.Vmax = 0;
        const int occ = stream_occupancy<T, WS>(ctx->device, nthr, mm, stream_lds_bytes<T, WS>(t0));
        int best_h = 0, last_h = -1;
        for (int r = 1; r <= std::max(1, g->ny / 16); ++r) {  // r tile rows (H >= 16)
            const int H = (g->ny + r - 1) / r;
            if (H == last_h) continue;
            last_h = H;
            RasArgs t = a;
            t.Vmax = tile_rows(H);
            const size_t l = stream_lds_bytes<T, WS>(t);
            const int64_t slots = slots_for(l, occ);
            if (slots < 1) continue;
            const int64_t nwg = (int64_t)ntx * ((g->ny + H - 1) / H);
            const double cost = (double)((nwg + slots - 1) / slots) * (tile_rows(H) + 2 * kt + 1);
            if (cost < best_cost) {
                best_cost = cost;
                best_h = H;
                lds = l;
            }
        }
        if (best_cost >= 1e300) return STK_OK;
        a.Ty = a.sy = best_h;
        a.Vmax = tile_rows(best_h);
        a.ntx = ntx;
        a.nwg = ntx * ((g->ny + best_h - 1) / best_h);
    } else {
        // Tiles per workgroup NT: a workgroup streams NT tiles (NT (rows of a tile) + 2kt + 1
        // steps); pick the NT of least cost.
        a.merge = 0;
        int best_nt = 1;
        for (int NT = 1; NT <= 8; ++NT) {
            RasArgs t = a;
            t.NT = NT;
            t.Vmax = NT * tile_rows(Ty);
            const size_t l = stream_lds_bytes<T, WS>(t);
            if (l > (size_t)ctx->lds_max) break;
            const int64_t slots = slots_for(l, stream_occupancy<T, WS>(ctx->device, nthr, mm, l));
            if (slots < 1) break;
            const int64_t nwg = (int64_t)ntx * ((nty + NT - 1) / NT);
            const double cost = (double)((nwg + slots - 1) / slots) * (NT * tile_rows(Ty) + 2 * kt + 1);
            if (cost < best_cost) {
                best_cost = cost;
                best_nt = NT;
                lds = l;
            }
        }
        if (best_cost >= 1e300) return STK_OK;
        a.NT = best_nt;
        a.Vmax = best_nt * tile_rows(Ty);
        a.ntx = ntx;
        a.nwg = ntx * ((nty + best_nt - 1) / best_nt);
    }
    const dim3 grid((unsigned)a.nwg);
    auto* a0 = static_cast<const T*>(vx);
    auto* a1 = static_cast<const T*>(vy);
    auto* b0 = static_cast<T*>(ox);
    auto* b1 = static_cast<T*>(oy);
    int rc;
    if constexpr (level_factors(WS)) rc = launch_mm<T, 1024, WS>(ctx, mm, gg, a, nthr, lds, grid, a0, a1, b0, b1);
    else if (nthr <= 256) rc = launch_mm<T, 256, WS>(ctx, mm, gg, a, nthr, lds, grid, a0, a1, b0, b1);
    else if (nthr <= 512) rc = launch_mm<T, 512, WS>(ctx, mm, gg, a, nthr, lds, grid, a0, a1, b0, b1);
    else rc = launch_mm<T, 1024, WS>(ctx, mm, gg, a, nthr, lds, grid, a0, a1, b0, b1);
    if (rc == STK_OK) *done = true;
    return rc;
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
    if constexpr (sizeof(T) == 8) {
        // FP64, many sweeps, full overlap: tiles of 63 - 2kt columns, so that the window
        // (63 columns) needs no remainder wave and the level-factor instance applies
        // (the owned values do not depend on the cuts)
        if (kt >= LG_MIN_K && h >= kt - 1 && 63 - 2 * kt >= 8) {
            a.Tx = Tx = 63 - 2 * kt;
            a.sx = sx % Tx;
        }
    }
    if (h >= kt - 1) {  // full overlap: the shift does not matter either; cut at multiples of the
                        // tile, the first tile at 0 (no partial tile column or row)
        a.sx = a.Tx;
        a.sy = a.Ty;
    }
    a.Wm = (int)std::min<int64_t>((int64_t)Tx + 2 * (int64_t)h, g->nx) + 2;
    // (the output stores address one row at a time through 32-bit buffer offsets)
    if (a.Wm > WS_WIDE || kt > 16 || g->ny + 1 > YMASK || (int64_t)(g->nx + 1) * (int64_t)sizeof(T) >= INT32_MAX ||
        (int64_t)g->ny * g->ld >= INT32_MAX)
        return STK_OK;
    if constexpr (sizeof(T) == 8)
        if (kt >= LG_MIN_K && h >= kt - 1 && a.Wm <= 63)
            return try_stream_ws<T, WS_LG>(ctx, g, gg, a, vx, vy, ox, oy, done);
    if (a.Wm <= WS_NARROW) return try_stream_ws<T, WS_NARROW>(ctx, g, gg, a, vx, vy, ox, oy, done);
    return try_stream_ws<T, WS_WIDE>(ctx, g, gg, a, vx, vy, ox, oy, done);
}

// ------------------------------------------------------------------ batched --
template <typename T, int NTMAX, int MM, int WS>
int launch_batch_t(stk_ctx* ctx, const RasShape& sh, const void* jobs, const int* pre, int n, T omega) {
    static size_t attr_set[64] = {};
    const int dev = ctx->device < 64 ? ctx->device : 63;
    if (sh.lds > attr_set[dev]) {
        STK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_ras_batch<T, NTMAX, MM, WS>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh.lds));
        attr_set[dev] = sh.lds;
    }
    RasArgs a{};
    a.Tx = sh.tile;
    a.Ty = sh.ty;
    a.h = sh.h;
    a.kt = sh.kt;
    a.sx = sh.tile;  // cuts at multiples of the tile (and of its height), the first tile at 0
    a.sy = sh.ty;
    a.NT = sh.NT;
    a.merge = sh.merge;
    a.Wm = sh.Wm;
    a.Vmax = sh.Vmax;
    hipLaunchKernelGGL((k_ras_batch<T, NTMAX, MM, WS>), dim3((unsigned)sh.nwg), dim3(sh.nthr), sh.lds, ctx->stream,
                       static_cast<const RasJob<T>*>(jobs), pre, n, a, omega);
    STK_HIP(hipGetLastError());
    return STK_OK;
}
template <typename T, int NTM, int WS>
int launch_batch_mm(stk_ctx* ctx, const RasShape& sh, const void* jobs, const int* pre, int n, T omega) {
    switch (sh.mm) {
        case 2: return launch_batch_t<T, NTM, 2, WS>(ctx, sh, jobs, pre, n, omega);
        default: return launch_batch_t<T, NTM, 3, WS>(ctx, sh, jobs, pre, n, omega);
    }
}
template <typename T, int WS>
int launch_batch_ws(stk_ctx* ctx, const RasShape& sh, const void* jobs, const int* pre, int n, T omega) {
    if constexpr (level_factors(WS)) return launch_batch_mm<T, 1024, WS>(ctx, sh, jobs, pre, n, omega);
    if (sh.nthr <= 256) return launch_batch_mm<T, 256, WS>(ctx, sh, jobs, pre, n, omega);
    if (sh.nthr <= 512) return launch_batch_mm<T, 512, WS>(ctx, sh, jobs, pre, n, omega);
    return launch_batch_mm<T, 1024, WS>(ctx, sh, jobs, pre, n, omega);
}

// Same model as try_stream_ws over the whole batch: the occupancy of the
// single-grid instance (same body) and the LDS granule bound.
template <typename T, int WS>
void batch_shape_ws(stk_ctx* ctx, const int* nx, const int* ny, int n, int tile, int h, int kt, int Wm,
                    RasShape* out, std::vector<int>* pre, std::vector<int>* ntxv, bool* ok) {
    *ok = false;
    const int nthr = 64 * (level_waves(Wm, kt) + NF);
    if (nthr > 1024) return;
    const int mm = feeder_loads(Wm);
    const int D = std::min(kt, h + 1);
    const bool merge = h >= kt - 1;  // full overlap: a workgroup's tiles are streamed as one
    // stream rows of a tile of height H, the most over the instances
    auto rows_h = [&](int64_t H) {
        int rows = 0;
        for (int q = 0; q < n; ++q)
            rows = std::max(rows, (int)std::min<int64_t>(std::min<int64_t>(H + 2 * (int64_t)h, ny[q]) + 2,
                                                         std::min<int64_t>(H, ny[q]) + 2 * D));
        return rows;
    };
    double best_cost = 1e300;
    int best_ty = tile;
    if (merge) {
        // Full overlap, as in try_stream_ws: one tile of H rows per workgroup, cut at
        // multiples of H, H chosen over the instances' heights ceil(ny / r) so that the
        // workgroups fill whole rounds.  Resident workgroups per CU are capped at 3 in
        // FP64 and 4 in FP32: in the 2048^2 V-cycle (k = 2) four FP64 workgroups of
        // 64-row tiles per CU took 84 us a launch against 68 us for three of 86 rows,
        // and five FP32 ones of 52 rows were slower than four of 64 (62 against 47 us),
        // although the occupancy query allows them.
        RasArgs t0{};
        t0.kt = kt;
        const int occ = std::min(stream_occupancy<T, WS>(ctx->device, nthr, mm, stream_lds_bytes<T, WS>(t0)),
                                 sizeof(T) == 8 ? 3 : 4);
        std::set<int> hs;
        for (int q = 0; q < n; ++q)
            for (int r = 1; r <= std::max(1, ny[q] / 16); ++r) hs.insert((ny[q] + r - 1) / r);
        for (int H : hs) {
            RasArgs t{};
            t.kt = kt;
            t.Vmax = rows_h(H);
            const size_t l = stream_lds_bytes<T, WS>(t);
            if (l > (size_t)ctx->lds_max) continue;
            int per_cu = occ;
            if (ctx->lds_cu > 0) per_cu = std::min<int>(per_cu, ctx->lds_cu / (int)((l + 2047) & ~size_t(2047)));
            if (per_cu < 1) continue;
            int64_t nwg = 0;
            for (int q = 0; q < n; ++q) nwg += (int64_t)((nx[q] + tile - 1) / tile) * ((ny[q] + H - 1) / H);
            const int64_t slots = (int64_t)per_cu * std::max(ctx->num_cu, 1);
            const double cost = (double)((nwg + slots - 1) / slots) * (t.Vmax + 2 * kt + 1);
            if (cost < best_cost && nwg < INT32_MAX) {
                best_cost = cost;
                best_ty = H;
                out->NT = 1;
                out->Vmax = t.Vmax;
                out->lds = l;
                out->nwg = (int)nwg;
            }
        }
    } else {
        for (int NT = 1; NT <= 8; ++NT) {
            RasArgs t{};
            t.kt = kt;
            t.Vmax = NT * rows_h(tile);  // NT tiles, each with its overlap rows
            const size_t l = stream_lds_bytes<T, WS>(t);
            if (l > (size_t)ctx->lds_max) break;
            int per_cu = stream_occupancy<T, WS>(ctx->device, nthr, mm, l);
            if (ctx->lds_cu > 0) per_cu = std::min<int>(per_cu, ctx->lds_cu / (int)((l + 2047) & ~size_t(2047)));
            if (per_cu < 1) break;
            int64_t nwg = 0;
            for (int q = 0; q < n; ++q) {
                const int ntx = (nx[q] + tile - 1) / tile, nty = (ny[q] + tile - 1) / tile;
                nwg += (int64_t)ntx * ((nty + NT - 1) / NT);
            }
            const int64_t slots = (int64_t)per_cu * std::max(ctx->num_cu, 1);
            const double cost = (double)((nwg + slots - 1) / slots) * (t.Vmax + 2 * kt + 1);
            if (cost < best_cost && nwg < INT32_MAX) {
                best_cost = cost;
                out->NT = NT;
                out->Vmax = t.Vmax;
                out->lds = l;
                out->nwg = (int)nwg;
            }
        }
    }
    if (best_cost >= 1e300) return;
    out->ty = best_ty;
    out->tile = tile;
    out->h = h;
    out->kt = kt;
    out->merge = merge ? 1 : 0;
    out->Wm = Wm;
    out->nthr = nthr;
    out->mm = mm;
    out->ws = WS;
    pre->assign(1, 0);
    ntxv->clear();
    for (int q = 0; q < n; ++q) {
        const int ntx = (nx[q] + tile - 1) / tile, nty = (ny[q] + best_ty - 1) / best_ty;
        ntxv->push_back(ntx);
        pre->push_back(pre->back() + ntx * ((nty + out->NT - 1) / out->NT));
    }
    *ok = true;
}

template <typename T>
void batch_shape(stk_ctx* ctx, const int* nx, const int* ny, const int64_t* ld, int n, int tile, int h, int kt,
                 RasShape* out, std::vector<int>* pre, std::vector<int>* ntx, bool* ok) {
    *ok = false;
    if (n < 1 || kt < 1 || kt > 16 || tile < 1) return;
    int Wm = 0;
    for (int q = 0; q < n; ++q) {
        if (ny[q] + 1 > YMASK || (int64_t)(nx[q] + 1) * (int64_t)sizeof(T) >= INT32_MAX ||
            (int64_t)ny[q] * ld[q] >= INT32_MAX)
            return;
        Wm = std::max<int>(Wm, (int)std::min<int64_t>((int64_t)tile + 2 * (int64_t)h, nx[q]) + 2);
    }
    if (Wm > WS_WIDE) return;
    if constexpr (sizeof(T) == 8)
        if (kt >= LG_MIN_K && h >= kt - 1 && Wm <= 63)
            return batch_shape_ws<T, WS_LG>(ctx, nx, ny, n, tile, h, kt, Wm, out, pre, ntx, ok);
    if (Wm <= WS_NARROW) batch_shape_ws<T, WS_NARROW>(ctx, nx, ny, n, tile, h, kt, Wm, out, pre, ntx, ok);
    else batch_shape_ws<T, WS_WIDE>(ctx, nx, ny, n, tile, h, kt, Wm, out, pre, ntx, ok);
}

}  // namespace

// Overlap beyond kt - 1 cannot reach the owned cells: after kt sweeps an owned
// value depends on the snapshot within kt cells, and a frozen ring at distance
// kt (overlap kt - 1) enters only sweep-1 values at distance kt - 1, which
// are exact.  Every overlap h >= kt - 1 therefore gives the same values (kt
// Jacobi sweeps), and the narrowest window is streamed.
inline int effective_halo(int h, int kt) { return std::min(h, std::max(kt - 1, 0)); }

int launch_ras_stream(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const FieldPtrs& f, double omega, int tile_x,
                      int tile_y, int halo, int kt, int sx, int sy, const void* vx, const void* vy, void* ox, void* oy,
                      bool* done) {
    halo = effective_halo(halo, kt);
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

namespace stk {

int ras_batch_shape(stk_ctx* ctx, stk_dtype dt, const int* nx, const int* ny, const int64_t* ld, int n, int tile,
                    int h, int kt, RasShape* out, std::vector<int>* pre, std::vector<int>* ntx, bool* ok) {
    h = effective_halo(h, kt);
    if (dt == STK_F64) batch_shape<double>(ctx, nx, ny, ld, n, tile, h, kt, out, pre, ntx, ok);
    else batch_shape<float>(ctx, nx, ny, ld, n, tile, h, kt, out, pre, ntx, ok);
    return STK_OK;
}

int ras_batch_launch(stk_ctx* ctx, stk_dtype dt, const RasShape& s, const void* jobs, const int* pre, int n,
                     double omega) {
    if (n < 1 || s.nwg < 1) return STK_OK;
    if (dt == STK_F64)
        return s.ws == WS_LG       ? launch_batch_ws<double, WS_LG>(ctx, s, jobs, pre, n, omega)
               : s.ws == WS_NARROW ? launch_batch_ws<double, WS_NARROW>(ctx, s, jobs, pre, n, omega)
                                   : launch_batch_ws<double, WS_WIDE>(ctx, s, jobs, pre, n, omega);
    return s.ws == WS_NARROW ? launch_batch_ws<float, WS_NARROW>(ctx, s, jobs, pre, n, float(omega))
                             : launch_batch_ws<float, WS_WIDE>(ctx, s, jobs, pre, n, float(omega));
}

}  // namespace stk
