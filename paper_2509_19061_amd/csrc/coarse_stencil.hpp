// Stored stencils of the Galerkin coarse operators A_c = P^T A P / 4
// (A = -M, bilinear P), on the staggered layout of the fine grid.
//
// With bilinear prolongation the coarse couplings of one unknown stay inside
// fixed windows on every coarse level (offsets of the neighbour's (i, j)
// relative to the row's own (i, j)):
//   vx row -> vx: x in [-1, 1], y in [-2, 2]   (15 slots,  0..14)
//   vx row -> vy: x in [-2, 1], y in [-1, 2]   (16 slots, 15..30)
//   vy row -> vx: x in [-1, 2], y in [-2, 1]   (16 slots,  0..15)
//   vy row -> vy: x in [-2, 2], y in [-1, 1]   (15 slots, 16..30)
// so a full row has 31 coefficients.  A_c is symmetric, and each coupling is
// stored once (32 planes instead of 62):
//   plane 0       vx row: diagonal
//   planes 1..7   vx row: vx -> vx "forward" offsets (dy > 0, or dy = 0 and dx > 0)
//   planes 8..23  vx row: all 16 vx -> vy couplings
//   plane 24      vy row: diagonal
//   planes 25..31 vy row: vy -> vy forward offsets
// A backward vx -> vx (vy -> vy) coupling is the forward one stored at the
// neighbour; a vy -> vx coupling is the vx -> vy one stored at the vx
// neighbour.  Each plane is (ny+1) x ld in the common row-stride layout;
// coefficients of rows that are not unknowns are 0.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "stencil.hpp"

namespace stk {

constexpr int NCOEF = 31;    // full row
constexpr int NPLANES = 32;  // stored planes per coarse level
constexpr int PL_VY = 24;    // first plane of the vy rows

// slot s of a row of component a -> neighbour component b and offset (dx, dy)
__host__ __device__ constexpr int slot_comp(int a, int s) { return a == 0 ? (s < 15 ? 0 : 1) : (s < 16 ? 0 : 1); }
__host__ __device__ constexpr int slot_dx(int a, int s) {
    return a == 0 ? (s < 15 ? s % 3 - 1 : (s - 15) % 4 - 2) : (s < 16 ? s % 4 - 1 : (s - 16) % 5 - 2);
}
__host__ __device__ constexpr int slot_dy(int a, int s) {
    return a == 0 ? (s < 15 ? s / 3 - 2 : (s - 15) / 4 - 1) : (s < 16 ? s / 4 - 2 : (s - 16) / 5 - 1);
}
// inverse map; -1 outside the window
__host__ __device__ constexpr int offset_slot(int a, int b, int dx, int dy) {
    if (a == 0 && b == 0) return (dx >= -1 && dx <= 1 && dy >= -2 && dy <= 2) ? (dy + 2) * 3 + (dx + 1) : -1;
    if (a == 0) return (dx >= -2 && dx <= 1 && dy >= -1 && dy <= 2) ? 15 + (dy + 1) * 4 + (dx + 2) : -1;
    if (b == 0) return (dx >= -1 && dx <= 2 && dy >= -2 && dy <= 1) ? (dy + 2) * 4 + (dx + 1) : -1;
    return (dx >= -2 && dx <= 2 && dy >= -1 && dy <= 1) ? 16 + (dy + 1) * 5 + (dx + 2) : -1;
}

__host__ __device__ constexpr bool forward(int dx, int dy) { return dy > 0 || (dy == 0 && dx > 0); }
// rank of same-component slot s among the forward offsets of its window
__host__ __device__ constexpr int forward_rank(int a, int s) {
    int r = 0;
    for (int q = (a == 0 ? 0 : 16); q < s; ++q) r += forward(slot_dx(a, q), slot_dy(a, q)) ? 1 : 0;
    return r;
}

// Where the coefficient of full slot s of a row of component a is stored:
// plane and the (i, j) offset of the row that stores it; own = the row itself
// stores it (a vy -> vx coupling at offset (0, 0) is stored by the vx row of
// the same (i, j), not by this row).
struct SlotSrc {
    int plane, ndx, ndy;
    bool own;
};
__host__ __device__ constexpr SlotSrc slot_src(int a, int s) {
    const int b = slot_comp(a, s), dx = slot_dx(a, s), dy = slot_dy(a, s);
    if (a == 0 && b == 0) {
        if (dx == 0 && dy == 0) return {0, 0, 0, true};
        if (forward(dx, dy)) return {1 + forward_rank(0, s), 0, 0, true};
        return {1 + forward_rank(0, offset_slot(0, 0, -dx, -dy)), dx, dy, false};
    }
    if (a == 0) return {8 + (s - 15), 0, 0, true};
    if (b == 1) {
        if (dx == 0 && dy == 0) return {PL_VY, 0, 0, true};
        if (forward(dx, dy)) return {PL_VY + 1 + forward_rank(1, s), 0, 0, true};
        return {PL_VY + 1 + forward_rank(1, offset_slot(1, 1, -dx, -dy)), dx, dy, false};
    }
    return {8 + (offset_slot(0, 1, -dx, -dy) - 15), dx, dy, false};  // vy -> vx: at the vx neighbour
}

// Full-row coefficient of slot s at row (a, i, j) of a level of nx x ny cells.
// A neighbour outside the (nx+1) x (ny+1) box reads as 0: its load is clamped
// onto the box and the value dropped, so no load sits under a branch and a
// row's 31 loads are issued back to back (under branches each one waited for
// the one before).
template <typename T>
__host__ __device__ __forceinline__ T stencil_coef(const T* st, int64_t plane, int64_t ld, int nx, int ny, int a, int s,
                                                   int i, int j) {
    const SlotSrc src = slot_src(a, s);
    const int pi = i + src.ndx, pj = j + src.ndy;
    // (i, j) itself is inside every plane: no bounds check
    if (src.ndx == 0 && src.ndy == 0) return st[src.plane * plane + (int64_t)j * ld + i];
    const bool in = pi >= 0 && pi <= nx && pj >= 0 && pj <= ny;
    const int ci = pi < 0 ? 0 : (pi > nx ? nx : pi), cj = pj < 0 ? 0 : (pj > ny ? ny : pj);
    const T c = st[src.plane * plane + (int64_t)cj * ld + ci];
    return in ? c : T(0);
}

// (A v) at the unknown (a, i, j) from the stored stencil, with v(c, i, j)
// given by the loader lv (component c, 0 outside the grid and on the walls);
// also returns the diagonal coefficient.  Fixed slot order: every kernel that
// applies a stored stencil goes through this function, so they agree bit for
// bit.
template <typename T, typename LV>
__device__ __forceinline__ T stencil_av_l(const T* __restrict__ st, int64_t plane, int a, const LV& lv, int64_t ld,
                                          int nx, int ny, int i, int j, T& diag) {
    T s = T(0);
    if (a == 0) {
#pragma unroll
        for (int q = 0; q < NCOEF; ++q) {
            const T v = lv(slot_comp(0, q), i + slot_dx(0, q), j + slot_dy(0, q));
            s += stencil_coef<T>(st, plane, ld, nx, ny, 0, q, i, j) * v;
        }
        diag = st[(int64_t)j * ld + i];
    } else {
#pragma unroll
        for (int q = 0; q < NCOEF; ++q) {
            const T v = lv(slot_comp(1, q), i + slot_dx(1, q), j + slot_dy(1, q));
            s += stencil_coef<T>(st, plane, ld, nx, ny, 1, q, i, j) * v;
        }
        diag = st[PL_VY * plane + (int64_t)j * ld + i];
    }
    return s;
}

// the velocity pair in global memory
template <typename T>
struct GlobalPair {
    const T *vx, *vy;
    int64_t ld;
    int nx, ny;
    __device__ __forceinline__ T operator()(int c, int i, int j) const {
        return c == 0 ? ldvx<T>(vx, ld, nx, ny, i, j) : ldvy<T>(vy, ld, nx, ny, i, j);
    }
};

template <typename T>
__device__ __forceinline__ T stencil_av(const T* __restrict__ st, int64_t plane, int a, const T* __restrict__ vx,
                                        const T* __restrict__ vy, int64_t ld, int nx, int ny, int i, int j,
                                        T& diag) {
    return stencil_av_l<T>(st, plane, a, GlobalPair<T>{vx, vy, ld, nx, ny}, ld, nx, ny, i, j, diag);
}

}  // namespace stk
