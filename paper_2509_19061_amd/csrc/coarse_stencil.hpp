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
// so each unknown stores 31 coefficients.  A level's stencil is 62 planes
// (31 for vx rows, then 31 for vy rows), each plane (ny+1) x ld in the common
// row-stride layout; coefficients to walls and outside the grid are 0.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "stencil.hpp"

namespace stk {

constexpr int NCOEF = 31;
constexpr int CENTER_X = 7;   // vx row, vx(0, 0)
constexpr int CENTER_Y = 23;  // vy row, vy(0, 0)

// slot s of a row of component a -> neighbour component b and offset (dx, dy)
__host__ __device__ constexpr int slot_comp(int a, int s) { return a == 0 ? (s < 15 ? 0 : 1) : (s < 16 ? 0 : 1); }
__host__ __device__ constexpr int slot_dx(int a, int s) {
    return a == 0 ? (s < 15 ? s % 3 - 1 : (s - 15) % 4 - 2) : (s < 16 ? s % 4 - 1 : (s - 16) % 5 - 2);
}
__host__ __device__ constexpr int slot_dy(int a, int s) {
    return a == 0 ? (s < 15 ? s / 3 - 2 : (s - 15) / 4 - 1) : (s < 16 ? s / 4 - 2 : (s - 16) / 5 - 1);
}
// inverse map; -1 outside the window
__host__ __device__ inline int offset_slot(int a, int b, int dx, int dy) {
    if (a == 0 && b == 0) return (dx >= -1 && dx <= 1 && dy >= -2 && dy <= 2) ? (dy + 2) * 3 + (dx + 1) : -1;
    if (a == 0) return (dx >= -2 && dx <= 1 && dy >= -1 && dy <= 2) ? 15 + (dy + 1) * 4 + (dx + 2) : -1;
    if (b == 0) return (dx >= -1 && dx <= 2 && dy >= -2 && dy <= 1) ? (dy + 2) * 4 + (dx + 1) : -1;
    return (dx >= -2 && dx <= 2 && dy >= -1 && dy <= 1) ? 16 + (dy + 1) * 5 + (dx + 2) : -1;
}

// (A v) at the unknown (a, i, j) from the stored stencil; also returns the
// diagonal coefficient.  Fixed slot order.
template <typename T>
__device__ __forceinline__ T stencil_av(const T* __restrict__ st, int64_t plane, int a, const T* __restrict__ vx,
                                        const T* __restrict__ vy, int64_t ld, int nx, int ny, int i, int j,
                                        T& diag) {
    const T* row = st + (int64_t)a * NCOEF * plane + (int64_t)j * ld + i;
    T s = T(0);
    if (a == 0) {
#pragma unroll
        for (int q = 0; q < NCOEF; ++q) {
            const int dx = slot_dx(0, q), dy = slot_dy(0, q);
            const T v = slot_comp(0, q) == 0 ? ldvx<T>(vx, ld, nx, ny, i + dx, j + dy) : ldvy<T>(vy, ld, nx, ny, i + dx, j + dy);
            s += row[q * plane] * v;
        }
        diag = row[CENTER_X * plane];
    } else {
#pragma unroll
        for (int q = 0; q < NCOEF; ++q) {
            const int dx = slot_dx(1, q), dy = slot_dy(1, q);
            const T v = slot_comp(1, q) == 0 ? ldvx<T>(vx, ld, nx, ny, i + dx, j + dy) : ldvy<T>(vy, ld, nx, ny, i + dx, j + dy);
            s += row[q * plane] * v;
        }
        diag = row[CENTER_Y * plane];
    }
    return s;
}

}  // namespace stk
