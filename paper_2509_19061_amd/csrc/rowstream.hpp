// Row-streaming engine for the one-sweep stencils on the finest (matrix-free)
// grid: fused Jacobi, residual, energy norms, and the finest level of the
// batched V-cycle.
//
// A wave owns a strip of SW = 62 columns and a segment of seg_rows rows.  Its 64
// lanes hold the columns x0 - 1 .. x0 + 62 (the strip and one neighbour
// column on each side); it walks up the rows, loading each row of every field
// once with coalesced buffer loads, keeps a window of three rows in registers
// and takes the columns i - 1 and i + 1 from the neighbouring lanes (DPP).
// Nothing goes through LDS and waves never wait for each other.
//
// Walls and everything outside the arrays read as 0 through the buffer
// resources (a lane offset past the row for a column outside a field, an
// empty row for a row outside it), so the operands are exactly those of a
// gather from global memory, and the results, through the shared stencil
// functions, are bit-identical to it.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "stencil.hpp"
#include "wave.hpp"

namespace stk {
namespace rows {

constexpr int SW = 62;  // columns a wave owns
constexpr int SR = 64;  // the most rows a wave walks
constexpr int WPB = 4;  // waves per workgroup (independent)
// Fewer waves than this (16 per CU of a 256-CU chip) leave the walk's latency
// exposed: a grid whose 64-row segments give fewer is cut into 32- or 16-row
// segments (each re-reads the two rows around it).  At 2048^2 (1122 waves of
// 64 rows) 16-row segments made the FCG iteration 2.7 % faster, at 1024^2 5 %;
// 4096^2 and larger keep 64.
constexpr int64_t MIN_WAVES = 4096;

__host__ __device__ inline int strips(int nx) { return (nx + 1 + SW - 1) / SW; }
// rows a wave walks on an nx x ny grid: SR, or SR / 2, SR / 4 (at least 16)
__host__ __device__ inline int seg_rows(int nx, int ny) {
    int r = SR;
    while (r > 16 && (int64_t)strips(nx) * ((ny + 1 + r - 1) / r) < MIN_WAVES) r >>= 1;
    return r;
}
__host__ __device__ inline int segments(int nx, int ny) {
    const int r = seg_rows(nx, ny);
    return (ny + 1 + r - 1) / r;
}
// workgroups for one (nx, ny) grid
__host__ __device__ inline int workgroups(int nx, int ny) {
    return (int)(((int64_t)strips(nx) * segments(nx, ny) + WPB - 1) / WPB);
}

// One grid row of the inputs at this lane's column: velocity, viscosities,
// right-hand side (b or f) and, for the residual with a pressure, p.
template <typename T>
struct Row {
    T vx, vy, ec, en, bx, by, p;
};

template <typename T>
struct Loader {
    const T *vx, *vy, *ec, *en, *bx, *by, *p;
    int64_t ld;
    int nx, ny;
    unsigned o_inner, o_cell;  // the column, or OOB: inner = 1..nx-1 (vx, eta_n-hat, bx), cell = 0..nx-1

    // vx, eta_c, bx, p live on rows 0..ny-1; vy, eta_n-hat (0 on boundary nodes), by on rows 1..ny-1
    __device__ __forceinline__ Row<T> load(int r) const {
        const size_t w = (size_t)(nx + 1) * sizeof(T);
        const size_t wx = (r >= 0 && r <= ny - 1) ? w : 0, wy = (r >= 1 && r <= ny - 1) ? w : 0;
        const int64_t o = (int64_t)r * ld;
        Row<T> q;
        q.vx = buf_load<T>(buf_rsrc(vx + o, wx), o_inner);
        q.vy = buf_load<T>(buf_rsrc(vy + o, wy), o_cell);
        q.ec = buf_load<T>(buf_rsrc(ec + o, wx), o_cell);
        q.en = buf_load<T>(buf_rsrc(en + o, wy), o_inner);
        q.bx = bx ? buf_load<T>(buf_rsrc(bx + o, wx), o_inner) : T(0);  // no right-hand side: b = 0
        q.by = by ? buf_load<T>(buf_rsrc(by + o, wy), o_cell) : T(0);
        q.p = p ? buf_load<T>(buf_rsrc(p + o, wx), o_cell) : T(0);
        return q;
    }
};

template <typename T>
__device__ __forceinline__ Loader<T> make_loader(const T* vx, const T* vy, const T* ec, const T* en, const T* bx,
                                                 const T* by, const T* p, int64_t ld, int nx, int ny, int i) {
    const unsigned col = (unsigned)i * (unsigned)sizeof(T);
    return Loader<T>{vx, vy, ec, en, bx, by, p, ld, nx, ny, (i >= 1 && i <= nx - 1) ? col : OOB,
                     (i >= 0 && i <= nx - 1) ? col : OOB};
}

// A wave's strip, segment and lane column, from its index wv among the
// strips x segments waves of one grid.
struct Place {
    int i, y0, y1;
    bool own;  // lane inside the strip and the grid
};
__device__ __forceinline__ Place place(int wv, int nx, int ny) {
    Place q;
    const int sr = seg_rows(nx, ny), nstrip = strips(nx), nseg = (ny + 1 + sr - 1) / sr, lane = threadIdx.x & 63;
    const int strip = wv % nstrip, seg = wv / nstrip;
    q.i = strip * SW - 1 + lane;
    q.y0 = seg * sr;
    q.y1 = seg < nseg ? min(q.y0 + sr, ny + 1) : q.y0;
    q.own = lane >= 1 && lane <= SW && q.i <= nx;
    return q;
}
// this wave's index within its workgroup (uniform)
__device__ __forceinline__ int wave_in_group() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// Walks rows y0 .. y1-1 with the window (a, b, c) = rows (j-1, j, j+1),
// loading row j+2 while row j is processed; body(a, b, c, j).  L is any
// loader with Row<T> load(int r).
template <typename T, typename LD, typename F>
__device__ __forceinline__ void walk_rows(const LD& L, int y0, int y1, F body) {
    Row<T> r0 = L.load(y0 - 1), r1 = L.load(y0), r2 = L.load(y0 + 1), r3;
    for (int j = y0; j < y1; j += 4) {  // four rows per trip: the window rotates by renaming
        r3 = L.load(j + 2);
        body(r0, r1, r2, j);
        if (j + 1 >= y1) break;
        r0 = L.load(j + 3);
        body(r1, r2, r3, j + 1);
        if (j + 2 >= y1) break;
        r1 = L.load(j + 4);
        body(r2, r3, r0, j + 2);
        if (j + 3 >= y1) break;
        r2 = L.load(j + 5);
        body(r3, r0, r1, j + 3);
    }
}

// Damped Jacobi at row j of this lane's column (a, b, c = rows j-1, j, j+1):
// the new vx(i, j), vy(i, j).
template <typename T>
__device__ __forceinline__ void jacobi_row(const Row<T>& a, const Row<T>& b, const Row<T>& c, T omega, T idx, T idy,
                                           T& ux, T& uy) {
    const T vxl = wave_shift<DPP_FROM_PREV>(b.vx), vxr = wave_shift<DPP_FROM_NEXT>(b.vx);
    const T vyl = wave_shift<DPP_FROM_PREV>(b.vy), vyr = wave_shift<DPP_FROM_NEXT>(b.vy);
    const T vytl = wave_shift<DPP_FROM_PREV>(c.vy);  // vy(i-1, j+1)
    const T vxrb = wave_shift<DPP_FROM_NEXT>(a.vx);  // vx(i+1, j-1)
    const T ecl = wave_shift<DPP_FROM_PREV>(b.ec), enr = wave_shift<DPP_FROM_NEXT>(b.en);
    ux = jac_vx<T>(b.vx, vxl, vxr, a.vx, c.vx, b.vy, vyl, c.vy, vytl, ecl, b.ec, b.en, c.en, b.bx, omega, idx, idy);
    uy = jac_vy<T>(b.vy, vyl, vyr, a.vy, c.vy, b.vx, vxr, a.vx, vxrb, a.ec, b.ec, b.en, enr, b.by, omega, idx, idy);
}

// Residuals at row j in the arithmetic type A (T widened on use), with the
// right-hand side b = f - G p when p is given (bx, by hold f).
template <typename A>
struct Res {
    A rx, ry, rp;  // r at vx(i, j), vy(i, j) and -D v at cell (i, j)
    A dx_, dy_;    // diag(-M) at vx(i, j), vy(i, j)
};
template <typename T, typename A>
__device__ __forceinline__ Res<A> residual_row(const Row<T>& a, const Row<T>& b, const Row<T>& c, bool has_p, A idx,
                                               A idy) {
    const T vxl = wave_shift<DPP_FROM_PREV>(b.vx), vxr = wave_shift<DPP_FROM_NEXT>(b.vx);
    const T vyl = wave_shift<DPP_FROM_PREV>(b.vy), vyr = wave_shift<DPP_FROM_NEXT>(b.vy);
    const T vytl = wave_shift<DPP_FROM_PREV>(c.vy);  // vy(i-1, j+1)
    const T vxrb = wave_shift<DPP_FROM_NEXT>(a.vx);  // vx(i+1, j-1)
    const T ecl = wave_shift<DPP_FROM_PREV>(b.ec), enr = wave_shift<DPP_FROM_NEXT>(b.en);
    Res<A> r;
    {  // vx(i, j)
        A bx = A(b.bx);
        if (has_p) bx += (A(b.p) - A(wave_shift<DPP_FROM_PREV>(b.p))) * idx;
        const A m = mv_x<A>(A(b.vx), A(vxl), A(vxr), A(a.vx), A(c.vx), A(b.vy), A(vyl), A(c.vy), A(vytl), A(ecl),
                            A(b.ec), A(b.en), A(c.en), idx, idy);
        r.rx = bx - m;
        r.dx_ = diag_x<A>(A(ecl), A(b.ec), A(b.en), A(c.en), idx, idy);
    }
    {  // vy(i, j)
        A by = A(b.by);
        if (has_p) by += (A(b.p) - A(a.p)) * idy;
        const A m = mv_y<A>(A(b.vy), A(vyl), A(vyr), A(a.vy), A(c.vy), A(b.vx), A(vxr), A(a.vx), A(vxrb), A(a.ec),
                            A(b.ec), A(b.en), A(enr), idx, idy);
        r.ry = by - m;
        r.dy_ = diag_y<A>(A(a.ec), A(b.ec), A(b.en), A(enr), idx, idy);
    }
    r.rp = -((A(vxr) - A(b.vx)) * idx + (A(c.vy) - A(b.vy)) * idy);
    return r;
}

// Row stores of a velocity-shaped pair at row j: vx has rows 0..ny-1 and
// columns 0..nx, vy rows 0..ny and columns 0..nx-1 (s_x, s_y: lane offsets).
template <typename T>
__device__ __forceinline__ void store_pair(T* ox, T* oy, int64_t ld, int nx, int ny, int j, T x, T y, unsigned s_x,
                                           unsigned s_y) {
    const int64_t o = (int64_t)j * ld;
    buf_store(x, buf_rsrc(ox + o, j <= ny - 1 ? (size_t)(nx + 1) * sizeof(T) : 0), s_x);
    buf_store(y, buf_rsrc(oy + o, j <= ny ? (size_t)nx * sizeof(T) : 0), s_y);
}

}  // namespace rows
}  // namespace stk
