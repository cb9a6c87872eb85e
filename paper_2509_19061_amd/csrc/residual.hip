// Residual and energy-norm kernels (paper Sec. 6.4).
//
// residual: r_v = b - M v on the velocity unknowns, r_p = -D v per cell, with
//           b = f - G p folded on the fly.
// energy:   FP64 sums N_v = sum r_v^2/d, N_p = sum r_p^2 eta_c/(2/dx^2 + 2/dy^2),
//           N_f = sum f^2/d.
//
// Both stream rows like the fused Jacobi kernel: a wave owns a strip of
// SW = 62 columns and SR rows, its 64 lanes hold the strip and one neighbour
// column on each side, each row of every field is loaded once (coalesced
// buffer loads; walls and outside read as 0), three rows stay in registers
// and the columns i +- 1 come from neighbouring lanes (DPP).  The energy sums
// accumulate per lane row by row, then over the wave's lanes (shuffles), one
// triple per wave; one workgroup adds the triples in a fixed order, so the
// result is bitwise reproducible.
#include <algorithm>

#include "stencil.hpp"
#include "stk_internal.hpp"
#include "wave.hpp"

namespace stk {
namespace {

constexpr int SW = 62;  // columns a wave owns
constexpr int SR = 64;  // rows a wave walks
constexpr int WPB = 4;  // waves per workgroup (independent)

// One grid row of the inputs at this lane's column.
template <typename T>
struct Row {
    T vx, vy, ec, en, fx, fy, p;
};

template <typename T>
struct Loader {
    const T *vx, *vy, *ec, *en, *fx, *fy, *p;
    int64_t ld;
    int nx, ny;
    unsigned o_inner, o_cell;  // the column, or OOB: inner = 1..nx-1 (vx, eta_n-hat, fx), cell = 0..nx-1

    // vx, eta_c, fx, p live on rows 0..ny-1; vy, eta_n-hat (0 on boundary nodes), fy on rows 1..ny-1
    __device__ __forceinline__ Row<T> load(int r) const {
        const size_t w = (size_t)(nx + 1) * sizeof(T);
        const size_t wx = (r >= 0 && r <= ny - 1) ? w : 0, wy = (r >= 1 && r <= ny - 1) ? w : 0;
        const int64_t o = (int64_t)r * ld;
        Row<T> q;
        q.vx = buf_load<T>(buf_rsrc(vx + o, wx), o_inner);
        q.vy = buf_load<T>(buf_rsrc(vy + o, wy), o_cell);
        q.ec = buf_load<T>(buf_rsrc(ec + o, wx), o_cell);
        q.en = buf_load<T>(buf_rsrc(en + o, wy), o_inner);
        q.fx = buf_load<T>(buf_rsrc(fx + o, wx), o_inner);
        q.fy = buf_load<T>(buf_rsrc(fy + o, wy), o_cell);
        q.p = p ? buf_load<T>(buf_rsrc(p + o, wx), o_cell) : T(0);
        return q;
    }
};

// Residuals at row j of this lane's column from rows a = j-1, b = j, c = j+1,
// in the arithmetic type A (T widened on use).
template <typename A>
struct Res {
    A rx, ry, rp;  // r at vx(i, j), vy(i, j) and cell (i, j)
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
    const T pl = wave_shift<DPP_FROM_PREV>(b.p);
    Res<A> r;
    {  // vx(i, j)
        A bx = A(b.fx);
        if (has_p) bx += (A(b.p) - A(pl)) * idx;
        const A m = mv_x<A>(A(b.vx), A(vxl), A(vxr), A(a.vx), A(c.vx), A(b.vy), A(vyl), A(c.vy), A(vytl), A(ecl),
                            A(b.ec), A(b.en), A(c.en), idx, idy);
        r.rx = bx - m;
        r.dx_ = diag_x<A>(A(ecl), A(b.ec), A(b.en), A(c.en), idx, idy);
    }
    {  // vy(i, j)
        A by = A(b.fy);
        if (has_p) by += (A(b.p) - A(a.p)) * idy;
        const A m = mv_y<A>(A(b.vy), A(vyl), A(vyr), A(a.vy), A(c.vy), A(b.vx), A(vxr), A(a.vx), A(vxrb), A(a.ec),
                            A(b.ec), A(b.en), A(enr), idx, idy);
        r.ry = by - m;
        r.dy_ = diag_y<A>(A(a.ec), A(b.ec), A(b.en), A(enr), idx, idy);
    }
    r.rp = -((A(vxr) - A(b.vx)) * idx + (A(c.vy) - A(b.vy)) * idy);
    return r;
}

// This wave's strip, segment and lane column (wave index uniform, so every
// row-dependent quantity stays scalar).
struct Place {
    int wv, i, y0, y1;
    bool own;  // lane inside the strip
};
__device__ __forceinline__ Place place(int nstrip, int nseg, int nx, int ny) {
    Place q;
    q.wv = xcd_tile((int)blockIdx.x, (int)gridDim.x) * WPB + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63, strip = q.wv % nstrip, seg = q.wv / nstrip;
    q.i = strip * SW - 1 + lane;
    q.y0 = seg * SR;
    q.y1 = seg < nseg ? std::min(q.y0 + SR, ny + 1) : q.y0;
    q.own = lane >= 1 && lane <= SW && q.i <= nx;
    return q;
}

template <typename T>
__device__ __forceinline__ Loader<T> make_loader(const T* vx, const T* vy, const T* ec, const T* en, const T* fx,
                                                 const T* fy, const T* p, int64_t ld, int nx, int ny, int i) {
    const unsigned col = (unsigned)i * (unsigned)sizeof(T);
    return Loader<T>{vx, vy, ec, en, fx, fy, p, ld, nx, ny, (i >= 1 && i <= nx - 1) ? col : OOB,
                     (i >= 0 && i <= nx - 1) ? col : OOB};
}

// Walks rows y0 .. y1-1 with the window (a, b, c) = rows (j-1, j, j+1),
// loading row j+2 while row j is processed; body(a, b, c, j).
template <typename T, typename F>
__device__ __forceinline__ void walk_rows(const Loader<T>& L, int y0, int y1, F body) {
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

template <typename T>
__global__ __launch_bounds__(64 * WPB) void k_residual(int nx, int ny, int64_t ld, T idx, T idy, int nstrip, int nseg,
                                                       const T* __restrict__ vx, const T* __restrict__ vy,
                                                       const T* __restrict__ p, const T* __restrict__ ec,
                                                       const T* __restrict__ en, const T* __restrict__ fx,
                                                       const T* __restrict__ fy, T* __restrict__ rx,
                                                       T* __restrict__ ry, T* __restrict__ rp) {
    const Place q = place(nstrip, nseg, nx, ny);
    if (q.y0 >= q.y1) return;  // the whole wave
    const Loader<T> L = make_loader<T>(vx, vy, ec, en, fx, fy, p, ld, nx, ny, q.i);
    const int i = q.i;
    const bool xcol = i >= 1 && i <= nx - 1, ycol = i >= 0 && i <= nx - 1;
    const unsigned col = (unsigned)i * (unsigned)sizeof(T);
    const unsigned s_x = q.own ? col : OOB, s_y = (q.own && ycol) ? col : OOB;
    walk_rows<T>(L, q.y0, q.y1, [&](const Row<T>& a, const Row<T>& b, const Row<T>& c, int j) {
        const Res<T> r = residual_row<T, T>(a, b, c, p != nullptr, idx, idy);
        const bool ux = xcol && j <= ny - 1, uy = ycol && j >= 1 && j <= ny - 1;
        const int64_t o = (int64_t)j * ld;
        // rx: rows 0..ny-1, columns 0..nx; ry: rows 0..ny, columns 0..nx-1; rp: cells
        buf_store(ux ? r.rx : T(0), buf_rsrc(rx + o, j <= ny - 1 ? (size_t)(nx + 1) * sizeof(T) : 0), s_x);
        buf_store(uy ? r.ry : T(0), buf_rsrc(ry + o, j <= ny ? (size_t)nx * sizeof(T) : 0), s_y);
        if (rp) buf_store(r.rp, buf_rsrc(rp + o, j <= ny - 1 ? (size_t)nx * sizeof(T) : 0), s_y);
    });
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// One triple (N_v, N_p, N_f) per wave -> part[3 wv + c].
template <typename T>
__global__ __launch_bounds__(64 * WPB) void k_energy(int nx, int ny, int64_t ld, double idx, double idy, double sp,
                                                     int nstrip, int nseg, const T* __restrict__ vx,
                                                     const T* __restrict__ vy, const T* __restrict__ p,
                                                     const T* __restrict__ ec, const T* __restrict__ en,
                                                     const T* __restrict__ fx, const T* __restrict__ fy,
                                                     double* __restrict__ part) {
    const Place q = place(nstrip, nseg, nx, ny);
    if (q.y0 >= q.y1) return;  // the whole wave (no triple: it is past the last one)
    const Loader<T> L = make_loader<T>(vx, vy, ec, en, fx, fy, p, ld, nx, ny, q.i);
    const int i = q.i;
    const bool xcol = q.own && i >= 1 && i <= nx - 1, ycol = q.own && i >= 0 && i <= nx - 1;
    double nv = 0.0, np = 0.0, nf = 0.0;
    walk_rows<T>(L, q.y0, q.y1, [&](const Row<T>& a, const Row<T>& b, const Row<T>& c, int j) {
        const Res<double> r = residual_row<T, double>(a, b, c, p != nullptr, idx, idy);
        if (xcol && j <= ny - 1) {
            const double f = b.fx;
            nv += r.rx * r.rx / r.dx_;
            nf += f * f / r.dx_;
        }
        if (ycol && j >= 1 && j <= ny - 1) {
            const double f = b.fy;
            nv += r.ry * r.ry / r.dy_;
            nf += f * f / r.dy_;
        }
        if (ycol && j <= ny - 1) np += r.rp * r.rp * double(b.ec) / sp;
    });
    nv = wave_sum(nv);
    np = wave_sum(np);
    nf = wave_sum(nf);
    if ((threadIdx.x & 63) == 0) {
        part[3 * (int64_t)q.wv + 0] = nv;
        part[3 * (int64_t)q.wv + 1] = np;
        part[3 * (int64_t)q.wv + 2] = nf;
    }
}

// Fixed-order sum of n triples -> dst[0..2].
__global__ __launch_bounds__(1024) void k_reduce_triples(const double* __restrict__ part, int64_t n,
                                                         double* __restrict__ dst) {
    __shared__ double red[3][1024 / 64];
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t q = threadIdx.x; q < n; q += 1024)
        for (int c = 0; c < 3; ++c) s[c] += part[3 * q + c];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int c = 0; c < 3; ++c) {
        const double v = wave_sum(s[c]);
        if (lane == 0) red[c][w] = v;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double v = 0.0;
        for (int q = 0; q < 1024 / 64; ++q) v += red[threadIdx.x][q];
        dst[threadIdx.x] = v;
    }
}

struct Shape {
    int nstrip, nseg;
    int64_t waves;
    dim3 grid;
};
inline Shape shape(const stk_grid* g) {
    Shape s;
    s.nstrip = (g->nx + 1 + SW - 1) / SW;
    s.nseg = (g->ny + 1 + SR - 1) / SR;
    s.waves = (int64_t)s.nstrip * s.nseg;
    s.grid = dim3((unsigned)((s.waves + WPB - 1) / WPB));
    return s;
}

}  // namespace

int launch_residual(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const void* vx, const void* vy, const void* p,
                    const void* eta_c, const void* eta_n, const void* fx, const void* fy, void* rx, void* ry,
                    void* rp) {
    const Shape s = shape(g);
    const dim3 block(64 * WPB);
    if (dt == STK_F64)
        hipLaunchKernelGGL(k_residual<double>, s.grid, block, 0, ctx->stream, g->nx, g->ny, g->ld, 1.0 / g->dx,
                           1.0 / g->dy, s.nstrip, s.nseg, (const double*)vx, (const double*)vy, (const double*)p,
                           (const double*)eta_c, (const double*)eta_n, (const double*)fx, (const double*)fy,
                           (double*)rx, (double*)ry, (double*)rp);
    else
        hipLaunchKernelGGL(k_residual<float>, s.grid, block, 0, ctx->stream, g->nx, g->ny, g->ld, float(1.0 / g->dx),
                           float(1.0 / g->dy), s.nstrip, s.nseg, (const float*)vx, (const float*)vy, (const float*)p,
                           (const float*)eta_c, (const float*)eta_n, (const float*)fx, (const float*)fy, (float*)rx,
                           (float*)ry, (float*)rp);
    STK_HIP(hipGetLastError());
    return STK_OK;
}

int launch_energy(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const void* vx, const void* vy, const void* p,
                  const void* eta_c, const void* eta_n, const void* fx, const void* fy, double* dst) {
    const Shape s = shape(g);
    void* part = nullptr;
    STK_TRY(scratch(ctx, stk_ctx::S_PART, sizeof(double) * 3 * (size_t)s.waves, &part));
    const double idx = 1.0 / g->dx, idy = 1.0 / g->dy, sp = 2.0 * idx * idx + 2.0 * idy * idy;
    const dim3 block(64 * WPB);
    if (dt == STK_F64)
        hipLaunchKernelGGL(k_energy<double>, s.grid, block, 0, ctx->stream, g->nx, g->ny, g->ld, idx, idy, sp,
                           s.nstrip, s.nseg, (const double*)vx, (const double*)vy, (const double*)p,
                           (const double*)eta_c, (const double*)eta_n, (const double*)fx, (const double*)fy,
                           (double*)part);
    else
        hipLaunchKernelGGL(k_energy<float>, s.grid, block, 0, ctx->stream, g->nx, g->ny, g->ld, idx, idy, sp,
                           s.nstrip, s.nseg, (const float*)vx, (const float*)vy, (const float*)p,
                           (const float*)eta_c, (const float*)eta_n, (const float*)fx, (const float*)fy,
                           (double*)part);
    hipLaunchKernelGGL(k_reduce_triples, dim3(1), dim3(1024), 0, ctx->stream, (const double*)part, s.waves, dst);
    STK_HIP(hipGetLastError());
    return STK_OK;
}

}  // namespace stk
