// Residual and energy-norm kernels (paper Sec. 6.4).
//
// residual: r_v = b - M v on the velocity unknowns, r_p = -D v per cell, with
//           b = f - G p folded on the fly.
// energy:   FP64 sums N_v = sum r_v^2/d, N_p = sum r_p^2 eta_c/(2/dx^2 + 2/dy^2),
//           N_f = sum f^2/d.
//
// Both stream rows like the fused Jacobi kernel: a wave owns a strip of
// SW = 62 columns and seg_rows rows, its 64 lanes hold the strip and one neighbour
// column on each side, each row of every field is loaded once (coalesced
// buffer loads; walls and outside read as 0), three rows stay in registers
// and the columns i +- 1 come from neighbouring lanes (DPP).  The energy sums
// accumulate per lane row by row, then over the wave's lanes (shuffles), one
// triple per wave; one workgroup adds the triples in a fixed order, so the
// result is bitwise reproducible.
#include "rowstream.hpp"
#include "stk_internal.hpp"

namespace stk {
namespace {

using namespace rows;

template <typename T>
__global__ __launch_bounds__(64 * WPB) void k_residual(int nx, int ny, int64_t ld, T idx, T idy,
                                                       const T* __restrict__ vx, const T* __restrict__ vy,
                                                       const T* __restrict__ p, const T* __restrict__ ec,
                                                       const T* __restrict__ en, const T* __restrict__ fx,
                                                       const T* __restrict__ fy, T* __restrict__ rx,
                                                       T* __restrict__ ry, T* __restrict__ rp) {
    const int wv = xcd_tile((int)blockIdx.x, (int)gridDim.x) * WPB + wave_in_group();
    const Place q = place(wv, nx, ny);
    if (q.y0 >= q.y1) return;  // the whole wave
    const int i = q.i;
    const Loader<T> L = make_loader<T>(vx, vy, ec, en, fx, fy, p, ld, nx, ny, i);
    const bool xcol = i >= 1 && i <= nx - 1, ycol = i >= 0 && i <= nx - 1;
    const unsigned col = (unsigned)i * (unsigned)sizeof(T);
    const unsigned s_x = q.own ? col : OOB, s_y = (q.own && ycol) ? col : OOB;
    walk_rows<T>(L, q.y0, q.y1, [&](const Row<T>& a, const Row<T>& b, const Row<T>& c, int j) {
        const Res<T> r = residual_row<T, T>(a, b, c, p != nullptr, idx, idy);
        const bool ux = xcol && j <= ny - 1, uy = ycol && j >= 1 && j <= ny - 1;
        // rx: rows 0..ny-1, columns 0..nx; ry: rows 0..ny, columns 0..nx-1; rp: cells
        store_pair<T>(rx, ry, ld, nx, ny, j, ux ? r.rx : T(0), uy ? r.ry : T(0), s_x, s_y);
        if (rp) buf_store(r.rp, buf_rsrc(rp + (int64_t)j * ld, j <= ny - 1 ? (size_t)nx * sizeof(T) : 0), s_y);
    });
}

// The FP64 residual r = b - M v rounded to FP32 for an FP32 V-cycle from
// zero: r32 <- (float) r, z32 <- 0 (FP32 arrays with the grid's row stride).
// The same rows and values as k_residual<double> followed by a rounding pass.
__global__ __launch_bounds__(64 * WPB) void k_residual_to32(int nx, int ny, int64_t ld, double idx, double idy,
                                                            const double* __restrict__ vx,
                                                            const double* __restrict__ vy,
                                                            const double* __restrict__ p,
                                                            const double* __restrict__ ec,
                                                            const double* __restrict__ en,
                                                            const double* __restrict__ fx,
                                                            const double* __restrict__ fy, float* __restrict__ r32x,
                                                            float* __restrict__ r32y, float* __restrict__ z32x,
                                                            float* __restrict__ z32y) {
    const int wv = xcd_tile((int)blockIdx.x, (int)gridDim.x) * WPB + wave_in_group();
    const Place q = place(wv, nx, ny);
    if (q.y0 >= q.y1) return;  // the whole wave
    const int i = q.i;
    const Loader<double> L = make_loader<double>(vx, vy, ec, en, fx, fy, p, ld, nx, ny, i);
    const bool xcol = i >= 1 && i <= nx - 1, ycol = i >= 0 && i <= nx - 1;
    const unsigned col = (unsigned)i * (unsigned)sizeof(float);
    const unsigned s_x = q.own ? col : OOB, s_y = (q.own && ycol) ? col : OOB;
    walk_rows<double>(L, q.y0, q.y1, [&](const Row<double>& a, const Row<double>& b, const Row<double>& c, int j) {
        const Res<double> r = residual_row<double, double>(a, b, c, p != nullptr, idx, idy);
        const bool ux = xcol && j <= ny - 1, uy = ycol && j >= 1 && j <= ny - 1;
        store_pair<float>(r32x, r32y, ld, nx, ny, j, ux ? (float)r.rx : 0.0f, uy ? (float)r.ry : 0.0f, s_x, s_y);
        store_pair<float>(z32x, z32y, ld, nx, ny, j, 0.0f, 0.0f, s_x, s_y);
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
                                                     const T* __restrict__ vx,
                                                     const T* __restrict__ vy, const T* __restrict__ p,
                                                     const T* __restrict__ ec, const T* __restrict__ en,
                                                     const T* __restrict__ fx, const T* __restrict__ fy,
                                                     double* __restrict__ part) {
    const int wv = xcd_tile((int)blockIdx.x, (int)gridDim.x) * WPB + wave_in_group();
    const Place q = place(wv, nx, ny);
    if (q.y0 >= q.y1) return;  // the whole wave (no triple: it is past the last one)
    const Loader<T> L = make_loader<T>(vx, vy, ec, en, fx, fy, p, ld, nx, ny, q.i);
    const int i = q.i;
    const bool xcol = q.own && i >= 1 && i <= nx - 1, ycol = q.own && i >= 0 && i <= nx - 1;
    double nv = 0.0, np = 0.0, nf = 0.0;
    walk_rows<T>(L, q.y0, q.y1, [&](const Row<T>& a, const Row<T>& b, const Row<T>& c, int j) {
        const Res<double> r = residual_row<T, double>(a, b, c, p != nullptr, idx, idy);
        if (xcol && j <= ny - 1) {
            const double f = b.bx;
            nv += r.rx * r.rx / r.dx_;
            nf += f * f / r.dx_;
        }
        if (ycol && j >= 1 && j <= ny - 1) {
            const double f = b.by;
            nv += r.ry * r.ry / r.dy_;
            nf += f * f / r.dy_;
        }
        if (ycol && j <= ny - 1) np += r.rp * r.rp * double(b.ec) / sp;
    });
    nv = wave_sum(nv);
    np = wave_sum(np);
    nf = wave_sum(nf);
    if ((threadIdx.x & 63) == 0) {
        part[3 * (int64_t)wv + 0] = nv;
        part[3 * (int64_t)wv + 1] = np;
        part[3 * (int64_t)wv + 2] = nf;
    }
}

// Fixed-order sum of n triples -> dst[0..2]; with `finish`, also
// dst[3] = sqrt((dst[0] + dst[1]) / dst[2]) and dst[4] = sqrt(dst[0] / dst[2]).
__global__ __launch_bounds__(1024) void k_reduce_triples(const double* __restrict__ part, int64_t n,
                                                         double* __restrict__ dst, int finish) {
    __shared__ double red[3][1024 / 64];
    __shared__ double tot[3];
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
        tot[threadIdx.x] = v;
    }
    if (!finish) return;
    __syncthreads();
    if (threadIdx.x == 0) {
        dst[3] = sqrt((tot[0] + tot[1]) / tot[2]);
        dst[4] = sqrt(tot[0] / tot[2]);
    }
}

}  // namespace

int launch_residual(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const void* vx, const void* vy, const void* p,
                    const void* eta_c, const void* eta_n, const void* fx, const void* fy, void* rx, void* ry,
                    void* rp) {
    const dim3 grid((unsigned)workgroups(g->nx, g->ny)), block(64 * WPB);
    if (dt == STK_F64)
        hipLaunchKernelGGL(k_residual<double>, grid, block, 0, ctx->stream, g->nx, g->ny, g->ld, 1.0 / g->dx,
                           1.0 / g->dy, (const double*)vx, (const double*)vy, (const double*)p,
                           (const double*)eta_c, (const double*)eta_n, (const double*)fx, (const double*)fy,
                           (double*)rx, (double*)ry, (double*)rp);
    else
        hipLaunchKernelGGL(k_residual<float>, grid, block, 0, ctx->stream, g->nx, g->ny, g->ld, float(1.0 / g->dx),
                           float(1.0 / g->dy), (const float*)vx, (const float*)vy, (const float*)p,
                           (const float*)eta_c, (const float*)eta_n, (const float*)fx, (const float*)fy, (float*)rx,
                           (float*)ry, (float*)rp);
    STK_HIP(hipGetLastError());
    return STK_OK;
}

int launch_residual_to32(stk_ctx* ctx, const stk_grid* g, const double* vx, const double* vy, const double* p,
                         const double* eta_c, const double* eta_n, const double* fx, const double* fy, float* r32x,
                         float* r32y, float* z32x, float* z32y) {
    hipLaunchKernelGGL(k_residual_to32, dim3((unsigned)workgroups(g->nx, g->ny)), dim3(64 * WPB), 0, ctx->stream,
                       g->nx, g->ny, g->ld, 1.0 / g->dx, 1.0 / g->dy, vx, vy, p, eta_c, eta_n, fx, fy, r32x, r32y,
                       z32x, z32y);
    STK_HIP(hipGetLastError());
    return STK_OK;
}

int64_t energy_partials(const stk_grid* g) { return (int64_t)strips(g->nx) * segments(g->nx, g->ny); }

int launch_energy(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const void* vx, const void* vy, const void* p,
                  const void* eta_c, const void* eta_n, const void* fx, const void* fy, double* dst) {
    void* part = nullptr;
    STK_TRY(scratch(ctx, stk_ctx::S_PART, sizeof(double) * 3 * (size_t)energy_partials(g), &part));
    return launch_energy_into(ctx, dt, g, vx, vy, p, eta_c, eta_n, fx, fy, static_cast<double*>(part), dst, false);
}

int launch_energy_into(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const void* vx, const void* vy, const void* p,
                       const void* eta_c, const void* eta_n, const void* fx, const void* fy, double* part,
                       double* dst, bool finish) {
    const int nwg = workgroups(g->nx, g->ny);
    const int64_t waves = energy_partials(g);  // one triple each (the rest leave at once)
    const double idx = 1.0 / g->dx, idy = 1.0 / g->dy, sp = 2.0 * idx * idx + 2.0 * idy * idy;
    const dim3 block(64 * WPB);
    if (dt == STK_F64)
        hipLaunchKernelGGL(k_energy<double>, dim3((unsigned)nwg), block, 0, ctx->stream, g->nx, g->ny, g->ld, idx,
                           idy, sp, (const double*)vx, (const double*)vy, (const double*)p,
                           (const double*)eta_c, (const double*)eta_n, (const double*)fx, (const double*)fy,
                           (double*)part);
    else
        hipLaunchKernelGGL(k_energy<float>, dim3((unsigned)nwg), block, 0, ctx->stream, g->nx, g->ny, g->ld, idx,
                           idy, sp, (const float*)vx, (const float*)vy, (const float*)p,
                           (const float*)eta_c, (const float*)eta_n, (const float*)fx, (const float*)fy,
                           (double*)part);
    hipLaunchKernelGGL(k_reduce_triples, dim3(1), dim3(1024), 0, ctx->stream, (const double*)part, waves, dst,
                       finish ? 1 : 0);
    STK_HIP(hipGetLastError());
    return STK_OK;
}

}  // namespace stk
