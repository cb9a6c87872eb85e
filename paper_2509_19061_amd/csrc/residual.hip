// Residual and energy-norm kernels (paper Sec. 6.4).
//
// residual: r_v = b - M v on the velocity unknowns, r_p = -D v per cell.
// energy:   per-workgroup FP64 partial sums of N_v = sum r_v^2/d,
//           N_p = sum r_p^2 eta_c/(2/dx^2 + 2/dy^2), N_f = sum f^2/d, reduced
//           with wave64 shuffles, then one workgroup adds the partials in a
//           fixed order (bitwise reproducible).
#include "stencil.hpp"
#include "stk_internal.hpp"

namespace stk {
namespace {

constexpr int BX = 64;
constexpr int BY = 4;
constexpr int NT = BX * BY;

template <typename T>
struct CellRes {
    T rx, ry, rp;     // residuals at vx(i,j), vy(i,j), cell (i,j)
    T dx_, dy_;       // diagonals of -M at vx(i,j), vy(i,j)
    bool ux, uy, uc;  // which of the three exist
};

// Residuals at cell (i,j): b = f - G p folded on the fly; A is the arithmetic
// type (the storage type T is widened on load).
template <typename T, typename A>
__device__ __forceinline__ CellRes<A> cell_residual(int nx, int ny, int64_t ld, A idx, A idy, const T* __restrict__ vx,
                                                    const T* __restrict__ vy, const T* __restrict__ p,
                                                    const T* __restrict__ ec, const T* __restrict__ en,
                                                    const T* __restrict__ fx, const T* __restrict__ fy, int i, int j) {
    CellRes<A> r{};
    auto VX = [&](int a, int b) { return A(ldvx(vx, ld, nx, ny, a, b)); };
    auto VY = [&](int a, int b) { return A(ldvy(vy, ld, nx, ny, a, b)); };
    auto ENH = [&](int a, int b) {
        return (a >= 1 && a <= nx - 1 && b >= 1 && b <= ny - 1) ? A(en[(int64_t)b * ld + a]) : A(0);
    };
    const int64_t k = (int64_t)j * ld + i;
    r.ux = is_vx_unknown(nx, ny, i, j);
    r.uy = is_vy_unknown(nx, ny, i, j);
    r.uc = i < nx && j < ny;
    if (r.ux) {
        const A ecl = A(ec[k - 1]), ecr = A(ec[k]), enb = ENH(i, j), ent = ENH(i, j + 1);
        A b = A(fx[k]);
        if (p) b += (A(p[k]) - A(p[k - 1])) * idx;
        const A m = mv_x<A>(VX(i, j), VX(i - 1, j), VX(i + 1, j), VX(i, j - 1), VX(i, j + 1), VY(i, j), VY(i - 1, j),
                            VY(i, j + 1), VY(i - 1, j + 1), ecl, ecr, enb, ent, idx, idy);
        r.rx = b - m;
        r.dx_ = diag_x<A>(ecl, ecr, enb, ent, idx, idy);
    }
    if (r.uy) {
        const A ecb = A(ec[k - ld]), ect = A(ec[k]), enl = ENH(i, j), enr = ENH(i + 1, j);
        A b = A(fy[k]);
        if (p) b += (A(p[k]) - A(p[k - ld])) * idy;
        const A m = mv_y<A>(VY(i, j), VY(i - 1, j), VY(i + 1, j), VY(i, j - 1), VY(i, j + 1), VX(i, j), VX(i + 1, j),
                            VX(i, j - 1), VX(i + 1, j - 1), ecb, ect, enl, enr, idx, idy);
        r.ry = b - m;
        r.dy_ = diag_y<A>(ecb, ect, enl, enr, idx, idy);
    }
    if (r.uc) r.rp = -((VX(i + 1, j) - VX(i, j)) * idx + (VY(i, j + 1) - VY(i, j)) * idy);
    return r;
}

template <typename T>
__global__ __launch_bounds__(NT) void k_residual(int nx, int ny, int64_t ld, T idx, T idy, const T* __restrict__ vx,
                                                 const T* __restrict__ vy, const T* __restrict__ p,
                                                 const T* __restrict__ ec, const T* __restrict__ en,
                                                 const T* __restrict__ fx, const T* __restrict__ fy,
                                                 T* __restrict__ rx, T* __restrict__ ry, T* __restrict__ rp) {
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    if (i > nx || j > ny) return;
    const CellRes<T> r = cell_residual<T, T>(nx, ny, ld, idx, idy, vx, vy, p, ec, en, fx, fy, i, j);
    const int64_t k = (int64_t)j * ld + i;
    if (j < ny) rx[k] = r.ux ? r.rx : T(0);
    if (i < nx) ry[k] = r.uy ? r.ry : T(0);
    if (rp && r.uc) rp[k] = r.rp;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Three partial sums per workgroup -> part[3*blk + c].
template <typename T>
__global__ __launch_bounds__(NT) void k_energy_partials(int nx, int ny, int64_t ld, double idx, double idy, double sp,
                                                        const T* __restrict__ vx, const T* __restrict__ vy,
                                                        const T* __restrict__ p, const T* __restrict__ ec,
                                                        const T* __restrict__ en, const T* __restrict__ fx,
                                                        const T* __restrict__ fy, double* __restrict__ part) {
    const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y;
    double nv = 0.0, np = 0.0, nf = 0.0;
    if (i <= nx && j <= ny) {
        const CellRes<double> r = cell_residual<T, double>(nx, ny, ld, idx, idy, vx, vy, p, ec, en, fx, fy, i, j);
        const int64_t k = (int64_t)j * ld + i;
        if (r.ux) {
            const double f = fx[k];
            nv += r.rx * r.rx / r.dx_;
            nf += f * f / r.dx_;
        }
        if (r.uy) {
            const double f = fy[k];
            nv += r.ry * r.ry / r.dy_;
            nf += f * f / r.dy_;
        }
        if (r.uc) np += r.rp * r.rp * double(ec[k]) / sp;
    }
    __shared__ double red[3][NT / 64];
    nv = wave_sum(nv);
    np = wave_sum(np);
    nf = wave_sum(nf);
    const int t = threadIdx.y * BX + threadIdx.x, lane = t & 63, w = t >> 6;
    if (lane == 0) {
        red[0][w] = nv;
        red[1][w] = np;
        red[2][w] = nf;
    }
    __syncthreads();
    if (t < 3) {
        double s = 0.0;
        for (int q = 0; q < NT / 64; ++q) s += red[t][q];
        part[3 * ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) + t] = s;
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

inline dim3 cell_grid(const stk_grid* g) {
    return dim3((unsigned)((g->nx + 1 + BX - 1) / BX), (unsigned)((g->ny + 1 + BY - 1) / BY));
}

}  // namespace

int launch_residual(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const void* vx, const void* vy, const void* p,
                    const void* eta_c, const void* eta_n, const void* fx, const void* fy, void* rx, void* ry,
                    void* rp) {
    const dim3 grid = cell_grid(g), block(BX, BY);
    if (dt == STK_F64)
        hipLaunchKernelGGL(k_residual<double>, grid, block, 0, ctx->stream, g->nx, g->ny, g->ld, 1.0 / g->dx,
                           1.0 / g->dy, (const double*)vx, (const double*)vy, (const double*)p, (const double*)eta_c,
                           (const double*)eta_n, (const double*)fx, (const double*)fy, (double*)rx, (double*)ry,
                           (double*)rp);
    else
        hipLaunchKernelGGL(k_residual<float>, grid, block, 0, ctx->stream, g->nx, g->ny, g->ld, float(1.0 / g->dx),
                           float(1.0 / g->dy), (const float*)vx, (const float*)vy, (const float*)p,
                           (const float*)eta_c, (const float*)eta_n, (const float*)fx, (const float*)fy, (float*)rx,
                           (float*)ry, (float*)rp);
    STK_HIP(hipGetLastError());
    return STK_OK;
}

int launch_energy(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const void* vx, const void* vy, const void* p,
                  const void* eta_c, const void* eta_n, const void* fx, const void* fy, double* dst) {
    const dim3 grid = cell_grid(g), block(BX, BY);
    const int64_t nb = (int64_t)grid.x * grid.y;
    void* part = nullptr;
    STK_TRY(scratch(ctx, stk_ctx::S_PART, sizeof(double) * 3 * (size_t)nb, &part));
    const double idx = 1.0 / g->dx, idy = 1.0 / g->dy, sp = 2.0 * idx * idx + 2.0 * idy * idy;
    if (dt == STK_F64)
        hipLaunchKernelGGL(k_energy_partials<double>, grid, block, 0, ctx->stream, g->nx, g->ny, g->ld, idx, idy, sp,
                           (const double*)vx, (const double*)vy, (const double*)p, (const double*)eta_c,
                           (const double*)eta_n, (const double*)fx, (const double*)fy, (double*)part);
    else
        hipLaunchKernelGGL(k_energy_partials<float>, grid, block, 0, ctx->stream, g->nx, g->ny, g->ld, idx, idy, sp,
                           (const float*)vx, (const float*)vy, (const float*)p, (const float*)eta_c,
                           (const float*)eta_n, (const float*)fx, (const float*)fy, (double*)part);
    hipLaunchKernelGGL(k_reduce_triples, dim3(1), dim3(1024), 0, ctx->stream, (const double*)part, nb, dst);
    STK_HIP(hipGetLastError());
    return STK_OK;
}

}  // namespace stk
