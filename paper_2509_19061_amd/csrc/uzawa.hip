// Inexact Uzawa iteration for the full Stokes system (Sec. 3.1, 3.2, 6.2).
//
// The pressure Schur complement of M v + G p = f, D v = 0 is never formed:
// a Richardson step on it, preconditioned by the cell viscosity, reads
//   p <- p + omega_p eta_c r_p,   r_p = -D v,
// with v the (approximate) velocity for the current pressure.  With the
// library's fold b = f - G p, (G p) = -grad p, the Schur complement of -M is
// positive and this sign is the convergent one.  The pressure is defined up
// to a constant; its domain mean is removed after every update (Sec. 6.2).
//
// Kernels (all FP64, bound by HBM bandwidth):
//   k_pressure_update  one pass over the cells: p <- p + omega_p eta_c r_p and
//                      a per-workgroup partial sum of the new p (fixed order)
//   k_litho            lithostatic pressure: one lane per column walks down
//                      from the top row, p(j-1) = p(j) + fy(j) dy
//   k_mean             one workgroup sums the partials in a fixed order
//   k_sub_mean         p <- p - mean
//   k_min_partial, k_min_final, k_rescale
//                      viscosity continuation (Sec. 6.2): eta_min over the
//                      cells, then (1 - theta) eta_min + theta eta on the cell
//                      and nodal fields of each stage's hierarchy
// The reductions never use atomics: results are bitwise reproducible.
#include <chrono>
#include <cmath>
#include <functional>

#include "mg_host.hpp"
#include "stk_internal.hpp"

namespace stk {
namespace {

constexpr int UX = 64;    // cells per workgroup row (one wave)
constexpr int UY = 4;     // waves per workgroup
constexpr int UROWS = 8;  // rows each lane walks

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Sum of one value per lane of a UX x UY workgroup, in a fixed order.
__device__ __forceinline__ double group_sum(double v) {
    __shared__ double red[UY];
    v = wave_sum64(v);
    if (threadIdx.x == 0) red[threadIdx.y] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0 && threadIdx.y == 0)
        for (int w = 0; w < UY; ++w) s += red[w];
    return s;
}

__global__ __launch_bounds__(UX* UY) void k_pressure_update(int nx, int ny, int64_t ld, double idx, double idy,
                                                            double omega_p, const double* __restrict__ vx,
                                                            const double* __restrict__ vy,
                                                            const double* __restrict__ ec, double* __restrict__ p,
                                                            double* __restrict__ part) {
    const int i = (int)blockIdx.x * UX + (int)threadIdx.x;
    const int j0 = ((int)blockIdx.y * UY + (int)threadIdx.y) * UROWS;
    double s = 0.0;
    if (i < nx && j0 < ny) {
        // the wall velocities vx(0, .), vx(nx, .), vy(., 0), vy(., ny) are read as 0
        const int j1 = min(j0 + UROWS, ny);
        const bool lw = i == 0, rw = i + 1 == nx;
        double below = j0 == 0 ? 0.0 : vy[(int64_t)j0 * ld + i];
        for (int j = j0; j < j1; ++j) {
            const int64_t c = (int64_t)j * ld + i;
            const double above = j + 1 == ny ? 0.0 : vy[c + ld];
            const double xl = lw ? 0.0 : vx[c], xr = rw ? 0.0 : vx[c + 1];
            const double div = (xr - xl) * idx + (above - below) * idy;
            const double q = p[c] - omega_p * ec[c] * div;  // + omega_p eta_c r_p, r_p = -D v
            p[c] = q;
            s += q;
            below = above;
        }
    }
    s = group_sum(s);
    if (threadIdx.x == 0 && threadIdx.y == 0) part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
}

__global__ __launch_bounds__(UX) void k_litho(int nx, int ny, int64_t ld, double dy, const double* __restrict__ fy,
                                              double* __restrict__ p, double* __restrict__ part) {
    const int i = (int)blockIdx.x * UX + (int)threadIdx.x;
    double s = 0.0;
    if (i < nx) {
        double q = 0.0;  // top row; the constant is removed afterwards
        p[(int64_t)(ny - 1) * ld + i] = q;
        for (int j = ny - 1; j >= 1; --j) {
            q = q + fy[(int64_t)j * ld + i] * dy;
            p[(int64_t)(j - 1) * ld + i] = q;
            s += q;
        }
    }
    s = wave_sum64(s);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(1024) void k_mean(const double* __restrict__ part, int64_t n, double inv_cells,
                                               double* __restrict__ mean) {
    __shared__ double red[1024 / 64];
    double s = 0.0;
    for (int64_t q = threadIdx.x; q < n; q += 1024) s += part[q];
    s = wave_sum64(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < 1024 / 64; ++w) t += red[w];
        *mean = t * inv_cells;
    }
}

__global__ __launch_bounds__(UX* UY) void k_sub_mean(int nx, int ny, int64_t ld, const double* __restrict__ mean,
                                                     double* __restrict__ p) {
    const int i = (int)blockIdx.x * UX + (int)threadIdx.x;
    const int j0 = ((int)blockIdx.y * UY + (int)threadIdx.y) * UROWS;
    if (i >= nx || j0 >= ny) return;
    const double m = *mean;
    const int j1 = min(j0 + UROWS, ny);
    for (int j = j0; j < j1; ++j) p[(int64_t)j * ld + i] -= m;
}

__device__ __forceinline__ double wave_min64(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_down(v, o, 64));
    return v;
}

// Per-workgroup minimum of eta_c over the cells (same tiling as the pressure step).
__global__ __launch_bounds__(UX* UY) void k_min_partial(int nx, int ny, int64_t ld, const double* __restrict__ ec,
                                                        double* __restrict__ part) {
    __shared__ double red[UY];
    const int i = (int)blockIdx.x * UX + (int)threadIdx.x;
    const int j0 = ((int)blockIdx.y * UY + (int)threadIdx.y) * UROWS;
    double m = INFINITY;
    if (i < nx && j0 < ny) {
        const int j1 = min(j0 + UROWS, ny);
        for (int j = j0; j < j1; ++j) m = fmin(m, ec[(int64_t)j * ld + i]);
    }
    m = wave_min64(m);
    if (threadIdx.x == 0) red[threadIdx.y] = m;
    __syncthreads();
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        for (int w = 1; w < UY; ++w) m = fmin(m, red[w]);
        part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = m;
    }
}

__global__ __launch_bounds__(1024) void k_min_final(const double* __restrict__ part, int64_t n,
                                                    double* __restrict__ out) {
    __shared__ double red[1024 / 64];
    double m = INFINITY;
    for (int64_t q = threadIdx.x; q < n; q += 1024) m = fmin(m, part[q]);
    m = wave_min64(m);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 1024 / 64; ++w) m = fmin(m, red[w]);
        *out = m;
    }
}

// Computational viscosity of the continuation, (1 - theta) eta_min + theta eta,
// on the cell and the nodal fields; every element of the (ny + 1) x ld arrays
// is written (0 outside the fields).  Products and sum rounded separately.
__global__ __launch_bounds__(256) void k_rescale(int nx, int ny, int64_t ld, double theta,
                                                 const double* __restrict__ emin, const double* __restrict__ ec,
                                                 const double* __restrict__ en, double* __restrict__ oc,
                                                 double* __restrict__ on) {
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= (int64_t)(ny + 1) * ld) return;
    const int j = (int)(q / ld), i = (int)(q - (int64_t)j * ld);
    const double a = __dmul_rn(1.0 - theta, *emin);
    oc[q] = (j < ny && i < nx) ? __dadd_rn(a, __dmul_rn(theta, ec[q])) : 0.0;
    on[q] = (i <= nx) ? __dadd_rn(a, __dmul_rn(theta, en[q])) : 0.0;
}

// v += (double) z32 on the unknowns; the walls vx(0, .), vx(nx, .), vy(., 0),
// vy(., ny) are written 0
__global__ __launch_bounds__(256) void k_add_z(int nx, int ny, int64_t ld, const float* __restrict__ z32x,
                                               const float* __restrict__ z32y, double* __restrict__ vx,
                                               double* __restrict__ vy) {
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= (int64_t)(ny + 1) * ld) return;
    const int j = (int)(q / ld), i = (int)(q - (int64_t)j * ld);
    if (j < ny && i <= nx) vx[q] = (i == 0 || i == nx) ? 0.0 : vx[q] + (double)z32x[q];
    if (i < nx) vy[q] = (j == 0 || j == ny) ? 0.0 : vy[q] + (double)z32y[q];
}

dim3 cell_grid_u(const stk_grid* g) {
    return dim3((unsigned)((g->nx + UX - 1) / UX), (unsigned)((g->ny + UY * UROWS - 1) / (UY * UROWS)));
}

// mean of p over the cells from `nblk` partials in `part`, then p -= mean;
// the mean lands in part[nblk].
int remove_mean(stk_ctx* ctx, const stk_grid* g, double* part, int64_t nblk, double* p) {
    hipLaunchKernelGGL(k_mean, dim3(1), dim3(1024), 0, ctx->stream, (const double*)part, nblk,
                       1.0 / ((double)g->nx * (double)g->ny), part + nblk);
    hipLaunchKernelGGL(k_sub_mean, cell_grid_u(g), dim3(UX, UY), 0, ctx->stream, g->nx, g->ny, g->ld,
                       (const double*)(part + nblk), p);
    STK_HIP(hipGetLastError());
    return STK_OK;
}

int pressure_update(stk_ctx* ctx, const stk_grid* g, const double* vx, const double* vy, const double* eta_c,
                    double omega_p, double* p) {
    const dim3 grid = cell_grid_u(g);
    const int64_t nblk = (int64_t)grid.x * grid.y;
    void* part = nullptr;
    STK_TRY(scratch(ctx, stk_ctx::S_PART, sizeof(double) * (size_t)(nblk + 1), &part));
    hipLaunchKernelGGL(k_pressure_update, grid, dim3(UX, UY), 0, ctx->stream, g->nx, g->ny, g->ld, 1.0 / g->dx,
                       1.0 / g->dy, omega_p, vx, vy, eta_c, p, (double*)part);
    STK_HIP(hipGetLastError());
    return remove_mean(ctx, g, (double*)part, nblk, p);
}

int check_omega_p(double w) {
    if (!(w > 0.0) || !std::isfinite(w)) return set_error(STK_EINVAL, "omega_p must be finite and > 0 (got %g)", w);
    return STK_OK;
}

// Device buffer owned for the duration of a call.
struct DevBuf {
    void* p = nullptr;
    int alloc(size_t bytes) {
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            return set_error(STK_ENOMEM, "cannot allocate %zu bytes", bytes);
        }
        return STK_OK;
    }
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

// Uzawa cycles with hierarchy `mm` and the stage's viscosities (ec_step,
// en_step), from the caller's (vx, vy, p); E (true system: eta_c, eta_n)
// after every cycle lands in out / hist[k].  The last stage runs while
// E > tol, earlier ones `stage_cycles` cycles; k counts all cycles against
// max_cycles.  The hierarchy's level 0 has the caller's row stride, so the
// FP64 cycles run in its own level-0 vectors (the V-cycle's iterate and
// right-hand side): the velocity is copied in and out once per stage instead
// of staging v and b through stk_mg_vcycle every cycle.
int uzawa_stage(stk_mg* mm, const stk_grid* g, double* vx, double* vy, double* p, const double* ec_step,
                const double* en_step, const double* eta_c, const double* eta_n, const double* fx, const double* fy,
                const stk_uzawa_opts& o, bool last, int& k, double* out, double* hist) {
    stk_ctx* ctx = mm->ctx;
    stk_mg* self = mm;
    if (!mm->plan[0]) STK_TRY(make_plan(ctx, &self, 1, 0, &mm->plan[0]));
    if (o.mode == STK_SOLVE_F32_REFINED) {
        // v += V32(0, (float)(f - G p - M v)) per V-cycle; the V-cycle is
        // consistent, so in exact arithmetic this is the FP64 cycle
        int n = 0;
        while (k < o.max_cycles && (last ? out[3] > o.tol : n < o.stage_cycles)) {
            for (int c = 0; c < o.vcycles; ++c)
                STK_TRY(mixed_correction(mm, g, vx, vy, p, ec_step, en_step, fx, fy));
            STK_TRY(pressure_update(ctx, g, vx, vy, ec_step, o.omega_p, p));
            ++k;
            ++n;
            STK_TRY(stk_energy_norm(ctx, STK_F64, g, vx, vy, p, eta_c, eta_n, fx, fy, out));
            if (hist) hist[k] = out[3];
        }
        return STK_OK;
    }
    double* wx = static_cast<double*>(mm->ks[0][VS_Z].x);
    double* wy = static_cast<double*>(mm->ks[0][VS_Z].y);
    double* bx = static_cast<double*>(mm->ks[0][VS_R].x);
    double* by = static_cast<double*>(mm->ks[0][VS_R].y);
    STK_TRY(copy_vel_in(mm, vx, vy, g->ld, wx, wy, g->ld, sizeof(double)));
    int n = 0;
    while (k < o.max_cycles && (last ? out[3] > o.tol : n < o.stage_cycles)) {
        STK_TRY(launch_fold_rhs(ctx, STK_F64, g, fx, fy, p, bx, by));  // b = f - G p
        for (int c = 0; c < o.vcycles; ++c) STK_TRY(run_vcycle(ctx, *mm->plan[0], mm->o, 0));
        STK_TRY(pressure_update(ctx, g, wx, wy, ec_step, o.omega_p, p));
        ++k;
        ++n;
        STK_TRY(stk_energy_norm(ctx, STK_F64, g, wx, wy, p, eta_c, eta_n, fx, fy, out));
        if (hist) hist[k] = out[3];
    }
    STK_TRY(copy_vel_in(mm, wx, wy, g->ld, vx, vy, g->ld, sizeof(double)));
    STK_HIP(hipStreamSynchronize(ctx->stream));
    return STK_OK;
}

}  // namespace

int mixed_correction(stk_mg* m, const stk_grid* g, double* vx, double* vy, const double* p, const double* ec,
                     const double* en, const double* fx, const double* fy) {
    stk_ctx* ctx = m->ctx;
    stk_mg* self = m;
    if (!m->plan[1]) STK_TRY(make_plan(ctx, &self, 1, 1, &m->plan[1]));
    float* z32x = static_cast<float*>(m->ks[1][VS_Z].x);
    float* z32y = static_cast<float*>(m->ks[1][VS_Z].y);
    const int64_t cnt = (int64_t)(g->ny + 1) * g->ld;
    const dim3 eg((unsigned)((cnt + 255) / 256)), eb(256);
    // r32 = (float)(f - G p - M v) and z32 = 0 in one pass
    STK_TRY(launch_residual_to32(ctx, g, vx, vy, p, ec, en, fx, fy, static_cast<float*>(m->ks[1][VS_R].x),
                                 static_cast<float*>(m->ks[1][VS_R].y), z32x, z32y));
    STK_TRY(run_vcycle(ctx, *m->plan[1], m->o, 1));
    hipLaunchKernelGGL(k_add_z, eg, eb, 0, ctx->stream, g->nx, g->ny, g->ld, (const float*)z32x, (const float*)z32y,
                       vx, vy);
    STK_HIP(hipGetLastError());
    return STK_OK;
}

int continuation(stk_mg* m, const stk_grid* g, const double* eta_c, const double* eta_n, const stk_uzawa_opts& o,
                 const int& k, const std::function<int(stk_mg*, const double*, const double*, bool)>& stage) {
    if (o.stages == 0) return stage(m, eta_c, eta_n, true);
    stk_ctx* ctx = m->ctx;
    const size_t fb = field_bytes(g, g->ny + 1, STK_F64);
    DevBuf ecs, ens, tmp;
    STK_TRY(ecs.alloc(fb));
    STK_TRY(ens.alloc(fb));
    STK_TRY(tmp.alloc(sizeof(double)));
    const dim3 grid = cell_grid_u(g);
    const int64_t nblk = (int64_t)grid.x * grid.y;
    void* part = nullptr;
    STK_TRY(scratch(ctx, stk_ctx::S_PART, sizeof(double) * (size_t)nblk, &part));
    hipLaunchKernelGGL(k_min_partial, grid, dim3(UX, UY), 0, ctx->stream, g->nx, g->ny, g->ld, eta_c, (double*)part);
    hipLaunchKernelGGL(k_min_final, dim3(1), dim3(1024), 0, ctx->stream, (const double*)part, nblk, (double*)tmp.p);
    STK_HIP(hipGetLastError());
    const int64_t cnt = (int64_t)(g->ny + 1) * g->ld;
    for (int st = 0; st < o.stages; ++st) {
        if (o.stage_cycles == 0 || k >= o.max_cycles) break;  // nothing would run on this stage's hierarchy
        const double theta = (double)st / (double)o.stages;
        hipLaunchKernelGGL(k_rescale, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, ctx->stream, g->nx, g->ny,
                           g->ld, theta, (const double*)tmp.p, eta_c, eta_n, (double*)ecs.p, (double*)ens.p);
        STK_HIP(hipGetLastError());
        stk_mg* ms = nullptr;
        STK_TRY(stk_mg_create(ctx, &ms, g, (const double*)ecs.p, (const double*)ens.p, &m->o));
        const int rc = stage(ms, (const double*)ecs.p, (const double*)ens.p, false);
        (void)stk_mg_destroy(ms);
        if (rc != STK_OK) return rc;
    }
    return stage(m, eta_c, eta_n, true);  // theta = 1: the true system and the caller's hierarchy
}

}  // namespace stk

using namespace stk;

extern "C" {

void stk_uzawa_opts_default(stk_uzawa_opts* o) {
    if (!o) return;
    o->omega_p = 0.6;
    o->vcycles = 1;
    o->tol = 1e-8;
    o->max_cycles = 1000;
    o->stages = 0;
    o->stage_cycles = 25;
    o->mode = STK_SOLVE_F64;
}

int stk_litho_pressure(stk_ctx* ctx, const stk_grid* g, const double* fy, double* p) {
    if (!ctx) return set_error(STK_EINVAL, "ctx is NULL");
    STK_TRY(check_grid(g));
    if (!fy || !p) return set_error(STK_EINVAL, "fy, p must be non-NULL");
    STK_TRY(use_device(ctx));
    const int64_t nblk = (g->nx + UX - 1) / UX;
    void* part = nullptr;
    STK_TRY(scratch(ctx, stk_ctx::S_PART, sizeof(double) * (size_t)(nblk + 1), &part));
    hipLaunchKernelGGL(k_litho, dim3((unsigned)nblk), dim3(UX), 0, ctx->stream, g->nx, g->ny, g->ld, g->dy, fy, p,
                       (double*)part);
    STK_HIP(hipGetLastError());
    return remove_mean(ctx, g, (double*)part, nblk, p);
}

int stk_uzawa_pressure(stk_ctx* ctx, const stk_grid* g, const double* vx, const double* vy, const double* eta_c,
                       double omega_p, double* p) {
    if (!ctx) return set_error(STK_EINVAL, "ctx is NULL");
    STK_TRY(check_grid(g));
    STK_TRY(check_omega_p(omega_p));
    if (!vx || !vy || !eta_c || !p) return set_error(STK_EINVAL, "vx, vy, eta_c, p must be non-NULL");
    STK_TRY(use_device(ctx));
    return pressure_update(ctx, g, vx, vy, eta_c, omega_p, p);
}

int stk_uzawa_solve(stk_mg* m, const stk_grid* g, double* vx, double* vy, double* p, const double* eta_c,
                    const double* eta_n, const double* fx, const double* fy, const stk_uzawa_opts* opts,
                    double* hist, stk_uzawa_report* rep) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!m) return set_error(STK_EINVAL, "mg is NULL");
    STK_TRY(check_grid(g));
    if (g->nx != m->L[0].nx || g->ny != m->L[0].ny || g->ld != m->user_ld)
        return set_error(STK_EINVAL, "grid (%d x %d, ld %lld) is not the handle's (%d x %d, ld %lld)", g->nx, g->ny,
                         (long long)g->ld, m->L[0].nx, m->L[0].ny, (long long)m->user_ld);
    if (!vx || !vy || !p || !eta_c || !eta_n || !fx || !fy)
        return set_error(STK_EINVAL, "vx, vy, p, eta_c, eta_n, fx, fy must be non-NULL");
    if (m->busy) return set_error(STK_EINVAL, "the handle is in a batch");
    stk_uzawa_opts o;
    stk_uzawa_opts_default(&o);
    if (opts) o = *opts;
    STK_TRY(check_omega_p(o.omega_p));
    if (o.vcycles < 1) return set_error(STK_EINVAL, "vcycles must be >= 1 (got %d)", o.vcycles);
    if (o.max_cycles < 0) return set_error(STK_EINVAL, "max_cycles must be >= 0 (got %d)", o.max_cycles);
    if (!(o.tol >= 0.0)) return set_error(STK_EINVAL, "tol must be >= 0");
    if (o.stages < 0 || o.stage_cycles < 0)
        return set_error(STK_EINVAL, "stages and stage_cycles must be >= 0 (got %d, %d)", o.stages, o.stage_cycles);
    if (o.mode != STK_SOLVE_F64 && o.mode != STK_SOLVE_F32_REFINED)
        return set_error(STK_EINVAL, "unknown mode %d", o.mode);
    stk_ctx* ctx = m->ctx;
    STK_TRY(use_device(ctx));
    double out[5];
    int rc = stk_energy_norm(ctx, STK_F64, g, vx, vy, p, eta_c, eta_n, fx, fy, out);
    if (rc != STK_OK) return rc;
    if (hist) hist[0] = out[3];
    int k = 0;
    STK_TRY(continuation(m, g, eta_c, eta_n, o, k, [&](stk_mg* mm, const double* ec, const double* en, bool last) {
        return uzawa_stage(mm, g, vx, vy, p, ec, en, eta_c, eta_n, fx, fy, o, last, k, out, hist);
    }));
    const bool conv = out[3] <= o.tol;
    if (rep) {
        rep->cycles = k;
        rep->converged = conv ? 1 : 0;
        rep->e = out[3];
        rep->ev = out[4];
        rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (!conv) return set_error(STK_ENOTCONV, "Uzawa: E = %g > tol = %g after %d cycles", out[3], o.tol, k);
    return STK_OK;
}

}  // extern "C"
