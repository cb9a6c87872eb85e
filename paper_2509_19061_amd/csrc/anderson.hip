// Anderson acceleration of the inexact Uzawa map (Sec. 3.3, Alg. 1).
//
// The fixed-point map F is one Uzawa cycle (fold, V-cycles, pressure step) on
// x = [v, p].  With r_i = F(x_i) - x_i, each step forms the combination of the
// last m_k + 1 values F(x_i) whose weights (summing to 1) minimise the l2 norm
// of the same combination of residuals.  The weights come from the Gram matrix
// H_ij = r_i . r_j, kept on the host: only the new residual's products are
// computed per step, in one fused pass.  The small bordered system of the
// constrained least squares is solved on the host.
//
// A vector is three planes of (ny + 1) x ld doubles (vx, vy, p in the grid's
// layout); only the used extents take part (vx: ny x (nx+1), vy: (ny+1) x nx,
// p: ny x nx).
//
// Kernels (FP64, bound by HBM bandwidth):
//   k_aa_diff_dots  r = F - x, and the products of r with the window's
//                 residuals (itself included), per-workgroup partials;
//                 k_aa_dots_final sums them in a fixed order (one workgroup
//                 per product)
//   k_aa_combine  x = sum_t a_t F_t (products and sums rounded separately, in
//                 the order t = 0, 1, ..)
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "mg_host.hpp"
#include "stk_internal.hpp"

namespace stk {
namespace {

constexpr int AA_MAX = 9;  // window of at most 9 residuals: depth m <= 8
constexpr int AT = 256;

struct Planes {
    const double* v[AA_MAX][3];
    double a[AA_MAX];
    int n;
};

// Used extents (ex, ey, ep) of the three planes at element q, and the
// unknowns among them (ux, uy: the walls vx(0, .), vx(nx, .), vy(., 0),
// vy(., ny) are not unknowns; every cell is a pressure unknown).
__device__ __forceinline__ void masks(int64_t q, int64_t ld, int nx, int ny, bool& ex, bool& ey, bool& ep, bool& ux,
                                      bool& uy) {
    const int j = (int)(q / ld), i = (int)(q - (int64_t)j * ld);
    ex = j < ny && i <= nx;
    ey = j <= ny && i < nx;
    ep = j < ny && i < nx;
    ux = ex && i >= 1 && i <= nx - 1;
    uy = ey && j >= 1 && j <= ny - 1;
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// r = F - x written to the new residual's planes (0 outside the used
// extents), and part[t * nblk + block] = sum over the block's elements of
// r . r_t for the window's older residuals t < n - 1 and r . r for t = n - 1
// (the window's newest entry is r itself and is not read back).
__global__ __launch_bounds__(AT) void k_aa_diff_dots(int nx, int ny, int64_t ld, const double* __restrict__ fx,
                                                     const double* __restrict__ fy, const double* __restrict__ fp,
                                                     const double* __restrict__ xx, const double* __restrict__ xy,
                                                     const double* __restrict__ xp, double* __restrict__ rx,
                                                     double* __restrict__ ry, double* __restrict__ rp, Planes o,
                                                     double* __restrict__ part) {
    __shared__ double red[AA_MAX][AT / 64];
    const int64_t q = (int64_t)blockIdx.x * AT + threadIdx.x;
    const int64_t cnt = (int64_t)(ny + 1) * ld;
    double a = 0.0, b = 0.0, c = 0.0;
    if (q < cnt) {
        bool ex, ey, ep, ux, uy;
        masks(q, ld, nx, ny, ex, ey, ep, ux, uy);
        a = ux ? fx[q] - xx[q] : 0.0;  // wall values of F and x take no part
        b = uy ? fy[q] - xy[q] : 0.0;
        c = ep ? fp[q] - xp[q] : 0.0;
        rx[q] = a;
        ry[q] = b;
        rp[q] = c;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int t = 0; t < o.n; ++t) {
        double s = 0.0;
        if (q < cnt) s = t == o.n - 1 ? a * a + b * b + c * c : a * o.v[t][0][q] + b * o.v[t][1][q] + c * o.v[t][2][q];
        s = wsum(s);
        if (lane == 0) red[t][w] = s;
    }
    __syncthreads();
    if ((int)threadIdx.x < o.n) {
        double s = 0.0;
        for (int k = 0; k < AT / 64; ++k) s += red[threadIdx.x][k];
        part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(1024) void k_aa_dots_final(const double* __restrict__ part, int64_t nblk,
                                                        double* __restrict__ dots) {
    __shared__ double red[1024 / 64];
    const double* p = part + (int64_t)blockIdx.x * nblk;
    double s = 0.0;
    for (int64_t q = threadIdx.x; q < nblk; q += 1024) s += p[q];
    s = wsum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < 1024 / 64; ++k) t += red[k];
        dots[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(AT) void k_aa_combine(int nx, int ny, int64_t ld, Planes f, double* __restrict__ ox,
                                                   double* __restrict__ oy, double* __restrict__ op) {
    const int64_t q = (int64_t)blockIdx.x * AT + threadIdx.x;
    if (q >= (int64_t)(ny + 1) * ld) return;
    bool ex, ey, ep, ux, uy;
    masks(q, ld, nx, ny, ex, ey, ep, ux, uy);
    const bool e3[3] = {ex, ey, ep}, u3[3] = {ux, uy, ep};
    double* o3[3] = {ox, oy, op};
    for (int c = 0; c < 3; ++c) {
        if (!e3[c]) continue;  // only the used extents are written: the unknowns, and 0 on the walls
        double s = 0.0;
        if (u3[c])
            for (int t = 0; t < f.n; ++t) s = __dadd_rn(s, __dmul_rn(f.a[t], f.v[t][c][q]));
        o3[c][q] = s;
    }
}

// alpha = argmin ||R alpha|| with sum(alpha) = 1 from the bordered system
// [H/s 1; 1^T 0] [alpha; mu] = [0; 1], s = max diag(H), by Gaussian
// elimination with partial pivoting; a singular system gives the plain step.
std::vector<double> aa_weights(const std::vector<double>& H, int n) {
    std::vector<double> plain(n, 0.0);
    plain[n - 1] = 1.0;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s = std::fmax(s, H[i * n + i]);
    if (!(s > 0.0) || !std::isfinite(s)) return plain;
    const int N = n + 1;
    std::vector<double> K(N * N, 0.0), b(N, 0.0);
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) K[i * N + j] = H[i * n + j] / s;
        K[i * N + n] = 1.0;
        K[n * N + i] = 1.0;
    }
    b[n] = 1.0;
    for (int c = 0; c < N; ++c) {
        int piv = c;
        for (int r = c + 1; r < N; ++r)
            if (std::fabs(K[r * N + c]) > std::fabs(K[piv * N + c])) piv = r;
        if (K[piv * N + c] == 0.0) return plain;
        if (piv != c) {
            for (int j = 0; j < N; ++j) std::swap(K[c * N + j], K[piv * N + j]);
            std::swap(b[c], b[piv]);
        }
        for (int r = c + 1; r < N; ++r) {
            const double f = K[r * N + c] / K[c * N + c];
            for (int j = c; j < N; ++j) K[r * N + j] -= f * K[c * N + j];
            b[r] -= f * b[c];
        }
    }
    std::vector<double> x(N);
    for (int r = N - 1; r >= 0; --r) {
        double t = b[r];
        for (int j = r + 1; j < N; ++j) t -= K[r * N + j] * x[j];
        x[r] = t / K[r * N + r];
    }
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(x[i])) return plain;
    return std::vector<double>(x.begin(), x.begin() + n);
}

struct Dev {
    void* p = nullptr;
    int alloc(size_t bytes) {
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            return set_error(STK_ENOMEM, "cannot allocate %zu bytes", bytes);
        }
        return STK_OK;
    }
    ~Dev() {
        if (p) (void)hipFree(p);
    }
};

}  // namespace
}  // namespace stk

using namespace stk;

extern "C" {

int stk_uzawa_anderson(stk_mg* m, const stk_grid* g, double* vx, double* vy, double* p, const double* eta_c,
                       const double* eta_n, const double* fx, const double* fy, int depth,
                       const stk_uzawa_opts* opts, double* hist, stk_uzawa_report* rep) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!m) return set_error(STK_EINVAL, "mg is NULL");
    STK_TRY(check_grid(g));
    if (g->nx != m->L[0].nx || g->ny != m->L[0].ny || g->ld != m->user_ld)
        return set_error(STK_EINVAL, "grid (%d x %d, ld %lld) is not the handle's (%d x %d, ld %lld)", g->nx, g->ny,
                         (long long)g->ld, m->L[0].nx, m->L[0].ny, (long long)m->user_ld);
    if (!vx || !vy || !p || !eta_c || !eta_n || !fx || !fy)
        return set_error(STK_EINVAL, "vx, vy, p, eta_c, eta_n, fx, fy must be non-NULL");
    if (m->busy) return set_error(STK_EINVAL, "the handle is in a batch");
    if (depth < 0 || depth > AA_MAX - 1)
        return set_error(STK_EINVAL, "depth must be in [0, %d] (got %d)", AA_MAX - 1, depth);
    stk_uzawa_opts o;
    stk_uzawa_opts_default(&o);
    if (opts) o = *opts;
    if (!(o.omega_p > 0.0) || !std::isfinite(o.omega_p)) return set_error(STK_EINVAL, "omega_p must be finite and > 0");
    if (o.vcycles < 1) return set_error(STK_EINVAL, "vcycles must be >= 1 (got %d)", o.vcycles);
    if (o.max_cycles < 0) return set_error(STK_EINVAL, "max_cycles must be >= 0 (got %d)", o.max_cycles);
    if (!(o.tol >= 0.0)) return set_error(STK_EINVAL, "tol must be >= 0");
    if (o.stages < 0 || o.stage_cycles < 0)
        return set_error(STK_EINVAL, "stages and stage_cycles must be >= 0 (got %d, %d)", o.stages, o.stage_cycles);
    if (o.mode != STK_SOLVE_F64 && o.mode != STK_SOLVE_F32_REFINED)
        return set_error(STK_EINVAL, "unknown mode %d", o.mode);
    stk_ctx* ctx = m->ctx;
    STK_TRY(use_device(ctx));
    const int W = depth + 1;                          // ring of W slots
    const int64_t plane = (int64_t)(g->ny + 1) * g->ld;
    const size_t pb = (size_t)plane * sizeof(double);
    Dev ring, dots;
    STK_TRY(ring.alloc(pb * 3 * 2 * (size_t)W));      // F and R vectors, 3 planes each
    STK_TRY(dots.alloc(sizeof(double) * AA_MAX));
    double* base = static_cast<double*>(ring.p);
    auto F = [&](int s, int c) { return base + ((int64_t)(2 * s) * 3 + c) * plane; };
    auto R = [&](int s, int c) { return base + ((int64_t)(2 * s + 1) * 3 + c) * plane; };
    const int64_t nblk = (plane + AT - 1) / AT;
    // the products' per-workgroup partials have a buffer of their own: the Uzawa
    // cycles and norms of every step use (and may regrow) the context's scratch
    Dev parts;
    STK_TRY(parts.alloc(sizeof(double) * (size_t)nblk * AA_MAX));
    double* part = static_cast<double*>(parts.p);
    const dim3 eg((unsigned)nblk), eb(AT);
    std::vector<double> H((size_t)W * W, 0.0);       // Gram matrix over ring slots
    double out[5];
    int rc = stk_energy_norm(ctx, STK_F64, g, vx, vy, p, eta_c, eta_n, fx, fy, out);
    if (rc != STK_OK) return rc;
    if (hist) hist[0] = out[3];
    int k = 0;  // F evaluations so far, all stages
    // One stage: Anderson steps on the system of hierarchy mm (viscosities ec,
    // en); the window restarts with the stage, since F changes with it.
    auto stage = [&](stk_mg* mm, const double* ec, const double* en, bool last) -> int {
        stk_mg* self = mm;
        if (!mm->plan[0]) STK_TRY(make_plan(ctx, &self, 1, 0, &mm->plan[0]));
        double* zx = static_cast<double*>(mm->ks[0][VS_Z].x);
        double* zy = static_cast<double*>(mm->ks[0][VS_Z].y);
        double* rx0 = static_cast<double*>(mm->ks[0][VS_R].x);
        double* ry0 = static_cast<double*>(mm->ks[0][VS_R].y);
        int kk = 0;  // index of the current iterate x_kk = (vx, vy, p) within the stage
        while (k < o.max_cycles && (last ? out[3] > o.tol : kk < o.stage_cycles)) {
            const int sk = kk % W;
            // F(x_k) into slot sk: one Uzawa cycle from x_k.  The hierarchy's
            // level 0 has the caller's row stride: the V-cycle runs in its own
            // level-0 vectors (iterate loaded from x_k, right-hand side folded in
            // place).
            const size_t rowb = (size_t)g->ld * sizeof(double);
            STK_HIP(hipMemcpy2DAsync(F(sk, 2), rowb, p, rowb, (size_t)g->nx * sizeof(double), g->ny,
                                     hipMemcpyDeviceToDevice, ctx->stream));
            if (o.mode == STK_SOLVE_F32_REFINED) {
                // FP32 V-cycles on the FP64 residual
                STK_TRY(copy_vel_in(mm, vx, vy, g->ld, F(sk, 0), F(sk, 1), g->ld, sizeof(double)));
                for (int c = 0; c < o.vcycles; ++c)
                    STK_TRY(mixed_correction(mm, g, F(sk, 0), F(sk, 1), p, ec, en, fx, fy));
            } else {
                STK_TRY(copy_vel_in(mm, vx, vy, g->ld, zx, zy, g->ld, sizeof(double)));
                STK_TRY(launch_fold_rhs(ctx, STK_F64, g, fx, fy, p, rx0, ry0));
                for (int c = 0; c < o.vcycles; ++c) STK_TRY(run_vcycle(ctx, *mm->plan[0], mm->o, 0));
                STK_TRY(copy_vel_in(mm, zx, zy, g->ld, F(sk, 0), F(sk, 1), g->ld, sizeof(double)));
            }
            STK_TRY(stk_uzawa_pressure(ctx, g, F(sk, 0), F(sk, 1), ec, o.omega_p, F(sk, 2)));
            // products of r_k with the window r_{k-mk} .. r_k (oldest first) into
            // the Gram matrix over ring slots
            const int mk = std::min(depth, kk);
            Planes D{};
            D.n = mk + 1;
            for (int t = 0; t <= mk; ++t)
                for (int c = 0; c < 3; ++c) D.v[t][c] = R((kk - mk + t) % W, c);
            hipLaunchKernelGGL(k_aa_diff_dots, eg, eb, 0, ctx->stream, g->nx, g->ny, g->ld, F(sk, 0), F(sk, 1),
                               F(sk, 2), vx, vy, p, R(sk, 0), R(sk, 1), R(sk, 2), D, part);
            hipLaunchKernelGGL(k_aa_dots_final, dim3((unsigned)D.n), dim3(1024), 0, ctx->stream, (const double*)part,
                               nblk, (double*)dots.p);
            STK_HIP(hipGetLastError());
            double d[AA_MAX];
            STK_HIP(hipMemcpyAsync(d, dots.p, sizeof(double) * D.n, hipMemcpyDeviceToHost, ctx->stream));
            STK_HIP(hipStreamSynchronize(ctx->stream));
            for (int t = 0; t <= mk; ++t) {
                const int st = (kk - mk + t) % W;
                H[(size_t)sk * W + st] = H[(size_t)st * W + sk] = d[t];
            }
            // x_1 = F(x_0); later x_{k+1} = sum alpha_t F(x_{k-mk+t})
            Planes P{};
            P.n = mk + 1;
            std::vector<double> al(1, 1.0);
            if (kk > 0) {
                std::vector<double> h((size_t)(mk + 1) * (mk + 1));
                for (int a = 0; a <= mk; ++a)
                    for (int b = 0; b <= mk; ++b)
                        h[(size_t)a * (mk + 1) + b] = H[(size_t)((kk - mk + a) % W) * W + (kk - mk + b) % W];
                al = aa_weights(h, mk + 1);
            }
            for (int t = 0; t <= mk; ++t) {
                P.a[t] = al[t];
                for (int c = 0; c < 3; ++c) P.v[t][c] = F((kk - mk + t) % W, c);
            }
            hipLaunchKernelGGL(k_aa_combine, eg, eb, 0, ctx->stream, g->nx, g->ny, g->ld, P, vx, vy, p);
            STK_HIP(hipGetLastError());
            ++k;
            ++kk;
            STK_TRY(stk_energy_norm(ctx, STK_F64, g, vx, vy, p, eta_c, eta_n, fx, fy, out));
            if (hist) hist[k] = out[3];
        }
        return STK_OK;
    };
    STK_TRY(continuation(m, g, eta_c, eta_n, o, k, stage));
    const bool conv = out[3] <= o.tol;
    if (rep) {
        rep->cycles = k;
        rep->converged = conv ? 1 : 0;
        rep->e = out[3];
        rep->ev = out[4];
        rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (!conv) return set_error(STK_ENOTCONV, "Anderson-Uzawa: E = %g > tol = %g after %d steps", out[3], o.tol, k);
    return STK_OK;
}

}  // extern "C"
