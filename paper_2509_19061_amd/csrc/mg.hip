// Host side of the geometric multigrid layer: hierarchy construction, the
// batched V-cycle, and the V-cycle-preconditioned flexible CG solves in FP64
// and in FP32 with FP64 iterative refinement.
//
// The paper solves the velocity block with a matrix-free geometric multigrid
// (Sec. 3.2, Sec. 6.2) and accelerates its fixed-point iteration with
// Anderson acceleration (Sec. 3.3, Alg. 1).  Here the V-cycle is used as the
// preconditioner of flexible conjugate gradients on the SPD system -M v = -b,
// always in FP64 (residual, operator, dot products, energy norms, coarsest
// solve); the mixed-precision mode applies the V-cycle in FP32 between two
// casts.  Coarse levels carry Galerkin operators P^T A P / 4 as stored
// 31-point stencils (galerkin.hip); the finest level stays matrix-free.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <thread>

#include <sched.h>
#include <vector>

#include "coarse_stencil.hpp"
#include "mg_host.hpp"
#include "rowstream.hpp"

namespace {
constexpr int RAS_TILE = 64;  // tile of the finest-level RAS smoothing (the paper's 64 x 64)
}

using namespace stk;

namespace stk {

static int dalloc(stk_mg* m, size_t bytes, void** out) {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return set_error(STK_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    m->mem.push_back(p);
    m->bytes += bytes;
    STK_HIP(hipMemsetAsync(p, 0, bytes, m->ctx->stream));
    *out = p;
    return STK_OK;
}
static int pdalloc(PlanT* P, size_t bytes, void** out, hipStream_t s) {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return set_error(STK_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    P->mem.push_back(p);
    STK_HIP(hipMemsetAsync(p, 0, bytes, s));
    *out = p;
    return STK_OK;
}
template <typename V>
static int upload(PlanT* P, const std::vector<V>& h, const void** out, hipStream_t s) {
    void* d = nullptr;
    STK_TRY(pdalloc(P, std::max<size_t>(1, h.size()) * sizeof(V), &d, s));
    if (!h.empty()) {  // the host copy stays alive until the plan's final synchronisation
        const auto* b = reinterpret_cast<const unsigned char*>(h.data());
        P->stage.emplace_back(b, b + h.size() * sizeof(V));
        STK_HIP(hipMemcpyAsync(d, P->stage.back().data(), P->stage.back().size(), hipMemcpyHostToDevice, s));
    }
    *out = d;
    return STK_OK;
}

static size_t level_field_bytes(const MgLevel& l, int t) { return (size_t)(l.ny + 1) * l.ld * (t ? 4 : 8); }
static int blocks_of(int nx, int ny) { return ((nx + 1 + 63) / 64) * ((ny + 1 + 3) / 4); }

// ---- host operator for the coarsest level (same discretisation as the device stencil)
struct HostGrid {
    int nx, ny;
    int64_t ld;
    double idx, idy;
    const double *ec, *en;
    double enh(int i, int j) const { return (i >= 1 && i <= nx - 1 && j >= 1 && j <= ny - 1) ? en[(int64_t)j * ld + i] : 0.0; }
};
// (-M v) at every unknown, v given as vx, vy on the level layout
static void host_apply_neg(const HostGrid& g, const std::vector<double>& vx, const std::vector<double>& vy,
                    std::vector<double>& ax, std::vector<double>& ay) {
    auto VX = [&](int i, int j) { return (i >= 1 && i <= g.nx - 1 && j >= 0 && j < g.ny) ? vx[(int64_t)j * g.ld + i] : 0.0; };
    auto VY = [&](int i, int j) { return (j >= 1 && j <= g.ny - 1 && i >= 0 && i < g.nx) ? vy[(int64_t)j * g.ld + i] : 0.0; };
    auto EC = [&](int i, int j) { return g.ec[(int64_t)j * g.ld + i]; };
    auto txy = [&](int i, int j) {
        const double e = g.enh(i, j);
        return e == 0.0 ? 0.0 : e * ((VX(i, j) - VX(i, j - 1)) * g.idy + (VY(i, j) - VY(i - 1, j)) * g.idx);
    };
    for (int j = 0; j <= g.ny; ++j)
        for (int i = 0; i <= g.nx; ++i) {
            const int64_t k = (int64_t)j * g.ld + i;
            if (i >= 1 && i <= g.nx - 1 && j < g.ny) {
                const double txr = 2.0 * EC(i, j) * (VX(i + 1, j) - VX(i, j)) * g.idx;
                const double txl = 2.0 * EC(i - 1, j) * (VX(i, j) - VX(i - 1, j)) * g.idx;
                ax[k] = -((txr - txl) * g.idx + (txy(i, j + 1) - txy(i, j)) * g.idy);
            }
            if (j >= 1 && j <= g.ny - 1 && i < g.nx) {
                const double tyt = 2.0 * EC(i, j) * (VY(i, j + 1) - VY(i, j)) * g.idy;
                const double tyb = 2.0 * EC(i, j - 1) * (VY(i, j) - VY(i, j - 1)) * g.idy;
                ay[k] = -((tyt - tyb) * g.idy + (txy(i + 1, j) - txy(i, j)) * g.idx);
            }
        }
}

// f(i) for i in [lo, hi) on up to hardware_concurrency host threads, in
// contiguous chunks (each f(i) independent of the others).
// Host threads for setup work: the CPUs this process may run on, at most
// OMP_NUM_THREADS when that is set (a machine's core count can far exceed a
// job's share of it, and oversubscribed threads also stall the caller's own).
static int host_threads() {
    static const int nt = [] {
        int c = (int)std::thread::hardware_concurrency();
        cpu_set_t set;
        if (sched_getaffinity(0, sizeof(set), &set) == 0) c = std::min(c, (int)CPU_COUNT(&set));
        if (const char* e = std::getenv("OMP_NUM_THREADS")) {
            const int v = std::atoi(e);
            if (v > 0) c = std::min(c, v);
        }
        return std::max(1, c);
    }();
    return nt;
}

// f(i) for i in [lo, hi) on up to host_threads() threads, in contiguous
// chunks (each f(i) independent of the others).
template <typename F>
static void par_for(int lo, int hi, const F& f) {
    const int n = hi - lo;
    const int nt = std::max(1, std::min(n / 16, host_threads()));
    if (nt <= 1) {
        for (int i = lo; i < hi; ++i) f(i);
        return;
    }
    std::vector<std::thread> th;
    int t = 0;
    try {  // a thread that cannot be started leaves its chunk (and the rest) to this one
        for (; t < nt; ++t) {
            const int a = lo + (int)((int64_t)n * t / nt), b = lo + (int)((int64_t)n * (t + 1) / nt);
            th.emplace_back([&f, a, b] {
                for (int i = a; i < b; ++i) f(i);
            });
        }
    } catch (...) {
        for (int i = lo + (int)((int64_t)n * t / nt); i < hi; ++i) f(i);
    }
    for (auto& x : th) x.join();
}

// Assemble A = -M on the coarsest level, invert it (Cholesky, A SPD) and
// upload the inverse column-major, so that the threads of the coarse solve
// (one per row) read consecutive addresses.  The coarsest level is the finest one (viscous stencil from the
// viscosities) when the grid is too small to coarsen, else a Galerkin level.
static int build_coarse(stk_mg* m) {
    MgLevel& l = m->L.back();
    const size_t cnt = (size_t)(l.ny + 1) * l.ld;
    const bool stored = l.st64 != nullptr;
    std::vector<double> ec, en, stc;
    if (stored) {
        stc.resize(cnt * NPLANES);
        STK_HIP(hipMemcpyAsync(stc.data(), l.st64, stc.size() * 8, hipMemcpyDeviceToHost, m->ctx->stream));
    } else {
        ec.resize(cnt);
        en.resize(cnt);
        STK_HIP(hipMemcpyAsync(ec.data(), l.ec64, cnt * 8, hipMemcpyDeviceToHost, m->ctx->stream));
        STK_HIP(hipMemcpyAsync(en.data(), l.en64, cnt * 8, hipMemcpyDeviceToHost, m->ctx->stream));
    }
    STK_HIP(hipStreamSynchronize(m->ctx->stream));
    // unknowns numbered by grid row, then column, vx before vy: every coupling
    // then reaches at most two grid rows, so A is banded (about 4 (nx + 1)
    // wide) and its Cholesky factor stays inside A's envelope
    std::vector<int> map;
    for (int j = 0; j < l.ny; ++j)
        for (int i = 0; i <= l.nx; ++i) {
            if (i >= 1 && i <= l.nx - 1) map.push_back((int)((int64_t)j * l.ld + i));
            if (j >= 1 && i < l.nx) map.push_back((1 << 30) | (int)((int64_t)j * l.ld + i));
        }
    const int n = (int)map.size();
    if (n > 4096)
        return set_error(STK_EUNSUPPORTED, "coarsest level %dx%d has %d unknowns (> 4096): choose sizes divisible by powers of 2",
                         l.nx, l.ny, n);
    std::vector<double> A((size_t)n * n);
    if (stored) {
        // row (a, i, j) from its full stencil (gathered from the stored half); neighbour -> column via pos
        std::vector<int> pos(cnt * 2, -1);
        for (int q = 0; q < n; ++q) pos[(size_t)(map[q] >> 30) * cnt + (map[q] & 0x3fffffff)] = q;
        for (int r = 0; r < n; ++r) {
            const int a = map[r] >> 30, off = map[r] & 0x3fffffff;
            const int i = (int)(off % l.ld), j = (int)(off / l.ld);
            for (int s2 = 0; s2 < NCOEF; ++s2) {
                const double v = stencil_coef<double>(stc.data(), (int64_t)cnt, l.ld, l.nx, l.ny, a, s2, i, j);
                const int b = slot_comp(a, s2), pi = i + slot_dx(a, s2), pj = j + slot_dy(a, s2);
                if (pi < 0 || pj < 0 || pi > l.nx || pj > l.ny) continue;
                const int c = pos[(size_t)b * cnt + (size_t)pj * l.ld + pi];
                if (c >= 0) A[(size_t)r * n + c] = v;
            }
        }
    }
    HostGrid g{l.nx, l.ny, l.ld, 1.0 / l.dx, 1.0 / l.dy, ec.data(), en.data()};
    std::vector<double> ex(stored ? 0 : cnt), ey(stored ? 0 : cnt), ax(stored ? 0 : cnt), ay(stored ? 0 : cnt);
    for (int c = 0; c < (stored ? 0 : n); ++c) {
        std::fill(ex.begin(), ex.end(), 0.0);
        std::fill(ey.begin(), ey.end(), 0.0);
        const int off = map[c] & 0x3fffffff;
        ((map[c] >> 30) ? ey : ex)[off] = 1.0;
        std::fill(ax.begin(), ax.end(), 0.0);
        std::fill(ay.begin(), ay.end(), 0.0);
        host_apply_neg(g, ex, ey, ax, ay);
        for (int r = 0; r < n; ++r) {
            const int o2 = map[r] & 0x3fffffff;
            A[(size_t)r * n + c] = (map[r] >> 30) ? ay[o2] : ax[o2];
        }
    }
    // Envelope of A: first[i] = the first column of row i that is not 0.  The
    // Cholesky factor has the same envelope, so every sum below starts there;
    // the terms it skips are exact zeros.
    std::vector<int> first(n), last(n);
    for (int i = 0; i < n; ++i) {
        int f = i;
        for (int k = 0; k < i; ++k)
            if (A[(size_t)i * n + k] != 0.0) {
                f = k;
                break;
            }
        first[i] = f;
    }
    // last[i] = the last row whose envelope reaches column i
    for (int i = 0, k = 0; i < n; ++i) {
        last[i] = i;
        for (k = n - 1; k > i; --k)
            if (first[k] <= i) {
                last[i] = k;
                break;
            }
    }
    // Cholesky A = L L^T (lower, in place), in panels of CPB columns: the
    // panel's own rows first, then the rows below it in parallel (each entry
    // the same sum in the same order however the work is split).
    constexpr int CPB = 32;
    bool spd = true;
    auto entry = [&](int i, int j) {
        double s = A[(size_t)i * n + j];
        for (int k = std::max(first[i], first[j]); k < j; ++k) s -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
        return s;
    };
    for (int p0 = 0; p0 < n && spd; p0 += CPB) {
        const int p1 = std::min(p0 + CPB, n);
        for (int i = p0; i < p1 && spd; ++i)
            for (int j = std::max(p0, first[i]); j <= i; ++j) {
                const double s = entry(i, j);
                if (j < i) {
                    A[(size_t)i * n + j] = s / A[(size_t)j * n + j];
                } else if (s > 0.0) {
                    A[(size_t)i * n + i] = std::sqrt(s);
                } else {
                    spd = false;
                    break;
                }
            }
        if (spd)
            par_for(p1, n, [&](int i) {
                for (int j = std::max(p0, first[i]); j < p1; ++j) A[(size_t)i * n + j] = entry(i, j) / A[(size_t)j * n + j];
            });
    }
    if (!spd) return set_error(STK_EINVAL, "coarsest operator not positive definite (check viscosities)");
    // inverse: solve L L^T X = I column by column (columns in parallel).  Row c
    // of the forward solve is the first nonzero (the rows above it stay 0, and
    // the terms with them are exact zeros).  The inverse is symmetric, so
    // column c is solved backward only down to row c (its rows below the
    // diagonal need no others) and its upper part is copied from the rows of
    // the columns before it.  The backward solve reads L^T by rows, over the
    // rows whose envelope reaches its column.
    std::vector<double> LT((size_t)n * n);
    par_for(0, n, [&](int i) {
        for (int k = first[i]; k <= i; ++k) LT[(size_t)k * n + i] = A[(size_t)i * n + k];
    });
    std::vector<double> inv((size_t)n * n);
    par_for(0, n, [&](int c) {
        double* y = &inv[(size_t)c * n];  // column c of the inverse, contiguous
        // forward, column-oriented: each y_i still takes its terms L_ik y_k in
        // ascending k, but the updates of one step k are independent
        for (int i = c; i < n; ++i) y[i] = (i == c) ? 1.0 : 0.0;
        for (int k = c; k < n; ++k) {
            const double yk = y[k] / A[(size_t)k * n + k];
            y[k] = yk;
            const double* lk = &LT[(size_t)k * n];
            for (int i = k + 1; i <= last[k]; ++i) y[i] -= lk[i] * yk;
        }
        for (int i = n - 1; i >= c; --i) {
            double s = y[i];
            for (int k = i + 1; k <= last[i]; ++k) s -= LT[(size_t)i * n + k] * y[k];
            y[i] = s / A[(size_t)i * n + i];
        }
    });
    par_for(0, n, [&](int c) {
        for (int i = 0; i < c; ++i) inv[(size_t)c * n + i] = inv[(size_t)i * n + c];
    });
    void *dm = nullptr, *di = nullptr;
    STK_TRY(dalloc(m, (size_t)n * sizeof(int), &dm));
    STK_TRY(dalloc(m, (size_t)n * n * sizeof(double), &di));
    STK_HIP(hipMemcpyAsync(dm, map.data(), (size_t)n * sizeof(int), hipMemcpyHostToDevice, m->ctx->stream));
    STK_HIP(hipMemcpyAsync(di, inv.data(), (size_t)n * n * 8, hipMemcpyHostToDevice, m->ctx->stream));
    STK_HIP(hipStreamSynchronize(m->ctx->stream));
    m->cn = n;
    m->cmap = static_cast<int*>(dm);
    m->cainv = static_cast<double*>(di);
    return STK_OK;
}

// FP32 copies of the viscosities and all per-dtype buffers
static __global__ void k_to_f32(const double* __restrict__ a, float* __restrict__ b, size_t n) {
    const size_t q = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (q < n) b[q] = (float)a[q];
}
int ensure_dtype(stk_mg* m, int t) {
    if (m->have[t]) return STK_OK;
    for (size_t l = 0; l < m->L.size(); ++l) {
        MgLevel& L = m->L[l];
        const size_t fb = level_field_bytes(L, t);
        if (t == 1 && l == 0) {
            void *a = nullptr, *b = nullptr;
            STK_TRY(dalloc(m, fb, &a));
            STK_TRY(dalloc(m, fb, &b));
            L.ec32 = static_cast<float*>(a);
            L.en32 = static_cast<float*>(b);
            const size_t cnt = (size_t)(L.ny + 1) * L.ld;
            hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, m->ctx->stream, L.ec64,
                               L.ec32, cnt);
            hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, m->ctx->stream, L.en64,
                               L.en32, cnt);
            STK_HIP(hipGetLastError());
        } else if (t == 1) {
            const size_t cnt = (size_t)L.plane * NPLANES;
            void* a = nullptr;
            STK_TRY(dalloc(m, cnt * 4, &a));
            L.st32 = static_cast<float*>(a);
            hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, m->ctx->stream, L.st64,
                               L.st32, cnt);
            STK_HIP(hipGetLastError());
        }
        Field2* fs[4] = {&L.v[t], &L.w[t], &L.b[t], &L.r[t]};
        for (int q = 0; q < 4; ++q) {
            if (l == 0 && (q == 0 || q == 2)) continue;  // bound to Krylov slots below
            STK_TRY(dalloc(m, fb, &fs[q]->x));
            STK_TRY(dalloc(m, fb, &fs[q]->y));
        }
    }
    const size_t fb0 = level_field_bytes(m->L[0], t);
    for (int sl = 0; sl < VS_N; ++sl) {
        if (t == 1 && sl != VS_R && sl != VS_Z) continue;
        STK_TRY(dalloc(m, fb0, &m->ks[t][sl].x));
        STK_TRY(dalloc(m, fb0, &m->ks[t][sl].y));
    }
    if (t == 0) {
        STK_TRY(dalloc(m, fb0, &m->zero64));
        STK_TRY(dalloc(m, fb0, &m->zero[0].x));
        STK_TRY(dalloc(m, fb0, &m->zero[0].y));
    }
    m->L[0].v[t] = m->ks[t][VS_Z];
    m->L[0].b[t] = m->ks[t][VS_R];
    m->have[t] = true;
    return STK_OK;
}

template <typename T>
static LevelJob<T> level_job(const stk_mg* m, size_t l, int t) {
    const MgLevel& L = m->L[l];
    LevelJob<T> J{};
    J.nx = L.nx;
    J.ny = L.ny;
    J.ld = L.ld;
    J.idx = T(1.0 / L.dx);
    J.idy = T(1.0 / L.dy);
    J.ec = t ? (gptr<const T>)L.ec32 : (gptr<const T>)L.ec64;
    J.en = t ? (gptr<const T>)L.en32 : (gptr<const T>)L.en64;
    J.st = t ? (gptr<const T>)L.st32 : (gptr<const T>)L.st64;
    J.plane = L.plane;
    J.vx = (gptr<T>)L.v[t].x;
    J.vy = (gptr<T>)L.v[t].y;
    J.wx = (gptr<T>)L.w[t].x;
    J.wy = (gptr<T>)L.w[t].y;
    J.bx = (gptr<T>)L.b[t].x;
    J.by = (gptr<T>)L.b[t].y;
    J.rx = (gptr<T>)L.r[t].x;
    J.ry = (gptr<T>)L.r[t].y;
    if (l + 1 < m->L.size()) {
        const MgLevel& C = m->L[l + 1];
        J.cnx = C.nx;
        J.cny = C.ny;
        J.cld = C.ld;
        J.cbx = (gptr<T>)C.b[t].x;
        J.cby = (gptr<T>)C.b[t].y;
        J.cvx = (gptr<T>)C.v[t].x;
        J.cvy = (gptr<T>)C.v[t].y;
        J.cwx = (gptr<T>)C.w[t].x;
        J.cwy = (gptr<T>)C.w[t].y;
        J.cst = t ? (gptr<const T>)C.st32 : (gptr<const T>)C.st64;
        J.cplane = C.plane;
    }
    return J;
}

template <typename T>
static int build_plan(stk_ctx* ctx, stk_mg* const* mgs, int n, int t, PlanT* P, bool z32) {
    hipStream_t s = ctx->stream;
    P->n = n;
    P->vec_z32 = t == 0 && z32;
    int maxl = 0;
    for (int q = 0; q < n; ++q) {
        STK_TRY(ensure_dtype(mgs[q], 0));  // the FP64 Krylov slots exist in both modes
        STK_TRY(ensure_dtype(mgs[q], t));
        if (P->vec_z32) STK_TRY(ensure_dtype(mgs[q], 1));  // the FP32 Z slot
        maxl = std::max(maxl, (int)mgs[q]->L.size());
        P->maxcn = std::max(P->maxcn, mgs[q]->cn);
    }
    P->depth = maxl - 1;
    P->fine.assign(maxl, Batch{});
    P->crs.assign(maxl, Batch{});
    P->cjobs.assign(maxl, nullptr);
    P->ncj.assign(maxl, 0);
    P->fine_t.assign(maxl, Batch{});
    P->relax.assign(maxl, Batch{});
    P->relax_t.assign(maxl, Batch{});
    const stk_mg_opts& o0 = mgs[0]->o;
    const bool cras = o0.coarse_smoother == 1;
    // Does the restriction into level l (>= 1) also take its first smoothing
    // sweep?  When it is smoothed by Jacobi from zero with at least one sweep
    // before its residual, or is a relaxed last level; not the solved
    // coarsest level, not with coarse RAS.  The V-cycle skips that sweep under
    // the same conditions (first_sweep_done).
    auto first_sweep = [&](const stk_mg* m, int l) {
        if (cras) return 0;
        if (l < (int)m->L.size() - 1) return level_sweeps(m->o.nu1, m->o.sweep_growth, l) >= 1 ? 1 : 0;
        return m->relaxed ? 1 : 0;
    };
    for (int d = 0; d < maxl; ++d) {
        std::vector<LevelJob<T>> jobs, rj;
        std::vector<int> pf{0}, pc{0}, pr{0}, pt{0}, rpf{0}, rpt{0};
        std::vector<CoarseJob<T>> cj;
        for (int q = 0; q < n; ++q) {
            const stk_mg* m = mgs[q];
            const int nl = (int)m->L.size();
            if (d < nl - 1) {
                jobs.push_back(level_job<T>(m, d, t));
                jobs.back().first = first_sweep(m, d + 1);
                pf.push_back(pf.back() + blocks_of(m->L[d].nx, m->L[d].ny));
                pr.push_back(pr.back() + rows::workgroups(m->L[d].nx, m->L[d].ny));
                pc.push_back(pc.back() + blocks_of(m->L[d + 1].nx, m->L[d + 1].ny));
                pt.push_back(pt.back() + mg_ras_tiles(m->L[d].nx, m->L[d].ny, o0.coarse_tile));
            } else if (d == nl - 1 && m->relaxed) {  // relaxed, not solved
                rj.push_back(level_job<T>(m, d, t));
                rpf.push_back(rpf.back() + blocks_of(m->L[d].nx, m->L[d].ny));
                rpt.push_back(rpt.back() + mg_ras_tiles(m->L[d].nx, m->L[d].ny, o0.coarse_tile));
            } else if (d == nl - 1) {
                const MgLevel& L = m->L[d];
                cj.push_back(CoarseJob<T>{m->cn, (gptr<const int>)m->cmap, (gptr<const double>)m->cainv,
                                          (gptr<const T>)L.b[t].x, (gptr<const T>)L.b[t].y,
                                          (gptr<T>)L.v[t].x, (gptr<T>)L.v[t].y});
            }
        }
        if (!rj.empty()) {
            const void *dj = nullptr, *dpf = nullptr, *dpt = nullptr;
            STK_TRY(upload(P, rj, &dj, s));
            STK_TRY(upload(P, rpf, &dpf, s));
            STK_TRY(upload(P, rpt, &dpt, s));
            P->relax[d] = Batch{dj, (const int*)dpf, (int)rj.size(), rpf.back()};
            P->relax_t[d] = Batch{dj, (const int*)dpt, (int)rj.size(), rpt.back()};
        }
        if (!jobs.empty()) {
            const void* dj = nullptr;
            const void *dpf = nullptr, *dpc = nullptr;
            STK_TRY(upload(P, jobs, &dj, s));
            STK_TRY(upload(P, pf, &dpf, s));
            STK_TRY(upload(P, pc, &dpc, s));
            P->fine[d] = Batch{dj, (const int*)dpf, (int)jobs.size(), pf.back()};
            P->crs[d] = Batch{dj, (const int*)dpc, (int)jobs.size(), pc.back()};
            if (d >= 1 && cras) {
                const void* dpt = nullptr;
                STK_TRY(upload(P, pt, &dpt, s));
                P->fine_t[d] = Batch{dj, (const int*)dpt, (int)jobs.size(), pt.back()};
            }
            if (d == 0) {  // the finest level is matrix-free: row-streaming smoothing and residual
                const void* dpr = nullptr;
                STK_TRY(upload(P, pr, &dpr, s));
                P->fine[d].rpre = (const int*)dpr;
                P->fine[d].rblocks = pr.back();
                // RAS smoothing v -> w -> v, and the level jobs with v and w exchanged
                std::vector<RasJob<T>> vw, wv;
                std::vector<LevelJob<T>> sw;
                for (const LevelJob<T>& J : jobs) {
                    const int ntx = (J.nx + RAS_TILE - 1) / RAS_TILE;
                    vw.push_back(RasJob<T>{J.ec, J.en, J.bx, J.by, J.ld, J.nx, J.ny, J.idx, J.idy, J.vx, J.vy, J.wx,
                                           J.wy, ntx});
                    wv.push_back(RasJob<T>{J.ec, J.en, J.bx, J.by, J.ld, J.nx, J.ny, J.idx, J.idy, J.wx, J.wy, J.vx,
                                           J.vy, ntx});
                    LevelJob<T> X = J;
                    std::swap(X.vx, X.wx);
                    std::swap(X.vy, X.wy);
                    sw.push_back(X);
                    P->l0nx.push_back(J.nx);
                    P->l0ny.push_back(J.ny);
                    P->l0ld.push_back(J.ld);
                }
                STK_TRY(upload(P, vw, &P->ras_jobs[0], s));
                STK_TRY(upload(P, wv, &P->ras_jobs[1], s));
                const void* dsw = nullptr;
                STK_TRY(upload(P, sw, &dsw, s));
                P->fine0w = P->fine[d];
                P->fine0w.jobs = dsw;
            }
        }
        if (!cj.empty()) {
            STK_TRY(upload(P, cj, &P->cjobs[d], s));
            P->ncj[d] = (int)cj.size();
        }
    }
    // operator apply on the finest level: Q = 0 - M P
    std::vector<LevelJob<T>> aj;
    std::vector<VecJob> vj;
    std::vector<XCastJob> xj;
    std::vector<int> pa{0}, pra{0};
    for (int q = 0; q < n; ++q) {
        stk_mg* m = mgs[q];
        LevelJob<T> J = level_job<T>(m, 0, t);
        J.vx = (gptr<T>)m->ks[t][VS_P].x;
        J.vy = (gptr<T>)m->ks[t][VS_P].y;
        J.bx = (gptr<T>)m->zero[t].x;
        J.by = (gptr<T>)m->zero[t].y;
        J.rx = (gptr<T>)m->ks[t][VS_Q].x;
        J.ry = (gptr<T>)m->ks[t][VS_Q].y;
        aj.push_back(J);
        pa.push_back(pa.back() + blocks_of(m->L[0].nx, m->L[0].ny));
        pra.push_back(pra.back() + rows::workgroups(m->L[0].nx, m->L[0].ny));
        VecJob V{};
        V.nx = m->L[0].nx;
        V.ny = m->L[0].ny;
        V.ld = m->L[0].ld;
        V.idx = 1.0 / m->L[0].dx;
        V.idy = 1.0 / m->L[0].dy;
        V.ec = (gptr<const double>)m->L[0].ec64;
        V.en = (gptr<const double>)m->L[0].en64;
        for (int sl = 0; sl < VS_N; ++sl) {
            const int ts = sl == VS_Z && P->vec_z32 ? 1 : t;
            V.v[sl][0] = (gptr<void>)m->ks[ts][sl].x;
            V.v[sl][1] = (gptr<void>)m->ks[ts][sl].y;
        }
        vj.push_back(V);
        XCastJob X{};
        X.nx = V.nx;
        X.ny = V.ny;
        X.ld = V.ld;
        for (int c = 0; c < 2; ++c) {
            X.r64[c] = (gptr<const double>)(c ? m->ks[0][VS_R].y : m->ks[0][VS_R].x);
            X.r32[c] = (gptr<float>)(c ? m->ks[1][VS_R].y : m->ks[1][VS_R].x);
            X.z32[c] = (gptr<float>)(c ? m->ks[1][VS_Z].y : m->ks[1][VS_Z].x);
        }
        xj.push_back(X);
    }
    const void *daj = nullptr, *dpa = nullptr, *dvj = nullptr, *dxj = nullptr;
    STK_TRY(upload(P, aj, &daj, s));
    STK_TRY(upload(P, pa, &dpa, s));
    STK_TRY(upload(P, vj, &dvj, s));
    P->apply = Batch{daj, (const int*)dpa, n, pa.back()};
    {  // row-streaming prefix of the operator batch and its reduction chunks
        const void* dpra = nullptr;
        STK_TRY(upload(P, pra, &dpra, s));
        P->apply.rpre = (const int*)dpra;
        P->apply.rblocks = pra.back();
        std::vector<int> cp{0};
        for (int q = 0; q < n; ++q) cp.push_back(cp.back() + (pra[q + 1] - pra[q] + SUM_CHUNK - 1) / SUM_CHUNK);
        const void* dcp = nullptr;
        STK_TRY(upload(P, cp, &dcp, s));
        P->applyr = Batch{nullptr, (const int*)dpra, n, pra.back()};
        P->applyr.cpre = static_cast<const int*>(dcp);
    }
    P->vec = Batch{dvj, (const int*)dpa, n, pa.back()};
    {  // reduction chunks of the vector batch
        std::vector<int> cp{0};
        for (int q = 0; q < n; ++q) cp.push_back(cp.back() + (pa[q + 1] - pa[q] + SUM_CHUNK - 1) / SUM_CHUNK);
        const void* dcp = nullptr;
        STK_TRY(upload(P, cp, &dcp, s));
        P->vec.cpre = static_cast<const int*>(dcp);
    }
    if (t == 1) {  // casts between the FP64 Krylov slots and this plan's FP32 V-cycle slots
        STK_TRY(upload(P, xj, &dxj, s));
        P->xcast = Batch{dxj, (const int*)dpa, n, pa.back()};
    }
    void *st = nullptr, *part = nullptr, *sums = nullptr;
    STK_TRY(pdalloc(P, sizeof(FcgState) * n, &st, s));
    STK_TRY(pdalloc(P, sizeof(double) * 2 * (size_t)pa.back(), &part, s));
    STK_TRY(pdalloc(P, sizeof(double) * 2 * (size_t)n, &sums, s));
    P->st = static_cast<FcgState*>(st);
    P->part = static_cast<double*>(part);
    P->sums = static_cast<double*>(sums);
    STK_HIP(hipStreamSynchronize(s));
    P->stage.clear();
    return STK_OK;
}

int make_plan(stk_ctx* ctx, stk_mg* const* mgs, int n, int t, PlanT** out, bool z32) {
    auto* P = new PlanT();
    const int rc = t ? build_plan<float>(ctx, mgs, n, t, P, false) : build_plan<double>(ctx, mgs, n, t, P, z32);
    if (rc != STK_OK) {
        P->release();
        delete P;
        return rc;
    }
    *out = P;
    return STK_OK;
}

// ---- the batched V-cycle on the level-0 binding (v = Z slot, b = R slot)
// Launch shape of the finest-level RAS smoothing for k sweeps (cached per k).
static const PlanT::RasK* ras_shape(stk_ctx* ctx, const PlanT& P, int kt, int h, stk_dtype dt) {
    for (const PlanT::RasK& r : P.ras_k)
        if (r.kt == kt && r.h == h) return r.ok ? &r : nullptr;
    PlanT::RasK r{kt, h, false, RasShape{}, nullptr};
    std::vector<int> pre, ntx;
    if (!P.l0nx.empty())
        ras_batch_shape(ctx, dt, P.l0nx.data(), P.l0ny.data(), P.l0ld.data(), (int)P.l0nx.size(), RAS_TILE, h, kt,
                        &r.shape, &pre, &ntx, &r.ok);
    if (r.ok) {
        void* d = nullptr;
        if (hipMalloc(&d, pre.size() * sizeof(int)) != hipSuccess) {
            r.ok = false;
        } else {
            P.mem.push_back(d);
            if (hipMemcpyAsync(d, pre.data(), pre.size() * sizeof(int), hipMemcpyHostToDevice, ctx->stream) !=
                    hipSuccess ||
                hipStreamSynchronize(ctx->stream) != hipSuccess)
                r.ok = false;
            r.pre = static_cast<const int*>(d);
        }
    }
    P.ras_k.push_back(r);
    return r.ok ? &P.ras_k.back() : nullptr;
}

// nu Jacobi sweeps v -> v; first_done: the first one (v -> w) was already
// taken (by the restriction into this level, from its zero iterate, or with
// the prolongation before the post-smoothing).
template <typename T>
static int smooth_stage(stk_ctx* ctx, const Batch& F, const stk_mg_opts& o, int nu, bool first_done = false) {
    for (int q = first_done ? 1 : 0; q < nu; ++q) STK_TRY(mg_jacobi<T>(ctx, F, o.omega, q & 1));
    if (nu & 1) STK_TRY(mg_copy_wv<T>(ctx, F));
    return STK_OK;
}

// The restriction into a coarse level took its first sweep (see first_sweep
// in build_plan): the pre-smoothing of a level d >= 1 smoothed by Jacobi with
// nu1 >= 1, or the relaxation of a relaxed last level.
static bool first_sweep_done(const stk_mg_opts& o, int nu) { return o.coarse_smoother != 1 && nu >= 1; }

// nu sweeps of a coarse level's smoother, v -> v: Jacobi, or (the mixed
// smoother) RAS outer iterations of min(coarse_k, sweeps left) sweeps.
template <typename T>
static int coarse_stage(stk_ctx* ctx, const Batch& F, const Batch& Ft, const stk_mg_opts& o, int nu,
                        bool first_done = false) {
    if (o.coarse_smoother != 1) return smooth_stage<T>(ctx, F, o, nu, first_done);
    int left = nu, q = 0;
    for (; left > 0; ++q) {
        const int kt = std::min(o.coarse_k, left);
        STK_TRY(mg_ras<T>(ctx, Ft, o.coarse_tile, o.coarse_halo, kt, o.omega, q & 1));
        left -= kt;
    }
    if (q & 1) STK_TRY(mg_copy_wv<T>(ctx, F));
    return STK_OK;
}

// The finest level's smoothing stage of nu sweeps as RAS outer iterations of
// min(k, sweeps left) sweeps each (k = fine_k, or nu), overlap fine_halo (or
// the iteration's sweep count: Jacobi exactly).  from_w: the iterate starts
// in w (post-smoothing) and must end in v; else starts in v and ends in w.
// Returns false (nothing launched) when a launch shape does not fit.
template <typename T>
static int fine_ras_stage(stk_ctx* ctx, const PlanT& P, const stk_mg_opts& o, int nu, bool from_w, bool* done) {
    const stk_dtype dt = sizeof(T) == 8 ? STK_F64 : STK_F32;
    *done = false;
    const int k = o.fine_k > 0 ? std::min(o.fine_k, nu) : nu;
    std::vector<const PlanT::RasK*> sh;
    for (int left = nu; left > 0; left -= std::min(k, left)) {
        const int kt = std::min(k, left);
        const PlanT::RasK* r = ras_shape(ctx, P, kt, o.fine_halo < 0 ? kt : o.fine_halo, dt);
        if (!r) return STK_OK;
        sh.push_back(r);
    }
    for (size_t q = 0; q < sh.size(); ++q) {
        const int jb = (q & 1) ^ (from_w ? 1 : 0);  // 0: v -> w, 1: w -> v
        STK_TRY(ras_batch_launch(ctx, dt, sh[q]->shape, P.ras_jobs[jb], sh[q]->pre, P.fine0w.n, o.omega));
    }
    // an even count ends where it started: move the iterate to its side
    if (!(sh.size() & 1)) STK_TRY(mg_copy_wv<T>(ctx, from_w ? P.fine[0] : P.fine0w));
    *done = true;
    return STK_OK;
}

template <typename T>
static int vcycle(stk_ctx* ctx, const PlanT& P, const stk_mg_opts& o) {
    // Finest level: pre-smoothing v -> w and post-smoothing w -> v as RAS outer
    // iterations (the iterate is in w in between), when the streaming kernel
    // takes the instances; else Jacobi sweeps (exactly the same values when
    // the overlap is the default).
    const bool paper_fine = o.fine_halo >= 0 || o.fine_k > 0;  // a smoother other than Jacobi
    bool ras0 = P.ras_jobs[0] && o.nu1 >= 1 && o.nu2 >= 1;
    if (ras0) {  // both stages must fit, checked before anything is launched
        const stk_dtype dt = sizeof(T) == 8 ? STK_F64 : STK_F32;
        for (int nu : {o.nu1, o.nu2}) {
            const int k = o.fine_k > 0 ? std::min(o.fine_k, nu) : nu;
            for (int left = nu; left > 0 && ras0; left -= std::min(k, left)) {
                const int kt = std::min(k, left);
                ras0 = ras_shape(ctx, P, kt, o.fine_halo < 0 ? kt : o.fine_halo, dt) != nullptr;
            }
        }
    }
    if (paper_fine && !ras0 && P.fine[0].n)
        return set_error(STK_EUNSUPPORTED, "the finest-level RAS smoother does not fit these instances");
    STK_TRY(mg_coarse<T>(ctx, P.cjobs[0], P.ncj[0], P.maxcn));
    for (int d = 0; d < P.depth; ++d) {
        const Batch& F = P.fine[d];
        if (!F.n) break;
        const int nu1 = level_sweeps(o.nu1, o.sweep_growth, d);
        if (d == 0 && ras0) {
            bool done = false;
            STK_TRY(fine_ras_stage<T>(ctx, P, o, nu1, false, &done));
            STK_TRY(mg_residual<T>(ctx, P.fine0w));
        } else {
            STK_TRY(d == 0 ? smooth_stage<T>(ctx, F, o, nu1)
                           : coarse_stage<T>(ctx, F, P.fine_t[d], o, nu1, first_sweep_done(o, nu1)));
            STK_TRY(mg_residual<T>(ctx, F));
        }
        STK_TRY(mg_restrict<T>(ctx, P.crs[d], o.omega));
        if (d + 1 < (int)P.cjobs.size()) {
            STK_TRY(mg_coarse<T>(ctx, P.cjobs[d + 1], P.ncj[d + 1], P.maxcn));
            if (P.relax[d + 1].n) {  // truncated hierarchies: the last level relaxed from 0
                const int nr = level_sweeps(o.nu1, o.sweep_growth, d + 1) + level_sweeps(o.nu2, o.sweep_growth, d + 1);
                STK_TRY(coarse_stage<T>(ctx, P.relax[d + 1], P.relax_t[d + 1], o, nr, first_sweep_done(o, nr)));
            }
        }
    }
    for (int d = P.depth - 1; d >= 0; --d) {
        const Batch& F = P.fine[d];
        if (!F.n) continue;
        const int nu2 = level_sweeps(o.nu2, o.sweep_growth, d);
        if (d == 0 && ras0) {
            STK_TRY(mg_prolong<T>(ctx, P.fine0w));
            bool done = false;
            STK_TRY(fine_ras_stage<T>(ctx, P, o, nu2, true, &done));
        } else if (d >= 1 && o.coarse_smoother != 1 && nu2 >= 1) {
            // the prolongation and the first post-sweep in one pass (v + P e -> w)
            STK_TRY(mg_jacobi_prolonged<T>(ctx, F, o.omega));
            STK_TRY(smooth_stage<T>(ctx, F, o, nu2, true));
        } else {
            STK_TRY(mg_prolong<T>(ctx, F));
            STK_TRY(d == 0 ? smooth_stage<T>(ctx, F, o, nu2) : coarse_stage<T>(ctx, F, P.fine_t[d], o, nu2));
        }
    }
    return STK_OK;
}

int run_vcycle(stk_ctx* ctx, const PlanT& P, const stk_mg_opts& o, int t) {
    return t ? vcycle<float>(ctx, P, o) : vcycle<double>(ctx, P, o);
}

int read_states(stk_ctx* ctx, const PlanT& P, std::vector<FcgState>& h) {
    h.resize(P.n);
    STK_HIP(hipMemcpyAsync(h.data(), P.st, sizeof(FcgState) * P.n, hipMemcpyDeviceToHost, ctx->stream));
    STK_HIP(hipStreamSynchronize(ctx->stream));
    return STK_OK;
}
int write_states(stk_ctx* ctx, const PlanT& P, const std::vector<FcgState>& h) {
    STK_HIP(hipMemcpyAsync(P.st, h.data(), sizeof(FcgState) * P.n, hipMemcpyHostToDevice, ctx->stream));
    return STK_OK;
}

void free_plan(PlanT*& P) {
    if (!P) return;
    P->release();
    delete P;
    P = nullptr;
}

int copy_vel_in(stk_mg* m, const void* sx, const void* sy, int64_t sld, void* dx, void* dy, int64_t dld, size_t es) {
    const MgLevel& L = m->L[0];
    STK_HIP(hipMemcpy2DAsync(dx, dld * es, sx, sld * es, (size_t)(L.nx + 1) * es, L.ny, hipMemcpyDeviceToDevice,
                             m->ctx->stream));
    STK_HIP(hipMemcpy2DAsync(dy, dld * es, sy, sld * es, (size_t)L.nx * es, L.ny + 1, hipMemcpyDeviceToDevice,
                             m->ctx->stream));
    return STK_OK;
}

int level_sweeps(int nu, double growth, int l) {
    const double v = std::floor((double)nu * std::pow(growth, (double)l) + 0.5);
    return v > 1e5 ? 100000 : (int)v;
}

bool same_smoothing(const stk_mg_opts& a, const stk_mg_opts& b) {
    return a.nu1 == b.nu1 && a.nu2 == b.nu2 && a.omega == b.omega && a.fine_k == b.fine_k &&
           a.fine_halo == b.fine_halo && a.coarse_smoother == b.coarse_smoother && a.coarse_tile == b.coarse_tile &&
           a.coarse_k == b.coarse_k && a.coarse_halo == b.coarse_halo && a.sweep_growth == b.sweep_growth;
}

}  // namespace stk

// ============================================================== C ABI ====
extern "C" {

void stk_mg_opts_default(stk_mg_opts* o) {
    if (!o) return;
    o->nu1 = 2;
    o->nu2 = 2;
    o->omega = 0.7;
    o->coarsest = 8;
    o->fine_k = 0;
    o->fine_halo = -1;
    o->coarse_smoother = 0;
    o->coarse_tile = 32;
    o->coarse_k = 4;
    o->coarse_halo = 0;
    o->sweep_growth = 1.0;
    o->max_levels = 0;
    o->stall_checks = 0;
}

static int check_mg_opts(const stk_mg_opts& o) {
    if (o.nu1 < 0 || o.nu2 < 0 || o.nu1 + o.nu2 < 1 || o.nu1 > 64 || o.nu2 > 64)
        return set_error(STK_EINVAL, "nu1, nu2 must be in [0, 64] with nu1 + nu2 >= 1");
    if (!(o.omega > 0.0 && o.omega < 2.0)) return set_error(STK_EINVAL, "omega must be in (0, 2)");
    if (o.coarsest < 2) return set_error(STK_EINVAL, "coarsest must be >= 2");
    if (o.fine_k < 0 || o.fine_k > 16) return set_error(STK_EINVAL, "fine_k must be in [0, 16]");
    if ((o.fine_k > 0 || o.fine_halo >= 0) && std::max(o.nu1, o.nu2) > 16 && o.fine_k == 0)
        return set_error(STK_EINVAL, "a finest-level RAS stage takes at most 16 sweeps per outer iteration");
    if (o.fine_halo < -1 || o.fine_halo > 15) return set_error(STK_EINVAL, "fine_halo must be in [-1, 15]");
    if (o.coarse_smoother != 0 && o.coarse_smoother != 1) return set_error(STK_EINVAL, "coarse_smoother must be 0 or 1");
    if (o.coarse_tile < 1 || o.coarse_k < 1 || o.coarse_halo < 0)
        return set_error(STK_EINVAL, "coarse_tile, coarse_k must be >= 1 and coarse_halo >= 0");
    if (!(o.sweep_growth >= 1.0 && o.sweep_growth <= 16.0))
        return set_error(STK_EINVAL, "sweep_growth must be in [1, 16]");
    if (o.max_levels < 0 || o.max_levels == 1) return set_error(STK_EINVAL, "max_levels must be 0 or >= 2");
    if (o.stall_checks < 0) return set_error(STK_EINVAL, "stall_checks must be >= 0");
    return STK_OK;
}

int stk_mg_footprint(const stk_grid* g, const stk_mg_opts* opts, int mode, size_t* bytes) {
    STK_TRY(check_grid(g));
    if (!bytes) return set_error(STK_EINVAL, "bytes is NULL");
    stk_mg_opts o;
    stk_mg_opts_default(&o);
    if (opts) o = *opts;
    STK_TRY(check_mg_opts(o));
    if (mode != STK_SOLVE_F64 && mode != STK_SOLVE_F32_REFINED) return set_error(STK_EINVAL, "unknown mode");
    size_t b = 0;
    int nx = g->nx, ny = g->ny, lvl = 0;
    const bool f32 = mode == STK_SOLVE_F32_REFINED;
    while (true) {
        const size_t cnt = (size_t)(ny + 1) * (lvl == 0 ? (size_t)g->ld : (size_t)pad_ld(nx));
        // fields of cnt words: finest = eta_c, eta_n, smoother partner w and residual r (2 components each),
        // 7 two-component Krylov slots, 3 zero fields; FP32 extra: eta, w, r, R, Z.
        // coarse = NPLANES stencil planes and v, w, b, r; FP32 extra: the same again.
        const size_t w64 = lvl == 0 ? 2 + 4 + 2 * VS_N + 3 : NPLANES + 8;
        const size_t w32 = lvl == 0 ? 2 + 4 + 4 : NPLANES + 8;
        b += cnt * (w64 * 8 + (f32 ? w32 * 4 : 0));
        if (std::min(nx, ny) <= o.coarsest || (nx & 1) || (ny & 1)) break;
        if (o.max_levels > 0 && lvl + 1 == o.max_levels) {  // truncated: relaxed, no dense inverse
            *bytes = b;
            return STK_OK;
        }
        nx /= 2;
        ny /= 2;
        ++lvl;
    }
    const size_t n = (size_t)(nx - 1) * ny + (size_t)nx * (ny - 1);
    b += n * n * 8 + n * 4;
    *bytes = b;
    return STK_OK;
}

int stk_mg_create(stk_ctx* ctx, stk_mg** out, const stk_grid* g, const double* eta_c, const double* eta_n,
                  const stk_mg_opts* opts) {
    if (!ctx || !out) return set_error(STK_EINVAL, "ctx/out is NULL");
    STK_TRY(check_grid(g));
    if (!eta_c || !eta_n) return set_error(STK_EINVAL, "eta_c, eta_n must be non-NULL");
    stk_mg_opts o;
    stk_mg_opts_default(&o);
    if (opts) o = *opts;
    STK_TRY(check_mg_opts(o));
    STK_TRY(use_device(ctx));
    auto* m = new stk_mg();
    m->ctx = ctx;
    m->o = o;
    m->user_ld = g->ld;
    auto fail = [&](int rc) {
        stk_mg_destroy(m);
        return rc;
    };
    int nx = g->nx, ny = g->ny;
    double dx = g->dx, dy = g->dy;
    while (true) {
        MgLevel L;
        L.nx = nx;
        L.ny = ny;
        L.ld = m->L.empty() ? g->ld : pad_ld(nx);
        L.dx = dx;
        L.dy = dy;
        m->L.push_back(L);
        if (std::min(nx, ny) <= o.coarsest || (nx & 1) || (ny & 1)) break;
        if (o.max_levels > 0 && (int)m->L.size() == o.max_levels) {  // cut here: relax the last level
            m->relaxed = true;
            break;
        }
        nx /= 2;
        ny /= 2;
        dx *= 2;
        dy *= 2;
    }
    for (size_t l = 0; l < m->L.size(); ++l) {
        MgLevel& L = m->L[l];
        L.plane = (int64_t)(L.ny + 1) * L.ld;
        if (l == 0) {
            void *a = nullptr, *b = nullptr;
            int rc = dalloc(m, level_field_bytes(L, 0), &a);
            if (rc == STK_OK) rc = dalloc(m, level_field_bytes(L, 0), &b);
            if (rc != STK_OK) return fail(rc);
            L.ec64 = static_cast<double*>(a);
            L.en64 = static_cast<double*>(b);
            hipError_t e1 = hipMemcpy2DAsync(L.ec64, L.ld * 8, eta_c, g->ld * 8, (size_t)g->nx * 8,
                                             g->ny, hipMemcpyDeviceToDevice, ctx->stream);
            hipError_t e2 = hipMemcpy2DAsync(L.en64, L.ld * 8, eta_n, g->ld * 8, (size_t)(g->nx + 1) * 8, g->ny + 1,
                                             hipMemcpyDeviceToDevice, ctx->stream);
            if (e1 != hipSuccess || e2 != hipSuccess) return fail(hip_fail(e1 != hipSuccess ? e1 : e2, "hipMemcpy2DAsync"));
        } else {
            void* a = nullptr;
            int rc = dalloc(m, (size_t)L.plane * NPLANES * 8, &a);
            if (rc != STK_OK) return fail(rc);
            L.st64 = static_cast<double*>(a);
            const MgLevel& F = m->L[l - 1];
            GalerkinArgs ga{F.nx, F.ny, F.ld, 1.0 / F.dx, 1.0 / F.dy, F.ec64, F.en64, F.st64, F.plane,
                            L.nx, L.ny, L.ld, L.st64, L.plane};
            rc = mg_galerkin(ctx, ga);
            if (rc != STK_OK) return fail(rc);
        }
    }
    if (o.coarse_smoother == 1 && mg_ras_lds_bytes(o.coarse_tile, o.coarse_halo, 8) > (size_t)ctx->lds_max)
        return fail(set_error(STK_EUNSUPPORTED, "coarse RAS tile %d with overlap %d exceeds the LDS of a workgroup",
                              o.coarse_tile, o.coarse_halo));
    int rc = m->relaxed ? STK_OK : build_coarse(m);
    if (rc != STK_OK) return fail(rc);
    *out = m;
    return STK_OK;
}

int stk_mg_destroy(stk_mg* m) {
    if (!m) return STK_OK;
    if (m->busy) return set_error(STK_EINVAL, "mg handle is solving in a batch: destroy the batch first");
    (void)hipSetDevice(m->ctx->device);
    (void)hipStreamSynchronize(m->ctx->stream);
    for (int t = 0; t < 2; ++t)
        if (m->plan[t]) {
            m->plan[t]->release();
            delete m->plan[t];
        }
    for (void* p : m->mem) (void)hipFree(p);
    delete m;
    return STK_OK;
}

int stk_mg_bind(stk_mg* m, stk_ctx* ctx, int mode) {
    if (!m || !ctx) return set_error(STK_EINVAL, "mg and ctx must be non-NULL");
    if (m->busy) return set_error(STK_EINVAL, "mg handle is solving in a batch");
    if (ctx->device != m->ctx->device)
        return set_error(STK_EINVAL, "ctx is on device %d, the handle on device %d", ctx->device, m->ctx->device);
    if (mode != STK_SOLVE_F64 && mode != STK_SOLVE_F32_REFINED) return set_error(STK_EINVAL, "unknown mode %d", mode);
    STK_TRY(use_device(m->ctx));
    // the buffers of `mode` are built on the old context's stream, which is drained
    STK_TRY(ensure_dtype(m, 0));
    if (mode == STK_SOLVE_F32_REFINED) STK_TRY(ensure_dtype(m, 1));
    STK_HIP(hipStreamSynchronize(m->ctx->stream));
    m->ctx = ctx;
    return STK_OK;
}

int stk_mg_info(const stk_mg* m, int* levels, int* coarse_unknowns, size_t* bytes) {
    if (!m) return set_error(STK_EINVAL, "mg is NULL");
    if (levels) *levels = (int)m->L.size();
    if (coarse_unknowns) *coarse_unknowns = m->cn;
    if (bytes) *bytes = m->bytes;
    return STK_OK;
}

int stk_mg_vcycle(stk_mg* m, stk_dtype dt, void* vx, void* vy, const void* bx, const void* by) {
    if (!m) return set_error(STK_EINVAL, "mg is NULL");
    if (dt != STK_F64 && dt != STK_F32) return set_error(STK_EINVAL, "unknown dtype");
    if (!vx || !vy || !bx || !by) return set_error(STK_EINVAL, "vx, vy, bx, by must be non-NULL");
    stk_ctx* ctx = m->ctx;
    STK_TRY(use_device(ctx));
    const int t = dt == STK_F32 ? 1 : 0;
    stk_mg* self = m;
    if (!m->plan[t]) STK_TRY(make_plan(ctx, &self, 1, t, &m->plan[t]));
    const size_t es = t ? 4 : 8;
    const int64_t ld0 = m->L[0].ld;
    STK_TRY(copy_vel_in(m, vx, vy, m->user_ld, m->ks[t][VS_Z].x, m->ks[t][VS_Z].y, ld0, es));
    STK_TRY(copy_vel_in(m, bx, by, m->user_ld, m->ks[t][VS_R].x, m->ks[t][VS_R].y, ld0, es));
    STK_TRY(run_vcycle(ctx, *m->plan[t], m->o, t));
    STK_TRY(copy_vel_in(m, m->ks[t][VS_Z].x, m->ks[t][VS_Z].y, ld0, vx, vy, m->user_ld, es));
    return STK_OK;
}

}  // extern "C"
