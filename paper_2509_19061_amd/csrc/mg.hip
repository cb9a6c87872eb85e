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
#include <cstring>
#include <vector>

#include "coarse_stencil.hpp"
#include "mg_internal.hpp"

namespace stk {
namespace {

struct Field2 {
    void* x = nullptr;
    void* y = nullptr;
};

struct MgLevel {
    int nx = 0, ny = 0;
    int64_t ld = 0;
    double dx = 0, dy = 0;
    double* ec64 = nullptr;  // viscosities (finest level only)
    double* en64 = nullptr;
    float* ec32 = nullptr;
    float* en32 = nullptr;
    double* st64 = nullptr;  // Galerkin stencil, 2 * NCOEF planes (coarse levels only)
    float* st32 = nullptr;
    int64_t plane = 0;
    Field2 v[2], w[2], b[2], r[2];  // [0] FP64, [1] FP32; level 0 binds v, b to the Krylov Z, R slots
};

int64_t pad_ld(int nx) { return ((int64_t)nx + 1 + 63) / 64 * 64; }

}  // namespace
}  // namespace stk

using namespace stk;

struct PlanT {  // one dtype, a fixed list of instances
    int n = 0, depth = 0, maxcn = 0;
    std::vector<Batch> fine, crs;       // per depth: fine-block and coarse-block batches of LevelJob
    std::vector<const void*> cjobs;     // per depth: CoarseJob array of instances whose coarsest it is
    std::vector<int> ncj;
    Batch apply;                        // finest: v = P, b = 0, r = Q  ->  Q = A P
    Batch vec;                          // VecJob array
    Batch xcast;                        // XCastJob array (FP32 plan only)
    FcgState* st = nullptr;
    double* part = nullptr;
    double* sums = nullptr;
    std::vector<void*> mem;
    std::vector<std::vector<unsigned char>> stage;  // host sources of pending uploads
    void release() {
        for (void* p : mem) (void)hipFree(p);
        mem.clear();
    }
};

struct stk_mg {
    stk_ctx* ctx = nullptr;
    stk_mg_opts o{};
    std::vector<MgLevel> L;
    int64_t user_ld = 0;
    int cn = 0;
    int* cmap = nullptr;
    double* cainv = nullptr;
    Field2 ks[2][VS_N];   // finest-level slots: row 0 FP64 (all), row 1 FP32 (R, Z only)
    Field2 zero[2];       // zero right-hand side for the operator apply
    void* zero64 = nullptr;  // FP64 zeros (pressure of a p = 0 fold)
    bool have[2] = {false, false};
    std::vector<void*> mem;
    size_t bytes = 0;
    PlanT* plan[2] = {nullptr, nullptr};  // single-instance plans
};

namespace stk {
namespace {

int dalloc(stk_mg* m, size_t bytes, void** out) {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return set_error(STK_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    m->mem.push_back(p);
    m->bytes += bytes;
    STK_HIP(hipMemsetAsync(p, 0, bytes, m->ctx->stream));
    *out = p;
    return STK_OK;
}
int pdalloc(PlanT* P, size_t bytes, void** out, hipStream_t s) {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return set_error(STK_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    P->mem.push_back(p);
    STK_HIP(hipMemsetAsync(p, 0, bytes, s));
    *out = p;
    return STK_OK;
}
template <typename V>
int upload(PlanT* P, const std::vector<V>& h, const void** out, hipStream_t s) {
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

size_t level_field_bytes(const MgLevel& l, int t) { return (size_t)(l.ny + 1) * l.ld * (t ? 4 : 8); }
int blocks_of(int nx, int ny) { return ((nx + 1 + 63) / 64) * ((ny + 1 + 3) / 4); }

// ---- host operator for the coarsest level (same discretisation as the device stencil)
struct HostGrid {
    int nx, ny;
    int64_t ld;
    double idx, idy;
    const double *ec, *en;
    double enh(int i, int j) const { return (i >= 1 && i <= nx - 1 && j >= 1 && j <= ny - 1) ? en[(int64_t)j * ld + i] : 0.0; }
};
// (-M v) at every unknown, v given as vx, vy on the level layout
void host_apply_neg(const HostGrid& g, const std::vector<double>& vx, const std::vector<double>& vy,
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

// Assemble A = -M on the coarsest level, invert it (Cholesky, A SPD) and
// upload.  The coarsest level is the finest one (viscous stencil from the
// viscosities) when the grid is too small to coarsen, else a Galerkin level.
int build_coarse(stk_mg* m) {
    MgLevel& l = m->L.back();
    const size_t cnt = (size_t)(l.ny + 1) * l.ld;
    const bool stored = l.st64 != nullptr;
    std::vector<double> ec, en, stc;
    if (stored) {
        stc.resize(cnt * 2 * NCOEF);
        STK_HIP(hipMemcpyAsync(stc.data(), l.st64, stc.size() * 8, hipMemcpyDeviceToHost, m->ctx->stream));
    } else {
        ec.resize(cnt);
        en.resize(cnt);
        STK_HIP(hipMemcpyAsync(ec.data(), l.ec64, cnt * 8, hipMemcpyDeviceToHost, m->ctx->stream));
        STK_HIP(hipMemcpyAsync(en.data(), l.en64, cnt * 8, hipMemcpyDeviceToHost, m->ctx->stream));
    }
    STK_HIP(hipStreamSynchronize(m->ctx->stream));
    std::vector<int> map;
    for (int j = 0; j < l.ny; ++j)
        for (int i = 1; i <= l.nx - 1; ++i) map.push_back((int)((int64_t)j * l.ld + i));
    for (int j = 1; j <= l.ny - 1; ++j)
        for (int i = 0; i < l.nx; ++i) map.push_back((1 << 30) | (int)((int64_t)j * l.ld + i));
    const int n = (int)map.size();
    if (n > 4096)
        return set_error(STK_EUNSUPPORTED, "coarsest level %dx%d has %d unknowns (> 4096): choose sizes divisible by powers of 2",
                         l.nx, l.ny, n);
    std::vector<double> A((size_t)n * n);
    if (stored) {
        // row (a, i, j) from its 31 stored coefficients; neighbour -> column via pos
        std::vector<int> pos(cnt * 2, -1);
        for (int q = 0; q < n; ++q) pos[(size_t)(map[q] >> 30) * cnt + (map[q] & 0x3fffffff)] = q;
        for (int r = 0; r < n; ++r) {
            const int a = map[r] >> 30, off = map[r] & 0x3fffffff;
            const int i = (int)(off % l.ld), j = (int)(off / l.ld);
            for (int s2 = 0; s2 < NCOEF; ++s2) {
                const double v = stc[((size_t)a * NCOEF + s2) * cnt + off];
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
    // Cholesky A = L L^T (lower, in place)
    for (int j = 0; j < n; ++j) {
        double d = A[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) d -= A[(size_t)j * n + k] * A[(size_t)j * n + k];
        if (!(d > 0.0)) return set_error(STK_EINVAL, "coarsest operator not positive definite (check viscosities)");
        const double Ljj = std::sqrt(d);
        A[(size_t)j * n + j] = Ljj;
        for (int i = j + 1; i < n; ++i) {
            double s = A[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) s -= A[(size_t)i * n + k] * A[(size_t)j * n + k];
            A[(size_t)i * n + j] = s / Ljj;
        }
    }
    // inverse: solve L L^T X = I column by column
    std::vector<double> inv((size_t)n * n), y(n);
    for (int c = 0; c < n; ++c) {
        for (int i = 0; i < n; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) s -= A[(size_t)i * n + k] * y[k];
            y[i] = s / A[(size_t)i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = y[i];
            for (int k = i + 1; k < n; ++k) s -= A[(size_t)k * n + i] * y[k];
            y[i] = s / A[(size_t)i * n + i];
        }
        for (int i = 0; i < n; ++i) inv[(size_t)i * n + c] = y[i];
    }
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
__global__ void k_to_f32(const double* __restrict__ a, float* __restrict__ b, size_t n) {
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
            const size_t cnt = (size_t)L.plane * 2 * NCOEF;
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
LevelJob<T> level_job(const stk_mg* m, size_t l, int t) {
    const MgLevel& L = m->L[l];
    LevelJob<T> J{};
    J.nx = L.nx;
    J.ny = L.ny;
    J.ld = L.ld;
    J.idx = T(1.0 / L.dx);
    J.idy = T(1.0 / L.dy);
    J.ec = t ? (const T*)L.ec32 : (const T*)L.ec64;
    J.en = t ? (const T*)L.en32 : (const T*)L.en64;
    J.st = t ? (const T*)L.st32 : (const T*)L.st64;
    J.plane = L.plane;
    J.vx = (T*)L.v[t].x;
    J.vy = (T*)L.v[t].y;
    J.wx = (T*)L.w[t].x;
    J.wy = (T*)L.w[t].y;
    J.bx = (T*)L.b[t].x;
    J.by = (T*)L.b[t].y;
    J.rx = (T*)L.r[t].x;
    J.ry = (T*)L.r[t].y;
    if (l + 1 < m->L.size()) {
        const MgLevel& C = m->L[l + 1];
        J.cnx = C.nx;
        J.cny = C.ny;
        J.cld = C.ld;
        J.cbx = (T*)C.b[t].x;
        J.cby = (T*)C.b[t].y;
        J.cvx = (T*)C.v[t].x;
        J.cvy = (T*)C.v[t].y;
    }
    return J;
}

template <typename T>
int build_plan(stk_ctx* ctx, stk_mg* const* mgs, int n, int t, PlanT* P) {
    hipStream_t s = ctx->stream;
    P->n = n;
    int maxl = 0;
    for (int q = 0; q < n; ++q) {
        STK_TRY(ensure_dtype(mgs[q], 0));  // the FP64 Krylov slots exist in both modes
        STK_TRY(ensure_dtype(mgs[q], t));
        maxl = std::max(maxl, (int)mgs[q]->L.size());
        P->maxcn = std::max(P->maxcn, mgs[q]->cn);
    }
    P->depth = maxl - 1;
    P->fine.assign(maxl, Batch{});
    P->crs.assign(maxl, Batch{});
    P->cjobs.assign(maxl, nullptr);
    P->ncj.assign(maxl, 0);
    for (int d = 0; d < maxl; ++d) {
        std::vector<LevelJob<T>> jobs;
        std::vector<int> pf{0}, pc{0};
        std::vector<CoarseJob<T>> cj;
        for (int q = 0; q < n; ++q) {
            const stk_mg* m = mgs[q];
            const int nl = (int)m->L.size();
            if (d < nl - 1) {
                jobs.push_back(level_job<T>(m, d, t));
                pf.push_back(pf.back() + blocks_of(m->L[d].nx, m->L[d].ny));
                pc.push_back(pc.back() + blocks_of(m->L[d + 1].nx, m->L[d + 1].ny));
            } else if (d == nl - 1) {
                const MgLevel& L = m->L[d];
                cj.push_back(CoarseJob<T>{m->cn, m->cmap, m->cainv, (const T*)L.b[t].x, (const T*)L.b[t].y,
                                          (T*)L.v[t].x, (T*)L.v[t].y});
            }
        }
        if (!jobs.empty()) {
            const void* dj = nullptr;
            const void *dpf = nullptr, *dpc = nullptr;
            STK_TRY(upload(P, jobs, &dj, s));
            STK_TRY(upload(P, pf, &dpf, s));
            STK_TRY(upload(P, pc, &dpc, s));
            P->fine[d] = Batch{dj, (const int*)dpf, (int)jobs.size(), pf.back()};
            P->crs[d] = Batch{dj, (const int*)dpc, (int)jobs.size(), pc.back()};
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
    std::vector<int> pa{0};
    for (int q = 0; q < n; ++q) {
        stk_mg* m = mgs[q];
        LevelJob<T> J = level_job<T>(m, 0, t);
        J.vx = (T*)m->ks[t][VS_P].x;
        J.vy = (T*)m->ks[t][VS_P].y;
        J.bx = (T*)m->zero[t].x;
        J.by = (T*)m->zero[t].y;
        J.rx = (T*)m->ks[t][VS_Q].x;
        J.ry = (T*)m->ks[t][VS_Q].y;
        aj.push_back(J);
        pa.push_back(pa.back() + blocks_of(m->L[0].nx, m->L[0].ny));
        VecJob V{};
        V.nx = m->L[0].nx;
        V.ny = m->L[0].ny;
        V.ld = m->L[0].ld;
        V.idx = 1.0 / m->L[0].dx;
        V.idy = 1.0 / m->L[0].dy;
        V.ec = m->L[0].ec64;
        V.en = m->L[0].en64;
        for (int sl = 0; sl < VS_N; ++sl) {
            V.v[sl][0] = m->ks[t][sl].x;
            V.v[sl][1] = m->ks[t][sl].y;
        }
        vj.push_back(V);
        XCastJob X{};
        X.nx = V.nx;
        X.ny = V.ny;
        X.ld = V.ld;
        for (int c = 0; c < 2; ++c) {
            X.r64[c] = static_cast<const double*>(c ? m->ks[0][VS_R].y : m->ks[0][VS_R].x);
            X.z64[c] = static_cast<double*>(c ? m->ks[0][VS_Z].y : m->ks[0][VS_Z].x);
            X.r32[c] = static_cast<float*>(c ? m->ks[1][VS_R].y : m->ks[1][VS_R].x);
            X.z32[c] = static_cast<const float*>(c ? m->ks[1][VS_Z].y : m->ks[1][VS_Z].x);
        }
        xj.push_back(X);
    }
    const void *daj = nullptr, *dpa = nullptr, *dvj = nullptr, *dxj = nullptr;
    STK_TRY(upload(P, aj, &daj, s));
    STK_TRY(upload(P, pa, &dpa, s));
    STK_TRY(upload(P, vj, &dvj, s));
    P->apply = Batch{daj, (const int*)dpa, n, pa.back()};
    P->vec = Batch{dvj, (const int*)dpa, n, pa.back()};
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

int make_plan(stk_ctx* ctx, stk_mg* const* mgs, int n, int t, PlanT** out) {
    auto* P = new PlanT();
    const int rc = t ? build_plan<float>(ctx, mgs, n, t, P) : build_plan<double>(ctx, mgs, n, t, P);
    if (rc != STK_OK) {
        P->release();
        delete P;
        return rc;
    }
    *out = P;
    return STK_OK;
}

// ---- the batched V-cycle on the level-0 binding (v = Z slot, b = R slot)
template <typename T>
int smooth_stage(stk_ctx* ctx, const Batch& F, const stk_mg_opts& o, int nu) {
    for (int q = 0; q < nu; ++q) STK_TRY(mg_jacobi<T>(ctx, F, o.omega, q & 1));
    if (nu & 1) STK_TRY(mg_copy_wv<T>(ctx, F));
    return STK_OK;
}
template <typename T>
int vcycle(stk_ctx* ctx, const PlanT& P, const stk_mg_opts& o) {
    STK_TRY(mg_coarse<T>(ctx, P.cjobs[0], P.ncj[0], P.maxcn));
    for (int d = 0; d < P.depth; ++d) {
        const Batch& F = P.fine[d];
        if (!F.n) break;
        STK_TRY(smooth_stage<T>(ctx, F, o, o.nu1));
        STK_TRY(mg_residual<T>(ctx, F));
        STK_TRY(mg_zero_coarse<T>(ctx, P.crs[d]));
        STK_TRY(mg_restrict<T>(ctx, P.crs[d]));
        if (d + 1 < (int)P.cjobs.size()) STK_TRY(mg_coarse<T>(ctx, P.cjobs[d + 1], P.ncj[d + 1], P.maxcn));
    }
    for (int d = P.depth - 1; d >= 0; --d) {
        const Batch& F = P.fine[d];
        if (!F.n) continue;
        STK_TRY(mg_prolong<T>(ctx, F));
        STK_TRY(smooth_stage<T>(ctx, F, o, o.nu2));
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
int write_active(stk_ctx* ctx, const PlanT& P, std::vector<FcgState>& h, const std::vector<int>& act) {
    for (int q = 0; q < P.n; ++q) h[q].active = act[q];
    STK_HIP(hipMemcpyAsync(P.st, h.data(), sizeof(FcgState) * P.n, hipMemcpyHostToDevice, ctx->stream));
    return STK_OK;
}

// One application of the preconditioner to every active instance:
// Z = V-cycle(R) from zero, in FP64 (P32 == nullptr) or in FP32 between casts.
int precondition(stk_ctx* ctx, const PlanT& P, const PlanT* P32, const stk_mg_opts& o) {
    if (!P32) {
        STK_TRY(vec_op<double>(ctx, P.vec, OP_ZERO_Z, P.st, P.part, nullptr));
        return vcycle<double>(ctx, P, o);
    }
    STK_TRY(prec_cast(ctx, P32->xcast, P.st, 0));
    STK_TRY(vec_op<float>(ctx, P32->vec, OP_ZERO_Z, P.st, P.part, nullptr));
    STK_TRY(vcycle<float>(ctx, *P32, o));
    return prec_cast(ctx, P32->xcast, P.st, 1);
}

// Flexible CG in FP64 on the Krylov slots of plan P: X and R are set by the
// caller and the per-instance stop thresholds are in the states; at most
// `maxit` iterations.  its[q] = iterations during which instance q was active;
// *loops = iterations run.  The V-cycle runs in FP32 when P32 is given.
int fcg(stk_ctx* ctx, const PlanT& P, const PlanT* P32, const stk_mg_opts& o, int maxit, std::vector<int>& its,
        int* loops) {
    std::vector<FcgState> h;
    its.assign(P.n, 0);
    *loops = 0;
    STK_TRY(read_states(ctx, P, h));
    std::vector<int> act(P.n);
    bool any = false;
    for (int q = 0; q < P.n; ++q) {
        act[q] = h[q].active;
        any = any || act[q];
    }
    if (!any) return STK_OK;
    STK_TRY(precondition(ctx, P, P32, o));
    STK_TRY(vec_op<double>(ctx, P.vec, OP_INIT_P, P.st, P.part, P.sums));
    STK_TRY(fcg_scalars(ctx, P.st, P.sums, P.n, PH_INIT, 0.0));
    for (int it = 0; it < maxit; ++it) {
        STK_TRY(mg_residual<double>(ctx, P.apply));  // Q = 0 - M P = A P
        STK_TRY(vec_op<double>(ctx, P.vec, OP_PQ, P.st, P.part, P.sums));
        STK_TRY(fcg_scalars(ctx, P.st, P.sums, P.n, PH_ALPHA, 0.0));
        STK_TRY(vec_op<double>(ctx, P.vec, OP_UPDATE, P.st, P.part, P.sums));
        STK_TRY(fcg_scalars(ctx, P.st, P.sums, P.n, PH_NV, 0.0));
        STK_TRY(read_states(ctx, P, h));
        ++*loops;
        any = false;
        for (int q = 0; q < P.n; ++q) {
            its[q] += act[q];
            act[q] = h[q].active;
            any = any || act[q];
        }
        if (!any) break;
        STK_TRY(precondition(ctx, P, P32, o));
        STK_TRY(vec_op<double>(ctx, P.vec, OP_RZ_ZQ, P.st, P.part, P.sums));
        STK_TRY(fcg_scalars(ctx, P.st, P.sums, P.n, PH_BETA, 0.0));
        STK_TRY(vec_op<double>(ctx, P.vec, OP_XPBY, P.st, P.part, nullptr));
    }
    return STK_OK;
}

int copy_vel_in(stk_mg* m, const void* sx, const void* sy, int64_t sld, void* dx, void* dy, int64_t dld, size_t es) {
    const MgLevel& L = m->L[0];
    STK_HIP(hipMemcpy2DAsync(dx, dld * es, sx, sld * es, (size_t)(L.nx + 1) * es, L.ny, hipMemcpyDeviceToDevice,
                             m->ctx->stream));
    STK_HIP(hipMemcpy2DAsync(dy, dld * es, sy, sld * es, (size_t)L.nx * es, L.ny + 1, hipMemcpyDeviceToDevice,
                             m->ctx->stream));
    return STK_OK;
}

}  // namespace
}  // namespace stk

// ============================================================== C ABI ====
extern "C" {

void stk_mg_opts_default(stk_mg_opts* o) {
    if (!o) return;
    o->nu1 = 2;
    o->nu2 = 2;
    o->omega = 0.7;
    o->coarsest = 8;
}

static int check_mg_opts(const stk_mg_opts& o) {
    if (o.nu1 < 0 || o.nu2 < 0 || o.nu1 + o.nu2 < 1 || o.nu1 > 64 || o.nu2 > 64)
        return set_error(STK_EINVAL, "nu1, nu2 must be in [0, 64] with nu1 + nu2 >= 1");
    if (!(o.omega > 0.0 && o.omega < 2.0)) return set_error(STK_EINVAL, "omega must be in (0, 2)");
    if (o.coarsest < 2) return set_error(STK_EINVAL, "coarsest must be >= 2");
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
        // coarse = 2 * NCOEF stencil planes and v, w, b, r; FP32 extra: the same again.
        const size_t w64 = lvl == 0 ? 2 + 4 + 2 * VS_N + 3 : 2 * NCOEF + 8;
        const size_t w32 = lvl == 0 ? 2 + 4 + 4 : 2 * NCOEF + 8;
        b += cnt * (w64 * 8 + (f32 ? w32 * 4 : 0));
        if (std::min(nx, ny) <= o.coarsest || (nx & 1) || (ny & 1)) break;
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
            int rc = dalloc(m, (size_t)L.plane * 2 * NCOEF * 8, &a);
            if (rc != STK_OK) return fail(rc);
            L.st64 = static_cast<double*>(a);
            const MgLevel& F = m->L[l - 1];
            GalerkinArgs ga{F.nx, F.ny, F.ld, 1.0 / F.dx, 1.0 / F.dy, F.ec64, F.en64, F.st64, F.plane,
                            L.nx, L.ny, L.ld, L.st64, L.plane};
            rc = mg_galerkin(ctx, ga);
            if (rc != STK_OK) return fail(rc);
        }
    }
    int rc = build_coarse(m);
    if (rc != STK_OK) return fail(rc);
    *out = m;
    return STK_OK;
}

int stk_mg_destroy(stk_mg* m) {
    if (!m) return STK_OK;
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

int stk_mg_solve_batch(stk_ctx* ctx, int n, stk_mg* const* mgs, stk_solve_mode mode, double* const* vx,
                       double* const* vy, const double* const* p, const double* const* fx, const double* const* fy,
                       double tol, int max_iters, stk_report* reps) {
    if (!ctx || n < 1 || !mgs || !vx || !vy || !fx || !fy) return set_error(STK_EINVAL, "bad batch arguments");
    if (mode != STK_SOLVE_F64 && mode != STK_SOLVE_F32_REFINED) return set_error(STK_EINVAL, "unknown mode");
    if (!(tol > 0.0) || max_iters < 0) return set_error(STK_EINVAL, "tol must be > 0 and max_iters >= 0");
    for (int q = 0; q < n; ++q) {
        if (!mgs[q] || mgs[q]->ctx != ctx) return set_error(STK_EINVAL, "instance %d: mg NULL or on another context", q);
        if (!vx[q] || !vy[q] || !fx[q] || !fy[q]) return set_error(STK_EINVAL, "instance %d: NULL field", q);
        for (int r = 0; r < q; ++r)
            if (mgs[r] == mgs[q]) return set_error(STK_EINVAL, "instance %d repeats an mg handle", q);
    }
    STK_TRY(use_device(ctx));
    const auto t0 = std::chrono::steady_clock::now();
    PlanT *P = nullptr, *P32 = nullptr;
    std::vector<stk_mg*> ms(mgs, mgs + n);
    auto cleanup = [&]() {
        for (PlanT* q : {P, P32})
            if (q) {
                q->release();
                delete q;
            }
    };
    auto chk = [&](int rc) {
        if (rc != STK_OK) cleanup();
        return rc;
    };
    if (int rc = make_plan(ctx, ms.data(), n, 0, &P)) return chk(rc);
    if (mode == STK_SOLVE_F32_REFINED)
        if (int rc = make_plan(ctx, ms.data(), n, 1, &P32)) return chk(rc);
    // inputs: x0 -> X, b = f - G p -> B, f -> F (FP64)
    for (int q = 0; q < n; ++q) {
        stk_mg* m = ms[q];
        const MgLevel& L = m->L[0];
        stk_grid g{L.nx, L.ny, L.ld, L.dx, L.dy};
        const Field2& X = m->ks[0][VS_X];
        const Field2& B = m->ks[0][VS_B];
        const Field2& F = m->ks[0][VS_F];
        if (int rc = copy_vel_in(m, vx[q], vy[q], m->user_ld, X.x, X.y, L.ld, 8)) return chk(rc);
        if (int rc = copy_vel_in(m, fx[q], fy[q], m->user_ld, F.x, F.y, L.ld, 8)) return chk(rc);
        const void* pres = m->zero64;  // p = 0
        void* ptmp = nullptr;
        if (p && p[q]) {  // the caller's pressure, restrided to the mg layout
            hipError_t e = hipMalloc(&ptmp, (size_t)L.ny * L.ld * 8);
            if (e != hipSuccess) return chk(set_error(STK_ENOMEM, "pressure staging: %s", hipGetErrorString(e)));
            e = hipMemcpy2DAsync(ptmp, L.ld * 8, p[q], m->user_ld * 8, (size_t)L.nx * 8, L.ny, hipMemcpyDeviceToDevice,
                                 ctx->stream);
            if (e != hipSuccess) {
                (void)hipFree(ptmp);
                return chk(hip_fail(e, "copy p"));
            }
            pres = ptmp;
        }
        const int rcf = launch_fold_rhs(ctx, STK_F64, &g, F.x, F.y, pres, B.x, B.y);
        if (ptmp) {
            (void)hipStreamSynchronize(ctx->stream);
            (void)hipFree(ptmp);
        }
        if (rcf) return chk(rcf);
    }
    std::vector<FcgState> h(n);
    for (auto& s : h) {
        std::memset(&s, 0, sizeof s);
        s.active = 1;
    }
    STK_HIP(hipMemcpyAsync(P->st, h.data(), sizeof(FcgState) * n, hipMemcpyHostToDevice, ctx->stream));
    if (int rc = vec_op<double>(ctx, P->vec, OP_FNORM, P->st, P->part, P->sums)) return chk(rc);
    if (int rc = fcg_scalars(ctx, P->st, P->sums, n, PH_NF, tol * tol)) return chk(rc);
    // FCG; when an instance's recurrence residual reaches tol its true residual
    // is recomputed and, if still above tol (rounding drift), CG restarts from
    // the current iterate within the same iteration budget.
    std::vector<int> running(n, 1), its(n, 0);
    int used = 0;
    while (true) {
        if (int rc = read_states(ctx, *P, h)) return chk(rc);
        if (int rc = write_active(ctx, *P, h, running)) return chk(rc);
        if (int rc = vec_residual64_st(ctx, P->vec, P->st, P->part, P->sums)) return chk(rc);
        if (int rc = fcg_scalars(ctx, P->st, P->sums, n, PH_NV, 0.0)) return chk(rc);
        if (int rc = read_states(ctx, *P, h)) return chk(rc);
        bool any = false;
        for (int q = 0; q < n; ++q) {
            running[q] = running[q] && h[q].active;
            any = any || running[q];
        }
        if (!any || used >= max_iters) break;
        std::vector<int> per;
        int loops = 0;
        if (int rc = fcg(ctx, *P, P32, ms[0]->o, max_iters - used, per, &loops)) return chk(rc);
        for (int q = 0; q < n; ++q) its[q] += per[q];
        used += loops;
    }
    // final true FP64 residual of every instance
    for (auto& s : h) s.active = 1;
    STK_HIP(hipMemcpyAsync(P->st, h.data(), sizeof(FcgState) * n, hipMemcpyHostToDevice, ctx->stream));
    if (int rc = vec_residual64_st(ctx, P->vec, P->st, P->part, P->sums)) return chk(rc);
    std::vector<double> sums(2 * (size_t)n);
    STK_HIP(hipMemcpyAsync(sums.data(), P->sums, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, ctx->stream));
    for (int q = 0; q < n; ++q) {
        stk_mg* m = ms[q];
        const Field2& X = m->ks[0][VS_X];
        if (int rc = copy_vel_in(m, X.x, X.y, m->L[0].ld, vx[q], vy[q], m->user_ld, 8)) return chk(rc);
    }
    STK_HIP(hipStreamSynchronize(ctx->stream));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int rc_all = STK_OK;
    for (int q = 0; q < n; ++q) {
        const double evt = std::sqrt(sums[2 * q] / h[q].nf);
        if (reps) {
            reps[q].iterations = its[q];
            reps[q].ev = evt;
            reps[q].nf = h[q].nf;
            reps[q].seconds = secs;
            reps[q].converged = std::isfinite(evt) && evt <= tol;
        }
        if (!std::isfinite(evt)) rc_all = set_error(STK_ENONFINITE, "instance %d: residual not finite", q);
        else if (evt > tol && rc_all == STK_OK) rc_all = set_error(STK_ENOTCONV, "instance %d: E_v = %.3e > tol", q, evt);
    }
    cleanup();
    return rc_all;
}

int stk_mg_solve(stk_mg* m, stk_solve_mode mode, double* vx, double* vy, const double* p, const double* fx,
                 const double* fy, double tol, int max_iters, stk_report* rep) {
    if (!m) return set_error(STK_EINVAL, "mg is NULL");
    return stk_mg_solve_batch(m->ctx, 1, &m, mode, &vx, &vy, p ? &p : nullptr, &fx, &fy, tol, max_iters, rep);
}

}  // extern "C"
