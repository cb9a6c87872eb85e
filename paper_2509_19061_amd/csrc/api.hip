// Host side of the stk C ABI: contexts, argument checks, the smoother driver
// (ping-pong buffers, RAS shift stream), residual and energy-norm calls.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "stk_internal.hpp"

namespace stk {

static thread_local char g_err[512] = "";

int set_error(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return set_error(e == hipErrorOutOfMemory ? STK_ENOMEM : STK_EHIP, "%s failed: %s", what, hipGetErrorString(e));
}

int use_device(stk_ctx* ctx) {
    STK_HIP(hipSetDevice(ctx->device));
    return STK_OK;
}

int scratch(stk_ctx* ctx, int s, size_t bytes, void** out) {
    if (ctx->slot_bytes[s] < bytes) {
        if (ctx->slot[s]) {
            // the old buffer may still be in use by queued work
            STK_HIP(hipStreamSynchronize(ctx->stream));
            STK_HIP(hipFree(ctx->slot[s]));
            ctx->slot[s] = nullptr;
            ctx->slot_bytes[s] = 0;
        }
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) return set_error(STK_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
        ctx->slot[s] = p;
        ctx->slot_bytes[s] = bytes;
    }
    *out = ctx->slot[s];
    return STK_OK;
}

int check_grid(const stk_grid* g) {
    if (!g) return set_error(STK_EINVAL, "grid is NULL");
    if (g->nx < 2 || g->ny < 2) return set_error(STK_EINVAL, "nx, ny must be >= 2 (got %d, %d)", g->nx, g->ny);
    if (g->ld < (int64_t)g->nx + 1) return set_error(STK_EINVAL, "ld (%lld) must be >= nx + 1", (long long)g->ld);
    if (!(g->dx > 0.0) || !(g->dy > 0.0) || !std::isfinite(g->dx) || !std::isfinite(g->dy))
        return set_error(STK_EINVAL, "dx, dy must be finite and > 0");
    if ((int64_t)(g->ny + 1) * g->ld > ((int64_t)1 << 40))
        return set_error(STK_EINVAL, "grid too large");
    return STK_OK;
}

size_t elem_size(stk_dtype dt) { return dt == STK_F64 ? sizeof(double) : sizeof(float); }

static int check_dtype(stk_dtype dt) {
    if (dt != STK_F64 && dt != STK_F32) return set_error(STK_EINVAL, "unknown dtype %d", (int)dt);
    return STK_OK;
}

static uint64_t splitmix64_next(uint64_t& state) {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace stk

using namespace stk;

extern "C" {

const char* stk_last_error(void) { return g_err; }

int stk_ctx_create(stk_ctx** out, int device, void* hip_stream) {
    if (!out) return set_error(STK_EINVAL, "out is NULL");
    int ndev = 0;
    STK_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return set_error(STK_EINVAL, "device %d out of range (%d devices)", device, ndev);
    STK_HIP(hipSetDevice(device));
    auto* c = new stk_ctx();
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    int a = 0, b = 0;
    (void)hipDeviceGetAttribute(&a, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
    (void)hipDeviceGetAttribute(&b, hipDeviceAttributeSharedMemPerBlockOptin, device);
    c->lds_max = a > b ? a : b;
    (void)hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, device);
    (void)hipDeviceGetAttribute(&c->lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device);
    if (const char* rk = std::getenv("STK_RAS_KERNEL")) {
        if (!std::strcmp(rk, "window")) c->ras_kernel = 1;
        else if (!std::strcmp(rk, "stream")) c->ras_kernel = 2;
    }
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&c->host_red), 64 * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "hipHostMalloc");
    }
    *out = c;
    return STK_OK;
}

int stk_ctx_destroy(stk_ctx* ctx) {
    if (!ctx) return STK_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (int s = 0; s < stk_ctx::S_NSLOT; ++s)
        if (ctx->slot[s]) (void)hipFree(ctx->slot[s]);
    if (ctx->host_red) (void)hipHostFree(ctx->host_red);
    delete ctx;
    return STK_OK;
}

int stk_ctx_set_stream(stk_ctx* ctx, void* hip_stream) {
    if (!ctx) return set_error(STK_EINVAL, "ctx is NULL");
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return STK_OK;
}

int stk_ctx_sync(stk_ctx* ctx) {
    if (!ctx) return set_error(STK_EINVAL, "ctx is NULL");
    STK_TRY(use_device(ctx));
    STK_HIP(hipStreamSynchronize(ctx->stream));
    return STK_OK;
}

int stk_ctx_scratch_bytes(const stk_ctx* ctx, size_t* bytes) {
    if (!ctx || !bytes) return set_error(STK_EINVAL, "NULL argument");
    size_t s = 0;
    for (int k = 0; k < stk_ctx::S_NSLOT; ++k) s += ctx->slot_bytes[k];
    *bytes = s;
    return STK_OK;
}

void stk_smooth_opts_default(stk_smooth_opts* o) {
    if (!o) return;
    o->omega = 0.0;
    o->tile_x = 64;
    o->tile_y = 64;
    o->halo = -1;
    o->k = 4;
    o->shifts = nullptr;
    o->seed = 0;
    o->last_partial = 1;
}

int stk_ras_shifts(uint64_t seed, int n_outer, int tile_x, int tile_y, int32_t* out) {
    if (n_outer < 0 || tile_x < 1 || tile_y < 1) return set_error(STK_EINVAL, "bad n_outer/tile");
    if (n_outer > 0 && !out) return set_error(STK_EINVAL, "out is NULL");
    uint64_t st = seed;
    for (int t = 0; t < n_outer; ++t) {
        out[2 * t] = (int32_t)((splitmix64_next(st) >> 32) % (uint64_t)tile_x);
        out[2 * t + 1] = (int32_t)((splitmix64_next(st) >> 32) % (uint64_t)tile_y);
    }
    return STK_OK;
}

int stk_smooth(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, void* vx, void* vy, const void* p, const void* eta_c,
               const void* eta_n, const void* fx, const void* fy, int sweeps, stk_variant variant,
               const stk_smooth_opts* opts) {
    if (!ctx) return set_error(STK_EINVAL, "ctx is NULL");
    STK_TRY(check_dtype(dt));
    STK_TRY(check_grid(g));
    if (!vx || !vy || !eta_c || !eta_n || !fx || !fy)
        return set_error(STK_EINVAL, "vx, vy, eta_c, eta_n, fx, fy must be non-NULL");
    if (sweeps < 0) return set_error(STK_EINVAL, "sweeps must be >= 0");
    if (variant < STK_JACOBI || variant > STK_RBGS) return set_error(STK_EINVAL, "unknown variant %d", (int)variant);
    stk_smooth_opts o;
    stk_smooth_opts_default(&o);
    if (opts) o = *opts;
    double omega = o.omega == 0.0 ? (variant == STK_RBGS ? 1.0 : 0.7) : o.omega;
    if (!(omega > 0.0 && omega < 2.0)) return set_error(STK_EINVAL, "omega must be in (0, 2)");
    if (variant == STK_RAS_JACOBI) {
        if (o.tile_x < 1 || o.tile_y < 1) return set_error(STK_EINVAL, "tile must be >= 1");
        if (o.k < 1) return set_error(STK_EINVAL, "k must be >= 1");
        if (o.halo < -1) return set_error(STK_EINVAL, "halo must be >= 0 (or -1 for k)");
        if (o.tile_x > (1 << 20) || o.tile_y > (1 << 20) || o.halo > (1 << 20))
            return set_error(STK_EINVAL, "tile/halo too large");
    }
    if (sweeps == 0) return STK_OK;
    STK_TRY(use_device(ctx));

    int h = 0, nouter = 0;
    std::vector<int32_t> shifts;
    if (variant == STK_RAS_JACOBI) {
        h = o.halo < 0 ? o.k : o.halo;
        size_t lds = 0;
        ras_lds_bytes(dt, g, o.tile_x, o.tile_y, h, &lds);
        if (lds > (size_t)ctx->lds_max)
            return set_error(STK_EUNSUPPORTED, "RAS tile %dx%d with halo %d needs %zu bytes of LDS (limit %d)",
                             o.tile_x, o.tile_y, h, lds, ctx->lds_max);
        nouter = (sweeps + o.k - 1) / o.k;
        shifts.resize(2 * (size_t)nouter);
        if (o.shifts) {
            for (int t = 0; t < 2 * nouter; ++t) shifts[t] = o.shifts[t];
        } else {
            stk_ras_shifts(o.seed, nouter, o.tile_x, o.tile_y, shifts.data());
        }
        for (int t = 0; t < nouter; ++t) {
            shifts[2 * t] = ((shifts[2 * t] % o.tile_x) + o.tile_x) % o.tile_x;
            shifts[2 * t + 1] = ((shifts[2 * t + 1] % o.tile_y) + o.tile_y) % o.tile_y;
        }
    }

    const size_t vbytes = field_bytes(g, g->ny + 1, dt);
    FieldPtrs f{eta_c, eta_n, fx, fy};
    if (p) {
        void *bx = nullptr, *by = nullptr;
        STK_TRY(scratch(ctx, stk_ctx::S_BX, vbytes, &bx));
        STK_TRY(scratch(ctx, stk_ctx::S_BY, vbytes, &by));
        STK_TRY(launch_fold_rhs(ctx, dt, g, fx, fy, p, bx, by));
        f.bx = bx;
        f.by = by;
    }
    if (variant == STK_RBGS) {
        STK_TRY(launch_zero_walls(ctx, dt, g, vx, vy));
        for (int s = 0; s < sweeps; ++s) STK_TRY(launch_rbgs(ctx, dt, g, f, omega, vx, vy));
        return STK_OK;
    }

    // Out-of-place steps: the first reads the caller's arrays, the last writes them, and the
    // ones between alternate over two scratch pairs, so no copy is needed for n >= 2 steps
    // (two buffers alone would end an odd count in scratch).
    const bool ras = !(variant == STK_JACOBI_FUSED || variant == STK_JACOBI);
    const int n = ras ? nouter : sweeps;
    void *tx = nullptr, *ty = nullptr, *ux = nullptr, *uy = nullptr;
    STK_TRY(scratch(ctx, stk_ctx::S_VX, vbytes, &tx));
    STK_TRY(scratch(ctx, stk_ctx::S_VY, vbytes, &ty));
    if (n >= 3) {
        STK_TRY(scratch(ctx, stk_ctx::S_VX2, vbytes, &ux));
        STK_TRY(scratch(ctx, stk_ctx::S_VY2, vbytes, &uy));
    }
    const void *cx = vx, *cy = vy;  // current iterate
    for (int t = 0; t < n; ++t) {
        void *dx = tx, *dy = ty;  // next
        if (t == n - 1 && n >= 2) {
            dx = vx;
            dy = vy;
        } else if (cx == tx) {
            dx = ux;
            dy = uy;
        }
        if (variant == STK_JACOBI_FUSED) {
            STK_TRY(launch_jacobi_fused(ctx, dt, g, f, omega, cx, cy, dx, dy));
        } else if (variant == STK_JACOBI) {
            STK_TRY(launch_jacobi_split(ctx, dt, g, f, omega, cx, cy, dx, dy));
        } else {
            int kt = o.k;
            if (o.last_partial && t == nouter - 1 && sweeps % o.k) kt = sweeps % o.k;
            STK_TRY(launch_ras(ctx, dt, g, f, omega, o.tile_x, o.tile_y, h, kt, shifts[2 * t], shifts[2 * t + 1], cx,
                               cy, dx, dy));
        }
        cx = dx;
        cy = dy;
    }
    if (cx != vx) STK_TRY(launch_copy_velocity(ctx, dt, g, cx, cy, vx, vy));
    return STK_OK;
}

int stk_ras_outer(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const void* vx, const void* vy, const void* eta_c,
                  const void* eta_n, const void* bx, const void* by, void* ox, void* oy, double omega, int tile_x,
                  int tile_y, int halo, int kt, int sx, int sy) {
    if (!ctx) return set_error(STK_EINVAL, "ctx is NULL");
    STK_TRY(check_dtype(dt));
    STK_TRY(check_grid(g));
    if (!vx || !vy || !eta_c || !eta_n || !bx || !by || !ox || !oy)
        return set_error(STK_EINVAL, "vx, vy, eta_c, eta_n, bx, by, ox, oy must be non-NULL");
    if (ox == vx || oy == vy || ox == vy || oy == vx) return set_error(STK_EINVAL, "outputs alias the inputs");
    if (!(omega > 0.0 && omega < 2.0)) return set_error(STK_EINVAL, "omega must be in (0, 2)");
    if (tile_x < 1 || tile_y < 1 || halo < 0 || kt < 0 || tile_x > (1 << 20) || tile_y > (1 << 20) || halo > (1 << 20))
        return set_error(STK_EINVAL, "bad tile/halo/kt");
    STK_TRY(use_device(ctx));
    FieldPtrs f{eta_c, eta_n, bx, by};
    sx = ((sx % tile_x) + tile_x) % tile_x;
    sy = ((sy % tile_y) + tile_y) % tile_y;
    return launch_ras(ctx, dt, g, f, omega, tile_x, tile_y, halo, kt, sx, sy, vx, vy, ox, oy);
}

int stk_residual(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const void* vx, const void* vy, const void* p,
                 const void* eta_c, const void* eta_n, const void* fx, const void* fy, void* rx, void* ry, void* rp) {
    if (!ctx) return set_error(STK_EINVAL, "ctx is NULL");
    STK_TRY(check_dtype(dt));
    STK_TRY(check_grid(g));
    if (!vx || !vy || !eta_c || !eta_n || !fx || !fy || !rx || !ry)
        return set_error(STK_EINVAL, "vx, vy, eta_c, eta_n, fx, fy, rx, ry must be non-NULL");
    if (rx == vx || ry == vy || rx == vy || ry == vx) return set_error(STK_EINVAL, "outputs alias the velocity");
    STK_TRY(use_device(ctx));
    return launch_residual(ctx, dt, g, vx, vy, p, eta_c, eta_n, fx, fy, rx, ry, rp);
}

int stk_energy_norm(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const void* vx, const void* vy, const void* p,
                    const void* eta_c, const void* eta_n, const void* fx, const void* fy, double out[5]) {
    if (!ctx) return set_error(STK_EINVAL, "ctx is NULL");
    STK_TRY(check_dtype(dt));
    STK_TRY(check_grid(g));
    if (!vx || !vy || !eta_c || !eta_n || !fx || !fy || !out)
        return set_error(STK_EINVAL, "vx, vy, eta_c, eta_n, fx, fy, out must be non-NULL");
    STK_TRY(use_device(ctx));
    void* red = nullptr;
    STK_TRY(scratch(ctx, stk_ctx::S_RED, 64 * sizeof(double), &red));
    STK_TRY(launch_energy(ctx, dt, g, vx, vy, p, eta_c, eta_n, fx, fy, static_cast<double*>(red)));
    STK_HIP(hipMemcpyAsync(ctx->host_red, red, 3 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    STK_HIP(hipStreamSynchronize(ctx->stream));
    const double nv = ctx->host_red[0], np = ctx->host_red[1], nf = ctx->host_red[2];
    out[0] = nv;
    out[1] = np;
    out[2] = nf;
    out[3] = std::sqrt((nv + np) / nf);
    out[4] = std::sqrt(nv / nf);
    for (int k = 0; k < 5; ++k)
        if (!std::isfinite(out[k])) return set_error(STK_ENONFINITE, "energy norm is not finite (out[%d] = %g)", k, out[k]);
    return STK_OK;
}

}  // extern "C"
