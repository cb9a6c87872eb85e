// The energy norm with no allocation (for callers that cannot allocate device
// memory: code under HIP graph capture, tight serving loops).
//
// stk_energy_norm keeps its per-wave partial sums in the context's scratch,
// which grows on demand (hipMalloc).  This variant takes them from a
// file-scope device array of fixed size instead, and writes the five results
// to device memory without waiting, so the call allocates nothing and never
// synchronises.  Each GPU holds its own copy of the array until the process
// ends; its address on a device is looked up once per device, with that
// device current, and only that address is passed to kernels.
#include <mutex>

#include "stk_internal.hpp"

namespace {

// Partial sums of the energy kernel: 3 doubles per wave of the row-streaming
// launch.  8 MiB holds the 349525 triples of square grids up to 37199 x 37199.
constexpr size_t SCRATCH_DOUBLES = (size_t)1 << 20;
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

constexpr int MAX_DEV = 64;
std::mutex g_mu;
double* g_ptr[MAX_DEV] = {};

// The device address of `scratch` on the current device `dev`.
int scratch_address(int dev, double** out) {
    if (dev < 0 || dev >= MAX_DEV) return stk::set_error(STK_EUNSUPPORTED, "device %d beyond %d", dev, MAX_DEV);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return stk::hip_fail(e != hipSuccess ? e : hipErrorUnknown, "hipGetSymbolAddress");
        g_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_ptr[dev];
    return STK_OK;
}

}  // namespace

extern "C" {

int stk_energy_norm_noalloc(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const void* vx, const void* vy,
                            const void* p, const void* eta_c, const void* eta_n, const void* fx, const void* fy,
                            double* out) {
    if (!ctx) return stk::set_error(STK_EINVAL, "ctx is NULL");
    if (dt != STK_F64 && dt != STK_F32) return stk::set_error(STK_EINVAL, "unknown dtype %d", (int)dt);
    STK_TRY(stk::check_grid(g));
    if (!vx || !vy || !eta_c || !eta_n || !fx || !fy || !out)
        return stk::set_error(STK_EINVAL, "vx, vy, eta_c, eta_n, fx, fy, out must be non-NULL");
    const int64_t triples = stk::energy_partials(g);
    if ((size_t)triples * 3 > SCRATCH_DOUBLES)
        return stk::set_error(STK_EUNSUPPORTED,
                              "grid %d x %d needs %lld partial triples; the static scratch holds %zu (use "
                              "stk_energy_norm)", g->nx, g->ny, (long long)triples, SCRATCH_DOUBLES / 3);
    STK_TRY(stk::use_device(ctx));
    double* part = nullptr;
    STK_TRY(scratch_address(ctx->device, &part));
    return stk::launch_energy_into(ctx, dt, g, vx, vy, p, eta_c, eta_n, fx, fy, part, out, true);
}

}  // extern "C"
