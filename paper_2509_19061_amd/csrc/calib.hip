// Measurement helper: a plain streaming pass with the traffic pattern of one
// RAS outer iteration (six planes read, two written, Sec. 4.3), used as the
// practical HBM ceiling the smoother kernels are compared against and as the
// calibration kernel of the HBM byte counters.  One element per thread over
// the whole (ny + 1) x ld extent of the planes, consecutive threads on
// consecutive elements: the access pattern HBM serves best.
#include "stk_internal.hpp"

namespace stk {
namespace {

template <typename T>
__global__ __launch_bounds__(256) void k_stream6(int64_t n, const T* __restrict__ a0, const T* __restrict__ a1,
                                                 const T* __restrict__ a2, const T* __restrict__ a3,
                                                 const T* __restrict__ a4, const T* __restrict__ a5,
                                                 T* __restrict__ o0, T* __restrict__ o1) {
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    o0[q] = a0[q] + a2[q] * a4[q];
    o1[q] = a1[q] + a3[q] * a5[q];
}

}  // namespace
}  // namespace stk

using namespace stk;

extern "C" {

int stk_stream_probe(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const void* a0, const void* a1, const void* a2,
                     const void* a3, const void* a4, const void* a5, void* o0, void* o1) {
    if (!ctx) return set_error(STK_EINVAL, "ctx is NULL");
    if (dt != STK_F64 && dt != STK_F32) return set_error(STK_EINVAL, "unknown dtype %d", (int)dt);
    STK_TRY(check_grid(g));
    if (!a0 || !a1 || !a2 || !a3 || !a4 || !a5 || !o0 || !o1)
        return set_error(STK_EINVAL, "all eight planes must be non-NULL");
    STK_TRY(use_device(ctx));
    const int64_t n = (int64_t)(g->ny + 1) * g->ld;
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (dt == STK_F64)
        hipLaunchKernelGGL(k_stream6<double>, grid, block, 0, ctx->stream, n, (const double*)a0, (const double*)a1,
                           (const double*)a2, (const double*)a3, (const double*)a4, (const double*)a5, (double*)o0,
                           (double*)o1);
    else
        hipLaunchKernelGGL(k_stream6<float>, grid, block, 0, ctx->stream, n, (const float*)a0, (const float*)a1,
                           (const float*)a2, (const float*)a3, (const float*)a4, (const float*)a5, (float*)o0,
                           (float*)o1);
    STK_HIP(hipGetLastError());
    return STK_OK;
}

}  // extern "C"
