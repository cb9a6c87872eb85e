// Internal declarations of the stk HIP library (host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "stk.h"

struct stk_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int lds_max = 0;  // bytes of LDS one workgroup may use on this device
    int lds_cu = 0;   // bytes of LDS per CU
    int num_cu = 0;
    int ras_kernel = 0;  // 0 auto (streaming when it fits), 1 LDS window only, 2 streaming only
    // Scratch slots, grown on demand (device memory).
    enum { S_VX = 0, S_VY, S_VX2, S_VY2, S_BX, S_BY, S_PART, S_RED, S_NSLOT };
    void* slot[S_NSLOT] = {};
    size_t slot_bytes[S_NSLOT] = {};
    double* host_red = nullptr;  // pinned host landing buffer for reductions
};

namespace stk {

// Device arrays named inside a job struct.  In device code they carry the
// global address space: a kernel reads them from a job array in memory, and
// without it the compiler cannot tell global from LDS and emits flat loads,
// which count against the LDS wait counter too, so that every use of an LDS
// value waited for all the loads in flight.  In host code they are plain
// pointers of the same size (host code sets them with an explicit cast).
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
#else
template <typename T>
using gptr = T*;
#endif


int set_error(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
#define STK_HIP(call)                                      \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return stk::hip_fail(e_, #call); \
    } while (0)
#define STK_TRY(call)              \
    do {                           \
        int rc_ = (call);          \
        if (rc_ != STK_OK) return rc_; \
    } while (0)

// Make sure slot `s` of the context holds at least `bytes`; returns its pointer.
int scratch(stk_ctx* ctx, int s, size_t bytes, void** out);
// Make `ctx->device` current.
int use_device(stk_ctx* ctx);

int check_grid(const stk_grid* g);
size_t elem_size(stk_dtype dt);
// Bytes spanned by a field of `rows` rows of the grid's stride.
inline size_t field_bytes(const stk_grid* g, int rows, stk_dtype dt) { return (size_t)rows * (size_t)g->ld * elem_size(dt); }

// ---- kernel launchers (defined in the .hip files) ---------------------------
struct FieldPtrs {
    const void* eta_c;
    const void* eta_n;
    const void* bx;  // right-hand side at vx points (f folded with p, or fx)
    const void* by;
};

int launch_fold_rhs(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const void* fx, const void* fy, const void* p,
                    void* bx, void* by);
// FP64 residual f - G p - M v rounded to FP32 into (r32x, r32y), and
// (z32x, z32y) zeroed, on the velocity extents (FP32 arrays, stride g->ld).
int launch_residual_to32(stk_ctx* ctx, const stk_grid* g, const double* vx, const double* vy, const double* p,
                         const double* eta_c, const double* eta_n, const double* fx, const double* fy, float* r32x,
                         float* r32y, float* z32x, float* z32y);
int launch_jacobi_rows(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const FieldPtrs& f, double omega,
                       const void* vx, const void* vy, void* ox, void* oy);
int launch_jacobi_fused(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const FieldPtrs& f, double omega,
                        const void* vx, const void* vy, void* ox, void* oy);
int launch_jacobi_split(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const FieldPtrs& f, double omega,
                        const void* vx, const void* vy, void* ox, void* oy);
int launch_zero_walls(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, void* vx, void* vy);
int launch_rbgs(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const FieldPtrs& f, double omega, void* vx, void* vy);
// RAS outer iteration; returns STK_EUNSUPPORTED when the tile does not fit.
int ras_lds_bytes(stk_dtype dt, const stk_grid* g, int tile_x, int tile_y, int halo, size_t* bytes);
int launch_ras(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const FieldPtrs& f, double omega, int tile_x,
               int tile_y, int halo, int kt, int sx, int sy, const void* vx, const void* vy, void* ox, void* oy);
// Streaming RAS kernel; *done = false when the configuration does not fit it.
int launch_ras_stream(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const FieldPtrs& f, double omega, int tile_x,
                      int tile_y, int halo, int kt, int sx, int sy, const void* vx, const void* vy, void* ox, void* oy,
                      bool* done);
// One instance of a batched RAS outer iteration: its grid's fields, the
// snapshot and the result (device pointers, common row stride ld).
template <typename T>
struct RasJob {
    gptr<const T> ec, en, bx, by;
    int64_t ld;
    int nx, ny;
    T idx, idy;
    gptr<const T> vx, vy;
    gptr<T> ox, oy;
    int ntx;  // tile columns
};
// Launch shape of a batched RAS outer iteration, shared by its instances.
struct RasShape {
    int tile, h, kt, NT, Wm, Vmax, nthr, mm, ws, nwg;
    int merge;  // full overlap: a workgroup's NT tiles are streamed as one
    int ty;     // tile height: the tile, or (full overlap) the height that fills whole rounds
    size_t lds;
};
// Shape for instances of nx[i] x ny[i] cells (square tiles cut at multiples
// of the tile, halo h, kt sweeps): fills the workgroup prefix pre[0..n] and
// each instance's tile columns; *ok = false when the streaming kernel cannot
// take them (window or LDS too large).
int ras_batch_shape(stk_ctx* ctx, stk_dtype dt, const int* nx, const int* ny, const int64_t* ld, int n, int tile,
                    int h, int kt, RasShape* out, std::vector<int>* pre, std::vector<int>* ntx, bool* ok);
// One outer iteration of every instance of a RasJob array (device) with the
// shape above; pre: the device copy of the prefix.
int ras_batch_launch(stk_ctx* ctx, stk_dtype dt, const RasShape& s, const void* jobs, const int* pre, int n,
                     double omega);
int launch_copy_velocity(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const void* vx, const void* vy, void* ox,
                         void* oy);
int launch_residual(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const void* vx, const void* vy, const void* p,
                    const void* eta_c, const void* eta_n, const void* fx, const void* fy, void* rx, void* ry,
                    void* rp);
// Energy partial sums -> 3 doubles in device memory `dst` (N_v, N_p, N_f).
int launch_energy(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const void* vx, const void* vy, const void* p,
                  const void* eta_c, const void* eta_n, const void* fx, const void* fy, double* dst);
// Triples of partial sums the energy kernel writes for grid g.
int64_t energy_partials(const stk_grid* g);
// The energy norm with caller-provided partials (3 * energy_partials(g)
// doubles); dst[0..2] = N_v, N_p, N_f and, with `finish`, dst[3] = E and
// dst[4] = E_v, all in device memory.  Allocates nothing.
int launch_energy_into(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const void* vx, const void* vy, const void* p,
                       const void* eta_c, const void* eta_n, const void* fx, const void* fy, double* part,
                       double* dst, bool finish);

}  // namespace stk
