// Host-side types of the multigrid / Krylov layer shared by the hierarchy
// code (mg.hip) and the solve and batch engine (solve.hip).
#pragma once

#include <deque>
#include <functional>
#include <vector>

#include "mg_internal.hpp"

namespace stk {

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
    double* st64 = nullptr;  // Galerkin stencil, NPLANES planes (coarse levels only)
    float* st32 = nullptr;
    int64_t plane = 0;
    Field2 v[2], w[2], b[2], r[2];  // [0] FP64, [1] FP32; level 0 binds v, b to the Krylov Z, R slots
};

inline int64_t pad_ld(int nx) { return ((int64_t)nx + 1 + 63) / 64 * 64; }

// Device job arrays of one dtype for a fixed, ordered list of instances.
struct PlanT {
    int n = 0, depth = 0, maxcn = 0;
    std::vector<Batch> fine, crs;       // per depth: fine-block and coarse-block batches of LevelJob
    std::vector<const void*> cjobs;     // per depth: CoarseJob array of instances whose coarsest it is
    std::vector<int> ncj;
    // finest level smoothed by batched RAS outer iterations (64 x 64 tiles, halo
    // = k = the sweep count, so each is k Jacobi sweeps exactly): job arrays
    // v -> w and w -> v, the finest-level jobs with v and w exchanged (residual
    // and prolongation while the iterate is in w), the instances' sizes, and
    // the launch shape per k (built on first use)
    const void* ras_jobs[2] = {nullptr, nullptr};
    Batch fine0w;
    // coarse levels: the same LevelJob arrays with a prefix over RAS tiles
    // (coarse RAS smoothing); relaxed coarsest levels of truncated hierarchies
    // (block and tile prefixes)
    std::vector<Batch> fine_t, relax, relax_t;
    std::vector<int> l0nx, l0ny;
    std::vector<int64_t> l0ld;
    struct RasK {
        int kt, h;
        bool ok;
        RasShape shape;
        const int* pre;
    };
    mutable std::deque<RasK> ras_k;  // deque: entries keep their address as more are added
    Batch apply;                        // finest: v = P, no right-hand side, r = Q  ->  Q = A P
    Batch applyr;                       // reduction chunks over the row-streaming prefix of `apply`
    Batch vec;                          // VecJob array
    bool vec_z32 = false;               // its Z slot is FP32 (mixed-precision solves)
    Batch xcast;                        // XCastJob array (FP32 plan only)
    FcgState* st = nullptr;
    double* part = nullptr;
    double* sums = nullptr;
    mutable std::vector<void*> mem;
    std::vector<std::vector<unsigned char>> stage;  // host sources of pending uploads
    void release() {
        for (void* p : mem) (void)hipFree(p);
        mem.clear();
    }
};

// Plans over mgs[0..n) for dtype t (0 FP64, 1 FP32); *out owns its memory.
// z32 (FP64 plans): the Krylov Z slot is the FP32 V-cycle's output vector.
int make_plan(stk_ctx* ctx, stk_mg* const* mgs, int n, int t, PlanT** out, bool z32 = false);
void free_plan(PlanT*& P);
// One V-cycle on the level-0 binding (v = Z slot, b = R slot) of every instance of P.
int run_vcycle(stk_ctx* ctx, const PlanT& P, const stk_mg_opts& o, int t);
int read_states(stk_ctx* ctx, const PlanT& P, std::vector<FcgState>& h);
int write_states(stk_ctx* ctx, const PlanT& P, const std::vector<FcgState>& h);
// 2D copy of the used extents of a velocity pair between two row strides
int copy_vel_in(stk_mg* m, const void* sx, const void* sy, int64_t sld, void* dx, void* dy, int64_t dld, size_t es);
int ensure_dtype(stk_mg* m, int t);
// FP32 V-cycle correction of an FP64 velocity (uzawa.hip): v += V32(0, (float) r)
// for the FP64 residual r = f - G p - M v of the finest level (viscosities ec,
// en), in the caller's layout.
int mixed_correction(stk_mg* m, const stk_grid* g, double* vx, double* vy, const double* p, const double* ec,
                     const double* en, const double* fx, const double* fy);
// Viscosity continuation (uzawa.hip, Sec. 6.2): for theta = s / o.stages,
// s < o.stages, calls stage(hierarchy of (1 - theta) eta_min + theta eta, its
// cell and nodal viscosities, false), then stage(m, eta_c, eta_n, true) for
// the true system; o.stages = 0 is the last call only.  A stage's hierarchy
// is skipped when no cycle is left to run on it (k >= o.max_cycles or
// o.stage_cycles = 0).
int continuation(stk_mg* m, const stk_grid* g, const double* eta_c, const double* eta_n, const stk_uzawa_opts& o,
                 const int& k, const std::function<int(stk_mg*, const double*, const double*, bool)>& stage);

}  // namespace stk

struct stk_mg {
    stk_ctx* ctx = nullptr;
    stk_mg_opts o{};
    std::vector<stk::MgLevel> L;
    int64_t user_ld = 0;
    bool relaxed = false;  // truncated by max_levels: the last level is relaxed, not solved
    int cn = 0;
    int* cmap = nullptr;
    double* cainv = nullptr;
    stk::Field2 ks[2][stk::VS_N];  // finest-level slots: row 0 FP64 (all), row 1 FP32 (R, Z only)
    stk::Field2 zero[2];           // zero right-hand side for the operator apply
    void* zero64 = nullptr;        // FP64 zeros (pressure of a p = 0 fold)
    bool have[2] = {false, false};
    std::vector<void*> mem;
    size_t bytes = 0;
    stk::PlanT* plan[2] = {nullptr, nullptr};  // single-instance plans of stk_mg_vcycle
    bool busy = false;                          // in a batch
};
