// Krylov solves and the continuous-batching engine.
//
// Every solve is flexible conjugate gradients on the SPD system -M v = -b in
// FP64 (residual, operator, dot products, energy norms), preconditioned by one
// V-cycle per iteration in FP64 or in FP32 (paper Sec. 3.2: multigrid for the
// velocity update; Sec. 6.4: the energy residual E_v used as the stop test).
//
// A batch (stk_batch) holds slots of in-flight solves.  A slot moves through
//   NEW    admitted: N_f and the stop threshold are still to be computed,
//   CHECK  the true residual b - M x is to be computed: the solve finishes if
//          E_v <= tol or its iteration budget is spent, and otherwise (re)starts
//          CG from x (first start, or a restart after the recurrence residual
//          drifted below tol while the true one did not),
//   ITER   iterating: member of the batch's main plan,
// and back to FREE when it finishes.  Every step runs the NEW / CHECK slots
// through one temporary plan, then advances all ITER slots together: each
// level kernel is one launch over every member's blocks.  Slots join and
// leave between steps; the per-slot CG scalars live in a host mirror that is
// re-uploaded whenever the main plan is rebuilt.  The arithmetic of a slot
// never depends on which other slots share its launches.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "mg_host.hpp"

namespace stk {
namespace {

enum SlotState { SL_FREE = 0, SL_NEW, SL_CHECK, SL_ITER };

struct Slot {
    stk_mg* m = nullptr;
    double* ux = nullptr;  // caller's solution arrays (written when the slot finishes)
    double* uy = nullptr;
    double tol = 0.0;
    int max_iters = 0;
    int its = 0;
    int state = SL_FREE;
    double last_nv = -1.0;  // N_v of the previous true-residual check (-1: none yet)
    int stalls = 0;         // consecutive checks that did not halve it
    FcgState fs{};
    std::chrono::steady_clock::time_point t0;
};

// Z = V-cycle(R) from zero for every active instance of P, in FP64 (P32 ==
// nullptr) or in FP32 between the casts R -> R32 and Z32 -> Z.  z_zeroed: the
// FP64 Z is already 0 (OP_UPDATE clears it).
int precondition(stk_ctx* ctx, const PlanT& P, const PlanT* P32, const stk_mg_opts& o, bool z_zeroed) {
    if (!P32) {
        if (!z_zeroed) STK_TRY(vec_op<double>(ctx, P.vec, OP_ZERO_Z, P.st, P.part));
        return run_vcycle(ctx, P, o, 0);
    }
    // r32 = (float) r and z32 = 0, the FP32 V-cycle, whose z32 the Krylov steps read in place
    STK_TRY(prec_cast(ctx, P32->xcast, P.st));
    return run_vcycle(ctx, *P32, o, 1);
}

}  // namespace
}  // namespace stk

using namespace stk;

struct stk_batch {
    stk_ctx* ctx = nullptr;
    stk_solve_mode mode = STK_SOLVE_F64;
    std::vector<Slot> slots;
    PlanT* P = nullptr;    // main plan over `members` (ITER slots), FP64
    PlanT* P32 = nullptr;  // its FP32 V-cycle plan (mixed-precision mode)
    std::vector<int> members;
    bool dirty = true;
    bool have_opts = false;
    stk_mg_opts o{};       // V-cycle options shared by every instance of the batch
    // Look-ahead (stk_mg_solve_batch, which runs its batch to the end alone): the
    // member states are read while the rest of the iteration is queued.  Batches
    // of the caller (serving) read them before queueing it: queueing a whole
    // iteration ahead made a serving loop that sets requests up on another
    // stream meanwhile 35 % slower.
    bool lookahead = false;
    // pinned host copy of the member states, read once per iteration; the reduction
    // kernel that updates them writes it on the solve's stream (a copy-engine
    // transfer would queue behind unrelated uploads: requests being set up on
    // another stream while the batch runs)
    FcgState* pin = nullptr;
    FcgState* pin_dev = nullptr;  // its device-side address
    int npin = 0;
    hipEvent_t ev = nullptr;  // marks that copy in the stream
};

namespace stk {
namespace {

int plans_for(stk_batch* b, const std::vector<int>& ids, PlanT** P, PlanT** P32) {
    std::vector<stk_mg*> ms;
    for (int id : ids) ms.push_back(b->slots[id].m);
    STK_TRY(make_plan(b->ctx, ms.data(), (int)ms.size(), 0, P, b->mode == STK_SOLVE_F32_REFINED));
    if (b->mode == STK_SOLVE_F32_REFINED) {
        const int rc = make_plan(b->ctx, ms.data(), (int)ms.size(), 1, P32);
        if (rc != STK_OK) {
            free_plan(*P);
            return rc;
        }
    }
    return STK_OK;
}

int ensure_pinned(stk_batch* b, int n) {
    if (!b->ev) STK_HIP(hipEventCreateWithFlags(&b->ev, hipEventDisableTiming));
    if (b->npin >= n) return STK_OK;
    if (b->pin) STK_HIP(hipHostFree(b->pin));
    b->pin = b->pin_dev = nullptr;
    b->npin = 0;
    STK_HIP(hipHostMalloc(reinterpret_cast<void**>(&b->pin), sizeof(FcgState) * (size_t)n, hipHostMallocCoherent));
    STK_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&b->pin_dev), b->pin, 0));
    b->npin = n;
    return STK_OK;
}


// Write the solution to the caller's arrays and fill the report (the true
// residual of the slot's last CHECK is in its state).
int finish(stk_batch* b, int id, stk_report* rep) {
    Slot& s = b->slots[id];
    stk_mg* m = s.m;
    const Field2& X = m->ks[0][VS_X];
    STK_TRY(copy_vel_in(m, X.x, X.y, m->L[0].ld, s.ux, s.uy, m->user_ld, 8));
    const double ev = std::sqrt(s.fs.nv / s.fs.nf);
    rep->iterations = s.its;
    rep->ev = ev;
    rep->nf = s.fs.nf;
    rep->converged = std::isfinite(ev) && ev <= s.tol;
    rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - s.t0).count();
    m->busy = false;
    s = Slot{};
    b->dirty = true;
    return STK_OK;
}

// NEW and CHECK slots: N_f (NEW), true residual, finish or (re)start CG.
int start_phase(stk_batch* b, int* done, stk_report* reps, int* ndone) {
    std::vector<int> ids;
    for (int i = 0; i < (int)b->slots.size(); ++i)
        if (b->slots[i].state == SL_NEW || b->slots[i].state == SL_CHECK) ids.push_back(i);
    if (ids.empty()) return STK_OK;
    stk_ctx* ctx = b->ctx;
    PlanT *Q = nullptr, *Q32 = nullptr;
    STK_TRY(plans_for(b, ids, &Q, &Q32));
    auto fail = [&](int rc) {
        free_plan(Q);
        free_plan(Q32);
        return rc;
    };
    const int n = (int)ids.size();
    const stk_mg_opts o = b->o;
    std::vector<FcgState> h(n);
    bool any_new = false;
    for (int q = 0; q < n; ++q) {
        h[q] = b->slots[ids[q]].fs;
        h[q].active = b->slots[ids[q]].state == SL_NEW;
        any_new = any_new || h[q].active;
    }
    if (any_new) {
        if (int rc = write_states(ctx, *Q, h)) return fail(rc);
        if (int rc = vec_op<double>(ctx, Q->vec, OP_FNORM, Q->st, Q->part)) return fail(rc);
        if (int rc = fcg_reduce(ctx, Q->vec, Q->part, Q->sums, Q->st, PH_NF)) return fail(rc);
        if (int rc = read_states(ctx, *Q, h)) return fail(rc);
    }
    for (auto& s : h) s.active = 1;
    if (int rc = write_states(ctx, *Q, h)) return fail(rc);
    if (int rc = vec_residual64_st(ctx, Q->vec, Q->st, Q->part)) return fail(rc);
    if (int rc = fcg_reduce(ctx, Q->vec, Q->part, Q->sums, Q->st, PH_TRUE)) return fail(rc);
    if (int rc = read_states(ctx, *Q, h)) return fail(rc);
    bool restart = false;
    for (int q = 0; q < n; ++q) {
        Slot& s = b->slots[ids[q]];
        s.fs = h[q];
        bool stalled = false;  // restarts no longer gain: E_v is at its FP64 floor
        if (h[q].active && s.m->o.stall_checks > 0) {
            s.stalls = (s.last_nv >= 0.0 && !(h[q].nv <= 0.5 * s.last_nv)) ? s.stalls + 1 : 0;
            s.last_nv = h[q].nv;
            stalled = s.stalls >= s.m->o.stall_checks;
        }
        if (!h[q].active || s.its >= s.max_iters || stalled) {
            h[q].active = 0;
            done[*ndone] = ids[q];
            if (int rc = finish(b, ids[q], &reps[*ndone])) return fail(rc);
            ++*ndone;
        } else {
            h[q].left = s.max_iters - s.its;  // the device stops the instance when its budget runs out
            restart = true;
        }
    }
    if (restart) {  // Z = V(R), P = Z, gamma for the slots that go on
        if (int rc = write_states(ctx, *Q, h)) return fail(rc);
        if (int rc = precondition(ctx, *Q, Q32, o, false)) return fail(rc);
        if (int rc = vec_op<double>(ctx, Q->vec, OP_INIT_P, Q->st, Q->part, Q->vec_z32)) return fail(rc);
        if (int rc = fcg_reduce(ctx, Q->vec, Q->part, Q->sums, Q->st, PH_INIT)) return fail(rc);
        if (int rc = read_states(ctx, *Q, h)) return fail(rc);
        for (int q = 0; q < n; ++q) {
            Slot& s = b->slots[ids[q]];
            if (s.state == SL_FREE || !h[q].active) continue;
            s.fs = h[q];
            s.state = SL_ITER;
            b->dirty = true;
        }
    }
    free_plan(Q);
    free_plan(Q32);
    return STK_OK;
}

// Up to `iters` CG iterations of every ITER slot, all in the same launches.
int iterate_phase(stk_batch* b, int iters) {
    stk_ctx* ctx = b->ctx;
    if (b->dirty) {
        free_plan(b->P);
        free_plan(b->P32);
        b->members.clear();
        for (int i = 0; i < (int)b->slots.size(); ++i)
            if (b->slots[i].state == SL_ITER) b->members.push_back(i);
        b->dirty = false;
        if (b->members.empty()) return STK_OK;
        STK_TRY(plans_for(b, b->members, &b->P, &b->P32));
    }
    if (b->members.empty()) return STK_OK;
    const PlanT& P = *b->P;
    const int n = (int)b->members.size();
    const stk_mg_opts o = b->o;
    std::vector<FcgState> h(n);
    for (int q = 0; q < n; ++q) h[q] = b->slots[b->members[q]].fs;
    STK_TRY(write_states(ctx, P, h));
    if (b->lookahead) STK_TRY(ensure_pinned(b, n));
    // the states after an iteration's update: ++its of the members that took part, CHECK
    // for those that stopped (below tol: verify with the true residual; or budget spent);
    // false when none goes on
    auto take = [&](const FcgState* hn) {
        bool any = false;
        for (int q = 0; q < n; ++q) {
            Slot& s = b->slots[b->members[q]];
            const bool was = h[q].active != 0;
            h[q] = hn[q];
            if (!was) continue;
            ++s.its;
            if (!h[q].active) {
                s.state = SL_CHECK;
                b->dirty = true;
            } else {
                any = true;
            }
        }
        return any;
    };
    std::vector<FcgState> hn;
    for (int it = 0; it < iters; ++it) {
        STK_TRY(fcg_apply_pq(ctx, P.apply, P.st, P.part));  // Q = A P and P . Q
        STK_TRY(fcg_reduce(ctx, P.applyr, P.part, P.sums, P.st, PH_ALPHA));
        // (the Z slot's dtype selects the kernel: OP_UPDATE clears an FP64 Z)
        STK_TRY(vec_op<double>(ctx, P.vec, OP_UPDATE, P.st, P.part, P.vec_z32));
        // stop below tol or at the end of the budget
        if (b->lookahead) {
            // The states go to the host while the rest of the iteration is queued behind
            // them: the GPU does not wait for the host between iterations.  An instance
            // that stopped here is skipped by the Krylov kernels, and its preconditioner
            // output is recomputed before it is used again.
            STK_TRY(fcg_reduce(ctx, P.vec, P.part, P.sums, P.st, PH_NV, b->pin_dev));
            STK_HIP(hipEventRecord(b->ev, ctx->stream));
        } else {
            STK_TRY(fcg_reduce(ctx, P.vec, P.part, P.sums, P.st, PH_NV));
            STK_TRY(read_states(ctx, P, hn));
            if (!take(hn.data())) break;
        }
        STK_TRY(precondition(ctx, P, b->P32, o, true));
        STK_TRY(vec_op<double>(ctx, P.vec, OP_RZ_ZQ, P.st, P.part, P.vec_z32));
        STK_TRY(fcg_reduce(ctx, P.vec, P.part, P.sums, P.st, PH_BETA));
        STK_TRY(vec_op<double>(ctx, P.vec, OP_XPBY, P.st, P.part, P.vec_z32));
        if (b->lookahead) {
            STK_HIP(hipEventSynchronize(b->ev));
            if (!take(b->pin)) break;
        }
    }
    STK_TRY(read_states(ctx, P, h));
    for (int q = 0; q < n; ++q) b->slots[b->members[q]].fs = h[q];
    return STK_OK;
}

}  // namespace
}  // namespace stk

// ============================================================== C ABI ====
extern "C" {

int stk_batch_create(stk_ctx* ctx, stk_solve_mode mode, int max_slots, stk_batch** out) {
    if (!ctx || !out) return set_error(STK_EINVAL, "ctx/out is NULL");
    if (mode != STK_SOLVE_F64 && mode != STK_SOLVE_F32_REFINED) return set_error(STK_EINVAL, "unknown mode");
    if (max_slots < 1) return set_error(STK_EINVAL, "max_slots must be >= 1");
    auto* b = new stk_batch();
    b->ctx = ctx;
    b->mode = mode;
    b->slots.resize(max_slots);
    *out = b;
    return STK_OK;
}

int stk_batch_destroy(stk_batch* b) {
    if (!b) return STK_OK;
    (void)hipSetDevice(b->ctx->device);
    (void)hipStreamSynchronize(b->ctx->stream);
    for (auto& s : b->slots)
        if (s.m) s.m->busy = false;
    free_plan(b->P);
    free_plan(b->P32);
    if (b->pin) (void)hipHostFree(b->pin);
    if (b->ev) (void)hipEventDestroy(b->ev);
    delete b;
    return STK_OK;
}

int stk_batch_add(stk_batch* b, stk_mg* m, double* vx, double* vy, const double* p, const double* fx,
                  const double* fy, double tol, int max_iters, int* slot) {
    if (!b || !m || !slot) return set_error(STK_EINVAL, "batch, mg and slot must be non-NULL");
    if (m->ctx != b->ctx) return set_error(STK_EINVAL, "mg was built on another context");
    if (!vx || !vy || !fx || !fy) return set_error(STK_EINVAL, "vx, vy, fx, fy must be non-NULL");
    if (!(tol > 0.0) || max_iters < 0) return set_error(STK_EINVAL, "tol must be > 0 and max_iters >= 0");
    if (m->busy) return set_error(STK_EINVAL, "mg handle is already solving in a batch");
    if (b->have_opts && !same_smoothing(m->o, b->o))
        return set_error(STK_EINVAL, "mg handle's smoothing options differ from the batch's (nu %d, %d, omega %g)",
                         b->o.nu1, b->o.nu2, b->o.omega);
    int id = -1;
    for (int i = 0; i < (int)b->slots.size() && id < 0; ++i)
        if (b->slots[i].state == SL_FREE) id = i;
    if (id < 0) return set_error(STK_EINVAL, "no free slot (%zu slots)", b->slots.size());
    stk_ctx* ctx = b->ctx;
    STK_TRY(use_device(ctx));
    STK_TRY(ensure_dtype(m, 0));
    if (b->mode == STK_SOLVE_F32_REFINED) STK_TRY(ensure_dtype(m, 1));
    // x0 -> X, f -> F, b = f - G p -> B (FP64, the handle's layout)
    const MgLevel& L = m->L[0];
    stk_grid g{L.nx, L.ny, L.ld, L.dx, L.dy};
    const Field2& X = m->ks[0][VS_X];
    const Field2& B = m->ks[0][VS_B];
    const Field2& F = m->ks[0][VS_F];
    STK_TRY(copy_vel_in(m, vx, vy, m->user_ld, X.x, X.y, L.ld, 8));
    STK_TRY(copy_vel_in(m, fx, fy, m->user_ld, F.x, F.y, L.ld, 8));
    const void* pres = m->zero64;  // p = 0
    void* ptmp = nullptr;
    if (p) {  // the caller's pressure, restrided to the handle's layout
        hipError_t e = hipMalloc(&ptmp, (size_t)L.ny * L.ld * 8);
        if (e != hipSuccess) return set_error(STK_ENOMEM, "pressure staging: %s", hipGetErrorString(e));
        e = hipMemcpy2DAsync(ptmp, L.ld * 8, p, m->user_ld * 8, (size_t)L.nx * 8, L.ny, hipMemcpyDeviceToDevice,
                             ctx->stream);
        if (e != hipSuccess) {
            (void)hipFree(ptmp);
            return hip_fail(e, "copy p");
        }
        pres = ptmp;
    }
    const int rc = launch_fold_rhs(ctx, STK_F64, &g, F.x, F.y, pres, B.x, B.y);
    if (ptmp) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipFree(ptmp);
    }
    if (rc) return rc;
    Slot& s = b->slots[id];
    s = Slot{};
    s.m = m;
    s.ux = vx;
    s.uy = vy;
    s.tol = tol;
    s.max_iters = max_iters;
    s.state = SL_NEW;
    s.fs.tol2 = tol * tol;
    s.t0 = std::chrono::steady_clock::now();
    m->busy = true;
    b->o = m->o;
    b->have_opts = true;
    *slot = id;
    return STK_OK;
}

int stk_batch_step(stk_batch* b, int iters, int* done, stk_report* reps, int* ndone) {
    if (!b || !done || !reps || !ndone) return set_error(STK_EINVAL, "batch, done, reps, ndone must be non-NULL");
    if (iters < 1) return set_error(STK_EINVAL, "iters must be >= 1");
    STK_TRY(use_device(b->ctx));
    *ndone = 0;
    STK_TRY(start_phase(b, done, reps, ndone));
    STK_TRY(iterate_phase(b, iters));
    if (*ndone) STK_HIP(hipStreamSynchronize(b->ctx->stream));
    return STK_OK;
}

int stk_batch_count(const stk_batch* b, int* in_flight) {
    if (!b || !in_flight) return set_error(STK_EINVAL, "batch/in_flight is NULL");
    int c = 0;
    for (const auto& s : b->slots) c += s.state != SL_FREE;
    *in_flight = c;
    return STK_OK;
}

int stk_mg_solve_batch(stk_ctx* ctx, int n, stk_mg* const* mgs, stk_solve_mode mode, double* const* vx,
                       double* const* vy, const double* const* p, const double* const* fx, const double* const* fy,
                       double tol, int max_iters, stk_report* reps) {
    if (!ctx || n < 1 || !mgs || !vx || !vy || !fx || !fy) return set_error(STK_EINVAL, "bad batch arguments");
    for (int q = 0; q < n; ++q)
        for (int r = 0; r < q; ++r)
            if (mgs[r] == mgs[q]) return set_error(STK_EINVAL, "instance %d repeats an mg handle", q);
    stk_batch* b = nullptr;
    STK_TRY(stk_batch_create(ctx, mode, n, &b));
    b->lookahead = true;  // this batch runs alone to the end
    std::vector<stk_report> out(n), got(n);
    std::vector<int> done(n);
    int rc = STK_OK;
    for (int q = 0; q < n && rc == STK_OK; ++q) {
        int slot = -1;
        rc = stk_batch_add(b, mgs[q], vx[q], vy[q], p ? p[q] : nullptr, fx[q], fy[q], tol, max_iters, &slot);
        if (rc != STK_OK) {
            const std::string msg = stk_last_error();
            rc = set_error(rc, "instance %d: %s", q, msg.c_str());
        }
    }
    int left = n;
    while (rc == STK_OK && left > 0) {
        int nd = 0;
        rc = stk_batch_step(b, 1 << 30, done.data(), got.data(), &nd);
        for (int k = 0; k < nd; ++k) out[done[k]] = got[k];  // slots 0..n-1 were taken in order
        left -= nd;
    }
    stk_batch_destroy(b);
    if (rc != STK_OK) return rc;
    int rc_all = STK_OK;
    for (int q = 0; q < n; ++q) {
        if (reps) reps[q] = out[q];
        if (!std::isfinite(out[q].ev)) rc_all = set_error(STK_ENONFINITE, "instance %d: residual not finite", q);
        else if (!out[q].converged && rc_all == STK_OK)
            rc_all = set_error(STK_ENOTCONV, "instance %d: E_v = %.3e > tol", q, out[q].ev);
    }
    return rc_all;
}

int stk_mg_solve(stk_mg* m, stk_solve_mode mode, double* vx, double* vy, const double* p, const double* fx,
                 const double* fy, double tol, int max_iters, stk_report* rep) {
    if (!m) return set_error(STK_EINVAL, "mg is NULL");
    return stk_mg_solve_batch(m->ctx, 1, &m, mode, &vx, &vy, p ? &p : nullptr, &fx, &fy, tol, max_iters, rep);
}

}  // extern "C"
