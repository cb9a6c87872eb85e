// Setup of the Galerkin coarse operators A_c = P^T A P / 4 (A = -M) as stored
// stencils (each coupling stored once, coarse_stencil.hpp), one level from the
// next finer one.
//
// The paper's multigrid (Sec. 3.2, Sec. 6.2) leaves the coarse operators
// unspecified.  Rediscretised coarse operators (averaged coarse viscosities)
// lose convergence at the viscosity contrasts of the sinker workloads
// (Sec. 6.1, contrast up to 1e8); the Galerkin product keeps the coarse
// correction an A-orthogonal projection at any contrast.
//
// One thread per coarse (I, J) builds the rows of vx(I, J) and vy(I, J):
//   A_c[q, q'] = 1/4 sum_f P[f, q] sum_f' A[f, f'] P[f', q']
// walking the fine support f of P's column q, the fine row of f (the
// viscous stencil on the finest level, the stored stencil below it) and the
// coarse support of P's row f'.  The accumulation order is fixed, so the
// result is deterministic.  Of the full row only the couplings this row
// stores are written; the coarse operator is exactly symmetric because each
// coupling is computed once.  Setup only.
#include "coarse_stencil.hpp"
#include "mg_internal.hpp"

namespace stk {
namespace {

constexpr int GBX = 64, GBY = 4;

// Prolongation weight of coarse index c for fine index f along one axis.
// Normal axis (faces): f even -> f/2 (1); f odd -> (f-1)/2, (f+1)/2 (1/2).
// Tangential axis (rows of cells): own coarse row f/2 gets 3/4, the nearer
// neighbour row (f/2 - 1 for even f, f/2 + 1 for odd f) 1/4; where that
// neighbour is outside [0, nc) (free-slip mirror) the own row gets 1.
__device__ __forceinline__ double pw_normal(int f, int c) {
    if ((f & 1) == 0) return c == (f >> 1) ? 1.0 : 0.0;
    return (c == ((f - 1) >> 1) || c == ((f + 1) >> 1)) ? 0.5 : 0.0;
}
__device__ __forceinline__ double pw_tangent(int f, int nc, int c) {
    const int J = f >> 1, nb = (f & 1) ? J + 1 : J - 1;
    if (nb < 0 || nb >= nc) return c == J ? 1.0 : 0.0;
    return c == J ? 0.75 : (c == nb ? 0.25 : 0.0);
}
// weight of coarse unknown (b, I, J) in the prolongation of fine (b, fi, fj)
__device__ __forceinline__ double pw(int b, int fi, int fj, int I, int J, int NX, int NY) {
    return b == 0 ? pw_normal(fi, I) * pw_tangent(fj, NY, J) : pw_tangent(fi, NX, I) * pw_normal(fj, J);
}

__device__ __forceinline__ bool unknown(int b, int nx, int ny, int i, int j) {
    return b == 0 ? is_vx_unknown(nx, ny, i, j) : is_vy_unknown(nx, ny, i, j);
}

// Up to 9 entries (component, dx, dy, coefficient) of the finest-level row of
// A = -M at unknown (a, i, j): the viscous stencil of the staggered grid.
__device__ int stokes_row(const GalerkinArgs& g, int a, int i, int j, int* cb, int* cdx, int* cdy, double* cv) {
    const int64_t ld = g.ld, k = (int64_t)j * ld + i;
    const int nx = g.nx, ny = g.ny;
    auto enh = [&](int p, int q) { return (p >= 1 && p <= nx - 1 && q >= 1 && q <= ny - 1) ? g.en[(int64_t)q * ld + p] : 0.0; };
    const double x2 = g.idx * g.idx, y2 = g.idy * g.idy, xy = g.idx * g.idy;
    int n = 0;
    auto put = [&](int b, int dx, int dy, double v) {
        cb[n] = b;
        cdx[n] = dx;
        cdy[n] = dy;
        cv[n] = v;
        ++n;
    };
    if (a == 0) {
        const double ecl = g.ec[k - 1], ecr = g.ec[k], enb = enh(i, j), ent = enh(i, j + 1);
        put(0, 0, 0, 2.0 * (ecl + ecr) * x2 + (enb + ent) * y2);
        put(0, -1, 0, -2.0 * ecl * x2);
        put(0, 1, 0, -2.0 * ecr * x2);
        put(0, 0, -1, -enb * y2);
        put(0, 0, 1, -ent * y2);
        put(1, 0, 1, -ent * xy);
        put(1, -1, 1, ent * xy);
        put(1, 0, 0, enb * xy);
        put(1, -1, 0, -enb * xy);
    } else {
        const double ecb = g.ec[k - ld], ect = g.ec[k], enl = enh(i, j), enr = enh(i + 1, j);
        put(1, 0, 0, 2.0 * (ecb + ect) * y2 + (enl + enr) * x2);
        put(1, 0, -1, -2.0 * ecb * y2);
        put(1, 0, 1, -2.0 * ect * y2);
        put(1, -1, 0, -enl * x2);
        put(1, 1, 0, -enr * x2);
        put(0, 1, 0, -enr * xy);
        put(0, 1, -1, enr * xy);
        put(0, 0, 0, enl * xy);
        put(0, 0, -1, -enl * xy);
    }
    return n;
}

template <bool STOKES>
__global__ __launch_bounds__(GBX * GBY) void k_galerkin(GalerkinArgs g) {
    const int I = blockIdx.x * GBX + threadIdx.x % GBX, J = blockIdx.y * GBY + threadIdx.x / GBX;
    const int NX = g.NX, NY = g.NY, nx = g.nx, ny = g.ny;
    if (I > NX || J > NY) return;
    for (int a = 0; a < 2; ++a) {
        if (a == 0 ? J >= NY : I >= NX) continue;
        double acc[NCOEF];
        for (int s = 0; s < NCOEF; ++s) acc[s] = 0.0;
        if (unknown(a, NX, NY, I, J)) {
            // fine support of P's column (a, I, J): 3 along the normal, 4 along the tangent
            const int fi1 = a == 0 ? 2 * I + 1 : 2 * I + 2, fj1 = a == 0 ? 2 * J + 2 : 2 * J + 1;
            for (int fj = 2 * J - 1; fj <= fj1; ++fj)
                for (int fi = 2 * I - 1; fi <= fi1; ++fi) {
                    if (!unknown(a, nx, ny, fi, fj)) continue;
                    const double wf = pw(a, fi, fj, I, J, NX, NY);
                    if (wf == 0.0) continue;
                    int cb[NCOEF], cdx[NCOEF], cdy[NCOEF];
                    double cv[NCOEF];
                    int ne = 0;
                    if (STOKES) {
                        ne = stokes_row(g, a, fi, fj, cb, cdx, cdy, cv);
                    } else {
                        for (int s = 0; s < NCOEF; ++s) {
                            cb[s] = slot_comp(a, s);
                            cdx[s] = slot_dx(a, s);
                            cdy[s] = slot_dy(a, s);
                            cv[s] = stencil_coef<double>(g.fst, g.fplane, g.ld, nx, ny, a, s, fi, fj);
                        }
                        ne = NCOEF;
                    }
                    for (int e = 0; e < ne; ++e) {
                        const int b = cb[e], pi = fi + cdx[e], pj = fj + cdy[e];
                        if (cv[e] == 0.0 || !unknown(b, nx, ny, pi, pj)) continue;
                        const double c = 0.25 * wf * cv[e];
                        // coarse support of P's row (b, pi, pj): at most 2 x 2 coarse indices
                        const int ci0 = (pi - 1) >> 1, cj0 = (pj - 1) >> 1;
                        for (int cj = cj0; cj <= cj0 + 2; ++cj)
                            for (int ci = ci0; ci <= ci0 + 2; ++ci) {
                                if (!unknown(b, NX, NY, ci, cj)) continue;
                                const double wq = pw(b, pi, pj, ci, cj, NX, NY);
                                if (wq == 0.0) continue;
                                const int s = offset_slot(a, b, ci - I, cj - J);
                                if (s >= 0) acc[s] += c * wq;
                            }
                    }
                }
        }
        double* out = g.cst + (int64_t)J * g.cld + I;
        for (int s = 0; s < NCOEF; ++s) {
            const SlotSrc src = slot_src(a, s);
            if (src.own) out[src.plane * g.cplane] = acc[s];
        }
    }
}

}  // namespace

int mg_galerkin(stk_ctx* ctx, const GalerkinArgs& g) {
    const dim3 grid((unsigned)((g.NX + 1 + GBX - 1) / GBX), (unsigned)((g.NY + 1 + GBY - 1) / GBY));
    if (g.fst)
        hipLaunchKernelGGL(k_galerkin<false>, grid, dim3(GBX * GBY), 0, ctx->stream, g);
    else
        hipLaunchKernelGGL(k_galerkin<true>, grid, dim3(GBX * GBY), 0, ctx->stream, g);
    STK_HIP(hipGetLastError());
    return STK_OK;
}

}  // namespace stk
