// Fused damped Jacobi (paper Sec. 4.1, loop fusion: vx and vy of a cell in
// one pass) on the row-streaming engine (rowstream.hpp).
#include "rowstream.hpp"
#include "stk_internal.hpp"

namespace stk {
namespace {

using namespace rows;

template <typename T>
__global__ __launch_bounds__(64 * WPB) void k_jacobi_rows(Grid<T> g, const T* __restrict__ vx,
                                                          const T* __restrict__ vy, T* __restrict__ ox,
                                                          T* __restrict__ oy) {
    const int wv = xcd_tile((int)blockIdx.x, (int)gridDim.x) * WPB + wave_in_group();
    const Place q = place(wv, g.nx, g.ny);
    if (q.y0 >= q.y1) return;  // the whole wave
    const int nx = g.nx, ny = g.ny, i = q.i;
    const Loader<T> L = make_loader<T>(vx, vy, g.ec, g.en, g.bx, g.by, nullptr, g.ld, nx, ny, i);
    const bool xcol = i >= 1 && i <= nx - 1, ycol = i >= 0 && i <= nx - 1;
    const unsigned col = (unsigned)i * (unsigned)sizeof(T);
    const unsigned s_x = q.own ? col : OOB, s_y = (q.own && ycol) ? col : OOB;
    walk_rows<T>(L, q.y0, q.y1, [&](const Row<T>& a, const Row<T>& b, const Row<T>& c, int j) {
        T ux, uy;
        jacobi_row<T>(a, b, c, g.omega, g.idx, g.idy, ux, uy);
        const bool xu = xcol && j <= ny - 1, yu = ycol && j >= 1 && j <= ny - 1;
        store_pair<T>(ox, oy, g.ld, nx, ny, j, xu ? ux : T(0), yu ? uy : T(0), s_x, s_y);
    });
}

}  // namespace

int launch_jacobi_rows(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const FieldPtrs& f, double omega,
                       const void* vx, const void* vy, void* ox, void* oy) {
    const dim3 grid((unsigned)workgroups(g->nx, g->ny)), block(64 * WPB);
    if (dt == STK_F64) {
        Grid<double> gg{static_cast<const double*>(f.eta_c), static_cast<const double*>(f.eta_n),
                        static_cast<const double*>(f.bx), static_cast<const double*>(f.by), g->ld, g->nx, g->ny,
                        1.0 / g->dx, 1.0 / g->dy, omega};
        hipLaunchKernelGGL(k_jacobi_rows<double>, grid, block, 0, ctx->stream, gg, (const double*)vx,
                           (const double*)vy, (double*)ox, (double*)oy);
    } else {
        Grid<float> gg{static_cast<const float*>(f.eta_c), static_cast<const float*>(f.eta_n),
                       static_cast<const float*>(f.bx), static_cast<const float*>(f.by), g->ld, g->nx, g->ny,
                       float(1.0 / g->dx), float(1.0 / g->dy), float(omega)};
        hipLaunchKernelGGL(k_jacobi_rows<float>, grid, block, 0, ctx->stream, gg, (const float*)vx, (const float*)vy,
                           (float*)ox, (float*)oy);
    }
    STK_HIP(hipGetLastError());
    return STK_OK;
}

}  // namespace stk
