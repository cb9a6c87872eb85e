// Row-streaming one-sweep stencils for gfx950: fused damped Jacobi (paper
// Sec. 4.1, loop fusion: vx and vy of a cell in one pass).
//
// A wave owns a strip of SW = 62 columns and a segment of SR rows.  Its 64
// lanes hold the columns x0 - 1 .. x0 + 62 (the strip and one neighbour
// column on each side); it walks up the rows, loading each row of every field
// once with coalesced buffer loads, keeps a window of three rows in registers
// and takes the columns i - 1 and i + 1 from the neighbouring lanes (DPP).
// Nothing goes through LDS and waves never wait for each other.
//
// Walls and everything outside the arrays read as 0 through the buffer
// resources (a lane offset past the row for a column outside a field, an
// empty row for a row outside it), so the operands are exactly those of the
// gather kernels and the update, through the same stencil functions, is
// bit-identical.
#include <algorithm>

#include "stencil.hpp"
#include "stk_internal.hpp"
#include "wave.hpp"

namespace stk {
namespace {

constexpr int SW = 62;  // columns a wave updates
constexpr int SR = 64;  // rows a wave walks
constexpr int WPB = 4;  // waves per workgroup (independent)

// One grid row of the six input fields at this lane's column.
template <typename T>
struct Row {
    T vx, vy, ec, en, bx, by;
};

template <typename T>
struct Loader {
    const T *vx, *vy, *ec, *en, *bx, *by;
    int64_t ld;
    int nx, ny;
    // lane offsets: the column, or OOB where the field reads as 0
    unsigned o_vx, o_vy, o_ec, o_en, o_bx, o_by;

    // vx, eta_c, bx live on rows 0..ny-1; vy, eta_n-hat (0 on boundary nodes), by on rows 1..ny-1
    __device__ __forceinline__ Row<T> load(int r) const {
        const size_t w = (size_t)(nx + 1) * sizeof(T);
        const size_t wx = (r >= 0 && r <= ny - 1) ? w : 0, wy = (r >= 1 && r <= ny - 1) ? w : 0;
        const int64_t o = (int64_t)r * ld;
        Row<T> q;
        q.vx = buf_load<T>(buf_rsrc(vx + o, wx), o_vx);
        q.vy = buf_load<T>(buf_rsrc(vy + o, wy), o_vy);
        q.ec = buf_load<T>(buf_rsrc(ec + o, wx), o_ec);
        q.en = buf_load<T>(buf_rsrc(en + o, wy), o_en);
        q.bx = buf_load<T>(buf_rsrc(bx + o, wx), o_bx);
        q.by = buf_load<T>(buf_rsrc(by + o, wy), o_by);
        return q;
    }
};

template <typename T>
__device__ __forceinline__ Loader<T> make_loader(const Grid<T>& g, const T* vx, const T* vy, int i) {
    const int nx = g.nx;
    const unsigned col = (unsigned)i * (unsigned)sizeof(T);
    const bool inner = i >= 1 && i <= nx - 1, cell = i >= 0 && i <= nx - 1;
    Loader<T> L{vx, vy, g.ec, g.en, g.bx, g.by, g.ld, g.nx, g.ny,
                inner ? col : OOB, cell ? col : OOB, cell ? col : OOB, inner ? col : OOB, inner ? col : OOB,
                cell ? col : OOB};
    return L;
}

// Damped Jacobi at row j of this lane's column from rows a = j-1, b = j,
// c = j+1; writes vx(i, j) and vy(i, j) (0 where they are walls).
template <typename T>
__device__ __forceinline__ void jacobi_row(const Grid<T>& g, T* __restrict__ ox, T* __restrict__ oy, const Row<T>& a,
                                           const Row<T>& b, const Row<T>& c, int j, bool xcol, bool ycol,
                                           unsigned s_ox, unsigned s_oy) {
    const T vxl = wave_shift<DPP_FROM_PREV>(b.vx), vxr = wave_shift<DPP_FROM_NEXT>(b.vx);
    const T vyl = wave_shift<DPP_FROM_PREV>(b.vy), vyr = wave_shift<DPP_FROM_NEXT>(b.vy);
    const T vytl = wave_shift<DPP_FROM_PREV>(c.vy);  // vy(i-1, j+1)
    const T vxrb = wave_shift<DPP_FROM_NEXT>(a.vx);  // vx(i+1, j-1)
    const T ecl = wave_shift<DPP_FROM_PREV>(b.ec), enr = wave_shift<DPP_FROM_NEXT>(b.en);
    const T ux = jac_vx<T>(b.vx, vxl, vxr, a.vx, c.vx, b.vy, vyl, c.vy, vytl, ecl, b.ec, b.en, c.en, b.bx, g.omega,
                           g.idx, g.idy);
    const T uy = jac_vy<T>(b.vy, vyl, vyr, a.vy, c.vy, b.vx, vxr, a.vx, vxrb, a.ec, b.ec, b.en, enr, b.by, g.omega,
                           g.idx, g.idy);
    const int nx = g.nx, ny = g.ny;
    const bool xu = xcol && j >= 0 && j <= ny - 1, yu = ycol && j >= 1 && j <= ny - 1;
    const int64_t o = (int64_t)j * g.ld;
    // vx has rows 0..ny-1 and columns 0..nx; vy rows 0..ny and columns 0..nx-1
    buf_store(xu ? ux : T(0), buf_rsrc(ox + o, j <= ny - 1 ? (size_t)(nx + 1) * sizeof(T) : 0), s_ox);
    buf_store(yu ? uy : T(0), buf_rsrc(oy + o, j <= ny ? (size_t)nx * sizeof(T) : 0), s_oy);
}

template <typename T>
__global__ __launch_bounds__(64 * WPB) void k_jacobi_rows(Grid<T> g, const T* __restrict__ vx,
                                                          const T* __restrict__ vy, T* __restrict__ ox,
                                                          T* __restrict__ oy, int nstrip, int nseg) {
    const int nwg = (int)gridDim.x;
    const int wv = xcd_tile((int)blockIdx.x, nwg) * WPB + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int strip = wv % nstrip, seg = wv / nstrip;
    if (seg >= nseg) return;  // the whole wave
    const int nx = g.nx, ny = g.ny;
    const int i = strip * SW - 1 + lane;
    const int y0 = seg * SR, y1 = std::min(y0 + SR, ny + 1);
    const Loader<T> L = make_loader<T>(g, vx, vy, i);
    const bool upd = lane >= 1 && lane <= SW;
    const bool xcol = i >= 1 && i <= nx - 1, ycol = i >= 0 && i <= nx - 1;
    const unsigned col = (unsigned)i * (unsigned)sizeof(T);
    const unsigned s_ox = (upd && i >= 0 && i <= nx) ? col : OOB, s_oy = (upd && ycol) ? col : OOB;

    Row<T> r0 = L.load(y0 - 1), r1 = L.load(y0), r2 = L.load(y0 + 1), r3;
    // four rows per trip so that the window rotates by renaming; the row two
    // ahead is loaded while the current one is computed
    for (int j = y0; j < y1; j += 4) {
        r3 = L.load(j + 2);
        jacobi_row<T>(g, ox, oy, r0, r1, r2, j, xcol, ycol, s_ox, s_oy);
        if (j + 1 >= y1) break;
        r0 = L.load(j + 3);
        jacobi_row<T>(g, ox, oy, r1, r2, r3, j + 1, xcol, ycol, s_ox, s_oy);
        if (j + 2 >= y1) break;
        r1 = L.load(j + 4);
        jacobi_row<T>(g, ox, oy, r2, r3, r0, j + 2, xcol, ycol, s_ox, s_oy);
        if (j + 3 >= y1) break;
        r2 = L.load(j + 5);
        jacobi_row<T>(g, ox, oy, r3, r0, r1, j + 3, xcol, ycol, s_ox, s_oy);
    }
}

}  // namespace

int launch_jacobi_rows(stk_ctx* ctx, stk_dtype dt, const stk_grid* g, const FieldPtrs& f, double omega,
                       const void* vx, const void* vy, void* ox, void* oy) {
    const int nstrip = (g->nx + 1 + SW - 1) / SW, nseg = (g->ny + 1 + SR - 1) / SR;
    const int64_t waves = (int64_t)nstrip * nseg;
    const dim3 grid((unsigned)((waves + WPB - 1) / WPB)), block(64 * WPB);
    if (dt == STK_F64) {
        Grid<double> gg{static_cast<const double*>(f.eta_c), static_cast<const double*>(f.eta_n),
                        static_cast<const double*>(f.bx), static_cast<const double*>(f.by), g->ld, g->nx, g->ny,
                        1.0 / g->dx, 1.0 / g->dy, omega};
        hipLaunchKernelGGL(k_jacobi_rows<double>, grid, block, 0, ctx->stream, gg, (const double*)vx,
                           (const double*)vy, (double*)ox, (double*)oy, nstrip, nseg);
    } else {
        Grid<float> gg{static_cast<const float*>(f.eta_c), static_cast<const float*>(f.eta_n),
                       static_cast<const float*>(f.bx), static_cast<const float*>(f.by), g->ld, g->nx, g->ny,
                       float(1.0 / g->dx), float(1.0 / g->dy), float(omega)};
        hipLaunchKernelGGL(k_jacobi_rows<float>, grid, block, 0, ctx->stream, gg, (const float*)vx,
                           (const float*)vy, (float*)ox, (float*)oy, nstrip, nseg);
    }
    STK_HIP(hipGetLastError());
    return STK_OK;
}

}  // namespace stk
