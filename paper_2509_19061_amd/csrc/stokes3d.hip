// The 3D extension of the smoother (the paper's future work, Sec. 9): the
// staggered variable-viscosity operator in three dimensions, damped Jacobi,
// RAS-type temporal blocking of 3D tiles ("4D blocking": three space
// dimensions and the inner sweeps, Alg. 2 with snapshot semantics), the
// residual and the velocity energy norm (Sec. 6.4).
//
// Layout: every field is a plane-major array with one row stride ld and one
// plane stride lp (elements); element (i, j, k) at base[k lp + j ld + i].
// vx: nz x ny x (nx+1), vy: nz x (ny+1) x nx, vz: (nz+1) x ny x nx, eta_c:
// cells, eta_xy / eta_xz / eta_yz: the z-, y- and x-parallel edges.
//
// Stencil (the 2D formulas of Sec. 2.1 axis by axis): normal stresses
// 2 eta_c dv/dn per cell, shear stresses eta_e (dvx/dy + dvy/dx) etc. per
// interior edge (0 on boundary edges: free slip), centred divergences; the
// wall values of the normal velocity are 0.  Jacobi: v' = v - (omega/d)(b - Mv),
// d = diag(-M).
//
// Kernels:
//   k_jacobi3d   one thread per (i, j, k), gathers from global memory; every
//                smoother and the residual call the same row functions, so
//                RAS with an overlap >= k - 1 is bit-identical to k Jacobi
//                sweeps.
//   k_jacobi3d_z the same sweep with the velocity staged plane by plane: a
//                64 x 4 workgroup walks up a segment of z-planes with a ring
//                of four planes (the planes k - 1, k, k + 1 it reads, and
//                k + 2, loaded meanwhile) of the three components in LDS,
//                halo included; the coefficients come from global memory,
//                addressed by one 32-bit offset per plane.  Same operands,
//                same row arithmetic: the same values as k_jacobi3d, which
//                serves the arrays beyond 2^32 bytes.
//   k_ras3d      one workgroup per T^3 tile: the tile grown by h plus the
//                one-cell frozen ring is staged in LDS (three components,
//                two buffers), k sweeps run there with a barrier between
//                sweeps, the owned unknowns are written back; coefficients
//                and right-hand side come from global memory (L2).
//   k_energy3d   per-workgroup FP64 sums of r^2/d and f^2/d, summed in a
//                fixed order by a second kernel (reproducible).
#include <algorithm>
#include <cmath>
#include <vector>

#include "stencil.hpp"
#include "stk_internal.hpp"
#include "wave.hpp"

namespace stk {
namespace {

template <typename T>
struct Fields3 {
    const T *ec, *exy, *exz, *eyz;  // viscosities
    const T *bx, *by, *bz;          // right-hand side
    int64_t ld, lp;
    int nx, ny, nz;
    T idx, idy, idz;
};

template <typename T>
__device__ __forceinline__ int64_t at3(const Fields3<T>& f, int i, int j, int k) {
    return (int64_t)k * f.lp + (int64_t)j * f.ld + i;
}
__device__ __forceinline__ bool vx_unknown3(int nx, int ny, int nz, int i, int j, int k) {
    return i >= 1 && i <= nx - 1 && j >= 0 && j < ny && k >= 0 && k < nz;
}
__device__ __forceinline__ bool vy_unknown3(int nx, int ny, int nz, int i, int j, int k) {
    return j >= 1 && j <= ny - 1 && i >= 0 && i < nx && k >= 0 && k < nz;
}
__device__ __forceinline__ bool vz_unknown3(int nx, int ny, int nz, int i, int j, int k) {
    return k >= 1 && k <= nz - 1 && i >= 0 && i < nx && j >= 0 && j < ny;
}
// edge viscosities, 0 on boundary edges.  In FP64 the load itself is
// unconditional, from the index clamped onto the array, and its value dropped
// off the inner edges, so no load waits under a branch for the one before it
// (256^3 fused sweep 30.3 -> 32.2 GLUP/s); in FP32 that form was slower
// (51.3 -> 48.3), so FP32 loads under the branch.  The same values either way.
template <typename T>
__device__ __forceinline__ T edge3(const Fields3<T>& f, const T* __restrict__ e, bool in, int i, int j, int k) {
    if constexpr (sizeof(T) == 8) {
        const T a = e[at3(f, min(max(i, 0), f.nx), min(max(j, 0), f.ny), min(max(k, 0), f.nz))];
        return in ? a : T(0);
    } else {
        return in ? e[at3(f, i, j, k)] : T(0);
    }
}
template <typename T>
__device__ __forceinline__ T exy3(const Fields3<T>& f, int i, int j, int k) {
    return edge3(f, f.exy, i >= 1 && i <= f.nx - 1 && j >= 1 && j <= f.ny - 1, i, j, k);
}
template <typename T>
__device__ __forceinline__ T exz3(const Fields3<T>& f, int i, int j, int k) {
    return edge3(f, f.exz, i >= 1 && i <= f.nx - 1 && k >= 1 && k <= f.nz - 1, i, j, k);
}
template <typename T>
__device__ __forceinline__ T eyz3(const Fields3<T>& f, int i, int j, int k) {
    return edge3(f, f.eyz, j >= 1 && j <= f.ny - 1 && k >= 1 && k <= f.nz - 1, i, j, k);
}

// Velocity values by a loader V(c, i, j, k) (c: 0 vx, 1 vy, 2 vz) that
// returns 0 for walls and anything outside the arrays.  The row functions
// return (M v) at the unknown and the diagonal d = diag(-M).
//
// The coefficients of one row come in a Row3: the cell viscosities behind and
// ahead of the face along its own axis (e0, e1), and the edge viscosities
// behind and ahead along each of the two other axes, in x, y, z order
// (s0, s1, t0, t1), boundary edges already 0.  The gathering forms below
// (mvx3, ...) load them through Fields3; the plane-streaming sweep loads
// them its own way and calls the same arithmetic (mvx3c, ...).
template <typename T>
struct Row3 {
    T e0, e1, s0, s1, t0, t1;
};
template <typename T, typename V>
__device__ __forceinline__ T mvx3c(const Fields3<T>& f, const V& v, int i, int j, int k, const Row3<T>& w, T& d) {
    const T c = v(0, i, j, k);
    const T e0 = w.e0, e1 = w.e1, s0 = w.s0, s1 = w.s1, t0 = w.t0, t1 = w.t1;
    const T txx1 = T(2) * e1 * (v(0, i + 1, j, k) - c) * f.idx, txx0 = T(2) * e0 * (c - v(0, i - 1, j, k)) * f.idx;
    const T txy1 = s1 * ((v(0, i, j + 1, k) - c) * f.idy + (v(1, i, j + 1, k) - v(1, i - 1, j + 1, k)) * f.idx);
    const T txy0 = s0 * ((c - v(0, i, j - 1, k)) * f.idy + (v(1, i, j, k) - v(1, i - 1, j, k)) * f.idx);
    const T txz1 = t1 * ((v(0, i, j, k + 1) - c) * f.idz + (v(2, i, j, k + 1) - v(2, i - 1, j, k + 1)) * f.idx);
    const T txz0 = t0 * ((c - v(0, i, j, k - 1)) * f.idz + (v(2, i, j, k) - v(2, i - 1, j, k)) * f.idx);
    d = T(2) * (e0 + e1) * f.idx * f.idx + (s0 + s1) * f.idy * f.idy + (t0 + t1) * f.idz * f.idz;
    return (txx1 - txx0) * f.idx + (txy1 - txy0) * f.idy + (txz1 - txz0) * f.idz;
}
template <typename T, typename V>
__device__ __forceinline__ T mvy3c(const Fields3<T>& f, const V& v, int i, int j, int k, const Row3<T>& w, T& d) {
    const T c = v(1, i, j, k);
    const T e0 = w.e0, e1 = w.e1, s0 = w.s0, s1 = w.s1, t0 = w.t0, t1 = w.t1;
    const T tyy1 = T(2) * e1 * (v(1, i, j + 1, k) - c) * f.idy, tyy0 = T(2) * e0 * (c - v(1, i, j - 1, k)) * f.idy;
    const T txy1 = s1 * ((v(0, i + 1, j, k) - v(0, i + 1, j - 1, k)) * f.idy + (v(1, i + 1, j, k) - c) * f.idx);
    const T txy0 = s0 * ((v(0, i, j, k) - v(0, i, j - 1, k)) * f.idy + (c - v(1, i - 1, j, k)) * f.idx);
    const T tyz1 = t1 * ((v(1, i, j, k + 1) - c) * f.idz + (v(2, i, j, k + 1) - v(2, i, j - 1, k + 1)) * f.idy);
    const T tyz0 = t0 * ((c - v(1, i, j, k - 1)) * f.idz + (v(2, i, j, k) - v(2, i, j - 1, k)) * f.idy);
    d = T(2) * (e0 + e1) * f.idy * f.idy + (s0 + s1) * f.idx * f.idx + (t0 + t1) * f.idz * f.idz;
    return (tyy1 - tyy0) * f.idy + (txy1 - txy0) * f.idx + (tyz1 - tyz0) * f.idz;
}
template <typename T, typename V>
__device__ __forceinline__ T mvz3c(const Fields3<T>& f, const V& v, int i, int j, int k, const Row3<T>& w, T& d) {
    const T c = v(2, i, j, k);
    const T e0 = w.e0, e1 = w.e1, s0 = w.s0, s1 = w.s1, t0 = w.t0, t1 = w.t1;
    const T tzz1 = T(2) * e1 * (v(2, i, j, k + 1) - c) * f.idz, tzz0 = T(2) * e0 * (c - v(2, i, j, k - 1)) * f.idz;
    const T txz1 = s1 * ((v(0, i + 1, j, k) - v(0, i + 1, j, k - 1)) * f.idz + (v(2, i + 1, j, k) - c) * f.idx);
    const T txz0 = s0 * ((v(0, i, j, k) - v(0, i, j, k - 1)) * f.idz + (c - v(2, i - 1, j, k)) * f.idx);
    const T tyz1 = t1 * ((v(1, i, j + 1, k) - v(1, i, j + 1, k - 1)) * f.idz + (v(2, i, j + 1, k) - c) * f.idy);
    const T tyz0 = t0 * ((v(1, i, j, k) - v(1, i, j, k - 1)) * f.idz + (c - v(2, i, j - 1, k)) * f.idy);
    d = T(2) * (e0 + e1) * f.idz * f.idz + (s0 + s1) * f.idx * f.idx + (t0 + t1) * f.idy * f.idy;
    return (tzz1 - tzz0) * f.idz + (txz1 - txz0) * f.idx + (tyz1 - tyz0) * f.idy;
}
template <typename T, typename V>
__device__ __forceinline__ T mvx3(const Fields3<T>& f, const V& v, int i, int j, int k, T& d) {
    const Row3<T> w{f.ec[at3(f, i - 1, j, k)], f.ec[at3(f, i, j, k)], exy3(f, i, j, k), exy3(f, i, j + 1, k),
                    exz3(f, i, j, k), exz3(f, i, j, k + 1)};
    return mvx3c(f, v, i, j, k, w, d);
}
template <typename T, typename V>
__device__ __forceinline__ T mvy3(const Fields3<T>& f, const V& v, int i, int j, int k, T& d) {
    const Row3<T> w{f.ec[at3(f, i, j - 1, k)], f.ec[at3(f, i, j, k)], exy3(f, i, j, k), exy3(f, i + 1, j, k),
                    eyz3(f, i, j, k), eyz3(f, i, j, k + 1)};
    return mvy3c(f, v, i, j, k, w, d);
}
template <typename T, typename V>
__device__ __forceinline__ T mvz3(const Fields3<T>& f, const V& v, int i, int j, int k, T& d) {
    const Row3<T> w{f.ec[at3(f, i, j, k - 1)], f.ec[at3(f, i, j, k)], exz3(f, i, j, k), exz3(f, i + 1, j, k),
                    eyz3(f, i, j, k), eyz3(f, i, j + 1, k)};
    return mvz3c(f, v, i, j, k, w, d);
}

// Loader of the global velocity arrays: walls and outside read as 0.
template <typename T>
struct GlobalV {
    const T *x, *y, *z;
    int64_t ld, lp;
    int nx, ny, nz;
    __device__ __forceinline__ T operator()(int c, int i, int j, int k) const {
        const int64_t q = (int64_t)k * lp + (int64_t)j * ld + i;
        if (c == 0) return vx_unknown3(nx, ny, nz, i, j, k) ? x[q] : T(0);
        if (c == 1) return vy_unknown3(nx, ny, nz, i, j, k) ? y[q] : T(0);
        return vz_unknown3(nx, ny, nz, i, j, k) ? z[q] : T(0);
    }
};

// ----------------------------------------------------------- Jacobi (3D) --
constexpr int J3X = 64, J3Y = 4;

template <typename T>
__global__ __launch_bounds__(J3X* J3Y) void k_jacobi3d(Fields3<T> f, T omega, const T* __restrict__ vx,
                                                        const T* __restrict__ vy, const T* __restrict__ vz,
                                                        T* __restrict__ ox, T* __restrict__ oy, T* __restrict__ oz) {
    const int i = blockIdx.x * J3X + threadIdx.x, j = blockIdx.y * J3Y + threadIdx.y, k = blockIdx.z;
    const int nx = f.nx, ny = f.ny, nz = f.nz;
    if (i > nx || j > ny || k > nz) return;
    const GlobalV<T> v{vx, vy, vz, f.ld, f.lp, nx, ny, nz};
    const int64_t q = at3(f, i, j, k);
    T d;
    if (k < nz && j < ny) {
        T o = T(0);
        if (vx_unknown3(nx, ny, nz, i, j, k)) {
            const T m = mvx3<T>(f, v, i, j, k, d);
            o = jac_step<T>(vx[q], omega / d, f.bx[q], m);
        }
        ox[q] = o;
    }
    if (k < nz && i < nx) {
        T o = T(0);
        if (vy_unknown3(nx, ny, nz, i, j, k)) {
            const T m = mvy3<T>(f, v, i, j, k, d);
            o = jac_step<T>(vy[q], omega / d, f.by[q], m);
        }
        oy[q] = o;
    }
    if (j < ny && i < nx) {
        T o = T(0);
        if (vz_unknown3(nx, ny, nz, i, j, k)) {
            const T m = mvz3<T>(f, v, i, j, k, d);
            o = jac_step<T>(vz[q], omega / d, f.bz[q], m);
        }
        oz[q] = o;
    }
}

// --------------------------------------------- Jacobi (3D), plane streaming --
// A 64 x 4 workgroup owns the cells [i0, i0 + 64) x [j0, j0 + 4) of a segment
// of up to 32 planes and walks up it.  The three velocity components of the
// window (the tile plus one halo cell on each side) live in an LDS ring of
// four planes: k - 1, k, k + 1 are read while plane k is relaxed and k + 2 is
// loaded into registers meanwhile.  The walls beyond the last cell, vx(nx),
// vy(ny) and vz(nz), are written by the threads of the cells below them, so
// no workgroup exists for them alone.
//
// Everything that depends on the thread but not on the plane is computed once:
// the window cells it loads and whether each holds an unknown, and the
// boundary tests of its edge viscosities.  Within a plane every address is one
// 32-bit byte offset from a uniform base (the host keeps the arrays within
// 2^32 bytes), and every load is made unconditionally from a place on the
// arrays and its value dropped where it does not count, so no load waits under
// a branch.  Same operands and same row arithmetic as the gathering kernel.
constexpr int ZX = 64, ZY = 4, ZS = 32;               // tile columns, rows, planes per segment
constexpr int ZNT = ZX * ZY;
constexpr int ZWX = ZX + 2, ZWY = ZY + 2;              // staged window (one halo cell each side)
constexpr int ZPL = ZWX * ZWY;                         // window cells of one component and plane
constexpr int ZSLOT = 3 * ZPL;                         // one ring slot: three components
static_assert(ZPL > ZNT && ZPL <= 2 * ZNT, "two window loads per thread and component");

// Velocity loader of the staged ring: (c, i, j, k) -> the window cell, for
// i0 - 1 <= i <= i0 + 64, j0 - 1 <= j <= j0 + 4 and any of the three planes
// in the ring.
template <typename T>
struct RingV {
    const T* w;
    int i0, j0;
    __device__ __forceinline__ T operator()(int c, int i, int j, int k) const {
        return w[(k & 3) * ZSLOT + c * ZPL + (j - j0 + 1) * ZWX + (i - i0 + 1)];
    }
};

template <typename T>
__device__ __forceinline__ T at_b(const T* __restrict__ base, uint32_t off) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off);
}
template <typename T>
__device__ __forceinline__ void put_b(T* __restrict__ base, uint32_t off, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + off) = v;
}

// The window cells of one thread: cell e = tid + 256 m of each component's
// window plane (m = 0, 1; the second only for e < ZPL), its byte offset within
// a plane (clamped onto the array where the cell is outside it) and whether it
// holds an unknown of vx, vy, vz in that plane's rows and columns.
struct ZWin {
    uint32_t off[2];
    bool x[2], y[2], z[2];
};

template <typename T>
__device__ __forceinline__ void zwin_load(const ZWin& w, const T* __restrict__ vx, const T* __restrict__ vy,
                                          const T* __restrict__ vz, uint32_t pb, bool kxy, bool kz,
                                          T (&r)[2][3]) {
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const T a = at_b(vx, w.off[m] + pb), b = at_b(vy, w.off[m] + pb), c = at_b(vz, w.off[m] + pb);
        r[m][0] = w.x[m] && kxy ? a : T(0);
        r[m][1] = w.y[m] && kxy ? b : T(0);
        r[m][2] = w.z[m] && kz ? c : T(0);
    }
}
template <typename T>
__device__ __forceinline__ void zwin_store(T* ring, int k, const T (&r)[2][3]) {
    T* s = ring + (k & 3) * ZSLOT + threadIdx.x;
#pragma unroll
    for (int c = 0; c < 3; ++c) s[c * ZPL] = r[0][c];
    if (threadIdx.x + ZNT < ZPL) {
#pragma unroll
        for (int c = 0; c < 3; ++c) s[c * ZPL + ZNT] = r[1][c];
    }
}

// The coefficients of the thread's cell (i, j) in one plane k, raw (boundary
// edges not yet dropped): eta_c at the cell and behind it along x, y, z;
// eta_xy at (i, j), (i, j + 1), (i + 1, j); eta_xz at (i, k), (i, k + 1),
// (i + 1, k); eta_yz at (j, k), (j, k + 1), (j + 1, k); b.  The loader
// fetches all but ecz, b0 and c0, which the plane below already had.
template <typename T>
struct Coef3 {
    T ec, ecx, ecy, ecz, a0, a1, a2, b0, b1, b2, c0, c1, c2, bx, by, bz;
};
template <typename T>
__device__ __forceinline__ Coef3<T> coef3_load(const Fields3<T>& f, uint32_t q, uint32_t dxm, uint32_t dym,
                                               uint32_t sld, uint32_t slp) {
    constexpr uint32_t es = sizeof(T);
    Coef3<T> c;
    c.ec = at_b(f.ec, q);
    c.ecx = at_b(f.ec, q - dxm);
    c.ecy = at_b(f.ec, q - dym);
    c.a0 = at_b(f.exy, q);
    c.a1 = at_b(f.exy, q + sld);
    c.a2 = at_b(f.exy, q + es);
    c.b1 = at_b(f.exz, q + slp);
    c.b2 = at_b(f.exz, q + es);
    c.c1 = at_b(f.eyz, q + slp);
    c.c2 = at_b(f.eyz, q + sld);
    c.bx = at_b(f.bx, q);
    c.by = at_b(f.by, q);
    c.bz = at_b(f.bz, q);
    return c;
}

template <typename T>
__global__ __launch_bounds__(ZNT) void k_jacobi3d_z(Fields3<T> f, T omega, const T* __restrict__ vx,
                                                     const T* __restrict__ vy, const T* __restrict__ vz,
                                                     T* __restrict__ ox, T* __restrict__ oy, T* __restrict__ oz,
                                                     int ntx, int nty) {
    __shared__ T ring[4 * ZSLOT];
    const int nx = f.nx, ny = f.ny, nz = f.nz;
    // tiles numbered x fastest, then y, then z segments, renumbered by XCD
    const int t = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    const int tx = t % ntx, ty = (t / ntx) % nty, tz = t / (ntx * nty);
    const int i0 = tx * ZX, j0 = ty * ZY, k0 = tz * ZS, k1 = min(k0 + ZS, nz);
    const int i = i0 + (int)(threadIdx.x % ZX), j = j0 + (int)(threadIdx.x / ZX);
    const bool act = i < nx && j < ny;
    const int ic = min(i, nx - 1), jc = min(j, ny - 1);  // inactive threads load from the last cell
    constexpr uint32_t es = sizeof(T);
    const uint32_t sld = (uint32_t)f.ld * es, slp = (uint32_t)f.lp * es;

    ZWin w;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int e = (int)threadIdx.x + m * ZNT, wy = e / ZWX, wx = e - wy * ZWX;
        const int gi = i0 - 1 + wx, gj = j0 - 1 + wy;
        const bool in = e < ZPL, ix = gi >= 0 && gi < nx, jy = gj >= 0 && gj < ny;
        w.off[m] = ((uint32_t)min(max(gj, 0), ny) * (uint32_t)f.ld + (uint32_t)min(max(gi, 0), nx)) * es;
        w.x[m] = in && gi >= 1 && gi <= nx - 1 && jy;
        w.y[m] = in && ix && gj >= 1 && gj <= ny - 1;
        w.z[m] = in && ix && jy;
    }
    // plane kk of the window: clamped onto the array, dropped outside the unknowns
    auto load = [&](int kk, T(&r)[2][3]) {
        zwin_load<T>(w, vx, vy, vz, (uint32_t)min(max(kk, 0), nz) * slp, kk >= 0 && kk < nz, kk >= 1 && kk < nz, r);
    };
    T r[2][3];
    load(k0 - 1, r);
    zwin_store<T>(ring, k0 - 1, r);
    load(k0, r);
    zwin_store<T>(ring, k0, r);
    load(k0 + 1, r);
    zwin_store<T>(ring, k0 + 1, r);
    __syncthreads();

    // boundary tests of the edges around the thread's cell (x and y parts)
    const bool xi0 = ic >= 1, xi1 = ic <= nx - 2, yj0 = jc >= 1, yj1 = jc <= ny - 2;
    const uint32_t dxm = xi0 ? es : 0u, dym = yj0 ? sld : 0u;  // the cell behind, or the cell itself at a wall
    uint32_t q = (uint32_t)k0 * slp + (uint32_t)jc * sld + (uint32_t)ic * es;
    // the coefficients of plane k0; those of plane k + 1 are loaded during
    // step k, and the three that planes k and k + 1 share are carried
    Coef3<T> c = coef3_load<T>(f, q, dxm, dym, sld, slp);
    c.ecz = at_b(f.ec, q - (k0 >= 1 ? slp : 0u));
    c.b0 = at_b(f.exz, q);
    c.c0 = at_b(f.eyz, q);
    const RingV<T> v{ring, i0, j0};
    for (int k = k0; k < k1; ++k, q += slp) {
        load(k + 2, r);  // in flight while plane k is relaxed
        Coef3<T> n = coef3_load<T>(f, k + 1 < k1 ? q + slp : q, dxm, dym, sld, slp);
        n.ecz = c.ec;
        n.b0 = c.b1;
        n.c0 = c.c1;
        const bool kz0 = k >= 1, kz1 = k <= nz - 2;
        const T sxy = xi0 && yj0 ? c.a0 : T(0), sxy_y = xi0 && yj1 ? c.a1 : T(0), sxy_x = xi1 && yj0 ? c.a2 : T(0);
        const T sxz = xi0 && kz0 ? c.b0 : T(0), sxz_z = xi0 && kz1 ? c.b1 : T(0), sxz_x = xi1 && kz0 ? c.b2 : T(0);
        const T syz = yj0 && kz0 ? c.c0 : T(0), syz_z = yj0 && kz1 ? c.c1 : T(0), syz_y = yj1 && kz0 ? c.c2 : T(0);
        T d;
        const T mx = mvx3c<T>(f, v, i, j, k, Row3<T>{c.ecx, c.ec, sxy, sxy_y, sxz, sxz_z}, d);
        const T nvx = jac_step<T>(v(0, i, j, k), omega / d, c.bx, mx);
        const T my = mvy3c<T>(f, v, i, j, k, Row3<T>{c.ecy, c.ec, sxy, sxy_x, syz, syz_z}, d);
        const T nvy = jac_step<T>(v(1, i, j, k), omega / d, c.by, my);
        const T mz = mvz3c<T>(f, v, i, j, k, Row3<T>{c.ecz, c.ec, sxz, sxz_x, syz, syz_y}, d);
        const T nvz = jac_step<T>(v(2, i, j, k), omega / d, c.bz, mz);
        if (act) {
            put_b(ox, q, xi0 ? nvx : T(0));  // vx(0) is a wall
            put_b(oy, q, yj0 ? nvy : T(0));  // vy(0)
            put_b(oz, q, kz0 ? nvz : T(0));  // vz(0)
            if (i == nx - 1) put_b(ox, q + es, T(0));
            if (j == ny - 1) put_b(oy, q + sld, T(0));
            if (k == nz - 1) put_b(oz, q + slp, T(0));
        }
        c = n;
        // slot (k + 2) & 3 held plane k - 2, last read in the previous step
        zwin_store<T>(ring, k + 2, r);
        __syncthreads();
    }
}

// ------------------------------------------------------------- RAS (3D) --
constexpr int R3NT = 512;

// LDS window of one tile: cells (i, j, k) in [X0 - 1, X1] x [Y0 - 1, Y1] x
// [Z0 - 1, Z1] (the region E plus the frozen ring; the upper index X1 also
// holds the right wall vx(nx) when E reaches it), three components, two
// buffers.  Window extent per axis: E + 2 <= T + 2h + 2.
template <typename T>
struct WinV {
    const T* w;  // buffer: component c at w + c * cs
    int cs, wx, wy;  // component stride, row and plane extents
    int x0, y0, z0;  // window origin (cell indices)
    __device__ __forceinline__ T operator()(int c, int i, int j, int k) const {
        return w[c * cs + ((k - z0) * wy + (j - y0)) * wx + (i - x0)];
    }
};

template <typename T>
__global__ __launch_bounds__(R3NT) void k_ras3d(Fields3<T> f, T omega, const T* __restrict__ vx,
                                                 const T* __restrict__ vy, const T* __restrict__ vz,
                                                 T* __restrict__ ox, T* __restrict__ oy, T* __restrict__ oz, int tile,
                                                 int h, int kt, int sx, int sy, int sz, int wmax) {
    extern __shared__ unsigned char smem_raw[];
    T* lds = reinterpret_cast<T*>(smem_raw);
    const int nx = f.nx, ny = f.ny, nz = f.nz;
    // tile (bx, by, bz): owned cells between the cuts s + (b - 1) T and s + b T, clipped
    const int x0 = max(0, sx + ((int)blockIdx.x - 1) * tile), x1 = min(nx, sx + (int)blockIdx.x * tile);
    const int y0 = max(0, sy + ((int)blockIdx.y - 1) * tile), y1 = min(ny, sy + (int)blockIdx.y * tile);
    const int z0 = max(0, sz + ((int)blockIdx.z - 1) * tile), z1 = min(nz, sz + (int)blockIdx.z * tile);
    if (x0 >= x1 || y0 >= y1 || z0 >= z1) return;  // empty tile: the whole workgroup leaves
    const int X0 = max(x0 - h, 0), X1 = min(x1 + h, nx), Y0 = max(y0 - h, 0), Y1 = min(y1 + h, ny);
    const int Z0 = max(z0 - h, 0), Z1 = min(z1 + h, nz);
    const int wx = X1 - X0 + 2, wy = Y1 - Y0 + 2, wz = Z1 - Z0 + 2;
    const int cs = wmax * wmax * wmax;  // component stride; a buffer is 3 cs
    const GlobalV<T> g{vx, vy, vz, f.ld, f.lp, nx, ny, nz};
    const int ncell = wx * wy * wz;
    for (int e = threadIdx.x; e < ncell; e += R3NT) {
        const int ci = e % wx, cj = (e / wx) % wy, ck = e / (wx * wy);
        const int i = X0 - 1 + ci, j = Y0 - 1 + cj, k = Z0 - 1 + ck;
        for (int c = 0; c < 3; ++c) {
            const T val = g(c, i, j, k);
            lds[c * cs + e] = val;
            lds[3 * cs + c * cs + e] = val;
        }
    }
    __syncthreads();
    // unknowns of E: the three faces owned by each cell of E
    const int ew = X1 - X0, eh = Y1 - Y0, ed = Z1 - Z0, ne = ew * eh * ed;
    for (int s = 0; s < kt; ++s) {
        const T* cur = lds + (s & 1) * 3 * cs;
        T* nxt = lds + ((s & 1) ^ 1) * 3 * cs;
        const WinV<T> v{cur, cs, wx, wy, X0 - 1, Y0 - 1, Z0 - 1};
        for (int e = threadIdx.x; e < 3 * ne; e += R3NT) {
            const int c = e / ne, r = e - c * ne;
            const int i = X0 + r % ew, j = Y0 + (r / ew) % eh, k = Z0 + r / (ew * eh);
            const bool unk = c == 0 ? vx_unknown3(nx, ny, nz, i, j, k)
                                    : c == 1 ? vy_unknown3(nx, ny, nz, i, j, k) : vz_unknown3(nx, ny, nz, i, j, k);
            if (!unk) continue;
            T d;
            const int64_t q = at3(f, i, j, k);
            const T m = c == 0 ? mvx3<T>(f, v, i, j, k, d) : c == 1 ? mvy3<T>(f, v, i, j, k, d) : mvz3<T>(f, v, i, j, k, d);
            const T b = c == 0 ? f.bx[q] : c == 1 ? f.by[q] : f.bz[q];
            const int o = ((k - (Z0 - 1)) * wy + (j - (Y0 - 1))) * wx + (i - (X0 - 1));
            nxt[c * cs + o] = jac_step<T>(cur[c * cs + o], omega / d, b, m);
        }
        __syncthreads();
    }
    // owned unknowns to the output; walls 0 (the right / top / back walls by the edge tiles)
    const T* fin = lds + (kt & 1) * 3 * cs;
    const int ow = x1 - x0 + 1, oh = y1 - y0 + 1, od = z1 - z0 + 1;
    for (int e = threadIdx.x; e < ow * oh * od; e += R3NT) {
        const int i = x0 + e % ow, j = y0 + (e / ow) % oh, k = z0 + e / (ow * oh);
        const bool ix = i < x1, iy = j < y1, iz = k < z1;
        const int o = ((k - (Z0 - 1)) * wy + (j - (Y0 - 1))) * wx + (i - (X0 - 1));
        const int64_t q = at3(f, i, j, k);
        if ((ix || i == nx) && iy && iz) ox[q] = vx_unknown3(nx, ny, nz, i, j, k) ? fin[o] : T(0);
        if (ix && (iy || j == ny) && iz) oy[q] = vy_unknown3(nx, ny, nz, i, j, k) ? fin[cs + o] : T(0);
        if (ix && iy && (iz || k == nz)) oz[q] = vz_unknown3(nx, ny, nz, i, j, k) ? fin[2 * cs + o] : T(0);
    }
}

// ------------------------------------------------------ residual, norms --
template <typename T>
__global__ __launch_bounds__(J3X* J3Y) void k_residual3d(Fields3<T> f, const T* __restrict__ vx,
                                                          const T* __restrict__ vy, const T* __restrict__ vz,
                                                          T* __restrict__ rx, T* __restrict__ ry,
                                                          T* __restrict__ rz) {
    const int i = blockIdx.x * J3X + threadIdx.x, j = blockIdx.y * J3Y + threadIdx.y, k = blockIdx.z;
    const int nx = f.nx, ny = f.ny, nz = f.nz;
    if (i > nx || j > ny || k > nz) return;
    const GlobalV<T> v{vx, vy, vz, f.ld, f.lp, nx, ny, nz};
    const int64_t q = at3(f, i, j, k);
    T d;
    if (k < nz && j < ny) rx[q] = vx_unknown3(nx, ny, nz, i, j, k) ? f.bx[q] - mvx3<T>(f, v, i, j, k, d) : T(0);
    if (k < nz && i < nx) ry[q] = vy_unknown3(nx, ny, nz, i, j, k) ? f.by[q] - mvy3<T>(f, v, i, j, k, d) : T(0);
    if (j < ny && i < nx) rz[q] = vz_unknown3(nx, ny, nz, i, j, k) ? f.bz[q] - mvz3<T>(f, v, i, j, k, d) : T(0);
}

__device__ __forceinline__ double wsum3(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Per-workgroup (N_v, N_f) partial sums in FP64, f = b: one workgroup per (x-y tile, plane).
template <typename T>
__global__ __launch_bounds__(J3X* J3Y) void k_energy3d(Fields3<T> f, const T* __restrict__ vx,
                                                        const T* __restrict__ vy, const T* __restrict__ vz,
                                                        double* __restrict__ part) {
    __shared__ double red[2][J3X * J3Y / 64];
    const int i = blockIdx.x * J3X + threadIdx.x, j = blockIdx.y * J3Y + threadIdx.y, k = blockIdx.z;
    const int nx = f.nx, ny = f.ny, nz = f.nz;
    double nv = 0.0, nf = 0.0;
    if (i <= nx && j <= ny && k <= nz) {
        const GlobalV<T> v{vx, vy, vz, f.ld, f.lp, nx, ny, nz};
        const int64_t q = at3(f, i, j, k);
        T d;
        if (vx_unknown3(nx, ny, nz, i, j, k)) {
            const double r = (double)f.bx[q] - (double)mvx3<T>(f, v, i, j, k, d);
            nv += r * r / (double)d;
            nf += (double)f.bx[q] * (double)f.bx[q] / (double)d;
        }
        if (vy_unknown3(nx, ny, nz, i, j, k)) {
            const double r = (double)f.by[q] - (double)mvy3<T>(f, v, i, j, k, d);
            nv += r * r / (double)d;
            nf += (double)f.by[q] * (double)f.by[q] / (double)d;
        }
        if (vz_unknown3(nx, ny, nz, i, j, k)) {
            const double r = (double)f.bz[q] - (double)mvz3<T>(f, v, i, j, k, d);
            nv += r * r / (double)d;
            nf += (double)f.bz[q] * (double)f.bz[q] / (double)d;
        }
    }
    const int t = threadIdx.y * J3X + threadIdx.x;
    nv = wsum3(nv);
    nf = wsum3(nf);
    if ((t & 63) == 0) {
        red[0][t >> 6] = nv;
        red[1][t >> 6] = nf;
    }
    __syncthreads();
    if (t < 2) {
        double s = 0.0;
        for (int w = 0; w < J3X * J3Y / 64; ++w) s += red[t][w];
        const int64_t b = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
        part[2 * b + t] = s;
    }
}

__global__ __launch_bounds__(1024) void k_energy3d_final(const double* __restrict__ part, int64_t n,
                                                         double* __restrict__ out) {
    __shared__ double red[2][1024 / 64];
    double s0 = 0.0, s1 = 0.0;
    for (int64_t q = threadIdx.x; q < n; q += 1024) {
        s0 += part[2 * q];
        s1 += part[2 * q + 1];
    }
    s0 = wsum3(s0);
    s1 = wsum3(s1);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = s0;
        red[1][threadIdx.x >> 6] = s1;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double s = 0.0;
        for (int w = 0; w < 1024 / 64; ++w) s += red[threadIdx.x][w];
        out[threadIdx.x] = s;
    }
}

template <typename T>
Fields3<T> fields3(const stk_grid3* g, const void* ec, const void* exy, const void* exz, const void* eyz,
                   const void* bx, const void* by, const void* bz) {
    Fields3<T> f;
    f.ec = static_cast<const T*>(ec);
    f.exy = static_cast<const T*>(exy);
    f.exz = static_cast<const T*>(exz);
    f.eyz = static_cast<const T*>(eyz);
    f.bx = static_cast<const T*>(bx);
    f.by = static_cast<const T*>(by);
    f.bz = static_cast<const T*>(bz);
    f.ld = g->ld;
    f.lp = g->lp;
    f.nx = g->nx;
    f.ny = g->ny;
    f.nz = g->nz;
    f.idx = T(1.0 / g->dx);
    f.idy = T(1.0 / g->dy);
    f.idz = T(1.0 / g->dz);
    return f;
}

dim3 grid3(const stk_grid3* g) {
    return dim3((unsigned)((g->nx + 1 + J3X - 1) / J3X), (unsigned)((g->ny + 1 + J3Y - 1) / J3Y),
                (unsigned)(g->nz + 1));
}

size_t ras3d_lds(int tile, int h, size_t es) {
    const size_t w = (size_t)tile + 2 * (size_t)h + 2;
    return 6 * w * w * w * es;
}

int check_grid3(const stk_grid3* g) {
    if (!g) return set_error(STK_EINVAL, "grid is NULL");
    if (g->nx < 2 || g->ny < 2 || g->nz < 2) return set_error(STK_EINVAL, "nx, ny, nz must be >= 2");
    if (g->ld < (int64_t)g->nx + 1) return set_error(STK_EINVAL, "ld must be >= nx + 1");
    if (g->lp < (int64_t)(g->ny + 1) * g->ld) return set_error(STK_EINVAL, "lp must be >= (ny + 1) ld");
    if (!(g->dx > 0.0 && g->dy > 0.0 && g->dz > 0.0) || !std::isfinite(g->dx) || !std::isfinite(g->dy) ||
        !std::isfinite(g->dz))
        return set_error(STK_EINVAL, "dx, dy, dz must be finite and > 0");
    if ((int64_t)(g->nz + 1) * g->lp > ((int64_t)1 << 40)) return set_error(STK_EINVAL, "grid too large");
    if (g->nz + 1 > 65535) return set_error(STK_EINVAL, "nz + 1 must be <= 65535");
    return STK_OK;
}

template <typename T>
int launch_jacobi3d(stk_ctx* ctx, const stk_grid3* g, const Fields3<T>& f, double omega, const void* vx,
                    const void* vy, const void* vz, void* ox, void* oy, void* oz) {
    const int ntx = (g->nx + ZX - 1) / ZX, nty = (g->ny + ZY - 1) / ZY, ntz = (g->nz + ZS - 1) / ZS;
    const int64_t nwg = (int64_t)ntx * nty * ntz;
    // the plane-streaming sweep addresses each array by 32-bit byte offsets
    if (nwg < INT32_MAX && (uint64_t)(g->nz + 1) * (uint64_t)g->lp * sizeof(T) <= UINT32_MAX) {
        hipLaunchKernelGGL(k_jacobi3d_z<T>, dim3((unsigned)nwg), dim3(ZX * ZY), 0, ctx->stream, f, T(omega),
                           static_cast<const T*>(vx), static_cast<const T*>(vy), static_cast<const T*>(vz),
                           static_cast<T*>(ox), static_cast<T*>(oy), static_cast<T*>(oz), ntx, nty);
    } else {
        hipLaunchKernelGGL(k_jacobi3d<T>, grid3(g), dim3(J3X, J3Y), 0, ctx->stream, f, T(omega),
                           static_cast<const T*>(vx), static_cast<const T*>(vy), static_cast<const T*>(vz),
                           static_cast<T*>(ox), static_cast<T*>(oy), static_cast<T*>(oz));
    }
    STK_HIP(hipGetLastError());
    return STK_OK;
}

template <typename T>
int launch_ras3d(stk_ctx* ctx, const stk_grid3* g, const Fields3<T>& f, double omega, int tile, int h, int kt,
                 int sx, int sy, int sz, const void* vx, const void* vy, const void* vz, void* ox, void* oy,
                 void* oz) {
    const size_t lds = ras3d_lds(tile, h, sizeof(T));
    if (lds > (size_t)ctx->lds_max)
        return set_error(STK_EUNSUPPORTED, "3D RAS tile %d with overlap %d needs %zu bytes of LDS (> %d)", tile, h,
                         lds, ctx->lds_max);
    static size_t attr_set[64] = {};
    const int dev = ctx->device < 64 ? ctx->device : 63;
    if (lds > attr_set[dev]) {
        STK_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_ras3d<T>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        attr_set[dev] = lds;
    }
    const dim3 grid((unsigned)((g->nx + tile - 1) / tile + 1), (unsigned)((g->ny + tile - 1) / tile + 1),
                    (unsigned)((g->nz + tile - 1) / tile + 1));
    hipLaunchKernelGGL(k_ras3d<T>, grid, dim3(R3NT), lds, ctx->stream, f, T(omega), static_cast<const T*>(vx),
                       static_cast<const T*>(vy), static_cast<const T*>(vz), static_cast<T*>(ox), static_cast<T*>(oy),
                       static_cast<T*>(oz), tile, h, kt, sx % tile, sy % tile, sz % tile, tile + 2 * h + 2);
    STK_HIP(hipGetLastError());
    return STK_OK;
}

}  // namespace
}  // namespace stk

using namespace stk;

extern "C" {

void stk_smooth3d_opts_default(stk_smooth3d_opts* o) {
    if (!o) return;
    o->omega = 0.7;
    o->tile = 8;
    o->halo = -1;
    o->k = 2;
    o->shifts = nullptr;
    o->seed = 0;
}

int stk_ras_outer3d(stk_ctx* ctx, stk_dtype dt, const stk_grid3* g, const void* vx, const void* vy, const void* vz,
                    const void* eta_c, const void* eta_xy, const void* eta_xz, const void* eta_yz, const void* bx,
                    const void* by, const void* bz, void* ox, void* oy, void* oz, double omega, int tile, int halo,
                    int kt, int sx, int sy, int sz) {
    if (!ctx) return set_error(STK_EINVAL, "ctx is NULL");
    if (dt != STK_F64 && dt != STK_F32) return set_error(STK_EINVAL, "unknown dtype %d", (int)dt);
    STK_TRY(check_grid3(g));
    if (!vx || !vy || !vz || !eta_c || !eta_xy || !eta_xz || !eta_yz || !bx || !by || !bz || !ox || !oy || !oz)
        return set_error(STK_EINVAL, "NULL array");
    if (ox == vx || oy == vy || oz == vz) return set_error(STK_EINVAL, "outputs alias inputs");
    if (!(omega > 0.0 && omega < 2.0)) return set_error(STK_EINVAL, "omega must be in (0, 2)");
    if (tile < 1 || halo < 0 || kt < 1 || sx < 0 || sy < 0 || sz < 0)
        return set_error(STK_EINVAL, "tile >= 1, halo >= 0, kt >= 1 and shifts >= 0 required");
    STK_TRY(use_device(ctx));
    if (dt == STK_F64)
        return launch_ras3d<double>(ctx, g, fields3<double>(g, eta_c, eta_xy, eta_xz, eta_yz, bx, by, bz), omega,
                                    tile, halo, kt, sx, sy, sz, vx, vy, vz, ox, oy, oz);
    return launch_ras3d<float>(ctx, g, fields3<float>(g, eta_c, eta_xy, eta_xz, eta_yz, bx, by, bz), omega, tile,
                               halo, kt, sx, sy, sz, vx, vy, vz, ox, oy, oz);
}

int stk_smooth3d(stk_ctx* ctx, stk_dtype dt, const stk_grid3* g, void* vx, void* vy, void* vz, const void* eta_c,
                 const void* eta_xy, const void* eta_xz, const void* eta_yz, const void* bx, const void* by,
                 const void* bz, int sweeps, stk_variant variant, const stk_smooth3d_opts* opts) {
    if (!ctx) return set_error(STK_EINVAL, "ctx is NULL");
    if (dt != STK_F64 && dt != STK_F32) return set_error(STK_EINVAL, "unknown dtype %d", (int)dt);
    STK_TRY(check_grid3(g));
    if (!vx || !vy || !vz || !eta_c || !eta_xy || !eta_xz || !eta_yz || !bx || !by || !bz)
        return set_error(STK_EINVAL, "NULL array");
    if (sweeps < 0) return set_error(STK_EINVAL, "sweeps must be >= 0");
    if (variant != STK_JACOBI_FUSED && variant != STK_RAS_JACOBI)
        return set_error(STK_EINVAL, "3D variants: STK_JACOBI_FUSED or STK_RAS_JACOBI");
    stk_smooth3d_opts o;
    stk_smooth3d_opts_default(&o);
    if (opts) o = *opts;
    if (!(o.omega > 0.0 && o.omega < 2.0)) return set_error(STK_EINVAL, "omega must be in (0, 2)");
    if (variant == STK_RAS_JACOBI && (o.tile < 1 || o.k < 1 || o.halo < -1))
        return set_error(STK_EINVAL, "tile >= 1, k >= 1, halo >= -1 required");
    if (variant == STK_RAS_JACOBI && ras3d_lds(o.tile, o.halo < 0 ? o.k : o.halo, elem_size(dt)) > (size_t)ctx->lds_max)
        return set_error(STK_EUNSUPPORTED, "3D RAS tile does not fit in LDS");
    if (sweeps == 0) return STK_OK;
    STK_TRY(use_device(ctx));
    // ping-pong through two scratch triples; the last step writes the caller's arrays
    const size_t fb = (size_t)(g->nz + 1) * (size_t)g->lp * elem_size(dt);
    void *t[6] = {};
    static const int slots[6] = {stk_ctx::S_VX, stk_ctx::S_VY, stk_ctx::S_VX2, stk_ctx::S_VY2, stk_ctx::S_BX,
                                 stk_ctx::S_BY};
    for (int q = 0; q < 6; ++q) STK_TRY(scratch(ctx, slots[q], fb, &t[q]));
    const int k = variant == STK_RAS_JACOBI ? o.k : 1;
    const int nsteps = (sweeps + k - 1) / k;
    std::vector<int32_t> sh;
    if (variant == STK_RAS_JACOBI) {
        sh.resize(3 * (size_t)nsteps);
        if (o.shifts) {
            for (size_t q = 0; q < sh.size(); ++q) sh[q] = o.shifts[q] % o.tile;
        } else {
            uint64_t s = o.seed;
            for (size_t q = 0; q < sh.size(); ++q) {  // SplitMix64 stream, x then y then z per outer iteration
                s += 0x9E3779B97F4A7C15ull;
                uint64_t z = s;
                z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
                z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
                z ^= z >> 31;
                sh[q] = (int32_t)((z >> 32) % (uint64_t)o.tile);
            }
        }
    }
    int left = sweeps;
    for (int st = 0; st < nsteps; ++st) {
        const bool first = st == 0, last = st == nsteps - 1;
        const void* src[3] = {first ? vx : t[3 * ((st - 1) & 1)], first ? vy : t[3 * ((st - 1) & 1) + 1],
                              first ? vz : t[3 * ((st - 1) & 1) + 2]};
        void* dst[3] = {last ? vx : t[3 * (st & 1)], last ? vy : t[3 * (st & 1) + 1], last ? vz : t[3 * (st & 1) + 2]};
        if (first && last) {  // one step: go through scratch, then copy back
            dst[0] = t[0];
            dst[1] = t[1];
            dst[2] = t[2];
        }
        const int kt = std::min(k, left);
        left -= kt;
        int rc;
        if (variant == STK_RAS_JACOBI) {
            const int h = o.halo < 0 ? kt : o.halo;
            rc = stk_ras_outer3d(ctx, dt, g, src[0], src[1], src[2], eta_c, eta_xy, eta_xz, eta_yz, bx, by, bz, dst[0],
                                 dst[1], dst[2], o.omega, o.tile, h, kt, sh[3 * st], sh[3 * st + 1], sh[3 * st + 2]);
        } else if (dt == STK_F64) {
            rc = launch_jacobi3d<double>(ctx, g, fields3<double>(g, eta_c, eta_xy, eta_xz, eta_yz, bx, by, bz), o.omega,
                                         src[0], src[1], src[2], dst[0], dst[1], dst[2]);
        } else {
            rc = launch_jacobi3d<float>(ctx, g, fields3<float>(g, eta_c, eta_xy, eta_xz, eta_yz, bx, by, bz), o.omega,
                                        src[0], src[1], src[2], dst[0], dst[1], dst[2]);
        }
        if (rc != STK_OK) return rc;
        if (first && last) {
            void* out[3] = {vx, vy, vz};
            for (int c = 0; c < 3; ++c)
                STK_HIP(hipMemcpyAsync(out[c], t[c], fb, hipMemcpyDeviceToDevice, ctx->stream));
        }
    }
    return STK_OK;
}

int stk_residual3d(stk_ctx* ctx, stk_dtype dt, const stk_grid3* g, const void* vx, const void* vy, const void* vz,
                   const void* eta_c, const void* eta_xy, const void* eta_xz, const void* eta_yz, const void* bx,
                   const void* by, const void* bz, void* rx, void* ry, void* rz) {
    if (!ctx) return set_error(STK_EINVAL, "ctx is NULL");
    if (dt != STK_F64 && dt != STK_F32) return set_error(STK_EINVAL, "unknown dtype %d", (int)dt);
    STK_TRY(check_grid3(g));
    if (!vx || !vy || !vz || !eta_c || !eta_xy || !eta_xz || !eta_yz || !bx || !by || !bz || !rx || !ry || !rz)
        return set_error(STK_EINVAL, "NULL array");
    STK_TRY(use_device(ctx));
    if (dt == STK_F64)
        hipLaunchKernelGGL(k_residual3d<double>, grid3(g), dim3(J3X, J3Y), 0, ctx->stream,
                           fields3<double>(g, eta_c, eta_xy, eta_xz, eta_yz, bx, by, bz), (const double*)vx,
                           (const double*)vy, (const double*)vz, (double*)rx, (double*)ry, (double*)rz);
    else
        hipLaunchKernelGGL(k_residual3d<float>, grid3(g), dim3(J3X, J3Y), 0, ctx->stream,
                           fields3<float>(g, eta_c, eta_xy, eta_xz, eta_yz, bx, by, bz), (const float*)vx,
                           (const float*)vy, (const float*)vz, (float*)rx, (float*)ry, (float*)rz);
    STK_HIP(hipGetLastError());
    return STK_OK;
}

int stk_energy_norm3d(stk_ctx* ctx, stk_dtype dt, const stk_grid3* g, const void* vx, const void* vy, const void* vz,
                      const void* eta_c, const void* eta_xy, const void* eta_xz, const void* eta_yz, const void* fx,
                      const void* fy, const void* fz, double out[3]) {
    if (!ctx) return set_error(STK_EINVAL, "ctx is NULL");
    if (dt != STK_F64 && dt != STK_F32) return set_error(STK_EINVAL, "unknown dtype %d", (int)dt);
    STK_TRY(check_grid3(g));
    if (!vx || !vy || !vz || !eta_c || !eta_xy || !eta_xz || !eta_yz || !fx || !fy || !fz || !out)
        return set_error(STK_EINVAL, "NULL argument");
    STK_TRY(use_device(ctx));
    const dim3 gr = grid3(g);
    const int64_t nblk = (int64_t)gr.x * gr.y * gr.z;
    void *part = nullptr, *red = nullptr;
    STK_TRY(scratch(ctx, stk_ctx::S_PART, sizeof(double) * 2 * (size_t)nblk, &part));
    STK_TRY(scratch(ctx, stk_ctx::S_RED, 64 * sizeof(double), &red));
    if (dt == STK_F64)
        hipLaunchKernelGGL(k_energy3d<double>, gr, dim3(J3X, J3Y), 0, ctx->stream,
                           fields3<double>(g, eta_c, eta_xy, eta_xz, eta_yz, fx, fy, fz), (const double*)vx,
                           (const double*)vy, (const double*)vz, (double*)part);
    else
        hipLaunchKernelGGL(k_energy3d<float>, gr, dim3(J3X, J3Y), 0, ctx->stream,
                           fields3<float>(g, eta_c, eta_xy, eta_xz, eta_yz, fx, fy, fz), (const float*)vx,
                           (const float*)vy, (const float*)vz, (double*)part);
    hipLaunchKernelGGL(k_energy3d_final, dim3(1), dim3(1024), 0, ctx->stream, (const double*)part, nblk,
                       (double*)red);
    STK_HIP(hipGetLastError());
    STK_HIP(hipMemcpyAsync(ctx->host_red, red, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    STK_HIP(hipStreamSynchronize(ctx->stream));
    out[0] = ctx->host_red[0];
    out[1] = ctx->host_red[1];
    out[2] = std::sqrt(out[0] / out[1]);
    for (int q = 0; q < 3; ++q)
        if (!std::isfinite(out[q])) return set_error(STK_ENONFINITE, "3D energy norm is not finite");
    return STK_OK;
}

}  // extern "C"
