// Device-side staggered-grid stencil shared by every smoother kernel.
//
// One damped-Jacobi update of a vx or vy unknown from its neighbourhood, in a
// single canonical expression order, so that fused, split, red-black and
// RAS-blocked kernels produce bit-identical values for identical inputs.
//
// Discretisation (paper Sec. 2.1, Cauchy form on the staggered grid of
// Fig. 1): normal stresses 2 eta_c du/dx at cell centres, shear stress
// eta_n (dvx/dy + dvy/dx) at nodes (zero at boundary nodes: free slip),
// centred divergences.  The damped Jacobi step is v' = v - (omega/d)(b - M v)
// with d = diag(-M) (Sec. 5 smoothers).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace stk {

// Read-only field set of one grid in the common-stride layout.
template <typename T>
struct Grid {
    const T* ec;  // eta_c, ny x nx
    const T* en;  // eta_n, (ny+1) x (nx+1)
    const T* bx;  // rhs at vx points, ny x (nx+1)
    const T* by;  // rhs at vy points, (ny+1) x nx
    int64_t ld;
    int nx, ny;
    T idx, idy, omega;
};

// Velocity loads with the Dirichlet walls (and anything outside the arrays)
// read as 0.
template <typename T>
__device__ __forceinline__ T ldvx(const T* __restrict__ v, int64_t ld, int nx, int ny, int i, int j) {
    return (i >= 1 && i <= nx - 1 && j >= 0 && j < ny) ? v[(int64_t)j * ld + i] : T(0);
}
template <typename T>
__device__ __forceinline__ T ldvy(const T* __restrict__ v, int64_t ld, int nx, int ny, int i, int j) {
    return (j >= 1 && j <= ny - 1 && i >= 0 && i < nx) ? v[(int64_t)j * ld + i] : T(0);
}
// Nodal viscosity with the free-slip boundary nodes read as 0.
template <typename T>
__device__ __forceinline__ T ldenh(const Grid<T>& g, int i, int j) {
    return (i >= 1 && i <= g.nx - 1 && j >= 1 && j <= g.ny - 1) ? g.en[(int64_t)j * g.ld + i] : T(0);
}

// The damped Jacobi step from the operator value m = (Mv) at the unknown and
// g = omega / diag(-M): v' = v - g (b - m).  Every kernel ends in this call.
template <typename T>
__device__ __forceinline__ T jac_step(T vc, T g, T b, T m) {
    return vc - g * (b - m);
}

// (M v)_x and (M v)_y in the same expression order (residual kernels).
template <typename T>
__device__ __forceinline__ T mv_x(T vc, T vl, T vr, T vb, T vt, T ybc, T ybl, T ytc, T ytl, T ecl, T ecr, T enb, T ent,
                                  T idx, T idy) {
    const T txr = T(2) * ecr * (vr - vc) * idx;
    const T txl = T(2) * ecl * (vc - vl) * idx;
    const T sxt = ent * ((vt - vc) * idy + (ytc - ytl) * idx);
    const T sxb = enb * ((vc - vb) * idy + (ybc - ybl) * idx);
    return (txr - txl) * idx + (sxt - sxb) * idy;
}
template <typename T>
__device__ __forceinline__ T mv_y(T vc, T vl, T vr, T vb, T vt, T xlc, T xrc, T xlb, T xrb, T ecb, T ect, T enl, T enr,
                                  T idx, T idy) {
    const T tyt = T(2) * ect * (vt - vc) * idy;
    const T tyb = T(2) * ecb * (vc - vb) * idy;
    const T syr = enr * ((xrc - xrb) * idy + (vr - vc) * idx);
    const T syl = enl * ((xlc - xlb) * idy + (vc - vl) * idx);
    return (tyt - tyb) * idy + (syr - syl) * idx;
}
template <typename T>
__device__ __forceinline__ T diag_x(T ecl, T ecr, T enb, T ent, T idx, T idy) {
    return T(2) * (ecl + ecr) * (idx * idx) + (enb + ent) * (idy * idy);
}
template <typename T>
__device__ __forceinline__ T diag_y(T ecb, T ect, T enl, T enr, T idx, T idy) {
    return T(2) * (ecb + ect) * (idy * idy) + (enl + enr) * (idx * idx);
}

// New vx(i,j).  vc = vx(i,j); vl/vr = vx(i-1/i+1, j); vb/vt = vx(i, j-1/j+1);
// ybc/ybl = vy(i/i-1, j); ytc/ytl = vy(i/i-1, j+1); ecl/ecr = eta_c(i-1/i, j);
// enb/ent = eta_n(i, j/j+1) (0 on boundary nodes).
template <typename T>
__device__ __forceinline__ T jac_vx(T vc, T vl, T vr, T vb, T vt, T ybc, T ybl, T ytc, T ytl, T ecl, T ecr, T enb,
                                    T ent, T b, T omega, T idx, T idy) {
    const T m = mv_x<T>(vc, vl, vr, vb, vt, ybc, ybl, ytc, ytl, ecl, ecr, enb, ent, idx, idy);
    const T g = omega / diag_x<T>(ecl, ecr, enb, ent, idx, idy);
    return jac_step<T>(vc, g, b, m);
}

// New vy(i,j).  vc = vy(i,j); vl/vr = vy(i-1/i+1, j); vb/vt = vy(i, j-1/j+1);
// xlc/xrc = vx(i/i+1, j); xlb/xrb = vx(i/i+1, j-1); ecb/ect = eta_c(i, j-1/j);
// enl/enr = eta_n(i/i+1, j) (0 on boundary nodes).
template <typename T>
__device__ __forceinline__ T jac_vy(T vc, T vl, T vr, T vb, T vt, T xlc, T xrc, T xlb, T xrb, T ecb, T ect, T enl,
                                    T enr, T b, T omega, T idx, T idy) {
    const T m = mv_y<T>(vc, vl, vr, vb, vt, xlc, xrc, xlb, xrb, ecb, ect, enl, enr, idx, idy);
    const T g = omega / diag_y<T>(ecb, ect, enl, enr, idx, idy);
    return jac_step<T>(vc, g, b, m);
}

// Gather-and-update at (i,j) straight from global memory (walls read as 0).
template <typename T>
__device__ __forceinline__ T jac_vx_global(const Grid<T>& g, const T* __restrict__ vx, const T* __restrict__ vy, int i,
                                           int j) {
    const int64_t ld = g.ld;
    const int nx = g.nx, ny = g.ny;
    return jac_vx<T>(ldvx(vx, ld, nx, ny, i, j), ldvx(vx, ld, nx, ny, i - 1, j), ldvx(vx, ld, nx, ny, i + 1, j),
                     ldvx(vx, ld, nx, ny, i, j - 1), ldvx(vx, ld, nx, ny, i, j + 1), ldvy(vy, ld, nx, ny, i, j),
                     ldvy(vy, ld, nx, ny, i - 1, j), ldvy(vy, ld, nx, ny, i, j + 1), ldvy(vy, ld, nx, ny, i - 1, j + 1),
                     g.ec[(int64_t)j * ld + i - 1], g.ec[(int64_t)j * ld + i], ldenh(g, i, j), ldenh(g, i, j + 1),
                     g.bx[(int64_t)j * ld + i], g.omega, g.idx, g.idy);
}
template <typename T>
__device__ __forceinline__ T jac_vy_global(const Grid<T>& g, const T* __restrict__ vx, const T* __restrict__ vy, int i,
                                           int j) {
    const int64_t ld = g.ld;
    const int nx = g.nx, ny = g.ny;
    return jac_vy<T>(ldvy(vy, ld, nx, ny, i, j), ldvy(vy, ld, nx, ny, i - 1, j), ldvy(vy, ld, nx, ny, i + 1, j),
                     ldvy(vy, ld, nx, ny, i, j - 1), ldvy(vy, ld, nx, ny, i, j + 1), ldvx(vx, ld, nx, ny, i, j),
                     ldvx(vx, ld, nx, ny, i + 1, j), ldvx(vx, ld, nx, ny, i, j - 1), ldvx(vx, ld, nx, ny, i + 1, j - 1),
                     g.ec[(int64_t)(j - 1) * ld + i], g.ec[(int64_t)j * ld + i], ldenh(g, i, j), ldenh(g, i + 1, j),
                     g.by[(int64_t)j * ld + i], g.omega, g.idx, g.idy);
}

__device__ __forceinline__ bool is_vx_unknown(int nx, int ny, int i, int j) { return i >= 1 && i <= nx - 1 && j >= 0 && j < ny; }
__device__ __forceinline__ bool is_vy_unknown(int nx, int ny, int i, int j) { return j >= 1 && j <= ny - 1 && i >= 0 && i < nx; }

}  // namespace stk
