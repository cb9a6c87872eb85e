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

// Fused multiply-add with a single rounding, written out so that no kernel
// depends on the compiler's contraction choices.
__host__ __device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__host__ __device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// The Jacobi factor g = omega / d (d = diag(-M) > 0): a reciprocal estimate
// refined by Newton steps r <- r + r (1 - d r), then one residual correction
// of the quotient q <- q + r (omega - d q) (Markstein's scheme).  No range
// scaling: a diagonal of the viscous operator is far from the limits of the
// format.  Every kernel takes its factor from here.
__device__ __forceinline__ double jac_factor(double omega, double d) {
    double r = __builtin_amdgcn_rcp(d);
    r = fmaT(r, fmaT(-d, r, 1.0), r);
    r = fmaT(r, fmaT(-d, r, 1.0), r);
    const double q = omega * r;
    return fmaT(fmaT(-d, q, omega), r, q);
}
__device__ __forceinline__ float jac_factor(float omega, float d) {
    float r = __builtin_amdgcn_rcpf(d);
    r = fmaT(r, fmaT(-d, r, 1.0f), r);
    const float q = omega * r;
    return fmaT(fmaT(-d, q, omega), r, q);
}

// The damped Jacobi step from the operator value m = (Mv) at the unknown and
// g = jac_factor(omega, diag(-M)): v' = v - g (b - m).  Every kernel ends in
// this call.
template <typename T>
__device__ __forceinline__ T jac_step(T vc, T g, T b, T m) {
    return fmaT(-g, b - m, vc);
}

// Scaled coefficients.  With A = 2 eta_c idx^2 and N = eta_n idx idy the
// operator rows read
//   (Mv)_x = A_r (vr - vc) - A_l (vc - vl)
//          + N_t (ry (vt - vc) + (ytc - ytl)) - N_b (ry (vc - vb) + (ybc - ybl))
//   (Mv)_y = B_t (vt - vc) - B_b (vc - vb)
//          + N_r (rx (vr - vc) + (xrc - xrb)) - N_l (rx (vc - vl) + (xlc - xlb))
// with B = A kap, kap = idy^2 / idx^2, ry = idy / idx, rx = idx / idy (all 1
// on square cells), and diag(-M) = (A_l + A_r) + ry (N_b + N_t) for vx,
// (B_b + B_t) + rx (N_l + N_r) for vy.  Per cell and sweep this is 12
// operations per component instead of about 17 with raw viscosities, and a
// kernel that keeps A and N (instead of eta_c and eta_n) computes the same
// values bit for bit.
template <typename T>
struct Scale {
    T a, n, kap, ry, rx;
};
template <typename T>
__host__ __device__ __forceinline__ Scale<T> stencil_scale(T idx, T idy) {
    return {T(2) * idx * idx, idx * idy, (idy * idy) / (idx * idx), idy / idx, idx / idy};
}
template <typename T>
__host__ __device__ __forceinline__ T coef_a(T ec, const Scale<T>& s) { return ec * s.a; }
template <typename T>
__host__ __device__ __forceinline__ T coef_n(T en, const Scale<T>& s) { return en * s.n; }
template <typename T>
__host__ __device__ __forceinline__ T coef_b(T a, const Scale<T>& s) { return a * s.kap; }

template <typename T>
__host__ __device__ __forceinline__ T mvx_scaled(T vc, T vl, T vr, T vb, T vt, T ybc, T ybl, T ytc, T ytl, T al, T ar,
                                                 T nb, T nt, T ry) {
    T m = ar * (vr - vc);
    m = fmaT(-al, vc - vl, m);
    m = fmaT(nt, fmaT(ry, vt - vc, ytc - ytl), m);
    return fmaT(-nb, fmaT(ry, vc - vb, ybc - ybl), m);
}
template <typename T>
__host__ __device__ __forceinline__ T mvy_scaled(T vc, T vl, T vr, T vb, T vt, T xlc, T xrc, T xlb, T xrb, T bb, T bt,
                                                 T nl, T nr, T rx) {
    T m = bt * (vt - vc);
    m = fmaT(-bb, vc - vb, m);
    m = fmaT(nr, fmaT(rx, vr - vc, xrc - xrb), m);
    return fmaT(-nl, fmaT(rx, vc - vl, xlc - xlb), m);
}
template <typename T>
__host__ __device__ __forceinline__ T diagx_scaled(T al, T ar, T nb, T nt, T ry) { return fmaT(nb + nt, ry, al + ar); }
template <typename T>
__host__ __device__ __forceinline__ T diagy_scaled(T bb, T bt, T nl, T nr, T rx) { return fmaT(nl + nr, rx, bb + bt); }

// (M v)_x and (M v)_y from raw viscosities (residual kernels and the
// gathering smoothers): scale, then the expressions above.
template <typename T>
__device__ __forceinline__ T mv_x(T vc, T vl, T vr, T vb, T vt, T ybc, T ybl, T ytc, T ytl, T ecl, T ecr, T enb, T ent,
                                  T idx, T idy) {
    const Scale<T> s = stencil_scale(idx, idy);
    return mvx_scaled<T>(vc, vl, vr, vb, vt, ybc, ybl, ytc, ytl, coef_a(ecl, s), coef_a(ecr, s), coef_n(enb, s),
                         coef_n(ent, s), s.ry);
}
template <typename T>
__device__ __forceinline__ T mv_y(T vc, T vl, T vr, T vb, T vt, T xlc, T xrc, T xlb, T xrb, T ecb, T ect, T enl, T enr,
                                  T idx, T idy) {
    const Scale<T> s = stencil_scale(idx, idy);
    return mvy_scaled<T>(vc, vl, vr, vb, vt, xlc, xrc, xlb, xrb, coef_b(coef_a(ecb, s), s), coef_b(coef_a(ect, s), s),
                         coef_n(enl, s), coef_n(enr, s), s.rx);
}
template <typename T>
__device__ __forceinline__ T diag_x(T ecl, T ecr, T enb, T ent, T idx, T idy) {
    const Scale<T> s = stencil_scale(idx, idy);
    return diagx_scaled<T>(coef_a(ecl, s), coef_a(ecr, s), coef_n(enb, s), coef_n(ent, s), s.ry);
}
template <typename T>
__device__ __forceinline__ T diag_y(T ecb, T ect, T enl, T enr, T idx, T idy) {
    const Scale<T> s = stencil_scale(idx, idy);
    return diagy_scaled<T>(coef_b(coef_a(ecb, s), s), coef_b(coef_a(ect, s), s), coef_n(enl, s), coef_n(enr, s), s.rx);
}

// New vx(i,j).  vc = vx(i,j); vl/vr = vx(i-1/i+1, j); vb/vt = vx(i, j-1/j+1);
// ybc/ybl = vy(i/i-1, j); ytc/ytl = vy(i/i-1, j+1); ecl/ecr = eta_c(i-1/i, j);
// enb/ent = eta_n(i, j/j+1) (0 on boundary nodes).
template <typename T>
__device__ __forceinline__ T jac_vx(T vc, T vl, T vr, T vb, T vt, T ybc, T ybl, T ytc, T ytl, T ecl, T ecr, T enb,
                                    T ent, T b, T omega, T idx, T idy) {
    const T m = mv_x<T>(vc, vl, vr, vb, vt, ybc, ybl, ytc, ytl, ecl, ecr, enb, ent, idx, idy);
    const T g = jac_factor(omega, diag_x<T>(ecl, ecr, enb, ent, idx, idy));
    return jac_step<T>(vc, g, b, m);
}

// New vy(i,j).  vc = vy(i,j); vl/vr = vy(i-1/i+1, j); vb/vt = vy(i, j-1/j+1);
// xlc/xrc = vx(i/i+1, j); xlb/xrb = vx(i/i+1, j-1); ecb/ect = eta_c(i, j-1/j);
// enl/enr = eta_n(i/i+1, j) (0 on boundary nodes).
template <typename T>
__device__ __forceinline__ T jac_vy(T vc, T vl, T vr, T vb, T vt, T xlc, T xrc, T xlb, T xrb, T ecb, T ect, T enl,
                                    T enr, T b, T omega, T idx, T idy) {
    const T m = mv_y<T>(vc, vl, vr, vb, vt, xlc, xrc, xlb, xrb, ecb, ect, enl, enr, idx, idy);
    const T g = jac_factor(omega, diag_y<T>(ecb, ect, enl, enr, idx, idy));
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
