/*
 * CPU ORACLE — TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct FP64 reference of the staggered-grid
 * variable-viscosity Stokes velocity smoother and its companions.  Only the
 * test-suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it.  It shares no code, header or constant with the HIP library.
 *
 * Layout (natural, row-major, x fastest; unit square, y up):
 *   vx, fx : ny   x (nx+1)   vx(i,j) at (i dx, (j+1/2) dy)   unknown iff 1<=i<=nx-1
 *   vy, fy : (ny+1) x nx     vy(i,j) at ((i+1/2) dx, j dy)   unknown iff 1<=j<=ny-1
 *   eta_c, p: ny x nx        cell centres (the paper's eta_P, pressure)
 *   eta_n  : (ny+1) x (nx+1) nodes (the paper's eta_B)
 * Wall entries of vx/vy (i=0, i=nx for vx; j=0, j=ny for vy) are Dirichlet 0:
 * inputs are read as if they held 0 and outputs hold 0 there.
 *
 * Operator (paper Sec. 2.1, eqs. for x-/y-momentum and the constitutive law
 * sigma'_ij = eta (dv_i/dx_j + dv_j/dx_i), discretised on the staggered grid of
 * Fig. 1 with eta_P for normal and eta_B for shear stress):
 *   txx(i,j) = 2 eta_c(i,j) (vx(i+1,j)-vx(i,j))/dx            per cell
 *   tyy(i,j) = 2 eta_c(i,j) (vy(i,j+1)-vy(i,j))/dy            per cell
 *   txy(i,j) = eta_n(i,j) ((vx(i,j)-vx(i,j-1))/dy + (vy(i,j)-vy(i-1,j))/dx)
 *              at interior nodes, 0 at boundary nodes (free slip)
 *   (Mv)_x(i,j) = (txx(i,j)-txx(i-1,j))/dx + (txy(i,j+1)-txy(i,j))/dy
 *   (Mv)_y(i,j) = (tyy(i,j)-tyy(i,j-1))/dy + (txy(i+1,j)-txy(i,j))/dx
 * The velocity subsystem is M v + G p = f (Sec. 3.1), G = D^T, so the
 * right-hand side for fixed p is b = f - G p with
 *   (Gp)_x(i,j) = -(p(i,j)-p(i-1,j))/dx,  (Gp)_y(i,j) = -(p(i,j)-p(i,j-1))/dy,
 *   (Dv)(i,j)   = (vx(i+1,j)-vx(i,j))/dx + (vy(i,j+1)-vy(i,j))/dy.
 * M is symmetric negative definite (Sec. 6.4); d = diag(-M) > 0.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Threads the OpenMP loops use (for reporting the CPU baseline's core count). */
int or_num_threads(void) { return omp_get_max_threads(); }
/* Threads for the following calls (the CPU baseline is timed at nproc and at 1). */
void or_set_num_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

typedef struct {
    int nx, ny;
    double dx, dy;
    const double *ec, *en; /* eta_c (ny x nx), eta_n ((ny+1) x (nx+1)) */
} grid_t;

/* A velocity state seen through a window: vx(i,j) = vx[(j-oy)*lx + (i-ox)],
 * vy(i,j) = vy[(j-oy)*ly + (i-ox)].  Full arrays use ox = oy = 0,
 * lx = nx+1, ly = nx. */
typedef struct {
    const double *vx, *vy;
    int ox, oy;
    long lx, ly;
} view_t;

#define VXV(V, i, j) ((V)->vx[(long)((j) - (V)->oy) * (V)->lx + ((i) - (V)->ox)])
#define VYV(V, i, j) ((V)->vy[(long)((j) - (V)->oy) * (V)->ly + ((i) - (V)->ox)])
#define EC(G, i, j) ((G)->ec[(long)(j) * (G)->nx + (i)])
#define EN(G, i, j) ((G)->en[(long)(j) * ((G)->nx + 1) + (i)])

static int vx_unknown(const grid_t* g, int i, int j) { return i >= 1 && i <= g->nx - 1 && j >= 0 && j < g->ny; }
static int vy_unknown(const grid_t* g, int i, int j) { return j >= 1 && j <= g->ny - 1 && i >= 0 && i < g->nx; }

/* Normal deviatoric stresses at cell (i,j). */
static double txx(const grid_t* g, const view_t* v, int i, int j) {
    return 2.0 * EC(g, i, j) * (VXV(v, i + 1, j) - VXV(v, i, j)) / g->dx;
}
static double tyy(const grid_t* g, const view_t* v, int i, int j) {
    return 2.0 * EC(g, i, j) * (VYV(v, i, j + 1) - VYV(v, i, j)) / g->dy;
}
/* Shear stress at node (i,j); zero on the boundary (free slip). */
static double txy(const grid_t* g, const view_t* v, int i, int j) {
    if (i <= 0 || i >= g->nx || j <= 0 || j >= g->ny) return 0.0;
    return EN(g, i, j) * ((VXV(v, i, j) - VXV(v, i, j - 1)) / g->dy + (VYV(v, i, j) - VYV(v, i - 1, j)) / g->dx);
}
/* (Mv)_x at the vx unknown (i,j) and (Mv)_y at the vy unknown (i,j). */
static double mvx(const grid_t* g, const view_t* v, int i, int j) {
    return (txx(g, v, i, j) - txx(g, v, i - 1, j)) / g->dx + (txy(g, v, i, j + 1) - txy(g, v, i, j)) / g->dy;
}
static double mvy(const grid_t* g, const view_t* v, int i, int j) {
    return (tyy(g, v, i, j) - tyy(g, v, i, j - 1)) / g->dy + (txy(g, v, i + 1, j) - txy(g, v, i, j)) / g->dx;
}
/* Diagonal of -M with the boundary conditions: the coefficient of the unknown
 * itself in -(Mv) (shear terms vanish at boundary nodes). */
static double enhat(const grid_t* g, int i, int j) {
    return (i <= 0 || i >= g->nx || j <= 0 || j >= g->ny) ? 0.0 : EN(g, i, j);
}
static double diag_x(const grid_t* g, int i, int j) {
    return 2.0 * (EC(g, i - 1, j) + EC(g, i, j)) / (g->dx * g->dx) + (enhat(g, i, j) + enhat(g, i, j + 1)) / (g->dy * g->dy);
}
static double diag_y(const grid_t* g, int i, int j) {
    return 2.0 * (EC(g, i, j - 1) + EC(g, i, j)) / (g->dy * g->dy) + (enhat(g, i, j) + enhat(g, i + 1, j)) / (g->dx * g->dx);
}

static grid_t mkgrid(int nx, int ny, double dx, double dy, const double* ec, const double* en) {
    grid_t g = {nx, ny, dx, dy, ec, en};
    return g;
}

/* Copy a velocity state into fresh arrays with the wall entries forced to 0. */
static void copy_state(int nx, int ny, const double* vx, const double* vy, double* ox, double* oy) {
    memcpy(ox, vx, sizeof(double) * (size_t)ny * (nx + 1));
    memcpy(oy, vy, sizeof(double) * (size_t)(ny + 1) * nx);
    for (int j = 0; j < ny; ++j) { ox[(long)j * (nx + 1)] = 0.0; ox[(long)j * (nx + 1) + nx] = 0.0; }
    for (int i = 0; i < nx; ++i) { oy[i] = 0.0; oy[(long)ny * nx + i] = 0.0; }
}

static view_t full_view(int nx, const double* vx, const double* vy) {
    view_t v = {vx, vy, 0, 0, nx + 1, nx};
    return v;
}

/* ---------------------------------------------------------------- apply -- */

/* mx, my <- M v on the unknowns, 0 on walls. */
void or_apply(int nx, int ny, double dx, double dy, const double* ec, const double* en,
              const double* vx, const double* vy, double* mx, double* my) {
    grid_t g = mkgrid(nx, ny, dx, dy, ec, en);
    double* wx = malloc(sizeof(double) * (size_t)ny * (nx + 1));
    double* wy = malloc(sizeof(double) * (size_t)(ny + 1) * nx);
    copy_state(nx, ny, vx, vy, wx, wy);
    view_t v = full_view(nx, wx, wy);
#pragma omp parallel for schedule(static)
    for (int j = 0; j <= ny; ++j) {
        for (int i = 0; i <= nx; ++i) {
            if (j < ny) mx[(long)j * (nx + 1) + i] = vx_unknown(&g, i, j) ? mvx(&g, &v, i, j) : 0.0;
            if (i < nx) my[(long)j * nx + i] = vy_unknown(&g, i, j) ? mvy(&g, &v, i, j) : 0.0;
        }
    }
    free(wx);
    free(wy);
}

/* d = diag(-M) on the unknowns, 0 on walls. */
void or_diag(int nx, int ny, double dx, double dy, const double* ec, const double* en, double* dxo, double* dyo) {
    grid_t g = mkgrid(nx, ny, dx, dy, ec, en);
#pragma omp parallel for schedule(static)
    for (int j = 0; j <= ny; ++j) {
        for (int i = 0; i <= nx; ++i) {
            if (j < ny) dxo[(long)j * (nx + 1) + i] = vx_unknown(&g, i, j) ? diag_x(&g, i, j) : 0.0;
            if (i < nx) dyo[(long)j * nx + i] = vy_unknown(&g, i, j) ? diag_y(&g, i, j) : 0.0;
        }
    }
}

/* b = f - G p on the unknowns (p may be NULL: b = f), 0 on walls. */
void or_rhs(int nx, int ny, double dx, double dy, const double* fx, const double* fy, const double* p,
            double* bx, double* by) {
#pragma omp parallel for schedule(static)
    for (int j = 0; j <= ny; ++j) {
        for (int i = 0; i <= nx; ++i) {
            if (j < ny) {
                long k = (long)j * (nx + 1) + i;
                double b = 0.0;
                if (i >= 1 && i <= nx - 1) {
                    b = fx[k];
                    if (p) b -= -(p[(long)j * nx + i] - p[(long)j * nx + i - 1]) / dx;
                }
                bx[k] = b;
            }
            if (i < nx) {
                long k = (long)j * nx + i;
                double b = 0.0;
                if (j >= 1 && j <= ny - 1) {
                    b = fy[k];
                    if (p) b -= -(p[(long)j * nx + i] - p[(long)(j - 1) * nx + i]) / dy;
                }
                by[k] = b;
            }
        }
    }
}

/* Divergence (Dv)(i,j) per cell. */
void or_divergence(int nx, int ny, double dx, double dy, const double* vx, const double* vy, double* dv) {
    double* wx = malloc(sizeof(double) * (size_t)ny * (nx + 1));
    double* wy = malloc(sizeof(double) * (size_t)(ny + 1) * nx);
    copy_state(nx, ny, vx, vy, wx, wy);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
            dv[(long)j * nx + i] = (wx[(long)j * (nx + 1) + i + 1] - wx[(long)j * (nx + 1) + i]) / dx +
                                   (wy[(long)(j + 1) * nx + i] - wy[(long)j * nx + i]) / dy;
    free(wx);
    free(wy);
}

/* ---------------------------------------------------------------- Jacobi -- */

/* Damped Jacobi update of one unknown (Sec. 4/5 smoothers):
 *   v' = v + omega (b - M v) / M_ii = v - omega (b - M v) / d.              */
static double jac_x(const grid_t* g, const view_t* v, const double* bx, double omega, int i, int j) {
    double r = bx[(long)j * (g->nx + 1) + i] - mvx(g, v, i, j);
    return VXV(v, i, j) - omega * r / diag_x(g, i, j);
}
static double jac_y(const grid_t* g, const view_t* v, const double* by, double omega, int i, int j) {
    double r = by[(long)j * g->nx + i] - mvy(g, v, i, j);
    return VYV(v, i, j) - omega * r / diag_y(g, i, j);
}

/* One damped Jacobi sweep, out-of-place: (ox, oy) <- J(vx, vy).  Both
 * components read the old iterate only (split and fused Jacobi have the same
 * values). */
void or_jacobi(int nx, int ny, double dx, double dy, const double* ec, const double* en, const double* bx,
               const double* by, double omega, const double* vx, const double* vy, double* ox, double* oy) {
    grid_t g = mkgrid(nx, ny, dx, dy, ec, en);
    double* wx = malloc(sizeof(double) * (size_t)ny * (nx + 1));
    double* wy = malloc(sizeof(double) * (size_t)(ny + 1) * nx);
    copy_state(nx, ny, vx, vy, wx, wy);
    view_t v = full_view(nx, wx, wy);
#pragma omp parallel for schedule(static)
    for (int j = 0; j <= ny; ++j) {
        for (int i = 0; i <= nx; ++i) {
            if (j < ny) ox[(long)j * (nx + 1) + i] = vx_unknown(&g, i, j) ? jac_x(&g, &v, bx, omega, i, j) : 0.0;
            if (i < nx) oy[(long)j * nx + i] = vy_unknown(&g, i, j) ? jac_y(&g, &v, by, omega, i, j) : 0.0;
        }
    }
    free(wx);
    free(wy);
}

/* ------------------------------------------------------------------ RBGS -- */

/* One red-black Gauss-Seidel sweep, in place (Sec. 4, smoother (i)).
 * Colour of vx(i,j) and vy(i,j) is (i+j) mod 2 (red = 0).  The four sets are
 * relaxed in the order vx-red, vx-black, vy-red, vy-black; each set uses the
 * current iterate.  Unknowns inside one set do not couple to each other. */
void or_rbgs(int nx, int ny, double dx, double dy, const double* ec, const double* en, const double* bx,
             const double* by, double omega, double* vx, double* vy) {
    grid_t g = mkgrid(nx, ny, dx, dy, ec, en);
    long nvx = (long)ny * (nx + 1), nvy = (long)(ny + 1) * nx;
    double* wx = malloc(sizeof(double) * nvx);
    double* wy = malloc(sizeof(double) * nvy);
    double* nw = malloc(sizeof(double) * (nvx > nvy ? nvx : nvy));
    copy_state(nx, ny, vx, vy, wx, wy);
    view_t v = full_view(nx, wx, wy);
    for (int comp = 0; comp < 2; ++comp) {
        for (int colour = 0; colour < 2; ++colour) {
            /* compute the whole set from the current iterate, then store it */
#pragma omp parallel for schedule(static)
            for (int j = 0; j <= ny; ++j)
                for (int i = 0; i <= nx; ++i) {
                    if (((i + j) & 1) != colour) continue;
                    if (comp == 0 && j < ny && vx_unknown(&g, i, j)) nw[(long)j * (nx + 1) + i] = jac_x(&g, &v, bx, omega, i, j);
                    if (comp == 1 && i < nx && vy_unknown(&g, i, j)) nw[(long)j * nx + i] = jac_y(&g, &v, by, omega, i, j);
                }
#pragma omp parallel for schedule(static)
            for (int j = 0; j <= ny; ++j)
                for (int i = 0; i <= nx; ++i) {
                    if (((i + j) & 1) != colour) continue;
                    if (comp == 0 && j < ny && vx_unknown(&g, i, j)) wx[(long)j * (nx + 1) + i] = nw[(long)j * (nx + 1) + i];
                    if (comp == 1 && i < nx && vy_unknown(&g, i, j)) wy[(long)j * nx + i] = nw[(long)j * nx + i];
                }
        }
    }
    memcpy(vx, wx, sizeof(double) * nvx);
    memcpy(vy, wy, sizeof(double) * nvy);
    free(wx);
    free(wy);
    free(nw);
}

/* ------------------------------------------------------------------- RAS -- */

/* Tile cuts along one axis for shift s and tile size T: cuts at the positions
 * congruent to s modulo T inside (0, n); tile t covers [lo, hi).  Returns
 * whether tile t is non-empty. */
static int tile_bounds(int n, int T, int s, int t, int* lo, int* hi) {
    s = ((s % T) + T) % T;
    int a = s + (t - 1) * T, b = s + t * T;
    if (a < 0) a = 0;
    if (b > n) b = n;
    *lo = a;
    *hi = b;
    return a < b;
}

/* One outer iteration of RAS-type temporal blocking (Sec. 4.3, Alg. 2) with
 * snapshot semantics: every tile starts from the same snapshot u = (vx, vy);
 * on its extended region E = owned box grown by h cells (clipped to the
 * domain) it runs kt damped Jacobi sweeps with every value outside E frozen
 * at u (walls 0), then writes back the unknowns of its owned box only.  The
 * tile grid is cut at positions congruent to the shift modulo the tile size,
 * so edge tiles may be partial.  Out-of-place: (ox, oy) <- RAS(vx, vy). */
void or_ras(int nx, int ny, double dx, double dy, const double* ec, const double* en, const double* bx,
            const double* by, double omega, int Tx, int Ty, int h, int kt, int sx, int sy, const double* vx,
            const double* vy, double* ox, double* oy) {
    grid_t g = mkgrid(nx, ny, dx, dy, ec, en);
    long nvx = (long)ny * (nx + 1), nvy = (long)(ny + 1) * nx;
    double* ux = malloc(sizeof(double) * nvx);
    double* uy = malloc(sizeof(double) * nvy);
    copy_state(nx, ny, vx, vy, ux, uy);
    memset(ox, 0, sizeof(double) * nvx);
    memset(oy, 0, sizeof(double) * nvy);
    int ntx = (nx + Tx - 1) / Tx + 1, nty = (ny + Ty - 1) / Ty + 1;
#pragma omp parallel for schedule(dynamic) collapse(2)
    for (int ty = 0; ty < nty; ++ty) {
        for (int tx = 0; tx < ntx; ++tx) {
            int x0, x1, y0, y1;
            if (!tile_bounds(nx, Tx, sx, tx, &x0, &x1) || !tile_bounds(ny, Ty, sy, ty, &y0, &y1)) continue;
            /* extended region E (cells) */
            int X0 = x0 - h < 0 ? 0 : x0 - h, X1 = x1 + h > nx ? nx : x1 + h;
            int Y0 = y0 - h < 0 ? 0 : y0 - h, Y1 = y1 + h > ny ? ny : y1 + h;
            /* window = E plus a one-cell ring, clipped to the arrays */
            int wx0 = X0 - 1 < 0 ? 0 : X0 - 1, wy0 = Y0 - 1 < 0 ? 0 : Y0 - 1;
            int wx1 = X1 > nx ? nx : X1, wy1 = Y1 > ny ? ny : Y1; /* inclusive */
            int W = wx1 - wx0 + 1, H = wy1 - wy0 + 1;
            double* cx = calloc((size_t)W * H, sizeof(double));
            double* cy = calloc((size_t)W * H, sizeof(double));
            double* nxv = calloc((size_t)W * H, sizeof(double));
            double* nyv = calloc((size_t)W * H, sizeof(double));
            for (int j = wy0; j <= wy1; ++j)
                for (int i = wx0; i <= wx1; ++i) {
                    long l = (long)(j - wy0) * W + (i - wx0);
                    if (j < ny) cx[l] = ux[(long)j * (nx + 1) + i];
                    if (i < nx) cy[l] = uy[(long)j * nx + i];
                }
            view_t cur = {cx, cy, wx0, wy0, W, W};
            for (int s = 0; s < kt; ++s) {
                for (int j = Y0; j < Y1; ++j)
                    for (int i = X0; i < X1; ++i) {
                        long l = (long)(j - wy0) * W + (i - wx0);
                        if (vx_unknown(&g, i, j)) nxv[l] = jac_x(&g, &cur, bx, omega, i, j);
                        if (vy_unknown(&g, i, j)) nyv[l] = jac_y(&g, &cur, by, omega, i, j);
                    }
                for (int j = Y0; j < Y1; ++j)
                    for (int i = X0; i < X1; ++i) {
                        long l = (long)(j - wy0) * W + (i - wx0);
                        if (vx_unknown(&g, i, j)) cx[l] = nxv[l];
                        if (vy_unknown(&g, i, j)) cy[l] = nyv[l];
                    }
            }
            for (int j = y0; j < y1; ++j)
                for (int i = x0; i < x1; ++i) {
                    long l = (long)(j - wy0) * W + (i - wx0);
                    if (vx_unknown(&g, i, j)) ox[(long)j * (nx + 1) + i] = cx[l];
                    if (vy_unknown(&g, i, j)) oy[(long)j * nx + i] = cy[l];
                }
            free(cx);
            free(cy);
            free(nxv);
            free(nyv);
        }
    }
    free(ux);
    free(uy);
}

/* ---------------------------------------------------------- energy norm -- */

/* Energy-norm pieces of Sec. 6.4 for the velocity state (vx, vy) and pressure
 * p (NULL = 0):
 *   r_v = b - M v  with b = f - G p,  r_p = -D v,
 *   out[0] = N_v = sum over unknowns r_v^2 / d           (||r_v||^2 in diag(-M)^-1)
 *   out[1] = N_p = sum over cells r_p^2 eta_c / (2/dx^2 + 2/dy^2)
 *   out[2] = N_f = sum over unknowns f^2 / d             (||f||^2 in diag(-M)^-1)
 *   out[3] = E   = sqrt((N_v + N_p) / N_f),  out[4] = E_v = sqrt(N_v / N_f).
 * Row partial sums are added in row order (deterministic). */
void or_energy(int nx, int ny, double dx, double dy, const double* ec, const double* en, const double* fx,
               const double* fy, const double* p, const double* vx, const double* vy, double* out) {
    grid_t g = mkgrid(nx, ny, dx, dy, ec, en);
    long nvx = (long)ny * (nx + 1), nvy = (long)(ny + 1) * nx;
    double* wx = malloc(sizeof(double) * nvx);
    double* wy = malloc(sizeof(double) * nvy);
    double* bx = malloc(sizeof(double) * nvx);
    double* by = malloc(sizeof(double) * nvy);
    double* dv = malloc(sizeof(double) * (size_t)nx * ny);
    double* part = calloc((size_t)3 * (ny + 1), sizeof(double));
    copy_state(nx, ny, vx, vy, wx, wy);
    or_rhs(nx, ny, dx, dy, fx, fy, p, bx, by);
    or_divergence(nx, ny, dx, dy, wx, wy, dv);
    view_t v = full_view(nx, wx, wy);
    double sp = 2.0 / (dx * dx) + 2.0 / (dy * dy);
#pragma omp parallel for schedule(static)
    for (int j = 0; j <= ny; ++j) {
        double nv = 0.0, np = 0.0, nf = 0.0;
        for (int i = 0; i <= nx; ++i) {
            if (j < ny && vx_unknown(&g, i, j)) {
                long k = (long)j * (nx + 1) + i;
                double d = diag_x(&g, i, j), r = bx[k] - mvx(&g, &v, i, j);
                nv += r * r / d;
                nf += fx[k] * fx[k] / d;
            }
            if (i < nx && vy_unknown(&g, i, j)) {
                long k = (long)j * nx + i;
                double d = diag_y(&g, i, j), r = by[k] - mvy(&g, &v, i, j);
                nv += r * r / d;
                nf += fy[k] * fy[k] / d;
            }
            if (j < ny && i < nx) {
                double rp = -dv[(long)j * nx + i];
                np += rp * rp * EC(&g, i, j) / sp;
            }
        }
        part[3 * j] = nv;
        part[3 * j + 1] = np;
        part[3 * j + 2] = nf;
    }
    double s[3] = {0, 0, 0};
    for (int j = 0; j <= ny; ++j)
        for (int c = 0; c < 3; ++c) s[c] += part[3 * j + c];
    out[0] = s[0];
    out[1] = s[1];
    out[2] = s[2];
    out[3] = sqrt((s[0] + s[1]) / s[2]);
    out[4] = sqrt(s[0] / s[2]);
    free(wx); free(wy); free(bx); free(by); free(dv); free(part);
}

/* ------------------------------------------------------------ multigrid -- */
/* The paper uses a matrix-free geometric multigrid for the velocity block
 * (Sec. 3.2, Sec. 6.2) but does not give its transfer operators; the oracle
 * follows this reading: coarsening by 2 in both directions, coarse cell (I,J)
 * = fine cells {2I,2I+1} x {2J,2J+1}; bilinear prolongation per component
 * (linear between coarse faces normal to the face, weights 3/4, 1/4 between
 * neighbouring coarse rows/columns tangentially, mirrored at walls); and
 * restriction R = P^T / 4.  Coarse operators are Galerkin products
 * (oracle/mg.py). */

/* Weights of the fine position f (index along one axis) on coarse positions.
 * normal=1: fine faces along their normal (n+1 faces on n cells): even f sits
 * on coarse face f/2; odd f is midway between faces (f-1)/2 and (f+1)/2.
 * normal=0: fine rows of face centres (n cells): fine f lies 1/4 coarse
 * spacing from coarse row f/2, towards row f/2-1 (even f) or f/2+1 (odd f);
 * outside the domain the neighbour is mirrored onto the row itself. */
static int axis_weights(int f, int ncoarse, int normal, int* idx, double* w) {
    if (normal) {
        if ((f & 1) == 0) { idx[0] = f / 2; w[0] = 1.0; return 1; }
        idx[0] = (f - 1) / 2; w[0] = 0.5;
        idx[1] = (f + 1) / 2; w[1] = 0.5;
        return 2;
    }
    int J = f / 2, nb = (f & 1) ? J + 1 : J - 1;
    if (nb < 0 || nb >= ncoarse) { idx[0] = J; w[0] = 1.0; return 1; }
    idx[0] = J; w[0] = 0.75;
    idx[1] = nb; w[1] = 0.25;
    return 2;
}

/* Fine <- fine + P coarse  (coarse grid NX x NY = nx/2 x ny/2). */
void or_prolong_add(int nx, int ny, const double* cx, const double* cy, double* fx, double* fy) {
    int NX = nx / 2, NY = ny / 2;
    for (int j = 0; j < ny; ++j)
        for (int i = 1; i <= nx - 1; ++i) {
            int ai[2], aj[2];
            double wi[2], wj[2];
            int ni = axis_weights(i, NX + 1, 1, ai, wi), nj = axis_weights(j, NY, 0, aj, wj);
            double s = 0.0;
            for (int a = 0; a < ni; ++a)
                for (int b = 0; b < nj; ++b) s += wi[a] * wj[b] * cx[(long)aj[b] * (NX + 1) + ai[a]];
            fx[(long)j * (nx + 1) + i] += s;
        }
    for (int j = 1; j <= ny - 1; ++j)
        for (int i = 0; i < nx; ++i) {
            int ai[2], aj[2];
            double wi[2], wj[2];
            int ni = axis_weights(i, NX, 0, ai, wi), nj = axis_weights(j, NY + 1, 1, aj, wj);
            double s = 0.0;
            for (int a = 0; a < ni; ++a)
                for (int b = 0; b < nj; ++b) s += wi[a] * wj[b] * cy[(long)aj[b] * NX + ai[a]];
            fy[(long)j * nx + i] += s;
        }
}

/* coarse <- R fine = P^T fine / 4, on coarse unknowns (coarse walls 0). */
void or_restrict(int nx, int ny, const double* fx, const double* fy, double* cx, double* cy) {
    int NX = nx / 2, NY = ny / 2;
    memset(cx, 0, sizeof(double) * (size_t)NY * (NX + 1));
    memset(cy, 0, sizeof(double) * (size_t)(NY + 1) * NX);
    for (int j = 0; j < ny; ++j)
        for (int i = 1; i <= nx - 1; ++i) {
            int ai[2], aj[2];
            double wi[2], wj[2];
            int ni = axis_weights(i, NX + 1, 1, ai, wi), nj = axis_weights(j, NY, 0, aj, wj);
            double r = fx[(long)j * (nx + 1) + i];
            for (int a = 0; a < ni; ++a)
                for (int b = 0; b < nj; ++b) cx[(long)aj[b] * (NX + 1) + ai[a]] += 0.25 * wi[a] * wj[b] * r;
        }
    for (int j = 1; j <= ny - 1; ++j)
        for (int i = 0; i < nx; ++i) {
            int ai[2], aj[2];
            double wi[2], wj[2];
            int ni = axis_weights(i, NX, 0, ai, wi), nj = axis_weights(j, NY + 1, 1, aj, wj);
            double r = fy[(long)j * nx + i];
            for (int a = 0; a < ni; ++a)
                for (int b = 0; b < nj; ++b) cy[(long)aj[b] * NX + ai[a]] += 0.25 * wi[a] * wj[b] * r;
        }
    for (int J = 0; J < NY; ++J) { cx[(long)J * (NX + 1)] = 0.0; cx[(long)J * (NX + 1) + NX] = 0.0; }
    for (int I = 0; I < NX; ++I) { cy[I] = 0.0; cy[(long)NY * NX + I] = 0.0; }
}
