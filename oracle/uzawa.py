"""FP64 inexact Uzawa iteration for the full Stokes system (test infrastructure).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline may use it; the HIP library never does.

The paper eliminates the velocity from M v + G p = f, D v = 0 (Sec. 3.1),
runs a Richardson iteration on the pressure Schur complement with the
viscosity as its diagonal approximate inverse, and solves each velocity update
only approximately with geometric multigrid (Sec. 3.2, inexact Uzawa).  Its
configuration (Sec. 6.2, 6.3) runs one V-cycle per Uzawa cycle, a pressure
relaxation omega_p = 0.6, starts from the lithostatic pressure and removes the
pressure mean after every update.

Readings taken here (the paper leaves them open):
  * sign of the update.  With G p = -grad p (the fold b = f - G p of the
    velocity block) the Schur complement D A^{-1} D^T of A = -M is positive,
    and the convergent Richardson step is p <- p + omega_p eta_c r_p with the
    continuity residual r_p = -D v of Sec. 6.4.  The paper's "+ alpha eta D v"
    is the same step in a sign convention where D carries the minus;
  * eta is the cell viscosity eta_c, where p lives;
  * lithostatic pressure: integrated from the top wall downwards so that the
    discrete vertical balance (p(i,j-1) - p(i,j))/dy = fy(i,j) holds on every
    interior vy face, then shifted to zero mean (the constant is free);
  * one Uzawa cycle: b = f - G p^k; v^{k+1} = `vcycles` V-cycles on M v = b
    from v^k; p^{k+1} = p^k + omega_p eta_c r_p(v^{k+1}); p^{k+1} -= mean;
    then the global energy residual E of Sec. 6.4 (with p^{k+1}) decides
    whether to stop.
"""
from __future__ import annotations

import numpy as np

from . import mg
from . import stokes as S


def litho(g, fy):
    """Lithostatic pressure (Sec. 6.2) balancing the vertical body force fy on
    every interior vy face, zero mean."""
    p = np.zeros((g.ny, g.nx))
    for j in range(g.ny - 1, 0, -1):        # top row first, walking down
        p[j - 1] = p[j] + np.asarray(fy)[j] * g.dy
    return p - p.mean()


def pressure_update(g, vx, vy, p, omega_p):
    """p + omega_p eta_c r_p with r_p = -D v (Sec. 3.1), then the domain mean
    removed (Sec. 6.2)."""
    q = np.asarray(p, float) + omega_p * np.asarray(g.eta_c, float) * (-S.divergence(g, vx, vy))
    return q - q.mean()


def uzawa(levels, g, fx, fy, vx, vy, p, omega_p=0.6, vcycles=1, tol=1e-8, max_cycles=100,
          nu1=2, nu2=2, omega=0.7):
    """Inexact Uzawa cycles from (vx, vy, p) until E <= tol or max_cycles.
    Returns (vx, vy, p, history of E): history[0] is E of the start, one entry
    per cycle follows."""
    vx, vy, p = np.array(vx, float), np.array(vy, float), np.array(p, float)
    hist = [S.energy(g, vx, vy, fx, fy, p)[3]]
    while hist[-1] > tol and len(hist) <= max_cycles:
        bx, by = S.rhs(g, fx, fy, p)
        for _ in range(vcycles):
            vx, vy = mg.vcycle(levels, 0, vx, vy, bx, by, nu1, nu2, omega)
        p = pressure_update(g, vx, vy, p, omega_p)
        hist.append(S.energy(g, vx, vy, fx, fy, p)[3])
    return vx, vy, p, hist


def rescaled(g, theta, eta_min=None):
    """The problem with the computational viscosity of Sec. 6.2,
    (1 - theta) eta_min + theta eta, applied to the cell and to the nodal
    viscosities alike; eta_min = the smallest cell viscosity."""
    from types import SimpleNamespace
    em = float(np.min(g.eta_c)) if eta_min is None else eta_min
    return SimpleNamespace(nx=g.nx, ny=g.ny, dx=g.dx, dy=g.dy,
                           eta_c=(1.0 - theta) * em + theta * np.asarray(g.eta_c, float),
                           eta_n=(1.0 - theta) * em + theta * np.asarray(g.eta_n, float))


def uzawa_continuation(g, fx, fy, vx, vy, p, stages=4, stage_cycles=25, omega_p=0.6, vcycles=1, tol=1e-8,
                       max_cycles=1000, coarsest=8, nu1=2, nu2=2, omega=0.7):
    """Uzawa cycles under viscosity continuation (Sec. 6.2): theta = s/stages
    for s = 0 .. stages; every stage with theta < 1 runs stage_cycles cycles
    on the rescaled system (its own hierarchy, and its eta_c in the pressure
    step); the last stage (theta = 1, the true system) runs until E <= tol.
    max_cycles bounds all cycles together.  history[k] is E of the TRUE
    system after k cycles."""
    vx, vy, p = np.array(vx, float), np.array(vy, float), np.array(p, float)
    hist = [S.energy(g, vx, vy, fx, fy, p)[3]]
    for s in range(stages + 1):
        theta = s / stages if stages > 0 else 1.0
        gs = rescaled(g, theta)
        levels = mg.hierarchy(gs, coarsest)
        last, n = s == stages, 0
        while len(hist) <= max_cycles and (hist[-1] > tol if last else n < stage_cycles):
            bx, by = S.rhs(gs, fx, fy, p)
            for _ in range(vcycles):
                vx, vy = mg.vcycle(levels, 0, vx, vy, bx, by, nu1, nu2, omega)
            p = pressure_update(gs, vx, vy, p, omega_p)
            hist.append(S.energy(g, vx, vy, fx, fy, p)[3])
            n += 1
    return vx, vy, p, hist


def _cycle(levels, g, fx, fy, vx, vy, p, omega_p, vcycles, nu1, nu2, omega):
    """F(x): one inexact Uzawa cycle from x = (vx, vy, p)."""
    bx, by = S.rhs(g, fx, fy, p)
    for _ in range(vcycles):
        vx, vy = mg.vcycle(levels, 0, vx, vy, bx, by, nu1, nu2, omega)
    return vx, vy, pressure_update(g, vx, vy, p, omega_p)


def anderson_weights(R):
    """alpha = argmin ||R alpha||_2 subject to sum(alpha) = 1 (Alg. 1), from the
    stationarity conditions of the Lagrangian: [H 1; 1^T 0] [alpha; mu] =
    [0; 1] with the Gram matrix H = R^T R (scaled by its largest diagonal
    entry, which leaves alpha unchanged).  A singular system falls back to
    alpha = (0, .., 0, 1), the plain step."""
    H = R.T @ R
    n = H.shape[0]
    s = np.max(np.diag(H))
    if not np.isfinite(s) or s <= 0.0:
        return np.eye(n)[-1]
    K = np.zeros((n + 1, n + 1))
    K[:n, :n] = H / s
    K[:n, n] = 1.0
    K[n, :n] = 1.0
    rhs = np.zeros(n + 1)
    rhs[n] = 1.0
    try:
        a = np.linalg.solve(K, rhs)[:n]
    except np.linalg.LinAlgError:
        return np.eye(n)[-1]
    return a if np.all(np.isfinite(a)) else np.eye(n)[-1]


def _anderson_steps(levels, gs, g, fx, fy, x, hist, m, omega_p, vcycles, nu1, nu2, omega, more):
    """Anderson steps on the system gs (hierarchy `levels`) from x, while
    more(n) holds (n = steps taken here); E of the true system g is appended
    to hist after every step."""
    def flat(y):
        return np.concatenate([np.ravel(y[0]), np.ravel(y[1]), np.ravel(y[2])])

    Fs, rs, n = [], [], 0
    while more(n):
        fxk = _cycle(levels, gs, fx, fy, *x, omega_p, vcycles, nu1, nu2, omega)
        Fs.append(fxk)
        rs.append(flat(fxk) - flat(x))
        k = len(Fs) - 1                      # the index of x_k
        if k == 0:
            x = fxk                          # x_1 = F(x_0)
        else:
            mk = min(m, k)
            Fs, rs = Fs[-(mk + 1):], rs[-(mk + 1):]
            a = anderson_weights(np.stack(rs, axis=1))
            x = tuple(sum(a[i] * Fs[i][c] for i in range(mk + 1)) for c in range(3))
        hist.append(S.energy(g, *x[:2], fx, fy, x[2])[3])
        n += 1
    return x


def anderson(levels, g, fx, fy, vx, vy, p, m=3, omega_p=0.6, vcycles=1, tol=1e-8, max_iters=200, nu1=2, nu2=2,
             omega=0.7):
    """Anderson acceleration of the inexact Uzawa fixed-point map F on
    x = [v, p] (Sec. 3.3, Alg. 1): x_1 = F(x_0); then with m_k = min(m, k),
    r_i = F(x_i) - x_i, the new iterate is the combination of the last m_k + 1
    values F(x_i) whose weights (summing to 1) minimise the l2 norm of the
    same combination of the r_i.  The norm runs over every velocity unknown
    and pressure cell as one vector.  Stops when E of the new iterate <= tol.
    Returns (vx, vy, p, history of E), one entry per F evaluation after the
    start's."""
    x = (np.array(vx, float), np.array(vy, float), np.array(p, float))
    hist = [S.energy(g, *x[:2], fx, fy, x[2])[3]]
    x = _anderson_steps(levels, g, g, fx, fy, x, hist, m, omega_p, vcycles, nu1, nu2, omega,
                        lambda n: hist[-1] > tol and len(hist) <= max_iters)
    return x[0], x[1], x[2], hist


def anderson_continuation(g, fx, fy, vx, vy, p, m=3, stages=4, stage_cycles=25, omega_p=0.6, vcycles=1, tol=1e-8,
                          max_iters=1000, coarsest=8, nu1=2, nu2=2, omega=0.7):
    """Anderson steps under the viscosity continuation of Sec. 6.2: each
    stage theta = s/stages < 1 runs stage_cycles steps on the rescaled system
    (its own hierarchy; the Anderson history restarts with the stage, whose
    map differs), then the true system runs until E <= tol.  max_iters bounds
    all steps together; history[k] is E of the TRUE system."""
    x = (np.array(vx, float), np.array(vy, float), np.array(p, float))
    hist = [S.energy(g, *x[:2], fx, fy, x[2])[3]]
    for s in range(stages + 1):
        theta = s / stages if stages > 0 else 1.0
        gs = rescaled(g, theta)
        last = s == stages
        x = _anderson_steps(mg.hierarchy(gs, coarsest), gs, g, fx, fy, x, hist, m, omega_p, vcycles, nu1, nu2, omega,
                            lambda n: len(hist) <= max_iters and (hist[-1] > tol if last else n < stage_cycles))
    return x[0], x[1], x[2], hist
