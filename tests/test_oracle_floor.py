"""Where the FP64 floor of the velocity energy residual E_v (Sec. 6.4) comes
from, on the refinement workload (16 sinkers of 1e6 over a smooth
log-uniform background, contrast up to 1e8).

Flexible CG preconditioned by V-cycles drives E_v down to a floor and no
further.  Both quantities below are measured in extended precision (numpy
longdouble, a 64-bit significand), with the assembled operator of the
oracle:
- the residual of the FP64 solution the oracle reaches;
- the residual change that rounding alone causes: the solution perturbed by
  up to half a unit in the last place of FP64 in every entry.
The two agree: the floor is the FP64 representation of the solution itself,
not the arithmetic that measures it, so no residual precision or solver
change lowers it while x is stored in FP64.  Measured: 8.0e-12 against
6.6e-12 at 128^2, 3.0e-11 against 2.5e-11 at 256^2, growing about 4x per
halving of h, which puts the floor near 2-3e-8 at 8192^2 (the GPU solves
stall at 1.77e-8 there), above a tolerance of 1e-8.
"""
import numpy as np

from oracle import mg as OM
from oracle import sparse as SP
from oracle import stokes as S
from paper_2509_19061_amd import inputs as I

LD = np.longdouble


def energy_ld(A, vec, d, nf):
    """E_v of the residual-shaped vector A vec, summed in longdouble."""
    data, idx, ptr = A.data.astype(LD), A.indices, A.indptr
    av = np.add.reduceat(data * vec[idx], ptr[:-1])
    return float(np.sqrt(np.sum(av * av / d) / nf))


def test_fp64_floor_is_the_rounding_of_the_solution():
    assert np.finfo(LD).eps < 1e-18  # an extended format, else the test says nothing
    prob = I.lognormal_background_workload(128)
    levels = OM.hierarchy(prob, coarsest=32)
    vx, vy, hist = OM.pcg(levels, prob.fx, prob.fy, tol=1e-16, max_iters=500)
    L = levels[0]
    A = L.A.tocsr()  # A = -M on the packed unknowns; M x = b is A x = -b
    x = SP.pack(L.nx, L.ny, vx, vy).astype(LD)
    bx, by = S.rhs(L, prob.fx, prob.fy)
    b = SP.pack(L.nx, L.ny, bx, by).astype(LD)
    d = A.diagonal().astype(LD)
    f = SP.pack(L.nx, L.ny, prob.fx, prob.fy).astype(LD)
    nf = np.sum(f * f / d)

    data, idx, ptr = A.data.astype(LD), A.indices, A.indptr
    r = -b - np.add.reduceat(data * x[idx], ptr[:-1])
    floor = float(np.sqrt(np.sum(r * r / d) / nf))

    rng = np.random.default_rng(1)
    rounding = np.mean([energy_ld(A, x * (rng.uniform(-1, 1, x.shape) * LD(2.0 ** -53)), d, nf) for _ in range(3)])

    # the solve is at its floor: far below the start, and the FP64 measurement agrees
    assert hist[0] > 1e6 * floor
    assert 0.5 < hist[-1] / floor < 2.0
    # ... and that floor is what rounding the solution to FP64 causes
    assert 0.5 < floor / rounding < 3.0, (floor, rounding)
