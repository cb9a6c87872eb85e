"""MI355X (gfx950) matrix-free velocity smoothers for 2D staggered-grid
variable-viscosity Stokes flow (Jacobi, fused Jacobi, RAS-type temporally
blocked Jacobi, red-black Gauss-Seidel), energy residual norms, and a
geometric multigrid solve, behind the C ABI of ``include/stk.h``.

``paper_2509_19061_amd.inputs`` (seeded synthetic problems) imports only
numpy.  The HIP binding is loaded on first use of ``api``/``fields``/``mg``;
without a built ``libstk.so`` that import fails — there is no CPU fallback.
"""
import importlib

__all__ = ["api", "fields", "inputs", "build"]


def __getattr__(name):
    if name in ("api", "fields", "inputs", "build", "mg", "serve"):
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
