"""ctypes binding of ``libstk.so`` (include/stk.h): argument marshalling only.

Every compute step runs in the HIP library.  If the library is not built
this module raises at import time — there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstk.so")

OK, EINVAL, ENOMEM, EHIP, ENOTCONV, ENONFINITE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
F64, F32 = 0, 1
JACOBI, JACOBI_FUSED, RAS_JACOBI, RBGS = 0, 1, 2, 3
VARIANTS = {"jacobi": JACOBI, "jacobi_fused": JACOBI_FUSED, "ras": RAS_JACOBI, "rbgs": RBGS}


class StkError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"stk error {code}: {msg}")
        self.code = code


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("ld", C.c_int64), ("dx", C.c_double), ("dy", C.c_double)]


class SmoothOpts(C.Structure):
    _fields_ = [("omega", C.c_double), ("tile_x", C.c_int), ("tile_y", C.c_int), ("halo", C.c_int), ("k", C.c_int),
                ("shifts", C.POINTER(C.c_int32)), ("seed", C.c_uint64), ("last_partial", C.c_int)]


class MgOpts(C.Structure):
    _fields_ = [("nu1", C.c_int), ("nu2", C.c_int), ("omega", C.c_double), ("coarsest", C.c_int),
                ("fine_k", C.c_int), ("fine_halo", C.c_int), ("coarse_smoother", C.c_int), ("coarse_tile", C.c_int),
                ("coarse_k", C.c_int), ("coarse_halo", C.c_int), ("sweep_growth", C.c_double),
                ("max_levels", C.c_int), ("stall_checks", C.c_int)]


class Report(C.Structure):
    _fields_ = [("iterations", C.c_int), ("converged", C.c_int), ("ev", C.c_double), ("nf", C.c_double),
                ("seconds", C.c_double)]


class Grid3(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("ld", C.c_int64), ("lp", C.c_int64),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double)]


class Smooth3dOpts(C.Structure):
    _fields_ = [("omega", C.c_double), ("tile", C.c_int), ("halo", C.c_int), ("k", C.c_int),
                ("shifts", C.POINTER(C.c_int32)), ("seed", C.c_uint64)]


class UzawaOpts(C.Structure):
    _fields_ = [("omega_p", C.c_double), ("vcycles", C.c_int), ("tol", C.c_double), ("max_cycles", C.c_int),
                ("stages", C.c_int), ("stage_cycles", C.c_int), ("mode", C.c_int)]


class UzawaReport(C.Structure):
    _fields_ = [("cycles", C.c_int), ("converged", C.c_int), ("e", C.c_double), ("ev", C.c_double),
                ("seconds", C.c_double)]


SOLVE_F64, SOLVE_F32_REFINED = 0, 1

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2509_19061_amd.build` "
                      "(there is no CPU fallback)")

lib = C.CDLL(LIB_PATH)

_P = C.c_void_p
_I = C.c_int
_G = C.POINTER(Grid)

_SIGS = {
    "stk_ctx_create": ([C.POINTER(_P), _I, _P], _I),
    "stk_ctx_destroy": ([_P], _I),
    "stk_ctx_set_stream": ([_P, _P], _I),
    "stk_ctx_sync": ([_P], _I),
    "stk_ctx_scratch_bytes": ([_P, C.POINTER(C.c_size_t)], _I),
    "stk_last_error": ([], C.c_char_p),
    "stk_smooth_opts_default": ([C.POINTER(SmoothOpts)], None),
    "stk_smooth": ([_P, _I, _G, _P, _P, _P, _P, _P, _P, _P, _I, _I, C.POINTER(SmoothOpts)], _I),
    "stk_ras_shifts": ([C.c_uint64, _I, _I, _I, C.POINTER(C.c_int32)], _I),
    "stk_ras_outer": ([_P, _I, _G, _P, _P, _P, _P, _P, _P, _P, _P, C.c_double, _I, _I, _I, _I, _I, _I], _I),
    "stk_residual": ([_P, _I, _G, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P], _I),
    "stk_energy_norm": ([_P, _I, _G, _P, _P, _P, _P, _P, _P, _P, C.POINTER(C.c_double)], _I),
    "stk_energy_norm_noalloc": ([_P, _I, _G, _P, _P, _P, _P, _P, _P, _P, _P], _I),
    "stk_stream_probe": ([_P, _I, _G, _P, _P, _P, _P, _P, _P, _P, _P], _I),
    "stk_smooth3d_opts_default": ([C.POINTER(Smooth3dOpts)], None),
    "stk_smooth3d": ([_P, _I, C.POINTER(Grid3)] + [_P] * 10 + [_I, _I, C.POINTER(Smooth3dOpts)], _I),
    "stk_ras_outer3d": ([_P, _I, C.POINTER(Grid3)] + [_P] * 13 + [C.c_double, _I, _I, _I, _I, _I, _I], _I),
    "stk_residual3d": ([_P, _I, C.POINTER(Grid3)] + [_P] * 13, _I),
    "stk_energy_norm3d": ([_P, _I, C.POINTER(Grid3)] + [_P] * 10 + [C.POINTER(C.c_double)], _I),
    "stk_mg_opts_default": ([C.POINTER(MgOpts)], None),
    "stk_mg_create": ([_P, C.POINTER(_P), _G, _P, _P, C.POINTER(MgOpts)], _I),
    "stk_mg_destroy": ([_P], _I),
    "stk_mg_bind": ([_P, _P, _I], _I),
    "stk_mg_info": ([_P, C.POINTER(_I), C.POINTER(_I), C.POINTER(C.c_size_t)], _I),
    "stk_mg_footprint": ([_G, C.POINTER(MgOpts), _I, C.POINTER(C.c_size_t)], _I),
    "stk_mg_vcycle": ([_P, _I, _P, _P, _P, _P], _I),
    "stk_mg_solve": ([_P, _I, _P, _P, _P, _P, _P, C.c_double, _I, C.POINTER(Report)], _I),
    "stk_mg_solve_batch": ([_P, _I, C.POINTER(_P), _I, C.POINTER(_P), C.POINTER(_P), C.POINTER(_P), C.POINTER(_P),
                            C.POINTER(_P), C.c_double, _I, C.POINTER(Report)], _I),
    "stk_batch_create": ([_P, _I, _I, C.POINTER(_P)], _I),
    "stk_batch_destroy": ([_P], _I),
    "stk_batch_add": ([_P, _P, _P, _P, _P, _P, _P, C.c_double, _I, C.POINTER(_I)], _I),
    "stk_batch_step": ([_P, _I, C.POINTER(_I), C.POINTER(Report), C.POINTER(_I)], _I),
    "stk_batch_count": ([_P, C.POINTER(_I)], _I),
    "stk_uzawa_opts_default": ([C.POINTER(UzawaOpts)], None),
    "stk_litho_pressure": ([_P, _G, _P, _P], _I),
    "stk_uzawa_pressure": ([_P, _G, _P, _P, _P, C.c_double, _P], _I),
    "stk_uzawa_solve": ([_P, _G, _P, _P, _P, _P, _P, _P, _P, C.POINTER(UzawaOpts), C.POINTER(C.c_double),
                         C.POINTER(UzawaReport)], _I),
    "stk_uzawa_anderson": ([_P, _G, _P, _P, _P, _P, _P, _P, _P, _I, C.POINTER(UzawaOpts), C.POINTER(C.c_double),
                            C.POINTER(UzawaReport)], _I),
}


def _bind(sigs):
    for name, (args, res) in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res


_bind(_SIGS)


def check(rc):
    if rc != OK:
        raise StkError(rc, lib.stk_last_error().decode())
    return rc
