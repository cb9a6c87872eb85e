"""The C-ABI library loads and exports every symbol of include/stk.h; host-only
entry points behave as documented (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "stk.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(stk_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2509_19061_amd import _lib
    return _lib


def test_library_exports_every_declared_symbol(L):
    names = header_functions()
    assert len(names) >= 10
    missing = [n for n in names if not hasattr(L.lib, n)]
    assert not missing, missing


def test_no_cpu_fallback_when_library_missing(tmp_path, monkeypatch):
    import importlib
    import sys
    import paper_2509_19061_amd._lib as mod
    monkeypatch.setattr(os.path, "exists", lambda p, _e=os.path.exists: False if p == mod.LIB_PATH else _e(p))
    sys.modules.pop("paper_2509_19061_amd._lib")
    try:
        with pytest.raises(ImportError, match="no CPU fallback"):
            importlib.import_module("paper_2509_19061_amd._lib")
    finally:
        sys.modules["paper_2509_19061_amd._lib"] = mod


def _splitmix64(seed):
    M = (1 << 64) - 1
    s = seed
    while True:
        s = (s + 0x9E3779B97F4A7C15) & M
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        yield z ^ (z >> 31)


def test_splitmix64_matches_published_vectors():
    lines = [l.strip() for l in open(os.path.join(ROOT, "tests", "golden", "splitmix64.txt")) if l.strip() and not l.startswith("#")]
    k = 0
    while k < len(lines):
        seed = int(lines[k].split()[1])
        gen = _splitmix64(seed)
        for v in lines[k + 1:k + 4]:
            assert next(gen) == int(v, 0)
        k += 4


@pytest.mark.parametrize("seed,T", [(0, 64), (3, 64), (12345, 17), (2**63 + 5, 1)])
def test_ras_shift_stream(L, seed, T):
    from paper_2509_19061_amd import api
    s = api.ras_shifts(seed, 25, T, T + 3)
    gen = _splitmix64(seed)
    for t in range(25):
        assert s[t, 0] == (next(gen) >> 32) % T
        assert s[t, 1] == (next(gen) >> 32) % (T + 3)


def test_host_side_argument_errors(L):
    g = L.Grid(8, 8, 9, 0.125, 0.125)
    rc = L.lib.stk_smooth(None, 0, C.byref(g), 1, 1, None, 1, 1, 1, 1, 1, 1, None)
    assert rc == L.EINVAL and b"ctx" in L.lib.stk_last_error()
    assert L.lib.stk_ras_shifts(0, -1, 4, 4, None) == L.EINVAL
    assert L.lib.stk_ras_shifts(0, 3, 0, 4, (C.c_int32 * 6)()) == L.EINVAL
    o = L.SmoothOpts()
    L.lib.stk_smooth_opts_default(C.byref(o))
    assert (o.omega, o.tile_x, o.tile_y, o.halo, o.k, o.seed, o.last_partial) == (0.0, 64, 64, -1, 4, 0, 1)
    assert not o.shifts
    assert L.lib.stk_ctx_destroy(None) == L.OK
    assert L.lib.stk_ctx_sync(None) == L.EINVAL


def test_uzawa_option_defaults(L):
    o = L.UzawaOpts()
    L.lib.stk_uzawa_opts_default(C.byref(o))
    assert (o.omega_p, o.vcycles, o.tol, o.max_cycles, o.stages, o.stage_cycles, o.mode) == \
        (0.6, 1, 1e-8, 1000, 0, 25, L.SOLVE_F64)


def test_mg_option_defaults(L):
    """The binding's struct and the library agree on every field, the last
    one (stall_checks) included: a sentinel behind it stays untouched."""
    class Padded(C.Structure):
        _fields_ = [("o", L.MgOpts), ("sentinel", C.c_int64)]
    p = Padded()
    p.sentinel = 0x5A5A5A5A
    p.o.stall_checks = 77
    L.lib.stk_mg_opts_default(C.byref(p.o))
    o = p.o
    assert (o.nu1, o.nu2, o.omega, o.coarsest, o.fine_k, o.fine_halo, o.coarse_smoother, o.max_levels,
            o.sweep_growth, o.stall_checks) == (2, 2, 0.7, 8, 0, -1, 0, 0, 1.0, 0)
    assert p.sentinel == 0x5A5A5A5A
