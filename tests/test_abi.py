"""C-ABI library checks that need no GPU: it loads, exports every symbol that
include/rt.h declares, rejects bad arguments before touching the device, and
its host-side geodesic grid agrees with the oracle's independent construction."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rt.h")


def _lib():
    from paper_2508_15532_amd import _native as N
    return N, N.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rt_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    N, lib = _lib()
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(N.EXPORTED) == names


def test_null_arguments_are_rejected_without_device_work():
    N, lib = _lib()
    assert lib.rt_init_grid(None, None) == N.RT_E_ARG
    ctx = C.c_void_p()
    assert lib.rt_init_grid(None, C.byref(ctx)) == N.RT_E_ARG
    assert ctx.value is None
    assert b"NULL" in lib.rt_last_error()
    assert lib.rt_set_metric(None, 0, 1.0, 0.0, 0.4, None) == N.RT_E_ARG
    assert lib.rt_step(None, None, None, 0.1, 1, None, None, None) == N.RT_E_ARG
    assert lib.rt_moments(None, None, None, None, 0, None) == N.RT_E_ARG
    assert lib.rt_step_adjoint(None, None, None, 0.1, None, None, None, None, None) == N.RT_E_ARG
    lib.rt_destroy(None)


def _desc(N, **kw):
    d = N.GridDesc()
    for a in range(3):
        d.n[a], d.xlo[a], d.xhi[a] = 4, 0.0, 4.0
    d.generation, d.abar, d.rho_floor, d.n0_cut = 1, 1.0, 5e-4, 0.1
    for k, v in kw.items():
        if k == "n":
            for a in range(3):
                d.n[a] = v[a]
        elif k in ("bc_lo", "bc_hi"):
            arr = getattr(d, k)
            for a in range(3):
                arr[a] = v[a]
        else:
            setattr(d, k, v)
    return d


@pytest.mark.parametrize("kw,msg", [
    (dict(n=(0, 4, 4)), b"n[a]"),
    (dict(generation=6), b"generation"),
    (dict(precision=7), b"precision"),
    (dict(limiter=3), b"limiter"),
    (dict(angular_recon=2), b"angular_recon"),
    (dict(bc_lo=(0, 0, 0), bc_hi=(1, 0, 0)), b"periodic"),
    (dict(coords=5), b"coords"),
    (dict(weights=4), b"weights"),
    (dict(coords=1, pole_zero_rows=3), b"pole_zero_rows"),
    (dict(coords=0, pole_zero_rows=1), b"pole_zero_rows"),
    (dict(n0_cut=-1.0), b"n0_cut"),
    # one direction's plane must stay below 4 GiB (32-bit byte offsets in the stage kernels)
    (dict(n=(1024, 1024, 512)), b"2^29"),
])
def test_bad_descriptors_are_rejected(kw, msg):
    N, lib = _lib()
    ctx = C.c_void_p()
    d = _desc(N, **kw)
    assert lib.rt_init_grid(C.byref(d), C.byref(ctx)) == N.RT_E_ARG
    assert msg in lib.rt_last_error()
    assert ctx.value is None


@pytest.mark.parametrize("g", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("weights", ["voronoi", "equal"])
def test_host_grid_matches_oracle_grid(g, weights):
    """The library's C++ grid builder and the oracle's numpy builder are
    independent implementations of the same numbering convention."""
    from oracle.grid import GeodesicGrid
    import paper_2508_15532_amd as P
    dirs, w, area = P.geodesic_grid(g, weights)
    G = GeodesicGrid(g, weights)
    assert dirs.shape == G.n.shape
    assert np.abs(dirs - G.n).max() < 1e-15
    assert np.abs(w - G.w).max() < 1e-14
    assert np.abs(area - G.area).max() < 1e-14
    assert abs(w.sum() - 4 * np.pi) < 1e-12


def test_host_grid_rejects_bad_generation():
    N, lib = _lib()
    n = C.c_int()
    assert lib.rt_geodesic_grid(9, 0, C.byref(n), None, None, None) == N.RT_E_ARG
