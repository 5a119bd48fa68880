"""MI355X-native gray covariant radiative transfer on a geodesic angular grid.

Python binding of the HIP library (include/rt.h).  Tensors are torch CUDA
(HIP) tensors used only as device memory; work is enqueued on torch's current
stream.  Every numerical step of the method runs in librt355.so.
"""
import ctypes as C

import numpy as np

from . import _native as N
from ._native import RTError  # noqa: F401

_BC = {"periodic": N.RT_BC_PERIODIC, "outflow": N.RT_BC_OUTFLOW,
       "zero_incoming": N.RT_BC_ZERO_INCOMING}
_MODEL = {"kirchhoff_const": N.RT_OPAC_KIRCHHOFF_CONST, "brems": N.RT_OPAC_BREMS,
          "fixed_emissivity": N.RT_OPAC_FIXED_EMISSIVITY, "brems_m3": N.RT_OPAC_BREMS_M3}
_PREC = {"fp64": N.RT_FP64, "fp32": N.RT_FP32_TRANSPORT}


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, name, dtype=None, numel=None, optional=False):
    import torch
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    if t.data_ptr() % 256:
        raise ValueError(f"{name} must be 256-byte aligned")
    return C.c_void_p(t.data_ptr())


def geodesic_grid(generation, weights="voronoi"):
    """Host-only: (directions [Ns,3], weights [Ns], solid angles [Ns]) of the
    library's geodesic grid (no GPU needed)."""
    lib = N.load()
    ns = 10 * 4 ** int(generation) + 2
    dirs, w, area = np.zeros((ns, 3)), np.zeros(ns), np.zeros(ns)
    n = C.c_int()
    N.check(lib.rt_geodesic_grid(int(generation), {"voronoi": N.RT_W_VORONOI, "equal": N.RT_W_EQUAL}[weights],
                                 C.byref(n), dirs.ctypes.data_as(C.c_void_p), w.ctypes.data_as(C.c_void_p),
                                 area.ctypes.data_as(C.c_void_p)))
    assert n.value == ns
    return dirs, w, area


class RTContext:
    """One problem: mesh, angular grid, metric, fluid and opacity model."""

    def __init__(self, n, xlo, xhi, generation, *, weights="voronoi", precision="fp64",
                 bc=("periodic",) * 3, bc_hi=None, limiter="mc", abar=1.0, rho_floor=5e-4,
                 n0_cut=0.1, coords="cart", pole_zero_rows=None, angular_recon="donor"):
        self._lib = N.load()
        d = N.GridDesc()
        bc_hi = bc if bc_hi is None else bc_hi
        for a in range(3):
            d.n[a] = int(n[a])
            d.xlo[a] = float(xlo[a])
            d.xhi[a] = float(xhi[a])
            d.bc_lo[a] = _BC[bc[a]]
            d.bc_hi[a] = _BC[bc_hi[a]]
        d.coords = {"cart": N.RT_CART, "logr_theta_phi": N.RT_LOGR_THETA_PHI}[coords]
        d.generation = int(generation)
        d.weights = {"voronoi": N.RT_W_VORONOI, "equal": N.RT_W_EQUAL}[weights]
        d.precision = _PREC[precision]
        d.limiter = {"mc": N.RT_LIM_MC, "minmod": N.RT_LIM_MINMOD}[limiter]
        d.angular_recon = {"donor": N.RT_AREC_DONOR, "mapr": N.RT_AREC_MAPR}[angular_recon]
        d.abar, d.rho_floor, d.n0_cut = float(abar), float(rho_floor), float(n0_cut)
        if pole_zero_rows is None:
            pole_zero_rows = 4 if coords == "logr_theta_phi" else 0
        d.pole_zero_rows = int(pole_zero_rows)
        ctx = C.c_void_p()
        N.check(self._lib.rt_init_grid(C.byref(d), C.byref(ctx)))
        self._ctx = ctx
        self.n = tuple(int(x) for x in n)
        self.nc = int(np.prod(self.n))
        self.precision = precision
        ns = C.c_int()
        N.check(self._lib.rt_grid_info(ctx, C.byref(ns), None, None, None))
        self.ns = ns.value
        self._keep = []
        self.dt_max = None
        self.ng = 0

    # -- grid ---------------------------------------------------------------
    def grid(self):
        """(directions [Ns,3], weights [Ns], Voronoi solid angles [Ns]) as numpy."""
        dirs = np.zeros((self.ns, 3))
        w = np.zeros(self.ns)
        area = np.zeros(self.ns)
        N.check(self._lib.rt_grid_info(self._ctx, None, dirs.ctypes.data_as(C.c_void_p),
                                       w.ctypes.data_as(C.c_void_p), area.ctypes.data_as(C.c_void_p)))
        return dirs, w, area

    @property
    def intensity_dtype(self):
        import torch
        return torch.float32 if self.precision == "fp32" else torch.float64

    # -- setup ----------------------------------------------------------------
    def set_metric(self, kind="flat", M=1.0, a=0.0, cfl=0.4):
        dt = C.c_double()
        k = {"flat": N.RT_FLAT, "kerr_schild": N.RT_KERR_SCHILD}[kind]
        N.check(self._lib.rt_set_metric(self._ctx, k, float(M), float(a), float(cfl), C.byref(dt)))
        self.dt_max = dt.value
        return self.dt_max

    def set_opacities(self, model, rho, u=None, kappa_a=None, kappa_s=None, j=None,
                      gamma=5.0 / 3.0, C_a=1.0, C_s=1.0, newton_max_iter=50, newton_rtol=1e-14):
        import torch
        f64 = torch.float64
        o = N.OpacityDesc()
        o.model = _MODEL[model]
        o.gamma, o.C_a, o.C_s = float(gamma), float(C_a), float(C_s)
        o.rho = _ptr(rho, "rho", f64, self.nc)
        o.u = _ptr(u, "u", f64, 4 * self.nc, optional=True)
        o.kappa_a = _ptr(kappa_a, "kappa_a", f64, self.nc, optional=True)
        o.kappa_s = _ptr(kappa_s, "kappa_s", f64, self.nc, optional=True)
        o.j = _ptr(j, "j", f64, self.nc, optional=True)
        o.newton_max_iter, o.newton_rtol = int(newton_max_iter), float(newton_rtol)
        N.check(self._lib.rt_set_opacities(self._ctx, C.byref(o), _stream()))
        # the copies are asynchronous: keep the sources alive until the stream passes
        self._keep = [rho, u, kappa_a, kappa_s, j]

    def set_groups(self, edges, kappa_a_groups):
        """Frequency bins (fluid at rest, flat space): edges, G + 1 increasing
        values (the last may be inf), kappa_a_groups [G, *n] float64 (per-bin
        absorption opacity).  Afterwards step() takes I as [G, Ns, *n] and
        returns R and G summed over the bins.  edges=None switches back to gray."""
        import torch
        if edges is None:
            N.check(self._lib.rt_set_groups(self._ctx, 0, None, None, _stream()))
            self.ng = 0
            return
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.float64).reshape(-1))
        ng = e.size - 1
        if ng < 1:
            raise ValueError("edges needs at least two values (one bin); edges=None means gray")
        ka = _ptr(kappa_a_groups, "kappa_a_groups", torch.float64, ng * self.nc)
        N.check(self._lib.rt_set_groups(self._ctx, int(ng), e.ctypes.data_as(C.c_void_p), ka, _stream()))
        self.ng = ng
        self._keep_groups = kappa_a_groups

    # -- hot path -------------------------------------------------------------
    def step(self, I, T, dt, nsteps=1, G=None, R=None):
        """Advance (I, T) in place by nsteps predictor-corrector steps; optional
        G [4, Nc] (4-force of the last step) and R [10, Nc] (moments of the new
        intensity) are filled in."""
        import torch
        st = self._lib.rt_step(self._ctx, _ptr(I, "I", self.intensity_dtype, max(self.ng, 1) * self.ns * self.nc),
                               _ptr(T, "T", torch.float64, self.nc), float(dt), int(nsteps),
                               _ptr(G, "G", torch.float64, 4 * self.nc, optional=True),
                               _ptr(R, "R", torch.float64, 10 * self.nc, optional=True), _stream())
        return N.check(st, allow_warning=True)

    def step_noalloc(self, I, T, dt, nsteps=1, G=None, R=None):
        """As step(), through rt_step_noalloc: the step scratch is the library's
        static per-device array (no device allocation in the call)."""
        import torch
        st = self._lib.rt_step_noalloc(self._ctx, _ptr(I, "I", self.intensity_dtype,
                                                       max(self.ng, 1) * self.ns * self.nc),
                                       _ptr(T, "T", torch.float64, self.nc), float(dt), int(nsteps),
                                       _ptr(G, "G", torch.float64, 4 * self.nc, optional=True),
                                       _ptr(R, "R", torch.float64, 10 * self.nc, optional=True), _stream())
        return N.check(st, allow_warning=True)

    def moments(self, I, R=None, J=None, frame="tetrad"):
        """R [10, *n] float64 (00,01,02,03,11,12,13,22,23,33) of I; optional J [*n]."""
        import torch
        if R is None:
            R = torch.empty((10,) + self.n, dtype=torch.float64, device=I.device)
        N.check(self._lib.rt_moments(self._ctx, _ptr(I, "I", self.intensity_dtype, self.ns * self.nc),
                                     _ptr(R, "R", torch.float64, 10 * self.nc),
                                     _ptr(J, "J", torch.float64, self.nc, optional=True),
                                     {"tetrad": N.RT_TETRAD, "coord": N.RT_COORD}[frame], _stream()))
        return R

    def step_adjoint(self, I_n, T_n, dt, gI_np1, gI_n=None, g_kappa_a=None, g_j=None):
        """Reverse of one step: returns gI_n (may be gI_np1 itself); accumulates
        into g_kappa_a and g_j."""
        import torch
        if gI_n is None:
            gI_n = torch.empty_like(gI_np1)
        dt_i = self.intensity_dtype
        N.check(self._lib.rt_step_adjoint(
            self._ctx, _ptr(I_n, "I_n", dt_i, self.ns * self.nc),
            _ptr(T_n, "T_n", torch.float64, self.nc, optional=True), float(dt),
            _ptr(gI_np1, "gI_np1", dt_i, self.ns * self.nc), _ptr(gI_n, "gI_n", dt_i, self.ns * self.nc),
            _ptr(g_kappa_a, "g_kappa_a", torch.float64, self.nc, optional=True),
            _ptr(g_j, "g_j", torch.float64, self.nc, optional=True), _stream()))
        return gI_n

    def step_adjoint_thermal(self, I_n, T_n, dt, gI_np1, gT_np1=None, gI_n=None, gT_n=None, g_kappa_a=None):
        """Reverse of one step of the bremsstrahlung model: returns (gI_n, gT_n);
        accumulates into g_kappa_a (the per-cell opacity factor's gradient)."""
        import torch
        if gI_n is None:
            gI_n = torch.empty_like(gI_np1)
        if gT_n is None:
            gT_n = torch.empty_like(T_n)
        dt_i, f64 = self.intensity_dtype, torch.float64
        N.check(self._lib.rt_step_adjoint_thermal(
            self._ctx, _ptr(I_n, "I_n", dt_i, self.ns * self.nc), _ptr(T_n, "T_n", f64, self.nc), float(dt),
            _ptr(gI_np1, "gI_np1", dt_i, self.ns * self.nc), _ptr(gT_np1, "gT_np1", f64, self.nc, optional=True),
            _ptr(gI_n, "gI_n", dt_i, self.ns * self.nc), _ptr(gT_n, "gT_n", f64, self.nc),
            _ptr(g_kappa_a, "g_kappa_a", f64, self.nc, optional=True), _stream()))
        return gI_n, gT_n

    def set_debug(self, flags=1):
        N.check(self._lib.rt_set_debug(self._ctx, int(flags)))

    def kernel_times(self):
        """{kernel kind: (launches, total ms)} since the previous call (timing
        is on when set_debug(flags) has bit 1 set)."""
        k = len(N.KERNELS)
        counts = (C.c_int * k)()
        ms = (C.c_double * k)()
        N.check(self._lib.rt_kernel_times(self._ctx, counts, ms))
        return {name: (counts[i], ms[i]) for i, name in enumerate(N.KERNELS)}

    def newton_failures(self):
        n = C.c_longlong()
        N.check(self._lib.rt_newton_failures(self._ctx, C.byref(n)))
        return n.value

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.rt_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
