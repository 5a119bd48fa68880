"""ctypes binding of the C ABI in include/rt.h (argument marshalling only).

Every numerical step runs in the HIP library librt355.so; this module only
converts Python arguments into the C structs and device pointers.  Loading
fails loudly when the library has not been built.
"""
import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librt355.so")

# enums of rt.h
RT_OK, RT_W_NEWTON = 0, 1
RT_E_ARG, RT_E_STATE, RT_E_HIP, RT_E_NOMEM, RT_E_NONFINITE = -1, -2, -3, -4, -5
RT_CART, RT_LOGR_THETA_PHI = 0, 1
RT_BC_PERIODIC, RT_BC_OUTFLOW, RT_BC_ZERO_INCOMING = 0, 1, 2
RT_W_VORONOI, RT_W_EQUAL = 0, 1
RT_FP64, RT_FP32_TRANSPORT = 0, 1
RT_LIM_MC, RT_LIM_MINMOD = 0, 1
RT_AREC_DONOR, RT_AREC_MAPR = 0, 1
RT_FLAT, RT_KERR_SCHILD = 0, 1
RT_OPAC_KIRCHHOFF_CONST, RT_OPAC_BREMS, RT_OPAC_FIXED_EMISSIVITY, RT_OPAC_BREMS_M3 = 0, 1, 2, 3
RT_TETRAD, RT_COORD = 0, 1
KERNELS = ["stage1", "stage2", "materialize", "moments", "adjoint", "angular", "mg_solve"]

EXPORTED = ["rt_init_grid", "rt_geodesic_grid", "rt_grid_info", "rt_set_metric", "rt_set_opacities", "rt_set_groups", "rt_step",
            "rt_step_noalloc", "rt_moments", "rt_step_adjoint", "rt_step_adjoint_thermal", "rt_set_debug", "rt_kernel_times", "rt_newton_failures",
            "rt_destroy", "rt_last_error"]


class GridDesc(C.Structure):
    _fields_ = [("n", C.c_int * 3), ("xlo", C.c_double * 3), ("xhi", C.c_double * 3),
                ("coords", C.c_int), ("bc_lo", C.c_int * 3), ("bc_hi", C.c_int * 3),
                ("generation", C.c_int), ("weights", C.c_int), ("precision", C.c_int),
                ("limiter", C.c_int), ("angular_recon", C.c_int), ("abar", C.c_double),
                ("rho_floor", C.c_double), ("n0_cut", C.c_double), ("pole_zero_rows", C.c_int)]


class OpacityDesc(C.Structure):
    _fields_ = [("model", C.c_int), ("gamma", C.c_double), ("C_a", C.c_double),
                ("C_s", C.c_double), ("rho", C.c_void_p), ("u", C.c_void_p),
                ("kappa_a", C.c_void_p), ("kappa_s", C.c_void_p), ("j", C.c_void_p),
                ("newton_max_iter", C.c_int), ("newton_rtol", C.c_double)]


_lib = None


def load():
    """Load librt355.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run python -m paper_2508_15532_amd.build)")
    import torch  # noqa: F401  (loads the HIP runtime the library links against)
    lib = C.CDLL(LIB_PATH)
    P, I, D = C.c_void_p, C.c_int, C.c_double
    sig = {
        "rt_init_grid": ([C.POINTER(GridDesc), C.POINTER(P)], I),
        "rt_geodesic_grid": ([I, I, C.POINTER(I), P, P, P], I),
        "rt_grid_info": ([P, C.POINTER(I), P, P, P], I),
        "rt_set_metric": ([P, I, D, D, D, C.POINTER(D)], I),
        "rt_set_opacities": ([P, C.POINTER(OpacityDesc), P], I),
        "rt_set_groups": ([P, I, P, P, P], I),
        "rt_step": ([P, P, P, D, I, P, P, P], I),
        "rt_step_noalloc": ([P, P, P, D, I, P, P, P], I),
        "rt_moments": ([P, P, P, P, I, P], I),
        "rt_step_adjoint": ([P, P, P, D, P, P, P, P, P], I),
        "rt_step_adjoint_thermal": ([P, P, P, D, P, P, P, P, P, P], I),
        "rt_set_debug": ([P, I], I),
        "rt_kernel_times": ([P, P, P], I),
        "rt_newton_failures": ([P, C.POINTER(C.c_longlong)], I),
        "rt_destroy": ([P], None),
        "rt_last_error": ([], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


class RTError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"status {status}: {msg}")
        self.status = status


def check(status, allow_warning=False):
    if status == RT_OK or (allow_warning and status > 0):
        return status
    raise RTError(status, load().rt_last_error().decode())
