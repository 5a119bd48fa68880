"""Turn a workload description (plain dict of numpy fields) into oracle inputs.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
import numpy as np
import torch

from . import interaction as src
from . import transport as tr
from .geometry import FlatCartesian
from .grid import GeodesicGrid
from .step import Problem

F64 = torch.float64
BC = {"periodic": tr.PERIODIC, "outflow": tr.OUTFLOW, "zero_incoming": tr.ZERO_INCOMING}
MODEL = {"kirchhoff_const": src.KIRCHHOFF_CONST, "brems": src.BREMS,
         "fixed_emissivity": src.FIXED_EMISSIVITY, "brems_m3": src.BREMS_M3}


def _t(x):
    return None if x is None else torch.as_tensor(np.asarray(x, dtype=np.float64))


def build_flat(wl, grid=None, limiter=tr.LIM_MC):
    """Problem, initial intensity [Ns,*n] (isotropic I0_iso) and temperature."""
    grid = grid or GeodesicGrid(wl["generation"], wl["weights"])
    geo = FlatCartesian(wl["n"], wl["xlo"], wl["xhi"], grid)
    shape = tuple(wl["n"])
    rho = _t(wl["rho"])
    if wl.get("u") is None:
        u_hat = torch.zeros((4,) + shape, dtype=F64)
        u_hat[0] = 1.0
    else:
        u_hat = geo.u_hat(_t(wl["u"]))
    v = u_hat[1:] / u_hat[0]
    bc = tuple(BC[b] for b in wl["bc"])
    bc_hi = tuple(BC[b] for b in wl.get("bc_hi") or wl["bc"])
    pb = Problem(geo=geo, rho=rho, u_hat=u_hat, v=v, model=MODEL[wl["model"]],
                 gamma=wl["gamma"], kappa_a=_t(wl.get("kappa_a")), kappa_s=_t(wl.get("kappa_s")),
                 j=_t(wl.get("j")), C_a=wl.get("C_a", 1.0), C_s=wl.get("C_s", 1.0),
                 bc_lo=bc, bc_hi=bc_hi, limiter=limiter)
    I0 = _t(wl["I0_iso"]).unsqueeze(0).expand((grid.ns,) + shape).clone()
    T0 = _t(wl["T"]).clone()
    return pb, I0, T0


def build_ks(wl, grid=None, limiter=tr.LIM_MC, fd_h=1e-3):
    """Problem on the Kerr-Schild (ln r, theta, phi) mesh; returns (pb, I0, T0, dt_max)."""
    from .kerr import KerrSchildLogR
    grid = grid or GeodesicGrid(wl["generation"], wl["weights"])
    geo = KerrSchildLogR(wl["n"], wl["xlo"], wl["xhi"], grid, wl["a"], wl.get("M", 1.0), fd_h,
                         recon=wl.get("angular_recon", "donor"), mapr_tie_rtol=wl.get("mapr_tie_rtol"))
    shape = tuple(wl["n"])
    u = np.asarray(wl["u"], dtype=np.float64)
    u_hat = geo.u_hat(u)
    v = torch.as_tensor(u[1:] / u[0])
    bc_lo = tuple(BC[b] for b in wl["bc"])
    bc_hi = tuple(BC[b] for b in wl.get("bc_hi", wl["bc"]))
    pb = Problem(geo=geo, rho=_t(wl["rho"]), u_hat=u_hat, v=v, model=MODEL[wl["model"]],
                 gamma=wl["gamma"], kappa_a=_t(wl.get("kappa_a")), kappa_s=_t(wl.get("kappa_s")),
                 j=_t(wl.get("j")), C_a=wl.get("C_a", 1.0), C_s=wl.get("C_s", 1.0),
                 bc_lo=bc_lo, bc_hi=bc_hi, limiter=limiter, n0_cut=wl.get("n0_cut"),
                 angular=geo.angular, pole_rows=wl.get("pole_rows", 0))
    I0 = _t(wl["I0_iso"]).unsqueeze(0).expand((grid.ns,) + shape).clone()
    return pb, I0, _t(wl["T"]).clone(), geo.dt_max(wl.get("cfl", 0.4))


def build_flat_mg(wl, grid=None, limiter=tr.LIM_MC):
    """Multi-group inputs: (Problem, kappa_a per bin [G, *n], bin edges,
    I0 [G, Ns, *n] (isotropic per bin), T0)."""
    pb, _, T0 = build_flat(wl, grid, limiter)
    ka = _t(wl["kappa_a_groups"])
    ns = pb.geo.grid.ns
    shape = tuple(wl["n"])
    I0 = _t(wl["I0_iso_groups"]).unsqueeze(1).expand((ka.shape[0], ns) + shape).clone()
    return pb, ka, tuple(wl["group_edges"]), I0, T0
