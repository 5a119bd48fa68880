"""Metric-dependent factors of the discrete transport equation.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The finite-volume form of the gray transfer equation (Sec. 3.1,
Eq. radiative_transfer_discrete) needs, per cell l, face l+1/2 and direction s:
  n^0, n_0       coordinate-frame time components of the photon direction
                 n^alpha = e^alpha_(beta-hat) n-hat^(beta-hat)  (Sec. 2.2)
  n^a            the spatial component along axis a, at the faces
  Delta V, Delta A_a   the sqrt(-g)-weighted cell volume and face areas
This module provides them for the flat Cartesian case: identity tetrad
(Sec. 2.1.1: "for a flat spacetime ... the identity matrix"), so n^0 = 1,
n_0 = -1, n^a = n-hat^a, and Delta V, Delta A are the plain Cartesian
volume and areas.

Every accessor returns a float64 tensor that broadcasts against the
direction-major intensity layout [N_s, N1, N2, N3]; face quantities along axis a
broadcast against [N_s, ..., N_a + 1, ...] (face f is the lower face of cell f).
"""
import numpy as np
import torch

F64 = torch.float64


class FlatCartesian:
    """Minkowski metric on a uniform Cartesian mesh with the identity tetrad."""

    kind = "flat"

    def __init__(self, n, xlo, xhi, grid):
        self.n = tuple(int(x) for x in n)
        self.dx = tuple((float(b) - float(a)) / m for a, b, m in zip(xlo, xhi, self.n))
        self.grid = grid
        self.nhat = torch.tensor(grid.n, dtype=F64)          # [Ns, 3]

    # -- cell-centre quantities ------------------------------------------
    def n_up0(self):
        """n^0 at cell centres: e^0_0-hat = 1."""
        return torch.ones((1, 1, 1, 1), dtype=F64)

    def n_low0(self):
        """n_0 = g_(0 mu) n^mu = -1 at cell centres, every direction."""
        return -torch.ones((1, 1, 1, 1), dtype=F64)

    def dV(self):
        return torch.full((1, 1, 1), self.dx[0] * self.dx[1] * self.dx[2], dtype=F64)

    # -- face quantities along axis a --------------------------------------
    def face_nu(self, a):
        """n^a at the faces normal to axis a: the tetrad component n-hat^a."""
        return self.nhat[:, a].reshape(-1, 1, 1, 1)

    def face_n_low0(self, a):
        return -torch.ones((1, 1, 1, 1), dtype=F64)

    def face_n_up0(self, a):
        return torch.ones((1, 1, 1, 1), dtype=F64)

    def face_dA(self, a):
        return torch.full((1, 1, 1), self.dx[0] * self.dx[1] * self.dx[2] / self.dx[a], dtype=F64)

    def u_hat(self, u_coord):
        """Tetrad-frame fluid 4-velocity u-hat = e^hat_gamma u^gamma (identity)."""
        return u_coord

    def dt_max(self, cfl):
        """Time-step bound of Sec. 3.8: cfl times the light-crossing time of the
        smallest cell, using the largest |n^a / n^0| on the angular grid."""
        vmax = np.abs(self.grid.n).max(axis=0)
        return cfl * min(d / v for d, v in zip(self.dx, vmax))
