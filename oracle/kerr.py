"""Kerr-Schild geometry on a (ln r, theta, phi) mesh, and the angular flux.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2.1.1 (tetrads): the tetrad satisfies e e g = eta (Eq. tetrad_def), its time
leg is the normal observer e_0 = -g^(0 mu)/sqrt(-g^00) (Eq. tetrad_restriction),
and the metric is stationary.  The spatial legs are built here by Gram-Schmidt
on (d_phi, d_theta, d_x1) with respect to the spatial metric and assigned to
(3, 2, 1); they have no time component, so they are orthogonal to e_0.  The
geodesic grid's pole therefore lies on 3 = phi-hat.

Sec. 2.2 (Eq. angular_n_vectors, Eq. ricci_rotation_coefficients): the
rotation coefficients omega^a_(c d) = e^a_b e^mu_c (d_mu e^b_d + Gamma^b_(mu l) e^l_d)
are evaluated with central differences of the analytic tetrad and metric
(the paper also takes the derivatives numerically; fourth-order stencil).  A photon with tetrad
direction n (n^0 = 1) changes direction along its ray, per unit of the
parameter with dx/dlambda = n^mu, at the rate
    r^i(n) = -omega^i_(c d) n^c n^d + n^i omega^0_(c d) n^c n^d,
which follows from the geodesic equation in the tetrad basis (this fixes the
sign that the printed r^zeta leaves ambiguous).  The angular flux across a
geodesic edge with outward unit normal u_e at midpoint m_e (Sec. 3.5,
Eq. angular_fluxes) is F_e = n_0(m_e) (r(m_e) . u_e) I_upwind, with donor-cell
or MAPR (oracle.mapr) upwind states.

Kerr-Schild metric (units G = c = M = 1 scaled by M), Sigma = r^2 + a^2 cos^2 th,
z = 2 M r / Sigma:
    g_tt = -(1 - z), g_tr = z, g_tph = -z a sin^2 th, g_rr = 1 + z,
    g_rph = -a (1 + z) sin^2 th, g_thth = Sigma,
    g_phph = sin^2 th (Sigma + a^2 (1 + z) sin^2 th);
with x1 = ln r every r index picks up a factor r.
"""
import math

import numpy as np
import torch

F64 = torch.float64


def ks_metric(x1, th, a, M=1.0):
    """g_(mu nu) [..., 4, 4] at logical (x1 = ln r, theta), any broadcast shape."""
    x1, th = np.broadcast_arrays(np.asarray(x1, float), np.asarray(th, float))
    r = np.exp(x1)
    s, c = np.sin(th), np.cos(th)
    Sig = r * r + a * a * c * c
    z = 2.0 * M * r / Sig
    g = np.zeros(x1.shape + (4, 4))
    g[..., 0, 0] = -(1.0 - z)
    g[..., 0, 1] = g[..., 1, 0] = z * r
    g[..., 0, 3] = g[..., 3, 0] = -z * a * s * s
    g[..., 1, 1] = (1.0 + z) * r * r
    g[..., 1, 3] = g[..., 3, 1] = -a * (1.0 + z) * s * s * r
    g[..., 2, 2] = Sig
    g[..., 3, 3] = s * s * (Sig + a * a * (1.0 + z) * s * s)
    return g


def ks_sqrt_minus_g(x1, th, a, M=1.0):
    r = np.exp(x1)
    return r * (r * r + a * a * np.cos(th) ** 2) * np.abs(np.sin(th))


def tetrad(g):
    """e^mu_(alpha-hat) [..., 4(mu), 4(alpha)] from g [..., 4, 4]: normal observer
    plus Gram-Schmidt of (d_phi, d_theta, d_x1) -> (3, 2, 1)."""
    ginv = np.linalg.inv(g)
    e = np.zeros(g.shape)
    e[..., :, 0] = -ginv[..., 0, :] / np.sqrt(-ginv[..., 0, 0])[..., None]
    gam = g[..., 1:, 1:]

    def dot(u, v):
        return np.einsum("...i,...ij,...j->...", u, gam, v)

    basis = np.zeros(g.shape[:-2] + (3, 3))
    legs = []
    for k in (2, 1, 0):  # d_phi, d_theta, d_x1
        v = np.zeros(g.shape[:-2] + (3,))
        v[..., k] = 1.0
        for u in legs:
            v = v - dot(v, u)[..., None] * u
        v = v / np.sqrt(dot(v, v))[..., None]
        legs.append(v)
    # legs = [e_3, e_2, e_1]
    for hat, v in zip((3, 2, 1), legs):
        e[..., 1:, hat] = v
    del basis
    return e


def inverse_tetrad(e, g):
    """e^(alpha-hat)_mu = eta^(ab) g_(mu nu) e^nu_b  [..., 4(alpha), 4(mu)]."""
    eta = np.diag([-1.0, 1.0, 1.0, 1.0])
    return np.einsum("ab,...mn,...nb->...am", eta, g, e)


def rotation_coefficients(x1, th, a, M=1.0, h=1e-3):
    """omega^(alpha-hat)_(gamma-hat delta-hat) [..., 4, 4, 4] by fourth-order
    central differences in x1 and theta (the metric does not depend on t, phi);
    with h = 1e-3 the truncation error is ~1e-12 and the rounding error ~1e-13."""
    x1 = np.asarray(x1, float)
    th = np.asarray(th, float)
    g = ks_metric(x1, th, a, M)
    e = tetrad(g)
    einv = inverse_tetrad(e, g)
    ginv = np.linalg.inv(g)
    dg = np.zeros(g.shape + (4,))        # d_mu g_(nu l) stored as [..., nu, l, mu]
    de = np.zeros(e.shape + (4,))        # d_mu e^b_d stored as [..., b, d, mu]
    for mu, (dx1, dth) in ((1, (h, 0.0)), (2, (0.0, h))):
        # fourth-order central differences: (-f(+2h) + 8 f(+h) - 8 f(-h) + f(-2h)) / 12h
        gs = {k: ks_metric(x1 + k * dx1, th + k * dth, a, M) for k in (-2, -1, 1, 2)}
        dg[..., mu] = (-gs[2] + 8 * gs[1] - 8 * gs[-1] + gs[-2]) / (12 * h)
        es = {k: tetrad(v) for k, v in gs.items()}
        de[..., mu] = (-es[2] + 8 * es[1] - 8 * es[-1] + es[-2]) / (12 * h)
    # Gamma^b_(mu l) = 1/2 g^(b n) (d_mu g_(n l) + d_l g_(n mu) - d_n g_(mu l))
    term = (np.einsum("...nlm->...nml", dg) + np.einsum("...nml->...nml", dg)
            - np.einsum("...mln->...nml", dg))
    Gam = 0.5 * np.einsum("...bn,...nml->...bml", ginv, term)
    # nabla_mu e^b_d = d_mu e^b_d + Gamma^b_(mu l) e^l_d
    nab = np.einsum("...bdm->...bmd", de) + np.einsum("...bml,...ld->...bmd", Gam, e)
    # omega^a_(c d) = e^a_b e^mu_c nabla_mu e^b_d
    return np.einsum("...ab,...mc,...bmd->...acd", einv, e, nab)


def angular_rate(omega, n3):
    """r^i(n) for tetrad directions n3 [S, 3] -> [..., S, 3]."""
    S = n3.shape[0]
    n4 = np.concatenate([np.ones((S, 1)), n3], axis=1)
    q = np.einsum("...acd,sc,sd->...sa", omega, n4, n4)   # omega^a_(n n)
    return -q[..., 1:] + n3 * q[..., :1]


class KerrSchildLogR:
    """Geometry provider for the oracle transport on a (ln r, theta, phi) mesh.

    Shapes follow the direction-major intensity [Ns, N1, N2, N3]; everything is
    independent of phi (axis 3 is broadcast)."""

    kind = "kerr_schild"

    def __init__(self, n, xlo, xhi, grid, a, M=1.0, fd_h=1e-3, recon="donor", mapr_tie_rtol=None):
        if recon not in ("donor", "mapr"):
            raise ValueError(recon)
        self.recon = recon
        self.mapr_tie_rtol = mapr_tie_rtol      # None: the FP64 band of oracle.mapr
        self.n = tuple(int(v) for v in n)
        self.xlo, self.xhi = tuple(map(float, xlo)), tuple(map(float, xhi))
        self.dx = tuple((b - c) / m for c, b, m in zip(self.xlo, self.xhi, self.n))
        self.grid, self.a, self.M = grid, float(a), float(M)
        N1, N2, _ = self.n
        x1c = self.xlo[0] + (np.arange(N1) + 0.5) * self.dx[0]
        thc = self.xlo[1] + (np.arange(N2) + 0.5) * self.dx[1]
        x1f = self.xlo[0] + np.arange(N1 + 1) * self.dx[0]
        thf = self.xlo[1] + np.arange(N2 + 1) * self.dx[1]
        self.x1c, self.thc, self.x1f, self.thf = x1c, thc, x1f, thf
        nh = np.concatenate([np.ones((grid.ns, 1)), grid.n], axis=1)   # [Ns, 4]
        self.nh = nh
        X1, TH = np.meshgrid(x1c, thc, indexing="ij")
        self.gc = ks_metric(X1, TH, a, M)
        self.ec = tetrad(self.gc)
        self.sqrtg_c = ks_sqrt_minus_g(X1, TH, a, M)
        # cell-centre factors
        nmu = np.einsum("ijma,sa->sijm", self.ec, nh)                 # n^mu [Ns, N1, N2, 4]
        self._n_up0 = self.ec[..., 0, 0]                                # 1/alpha [N1, N2]
        self._n_low0 = np.einsum("ijm,sijm->sij", self.gc[..., 0, :], nmu)
        # faces along x1 (axis 0) and theta (axis 1); phi faces equal the centres
        self._face = {}
        for ax, (xa, xb) in enumerate(((x1f, thc), (x1c, thf))):
            A, B = np.meshgrid(xa, xb, indexing="ij")
            # the tetrad is singular on the axis; pole faces carry no flux (their
            # area vanishes), so their factors are taken just off the axis
            pole = (np.abs(np.sin(B)) < 1e-12) if ax == 1 else np.zeros(A.shape, bool)
            Bs = np.where(pole, B + np.where(B < 1.0, 1e-8, -1e-8), B)
            g = ks_metric(A, Bs, a, M)
            e = tetrad(g)
            nm = np.einsum("ijma,sa->sijm", e, nh)
            nu = nm[..., 1 + ax]
            nl0 = np.einsum("ijm,sijm->sij", g[..., 0, :], nm)
            nu0 = e[..., 0, 0]
            sg = ks_sqrt_minus_g(A, B, a, M)
            nu = np.where(pole[None], 0.0, nu)
            other = [self.dx[k] for k in range(3) if k != ax]
            self._face[ax] = (nu, nl0, nu0, sg * other[0] * other[1])
        # phi faces (axis 2): the metric does not depend on phi
        self._face[2] = (nmu[..., 3], self._n_low0, self._n_up0,
                         self.sqrtg_c * self.dx[0] * self.dx[1])
        self._dV = self.sqrtg_c * self.dx[0] * self.dx[1] * self.dx[2]
        # angular (geodesic-edge) velocities v_e = r(m_e) . u_e and n_0(m_e) per cell
        self.omega = rotation_coefficients(X1, TH, a, M, fd_h)
        rate = angular_rate(self.omega, grid.emid)                      # [N1, N2, Ne, 3]
        self.v_edge = np.einsum("ijes,es->eij", rate, grid.enorm)       # [Ne, N1, N2]
        me4 = np.concatenate([np.ones((len(grid.emid), 1)), grid.emid], axis=1)
        nme = np.einsum("ijma,ea->eijm", self.ec, me4)
        self.n0_edge = np.einsum("ijm,eijm->eij", self.gc[..., 0, :], nme)

    # -- providers used by oracle.transport --------------------------------
    def _t(self, x, shape):
        return torch.as_tensor(np.ascontiguousarray(x), dtype=F64).reshape(shape)

    def n_up0(self):
        return self._t(self._n_up0, (1, self.n[0], self.n[1], 1))

    def n_low0(self):
        return self._t(self._n_low0, (-1, self.n[0], self.n[1], 1))

    def dV(self):
        return self._t(self._dV, (self.n[0], self.n[1], 1))

    def face_nu(self, ax):
        nu = self._face[ax][0]
        return self._t(nu, (-1,) + nu.shape[1:] + (1,))

    def face_n_low0(self, ax):
        x = self._face[ax][1]
        return self._t(x, (-1,) + x.shape[1:] + (1,))

    def face_n_up0(self, ax):
        x = self._face[ax][2]
        return self._t(x, (1,) + x.shape + (1,))

    def face_dA(self, ax):
        x = self._face[ax][3]
        return self._t(x, x.shape + (1,))

    def face_sign_ok(self, ax, periodic):
        """n_0 keeps its sign across the face (Sec. 3.5); False zeroes the flux.
        Evaluated between interior neighbours; boundary faces are kept."""
        n0 = self._n_low0 if ax < 2 else None
        if ax == 2:
            return None   # phi neighbours share the same geometry
        N = self.n[ax]
        ok = np.ones((n0.shape[0],) + tuple(N + 1 if k == ax else self.n[k] for k in range(2)), bool)
        if ax == 0:
            ok[:, 1:N] = np.sign(n0[:, :-1]) == np.sign(n0[:, 1:])
        else:
            ok[:, :, 1:N] = np.sign(n0[:, :, :-1]) == np.sign(n0[:, :, 1:])
        return torch.as_tensor(ok).reshape((-1,) + ok.shape[1:] + (1,))

    def u_hat(self, u_coord):
        """u-hat^a = e^a_mu u^mu at the cell centres; u_coord [4, N1, N2, N3]."""
        einv = inverse_tetrad(self.ec, self.gc)                          # [N1, N2, 4, 4]
        uh = np.einsum("ijam,mijk->aijk", einv, np.asarray(u_coord))
        return torch.as_tensor(uh, dtype=F64)

    def dt_max(self, cfl):
        """cfl times min over cells and axes of dx^a / max_s |n^a / n^0| (Sec. 3.8)."""
        nmu = np.einsum("ijma,sa->sijm", self.ec, self.nh)
        best = math.inf
        for ax in range(3):
            speed = np.abs(nmu[..., 1 + ax] / nmu[..., 0]).max()
            best = min(best, self.dx[ax] / speed)
        return cfl * best

    def angular(self, I):
        """(1/w_s) sum_e dlambda_e F_e for every direction and cell; the edge
        states are the upwind direction's own intensity (donor cell) or its
        MAPR reconstruction at the edge midpoint (oracle.mapr)."""
        g = self.grid
        es, et = torch.as_tensor(g.edges[:, 0]), torch.as_tensor(g.edges[:, 1])
        v = self._t(self.v_edge, (-1, self.n[0], self.n[1], 1))
        n0 = self._t(self.n0_edge, (-1, self.n[0], self.n[1], 1))
        if self.recon == "mapr":
            from . import mapr
            if not hasattr(self, "_ring"):
                self._ring = mapr.rings(g)
            tie = mapr.TIE_RTOL if self.mapr_tie_rtol is None else self.mapr_tie_rtol
            first, second = mapr.edge_states(g, I, self._ring, tie)
            Iup = torch.where(v > 0, first, second)
        else:
            Iup = torch.where(v > 0, I[es], I[et])
        F = n0 * v * Iup * torch.as_tensor(g.dlam, dtype=F64).reshape(-1, 1, 1, 1)
        w = torch.as_tensor(g.w, dtype=F64).reshape(-1, 1, 1, 1)
        div = torch.zeros_like(I)
        div = div.index_add(0, es, F)
        div = div.index_add(0, et, -F)
        return div / w


def coordinate_moments(R_hat, e):
    """R^(mu nu) = e^mu_a e^nu_b R-hat^(ab) (Eq. R in the coordinate frame).
    R_hat [10, N1, N2, N3] in the order 00,01,02,03,11,12,13,22,23,33; e the
    tetrad e^mu_a [N1, N2, 4, 4] (phi-independent).  Same storage order out."""
    from .step import SYM10
    R_hat = torch.as_tensor(R_hat, dtype=F64)
    full = torch.zeros((4, 4) + tuple(R_hat.shape[1:]), dtype=F64)
    for k, (p, q) in enumerate(SYM10):
        full[p, q] = R_hat[k]
        full[q, p] = R_hat[k]
    E = torch.as_tensor(e, dtype=F64)                                   # [N1, N2, mu, a]
    Rc = torch.einsum("ijma,abijk,ijnb->mnijk", E, full, E)
    return torch.stack([Rc[p, q] for p, q in SYM10])
