"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module only draws and shapes input fields (numpy, float64); it contains
none of the transfer method's arithmetic.  Every generator takes an explicit
seed; the default seed of workload k is 2508153 + k.

Workloads (sizes of the paper-scale runs; every builder accepts a reduced
`n` for parity tests that the oracle finishes in seconds):

  blob_flat      flat 16^3 on [0,16]^3, periodic, generation 1, equal weights,
                 isotropic Gaussian blob (amplitude 1, sigma 3 cells) + 1e-6,
                 rho = 1, T = 1, kappa_a = 1, no scattering, Method 1, dt 0.4.
  brems_flat     flat 128^3, periodic, generation 2, Voronoi weights;
                 rho lognormal (sigma_ln = 1, k^-2 Gaussian random field),
                 T ~ U[0.5, 2] per cell, alpha^a = rho^2 T^-3.5, alpha^s = rho,
                 Gamma = 5/3, Method 2, I0 = T^4/(4 pi) isotropic, dt 0.4.
  adjoint_flat   flat 64^3, zero-incoming on all faces, generation 2,
                 kappa_a lognormal (sigma_ln = 0.5), j ~ U[0,1], rho = 1,
                 fixed emissivity, I0 = 0, dt 0.4, 20 steps.
  multigroup_flat  the flat recipe with 4 frequency bins, per-bin absorption
                 opacities rho^2 (3, 1, 0.3, 0.1), alpha^s = rho, bins
                 starting with equal shares of T^4/(4 pi).
  torus_ks       Kerr-Schild a = 0.9, log r in [ln 1.5, ln 50], theta in
                 [0, pi], phi in [0, 2 pi); synthetic torus density, Keplerian
                 4-velocity outside the ISCO, T0 = 1, Method 2.
"""
import math
import numpy as np

BASE_SEED = 2508153


def rng_for(k, seed=None):
    return np.random.default_rng(BASE_SEED + k if seed is None else seed)


def gaussian_random_field(shape, rng):
    """Unit-variance Gaussian random field with power spectrum |k|^-2 (amplitude
    |k|^-1), zero mean (k = 0 removed), periodic on the grid."""
    noise = rng.standard_normal(shape)
    fk = np.fft.rfftn(noise)
    ks = [np.fft.fftfreq(n) for n in shape[:-1]] + [np.fft.rfftfreq(shape[-1])]
    kk = np.meshgrid(*ks, indexing="ij")
    kmag = np.sqrt(sum(k * k for k in kk))
    amp = np.zeros_like(kmag)
    nz = kmag > 0
    amp[nz] = 1.0 / kmag[nz]
    g = np.fft.irfftn(fk * amp, s=shape, axes=tuple(range(len(shape))))
    g -= g.mean()
    return g / g.std()


def lognormal(shape, sigma_ln, rng):
    """exp(sigma g - sigma^2/2) for a unit-variance GRF g (mean 1)."""
    return np.exp(sigma_ln * gaussian_random_field(shape, rng) - 0.5 * sigma_ln ** 2)


def blob_flat(n=16, seed=None):
    shape = (n, n, n)
    c = n / 2.0
    x = np.arange(n) + 0.5 - c
    r2 = x[:, None, None] ** 2 + x[None, :, None] ** 2 + x[None, None, :] ** 2
    I0 = np.exp(-r2 / 18.0) + 1e-6
    return dict(
        name="blob_flat", n=shape, xlo=(0.0, 0.0, 0.0), xhi=(float(n),) * 3,
        generation=1, weights="equal", bc=("periodic",) * 3,
        model="kirchhoff_const", gamma=5.0 / 3.0,
        rho=np.ones(shape), T=np.ones(shape), kappa_a=np.ones(shape),
        kappa_s=np.zeros(shape), j=None, u=None,
        I0_iso=I0, dt=0.4, steps=10,
    )


def brems_flat(n=128, generation=2, seed=None):
    rng = rng_for(1, seed)
    shape = (n, n, n) if np.isscalar(n) else tuple(n)
    rho = lognormal(shape, 1.0, rng)
    T = rng.uniform(0.5, 2.0, size=shape)
    return dict(
        name="brems_flat", n=shape, xlo=(0.0, 0.0, 0.0), xhi=tuple(float(m) for m in shape),
        generation=generation, weights="voronoi", bc=("periodic",) * 3,
        model="brems", gamma=5.0 / 3.0, C_a=1.0, C_s=1.0,
        rho=rho, T=T, kappa_a=None, kappa_s=None, j=None, u=None,
        I0_iso=T ** 4 / (4.0 * math.pi), dt=0.4, steps=100,
    )


def adjoint_flat(n=64, generation=2, seed=None, n_probe=32):
    rng = rng_for(3, seed)
    shape = (n, n, n) if np.isscalar(n) else tuple(n)
    kappa = lognormal(shape, 0.5, rng)
    j = rng.uniform(0.0, 1.0, size=shape)
    # probe cells for finite differences: x-layers within 8 of the +x face
    lo = max(0, shape[0] - 8)
    probes = np.stack([rng.integers(lo, shape[0], n_probe),
                       rng.integers(0, shape[1], n_probe),
                       rng.integers(0, shape[2], n_probe)], axis=1)
    return dict(
        name="adjoint_flat", n=shape, xlo=(0.0, 0.0, 0.0), xhi=tuple(float(m) for m in shape),
        generation=generation, weights="voronoi", bc=("zero_incoming",) * 3,
        model="fixed_emissivity", gamma=5.0 / 3.0,
        rho=np.ones(shape), T=np.ones(shape), kappa_a=kappa, kappa_s=np.zeros(shape), j=j,
        u=None, I0_iso=np.zeros(shape), dt=0.4, steps=20, checkpoint=5, probes=probes,
    )


def multigroup_flat(n=128, generation=2, seed=None,
                    edges=(0.0, 1.0, 3.0, 9.0, math.inf), kappa_groups=(3.0, 1.0, 0.3, 0.1)):
    """Multi-group version of the flat recipe: rho lognormal (sigma_ln 1), T ~
    U[0.5, 2], bins [0, 1), [1, 3), [3, 9), [9, inf) of fluid-frame frequency
    (units of k_B/h), absorption opacity per bin kappa_a,g = rho kappa_g with
    kappa_g = 3, 1, 0.3, 0.1 (alpha^a_g = rho^2 kappa_g, falling with
    frequency), alpha^s = rho, periodic, dt 0.4; every bin starts isotropic
    with an equal share T^4/(4 pi G) of the gray energy (out of equilibrium
    across bins)."""
    rng = rng_for(5, seed)
    shape = (n, n, n) if np.isscalar(n) else tuple(n)
    rho = lognormal(shape, 1.0, rng)
    T = rng.uniform(0.5, 2.0, size=shape)
    G = len(kappa_groups)
    assert len(edges) == G + 1
    return dict(
        name="multigroup_flat", n=shape, xlo=(0.0, 0.0, 0.0), xhi=tuple(float(m) for m in shape),
        generation=generation, weights="voronoi", bc=("periodic",) * 3,
        model="kirchhoff_const", gamma=5.0 / 3.0,
        rho=rho, T=T, kappa_a=None, kappa_s=np.ones(shape), j=None, u=None,
        group_edges=tuple(float(e) for e in edges),
        kappa_a_groups=np.stack([rho * k for k in kappa_groups]),
        I0_iso_groups=np.stack([T ** 4 / (4.0 * math.pi * G)] * G),
        I0_iso=T ** 4 / (4.0 * math.pi), dt=0.4, steps=20,
    )


def random_intensity(ns, shape, seed, lo=0.0, hi=1.0):
    """Anisotropic positive intensity field [ns, *shape] for kernel-level parity."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(ns,) + tuple(shape))


def _ks_equatorial_block(r, th, a):
    """g_tt, g_tph, g_phph of the Kerr-Schild metric (M = 1); input preparation
    for the fluid 4-velocity only."""
    Sig = r * r + a * a * np.cos(th) ** 2
    z = 2.0 * r / Sig
    s2 = np.sin(th) ** 2
    return -(1.0 - z), -z * a * s2, s2 * (Sig + a * a * (1.0 + z) * s2)


def torus_ks(n=(256, 128, 64), a=0.9, generation=2, sigma_ln=None, scattering=False, seed=None,
             r_in=1.5, r_out=50.0):
    """Synthetic torus in Kerr-Schild coordinates (x1 = ln r, theta, phi), r in [r_in, r_out]
    (default [1.5, 50]):
    rho = exp(-(r-12)^2/(2*3^2) - (theta-pi/2)^2/(2*0.3^2)) (times a lognormal field
    when sigma_ln is given); circular Keplerian flow u = u^t (1, 0, 0, Omega),
    Omega = 1/(r^1.5 + a), where r >= r_isco(a) and the orbit is timelike, else
    the normal observer; T0 = 1; alpha^a = rho^2 T^-3.5 (Method 2); alpha^s = rho
    if scattering; I0 = 0; r: outflow inside, zero-incoming outside; theta:
    outflow; phi periodic; rows next to the poles zeroed."""
    rng = rng_for(5 if sigma_ln else 2, seed)
    shape = tuple(int(v) for v in n)
    xlo = (math.log(r_in), 0.0, 0.0)
    xhi = (math.log(r_out), math.pi, 2.0 * math.pi)
    x1 = xlo[0] + (np.arange(shape[0]) + 0.5) * (xhi[0] - xlo[0]) / shape[0]
    th = xlo[1] + (np.arange(shape[1]) + 0.5) * (xhi[1] - xlo[1]) / shape[1]
    r = np.exp(x1)[:, None, None] * np.ones(shape)
    TH = th[None, :, None] * np.ones(shape)
    rho = np.exp(-(r - 12.0) ** 2 / 18.0 - (TH - math.pi / 2) ** 2 / (2 * 0.09))
    if sigma_ln:
        rho = rho * lognormal(shape, sigma_ln, rng)
    # ISCO radius of a prograde orbit (Bardeen, Press & Teukolsky 1972)
    z1 = 1 + (1 - a * a) ** (1 / 3) * ((1 + a) ** (1 / 3) + (1 - a) ** (1 / 3))
    z2 = math.sqrt(3 * a * a + z1 * z1)
    r_isco = 3 + z2 - math.sqrt((3 - z1) * (3 + z1 + 2 * z2))
    Om = 1.0 / (r ** 1.5 + a)
    gtt, gtp, gpp = _ks_equatorial_block(r, TH, a)
    norm = gtt + 2 * gtp * Om + gpp * Om * Om
    kep = (r >= r_isco) & (norm < 0)
    u = np.zeros((4,) + shape)
    ut = np.where(kep, 1.0 / np.sqrt(np.where(kep, -norm, 1.0)), 0.0)
    # normal observer: u = (1/alpha, -beta^i/alpha), alpha = 1/sqrt(1+z),
    # beta^r = z/(1+z); in x1 = ln r the radial component is divided by r
    Sig = r * r + a * a * np.cos(TH) ** 2
    zz = 2.0 * r / Sig
    u[0] = np.where(kep, ut, np.sqrt(1 + zz))
    u[1] = np.where(kep, 0.0, -zz / (1 + zz) * np.sqrt(1 + zz) / r)
    u[3] = np.where(kep, ut * Om, 0.0)
    return dict(
        name="torus_ks", n=shape, xlo=xlo, xhi=xhi, coords="logr_theta_phi", metric="kerr_schild",
        a=a, M=1.0, generation=generation, weights="voronoi",
        bc=("outflow", "outflow", "periodic"), bc_hi=("zero_incoming", "outflow", "periodic"),
        model="brems", gamma=5.0 / 3.0, C_a=1.0, C_s=1.0 if scattering else 0.0,
        rho=rho, T=np.ones(shape), kappa_a=None, kappa_s=None, j=None, u=u,
        I0_iso=np.zeros(shape), cfl=0.4, steps=50, pole_rows=4, n0_cut=0.1,
    )


def bright_sphere(n=(32, 12, 4), r_in=1.0, r_out=12.0, r_src=2.0, kappa=5.0, generation=1):
    """Flat space in spherical coordinates (x1 = ln r, theta, phi; M = 0): an
    opaque ball r < r_src (fixed emissivity j = kappa / (4 pi) per unit
    density, absorption kappa, so the intensity inside tends to
    I_s = 1 / (4 pi)) in vacuum out to r_out (density below the floor);
    inner boundary outflow, outer boundary zero-incoming, phi periodic.
    The steady state outside the ball is the field of a uniformly bright
    sphere, J(r) = (I_s / 2) (1 - sqrt(1 - R^2 / r^2)), R the ball's radius."""
    shape = tuple(int(v) for v in n)
    xlo = (math.log(r_in), 0.0, 0.0)
    xhi = (math.log(r_out), math.pi, 2.0 * math.pi)
    x1 = xlo[0] + (np.arange(shape[0]) + 0.5) * (xhi[0] - xlo[0]) / shape[0]
    r = np.exp(x1)[:, None, None] * np.ones(shape)
    src = r < r_src
    u = np.zeros((4,) + shape)
    u[0] = 1.0
    return dict(
        name="bright_sphere", n=shape, xlo=xlo, xhi=xhi, coords="logr_theta_phi", metric="kerr_schild",
        a=0.0, M=0.0, generation=generation, weights="voronoi",
        bc=("outflow", "outflow", "periodic"), bc_hi=("zero_incoming", "outflow", "periodic"),
        model="fixed_emissivity", gamma=5.0 / 3.0, C_a=1.0, C_s=0.0,
        rho=np.where(src, 1.0, 1e-6), T=np.ones(shape), kappa_a=np.where(src, kappa, 0.0),
        kappa_s=np.zeros(shape), j=np.where(src, kappa / (4.0 * math.pi), 0.0), u=u,
        I0_iso=np.zeros(shape), cfl=0.4, pole_rows=0, n0_cut=0.1,
        r_src_face=float(np.exp(xlo[0] + np.count_nonzero(src[:, 0, 0]) * (xhi[0] - xlo[0]) / shape[0])),
    )
