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


def random_intensity(ns, shape, seed, lo=0.0, hi=1.0):
    """Anisotropic positive intensity field [ns, *shape] for kernel-level parity."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(ns,) + tuple(shape))
