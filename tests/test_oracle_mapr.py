"""Pins of the oracle's MAPR angular reconstruction (Sec. 3.4, edge states of
the angular fluxes) against properties its reading implies, each computed by
a route the oracle does not take:
  * cyclic order: consecutive neighbours of a direction share a Delaunay
    triangle with it (the grid's own triangle list);
  * exactness on planes: a field linear in the gnomonic coordinates of n_s is
    reconstructed exactly at every point;
  * minimum slope: the chosen slope is one of the consecutive-pair planes and
    no pair plane is flatter (planes from 3D cross products of the lifted
    points, not the Gram system the oracle solves);
  * positivity: states are never negative and fall back to I_s exactly where
    the linear state is negative;
  * second order: the edge-state error of a smooth field falls ~4x per
    grid generation (donor cell ~2x);
  * conservation: the angular divergence has zero quadrature sum over the
    directions, and a constant field has the donor-cell divergence.
"""
import numpy as np
import pytest
import torch

from oracle import mapr
from oracle.grid import GeodesicGrid

F64 = torch.float64


@pytest.fixture(scope="module", params=[1, 2])
def grid(request):
    return GeodesicGrid(request.param)


def _tangent_basis(n):
    a = np.array([1.0, 0.0, 0.0]) if abs(n[0]) < 0.8 else np.array([0.0, 1.0, 0.0])
    e1 = np.cross(n, a)
    e1 /= np.linalg.norm(e1)
    return e1, np.cross(n, e1)


def test_ring_pairs_are_delaunay_triangles(grid):
    tris = {tuple(sorted(t)) for t in grid.tris.tolist()}
    ring = mapr.rings(grid)
    for s, r in enumerate(ring):
        assert len(r) == grid.degree[s]
        for k in range(len(r)):
            assert tuple(sorted((s, r[k], r[(k + 1) % len(r)]))) in tris


def test_plane_fields_are_exact(grid):
    """I(x) = c + g0 . p_s(x) on s and its ring: slope g0 and the exact value at
    every edge midpoint of s."""
    rng = np.random.default_rng(3)
    ring = mapr.rings(grid)
    for s in range(grid.ns):
        n = grid.n[s]
        e1, e2 = _tangent_basis(n)
        g0 = rng.normal(size=2)
        g3 = g0[0] * e1 + g0[1] * e2
        c = 5.0 + rng.random()
        I = torch.zeros((grid.ns, 1), dtype=F64)
        for x in [s] + ring[s]:
            I[x, 0] = c + float(mapr.gnomonic(n, grid.n[x]) @ g3)
        g = mapr.slopes(grid, I, ring)[s, 0].numpy()
        assert np.allclose(g, g3, rtol=0, atol=1e-12)
        for e in np.nonzero((grid.edges == s).any(1))[0]:
            m = grid.emid[e]
            v = mapr.state(n, I[s], torch.as_tensor(g)[None], m)
            assert abs(float(v) - (c + float(mapr.gnomonic(n, m) @ g3))) < 1e-12


def _lifted_plane_slope(pa, pb, dA, dB, e1, e2):
    """Slope of the plane through (0,0,0), (a1,a2,dA), (b1,b2,dB) in tangent
    coordinates, from the normal vector (a x b)."""
    a = np.array([pa @ e1, pa @ e2, dA])
    b = np.array([pb @ e1, pb @ e2, dB])
    N = np.cross(a, b)
    return np.array([-N[0] / N[2], -N[1] / N[2]])


def test_minimum_slope_choice(grid):
    rng = np.random.default_rng(5)
    ring = mapr.rings(grid)
    I = torch.as_tensor(rng.random((grid.ns, 4)) * 2.0, dtype=F64)
    g = mapr.slopes(grid, I, ring)
    for s in range(grid.ns):
        n = grid.n[s]
        e1, e2 = _tangent_basis(n)
        P = mapr.gnomonic(n, grid.n[ring[s]])
        for c in range(I.shape[1]):
            cand = []
            for k in range(len(ring[s])):
                a, b = k, (k + 1) % len(ring[s])
                cand.append(_lifted_plane_slope(P[a], P[b], float(I[ring[s][a], c] - I[s, c]),
                                                float(I[ring[s][b], c] - I[s, c]), e1, e2))
            norms = [float(x @ x) for x in cand]
            got = np.array([float(g[s, c] @ torch.as_tensor(e1)), float(g[s, c] @ torch.as_tensor(e2))])
            assert abs(float(g[s, c] @ torch.as_tensor(n))) < 1e-12        # tangent
            assert float(got @ got) <= min(norms) * (1 + 1e-7) + 1e-30
            assert min(np.abs(got - x).max() for x in cand) < 1e-10


def test_ties_are_not_decided_by_rounding(grid):
    """Fields with many exact ties (zeroed neighbours around symmetric
    neighbourhoods): the slopes do not change when the inputs move by 1e-14
    relative, and a tie goes to the first minimal plane counter-clockwise from
    the neighbour with the smallest index."""
    rng = np.random.default_rng(11)
    ring = mapr.rings(grid)
    for s, r in enumerate(ring):
        assert r[0] == min(r)
    I = rng.random((grid.ns, 32)) + 0.5
    I[rng.random(I.shape) < 0.5] = 0.0
    It = torch.as_tensor(I, dtype=F64)
    g = mapr.slopes(grid, It, ring)
    gp = mapr.slopes(grid, It * (1.0 + 1e-14 * torch.as_tensor(rng.standard_normal(I.shape))), ring)
    assert float((g - gp).abs().max()) < 1e-9
    # the pole (a pentagon with five-fold symmetry): I_s = 1, neighbours zero:
    # five congruent planes, the first (smallest-index neighbour and its
    # counter-clockwise successor) is taken
    s = 0
    J = torch.zeros((grid.ns, 1), dtype=F64)
    J[s] = 1.0
    P = mapr.gnomonic(grid.n[s], grid.n[ring[s]])
    m1 = torch.tensor([-1.0], dtype=F64)
    want = mapr.pair_slope(P[0], P[1], m1, m1)[0]
    assert float((mapr.slopes(grid, J, ring)[s, 0] - want).abs().max()) < 1e-14
    n = grid.n[s]
    assert float(np.cross(P[0], P[1]) @ n) > 0          # counter-clockwise from outside


def test_tie_band_of_the_fp32_form(grid):
    """The FP32 form counts planes within 1e-4 (relative |g|^2) of the
    flattest as tied, the FP64 form within 1e-8: break the pole's five-fold
    symmetry so that the third pair plane is flatter by a relative 1e-6; the
    FP64 band takes it, the FP32 band keeps the first plane of the ring."""
    ring = mapr.rings(grid)
    s = 0
    r = ring[s]
    P = mapr.gnomonic(grid.n[s], grid.n[r])
    J = torch.zeros((grid.ns, 1), dtype=F64)
    J[s] = 1.0
    # neighbours 2 and 3 (the third pair) rise a little: that plane flattens
    J[r[2]] = J[r[3]] = 5e-7
    cand = [mapr.pair_slope(P[k], P[(k + 1) % 5], J[r[k]] - 1.0, J[r[(k + 1) % 5]] - 1.0)[0]
            for k in range(5)]
    norms = [float(c @ c) for c in cand]
    assert min(norms) == norms[2] and 1e-8 < (norms[0] - norms[2]) / norms[2] < 1e-4
    g64 = mapr.slopes(grid, J, ring)[s, 0]
    g32 = mapr.slopes(grid, J, ring, tie_rtol=mapr.TIE_RTOL_FP32)[s, 0]
    assert float((g64 - cand[2]).abs().max()) < 1e-15
    assert float((g32 - cand[0]).abs().max()) < 1e-15


def test_positivity_fallback(grid):
    rng = np.random.default_rng(7)
    I = torch.as_tensor(rng.random((grid.ns, 64)) ** 6, dtype=F64)   # steep, near zero
    first, second = mapr.edge_states(grid, I)
    g = mapr.slopes(grid, I)
    assert (first >= 0).all() and (second >= 0).all()
    hit = 0
    for e, (s, t) in enumerate(grid.edges):
        lin = I[s] + (g[s] * torch.as_tensor(mapr.gnomonic(grid.n[s], grid.emid[e]))).sum(-1)
        neg = lin < 0
        hit += int(neg.sum())
        assert torch.equal(first[e][neg], I[s][neg])
        assert torch.equal(first[e][~neg], lin[~neg])
    assert hit > 0          # the fallback was exercised


def _edge_error(gen, field):
    grid = GeodesicGrid(gen)
    I = torch.as_tensor(field(grid.n), dtype=F64)[:, None]
    first, second = mapr.edge_states(grid, I)
    exact = torch.as_tensor(field(grid.emid), dtype=F64)
    e_mapr = max(float((first[:, 0] - exact).abs().max()), float((second[:, 0] - exact).abs().max()))
    e_donor = float((I[grid.edges[:, 0], 0] - exact).abs().max())
    return e_mapr, e_donor


def test_second_order_convergence():
    k = np.array([0.3, -0.5, 0.8])

    def field(x):
        return np.exp(x @ k) + 0.2 * (x[..., 0] * x[..., 1])

    (m2, d2), (m3, d3), (m4, d4) = (_edge_error(g, field) for g in (2, 3, 4))
    assert m2 / m3 > 3.2 and m3 / m4 > 3.5, (m2, m3, m4)
    assert 1.6 < d3 / d4 < 2.5, (d3, d4)
    assert m4 < d4 / 5


def test_angular_divergence_conservation_and_constant_field():
    """Through the Kerr-Schild geometry provider: sum_s w_s D_s = 0 for MAPR
    states; a constant field gives the donor-cell divergence."""
    import workloads as W
    from oracle.kerr import KerrSchildLogR
    wl = W.torus_ks(n=(4, 6, 2), a=0.9, generation=1, r_in=1.5, r_out=20.0)
    grid = GeodesicGrid(1)
    mk = lambda rec: KerrSchildLogR(wl["n"], wl["xlo"], wl["xhi"], grid, wl["a"], 1.0, recon=rec)
    geo_m, geo_d = mk("mapr"), mk("donor")
    rng = np.random.default_rng(9)
    I = torch.as_tensor(rng.random((grid.ns,) + tuple(wl["n"])) + 0.1, dtype=F64)
    D = geo_m.angular(I)
    w = torch.as_tensor(grid.w, dtype=F64).reshape(-1, 1, 1, 1)
    tot = (w * D).sum(0)
    assert float(tot.abs().max()) <= 1e-13 * float((w * D).abs().sum(0).max())
    assert float((D - geo_d.angular(I)).abs().max()) > 1e-3          # MAPR differs from donor
    C = torch.full_like(I, 0.7)
    assert torch.allclose(geo_m.angular(C), geo_d.angular(C), rtol=1e-13, atol=1e-15)
