"""MAPR angular reconstruction on the geodesic grid (Sec. 3.4; the states at
the Voronoi edges for the angular fluxes; the paper names the minimum-angle
plane reconstruction of its cited source and donor cell as the alternative).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper names the method without spelling it out.  Reading used here:
  * the neighbours x_j of a direction n_s are projected gnomonically onto the
    plane tangent to the unit sphere at n_s: p_s(x) = x / (x . n_s) - n_s
    (a tangent vector: p_s(x) . n_s = 0);
  * the neighbours are taken in their cyclic order around n_s; each
    consecutive pair (a, b) fixes the plane through (0, I_s), (p_a, I_a),
    (p_b, I_b): the tangent slope vector g in span(p_a, p_b) with
    g . p_a = I_a - I_s and g . p_b = I_b - I_s;
  * of these planes the one with the smallest slope |g| (the smallest angle
    with the tangent plane) is taken.  Ties are common (a symmetric
    neighbourhood with equal or zeroed intensities gives congruent planes of
    equal slope) and rounding must not decide them: every plane whose |g|^2 is
    within a relative TIE_RTOL of the smallest counts as minimal, and the first
    of them is taken, in counter-clockwise order (seen from outside the sphere)
    starting at the neighbour with the smallest direction index;
  * the state of s at a point m of its Voronoi cell is I_s + g . p_s(m),
    replaced by I_s where that is negative.
The angular flux across an edge takes the state of its upwind direction at the
edge midpoint.

Parity unpinned as a reading (the paper does not fix these details); the
functions below are pinned to the properties that the reading implies.
"""
import numpy as np
import torch

F64 = torch.float64
# relative |g|^2 band of the minimal planes: at the rounding level of the
# arithmetic that compares them, 1e-8 for the FP64 form and 1e-4 for the FP32
# transport form (whose slopes carry ~1e-7 relative rounding)
TIE_RTOL = 1e-8
TIE_RTOL_FP32 = 1e-4


def gnomonic(n_s, x):
    """p_s(x) = x / (x . n_s) - n_s for x [..., 3] (points of the hemisphere of n_s)."""
    x = np.asarray(x, dtype=np.float64)
    return x / (x @ n_s)[..., None] - n_s


def rings(grid):
    """For every direction, its neighbours in counter-clockwise order seen from
    outside the sphere, starting at the neighbour with the smallest index."""
    nb = [[] for _ in range(grid.ns)]
    for a, b in grid.edges:
        nb[a].append(int(b))
        nb[b].append(int(a))
    out = []
    for s in range(grid.ns):
        n = grid.n[s]
        P = gnomonic(n, grid.n[nb[s]])
        ref = P[0] / np.linalg.norm(P[0])
        perp = np.cross(n, ref)
        ang = np.arctan2(P @ perp, P @ ref)
        r = [nb[s][k] for k in np.argsort(ang, kind="stable")]
        k0 = r.index(min(r))
        out.append(r[k0:] + r[:k0])
    return out


def pair_slope(pa, pb, dA, dB):
    """The tangent vector g = alpha p_a + beta p_b with g . p_a = dA, g . p_b = dB
    (the 2x2 Gram system); dA, dB tensors of any shape -> [..., 3]."""
    g00, g01, g11 = float(pa @ pa), float(pa @ pb), float(pb @ pb)
    det = g00 * g11 - g01 * g01
    alpha = (g11 * dA - g01 * dB) / det
    beta = (g00 * dB - g01 * dA) / det
    return (alpha[..., None] * torch.as_tensor(pa, dtype=F64)
            + beta[..., None] * torch.as_tensor(pb, dtype=F64))


def slopes(grid, I, ring=None, tie_rtol=TIE_RTOL):
    """Minimum-norm slope vector g_s for every direction and cell: [Ns, *cells, 3]."""
    ring = ring if ring is not None else rings(grid)
    I = torch.as_tensor(I, dtype=F64)
    out = torch.zeros(I.shape + (3,), dtype=F64)
    for s in range(grid.ns):
        n = grid.n[s]
        r = ring[s]
        P = gnomonic(n, grid.n[r])
        cand = []
        for k in range(len(r)):
            a, b = k, (k + 1) % len(r)
            cand.append(pair_slope(P[a], P[b], I[r[a]] - I[s], I[r[b]] - I[s]))
        cand = torch.stack(cand)                               # [deg, *cells, 3]
        norms = (cand * cand).sum(-1)                          # [deg, *cells]
        minimal = norms <= norms.min(0).values * (1.0 + tie_rtol)
        first = minimal.to(torch.int64).argmax(0)              # first minimal plane
        out[s] = torch.gather(cand, 0, first[None, ..., None].expand((1,) + cand.shape[1:]))[0]
    return out


def state(n_s, I_s, g_s, m):
    """State of direction n_s at the point m of its cell: I_s + g_s . p_s(m),
    I_s where that is negative."""
    p = torch.as_tensor(gnomonic(n_s, m), dtype=F64)
    v = I_s + (g_s * p).sum(-1)
    return torch.where(v < 0, I_s, v)


def edge_states(grid, I, ring=None, tie_rtol=TIE_RTOL):
    """States at every Voronoi edge midpoint from the edge's first and its second
    direction: two tensors [Ne, *cells]."""
    I = torch.as_tensor(I, dtype=F64)
    g = slopes(grid, I, ring, tie_rtol)
    ne = len(grid.edges)
    first = torch.zeros((ne,) + I.shape[1:], dtype=F64)
    second = torch.zeros_like(first)
    for e, (s, t) in enumerate(grid.edges):
        m = grid.emid[e]
        first[e] = state(grid.n[s], I[s], g[s], m)
        second[e] = state(grid.n[t], I[t], g[t], m)
    return first, second
