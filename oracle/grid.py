"""Geodesic angular grid, paper Sec. 3.3 ("Geodesic Grid").

TEST INFRASTRUCTURE ONLY (see the package docstring).

Construction (Sec. 3.3): inscribe an icosahedron in the unit sphere, then g
times bisect every edge of the Delaunay triangulation, project the new points
onto the sphere and re-triangulate.  The angular cells are the Voronoi cells
of the resulting points: N_s = 10 * 4**g + 2, twelve pentagons, the rest
hexagons.

Conventions shared with the product through the documented interface only
(not through code):
  * the generation-0 icosahedron has a vertex on the +3 axis and a second one
    in the 1-3 half plane with positive 1 component (upper ring at azimuths
    2*pi*k/5, lower ring at 2*pi*k/5 + pi/5, then the south pole);
  * the points created by one subdivision are numbered after the existing
    ones, in lexicographic order of the (lower, higher) index pair of the edge
    they bisect.

Cell solid angles are computed here as a fan of spherical triangles
(n_s, c_k, c_k+1) over the circumcentres c_k ordered around n_s, with the
Van Oosterom-Strackee formula.
"""
import numpy as np


def _normalize(v):
    return v / np.sqrt(np.sum(v * v, axis=-1, keepdims=True))


def icosahedron():
    """Generation-0 grid: 12 unit vectors and 20 outward-oriented triangles."""
    zc = 1.0 / np.sqrt(5.0)
    rc = 2.0 / np.sqrt(5.0)
    pts = [(0.0, 0.0, 1.0)]
    for k in range(5):
        a = 2.0 * np.pi * k / 5.0
        pts.append((rc * np.cos(a), rc * np.sin(a), zc))
    for k in range(5):
        a = 2.0 * np.pi * k / 5.0 + np.pi / 5.0
        pts.append((rc * np.cos(a), rc * np.sin(a), -zc))
    pts.append((0.0, 0.0, -1.0))
    tris = []
    for k in range(5):
        k1 = (k + 1) % 5
        tris += [(0, 1 + k, 1 + k1), (1 + k, 6 + k, 1 + k1),
                 (1 + k1, 6 + k, 6 + k1), (11, 6 + k1, 6 + k)]
    V = np.array(pts, dtype=np.float64)
    return V, _orient(V, np.array(tris, dtype=np.int64))


def _orient(V, T):
    """Make every triangle counter-clockwise seen from outside the sphere."""
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    s = np.einsum("ij,ij->i", np.cross(b - a, c - a), a + b + c)
    T = T.copy()
    flip = s < 0
    T[flip] = T[flip][:, [0, 2, 1]]
    return T


def subdivide(V, T):
    """One refinement: bisect each edge, project to the sphere, split 1 -> 4."""
    edges = set()
    for t in T:
        for i, j in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
            edges.add((min(i, j), max(i, j)))
    edges = sorted(edges)
    mid = {}
    newpts = []
    for n, (i, j) in enumerate(edges):
        mid[(i, j)] = len(V) + n
        newpts.append(_normalize(V[i] + V[j]))
    V2 = np.vstack([V, np.array(newpts)])

    def m(i, j):
        return mid[(min(i, j), max(i, j))]

    T2 = []
    for a, b, c in T:
        ab, bc, ca = m(a, b), m(b, c), m(c, a)
        T2 += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
    return V2, _orient(V2, np.array(T2, dtype=np.int64))


def solid_angle(a, b, c):
    """Solid angle of the spherical triangle (a, b, c), Van Oosterom-Strackee."""
    num = abs(np.dot(a, np.cross(b, c)))
    den = 1.0 + np.dot(a, b) + np.dot(b, c) + np.dot(c, a)
    return 2.0 * np.arctan2(num, den)


class GeodesicGrid:
    """Directions, Voronoi solid angles and Voronoi edges of generation g.

    Attributes
      n      [N_s, 3] unit direction vectors n^hat (tetrad frame, Eq. n_vector)
      area   [N_s] Voronoi solid angles Delta Omega_s
      w      [N_s] quadrature weights (area, or 4 pi / N_s for 'equal')
      tris   [N_t, 3] Delaunay triangles (outward oriented)
      edges  [N_e, 2] neighbour pairs (s, s'), s < s'
      dlam   [N_e] Voronoi edge arc lengths Delta lambda
      emid   [N_e, 3] Voronoi edge midpoints
      enorm  [N_e, 3] unit edge normals, tangent at emid, pointing s -> s'
    """

    def __init__(self, generation, weights="voronoi"):
        V, T = icosahedron()
        for _ in range(generation):
            V, T = subdivide(V, T)
        self.generation = generation
        self.n = V
        self.tris = T
        ns = len(V)
        # circumcentres of the Delaunay triangles = Voronoi vertices
        a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
        cc = _normalize(np.cross(b - a, c - a))
        self.circum = cc
        # Voronoi polygon of each point: circumcentres ordered around it
        inc = [[] for _ in range(ns)]
        for t, tri in enumerate(T):
            for v in tri:
                inc[v].append(t)
        area = np.zeros(ns)
        for s in range(ns):
            p = V[s]
            e1 = _normalize(np.cross(p, [0.0, 0.0, 1.0]) if abs(p[2]) < 0.9
                            else np.cross(p, [1.0, 0.0, 0.0]))
            e2 = np.cross(p, e1)
            ang = [np.arctan2(np.dot(cc[t], e2), np.dot(cc[t], e1)) for t in inc[s]]
            ring = [inc[s][k] for k in np.argsort(ang)]
            for k in range(len(ring)):
                area[s] += solid_angle(p, cc[ring[k]], cc[ring[(k + 1) % len(ring)]])
        self.area = area
        self.degree = np.array([len(x) for x in inc])
        if weights == "voronoi":
            self.w = area.copy()
        elif weights == "equal":
            self.w = np.full(ns, 4.0 * np.pi / ns)
        else:
            raise ValueError(weights)
        # Voronoi edges: the two triangles sharing each Delaunay edge
        share = {}
        for t, (i, j, k) in enumerate(T):
            for u, v in ((i, j), (j, k), (k, i)):
                share.setdefault((min(u, v), max(u, v)), []).append(t)
        keys = sorted(share)
        self.edges = np.array(keys, dtype=np.int64)
        c1 = cc[[share[k][0] for k in keys]]
        c2 = cc[[share[k][1] for k in keys]]
        cr = np.cross(c1, c2)
        self.dlam = np.arctan2(np.sqrt(np.sum(cr * cr, axis=1)), np.sum(c1 * c2, axis=1))
        self.emid = _normalize(c1 + c2)
        d = V[self.edges[:, 1]] - V[self.edges[:, 0]]
        # tangent at the midpoint, perpendicular to the edge, towards s'
        d = d - np.sum(d * self.emid, axis=1, keepdims=True) * self.emid
        self.enorm = _normalize(d)

    @property
    def ns(self):
        return len(self.n)
