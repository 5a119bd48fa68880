// Geodesic grid construction (paper Sec. 3.3): an icosahedron inscribed in
// the unit sphere, refined g times by bisecting every Delaunay edge and
// projecting the midpoints onto the sphere; the angular cells are the Voronoi
// cells of the points.
//
// Solid angles are accumulated per Delaunay triangle: the part of triangle
// (a, b, c) closest to vertex a is the spherical quadrilateral bounded by the
// arc midpoints of ab and ac and the triangle's circumcentre, split into two
// spherical triangles whose solid angles use the Van Oosterom-Strackee
// formula.  (All geodesic-grid triangles are acute, so every circumcentre
// lies inside its triangle.)
#include "grid.hpp"

#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <utility>

namespace rt {
namespace {

using V3 = std::array<double, 3>;

V3 add(const V3& a, const V3& b) { return {a[0] + b[0], a[1] + b[1], a[2] + b[2]}; }
V3 sub(const V3& a, const V3& b) { return {a[0] - b[0], a[1] - b[1], a[2] - b[2]}; }
V3 scale(const V3& a, double s) { return {a[0] * s, a[1] * s, a[2] * s}; }
double dot(const V3& a, const V3& b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
V3 cross(const V3& a, const V3& b) {
  return {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
}
V3 unit(const V3& a) { return scale(a, 1.0 / std::sqrt(dot(a, a))); }

double tri_solid_angle(const V3& a, const V3& b, const V3& c) {
  double num = std::fabs(dot(a, cross(b, c)));
  double den = 1.0 + dot(a, b) + dot(b, c) + dot(c, a);
  return 2.0 * std::atan2(num, den);
}

void orient_outward(const std::vector<V3>& p, std::array<int, 3>& t) {
  V3 n = cross(sub(p[t[1]], p[t[0]]), sub(p[t[2]], p[t[0]]));
  if (dot(n, add(add(p[t[0]], p[t[1]]), p[t[2]])) < 0) std::swap(t[1], t[2]);
}

std::pair<int, int> key(int i, int j) { return i < j ? std::make_pair(i, j) : std::make_pair(j, i); }

}  // namespace

GeodesicGrid build_geodesic_grid(int g, bool equal_weights) {
  if (g < 0 || g > 5) throw std::invalid_argument("generation must be in 0..5");
  const double kPi = 3.14159265358979323846;
  std::vector<V3> p;
  std::vector<std::array<int, 3>> tris;
  // generation 0: pole-aligned regular icosahedron
  const double zc = 1.0 / std::sqrt(5.0), rc = 2.0 / std::sqrt(5.0);
  p.push_back({0.0, 0.0, 1.0});
  for (int k = 0; k < 5; ++k) {
    double phi = 2.0 * kPi * k / 5.0;
    p.push_back({rc * std::cos(phi), rc * std::sin(phi), zc});
  }
  for (int k = 0; k < 5; ++k) {
    double phi = 2.0 * kPi * k / 5.0 + kPi / 5.0;
    p.push_back({rc * std::cos(phi), rc * std::sin(phi), -zc});
  }
  p.push_back({0.0, 0.0, -1.0});
  for (int k = 0; k < 5; ++k) {
    int k1 = (k + 1) % 5;
    tris.push_back({0, 1 + k, 1 + k1});
    tris.push_back({1 + k, 6 + k, 1 + k1});
    tris.push_back({1 + k1, 6 + k, 6 + k1});
    tris.push_back({11, 6 + k1, 6 + k});
  }
  for (auto& t : tris) orient_outward(p, t);

  for (int level = 0; level < g; ++level) {
    std::vector<std::pair<int, int>> edges;
    edges.reserve(tris.size() * 3);
    for (const auto& t : tris)
      for (int e = 0; e < 3; ++e) edges.push_back(key(t[e], t[(e + 1) % 3]));
    std::sort(edges.begin(), edges.end());
    edges.erase(std::unique(edges.begin(), edges.end()), edges.end());
    const int base = static_cast<int>(p.size());
    for (const auto& e : edges) p.push_back(unit(add(p[e.first], p[e.second])));
    auto mid = [&](int i, int j) {
      auto it = std::lower_bound(edges.begin(), edges.end(), key(i, j));
      return base + static_cast<int>(it - edges.begin());
    };
    std::vector<std::array<int, 3>> next;
    next.reserve(tris.size() * 4);
    for (const auto& t : tris) {
      int a = t[0], b = t[1], c = t[2];
      int ab = mid(a, b), bc = mid(b, c), ca = mid(c, a);
      next.push_back({a, ab, ca});
      next.push_back({b, bc, ab});
      next.push_back({c, ca, bc});
      next.push_back({ab, bc, ca});
    }
    for (auto& t : next) orient_outward(p, t);
    tris.swap(next);
  }

  GeodesicGrid G;
  G.generation = g;
  G.ns = static_cast<int>(p.size());
  G.dir = p;
  G.tri = tris;
  G.area.assign(G.ns, 0.0);
  std::vector<V3> cc(tris.size());
  for (size_t t = 0; t < tris.size(); ++t) {
    const V3 &a = p[tris[t][0]], &b = p[tris[t][1]], &c = p[tris[t][2]];
    cc[t] = unit(cross(sub(b, a), sub(c, a)));
    for (int v = 0; v < 3; ++v) {
      const V3& x = p[tris[t][v]];
      V3 m1 = unit(add(x, p[tris[t][(v + 1) % 3]]));
      V3 m2 = unit(add(x, p[tris[t][(v + 2) % 3]]));
      G.area[tris[t][v]] += tri_solid_angle(x, m1, cc[t]) + tri_solid_angle(x, cc[t], m2);
    }
  }
  G.w = equal_weights ? std::vector<double>(G.ns, 4.0 * kPi / G.ns) : G.area;

  // Voronoi edges: circumcentres of the two triangles sharing each Delaunay edge
  std::vector<std::pair<std::pair<int, int>, int>> half;
  half.reserve(tris.size() * 3);
  for (size_t t = 0; t < tris.size(); ++t)
    for (int e = 0; e < 3; ++e)
      half.push_back({key(tris[t][e], tris[t][(e + 1) % 3]), static_cast<int>(t)});
  std::sort(half.begin(), half.end());
  for (size_t k = 0; k + 1 < half.size(); k += 2) {
    if (half[k].first != half[k + 1].first) throw std::runtime_error("non-manifold triangulation");
    int s = half[k].first.first, t = half[k].first.second;
    const V3 &c1 = cc[half[k].second], &c2 = cc[half[k + 1].second];
    V3 cr = cross(c1, c2);
    G.edge.push_back({s, t});
    G.dlam.push_back(std::atan2(std::sqrt(dot(cr, cr)), dot(c1, c2)));
    V3 m = unit(add(c1, c2));
    G.emid.push_back(m);
    V3 d = sub(p[t], p[s]);
    G.enorm.push_back(unit(sub(d, scale(m, dot(d, m)))));
  }
  return G;
}

}  // namespace rt
