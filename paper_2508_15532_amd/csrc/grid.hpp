// Host-side geodesic angular grid (paper Sec. 3.3) and the per-direction
// tables the kernels read.
#pragma once
#include <array>
#include <vector>

namespace rt {

struct GeodesicGrid {
  int generation = 0;
  int ns = 0;
  std::vector<std::array<double, 3>> dir;   // unit directions n-hat_s
  std::vector<std::array<int, 3>> tri;      // Delaunay triangles, outward CCW
  std::vector<double> area;                 // Voronoi solid angle of each cell
  std::vector<double> w;                    // quadrature weights
  // Voronoi edges, one per Delaunay edge (s < t)
  std::vector<std::array<int, 2>> edge;
  std::vector<double> dlam;                 // arc length of the Voronoi edge
  std::vector<std::array<double, 3>> emid;  // its midpoint (unit vector)
  std::vector<std::array<double, 3>> enorm; // unit tangent normal, s -> t
};

// Builds generation g (0..5) with Voronoi (equal_weights = false) or
// 4 pi / Ns weights.  Numbering: see rt_init_grid in rt.h.
GeodesicGrid build_geodesic_grid(int g, bool equal_weights);

}  // namespace rt
