// Host-built geometry of the Kerr-Schild metric on a (x1 = ln r, theta, phi)
// mesh: everything the transport needs per (r, theta) position and direction.
// The metric is stationary and axisymmetric, so no table depends on phi.
#pragma once
#include <vector>

#include "grid.hpp"

namespace rt {

struct KsTables {
  int n1 = 0, n2 = 0, ns = 0, ne = 0;
  // Per direction s and face: {gP, gN, gA, x}.  The area-weighted flux through
  // a face is gP F+(...) + gN F-(...) + gA adv(...), where
  //   gP = dA n_0 n^a   if n^a > 0 (else 0),   gN = dA n_0 n^a   if n^a < 0,
  //   gA = dA n_0 n^0   (advection term),
  // all zero where n_0 changes sign between the two cells of the face.
  // For centre records x = 1 / (dV n^0 n_0), zero where |n_0| < n0_cut.
  std::vector<double> fr;  // [ns][(n1+1)*n2][4]  faces normal to x1
  std::vector<double> ft;  // [ns][n1*(n2+1)][4]  faces normal to theta
  std::vector<double> fp;  // [ns][n1*n2][4]      faces normal to phi (x = centre record)
  // incoming flags of the boundary faces for zero-incoming ghosts:
  // [ns][2*n2 (x1 lo, hi) + 2*n1 (theta lo, hi) + 2*n1*n2 (phi lo, hi)]
  std::vector<unsigned char> zin;
  int zin_stride = 0;
  // geodesic-edge fluxes per (r, theta): F_e = vP_e I_s + vN_e I_t with
  // vP = dlambda n_0(m_e) v_e for v_e > 0 (else 0), vN likewise for v_e <= 0
  std::vector<double> ve;  // [n1*n2][ne][2]
  std::vector<double> dV;  // [n1*n2] cell volume sqrt(-g) dx1 dtheta dphi
  std::vector<double> nu0; // [n1*n2] n^0 = 1/lapse at the centre
  std::vector<double> e;    // [n1*n2][16] tetrad e^mu_a at the centre, [mu*4 + a]
  std::vector<double> einv; // [n1*n2][16] inverse tetrad e^a_mu, [a*4 + mu]
  // incidence lists of the directions: for direction s, entries
  // inc[inc_off[s] .. inc_off[s+1]) = (edge, other direction, +1 if s is the
  // edge's first vertex else -1)
  std::vector<int> inc_off, inc_edge, inc_other, inc_side;
  // angular flux divergence as the update needs it, per (r, theta):
  // D'_s = acoef[s] I_s + sum_k acoef[ns + k] I_(other k), k over the incidences
  // of s; the factors 1/w_s and 1/(n^0 n_0) (zero below the n_0 cut) are folded in
  std::vector<double> acoef;  // [n1*n2][ns + ninc]
  double dt_max = 0.0;  // cfl * min over cells and axes of dx^a / max_s |n^a / n^0|
};

// Builds the tables for spin a and mass M on the mesh n, [xlo, xhi] with the
// given geodesic grid.  Rotation coefficients come from fourth-order central
// differences with step fd_h of the analytic metric and tetrad.  Throws std::invalid_argument
// when the mesh reaches r <= 0 or theta outside [0, pi].
KsTables build_ks_tables(const GeodesicGrid& g, const int n[3], const double xlo[3],
                         const double xhi[3], double a, double M, double n0_cut, double cfl,
                         double fd_h);

}  // namespace rt
