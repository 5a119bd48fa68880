// Kerr-Schild geometry tables (host, FP64).
//
// Metric (Sec. 2.1.1 uses a fixed stationary metric; the torus tests of Sec. 5
// use Kerr-Schild coordinates), with Sigma = r^2 + a^2 cos^2 theta and
// z = 2 M r / Sigma, in (t, x1 = ln r, theta, phi) -- every r index carries a
// factor r:
//   g_tt = -(1 - z)      g_t1 = z r             g_tph = -z a sin^2
//   g_11 = (1 + z) r^2   g_1ph = -a (1 + z) r sin^2
//   g_thth = Sigma       g_phph = sin^2 (Sigma + a^2 (1 + z) sin^2)
//
// Tetrad (Sec. 2.1.1): the time leg is the normal observer, e_0 = -g^(0 mu) /
// sqrt(-g^00); the spatial legs come from Gram-Schmidt of (d_phi, d_theta,
// d_x1) in the spatial metric and are numbered (3, 2, 1).  The tetrad then
// satisfies e e g = eta, and the geodesic grid's pole lies along phi-hat.
//
// Angular motion (Sec. 2.2): with the rotation coefficients
// omega^a_(c d) = e^a_b e^mu_c (d_mu e^b_d + Gamma^b_(mu l) e^l_d), a photon of
// tetrad direction n (n^0 = 1) turns at the rate
// r^i = -omega^i_(c d) n^c n^d + n^i omega^0_(c d) n^c n^d per unit of the
// affine parameter with dx/dlambda = n^mu (the geodesic equation written in
// the tetrad basis).  The flux through a Voronoi edge of the geodesic grid
// (Sec. 3.5, donor-cell states) is n_0(m_e) (r(m_e) . u_e) dlambda_e I_upwind.
// Derivatives are fourth-order central differences of the analytic metric and
// tetrad.
#include "kerr.hpp"

#include <cmath>
#include <stdexcept>

namespace rt {
namespace {

using M4 = double[4][4];

void ks_metric(double x1, double th, double a, double M, M4 g) {
  const double r = std::exp(x1), s = std::sin(th), c = std::cos(th);
  const double Sig = r * r + a * a * c * c, z = 2.0 * M * r / Sig, s2 = s * s;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) g[i][j] = 0.0;
  g[0][0] = -(1.0 - z);
  g[0][1] = g[1][0] = z * r;
  g[0][3] = g[3][0] = -z * a * s2;
  g[1][1] = (1.0 + z) * r * r;
  g[1][3] = g[3][1] = -a * (1.0 + z) * s2 * r;
  g[2][2] = Sig;
  g[3][3] = s2 * (Sig + a * a * (1.0 + z) * s2);
}

double ks_sqrt_mg(double x1, double th, double a) {
  const double r = std::exp(x1), c = std::cos(th);
  return r * (r * r + a * a * c * c) * std::fabs(std::sin(th));
}

// Gauss-Jordan inverse with partial pivoting
void inverse4(const M4 A, M4 out) {
  double m[4][8];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      m[i][j] = A[i][j];
      m[i][j + 4] = i == j ? 1.0 : 0.0;
    }
  for (int col = 0; col < 4; ++col) {
    int piv = col;
    for (int r = col + 1; r < 4; ++r)
      if (std::fabs(m[r][col]) > std::fabs(m[piv][col])) piv = r;
    if (piv != col)
      for (int j = 0; j < 8; ++j) std::swap(m[col][j], m[piv][j]);
    const double inv = 1.0 / m[col][col];
    for (int j = 0; j < 8; ++j) m[col][j] *= inv;
    for (int r = 0; r < 4; ++r) {
      if (r == col) continue;
      const double f = m[r][col];
      if (f != 0.0)
        for (int j = 0; j < 8; ++j) m[r][j] -= f * m[col][j];
    }
  }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) out[i][j] = m[i][j + 4];
}

// e[mu][a] = e^mu_(a-hat)
void tetrad(const M4 g, M4 e) {
  M4 gi;
  inverse4(g, gi);
  for (int mu = 0; mu < 4; ++mu) e[mu][0] = -gi[0][mu] / std::sqrt(-gi[0][0]);
  auto dot = [&](const double* u, const double* v) {
    double s = 0.0;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) s += u[i] * g[i + 1][j + 1] * v[j];
    return s;
  };
  double legs[3][3];
  const int order[3] = {2, 1, 0};  // d_phi, d_theta, d_x1 -> legs 3, 2, 1
  for (int q = 0; q < 3; ++q) {
    double v[3] = {0.0, 0.0, 0.0};
    v[order[q]] = 1.0;
    for (int p = 0; p < q; ++p) {
      const double d = dot(v, legs[p]);
      for (int i = 0; i < 3; ++i) v[i] -= d * legs[p][i];
    }
    const double nrm = std::sqrt(dot(v, v));
    for (int i = 0; i < 3; ++i) legs[q][i] = v[i] / nrm;
  }
  for (int q = 0; q < 3; ++q) {
    const int hat = 3 - q;
    e[0][hat] = 0.0;
    for (int i = 0; i < 3; ++i) e[i + 1][hat] = legs[q][i];
  }
}

// einv[a][mu] = eta^(a b) g_(mu nu) e^nu_b
void inverse_tetrad(const M4 g, const M4 e, M4 einv) {
  for (int a = 0; a < 4; ++a)
    for (int mu = 0; mu < 4; ++mu) {
      double s = 0.0;
      for (int nu = 0; nu < 4; ++nu) s += g[mu][nu] * e[nu][a];
      einv[a][mu] = a == 0 ? -s : s;
    }
}

struct Point {
  M4 g, e, einv;
};

Point at(double x1, double th, double a, double M) {
  Point p;
  ks_metric(x1, th, a, M, p.g);
  tetrad(p.g, p.e);
  inverse_tetrad(p.g, p.e, p.einv);
  return p;
}

// omega[a][c][d] at (x1, theta)
void rotation_coefficients(double x1, double th, double a, double M, double h, double om[4][4][4]) {
  const Point P = at(x1, th, a, M);
  M4 gi;
  inverse4(P.g, gi);
  double dg[4][4][4] = {};  // dg[mu][n][l] = d_mu g_(n l)
  double de[4][4][4] = {};  // de[mu][b][d] = d_mu e^b_d
  // fourth-order central differences, weights (1, -8, 8, -1) / 12h at -2h .. 2h
  for (int mu = 1; mu <= 2; ++mu) {
    const double d1 = mu == 1 ? h : 0.0, d2 = mu == 2 ? h : 0.0;
    const Point p2 = at(x1 + 2 * d1, th + 2 * d2, a, M), p1 = at(x1 + d1, th + d2, a, M);
    const Point m1 = at(x1 - d1, th - d2, a, M), m2 = at(x1 - 2 * d1, th - 2 * d2, a, M);
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) {
        dg[mu][i][j] = (8.0 * (p1.g[i][j] - m1.g[i][j]) - (p2.g[i][j] - m2.g[i][j])) / (12.0 * h);
        de[mu][i][j] = (8.0 * (p1.e[i][j] - m1.e[i][j]) - (p2.e[i][j] - m2.e[i][j])) / (12.0 * h);
      }
  }
  // Gamma^b_(mu l) = 1/2 g^(b n) (d_mu g_(n l) + d_l g_(n mu) - d_n g_(mu l))
  double Gam[4][4][4];
  for (int b = 0; b < 4; ++b)
    for (int mu = 0; mu < 4; ++mu)
      for (int l = 0; l < 4; ++l) {
        double s = 0.0;
        for (int n = 0; n < 4; ++n) s += gi[b][n] * (dg[mu][n][l] + dg[l][n][mu] - dg[n][mu][l]);
        Gam[b][mu][l] = 0.5 * s;
      }
  // nab[b][mu][d] = d_mu e^b_d + Gamma^b_(mu l) e^l_d
  double nab[4][4][4];
  for (int b = 0; b < 4; ++b)
    for (int mu = 0; mu < 4; ++mu)
      for (int d = 0; d < 4; ++d) {
        double s = de[mu][b][d];
        for (int l = 0; l < 4; ++l) s += Gam[b][mu][l] * P.e[l][d];
        nab[b][mu][d] = s;
      }
  for (int A = 0; A < 4; ++A)
    for (int c = 0; c < 4; ++c)
      for (int d = 0; d < 4; ++d) {
        double s = 0.0;
        for (int b = 0; b < 4; ++b)
          for (int mu = 0; mu < 4; ++mu) s += P.einv[A][b] * P.e[mu][c] * nab[b][mu][d];
        om[A][c][d] = s;
      }
}

int sgn(double x) { return (x > 0.0) - (x < 0.0); }

}  // namespace

KsTables build_ks_tables(const GeodesicGrid& G, const int n[3], const double xlo[3],
                         const double xhi[3], double a, double M, double n0_cut, double cfl,
                         double fd_h) {
  if (!(xlo[1] >= 0.0) || !(xhi[1] <= M_PI + 1e-12))
    throw std::invalid_argument("theta range must lie in [0, pi]");
  KsTables T;
  const int N1 = n[0], N2 = n[1], N3 = n[2], ns = G.ns, ne = (int)G.edge.size();
  T.n1 = N1;
  T.n2 = N2;
  T.ns = ns;
  T.ne = ne;
  const double dx[3] = {(xhi[0] - xlo[0]) / N1, (xhi[1] - xlo[1]) / N2, (xhi[2] - xlo[2]) / N3};
  // the difference stencil of the rotation coefficients must stay off the axis
  if (!(xlo[1] + 0.5 * dx[1] - 2.0 * fd_h > 0.0) || !(xlo[1] + (N2 - 0.5) * dx[1] + 2.0 * fd_h < M_PI))
    throw std::invalid_argument("theta cell centres must lie more than 2 fd_h from the axis");
  auto x1c = [&](int i) { return xlo[0] + (i + 0.5) * dx[0]; };
  auto thc = [&](int j) { return xlo[1] + (j + 0.5) * dx[1]; };
  auto x1f = [&](int i) { return xlo[0] + i * dx[0]; };
  auto thf = [&](int j) { return xlo[1] + j * dx[1]; };
  const size_t nrt = (size_t)N1 * N2;

  // n^mu of every direction at a point: e^mu_0 + e^mu_i n-hat^i
  auto nup = [&](const Point& P, int s, int mu) {
    return P.e[mu][0] + P.e[mu][1] * G.dir[s][0] + P.e[mu][2] * G.dir[s][1] + P.e[mu][3] * G.dir[s][2];
  };
  auto nlow0 = [&](const Point& P, int s) {
    double v = 0.0;
    for (int mu = 0; mu < 4; ++mu) v += P.g[0][mu] * nup(P, s, mu);
    return v;
  };

  // ---- centres
  std::vector<double> nl0c((size_t)ns * nrt);
  T.dV.resize(nrt);
  T.nu0.resize(nrt);
  T.e.resize(nrt * 16);
  T.einv.resize(nrt * 16);
  T.fp.assign((size_t)ns * nrt * 4, 0.0);
  double vmax[3] = {0.0, 0.0, 0.0};
  std::vector<double> nuphi((size_t)ns * nrt);
  for (int i = 0; i < N1; ++i)
    for (int j = 0; j < N2; ++j) {
      const size_t q = (size_t)i * N2 + j;
      const Point P = at(x1c(i), thc(j), a, M);
      const double sg = ks_sqrt_mg(x1c(i), thc(j), a);
      T.dV[q] = sg * dx[0] * dx[1] * dx[2];
      T.nu0[q] = P.e[0][0];
      for (int mu = 0; mu < 4; ++mu)
        for (int b = 0; b < 4; ++b) {
          T.e[q * 16 + mu * 4 + b] = P.e[mu][b];
          T.einv[q * 16 + b * 4 + mu] = P.einv[b][mu];
        }
      const double dAphi = sg * dx[0] * dx[1];
      for (int s = 0; s < ns; ++s) {
        const double n0 = nup(P, s, 0), nl = nlow0(P, s), nph = nup(P, s, 3);
        nl0c[(size_t)s * nrt + q] = nl;
        nuphi[(size_t)s * nrt + q] = nph;
        for (int ax = 0; ax < 3; ++ax) vmax[ax] = std::max(vmax[ax], std::fabs(nup(P, s, ax + 1) / n0));
        double* r = &T.fp[((size_t)s * nrt + q) * 4];
        const double base = dAphi * nl;
        r[0] = nph > 0.0 ? base * nph : 0.0;
        r[1] = nph < 0.0 ? base * nph : 0.0;
        r[2] = base * T.nu0[q];
        r[3] = std::fabs(nl) < n0_cut ? 0.0 : 1.0 / (T.dV[q] * (T.nu0[q] * nl));
      }
    }
  T.dt_max = INFINITY;
  for (int ax = 0; ax < 3; ++ax) T.dt_max = std::min(T.dt_max, dx[ax] / vmax[ax]);
  T.dt_max *= cfl;

  // ---- faces normal to x1 and theta
  T.fr.assign((size_t)ns * (N1 + 1) * N2 * 4, 0.0);
  T.ft.assign((size_t)ns * N1 * (N2 + 1) * 4, 0.0);
  T.zin_stride = 2 * N2 + 2 * N1 + 2 * N1 * N2;
  T.zin.assign((size_t)ns * T.zin_stride, 0);
  for (int i = 0; i <= N1; ++i)
    for (int j = 0; j < N2; ++j) {
      const Point P = at(x1f(i), thc(j), a, M);
      const double dA = ks_sqrt_mg(x1f(i), thc(j), a) * dx[1] * dx[2];
      const size_t q = (size_t)i * N2 + j, nf = (size_t)(N1 + 1) * N2;
      for (int s = 0; s < ns; ++s) {
        const double nu = nup(P, s, 1), nl = nlow0(P, s);
        bool ok = true;
        if (i > 0 && i < N1)
          ok = sgn(nl0c[(size_t)s * nrt + (size_t)(i - 1) * N2 + j]) ==
               sgn(nl0c[(size_t)s * nrt + (size_t)i * N2 + j]);
        double* r = &T.fr[((size_t)s * nf + q) * 4];
        const double base = ok ? dA * nl : 0.0;
        r[0] = nu > 0.0 ? base * nu : 0.0;
        r[1] = nu < 0.0 ? base * nu : 0.0;
        r[2] = base * P.e[0][0];
        unsigned char* z = &T.zin[(size_t)s * T.zin_stride];
        if (i == 0) z[j] = nu > 0.0;
        if (i == N1) z[N2 + j] = nu < 0.0;
      }
    }
  for (int i = 0; i < N1; ++i)
    for (int j = 0; j <= N2; ++j) {
      double th = thf(j);
      // the tetrad is singular on the axis; pole faces have zero area and no
      // flux, so their factors are taken just off the axis
      const bool pole = std::fabs(std::sin(th)) < 1e-12;
      const double ths = pole ? th + (th < 1.0 ? 1e-8 : -1e-8) : th;
      const Point P = at(x1c(i), ths, a, M);
      const double dA = ks_sqrt_mg(x1c(i), th, a) * dx[0] * dx[2];
      const size_t q = (size_t)i * (N2 + 1) + j, nf = (size_t)N1 * (N2 + 1);
      for (int s = 0; s < ns; ++s) {
        const double nu = pole ? 0.0 : nup(P, s, 2), nl = nlow0(P, s);
        bool ok = true;
        if (j > 0 && j < N2)
          ok = sgn(nl0c[(size_t)s * nrt + (size_t)i * N2 + j - 1]) ==
               sgn(nl0c[(size_t)s * nrt + (size_t)i * N2 + j]);
        double* r = &T.ft[((size_t)s * nf + q) * 4];
        const double base = ok ? dA * nl : 0.0;
        r[0] = nu > 0.0 ? base * nu : 0.0;
        r[1] = nu < 0.0 ? base * nu : 0.0;
        r[2] = base * P.e[0][0];
        unsigned char* z = &T.zin[(size_t)s * T.zin_stride];
        if (j == 0) z[2 * N2 + i] = nu > 0.0;
        if (j == N2) z[2 * N2 + N1 + i] = nu < 0.0;
      }
    }
  for (int s = 0; s < ns; ++s) {
    unsigned char* z = &T.zin[(size_t)s * T.zin_stride + 2 * N2 + 2 * N1];
    for (size_t q = 0; q < nrt; ++q) {
      const double nph = nuphi[(size_t)s * nrt + q];
      z[q] = nph > 0.0;
      z[nrt + q] = nph < 0.0;
    }
  }

  // ---- geodesic-edge velocities per (r, theta)
  T.ve.assign(nrt * ne * 2, 0.0);
  for (int i = 0; i < N1; ++i)
    for (int j = 0; j < N2; ++j) {
      const size_t q = (size_t)i * N2 + j;
      double om[4][4][4];
      rotation_coefficients(x1c(i), thc(j), a, M, fd_h, om);
      M4 g;
      ks_metric(x1c(i), thc(j), a, M, g);
      const Point P = at(x1c(i), thc(j), a, M);
      for (int e = 0; e < ne; ++e) {
        const double m4[4] = {1.0, G.emid[e][0], G.emid[e][1], G.emid[e][2]};
        double qv[4];
        for (int A = 0; A < 4; ++A) {
          double s = 0.0;
          for (int c = 0; c < 4; ++c)
            for (int d = 0; d < 4; ++d) s += om[A][c][d] * m4[c] * m4[d];
          qv[A] = s;
        }
        double v = 0.0;
        for (int k = 0; k < 3; ++k) v += (-qv[k + 1] + m4[k + 1] * qv[0]) * G.enorm[e][k];
        double n0e = 0.0;
        for (int mu = 0; mu < 4; ++mu) {
          double nm = 0.0;
          for (int b = 0; b < 4; ++b) nm += P.e[mu][b] * m4[b];
          n0e += g[0][mu] * nm;
        }
        const double f = G.dlam[e] * n0e * v;
        T.ve[(q * ne + e) * 2 + 0] = v > 0.0 ? f : 0.0;
        T.ve[(q * ne + e) * 2 + 1] = v > 0.0 ? 0.0 : f;
      }
    }

  // ---- incidence lists
  T.inc_off.assign(ns + 1, 0);
  for (int e = 0; e < ne; ++e) {
    ++T.inc_off[G.edge[e][0] + 1];
    ++T.inc_off[G.edge[e][1] + 1];
  }
  for (int s = 0; s < ns; ++s) T.inc_off[s + 1] += T.inc_off[s];
  T.inc_edge.resize(T.inc_off[ns]);
  T.inc_other.resize(T.inc_off[ns]);
  T.inc_side.resize(T.inc_off[ns]);
  std::vector<int> fill(T.inc_off.begin(), T.inc_off.end() - 1);
  for (int e = 0; e < ne; ++e) {
    const int s = G.edge[e][0], t = G.edge[e][1];
    int k = fill[s]++;
    T.inc_edge[k] = e;
    T.inc_other[k] = t;
    T.inc_side[k] = 1;
    k = fill[t]++;
    T.inc_edge[k] = e;
    T.inc_other[k] = s;
    T.inc_side[k] = -1;
  }

  // ---- angular coefficients: the edge flux F_e = vP I_first + vN I_second
  // enters direction s with + (s first) or - (s second)
  const int ninc = T.inc_off[ns];
  T.acoef.assign(nrt * (ns + ninc), 0.0);
  for (size_t q = 0; q < nrt; ++q) {
    double* A = &T.acoef[q * (ns + ninc)];
    for (int s = 0; s < ns; ++s) {
      const double x = T.fp[((size_t)s * nrt + q) * 4 + 3];
      const double scale = x * T.dV[q] / G.w[s];  // 1/(w_s n^0 n_0), 0 below the cut
      double diag = 0.0;
      for (int k = T.inc_off[s]; k < T.inc_off[s + 1]; ++k) {
        const double vP = T.ve[(q * ne + T.inc_edge[k]) * 2], vN = T.ve[(q * ne + T.inc_edge[k]) * 2 + 1];
        if (T.inc_side[k] > 0) {
          diag += vP;
          A[ns + k] = scale * vN;
        } else {
          diag -= vN;
          A[ns + k] = -scale * vP;
        }
      }
      A[s] = scale * diag;
    }
  }
  return T;
}

}  // namespace rt
