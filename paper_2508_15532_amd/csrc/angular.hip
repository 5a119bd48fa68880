// Angular flux divergence of the curved geometry (Sec. 3.5, geodesic-edge
// fluxes; donor-cell states).
//
// In a curved metric a photon's tetrad direction turns along its ray, so the
// intensity also flows between neighbouring directions of the geodesic grid
// through the Voronoi edges.  For direction s at a cell,
//   D_s = (1/w_s) sum_(edges e of s) +-F_e,   F_e = vP_e I_first + vN_e I_second,
// with vP, vN the edge coefficients dlambda n_0(m_e) v_e split by the sign of
// the edge velocity v_e (the upwind direction carries the flux) and the sign
// + for the edge's first direction.  The update uses D_s / (n^0 n_0), zero
// where |n_0| is below the cut; that factor is applied here, so the stage
// kernel adds h D' to the spatial update.
//
// One workgroup owns a run of up to `cw` cells along phi at one (r, theta)
// position and holds all their directions in LDS; the geometry of the run is
// shared (it does not depend on phi), so the edge coefficients are read once
// per workgroup.
#include <hip/hip_runtime.h>

#include "ctx.hpp"
#include "stage.hpp"

namespace rt {
namespace {

template <typename S>
__global__ void __launch_bounds__(256)
k_angular(long long nc, int n3, int ns, int cw, const S* __restrict__ I, S* __restrict__ D,
          const S* __restrict__ ve, int ne, const S* __restrict__ recp, long long nrt,
          const S* __restrict__ dV, const int* __restrict__ inc, const double* __restrict__ w) {
  extern __shared__ unsigned char smem_raw[];
  S* col = reinterpret_cast<S*>(smem_raw);  // [ns][cw]
  const int chunks = (n3 + cw - 1) / cw;
  const long long row = blockIdx.x / chunks;  // (i1, i2) position
  const int x0 = (int)(blockIdx.x % chunks) * cw;
  const long long cbase = row * n3 + x0;
  const int t = threadIdx.x;
  const int ncol = min(cw, n3 - x0);
  for (int k = t; k < ns * cw; k += 256) {
    const int s = k / cw, l = k % cw;
    col[k] = l < ncol ? I[(long long)s * nc + cbase + l] : S(0);
  }
  __syncthreads();
  const int l = t % cw, grp = t / cw, ngrp = 256 / cw;
  if (l >= ncol) return;  // no barrier follows
  const S* v = ve + row * ne * 2;
  const int* off = inc;
  const int* ent = inc + ns + 1;
  const S dv = dV[row];
  for (int s = grp; s < ns; s += ngrp) {
    const S Is = col[s * cw + l];
    S acc = S(0);
    for (int k = off[s]; k < off[s + 1]; ++k) {
      const int e = ent[3 * k], o = ent[3 * k + 1], side = ent[3 * k + 2];
      const S vP = v[2 * e], vN = v[2 * e + 1];
      const S It = col[o * cw + l];
      acc += side > 0 ? vP * Is + vN * It : -(vN * Is + vP * It);
    }
    const S x = recp[((long long)s * nrt + row) * 4 + 3];
    D[(long long)s * nc + cbase + l] = acc * (x * dv / (S)w[s]);
  }
}

}  // namespace

hipError_t launch_angular(rt_ctx* c, const void* I, hipStream_t st) {
  const long long nrt = (long long)c->n[0] * c->n[1];
  const int cw = c->ks_cw;
  const long long blocks = nrt * ((c->n[2] + cw - 1) / cw);
  const size_t lds = (size_t)c->ns * cw * c->elem;
  if (c->fp32)
    hipLaunchKernelGGL(k_angular<float>, dim3((unsigned)blocks), dim3(256), lds, st, c->nc, c->n[2],
                       c->ns, cw, (const float*)I, (float*)c->d_angD, (const float*)c->d_ve, c->ks_ne,
                       (const float*)c->d_rec_p, nrt, (const float*)c->d_dV, c->d_inc, c->d_w);
  else
    hipLaunchKernelGGL(k_angular<double>, dim3((unsigned)blocks), dim3(256), lds, st, c->nc, c->n[2],
                       c->ns, cw, (const double*)I, (double*)c->d_angD, (const double*)c->d_ve,
                       c->ks_ne, (const double*)c->d_rec_p, nrt, (const double*)c->d_dV, c->d_inc,
                       c->d_w);
  return hipGetLastError();
}

}  // namespace rt
