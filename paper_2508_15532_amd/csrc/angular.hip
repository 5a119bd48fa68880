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
// One workgroup owns a run of up to CW cells along phi at one (r, theta)
// position and holds all their directions in LDS; the geometry of the run is
// shared (it does not depend on phi), so the coefficients are read once per
// workgroup.
#include <hip/hip_runtime.h>

#include "ctx.hpp"
#include "stage.hpp"

namespace rt {
namespace {

// D'_s(c) = A_s I_s(c) + sum_k A_(ns+k) I_(o_k)(c) for the incidences k of s,
// with the per-(r, theta) coefficients A (scaled to the update on the host).
// CW cells along phi per workgroup; with CW = 64 a wave owns one direction
// at a time, so the coefficient and incidence reads are wave-uniform.
template <typename S, int CW>
__global__ void __launch_bounds__(256)
k_angular(long long nc, int n3, int ns, int ninc, const S* __restrict__ I, S* __restrict__ D,
          const S* __restrict__ coef, const int* __restrict__ inc) {
  extern __shared__ unsigned char smem_raw[];
  S* col = reinterpret_cast<S*>(smem_raw);  // [ns][CW]
  const int chunks = (n3 + CW - 1) / CW;
  const long long row = blockIdx.x / chunks;  // (i1, i2) position
  const int x0 = (int)(blockIdx.x % chunks) * CW;
  const long long cbase = row * n3 + x0;
  const int t = threadIdx.x;
  const int ncol = min(CW, n3 - x0);
  // batches of 16 independent loads per thread keep enough reads in flight
  constexpr int B = 16;
  const int total = ns * CW;
  for (int k0 = t; k0 < total; k0 += B * 256) {
    S v[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      // clamped indices keep every load in bounds, so none needs a branch
      const int k = min(k0 + u * 256, total - 1);
      const int s = k / CW, l = k % CW;
      const S x = I[(long long)s * nc + cbase + min(l, ncol - 1)];
      v[u] = l < ncol ? x : S(0);
    }
#pragma unroll
    for (int u = 0; u < B; ++u)
      if (k0 + u * 256 < total) col[k0 + u * 256] = v[u];
  }
  __syncthreads();
  const int l = t % CW;
  constexpr int NGRP = 256 / CW;
  int grp = t / CW;
  if (CW == 64) grp = __builtin_amdgcn_readfirstlane(grp);
  const S* A = coef + row * (long long)(ns + ninc);
  const int* off = inc;
  const int* other = inc + ns + 1;
  for (int s = grp; s < ns; s += NGRP) {
    S acc = A[s] * col[s * CW + l];
    const int k1 = off[s + 1];
    for (int k = off[s]; k < k1; ++k) acc += A[ns + k] * col[other[k] * CW + l];
    if (l < ncol) D[(long long)s * nc + cbase + l] = acc;
  }
}

template <typename S>
hipError_t launch_cw(rt_ctx* c, const void* I, hipStream_t st) {
  const long long nrt = (long long)c->n[0] * c->n[1];
  const int cw = c->ks_cw;
  const dim3 grid((unsigned)(nrt * ((c->n[2] + cw - 1) / cw))), block(256);
  const size_t lds = (size_t)c->ns * cw * sizeof(S);
  const S* in = (const S*)I;
  S* out = (S*)c->d_angD;
  const S* A = (const S*)c->d_acoef;
  switch (cw) {
    case 64: hipLaunchKernelGGL((k_angular<S, 64>), grid, block, lds, st, c->nc, c->n[2], c->ns, c->ks_ninc, in, out, A, c->d_inc); break;
    case 32: hipLaunchKernelGGL((k_angular<S, 32>), grid, block, lds, st, c->nc, c->n[2], c->ns, c->ks_ninc, in, out, A, c->d_inc); break;
    case 16: hipLaunchKernelGGL((k_angular<S, 16>), grid, block, lds, st, c->nc, c->n[2], c->ns, c->ks_ninc, in, out, A, c->d_inc); break;
    case 8: hipLaunchKernelGGL((k_angular<S, 8>), grid, block, lds, st, c->nc, c->n[2], c->ns, c->ks_ninc, in, out, A, c->d_inc); break;
    case 4: hipLaunchKernelGGL((k_angular<S, 4>), grid, block, lds, st, c->nc, c->n[2], c->ns, c->ks_ninc, in, out, A, c->d_inc); break;
    case 2: hipLaunchKernelGGL((k_angular<S, 2>), grid, block, lds, st, c->nc, c->n[2], c->ns, c->ks_ninc, in, out, A, c->d_inc); break;
    default: hipLaunchKernelGGL((k_angular<S, 1>), grid, block, lds, st, c->nc, c->n[2], c->ns, c->ks_ninc, in, out, A, c->d_inc); break;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_angular(rt_ctx* c, const void* I, hipStream_t st) {
  return c->fp32 ? launch_cw<float>(c, I, st) : launch_cw<double>(c, I, st);
}

}  // namespace rt
