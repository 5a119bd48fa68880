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
// workgroup.  The neighbour lists of the geodesic grid are padded to KS_DEG
// entries (zero weights), so the sum over a direction's neighbours is a fixed,
// fully unrolled one.
#include <hip/hip_runtime.h>

#include "ctx.hpp"
#include "stage.hpp"

namespace rt {
namespace {

// D'_s(c) = A_s0 I_s(c) + sum_j A_sj I_(o_sj)(c) over the KS_DEG padded
// neighbours o_sj of s, with the per-(r, theta) coefficients A (scaled to the
// update on the host).  CW cells along phi per workgroup, 256 / CW groups of
// CW threads; a thread keeps one cell (t % CW) throughout and its group takes
// every (256 / CW)-th direction, so a load's address advances by a uniform
// stride and the LDS slots by immediate offsets.
template <typename S, int CW>
__global__ void __launch_bounds__(256)
k_angular(long long nc, int n3, int ns, const S* __restrict__ I, S* __restrict__ D,
          const S* __restrict__ coef, const int* __restrict__ nbr) {
  constexpr int NGRP = 256 / CW;
  extern __shared__ unsigned char smem_raw[];
  // LDS: the run's intensities [ns][CW], its coefficient rows [ns][KS_ROW]
  // and the neighbour lists [ns][KS_ROW] as byte offsets of the neighbours'
  // rows in the intensity block (16 bits: ns CW elem < 64 KiB)
  S* col = reinterpret_cast<S*>(smem_raw);
  S* lco = col + ns * CW;
  unsigned short* lnb = reinterpret_cast<unsigned short*>(lco + ns * KS_ROW);
  const int chunks = (n3 + CW - 1) / CW;
  const long long row = blockIdx.x / chunks;  // (i1, i2) position
  const int x0 = (int)(blockIdx.x % chunks) * CW;
  const long long cbase = row * n3 + x0;
  const int t = threadIdx.x;
  const int ncol = min(CW, n3 - x0);
  const int l = t % CW;
  int grp = t / CW;
  if (CW == 64) grp = __builtin_amdgcn_readfirstlane(grp);
  const bool inrun = l < ncol;
  // the coefficient rows and neighbour lists go to LDS first; their reads
  // overlap those of the intensities
  const S* A = coef + row * (long long)ns * KS_ROW;
  for (int k = t; k < ns * KS_ROW; k += 256) {
    lco[k] = A[k];
    lnb[k] = (unsigned short)(nbr[k] * CW * (int)sizeof(S));
  }
  // this thread's cell in every direction of its group (cells past the run
  // re-read the run's last cell and stage zeros)
  const S* src = I + (long long)grp * nc + cbase + min(l, ncol - 1);
  const long long stride = (long long)NGRP * nc;
  const int nper = (ns - grp + NGRP - 1) / NGRP;  // directions of this group
  // batches of B loads per thread: the run is in flight at once
  constexpr int B = CW >= 64 ? 48 : 24;
  for (int u0 = 0; u0 < nper; u0 += B) {
    S v[B];
#pragma unroll
    for (int u = 0; u < B; ++u) v[u] = src[min(u0 + u, nper - 1) * stride];
#pragma unroll
    for (int u = 0; u < B; ++u)
      if (u0 + u < nper) col[(grp + (u0 + u) * NGRP) * CW + l] = inrun ? v[u] : S(0);
  }
  __syncthreads();
  static_assert(KS_DEG + 1 <= KS_ROW, "row layout");
  const char* lane = reinterpret_cast<const char*>(col + l);
  S* dst = D + (long long)grp * nc + cbase + l;
#pragma unroll 2
  for (int s = grp; s < ns; s += NGRP) {
    const S* a = lco + s * KS_ROW;
    const unsigned short* o = lnb + s * KS_ROW;
    S acc = a[0] * col[s * CW + l];
#pragma unroll
    for (int j = 1; j <= KS_DEG; ++j) acc += a[j] * *reinterpret_cast<const S*>(lane + o[j]);
    if (inrun) *dst = acc;
    dst += stride;
  }
}

// The same divergence for many directions (all of a cell's directions no
// longer fit LDS beside a useful run): workgroup (patch p, position, run of CW
// cells) stages the rows of its load list -- the patch's own directions, then
// the neighbours outside it -- and forms D' for the patch's own directions.
// lnb holds, per direction, the positions of its row set (itself, then its
// padded neighbours) in its patch's list.  With CW elem = 256 bytes the rows
// move in 256-byte pieces.
template <typename S, int CW>
__global__ void __launch_bounds__(256)
k_angular_patch(long long nc, int n3, int ns, long long nruns, const S* __restrict__ I,
                S* __restrict__ D, const S* __restrict__ coef, const int* __restrict__ plist,
                const int* __restrict__ poff, const int* __restrict__ pnout,
                const int* __restrict__ lnb) {
  constexpr int NGRP = 256 / CW;
  // LDS: the rows of the load list; for the patch's own directions their
  // direction number, coefficient row and local row-set positions (so that
  // the sum below reads LDS only)
  __shared__ S col[KS_PATCH_LOADS][CW];
  __shared__ S lco[KS_PATCH_LOADS][KS_ROW];
  __shared__ unsigned short lnl[KS_PATCH_LOADS][KS_ROW];
  __shared__ int ldir[KS_PATCH_LOADS];
  // the patch is the slowest index: consecutive workgroups read the same rows
  // at neighbouring cells
  const int p = (int)(blockIdx.x / nruns);
  const long long run = blockIdx.x % nruns;
  const int chunks = (n3 + CW - 1) / CW;
  const long long row = run / chunks;  // (i1, i2) position
  const int x0 = (int)(run % chunks) * CW;
  const long long cbase = row * n3 + x0;
  const int t = threadIdx.x;
  const int ncol = min(CW, n3 - x0);
  const int l = t % CW;
  int grp = t / CW;
  if (CW == 64) grp = __builtin_amdgcn_readfirstlane(grp);
  const bool inrun = l < ncol;
  const int* list = plist + poff[p];
  const int nl = poff[p + 1] - poff[p], nout = pnout[p];
  const S* A = coef + row * (long long)ns * KS_ROW;
  for (int k = t; k < nout * KS_ROW; k += 256) {
    const int li = k / KS_ROW, j = k % KS_ROW;
    const int s = list[li];
    lco[li][j] = A[s * KS_ROW + j];
    lnl[li][j] = (unsigned short)lnb[s * KS_ROW + j];
    if (j == 0) ldir[li] = s;
  }
  const long long cell = cbase + min(l, ncol - 1);
  constexpr int B = 16;
  for (int u0 = grp; u0 < nl; u0 += B * NGRP) {
    S v[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int li = min(u0 + u * NGRP, nl - 1);
      v[u] = I[(long long)list[li] * nc + cell];
    }
#pragma unroll
    for (int u = 0; u < B; ++u)
      if (u0 + u * NGRP < nl) col[u0 + u * NGRP][l] = inrun ? v[u] : S(0);
  }
  __syncthreads();
#pragma unroll 2
  for (int li = grp; li < nout; li += NGRP) {
    const S* a = lco[li];
    const unsigned short* o = lnl[li];
    S acc = a[0] * col[li][l];
#pragma unroll
    for (int j = 1; j <= KS_DEG; ++j) acc += a[j] * col[o[j]][l];
    if (inrun) D[(long long)ldir[li] * nc + cbase + l] = acc;
  }
}

template <typename S>
hipError_t launch_cw(rt_ctx* c, const void* I, hipStream_t st) {
  const long long nrt = (long long)c->n[0] * c->n[1];
  const int cw = c->ks_cw;
  const dim3 grid((unsigned)(nrt * ((c->n[2] + cw - 1) / cw))), block(256);
  const S* in = (const S*)I;
  S* out = (S*)c->d_angD;
  const S* A = (const S*)c->d_acoef;
  if (!c->ks_lco) {
    constexpr int PCW = 256 / (int)sizeof(S);  // 256-byte rows
    const long long nruns = nrt * ((c->n[2] + PCW - 1) / PCW);
    const dim3 pgrid((unsigned)(nruns * c->ks_npatch));
    hipLaunchKernelGGL((k_angular_patch<S, PCW>), pgrid, block, 0, st, c->nc, c->n[2], c->ns, nruns,
                       in, out, A, c->d_plist, c->d_poff, c->d_pnout, c->d_plnb);
    return hipGetLastError();
  }
  const size_t lds = angular_lds_bytes(c->ns, cw, sizeof(S), true);
#define RT_ANG(CW) \
  hipLaunchKernelGGL((k_angular<S, CW>), grid, block, lds, st, c->nc, c->n[2], c->ns, in, out, A, c->d_inc)
  switch (cw) {
    case 64: RT_ANG(64); break;
    case 32: RT_ANG(32); break;
    case 16: RT_ANG(16); break;
    case 8: RT_ANG(8); break;
    case 4: RT_ANG(4); break;
    case 2: RT_ANG(2); break;
    default: RT_ANG(1); break;
  }
#undef RT_ANG
  return hipGetLastError();
}

}  // namespace

hipError_t launch_angular(rt_ctx* c, const void* I, hipStream_t st) {
  return c->fp32 ? launch_cw<float>(c, I, st) : launch_cw<double>(c, I, st);
}

}  // namespace rt
