// Angular flux divergence of the curved geometry (Sec. 3.5, geodesic-edge
// fluxes; donor-cell states, or MAPR states in the two kernels at the end).
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
hipError_t launch_cw(rt_ctx* c, const void* I, void* angD, hipStream_t st) {
  const long long nrt = (long long)c->n[0] * c->n[1];
  const int cw = c->ks_cw;
  const dim3 grid((unsigned)(nrt * ((c->n[2] + cw - 1) / cw))), block(256);
  const S* in = (const S*)I;
  S* out = (S*)angD;
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

// MAPR edge states (Sec. 3.4; used by the angular fluxes of Sec. 3.5).  Pass 1: per direction s and cell, the slope of
// the flattest plane through (0, I_s) and a consecutive pair (a, b) of the
// neighbours in the gnomonic coordinates of s:
//   g = Minv_(s,ab) (I_a - I_s, I_b - I_s).
// Planes of equal slope are frequent (symmetric neighbourhoods with equal or
// zeroed intensities), so rounding must not choose among them: every plane with
// |g|^2 within the relative band tie_band<S>() of the smallest counts as
// minimal and the first of them in the cyclic order is taken.  One thread per
// cell and one direction per workgroup (uniform, scalar table loads); see
// mapr_block for the order of the workgroups.
template <typename S>
__device__ constexpr S tie_band() { return sizeof(S) == 8 ? S(1e-8) : S(1e-4); }

// Workgroup -> (256-cell chunk, direction).  Consecutive workgroups go to the
// eight XCDs in turn, so workgroup b runs on XCD b % 8; each XCD takes whole
// chunks (chunk = 8 k + xcd) and runs all directions of a chunk back to back,
// so the neighbour rows of the chunk (ns x 256 cells) are reused from that
// XCD's L2.  The grid has ceil(chunks / 8) * 8 * ns workgroups; those past the
// last chunk exit.
__device__ inline long long mapr_block(int ns, int& s) {
  const unsigned b = blockIdx.x, local = b >> 3;
  s = (int)(local % (unsigned)ns);
  return (long long)(local / (unsigned)ns) * 8 + (b & 7u);
}

template <typename S>
__global__ void __launch_bounds__(256)
k_mapr_slope(long long nc, int ns, const S* __restrict__ I, S* __restrict__ G,
             const int* __restrict__ ring, const S* __restrict__ minv) {
  int s;
  const long long c = mapr_block(ns, s) * 256 + threadIdx.x;
  if (c >= nc) return;
  const S Is = I[(long long)s * nc + c];
  const int* r = ring + s * KS_ROW;  // [0] neighbour count, [1..6] cyclic order
  const bool pentagon = r[0] == 5;   // uniform: its sixth pair is degenerate
  const S* m = minv + s * KS_DEG * 4;
  S d[KS_DEG];
#pragma unroll
  for (int j = 0; j < KS_DEG; ++j) d[j] = I[(long long)r[1 + j] * nc + c] - Is;
  S h0[KS_DEG], h1[KS_DEG], nn[KS_DEG];
  S lo = 0;
#pragma unroll
  for (int i = 0; i < KS_DEG; ++i) {
    const S dA = d[i], dB = d[(i + 1) % KS_DEG];
    h0[i] = m[4 * i] * dA + m[4 * i + 1] * dB;
    h1[i] = m[4 * i + 2] * dA + m[4 * i + 3] * dB;
    nn[i] = h0[i] * h0[i] + h1[i] * h1[i];
    if (i == KS_DEG - 1 && pentagon) continue;
    lo = i == 0 ? nn[i] : (nn[i] < lo ? nn[i] : lo);
  }
  const S thr = lo * (S(1) + tie_band<S>());
  S g0 = h0[0], g1 = h1[0];
#pragma unroll
  for (int i = KS_DEG - 1; i >= 0; --i)
    if (nn[i] <= thr && !(i == KS_DEG - 1 && pentagon)) {
      g0 = h0[i];
      g1 = h1[i];
    }
  G[2LL * s * nc + c] = g0;
  G[(2LL * s + 1) * nc + c] = g1;
}

// Pass 2: D'_s = sum_j a_sj R_j over the neighbour slots j of s, with R_j the
// state at the edge midpoint of the slot's upwind side: I_u + g_u . p_u(m),
// I_u where that is negative (u = s or its neighbour, by the slot's flag).
// WROW: n3 is a multiple of 64, so a wave's 64 cells share one (i1, i2)
// position and its coefficient row and flags are loaded once per wave.
template <typename S, bool WROW>
__global__ void __launch_bounds__(256)
k_mapr_flux(long long nc, int n3, int ns, const S* __restrict__ I, const S* __restrict__ G,
            S* __restrict__ D, const int* __restrict__ nbr, const S* __restrict__ pq,
            const S* __restrict__ coef, const unsigned char* __restrict__ self) {
  int s;
  const long long c = mapr_block(ns, s) * 256 + threadIdx.x;
  if (c >= nc) return;
  long long q = c / n3;  // (i1, i2) position
  if (WROW) q = __builtin_amdgcn_readfirstlane((int)q);
  const S* a = coef + (q * ns + s) * KS_ROW;
  const unsigned f = self[q * ns + s];
  const int* o = nbr + s * KS_ROW;
  const S* w = pq + s * KS_ROW * 4;
  const S Is = I[(long long)s * nc + c];
  const S gs0 = G[2LL * s * nc + c], gs1 = G[(2LL * s + 1) * nc + c];
  // the upwind neighbours' intensities and slopes: every load is issued before
  // the first is used (the slot flags only decide which loads are needed); the
  // neighbour numbers are read first, all at once, rather than one per slot
  // behind each slot's flag
  int on[KS_DEG];
#pragma unroll
  for (int j = 1; j <= KS_DEG; ++j) on[j - 1] = o[j];
  S Iu[KS_DEG], Gu0[KS_DEG], Gu1[KS_DEG];
#pragma unroll
  for (int j = 1; j <= KS_DEG; ++j) {
    Iu[j - 1] = Gu0[j - 1] = Gu1[j - 1] = S(0);
    if (!((f >> j) & 1u)) {
      const long long u = on[j - 1];
      Iu[j - 1] = I[u * nc + c];
      Gu0[j - 1] = G[2 * u * nc + c];
      Gu1[j - 1] = G[(2 * u + 1) * nc + c];
    }
  }
  S acc = 0;
#pragma unroll
  for (int j = 1; j <= KS_DEG; ++j) {
    S r;
    if ((f >> j) & 1u) {
      r = Is + gs0 * w[4 * j] + gs1 * w[4 * j + 1];
      if (r < S(0)) r = Is;
    } else {
      r = Iu[j - 1] + Gu0[j - 1] * w[4 * j + 2] + Gu1[j - 1] * w[4 * j + 3];
      if (r < S(0)) r = Iu[j - 1];
    }
    acc += a[j] * r;
  }
  D[(long long)s * nc + c] = acc;
}

template <typename S>
hipError_t launch_mapr(rt_ctx* c, const void* I, void* angD, void* grad, hipStream_t st) {
  const long long chunks8 = ((c->nc + 255) / 256 + 7) / 8 * 8;
  const long long nblk = chunks8 * c->ns;
  if (nblk > 0xffffffffLL) return hipErrorInvalidConfiguration;
  const dim3 grid((unsigned)nblk), block(256);
  const S* in = (const S*)I;
  S* G = (S*)grad;
  hipLaunchKernelGGL((k_mapr_slope<S>), grid, block, 0, st, c->nc, c->ns, in, G, c->d_mp_ring,
                     (const S*)c->d_mp_minv);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (c->n[2] % 64 == 0)
    hipLaunchKernelGGL((k_mapr_flux<S, true>), grid, block, 0, st, c->nc, c->n[2], c->ns, in,
                       (const S*)G, (S*)angD, c->d_inc, (const S*)c->d_mp_pq,
                       (const S*)c->d_mp_coef, c->d_mp_self);
  else
    hipLaunchKernelGGL((k_mapr_flux<S, false>), grid, block, 0, st, c->nc, c->n[2], c->ns, in,
                       (const S*)G, (S*)angD, c->d_inc, (const S*)c->d_mp_pq,
                       (const S*)c->d_mp_coef, c->d_mp_self);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_angular(rt_ctx* c, const void* I, void* angD, void* grad, hipStream_t st) {
  if (c->mapr)
    return c->fp32 ? launch_mapr<float>(c, I, angD, grad, st) : launch_mapr<double>(c, I, angD, grad, st);
  return c->fp32 ? launch_cw<float>(c, I, angD, st) : launch_cw<double>(c, I, angD, st);
}

}  // namespace rt
