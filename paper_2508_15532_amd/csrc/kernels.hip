// HIP kernels (gfx950) outside the fused stage: fluid-velocity setup, the
// FP64 MFMA moment contraction and the non-finite check.
//
// Data layout: intensities direction-major I[s*nc + c], c = (i1*n2 + i2)*n3 + i3,
// so a wavefront's 64 lanes read 64 consecutive cells of one direction.
// Template parameter S is the intensity storage type (float in the FP32
// transport form, double otherwise); the moments always accumulate in double.
#include <hip/hip_runtime.h>

#include <cmath>

#include "ctx.hpp"

namespace rt {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// moments R[k][c] = sum_s I[s][c] W[s][k] (Eq. R) on the FP64 matrix cores:
// v_mfma_f64_16x16x4_f64 computes D(16x16) += A(16x4) B(4x16) with
//   A[i][k] = I[s0 + k][cell0 + i]  (lane l: i = l % 16, k = l / 16),
//   B[k][j] = W[s0 + k][j]          (lane l: k = l / 16, j = l % 16),
//   D[i][j] in lane l = j + 16 * (i % 4), element i / 4 (measured on gfx950).
// Each wavefront owns 64 consecutive cells (four 16-cell tiles).
// ---------------------------------------------------------------------------
typedef double d4 __attribute__((ext_vector_type(4)));

// FP32 intensities, nc a multiple of 4, whole waves of cells only: lane (r, kq)
// loads the four consecutive cells cell0 + 4r .. 4r + 3 of direction s0 + kq in
// one 16-byte load, component m being row r of tile m (tile m's row i is cell
// cell0 + 4i + m).  Batches of B four-direction steps; the loads of the next
// batch are issued before the products of the current one, so every wave keeps
// 2 B loads in flight while its matrix products run.  A kernel of its own so
// that its register budget (and occupancy) is not set by the general path.
template <int B>
__global__ void __launch_bounds__(kBlock)
k_moments_f32(long long nc, int ns, const float* __restrict__ I, const double* __restrict__ W16,
              double* __restrict__ R, double* __restrict__ J) {
  const int lane = threadIdx.x & 63;
  const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const long long cell0 = wave * 64;
  if (cell0 + 64 > nc) return;
  const int r = lane & 15, kq = lane >> 4;
  d4 acc[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) acc[m] = d4{0.0, 0.0, 0.0, 0.0};
  const float* base = I + cell0 + 4 * r;
  auto load = [&](int s00, float4* av, double* b) {
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int s = s00 + 4 * u + kq;
      b[u] = s < ns ? W16[s * 16 + r] : 0.0;
      av[u] = s < ns ? *reinterpret_cast<const float4*>(base + (long long)s * nc) : float4{0.f, 0.f, 0.f, 0.f};
    }
  };
  float4 av[B], an[B];
  double b[B], bn[B];
  load(0, av, b);
  for (int s00 = 0; s00 < ns; s00 += 4 * B) {
    const bool more = s00 + 4 * B < ns;
    if (more) load(s00 + 4 * B, an, bn);
#pragma unroll
    for (int u = 0; u < B; ++u) {
      acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)av[u].x, b[u], acc[0], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)av[u].y, b[u], acc[1], 0, 0, 0);
      acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)av[u].z, b[u], acc[2], 0, 0, 0);
      acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)av[u].w, b[u], acc[3], 0, 0, 0);
    }
    if (more) {
#pragma unroll
      for (int u = 0; u < B; ++u) {
        av[u] = an[u];
        b[u] = bn[u];
      }
    }
  }
  // D[i][j] of tile m sits in lane j + 16 (i % 4), element i / 4: lane (r, kq)
  // holds component r of cells cell0 + 4 (4e + kq) + m, m = 0..3 contiguous
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const long long cc = cell0 + 16 * e + 4 * kq;
    if (r < 10) {
      double* o = R + (long long)r * nc + cc;
      *reinterpret_cast<d4*>(o) = d4{acc[0][e], acc[1][e], acc[2][e], acc[3][e]};
    }
    if (J && r == 0) {
      const double q = 1.0 / (4.0 * kPi);
      *reinterpret_cast<d4*>(J + cc) = d4{acc[0][e] * q, acc[1][e] * q, acc[2][e] * q, acc[3][e] * q};
    }
  }
}

// General path: FP64 intensities, and FP32 ones where k_moments_f32 does not
// apply; waves start at cell first + 64 w.
template <typename S>
__global__ void __launch_bounds__(kBlock)
k_moments(long long nc, int ns, const S* __restrict__ I, const double* __restrict__ W16,
          double* __restrict__ R, double* __restrict__ J, long long first) {
  const int lane = threadIdx.x & 63;
  const long long wave = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const long long cell0 = first + wave * 64;
  if (cell0 >= nc) return;
  const int r = lane & 15, kq = lane >> 4;
  d4 acc[4];
  for (int m = 0; m < 4; ++m) acc[m] = d4{0.0, 0.0, 0.0, 0.0};
  if constexpr (sizeof(S) == 4) {
    for (int s0 = 0; s0 < ns; s0 += 4) {
      const int s = s0 + kq;
      const double b = W16[s * 16 + r];  // W16 is zero-padded to a multiple of 4 rows
      for (int m = 0; m < 4; ++m) {
        long long cc = cell0 + 16 * m + r;
        double av = (s < ns && cc < nc) ? (double)I[(long long)s * nc + cc] : 0.0;
        acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b, acc[m], 0, 0, 0);
      }
    }
  } else {
    // FP64 intensities: batches of B four-direction steps, all loads of a batch
    // issued before its matrix products (4 B loads per lane in flight); with
    // FP32 ones the plain loop, with more resident waves, is faster (measured)
    constexpr int B = 4;
    for (int s00 = 0; s00 < ns; s00 += 4 * B) {
      double av[B][4], b[B];
#pragma unroll
      for (int u = 0; u < B; ++u) {
        const int s = s00 + 4 * u + kq;
        b[u] = s < ns ? W16[s * 16 + r] : 0.0;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const long long cc = cell0 + 16 * m + r;
          av[u][m] = (s < ns && cc < nc) ? (double)I[(long long)s * nc + cc] : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < B; ++u)
#pragma unroll
        for (int m = 0; m < 4; ++m)
          acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][m], b[u], acc[m], 0, 0, 0);
    }
  }
  for (int m = 0; m < 4; ++m) {
    for (int e = 0; e < 4; ++e) {
      long long cc = cell0 + 16 * m + 4 * e + kq;
      if (cc < nc && r < 10) R[(long long)r * nc + cc] = acc[m][e];
      if (J && cc < nc && r == 0) J[cc] = acc[m][e] / (4.0 * kPi);
    }
  }
}

template <typename S>
__global__ void k_nonfinite(long long n, const S* __restrict__ I, long long nT,
                            const double* __restrict__ T, unsigned long long* __restrict__ count) {
  long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  unsigned long long bad = 0;
  for (long long i = k; i < n; i += stride) bad += !isfinite((double)I[i]);
  for (long long i = k; i < nT; i += stride) bad += !isfinite(T[i]);
  if (bad) atomicAdd(count, bad);
}

// tetrad-frame fluid velocity (identity tetrad) and coordinate 3-velocity
// Tetrad-frame fluid 4-velocity u-hat^a = e^a_mu u^mu and coordinate
// 3-velocity v^i = u^i / u^0 per cell.  Flat: identity tetrad.  Curved: einv
// holds e^a_mu per (r, theta) position (index c / n3); a NULL u means the
// normal observer, u-hat = (1, 0, 0, 0), u^mu = e^mu_0 (etet per position).
__global__ void k_fluid(long long nc, int n3, const double* __restrict__ u,
                        const double* __restrict__ einv, const double* __restrict__ etet,
                        double* __restrict__ uhat, double* __restrict__ v) {
  long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  double u4[4] = {1.0, 0.0, 0.0, 0.0};
  if (einv && !u) {
    const double* e = etet + (c / n3) * 16;
    for (int k = 0; k < 4; ++k) u4[k] = e[k * 4 + 0];
  } else if (u) {
    for (int k = 0; k < 4; ++k) u4[k] = u[k * nc + c];
  }
  for (int a = 0; a < 4; ++a) {
    double x = u4[a];
    if (einv) {
      const double* L = einv + (c / n3) * 16 + a * 4;
      x = (u ? L[0] * u4[0] + L[1] * u4[1] + L[2] * u4[2] + L[3] * u4[3] : (a == 0 ? 1.0 : 0.0));
    }
    uhat[a * nc + c] = x;
  }
  for (int k = 0; k < 3; ++k) v[k * nc + c] = u4[k + 1] / u4[0];
}

// R^(mu nu) = e^mu_a e^nu_b R^(ab) in place, symmetric storage of 10 components
__global__ void k_to_coord(long long nc, int n3, const double* __restrict__ etet, double* __restrict__ R) {
  long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const int pa[10] = {0, 0, 0, 0, 1, 1, 1, 2, 2, 3};
  const int pb[10] = {0, 1, 2, 3, 1, 2, 3, 2, 3, 3};
  double full[4][4];
  for (int k = 0; k < 10; ++k) full[pa[k]][pb[k]] = full[pb[k]][pa[k]] = R[k * nc + c];
  const double* e = etet + (c / n3) * 16;  // e[mu*4 + a]
  double t[4][4];
  for (int m = 0; m < 4; ++m)
    for (int b = 0; b < 4; ++b) {
      double x = 0.0;
      for (int a = 0; a < 4; ++a) x += e[m * 4 + a] * full[a][b];
      t[m][b] = x;
    }
  for (int k = 0; k < 10; ++k) {
    const int m = pa[k], n = pb[k];
    double x = 0.0;
    for (int b = 0; b < 4; ++b) x += t[m][b] * e[n * 4 + b];
    R[k * nc + c] = x;
  }
}

inline unsigned blocks_for(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_fluid(rt_ctx* c, const double* u, hipStream_t st) {
  hipLaunchKernelGGL(k_fluid, dim3(blocks_for(c->nc)), dim3(kBlock), 0, st, c->nc, c->n[2], u,
                     c->curved ? c->d_einv : nullptr, c->d_e, c->d_uhat, c->d_v);
  return hipGetLastError();
}

hipError_t launch_to_coord(rt_ctx* c, double* R, hipStream_t st) {
  hipLaunchKernelGGL(k_to_coord, dim3(blocks_for(c->nc)), dim3(kBlock), 0, st, c->nc, c->n[2], c->d_e, R);
  return hipGetLastError();
}

hipError_t launch_moments(rt_ctx* c, const void* I, double* R, double* J, hipStream_t st) {
  auto blocks_of = [](long long waves) { return (unsigned)((waves * 64 + kBlock - 1) / kBlock); };
  if (!c->fp32) {
    hipLaunchKernelGGL(k_moments<double>, dim3(blocks_of((c->nc + 63) / 64)), dim3(kBlock), 0, st, c->nc,
                       c->ns, (const double*)I, c->d_W16, R, J, 0ll);
    return hipGetLastError();
  }
  // FP32: whole waves through the 16-byte-load kernel when nc is a multiple of
  // 4 (alignment of the loads), the ragged rest through the general path
  const long long full = (c->nc % 4 == 0) ? c->nc / 64 : 0;
  if (full > 0)
    hipLaunchKernelGGL(k_moments_f32<4>, dim3(blocks_of(full)), dim3(kBlock), 0, st, c->nc, c->ns,
                       (const float*)I, c->d_W16, R, J);
  const long long first = full * 64;
  if (first < c->nc)
    hipLaunchKernelGGL(k_moments<float>, dim3(blocks_of((c->nc - first + 63) / 64)), dim3(kBlock), 0, st,
                       c->nc, c->ns, (const float*)I, c->d_W16, R, J, first);
  return hipGetLastError();
}

hipError_t launch_nonfinite(rt_ctx* c, const void* I, const double* T, hipStream_t st) {
  long long n = (long long)c->ns * c->nc;
  if (c->fp32)
    hipLaunchKernelGGL(k_nonfinite<float>, dim3(1024), dim3(kBlock), 0, st, n, (const float*)I, c->nc,
                       T, c->d_count + 1);
  else
    hipLaunchKernelGGL(k_nonfinite<double>, dim3(1024), dim3(kBlock), 0, st, n, (const double*)I,
                       c->nc, T, c->d_count + 1);
  return hipGetLastError();
}


}  // namespace rt
