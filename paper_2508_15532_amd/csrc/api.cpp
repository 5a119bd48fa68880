// C ABI of the library (declared in include/rt.h): argument checking, context
// and device-memory management, and the order of kernel launches of a step.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "ctx.hpp"
#include "kerr.hpp"
#include "stage.hpp"

namespace rt {
namespace {
thread_local std::string g_err;
}

void set_error(const std::string& msg) { g_err = msg; }

namespace {

rt_status fail(rt_status s, const std::string& msg) {
  set_error(msg);
  return s;
}

rt_status hip_fail(hipError_t e, const char* what) {
  return fail(RT_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define RT_HIP(call)                                        \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return hip_fail(e_, #call);       \
  } while (0)

template <typename T>
rt_status alloc(T** p, size_t bytes) {
  if (*p) return RT_OK;
  hipError_t e = hipMalloc((void**)p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(RT_E_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " +
                                hipGetErrorString(e));
  }
  return RT_OK;
}

template <typename T>
void release(T*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

bool aligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

rt_status use_device(const rt_ctx* c) {
  int cur = -1;
  RT_HIP(hipGetDevice(&cur));
  if (cur != c->device) RT_HIP(hipSetDevice(c->device));
  return RT_OK;
}

hipEvent_t take_event(rt_ctx* c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Enqueue one launch; with timing on, bracket it with events on the same stream.
template <typename F>
hipError_t timed(rt_ctx* c, int kind, hipStream_t st, F&& launch) {
  if (!(c->debug & 2)) return launch();
  hipEvent_t a = take_event(c), b = take_event(c);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, st);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, st);
  if (e != hipSuccess) return e;
  c->timed.push_back({kind, a, b});
  return hipSuccess;
}

}  // namespace
}  // namespace rt

namespace rt {
namespace {
// host FP64 vector -> device array of the transport type
rt_status upload_as(rt_ctx* c, void** dst, const std::vector<double>& v) {
  rt_status st = alloc((char**)dst, v.size() * c->elem);
  if (st) return st;
  if (c->fp32) {
    std::vector<float> f(v.begin(), v.end());
    RT_HIP(hipMemcpy(*dst, f.data(), f.size() * 4, hipMemcpyHostToDevice));
  } else {
    RT_HIP(hipMemcpy(*dst, v.data(), v.size() * 8, hipMemcpyHostToDevice));
  }
  return RT_OK;
}

template <typename T>
rt_status upload(T** dst, const std::vector<T>& v) {
  rt_status st = alloc(dst, v.size() * sizeof(T));
  if (st) return st;
  RT_HIP(hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return RT_OK;
}

// MAPR tables (Sec. 3.4, angular edge states of the Sec. 3.5 fluxes).  Per direction s, with an
// orthonormal basis (e1, e2) of its tangent plane, a point x has the gnomonic
// coordinates of p = x / (x . n_s) - n_s.  The neighbours of s, sorted by the
// angle of their coordinates (counter-clockwise seen from outside, from the
// neighbour with the smallest index), give the consecutive pairs (a, b); the slope of
// the plane through (0, I_s), (p_a, I_a), (p_b, I_b) is
// g = [p_a; p_b]^-1 (I_a - I_s, I_b - I_s), and the kernels keep the inverse.
// Pentagons have five pairs (the sixth is skipped).  Per neighbour slot the
// edge midpoint gets its coordinates for s and for the neighbour.  Per
// (r, theta) and slot, the edge flux enters the update of s with one signed
// coefficient (the donor-cell coefficients of the slot) applied to the state
// of the edge's upwind side, and a flag tells whether that side is s.
rt_status build_mapr(rt_ctx* c, const KsTables& T) {
  const GeodesicGrid& G = c->grid;
  const int ns = c->ns, ne = (int)G.edge.size();
  const size_t nrt = (size_t)c->n[0] * c->n[1];
  std::vector<double> E((size_t)ns * 6);
  for (int s = 0; s < ns; ++s) {
    const double* n = G.dir[s].data();
    // e1 = normalise(a x n) for the coordinate axis a least aligned with n
    int k = 0;
    for (int q = 1; q < 3; ++q)
      if (std::fabs(n[q]) < std::fabs(n[k])) k = q;
    double a[3] = {0, 0, 0};
    a[k] = 1.0;
    double e1[3] = {a[1] * n[2] - a[2] * n[1], a[2] * n[0] - a[0] * n[2], a[0] * n[1] - a[1] * n[0]};
    const double l = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    for (int q = 0; q < 3; ++q) e1[q] /= l;
    const double e2[3] = {n[1] * e1[2] - n[2] * e1[1], n[2] * e1[0] - n[0] * e1[2], n[0] * e1[1] - n[1] * e1[0]};
    for (int q = 0; q < 3; ++q) {
      E[(size_t)s * 6 + q] = e1[q];
      E[(size_t)s * 6 + 3 + q] = e2[q];
    }
  }
  auto coords = [&](int s, const double* x, double out[2]) {
    const double* n = G.dir[s].data();
    const double d = x[0] * n[0] + x[1] * n[1] + x[2] * n[2];
    double p[3];
    for (int q = 0; q < 3; ++q) p[q] = x[q] / d - n[q];
    const double* e = &E[(size_t)s * 6];
    out[0] = p[0] * e[0] + p[1] * e[1] + p[2] * e[2];
    out[1] = p[0] * e[3] + p[1] * e[4] + p[2] * e[5];
  };
  std::vector<int> ring((size_t)ns * KS_ROW);
  std::vector<double> minv((size_t)ns * KS_DEG * 4), pq((size_t)ns * KS_ROW * 4, 0.0);
  for (int s = 0; s < ns; ++s) {
    const int k0 = T.inc_off[s], deg = T.inc_off[s + 1] - k0;
    if (deg < 5) return fail(RT_E_ARG, "rt_set_metric: MAPR needs 5 or 6 neighbours per direction");
    double xy[KS_DEG][2];
    std::vector<std::pair<double, int>> ang;
    for (int j = 0; j < deg; ++j) {
      coords(s, G.dir[T.inc_other[k0 + j]].data(), xy[j]);
      ang.push_back({std::atan2(xy[j][1], xy[j][0]), j});
    }
    std::sort(ang.begin(), ang.end());
    // the cycle starts at the neighbour with the smallest direction index (the
    // kernel breaks ties between planes of equal slope by this order)
    std::rotate(ang.begin(), std::min_element(ang.begin(), ang.end(),
                                              [&](const std::pair<double, int>& x, const std::pair<double, int>& y) {
                                                return T.inc_other[k0 + x.second] < T.inc_other[k0 + y.second];
                                              }),
                ang.end());
    // ring slots: [0] the number of neighbours, [1..6] the neighbours in cyclic
    // order, [7] unused; pair i is slots 1 + i and 1 + (i + 1) mod 6 (a pentagon
    // repeats its first neighbour in slot 6, so its pair 4 closes the cycle;
    // its pair 5 is degenerate and the kernel skips it)
    ring[(size_t)s * KS_ROW] = deg;
    ring[(size_t)s * KS_ROW + KS_ROW - 1] = s;
    for (int i = 0; i < KS_DEG; ++i) {
      const int ja = ang[i % deg].second, jb = ang[(i + 1) % deg].second;
      const double* pa = xy[ja];
      const double* pb = xy[jb];
      const double det = pa[0] * pb[1] - pa[1] * pb[0];
      ring[(size_t)s * KS_ROW + 1 + i] = T.inc_other[k0 + ja];
      double* m = &minv[((size_t)s * KS_DEG + i) * 4];
      m[0] = pb[1] / det;
      m[1] = -pa[1] / det;
      m[2] = -pb[0] / det;
      m[3] = pa[0] / det;
    }
    for (int j = 0; j < deg; ++j) {
      const int k = k0 + j, e = T.inc_edge[k];
      double* w = &pq[((size_t)s * KS_ROW + 1 + j) * 4];
      coords(s, G.emid[e].data(), w);
      coords(T.inc_other[k], G.emid[e].data(), w + 2);
    }
  }
  std::vector<double> coef;
  std::vector<unsigned char> self;
  try {
    coef.assign(nrt * ns * KS_ROW, 0.0);
    self.assign(nrt * ns, 0);
  } catch (const std::bad_alloc&) {
    return fail(RT_E_NOMEM, "rt_set_metric: host allocation failed");
  }
  for (size_t q = 0; q < nrt; ++q)
    for (int s = 0; s < ns; ++s) {
      const double scale = T.fp[((size_t)s * nrt + q) * 4 + 3] * T.dV[q] / G.w[s];
      const int k0 = T.inc_off[s], deg = T.inc_off[s + 1] - k0;
      unsigned char f = 0;
      for (int j = 0; j < deg; ++j) {
        const int k = k0 + j;
        const double vP = T.ve[(q * ne + T.inc_edge[k]) * 2], vN = T.ve[(q * ne + T.inc_edge[k]) * 2 + 1];
        // one of vP (upwind: the edge's first direction), vN (its second) is zero
        const bool first = T.inc_side[k] > 0;
        if (first ? vP != 0.0 : vN != 0.0) f |= (unsigned char)(1u << (1 + j));
        coef[(q * ns + s) * KS_ROW + 1 + j] = (first ? scale : -scale) * (vP + vN);
      }
      self[q * ns + s] = f;
    }
  rt_status st = RT_OK;
  if ((st = upload(&c->d_mp_ring, ring)) || (st = upload_as(c, &c->d_mp_minv, minv)) ||
      (st = upload_as(c, &c->d_mp_pq, pq)) || (st = upload_as(c, &c->d_mp_coef, coef)) ||
      (st = upload(&c->d_mp_self, self)) ||
      (st = alloc((char**)&c->d_mp_grad, (size_t)2 * c->ns * c->nc * c->elem)))
    return st;
  c->mapr = true;
  return RT_OK;
}

rt_status set_kerr_schild(rt_ctx* c, double M, double a, double cfl) {
  KsTables T;
  try {
    T = build_ks_tables(c->grid, c->desc.n, c->desc.xlo, c->desc.xhi, a, M, c->desc.n0_cut, cfl, 1e-3);
  } catch (const std::bad_alloc&) {
    return fail(RT_E_NOMEM, "rt_set_metric: host allocation failed");
  } catch (const std::exception& e) {
    return fail(RT_E_ARG, std::string("rt_set_metric: ") + e.what());
  }
  // angular kernel: runs of up to 32 phi cells with the coefficient rows in LDS
  // as long as the run's LDS stays within 40 KiB (four workgroups per compute
  // unit) and the run keeps at least 16 cells.  With more directions the
  // directions are split into patches (below) and a workgroup stages one
  // patch's directions and their neighbours for a run of 256-byte rows.
  int cw = 32;
  bool lco = true;
  while (cw > 16 && angular_lds_bytes(c->ns, cw, c->elem, true) > 40960) cw /= 2;
  if (angular_lds_bytes(c->ns, cw, c->elem, true) > 40960) {
    lco = false;
    cw = (int)(256 / c->elem);
  }
  // (the LCO kernel keeps 16-bit byte offsets into the run's intensity block)
  if (lco && (size_t)c->ns * cw * c->elem > 65535)
    return fail(RT_E_ARG, "rt_set_metric: too many directions for the curved form");
  c->ks_lco = lco;
  c->ks_cw = cw;
  c->ks_ninc = T.inc_off[c->ns];
  c->ks_zin_stride = T.zin_stride;
  // angular coefficients padded to a fixed width per direction: slot 0 the
  // direction itself, slots 1..KS_DEG its neighbours (zero weight and the
  // direction itself where it has fewer), the rest zero
  const int ns = c->ns;
  const size_t nrt = (size_t)c->n[0] * c->n[1];
  std::vector<int> inc((size_t)ns * KS_ROW, 0);
  std::vector<double> coef8;
  try {
    coef8.assign(nrt * ns * KS_ROW, 0.0);
  } catch (const std::bad_alloc&) {
    return fail(RT_E_NOMEM, "rt_set_metric: host allocation failed");
  }
  for (int s = 0; s < ns; ++s) {
    const int k0 = T.inc_off[s], deg = T.inc_off[s + 1] - k0;
    if (deg > KS_DEG) return fail(RT_E_ARG, "rt_set_metric: a direction has more than 6 neighbours");
    for (int j = 0; j < KS_ROW; ++j) inc[(size_t)s * KS_ROW + j] = s;
    for (int j = 0; j < deg; ++j) inc[(size_t)s * KS_ROW + 1 + j] = T.inc_other[k0 + j];
    for (size_t q = 0; q < nrt; ++q) {
      const double* A = &T.acoef[q * (ns + c->ks_ninc)];
      double* D = &coef8[(q * ns + s) * KS_ROW];
      D[0] = A[s];
      for (int j = 0; j < deg; ++j) D[1 + j] = A[ns + k0 + j];
    }
  }
  // Patches (many directions): grow compact sets of directions over the
  // neighbour graph, breadth first, while the set and its outside neighbours
  // (the halo) fit the workgroup's LDS (KS_PATCH_LOADS rows); a patch's load
  // list is its own directions, then the halo.  Per direction the kernel gets
  // the local positions of itself and its padded neighbours in its patch's list.
  std::vector<int> plist, poff(1, 0), pnout, lnb;
  if (!lco) {
    std::vector<int> owner(ns, -1);
    lnb.assign((size_t)ns * KS_ROW, 0);
    for (int seed = 0; seed < ns; ++seed) {
      if (owner[seed] >= 0) continue;
      const int p = (int)pnout.size();
      std::vector<int> out, halo, queue(1, seed);
      for (size_t qi = 0; qi < queue.size(); ++qi) {
        const int v = queue[qi];
        if (owner[v] >= 0) continue;
        // halo after adding v: without v, with v's neighbours outside the patch
        std::vector<int> h2;
        for (int x : halo)
          if (x != v) h2.push_back(x);
        for (int j = 1; j <= KS_DEG; ++j) {
          const int u = inc[(size_t)v * KS_ROW + j];
          if (u == v || owner[u] == p || std::find(h2.begin(), h2.end(), u) != h2.end()) continue;
          h2.push_back(u);
        }
        if ((int)(out.size() + 1 + h2.size()) > KS_PATCH_LOADS) continue;
        owner[v] = p;
        out.push_back(v);
        halo.swap(h2);
        for (int j = 1; j <= KS_DEG; ++j) {
          const int u = inc[(size_t)v * KS_ROW + j];
          if (owner[u] < 0) queue.push_back(u);
        }
      }
      std::sort(halo.begin(), halo.end());
      const int base = (int)plist.size();
      plist.insert(plist.end(), out.begin(), out.end());
      plist.insert(plist.end(), halo.begin(), halo.end());
      poff.push_back((int)plist.size());
      pnout.push_back((int)out.size());
      for (size_t k = 0; k < out.size(); ++k) {
        const int sd = out[k];
        for (int j = 0; j < KS_ROW; ++j) {
          const int u = inc[(size_t)sd * KS_ROW + j];
          const auto it = std::find(plist.begin() + base, plist.end(), u);
          lnb[(size_t)sd * KS_ROW + j] = (int)(it - (plist.begin() + base));
        }
      }
    }
  }
  c->ks_npatch = (int)pnout.size();
  rt_status st = RT_OK;
  if (!lco && ((st = upload(&c->d_plist, plist)) || (st = upload(&c->d_poff, poff)) ||
               (st = upload(&c->d_pnout, pnout)) || (st = upload(&c->d_plnb, lnb))))
    return st;
  if ((st = upload_as(c, &c->d_rec_r, T.fr)) || (st = upload_as(c, &c->d_rec_t, T.ft)) ||
      (st = upload_as(c, &c->d_rec_p, T.fp)) || (st = upload_as(c, &c->d_acoef, coef8)) ||
      (st = upload(&c->d_zin, T.zin)) ||
      (st = upload(&c->d_nu0, T.nu0)) || (st = upload(&c->d_e, T.e)) ||
      (st = upload(&c->d_einv, T.einv)) || (st = upload(&c->d_inc, inc)) ||
      (st = alloc((char**)&c->d_angD, (size_t)c->ns * c->nc * c->elem)))
    return st;
  if (c->desc.angular_recon == RT_AREC_MAPR && (st = build_mapr(c, T))) return st;
  c->dt_max = T.dt_max;
  c->curved = true;
  return RT_OK;
}
}  // namespace

namespace {
size_t round256(size_t b) { return (b + 255) / 256 * 256; }
}  // namespace

// doubles per cell of one lazy interaction map: (Q, abar, code) with a moving
// fluid, (alpha, beta) at rest, (alpha, beta) per bin with frequency bins
size_t map_words(const rt_ctx* c) { return std::max<size_t>(3, 2 * (size_t)c->ng); }

size_t step_scratch_bytes(const rt_ctx* c) {
  const size_t nc = (size_t)c->nc, ns = (size_t)c->ns, ng = (size_t)std::max(c->ng, 1);
  size_t b = round256(ng * ns * nc * c->elem) + 2 * round256(map_words(c) * nc * 8) + round256(nc * 8);
  if (c->curved) b += round256(ns * nc * c->elem);
  if (c->mapr) b += round256(2 * ns * nc * c->elem);
  if (c->ng) b += round256(ng * nc * 8);
  return b;
}

StepScratch carve_step_scratch(const rt_ctx* c, void* base) {
  const size_t nc = (size_t)c->nc, ns = (size_t)c->ns;
  char* q = (char*)base;
  auto take = [&](size_t bytes) -> void* {
    void* r = q;
    q += round256(bytes);
    return r;
  };
  const size_t ng = (size_t)std::max(c->ng, 1);
  StepScratch w{};
  w.Itil = take(ng * ns * nc * c->elem);
  w.mapA = (double*)take(map_words(c) * nc * 8);
  w.mapB = (double*)take(map_words(c) * nc * 8);
  w.Tstar = (double*)take(nc * 8);
  w.angD = c->curved ? take(ns * nc * c->elem) : nullptr;
  w.mp_grad = c->mapr ? take(2 * ns * nc * c->elem) : nullptr;
  w.Emg = c->ng ? (double*)take(ng * nc * 8) : nullptr;
  return w;
}

namespace {
// The steps of rt_step on a given scratch.  may_alloc = false: nothing is
// allocated (no kernel timing events, no new tile order).
rt_status step_impl(rt_ctx* c, const StepScratch& ws, bool may_alloc, void* I, double* T, double dt,
                    int nsteps, double* G_out, double* R_out, hipStream_t stream) {
  StageArgs a{};
  a.n1 = c->n[0];
  a.n2 = c->n[1];
  a.n3 = c->n[2];
  a.nc = c->nc;
  a.ns = c->ns;
  for (int ax = 0; ax < 3; ++ax) {
    a.bc_lo[ax] = c->desc.bc_lo[ax];
    a.bc_hi[ax] = c->desc.bc_hi[ax];
    a.inv_dx[ax] = 1.0 / c->dx[ax];
  }
  a.dt = dt;
  a.abar = c->desc.abar;
  a.limiter = c->desc.limiter;
  a.model = c->opac.model;
  a.gamma = c->opac.gamma;
  a.C_a = c->opac.C_a;
  a.C_s = c->opac.C_s;
  a.rho_floor = c->desc.rho_floor;
  a.max_iter = c->opac.newton_max_iter;
  a.rtol = c->opac.newton_rtol;
  a.W0 = c->W0;
  for (int k = 0; k < 10; ++k) a.Wsum[k] = c->Wsum[k];
  a.curved = c->curved ? 1 : 0;
  a.zin_stride = c->ks_zin_stride;
  a.pole_rows = c->desc.pole_zero_rows;
  StagePtrs p{};
  p.rho = c->d_rho;
  p.ka = c->d_ka;
  p.ks = c->d_ks;
  p.jv = c->d_j;
  p.uhat = c->d_uhat;
  p.vel = c->d_v;
  p.dirF_v = c->fp32 ? (const void*)c->d_dir_f : (const void*)c->d_dir;
  p.dirD = c->d_dir;
  p.w = c->d_w;
  p.W16 = c->d_W16;
  p.fail = c->d_count;
  if (c->curved) {
    p.rec_r_v = c->d_rec_r;
    p.rec_t_v = c->d_rec_t;
    p.rec_p_v = c->d_rec_p;
    p.zin = c->d_zin;
    p.angD_v = ws.angD;
    p.nu0 = c->d_nu0;
  }
  // kernel timing creates events: only where the call may allocate
  auto run = [&](int kind, auto&& launch) -> hipError_t {
    return may_alloc ? timed(c, kind, stream, launch) : launch();
  };
  // (a failed reconfiguration, e.g. an allocation in rt_set_groups, can leave
  // the context without its step scratch: refuse rather than launch on NULL)
  if (!ws.Itil || !ws.mapA || !ws.mapB || !ws.Tstar || (c->curved && !ws.angD) || (c->mapr && !ws.mp_grad))
    return fail(RT_E_STATE, "rt_step: the step scratch is not allocated");
  if (c->ng && (!ws.Emg || !c->d_ka_g))
    return fail(RT_E_STATE, "rt_step: the frequency-bin scratch is not allocated");
  if (c->ng) {
    // frequency bins (at rest, flat): each stage transports every bin with its
    // own opacity, the stage kernels leaving the per-bin E_- only; one solve
    // per stage couples the bins through the temperature and writes the
    // per-bin lazy maps
    const size_t bin = (size_t)c->ns * c->nc * c->elem;
    const long long nc = c->nc;
    char* Ib = static_cast<char*>(I);
    char* Jb = static_cast<char*>(ws.Itil);
    const double* mapA = nullptr;  // the caller's I is materialised on entry
    for (int k = 0; k < nsteps; ++k) {
      a.h = 0.5 * dt;
      for (int g = 0; g < c->ng; ++g) {
        p.Iflux_v = Ib + g * bin;
        p.mapF = mapA ? mapA + 2 * g * nc : nullptr;
        p.Ibase_v = nullptr;
        p.mapB = nullptr;
        p.Iout_v = Jb + g * bin;
        p.mapO = nullptr;
        p.Tstart = T;
        p.Tcoef = T;
        p.Tout = nullptr;
        p.ka = c->d_ka_g + g * nc;
        p.sumE = ws.Emg + g * nc;
        RT_HIP(run(RT_K_STAGE1, [&] { return launch_stage(c, a, p, false, stream, may_alloc); }));
      }
      RT_HIP(run(RT_K_MG_SOLVE, [&] { return launch_mg_solve(c, a.h, ws.Emg, T, T, ws.Tstar, ws.mapB, stream); }));
      a.h = dt;
      for (int g = 0; g < c->ng; ++g) {
        p.Iflux_v = Jb + g * bin;
        p.mapF = ws.mapB + 2 * g * nc;
        p.Ibase_v = Ib + g * bin;
        p.mapB = mapA ? mapA + 2 * g * nc : nullptr;
        p.Iout_v = Ib + g * bin;
        p.mapO = nullptr;
        p.Tstart = T;
        p.Tcoef = ws.Tstar;
        p.Tout = nullptr;
        p.ka = c->d_ka_g + g * nc;
        p.sumE = ws.Emg + g * nc;
        RT_HIP(run(RT_K_STAGE2, [&] { return launch_stage(c, a, p, true, stream, may_alloc); }));
      }
      RT_HIP(run(RT_K_MG_SOLVE, [&] { return launch_mg_solve(c, dt, ws.Emg, T, ws.Tstar, T, ws.mapA, stream); }));
      mapA = ws.mapA;
    }
    if (mapA) {
      // the bins' last maps, with R^(ab) and the 4-force summed over the bins
      for (int g = 0; g < c->ng; ++g)
        RT_HIP(run(RT_K_MATERIALIZE, [&] {
          return launch_materialize(c, Ib + g * bin, mapA + 2 * g * nc, dt, R_out, G_out, stream, g > 0);
        }));
    }
  } else {
    const double* mapA = nullptr;  // the caller's I is materialised on entry
    for (int k = 0; k < nsteps; ++k) {
      const bool last = k == nsteps - 1;
      // stage 1: fluxes of I^n, half step, interaction from T^n with opacities at T^n
      a.h = 0.5 * dt;
      p.Iflux_v = I;
      p.mapF = mapA;
      p.Ibase_v = nullptr;
      p.mapB = nullptr;
      p.Iout_v = ws.Itil;
      p.mapO = ws.mapB;
      p.Tstart = T;
      p.Tcoef = T;
      p.Tout = ws.Tstar;
      if (c->curved)
        RT_HIP(run(RT_K_ANGULAR, [&] { return launch_angular(c, I, ws.angD, ws.mp_grad, stream); }));
      RT_HIP(run(RT_K_STAGE1, [&] { return launch_stage(c, a, p, false, stream, may_alloc); }));
      const double* mapB = ws.mapB;
      if (c->moving) {
        RT_HIP(run(RT_K_MATERIALIZE, [&] {
          return launch_materialize(c, ws.Itil, ws.mapB, a.h, nullptr, nullptr, stream);
        }));
        mapB = nullptr;
      }
      // stage 2: fluxes of I*, full step from I^n, energy balance from T^n, opacities at T*
      a.h = dt;
      p.Iflux_v = ws.Itil;
      p.mapF = mapB;
      p.Ibase_v = I;
      p.mapB = mapA;
      p.Iout_v = I;
      p.mapO = ws.mapA;
      p.Tstart = T;
      p.Tcoef = ws.Tstar;
      p.Tout = T;
      if (c->curved)
        RT_HIP(run(RT_K_ANGULAR, [&] { return launch_angular(c, ws.Itil, ws.angD, ws.mp_grad, stream); }));
      RT_HIP(run(RT_K_STAGE2, [&] { return launch_stage(c, a, p, true, stream, may_alloc); }));
      if (c->moving) {
        RT_HIP(run(RT_K_MATERIALIZE, [&] {
          return launch_materialize(c, I, ws.mapA, dt, last ? R_out : nullptr, last ? G_out : nullptr,
                                    stream);
        }));
        mapA = nullptr;
      } else {
        mapA = ws.mapA;
      }
    }
    if (mapA) {
      // at rest the last interaction is still a lazy map: apply it, with the
      // moments and the 4-force of the last step
      RT_HIP(run(RT_K_MATERIALIZE, [&] { return launch_materialize(c, I, mapA, dt, R_out, G_out, stream); }));
    }
  }
  if (c->debug & 1) {
    RT_HIP(launch_nonfinite(c, I, T, stream));
    unsigned long long h[2];
    RT_HIP(hipMemcpyAsync(h, c->d_count, sizeof h, hipMemcpyDeviceToHost, stream));
    RT_HIP(hipStreamSynchronize(stream));
    RT_HIP(launch_fill_u64(c->d_count + 1, 1, 0ull, stream));
    if (h[1]) return fail(RT_E_NONFINITE, "rt_step: " + std::to_string(h[1]) + " non-finite values");
    if (h[0]) {
      set_error("rt_step: " + std::to_string(h[0]) + " cells without a valid temperature root");
      return RT_W_NEWTON;
    }
  }
  return RT_OK;
}

// argument checks shared by rt_step and rt_step_noalloc
rt_status check_step_args(const rt_ctx* c, const char* who, const void* I, const double* T, double dt,
                          int nsteps, const double* G_out, const double* R_out) {
  const std::string w(who);
  if (!c) return fail(RT_E_ARG, w + ": ctx is NULL");
  if (!c->metric_set || !c->opac_set) return fail(RT_E_STATE, w + ": set metric and opacities first");
  if (!I || !T) return fail(RT_E_ARG, w + ": I and T are required");
  if (!aligned(I) || !aligned(T) || (G_out && !aligned(G_out)) || (R_out && !aligned(R_out)))
    return fail(RT_E_ARG, w + ": arrays must be 256-byte aligned");
  if (nsteps < 0) return fail(RT_E_ARG, w + ": nsteps must be >= 0");
  if (!(dt > 0.0) || dt > c->dt_max * (1.0 + 1e-12))
    return fail(RT_E_ARG, w + ": need 0 < dt <= dt_max (" + std::to_string(c->dt_max) + ")");
  if (c->ng && (c->curved || c->moving || c->opac.model != RT_OPAC_KIRCHHOFF_CONST))
    return fail(RT_E_STATE, w + ": frequency bins need a fluid at rest and RT_OPAC_KIRCHHOFF_CONST");
  return RT_OK;
}
}  // namespace
}  // namespace rt

using namespace rt;

extern "C" {

const char* rt_last_error(void) { return rt::g_err.c_str(); }

rt_status rt_init_grid(const rt_grid_desc* d, rt_ctx** out) {
  if (!out) return fail(RT_E_ARG, "rt_init_grid: out is NULL");
  *out = nullptr;
  if (!d) return fail(RT_E_ARG, "rt_init_grid: descriptor is NULL");
  for (int a = 0; a < 3; ++a) {
    if (d->n[a] < 1) return fail(RT_E_ARG, "rt_init_grid: n[a] must be >= 1");
    if (!(d->xhi[a] > d->xlo[a])) return fail(RT_E_ARG, "rt_init_grid: xhi must exceed xlo");
    for (int side = 0; side < 2; ++side) {
      int b = side ? d->bc_hi[a] : d->bc_lo[a];
      if (b < RT_BC_PERIODIC || b > RT_BC_ZERO_INCOMING) return fail(RT_E_ARG, "rt_init_grid: bad bc");
    }
    if ((d->bc_lo[a] == RT_BC_PERIODIC) != (d->bc_hi[a] == RT_BC_PERIODIC))
      return fail(RT_E_ARG, "rt_init_grid: periodic must be set on both sides of an axis");
  }
  if (d->coords != RT_CART && d->coords != RT_LOGR_THETA_PHI) return fail(RT_E_ARG, "rt_init_grid: bad coords");
  if (d->pole_zero_rows < 0 || 2 * d->pole_zero_rows > d->n[1])
    return fail(RT_E_ARG, "rt_init_grid: pole_zero_rows must be in 0..n[1]/2");
  if (d->coords == RT_CART && d->pole_zero_rows != 0)
    return fail(RT_E_ARG, "rt_init_grid: pole_zero_rows needs RT_LOGR_THETA_PHI");
  if (!(d->n0_cut >= 0.0)) return fail(RT_E_ARG, "rt_init_grid: n0_cut must be >= 0");
  if (d->generation < 0 || d->generation > 5) return fail(RT_E_ARG, "rt_init_grid: generation in 0..5");
  if (d->weights != RT_W_VORONOI && d->weights != RT_W_EQUAL) return fail(RT_E_ARG, "rt_init_grid: bad weights");
  if (d->precision != RT_FP64 && d->precision != RT_FP32_TRANSPORT)
    return fail(RT_E_ARG, "rt_init_grid: bad precision");
  if (d->limiter != RT_LIM_MC && d->limiter != RT_LIM_MINMOD) return fail(RT_E_ARG, "rt_init_grid: bad limiter");
  if (d->angular_recon != RT_AREC_DONOR && d->angular_recon != RT_AREC_MAPR)
    return fail(RT_E_ARG, "rt_init_grid: bad angular_recon");
  if (!(d->abar >= 0.0) || !(d->rho_floor >= 0.0)) return fail(RT_E_ARG, "rt_init_grid: abar, rho_floor >= 0");
  long long nc = (long long)d->n[0] * d->n[1] * d->n[2];
  // the stage kernels address one direction's plane with 32-bit byte offsets
  if (nc >= (1ll << 29)) return fail(RT_E_ARG, "rt_init_grid: at most 2^29 - 1 cells");

  rt_ctx* c = nullptr;
  try {
    c = new rt_ctx();
    c->grid = build_geodesic_grid(d->generation, d->weights == RT_W_EQUAL);
  } catch (const std::bad_alloc&) {
    delete c;
    return fail(RT_E_NOMEM, "rt_init_grid: host allocation failed");
  } catch (const std::exception& e) {
    delete c;
    return fail(RT_E_ARG, std::string("rt_init_grid: ") + e.what());
  }
  c->desc = *d;
  c->ns = c->grid.ns;
  for (int a = 0; a < 3; ++a) {
    c->n[a] = d->n[a];
    c->dx[a] = (d->xhi[a] - d->xlo[a]) / d->n[a];
  }
  c->nc = nc;
  c->fp32 = d->precision == RT_FP32_TRANSPORT;
  c->elem = c->fp32 ? 4 : 8;
  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "hipGetDevice");
  }
  // the allocation-free entry point's static scratch: its address on this
  // device, resolved once per device with the device current (a failure here
  // only disables rt_step_noalloc, which then reports it)
  if ((e = noalloc_scratch_init(c->device)) != hipSuccess) {
    c->noalloc_error = std::string("hipGetSymbolAddress of the static scratch: ") + hipGetErrorString(e);
    (void)hipGetLastError();
  }
  const int ns = c->ns;
  const int ns4 = (ns + 3) / 4 * 4;
  std::vector<double> dir(3 * ns), w(ns), W16((size_t)ns4 * 16, 0.0);
  std::vector<float> dirf(3 * ns);
  for (int s = 0; s < ns; ++s) {
    for (int k = 0; k < 3; ++k) {
      dir[k * ns + s] = c->grid.dir[s][k];
      dirf[k * ns + s] = (float)c->grid.dir[s][k];
    }
    w[s] = c->grid.w[s];
    double n4[4] = {1.0, c->grid.dir[s][0], c->grid.dir[s][1], c->grid.dir[s][2]};
    static const int pa[10] = {0, 0, 0, 0, 1, 1, 1, 2, 2, 3};
    static const int pb[10] = {0, 1, 2, 3, 1, 2, 3, 2, 3, 3};
    for (int k = 0; k < 10; ++k) W16[(size_t)s * 16 + k] = w[s] * n4[pa[k]] * n4[pb[k]];
  }
  for (int s = 0; s < ns; ++s) {
    c->W0 += w[s];
    for (int k = 0; k < 10; ++k) c->Wsum[k] += W16[(size_t)s * 16 + k];
  }
  rt_status st = RT_OK;
  if ((st = alloc(&c->d_dir, dir.size() * 8)) || (st = alloc(&c->d_dir_f, dirf.size() * 4)) ||
      (st = alloc(&c->d_w, w.size() * 8)) || (st = alloc(&c->d_W16, W16.size() * 8)) ||
      (st = alloc(&c->d_count, 2 * sizeof(unsigned long long)))) {
    rt_destroy(c);
    return st;
  }
  if ((e = hipMemcpy(c->d_dir, dir.data(), dir.size() * 8, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(c->d_dir_f, dirf.data(), dirf.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(c->d_w, w.data(), w.size() * 8, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(c->d_W16, W16.data(), W16.size() * 8, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemset(c->d_count, 0, 2 * sizeof(unsigned long long))) != hipSuccess) {
    rt_destroy(c);
    return hip_fail(e, "rt_init_grid upload");
  }
  *out = c;
  return RT_OK;
}

rt_status rt_geodesic_grid(int generation, int weights, int* n_dirs, double* dirs_host,
                           double* w_host, double* area_host) {
  if (generation < 0 || generation > 5) return fail(RT_E_ARG, "rt_geodesic_grid: generation in 0..5");
  if (weights != RT_W_VORONOI && weights != RT_W_EQUAL) return fail(RT_E_ARG, "rt_geodesic_grid: bad weights");
  GeodesicGrid G;
  try {
    G = build_geodesic_grid(generation, weights == RT_W_EQUAL);
  } catch (const std::exception& e) {
    return fail(RT_E_NOMEM, std::string("rt_geodesic_grid: ") + e.what());
  }
  if (n_dirs) *n_dirs = G.ns;
  for (int s = 0; s < G.ns; ++s) {
    if (dirs_host)
      for (int k = 0; k < 3; ++k) dirs_host[3 * s + k] = G.dir[s][k];
    if (w_host) w_host[s] = G.w[s];
    if (area_host) area_host[s] = G.area[s];
  }
  return RT_OK;
}

rt_status rt_grid_info(const rt_ctx* c, int* n_dirs, double* dirs_host, double* w_host,
                       double* area_host) {
  if (!c) return fail(RT_E_ARG, "rt_grid_info: ctx is NULL");
  if (n_dirs) *n_dirs = c->ns;
  for (int s = 0; s < c->ns; ++s) {
    if (dirs_host)
      for (int k = 0; k < 3; ++k) dirs_host[3 * s + k] = c->grid.dir[s][k];
    if (w_host) w_host[s] = c->grid.w[s];
    if (area_host) area_host[s] = c->grid.area[s];
  }
  return RT_OK;
}

rt_status rt_set_metric(rt_ctx* c, int kind, double M, double a, double cfl, double* dt_max_out) {
  if (!c) return fail(RT_E_ARG, "rt_set_metric: ctx is NULL");
  if (!(cfl > 0.0)) return fail(RT_E_ARG, "rt_set_metric: cfl must be > 0");
  if (kind != RT_FLAT && kind != RT_KERR_SCHILD) return fail(RT_E_ARG, "rt_set_metric: bad kind");
  if (kind == RT_FLAT && c->desc.coords != RT_CART)
    return fail(RT_E_ARG, "rt_set_metric: RT_FLAT needs RT_CART coordinates");
  if (kind == RT_KERR_SCHILD && c->desc.coords != RT_LOGR_THETA_PHI)
    return fail(RT_E_ARG, "rt_set_metric: RT_KERR_SCHILD needs RT_LOGR_THETA_PHI coordinates");
  if (kind == RT_KERR_SCHILD && (!(M >= 0.0) || !(std::fabs(a) <= M || M == 0.0) || (M == 0.0 && a != 0.0)))
    return fail(RT_E_ARG, "rt_set_metric: need M >= 0 and |a| <= M");
  if (c->metric_set) return fail(RT_E_STATE, "rt_set_metric: the metric is already set");
  rt_status st = use_device(c);
  if (st) return st;
  c->metric_kind = kind;
  if (kind == RT_FLAT) {
    double vmax[3] = {0, 0, 0};
    for (int s = 0; s < c->ns; ++s)
      for (int k = 0; k < 3; ++k) vmax[k] = std::max(vmax[k], std::fabs(c->grid.dir[s][k]));
    double dtm = INFINITY;
    for (int k = 0; k < 3; ++k) dtm = std::min(dtm, c->dx[k] / vmax[k]);
    c->dt_max = cfl * dtm;
  } else if ((st = set_kerr_schild(c, M, a, cfl))) {
    return st;
  }
  // per-stage scratch: one intensity copy (the half-step state) and two lazy maps
  const size_t nc = (size_t)c->nc, ns = (size_t)c->ns;
  if ((st = alloc(&c->d_Tstar, nc * 8)) || (st = alloc(&c->d_mapA, 3 * nc * 8)) ||
      (st = alloc(&c->d_mapB, 3 * nc * 8)) || (st = alloc(&c->d_Itil, ns * nc * c->elem)))
    return st;
  c->metric_set = true;
  if (dt_max_out) *dt_max_out = c->dt_max;
  return RT_OK;
}

rt_status rt_set_opacities(rt_ctx* c, const rt_opacity_desc* o, hipStream_t stream) {
  if (!c || !o) return fail(RT_E_ARG, "rt_set_opacities: NULL argument");
  if (!c->metric_set) return fail(RT_E_STATE, "rt_set_opacities: call rt_set_metric first");
  if (o->model < RT_OPAC_KIRCHHOFF_CONST || o->model > RT_OPAC_BREMS_M3)
    return fail(RT_E_ARG, "rt_set_opacities: bad model");
  if (!(o->gamma > 1.0)) return fail(RT_E_ARG, "rt_set_opacities: gamma must be > 1");
  if (!o->rho) return fail(RT_E_ARG, "rt_set_opacities: rho is required");
  if (o->newton_max_iter < 1 || !(o->newton_rtol > 0.0))
    return fail(RT_E_ARG, "rt_set_opacities: newton_max_iter >= 1 and newton_rtol > 0");
  const void* ptrs[] = {o->rho, o->u, o->kappa_a, o->kappa_s, o->j};
  for (const void* p : ptrs)
    if (p && !aligned(p)) return fail(RT_E_ARG, "rt_set_opacities: arrays must be 256-byte aligned");
  rt_status st = use_device(c);
  if (st) return st;
  const size_t nb = (size_t)c->nc * 8;
  if ((st = alloc(&c->d_rho, nb)) || (st = alloc(&c->d_uhat, 4 * nb)) || (st = alloc(&c->d_v, 3 * nb)))
    return st;
  RT_HIP(hipMemcpyAsync(c->d_rho, o->rho, nb, hipMemcpyDeviceToDevice, stream));
  // u-hat^a = e^a_mu u^mu (identity when flat); v^a = u^a / u^0 for the advection
  // term.  The curved geometry always takes the direction-dependent map.
  c->moving = o->u != nullptr || c->curved;
  RT_HIP(launch_fluid(c, o->u, stream));
  auto copy_opt = [&](double** dst, const double* src) -> rt_status {
    if (!src) {
      release(*dst);
      return RT_OK;
    }
    rt_status s2 = alloc(dst, nb);
    if (s2) return s2;
    RT_HIP(hipMemcpyAsync(*dst, src, nb, hipMemcpyDeviceToDevice, stream));
    return RT_OK;
  };
  if ((st = copy_opt(&c->d_ka, o->kappa_a)) || (st = copy_opt(&c->d_ks, o->kappa_s)) ||
      (st = copy_opt(&c->d_j, o->j)))
    return st;
  c->opac = *o;
  c->opac.rho = c->opac.u = c->opac.kappa_a = c->opac.kappa_s = c->opac.j = nullptr;
  c->opac_set = true;
  return RT_OK;
}

rt_status rt_set_groups(rt_ctx* c, int ng, const double* nu_edges_host, const double* kappa_a_groups,
                        hipStream_t stream) {
  if (!c) return fail(RT_E_ARG, "rt_set_groups: ctx is NULL");
  if (!c->metric_set || !c->opac_set) return fail(RT_E_STATE, "rt_set_groups: set metric and opacities first");
  if (ng < 0 || ng > RT_MAX_GROUPS)
    return fail(RT_E_ARG, "rt_set_groups: ng must be in 0.." + std::to_string(RT_MAX_GROUPS));
  if (ng > 0) {
    if (c->curved || c->moving || c->opac.model != RT_OPAC_KIRCHHOFF_CONST)
      return fail(RT_E_STATE,
                  "rt_set_groups: frequency bins need the flat metric, a fluid at rest and RT_OPAC_KIRCHHOFF_CONST");
    if (!nu_edges_host || !kappa_a_groups) return fail(RT_E_ARG, "rt_set_groups: NULL argument");
    if (!aligned(kappa_a_groups)) return fail(RT_E_ARG, "rt_set_groups: kappa_a_groups must be 256-byte aligned");
    if (!(nu_edges_host[0] >= 0.0) || std::isinf(nu_edges_host[0]))
      return fail(RT_E_ARG, "rt_set_groups: the first edge must be finite and >= 0");
    for (int g = 0; g < ng; ++g)
      if (!(nu_edges_host[g + 1] > nu_edges_host[g]) || (g + 1 < ng && std::isinf(nu_edges_host[g + 1])))
        return fail(RT_E_ARG, "rt_set_groups: edges must increase (only the last may be +inf)");
  }
  rt_status st = use_device(c);
  if (st) return st;
  const size_t nc = (size_t)c->nc, ns = (size_t)c->ns;
  const int old = c->ng;
  const size_t ngo = (size_t)std::max(old, 1), ngn = (size_t)std::max(ng, 1);
  // the scratch of the old layout may still be in use by enqueued work
  RT_HIP(hipStreamSynchronize(stream));
  release(c->d_ka_g);
  release(c->d_Emg);
  c->ng = 0;
  c->nu_edges.clear();
  if (ngn != ngo || std::max<size_t>(3, 2 * (size_t)ng) != std::max<size_t>(3, 2 * (size_t)old)) {
    release(c->d_Itil);
    release(c->d_mapA);
    release(c->d_mapB);
  }
  const size_t mw = std::max<size_t>(3, 2 * (size_t)ng);
  if ((st = alloc(&c->d_Itil, ngn * ns * nc * c->elem)) || (st = alloc(&c->d_mapA, mw * nc * 8)) ||
      (st = alloc(&c->d_mapB, mw * nc * 8)))
    return st;
  if (ng == 0) return RT_OK;
  if ((st = alloc(&c->d_ka_g, (size_t)ng * nc * 8)) || (st = alloc(&c->d_Emg, (size_t)ng * nc * 8))) return st;
  RT_HIP(hipMemcpyAsync(c->d_ka_g, kappa_a_groups, (size_t)ng * nc * 8, hipMemcpyDeviceToDevice, stream));
  c->nu_edges.assign(nu_edges_host, nu_edges_host + ng + 1);
  c->ng = ng;
  return RT_OK;
}

rt_status rt_step(rt_ctx* c, void* I, double* T, double dt, int nsteps, double* G_out,
                  double* R_out, hipStream_t stream) {
  rt_status st = check_step_args(c, "rt_step", I, T, dt, nsteps, G_out, R_out);
  if (st) return st;
  if ((st = use_device(c))) return st;
  StepScratch ws{};
  ws.Itil = c->d_Itil;
  ws.mapA = c->d_mapA;
  ws.mapB = c->d_mapB;
  ws.Tstar = c->d_Tstar;
  ws.angD = c->d_angD;
  ws.mp_grad = c->d_mp_grad;
  ws.Emg = c->d_Emg;
  return step_impl(c, ws, true, I, T, dt, nsteps, G_out, R_out, stream);
}

rt_status rt_step_noalloc(rt_ctx* c, void* I, double* T, double dt, int nsteps, double* G_out,
                          double* R_out, hipStream_t stream) {
  rt_status st = check_step_args(c, "rt_step_noalloc", I, T, dt, nsteps, G_out, R_out);
  if (st) return st;
  const size_t need = step_scratch_bytes(c);
  if (need > kNoallocScratchBytes)
    return fail(RT_E_ARG, "rt_step_noalloc: this grid needs " + std::to_string(need) +
                              " bytes of step scratch; the static scratch holds " +
                              std::to_string(kNoallocScratchBytes));
  if ((st = use_device(c))) return st;
  void* base = noalloc_scratch_ptr(c->device);
  if (!base)
    return fail(RT_E_STATE, "rt_step_noalloc: the static scratch of this device is not resolved (" +
                                c->noalloc_error + ")");
  return step_impl(c, carve_step_scratch(c, base), false, I, T, dt, nsteps, G_out, R_out, stream);
}

rt_status rt_moments(rt_ctx* c, const void* I, double* R, double* J, int frame, hipStream_t stream) {
  if (!c) return fail(RT_E_ARG, "rt_moments: ctx is NULL");
  if (!I || !R) return fail(RT_E_ARG, "rt_moments: I and R are required");
  if (!aligned(I) || !aligned(R) || (J && !aligned(J)))
    return fail(RT_E_ARG, "rt_moments: arrays must be 256-byte aligned");
  if (frame != RT_TETRAD && frame != RT_COORD) return fail(RT_E_ARG, "rt_moments: bad frame");
  rt_status st = use_device(c);
  if (st) return st;
  RT_HIP(timed(c, RT_K_MOMENTS, stream, [&] { return launch_moments(c, I, R, J, stream); }));
  // flat metric: the identity tetrad makes both frames coincide
  if (frame == RT_COORD && c->curved) RT_HIP(launch_to_coord(c, R, stream));
  return RT_OK;
}

rt_status rt_step_adjoint(rt_ctx* c, const void* I_n, const double* T_n, double dt,
                          const void* gI_np1, void* gI_n, double* g_kappa_a, double* g_j,
                          hipStream_t stream) {
  if (!c) return fail(RT_E_ARG, "rt_step_adjoint: ctx is NULL");
  if (!c->metric_set || !c->opac_set) return fail(RT_E_STATE, "rt_step_adjoint: set metric and opacities first");
  if (c->opac.model != RT_OPAC_FIXED_EMISSIVITY)
    return fail(RT_E_ARG, "rt_step_adjoint: only the FIXED_EMISSIVITY model is differentiated");
  if (c->curved) return fail(RT_E_ARG, "rt_step_adjoint: only the flat metric is differentiated");
  if (c->moving) return fail(RT_E_ARG, "rt_step_adjoint: fluid must be at rest");
  if (c->ng) return fail(RT_E_ARG, "rt_step_adjoint: frequency bins are not differentiated");
  if (!I_n || !T_n || !gI_np1 || !gI_n) return fail(RT_E_ARG, "rt_step_adjoint: NULL argument");
  if (!aligned(I_n) || !aligned(T_n) || !aligned(gI_np1) || !aligned(gI_n) ||
      (g_kappa_a && !aligned(g_kappa_a)) || (g_j && !aligned(g_j)))
    return fail(RT_E_ARG, "rt_step_adjoint: arrays must be 256-byte aligned");
  if (!(dt > 0.0) || dt > c->dt_max * (1.0 + 1e-12)) return fail(RT_E_ARG, "rt_step_adjoint: bad dt");
  rt_status st = use_device(c);
  if (st) return st;
  const size_t bytes = (size_t)c->ns * c->nc * c->elem;
  if ((st = alloc(&c->d_gA, bytes)) || (st = alloc(&c->d_gB, bytes)) || (st = alloc(&c->d_gC, bytes)) ||
      (st = alloc(&c->d_gD, bytes)) || (st = alloc(&c->d_gcell, 6 * (size_t)adjoint_dir_groups(c) * c->nc * 8)) ||
      (st = alloc(&c->d_gT, 2 * (size_t)c->nc * 8)))
    return st;
  RT_HIP(timed(c, RT_K_ADJOINT, stream, [&] {
    return launch_adjoint_step(c, I_n, T_n, dt, gI_np1, nullptr, gI_n, nullptr, g_kappa_a, g_j, stream);
  }));
  return RT_OK;
}

rt_status rt_step_adjoint_thermal(rt_ctx* c, const void* I_n, const double* T_n, double dt,
                                  const void* gI_np1, const double* gT_np1, void* gI_n, double* gT_n,
                                  double* g_kappa_a, hipStream_t stream) {
  if (!c) return fail(RT_E_ARG, "rt_step_adjoint_thermal: ctx is NULL");
  if (!c->metric_set || !c->opac_set)
    return fail(RT_E_STATE, "rt_step_adjoint_thermal: set metric and opacities first");
  if (c->opac.model != RT_OPAC_BREMS)
    return fail(RT_E_ARG, "rt_step_adjoint_thermal: only the BREMS model (Method 2) is differentiated");
  if (c->curved) return fail(RT_E_ARG, "rt_step_adjoint_thermal: only the flat metric is differentiated");
  if (c->moving) return fail(RT_E_ARG, "rt_step_adjoint_thermal: fluid must be at rest");
  if (c->ng) return fail(RT_E_ARG, "rt_step_adjoint_thermal: frequency bins are not differentiated");
  if (!I_n || !T_n || !gI_np1 || !gI_n || !gT_n) return fail(RT_E_ARG, "rt_step_adjoint_thermal: NULL argument");
  if (!aligned(I_n) || !aligned(T_n) || !aligned(gI_np1) || !aligned(gI_n) || !aligned(gT_n) ||
      (gT_np1 && !aligned(gT_np1)) || (g_kappa_a && !aligned(g_kappa_a)))
    return fail(RT_E_ARG, "rt_step_adjoint_thermal: arrays must be 256-byte aligned");
  if (gT_n == T_n || (const void*)gT_n == (const void*)gT_np1)
    return fail(RT_E_ARG, "rt_step_adjoint_thermal: gT_n may alias neither T_n nor gT_np1");
  if (!(dt > 0.0) || dt > c->dt_max * (1.0 + 1e-12)) return fail(RT_E_ARG, "rt_step_adjoint_thermal: bad dt");
  rt_status st = use_device(c);
  if (st) return st;
  const size_t bytes = (size_t)c->ns * c->nc * c->elem;
  if ((st = alloc(&c->d_gA, bytes)) || (st = alloc(&c->d_gB, bytes)) || (st = alloc(&c->d_gC, bytes)) ||
      (st = alloc(&c->d_gD, bytes)) || (st = alloc(&c->d_gcell, 6 * (size_t)adjoint_dir_groups(c) * c->nc * 8)) ||
      (st = alloc(&c->d_gT, 2 * (size_t)c->nc * 8)))
    return st;
  RT_HIP(timed(c, RT_K_ADJOINT, stream, [&] {
    return launch_adjoint_step(c, I_n, T_n, dt, gI_np1, gT_np1, gI_n, gT_n, g_kappa_a, nullptr, stream);
  }));
  return RT_OK;
}

rt_status rt_set_debug(rt_ctx* c, int flags) {
  if (!c) return fail(RT_E_ARG, "rt_set_debug: ctx is NULL");
  c->debug = flags;
  return RT_OK;
}

rt_status rt_kernel_times(rt_ctx* c, int* counts, double* ms) {
  if (!c) return fail(RT_E_ARG, "rt_kernel_times: ctx is NULL");
  rt_status st = use_device(c);
  if (st) return st;
  int cnt[RT_NKERNELS] = {0};
  double tot[RT_NKERNELS] = {0.0};
  for (auto& t : c->timed) {
    RT_HIP(hipEventSynchronize(t.b));
    float m = 0.f;
    RT_HIP(hipEventElapsedTime(&m, t.a, t.b));
    cnt[t.kind] += 1;
    tot[t.kind] += m;
    c->event_pool.push_back(t.a);
    c->event_pool.push_back(t.b);
  }
  c->timed.clear();
  for (int k = 0; k < RT_NKERNELS; ++k) {
    if (counts) counts[k] = cnt[k];
    if (ms) ms[k] = tot[k];
  }
  return RT_OK;
}

rt_status rt_newton_failures(rt_ctx* c, long long* count) {
  if (!c || !count) return fail(RT_E_ARG, "rt_newton_failures: NULL argument");
  rt_status st = use_device(c);
  if (st) return st;
  unsigned long long h = 0;
  RT_HIP(hipMemcpy(&h, c->d_count, sizeof h, hipMemcpyDeviceToHost));
  RT_HIP(hipMemset(c->d_count, 0, sizeof h));
  *count = (long long)h;
  return RT_OK;
}

void rt_destroy(rt_ctx* c) {
  if (!c) return;
  (void)use_device(c);
  (void)hipDeviceSynchronize();
  release(c->d_dir);
  release(c->d_dir_f);
  release(c->d_w);
  release(c->d_W16);
  release(c->d_rho);
  release(c->d_uhat);
  release(c->d_v);
  release(c->d_ka);
  release(c->d_ks);
  release(c->d_j);
  release(c->d_Tstar);
  release(c->d_mapA);
  release(c->d_mapB);
  release(c->d_Itil);
  release(c->d_ka_g);
  release(c->d_Emg);
  release(c->d_gA);
  release(c->d_gB);
  release(c->d_gC);
  release(c->d_gD);
  release(c->d_gcell);
  release(c->d_gT);
  release(c->d_count);
  release(c->d_tile_order);
  release(c->d_rec_r);
  release(c->d_rec_t);
  release(c->d_rec_p);
  release(c->d_zin);
  release(c->d_acoef);
  release(c->d_nu0);
  release(c->d_e);
  release(c->d_einv);
  release(c->d_inc);
  release(c->d_plist);
  release(c->d_poff);
  release(c->d_pnout);
  release(c->d_plnb);
  release(c->d_angD);
  release(c->d_mp_ring);
  release(c->d_mp_minv);
  release(c->d_mp_pq);
  release(c->d_mp_coef);
  release(c->d_mp_self);
  release(c->d_mp_grad);
  for (auto& t : c->timed) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (auto e : c->event_pool) (void)hipEventDestroy(e);
  delete c;
}

}  // extern "C"
