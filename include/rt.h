/*
 * rt.h -- C ABI of the MI355X (gfx950) gray covariant radiative-transfer step.
 *
 * The library evolves the tetrad-frame gray specific intensity I-hat on a
 * geodesic angular grid in a fixed (stationary) metric, as in arXiv
 * 2508.15532 (Wallace, Begue, Pe'er): the finite-volume transport of the
 * covariant transfer equation (Sec. 3.1, Eq. radiative_transfer_discrete;
 * spatial fluxes of Sec. 3.5; in curved space the angular fluxes between
 * directions of Sec. 2.2 and 3.5), the implicit radiation-fluid interaction (Sec. 3.6.2,
 * Eq. fluid_interaction_discrete and the temperature equations), the
 * predictor-corrector step (Sec. 3.7), and the moments R^(ab) = int n^a n^b I
 * dOmega (Eq. R).  Units are scale free: c = G = a_rad = k_B/(mu m_p) = 1.
 *
 * Layout.  Spatial cells are indexed c = (i1*N2 + i2)*N3 + i3 (i3 fastest).
 * Intensities are direction-major: I[s*Nc + c], s = 0..Ns-1, Nc = N1*N2*N3.
 * Element type of I: double for RT_FP64, float for RT_FP32_TRANSPORT.
 * Per-cell fields are double [Nc]; multi-component fields are
 * component-major ([k*Nc + c]).
 *
 * Pointers: every array argument is a device pointer (HIP global memory)
 * unless its name ends in _host.  The caller owns every array it passes; the
 * library owns the context, the angular grid, the geometry tables and its own
 * copies of the fluid fields.  Device arrays must be 256-byte aligned and
 * dense.  Calls that take a stream enqueue work on that stream and return
 * without synchronising (unless debug checking is enabled, see
 * rt_set_debug); rt_init_grid and rt_set_metric are synchronous host calls.
 *
 * Errors: every call returns an rt_status; a negative value means the call
 * did nothing observable except possibly partial writes to its outputs, which
 * are then unspecified.  rt_last_error() returns a message describing the
 * last non-OK status raised on the calling thread.
 */
#ifndef RT_H
#define RT_H

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rt_ctx rt_ctx;

typedef enum {
  RT_OK = 0,
  RT_W_NEWTON = 1,      /* step done; some cells had no valid temperature root
                           and kept their pre-interaction state.  Returned only
                           with debug checking on (rt_set_debug bit 0): without
                           it rt_step returns before the device has run, so the
                           count is read with rt_newton_failures instead */
  RT_E_ARG = -1,        /* invalid argument (null pointer, size, enum, dt) */
  RT_E_STATE = -2,      /* call order violated (e.g. step before set_metric) */
  RT_E_HIP = -3,        /* a HIP runtime call failed */
  RT_E_NOMEM = -4,      /* device allocation failed */
  RT_E_NONFINITE = -5   /* non-finite intensity or temperature (debug mode) */
} rt_status;

/* coordinates of the logical mesh (Sec. 3.2) */
enum { RT_CART = 0, RT_LOGR_THETA_PHI = 1 };
/* boundary conditions per axis side */
enum { RT_BC_PERIODIC = 0, RT_BC_OUTFLOW = 1, RT_BC_ZERO_INCOMING = 2 };
/* quadrature weights of the geodesic grid */
enum { RT_W_VORONOI = 0, RT_W_EQUAL = 1 };
/* numerical forms: plain FP64, or FP32 intensities and transport with the
   interaction solve and the moment accumulation in FP64 */
enum { RT_FP64 = 0, RT_FP32_TRANSPORT = 1 };
/* PLI slope limiter (Sec. 3.4) */
enum { RT_LIM_MC = 0, RT_LIM_MINMOD = 1 };
/* states at the Voronoi edges for the angular fluxes of the curved geometry
   (Sec. 3.5; reconstruction of Sec. 3.4): the upwind direction's own intensity (donor cell), or its MAPR
   reconstruction: the flattest of the planes through the direction and
   consecutive pairs of its neighbours in gnomonic coordinates, evaluated at
   the edge midpoint and replaced by the cell value where negative */
enum { RT_AREC_DONOR = 0, RT_AREC_MAPR = 1 };
/* metric (fixed in time, Sec. 2.1.1) */
enum { RT_FLAT = 0, RT_KERR_SCHILD = 1 };
/* opacity / emission model (Sec. 3.6.2):
   KIRCHHOFF_CONST  alpha^a = rho kappa_a, alpha^s = rho kappa_s, Kirchhoff
                    emission with a constant Planck opacity (Method 1 quartic);
   BREMS            alpha^a = C_a rho^2 T^-7/2 (times kappa_a, a per-cell
                    dimensionless factor, when given), alpha^s = C_s rho,
                    Planck opacity implicit in T (Method 2);
   FIXED_EMISSIVITY alpha^a = rho kappa_a, alpha^s = rho kappa_s, emission
                    4 pi j fixed per cell, temperature unchanged;
   BREMS_M3         the BREMS opacities with Method 3 (Eq. T_almost_fully_implicit):
                    the angular integrals use the explicit total opacity
                    alpha_- = alpha(T_coef), the factor outside them the implicit
                    alpha_+ = alpha(T_+), so every direction's update carries
                    alpha_-/alpha_+; T_+ is the root with non-negative gas energy
                    (safeguarded Newton; at least 120 iterations allowed) */
enum { RT_OPAC_KIRCHHOFF_CONST = 0, RT_OPAC_BREMS = 1, RT_OPAC_FIXED_EMISSIVITY = 2, RT_OPAC_BREMS_M3 = 3 };
/* frame of the moments returned by rt_moments */
enum { RT_TETRAD = 0, RT_COORD = 1 };

typedef struct {
  int n[3];            /* cells per axis (>= 1); at most 2^29 - 1 cells in total */
  double xlo[3];       /* logical lower bounds */
  double xhi[3];       /* logical upper bounds (> xlo) */
  int coords;          /* RT_CART or RT_LOGR_THETA_PHI (x1 = ln r, theta in [0, pi]) */
  int bc_lo[3];        /* RT_BC_* per axis; periodic must be set on both sides */
  int bc_hi[3];
  int generation;      /* geodesic generation g in 0..5: Ns = 10*4^g + 2 */
  int weights;         /* RT_W_VORONOI or RT_W_EQUAL (4 pi / Ns) */
  int precision;       /* RT_FP64 or RT_FP32_TRANSPORT */
  int limiter;         /* RT_LIM_MC or RT_LIM_MINMOD */
  int angular_recon;   /* RT_AREC_DONOR or RT_AREC_MAPR (curved geometry only) */
  double abar;         /* coefficient in tau = abar alpha-hat dt (Sec. 3.5); 1 */
  double rho_floor;    /* no interaction below this density (Sec. 3.8); 5e-4 */
  double n0_cut;       /* |n_0| below which I is zeroed (Sec. 3.5, curved only); 0.1 */
  int pole_zero_rows;  /* theta rows next to each pole whose I is zeroed after each
                          interaction (RT_LOGR_THETA_PHI only, 0..n[1]/2; 4 in the
                          torus setup of Sec. 5); must be 0 for RT_CART */
} rt_grid_desc;

typedef struct {
  int model;           /* RT_OPAC_* */
  double gamma;        /* adiabatic index (> 1) */
  double C_a, C_s;     /* coefficients of the BREMS model */
  const double* rho;   /* [Nc] mass density (required) */
  const double* u;     /* [4][Nc] coordinate-frame fluid 4-velocity u^mu; NULL: at rest
                          (flat), the normal observer (Kerr-Schild) */
  const double* kappa_a; /* [Nc] absorption opacity (KIRCHHOFF_CONST, FIXED_EMISSIVITY; NULL: 0),
                            or the factor of the bremsstrahlung opacity (BREMS, BREMS_M3; NULL: 1) */
  const double* kappa_s; /* [Nc] scattering opacity; NULL: 0 */
  const double* j;     /* [Nc] fluid-frame gray emissivity (FIXED_EMISSIVITY); NULL: 0 */
  int newton_max_iter; /* cap of the temperature Newton iteration (>= 1); 50 */
  double newton_rtol;  /* relative step tolerance; 1e-14 */
} rt_opacity_desc;

/* Build the geodesic grid (Sec. 3.3) and an empty context.  Host-only and
   synchronous; allocates the grid tables on the current device.
   Directions are numbered as follows: a regular icosahedron with a vertex on
   +3 and the second in the 1-3 half plane (x > 0): upper ring at azimuths
   2 pi k/5, lower ring at 2 pi k/5 + pi/5, then -3; each subdivision appends
   the normalised edge midpoints in lexicographic order of the edge's
   (lower, higher) vertex-index pair.  On error *out is NULL. */
rt_status rt_init_grid(const rt_grid_desc* d, rt_ctx** out);

/* Host-only helper, no device work: the geodesic grid of generation g with the
   numbering of rt_init_grid.  n_dirs receives Ns; dirs_host [3*Ns], w_host [Ns]
   and area_host [Ns] may each be NULL (otherwise sized by the caller for Ns =
   10*4^g + 2).  weights is RT_W_VORONOI or RT_W_EQUAL. */
rt_status rt_geodesic_grid(int generation, int weights, int* n_dirs, double* dirs_host,
                           double* w_host, double* area_host);

/* Copy the grid to host arrays: *n_dirs = Ns; dirs_host[3*s + k] = n-hat^k of
   direction s (may be NULL); w_host[s] = quadrature weight (may be NULL);
   area_host[s] = Voronoi solid angle (may be NULL). */
rt_status rt_grid_info(const rt_ctx* ctx, int* n_dirs, double* dirs_host, double* w_host,
                       double* area_host);

/* Set the stationary metric and tetrads (Sec. 2.1.1) and build the geometry
   tables (host, once per context; a second call returns RT_E_STATE).
   kind = RT_FLAT needs coords RT_CART (identity tetrad; M, a ignored).
   kind = RT_KERR_SCHILD needs coords RT_LOGR_THETA_PHI: the Kerr metric of
   mass M >= 0 and spin |a| <= M in Kerr-Schild coordinates with x1 = ln r
   (M = 0, a = 0 is flat space in spherical coordinates); the tetrad's time leg
   is the normal observer and its spatial legs come from Gram-Schmidt of
   (d_phi, d_theta, d_x1) -> (3, 2, 1); the rotation coefficients that drive the
   angular fluxes (Sec. 2.2) use fourth-order central differences of the
   analytic tetrad (step 1e-3), so theta cell centres must lie more than 2e-3
   from the axis.
   Returns in *dt_max_out (may be NULL) the largest admissible step:
   cfl * min over cells and axes of dx^a / max_s |n^a_s / n^0_s| (Sec. 3.8). */
rt_status rt_set_metric(rt_ctx* ctx, int kind, double M, double a, double cfl, double* dt_max_out);

/* Copy the fluid state and opacity model (held fixed during steps, Sec. 3.6.2)
   into library-owned device memory, on `stream`.  The source arrays may be
   freed once the stream has passed this call. */
rt_status rt_set_opacities(rt_ctx* ctx, const rt_opacity_desc* desc, hipStream_t stream);

/* Multi-group transport: split the radiation into ng bins of fluid-frame
   frequency (Sec. 3.1, Eq. radiative_transfer_discrete_non_gray).  Read here
   for a fluid at rest in flat space, where the photon frequency does not change
   along a path, so the frequency flux r^nu vanishes and each bin is
   transported as the gray equation with its own optical depth; the bins couple
   through the gas temperature.  Per bin: absorption alpha^a_g = rho
   kappa_a,g, emission by Kirchhoff's law with the bin-integrated Planck
   function B_g(T) = int B_nu(T) dnu (units a_rad = k_B = h = 1, so the bins
   of [0, inf) sum to T^4/(4 pi)), elastic isotropic scattering alpha^s = rho
   kappa_s (kappa_s of rt_set_opacities) inside the bin.  The interaction is
   Method 1's semi-implicit update in every bin with the temperature equation
   Y (T_+ - T_-) = -sum_g (E+_g - E-_g), solved per cell by safeguarded
   Newton (failures counted as for rt_step).
     ng              number of bins, 1..RT_MAX_GROUPS; 0 switches back to gray.
     nu_edges_host   host [ng + 1]: 0 <= nu_0 < nu_1 < ... < nu_ng; nu_ng may
                     be +INFINITY.  Copied.
     kappa_a_groups  device [ng][Nc] FP64, 256-byte aligned: kappa_a,g per
                     cell.  Copied on `stream` (the source may be freed once
                     the stream has passed this call).
   Needs rt_set_metric (RT_FLAT) and rt_set_opacities (RT_OPAC_KIRCHHOFF_CONST,
   fluid at rest) first, else RT_E_STATE; bad sizes or edges give RT_E_ARG.
   While bins are set, rt_step and rt_step_noalloc take I as [ng][Ns][Nc] (bin
   major) and return R_out and G_out summed over the bins; a later
   rt_set_opacities that leaves this configuration makes rt_step return
   RT_E_STATE.  The adjoints do not support bins (RT_E_ARG).  The call
   reallocates the step scratch after synchronising `stream` (work enqueued on
   other streams must be complete); if an allocation fails (RT_E_NOMEM) the
   context is left gray and without its scratch, and rt_step returns
   RT_E_STATE until a later rt_set_groups succeeds. */
#define RT_MAX_GROUPS 64
rt_status rt_set_groups(rt_ctx* ctx, int ng, const double* nu_edges_host, const double* kappa_a_groups,
                        hipStream_t stream);

/* Advance nsteps predictor-corrector steps (Sec. 3.7):
     stage 1: I~ = I^n - dt/2 div F(I^n); (I*, T*) = interaction(I~, dt/2, T^n, T^n)
     stage 2: I~ = I^n - dt   div F(I*);  (I^n+1, T^n+1) = interaction(I~, dt, T^n, T*)
   where interaction(I~, h, T_start, T_coef) uses explicit opacities at T_coef
   and starts the energy balance from T_start.
   I     in/out [Ns][Nc] (element type per precision; [ng][Ns][Nc] while
         frequency bins are set, see rt_set_groups), T in/out [Nc].
   G_out optional [4][Nc]: tetrad-frame 4-force on the fluid of the last
         step's second interaction, -(R^(0a)(after) - R^(0a)(before))/dt.
   R_out optional [10][Nc]: moments (as rt_moments, tetrad frame, FP64 sums of
         the stored intensity) of the intensity returned, i.e. of the last
         step; computed in the pass that applies the last interaction, where
         the intensity is already in registers (an argument added to the
         step for that reason: it saves the separate read of I that
         rt_moments would make).
   0 < dt <= dt_max of rt_set_metric, else RT_E_ARG. */
rt_status rt_step(rt_ctx* ctx, void* I, double* T, double dt, int nsteps, double* G_out,
                  double* R_out, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): rt_step with
   the same arguments, semantics and results, whose step scratch (the
   half-step intensity, the lazy interaction maps, the half-step temperature,
   and in curved space the angular divergence and the MAPR slopes) lives in a
   static device array of 64 MiB per device instead of context allocations.
   The call allocates nothing and records no kernel timing events; the tile
   launch order of the stage kernels is the context's cached one when it was
   built by an earlier rt_step call, else the natural order (same results).
   Every call on one device shares that array and leaves it holding its last
   contents: calls that overlap on one device (two streams, two threads, two
   contexts) race and must be serialised by the caller.  Errors: RT_E_ARG as
   rt_step, and when the grid needs more than 64 MiB of step scratch
   (about Nc * (Ns * elem + 56) bytes flat, plus Ns * Nc * elem curved and
   2 Ns * Nc * elem more with MAPR; with ng frequency bins about
   Nc * (ng (Ns * elem + 40) + 8)); RT_E_STATE when the array's device address
   could not be resolved at rt_init_grid. */
rt_status rt_step_noalloc(rt_ctx* ctx, void* I, double* T, double dt, int nsteps, double* G_out,
                          double* R_out, hipStream_t stream);

/* Moments (Eq. R): R[k][c] = sum_s w_s n^a n^b I[s][c] for the 10 pairs
   (a,b) = 00,01,02,03,11,12,13,22,23,33 (n^0 = 1), accumulated in FP64.
   frame RT_COORD returns e^mu_a e^nu_b R^(ab) instead (identity when flat;
   coordinate indices (t, x1, x2, x3) in the same storage order).
   J optional [Nc]: R-hat^00 / (4 pi). */
rt_status rt_moments(rt_ctx* ctx, const void* I, double* R, double* J, int frame,
                     hipStream_t stream);

/* Adjoint of one rt_step step (nsteps = 1) for the FIXED_EMISSIVITY model
   (temperature-independent opacities), flat metric, fluid at rest (other
   configurations return RT_E_ARG): given I^n and the loss gradient
   gI_np1 = dL/dI^(n+1), writes gI_n = dL/dI^n (may alias gI_np1) and ADDS
   dL/dkappa_a and dL/dj of this step into g_kappa_a, g_j ([Nc] each, either
   may be NULL).  T_n is read only. */
rt_status rt_step_adjoint(rt_ctx* ctx, const void* I_n, const double* T_n, double dt,
                          const void* gI_np1, void* gI_n, double* g_kappa_a, double* g_j,
                          hipStream_t stream);

/* Adjoint of one rt_step step (nsteps = 1) for the BREMS model (Method 2,
   Eq. implicit_T; temperature-dependent opacities), flat metric, fluid at
   rest (other configurations return RT_E_ARG).  Given I^n, T^n and the loss
   gradients gI_np1 = dL/dI^(n+1) and gT_np1 = dL/dT^(n+1) ([Nc]; NULL: 0),
   writes gI_n = dL/dI^n (may alias gI_np1) and gT_n = dL/dT^n ([Nc]; may
   alias neither T_n nor gT_np1), and ADDS dL/dkappa_a of this step into
   g_kappa_a ([Nc], may be NULL; kappa_a being the per-cell factor of the
   bremsstrahlung opacity, 1 where the context has none).  The temperature
   solve is differentiated by the implicit-function theorem; T^n enters
   through both stages' energy balances and stage 1's opacities, the
   half-step temperature through stage 2's opacities and optical depths. */
rt_status rt_step_adjoint_thermal(rt_ctx* ctx, const void* I_n, const double* T_n, double dt,
                                  const void* gI_np1, const double* gT_np1, void* gI_n, double* gT_n,
                                  double* g_kappa_a, hipStream_t stream);

/* Debug checking: flags bit 0 -> after each rt_step, synchronise the stream,
   count cells without a valid temperature root (RT_W_NEWTON) and check
   intensities/temperatures for non-finite values (RT_E_NONFINITE). */
rt_status rt_set_debug(rt_ctx* ctx, int flags);

/* Kernel timing: with bit 1 of rt_set_debug's flags set, HIP events bracket
   every kernel launch on its stream.  rt_kernel_times waits for those events
   and returns, for each kernel kind k < RT_NKERNELS, the number of launches
   (counts[k]) and their summed duration in milliseconds (ms[k]) since the
   previous call, then starts a new tally.  Either output may be NULL. */
enum { RT_K_STAGE1 = 0, RT_K_STAGE2, RT_K_MATERIALIZE, RT_K_MOMENTS, RT_K_ADJOINT,
       RT_K_ANGULAR /* curved: angular flux divergence before each stage */,
       RT_K_MG_SOLVE /* frequency bins: temperature solve and per-bin maps of each stage */,
       RT_NKERNELS };
rt_status rt_kernel_times(rt_ctx* ctx, int* counts, double* ms);

/* Number of cells whose interaction found no valid temperature root (they
   kept their pre-interaction state), counted by every rt_step and
   rt_step_noalloc since the previous call of this function; synchronises the
   device. */
rt_status rt_newton_failures(rt_ctx* ctx, long long* count);

void rt_destroy(rt_ctx* ctx);

/* Message of the last non-OK status on this thread ("" if none). */
const char* rt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RT_H */
