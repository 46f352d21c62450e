/*
 * vbrdf — polarized subsurface BRDF of flat homogeneous particulate layers on MI355X (gfx950).
 *
 * Discrete-ordinate solution of the vector radiative transfer equation (Collin & Pattanaik,
 * "GPU accelerated computation of Polarized Subsurface BRDF for Flat Particulate Layers",
 * Sec. 2-3): the phase matrix and the radiance are split into Fourier orders (Sec. 2.B, eq. 6-15),
 * each order is solved independently through the half-size homogeneous eigenproblem
 * (Sec. 3.A, eq. 40-45) and the black-base boundary conditions (Sec. 3.C, eq. 49-56), for all
 * incident Gauss-node directions at once, and the orders are summed into the BRDF Mueller matrix
 * (Sec. 2.D, eq. 1, 12 and 39).
 *
 * Conventions shared by every entry point
 *   - Layer: optical thickness tau0 > 0, single-scattering albedo 0 < omega <= 1 (clamped to
 *     1 - 1e-12 internally), expansion coefficients coef[6][L] with rows
 *     (alpha1, alpha2, alpha3, alpha4, beta1, beta2), l = 0..L-1, alpha1_0 = 1. The scattering
 *     matrix is F = [[a1,b1,0,0],[b1,a2,0,0],[0,0,a3,b2],[0,0,-b2,a4]] with a1 = sum alpha1_l
 *     d^l_00, a4 = sum alpha4_l d^l_00, a2 +- a3 = sum (alpha2 +- alpha3)_l d^l_{2,+-2},
 *     b1 = -sum beta1_l d^l_02, b2 = -sum beta2_l d^l_02 (Wigner d-functions of cos Theta).
 *   - Zenith grid: N-point Gauss-Legendre on [0, 1] per hemisphere (eq. 15), mu ascending.
 *     Incident and outgoing zenith directions are these nodes.
 *   - Azimuth grid: dphi_k = 2 pi k / n_dphi, the difference (outgoing - incident) azimuth.
 *   - Geometry: tau grows downward, mu > 0 propagates downward; incidence (mu_q, phi0),
 *     reflection towards (-mu_i, phi). F_r is referred to the horizontal irradiance mu_q I0.
 *   - F_r layout per layer: [N_out = i][N_in = q][n_dphi = k][4 = r][4 = p], Stokes (I,Q,U,V).
 *     Layers are packed back to back in the order of the plan.
 *   - Stacks and bases: by default every layer lies alone over a black base. A plan may instead
 *     put layers on top of one another (vbrdf_plan_desc.below) and give the bottom of each stack
 *     a reflecting base (vbrdf_plan_desc.base); a layer's F_r is then the BRDF of its sub-stack,
 *     from that layer down to the base.
 *
 * Memory ownership: every pointer passed to these functions stays owned by the caller. Device
 * pointers must stay valid until the enqueued work on the given stream has completed. The plan
 * owns its device workspace (released by vbrdf_plan_destroy).
 *
 * Errors: functions return a vbrdf_status. A negative value is an error; vbrdf_last_error()
 * returns a message for the calling thread's last failed call.
 */
#ifndef VBRDF_H
#define VBRDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VBRDF_ABI_VERSION 3

typedef int32_t vbrdf_status;
#define VBRDF_OK 0
#define VBRDF_E_INVALID (-1)     /* bad pointer, shape or value */
#define VBRDF_E_UNSUPPORTED (-2) /* valid request this library does not implement */
#define VBRDF_E_NOMEM (-3)       /* workspace above the cap, or device allocation failed */
#define VBRDF_E_DEVICE (-4)      /* HIP runtime error (message kept in vbrdf_last_error) */
#define VBRDF_E_NUMERIC (-5)     /* eigen iteration did not converge, zero pivot, NaN/Inf */
#define VBRDF_E_NONCONVERGED (-6) /* FP32 refinement stalled and the FP64 fallback is disabled */

/* Arithmetic of the per-order solves. */
#define VBRDF_PRECISION_FP64 0
/* Boundary factorisations and right divisions in FP32 on the matrix cores, recovered by iterative
 * refinement against FP64 residuals (eigen-decomposition and products stay FP64). */
#define VBRDF_PRECISION_FP32_REFINED 1

/* Plan flags. */
#define VBRDF_FLAG_STAGE_TIMING 1 /* record a hipEvent between the stages of every solve */
/* Capture the launch sequence of vbrdf_solve into a hipGraph on first use and replay it; the graph
 * is captured again whenever the device pointers or the stream of a call differ from the previous
 * call's. Needs a non-default stream; cannot be combined with VBRDF_FLAG_STAGE_TIMING. */
#define VBRDF_FLAG_GRAPH 2
/* Keep the per-order diffuse-plus-direct transmission at the base (the downward field at tau0 for
 * the same unit stream inputs, direct stream included) for vbrdf_plan_inspect. */
#define VBRDF_FLAG_EMIT_TRANSMISSION 4
/* Keep what the adjoint needs (copies of E~ and F~ per order, the layer status) so that
 * vbrdf_backward can follow vbrdf_solve; adds 8 (4N)^2 doubles of workspace per order. */
#define VBRDF_FLAG_SAVE_FOR_BACKWARD 8
/* FP32_REFINED only: report VBRDF_E_NONCONVERGED for a layer whose refinement stalls instead of
 * redoing its boundary solve in FP64. */
#define VBRDF_FLAG_DISABLE_FP64_FALLBACK 16

/* Reflecting base under the bottom layer of every stack (Sec. 2.C, base condition; Sec. 3.C,
 * "Base Reflection", eq. 57-66). The base data are passed to vbrdf_solve_base. */
#define VBRDF_BASE_BLACK 0      /* nothing is reflected (no base data) */
#define VBRDF_BASE_LAMBERTIAN 1 /* ideal depolarising Lambertian base of albedo rho (R_00 = 2 rho,
                                   eq. 66): one double per layer, read for bottom layers only */
#define VBRDF_BASE_MUELLER 2    /* general per-order Mueller base: for every bottom layer (in plan
                                   order) M blocks of (4N)^2 doubles, Rb^m[(i,r)][(j,p)] = Stokes r of
                                   the upward radiance on node i per unit Stokes p of the downward
                                   radiance on node j in order m, in the per-order representation of
                                   the phase matrix (cos part on the IQ-IQ and UV-UV blocks, sin part
                                   on the cross blocks); the base condition is
                                   I_up(i) = sum_j alpha_j mu_j Rb^m(i, j) I_down(j) (eq. 58). */

/* Largest supported quadrature order per hemisphere (Stokes system size 4N = 512). */
#define VBRDF_MAX_N 128

typedef struct vbrdf_plan vbrdf_plan;

typedef struct vbrdf_plan_desc {
  int32_t abi_version;       /* must equal VBRDF_ABI_VERSION */
  int32_t n_layers;          /* >= 1 */
  const int32_t* N;          /* host [n_layers]: nodes per hemisphere, 1..VBRDF_MAX_N */
  const int32_t* L;          /* host [n_layers]: number of expansion coefficients, >= 1 */
  const int32_t* M;          /* host [n_layers]: Fourier orders m = 0..M-1, 1 <= M <= L */
  const int32_t* n_dphi;     /* host [n_layers]: azimuth samples, >= 1 */
  int32_t precision;         /* VBRDF_PRECISION_FP64 or VBRDF_PRECISION_FP32_REFINED */
  int32_t flags;             /* OR of VBRDF_FLAG_* (STAGE_TIMING and GRAPH exclude each other) */
  uint64_t workspace_cap_bytes; /* 0 = no cap; otherwise plan creation fails with NOMEM above it */
  /* Optional caller-owned device workspace (256-byte aligned, at least vbrdf_workspace_query bytes)
   * that the plan borrows instead of allocating its own; NULL = the plan allocates. It must stay
   * valid until the plan is destroyed. */
  void* workspace;
  uint64_t workspace_bytes;
  /* Largest number of QR sweeps per eigenproblem before the layer is reported NUMERIC; 0 = the
   * default of 60 sweeps per row. A small cap forces the NUMERIC status (for tests). */
  int32_t qr_sweep_cap;
  /* FP32_REFINED: correction steps of the boundary solve after the first FP32 solve; 0 = the
   * default (2), -1 = none (the unrefined FP32 solve then fails the convergence test: for tests of
   * the fallback and of NONCONVERGED). Must be 0 for FP64. */
  int32_t refine_steps;
  /* Layer stacks (Sec. 2.C: one homogeneous solution per layer, radiance continuous across each
   * interface). NULL = every layer alone. Otherwise host [n_layers]: below[l] is the index of the
   * layer directly beneath layer l, or -1 when layer l is the bottom of its stack. Each layer lies
   * on at most one other, chains end (no cycles), at most 64 layers per stack, and the layers of a
   * stack share N and M. Layer l's F_r is the BRDF of the stack from l down to the base. */
  const int32_t* below;
  /* VBRDF_BASE_* under the bottom layer of every stack (also for a layer alone). Plans with stacks
   * or a non-black base accept neither VBRDF_FLAG_SAVE_FOR_BACKWARD nor
   * VBRDF_FLAG_EMIT_TRANSMISSION. */
  int32_t base;
  /* Off-node incidence (Sec. 2.C particular solution, eq. 28-33, in its half-size form of Sec. 3.B,
   * eq. 46-48): n_mu0 incident cosines (host array mu0[n_mu0], each in (0, 1], at most 64 and at
   * most N of every layer), for which vbrdf_solve_ex also writes the BRDF towards the Gauss nodes.
   * 0 = none. Not with stacks, a reflecting base or VBRDF_FLAG_SAVE_FOR_BACKWARD. */
  int32_t n_mu0;
  const double* mu0;
  /* Extra outgoing directions of the beams (Sec. 2.C "Reconstruction", eq. 36-38): n_mu_out cosines
   * (host array mu_out[n_mu_out], each in (0, 1], at most 64 and at most N of every layer; needs
   * n_mu0 > 0) towards which vbrdf_solve_ex also writes the beams' BRDF, by integrating the
   * source function of the per-order solution along each direction in closed form. 0 = none. */
  int32_t n_mu_out;
  const double* mu_out;
} vbrdf_plan_desc;

/* ABI version of the loaded library (VBRDF_ABI_VERSION). */
int32_t vbrdf_abi_version(void);

/* Message for the calling thread's last failed call ("" if none). Valid until the next call
 * into this library on the same thread. */
const char* vbrdf_last_error(void);

/* Double-Gauss nodes of eq. 15: mu[i] = (1 + x_i)/2 and alpha[i] = w_i/2 for the N-point
 * Gauss-Legendre rule (x_i, w_i) on [-1, 1]; ascending, sum(alpha) = 1. Host only: mu and alpha
 * are caller-owned host arrays of N doubles. Returns INVALID for N < 1 or null pointers. */
vbrdf_status vbrdf_gauss_nodes(int32_t N, double* mu, double* alpha);

/* Create a plan specialised to the layer shapes in *desc (Sec. 3: one homogeneous solution per
 * Fourier order, shared by all incident directions). Allocates the device workspace on the
 * current HIP device. On success *out receives the plan; on failure *out is set to NULL.
 * Errors: INVALID (bad desc), UNSUPPORTED (N > VBRDF_MAX_N, M > 512, n_dphi > 1024, unknown
 * precision or flags),
 * NOMEM (cap exceeded or allocation failed), DEVICE. */
vbrdf_status vbrdf_plan_create(const vbrdf_plan_desc* desc, vbrdf_plan** out);

/* Device workspace, in bytes, that a plan for *desc needs (the size a caller-owned workspace must
 * have). Host only. Errors as for vbrdf_plan_create's descriptor checks. */
vbrdf_status vbrdf_workspace_query(const vbrdf_plan_desc* desc, uint64_t* bytes);

/* Release the plan and its workspace. Waits for nothing: the caller must make sure no enqueued
 * solve still uses it. NULL is accepted. */
vbrdf_status vbrdf_plan_destroy(vbrdf_plan* plan);

/* Bytes of F_r the plan writes (sum over layers of N*N*n_dphi*16 doubles). */
size_t vbrdf_plan_output_bytes(const vbrdf_plan* plan);

/* Device workspace held by the plan, in bytes. */
size_t vbrdf_plan_workspace_bytes(const vbrdf_plan* plan);

/* Enqueue the BRDF of every layer on `stream` (a hipStream_t; NULL = default stream).
 *   tau[n_layers], omega[n_layers]       device doubles
 *   coef                                 device doubles, per layer [6][L_l] packed back to back
 *   F_r                                  device doubles, per layer [N][N][n_dphi][4][4] packed
 *   layer_status[n_layers]               device int32, written with VBRDF_OK or a negative code
 * Steps per (layer, order): Legendre matrices and assembly of E and F (eq. 9-11, 41-42), the
 * product FE (eq. 43), its eigen-decomposition (eq. 43-45), the mode vectors (eq. 45), the
 * black-base boundary solve for all 4N incident (node, Stokes) pairs (eq. 49-56), the emergent
 * response at tau = 0, then the Fourier synthesis of F_r (eq. 12, 39).
 * Returns after enqueueing. Host-detectable errors (null pointers, null plan) return INVALID
 * without enqueueing. Data-dependent problems are reported per layer in layer_status (INVALID:
 * tau0 <= 0, omega outside (0,1], alpha1_0 != 1, non-finite input; NUMERIC: eigen iteration or
 * boundary solve failed); such a layer's F_r is filled with NaN. */
vbrdf_status vbrdf_solve(vbrdf_plan* plan, const double* tau, const double* omega, const double* coef,
                         double* F_r, int32_t* layer_status, void* stream);

/* vbrdf_solve for plans with stacks or a reflecting base. Every layer is first solved over a black
 * base as above; the stacks are then combined per order from the bottom up: with R~, T~ a layer's
 * reflection and transmission operators on radiance at the nodes (upward fields stored mirrored,
 * Stokes U and V negated) and X~ the reflection of what lies beneath it (the sub-stack, or the base
 * as the matrix of eq. 58 in the same storage),
 *     R~_stack = R~ + T~ (I - X~ R~)^-1 (X~ T~),
 * which is the solution of the full boundary system with interface continuity and the base
 * condition (the two agree exactly; the combined system is never formed).
 *   base      device doubles as described for the plan's VBRDF_BASE_* (NULL for a black base):
 *             LAMBERTIAN: rho[n_layers], 0 <= rho <= 1; MUELLER: vbrdf_plan_base_bytes() bytes
 * Other arguments and the per-layer status as for vbrdf_solve. A layer whose sub-stack contains a
 * failed layer gets that layer's status; an invalid rho or a non-finite Mueller entry gives INVALID
 * for the stack's bottom layer (and so for the layers above it); a singular adding system gives
 * NUMERIC. Errors: INVALID (null pointers; base NULL for a non-black base), as vbrdf_solve. */
vbrdf_status vbrdf_solve_base(vbrdf_plan* plan, const double* tau, const double* omega, const double* coef,
                              const double* base, double* F_r, int32_t* layer_status, void* stream);

/* Bytes of base data vbrdf_solve_base reads for this plan (0 for a black base). */
size_t vbrdf_plan_base_bytes(const vbrdf_plan* plan);

/* The general solve: vbrdf_solve_base plus, for a plan with off-node beams (n_mu0 > 0), the BRDF
 * of each beam towards the Gauss nodes:
 *   F_beam    device doubles, per layer [N + n_mu_out = i][n_mu0 = j][n_dphi = k][4 = r][4 = p],
 *             packed back to back (vbrdf_plan_beam_bytes() bytes): F_r for incidence at mu0_j,
 *             outgoing direction i (the Gauss nodes for i < N, then mu_out[i - N]), azimuth
 *             difference 2 pi k / n_dphi, referred to the horizontal irradiance mu0_j I0 as the
 *             node table.
 * Per order the particular solution of the beam's source is found through the eigen-decomposition
 * of the half-size problem, (F E - mu0^-2) G = (F X+ + X- / mu0) M^-1 (eq. 47) solved as
 * U (Lambda - mu0^-2)^-1 U^-1, and the homogeneous part that cancels its incoming diffuse light at
 * the top and the black base comes from the layer's boundary operators. A beam within a relative
 * 1e-12 of a resonance (mu0^-2 equal to an eigenvalue of FE, which in weakly scattering orders
 * happens at the Gauss nodes, where the node table is exact) makes the layer NUMERIC. Towards an
 * extra outgoing direction the radiance is the source function of eq. 38 (the per-order field at
 * the nodes, a sum of exponentials in depth, scattered towards -mu, plus the beam's own single
 * scattering) integrated along the direction in closed form (eq. 37, with the 1/mu its printed form
 * lacks); at a Gauss node this is the discrete-ordinate value itself.
 * base and the other arguments as for vbrdf_solve_base (base NULL for a black base). vbrdf_solve
 * on a plan with beams computes the node table only. Errors: INVALID (null pointers; F_beam NULL
 * for a plan with beams), as vbrdf_solve. */
vbrdf_status vbrdf_solve_ex(vbrdf_plan* plan, const double* tau, const double* omega, const double* coef,
                            const double* base, double* F_r, double* F_beam, int32_t* layer_status, void* stream);

/* Bytes of F_beam a plan writes (0 without beams). */
size_t vbrdf_plan_beam_bytes(const vbrdf_plan* plan);

/* Inspection of the last solve's per-order intermediates for one (layer, order), copied
 * synchronously (after waiting for `stream`) into caller-owned host arrays:
 *   R_out[4N*4N]   emergent response R^m[(i,r),(q,p)]: Stokes r of the upward radiance at the
 *                  top on node i for a unit Stokes e_p entering on node q (order m), may be NULL
 *   lam_re[4N], lam_im[4N]   eigenvalues of FE (1/nu^2), may be NULL
 *   T_out[4N*4N]   transmission T^m[(i,r),(q,p)]: Stokes r of the downward radiance at the base on
 *                  node i for the same inputs, the attenuated incident stream included (plan created
 *                  with VBRDF_FLAG_EMIT_TRANSMISSION; INVALID otherwise), may be NULL
 * Returns INVALID for an out-of-range layer or order. */
vbrdf_status vbrdf_plan_inspect(const vbrdf_plan* plan, int32_t layer, int32_t m, double* R_out,
                                double* lam_re, double* lam_im, double* T_out, void* stream);

/* Per-stage device times (milliseconds) of the solves enqueued on a plan created with
 * VBRDF_FLAG_STAGE_TIMING since the previous call (at most the first 256 of them), averaged per
 * stage. hipEvents are recorded on each solve's stream between its kernel launches, so the times
 * are those of the stream the kernels ran on. Waits for the last recorded solve, then starts a new
 * averaging window. Writes min(cap, count) floats to ms_out (host array, may be NULL) and returns
 * the number of stages, or a negative status (INVALID without the flag or with no recorded solve).
 * Stage names: vbrdf_stage_name. */
int32_t vbrdf_plan_stage_times(vbrdf_plan* plan, float* ms_out, int32_t cap);

/* Name of stage i (static string), or NULL when out of range. */
const char* vbrdf_stage_name(int32_t i);

/* Gradients of a scalar loss with respect to the layer parameters, given its gradient dF_r with
 * respect to F_r (same layout as F_r): reverse mode through the synthesis (eq. 12, 39), the
 * boundary solve (eq. 49-56), the matrix functions of the eigen-decomposition (eq. 43-45, by the
 * Daleckii-Krein form of their derivative) and the assembly (eq. 41-42, 9). The plan must have
 * been created with VBRDF_FLAG_SAVE_FOR_BACKWARD, and the last vbrdf_solve on it must have had the
 * same tau, omega and coef (its per-order state is reused; it must not be overwritten by another
 * solve before this call's work has run). Device pointers, enqueued on `stream`:
 *   tau, omega, coef        the forward's inputs
 *   dF_r                    dLoss / dF_r, doubles in the F_r layout
 *   dtau[n_layers], domega[n_layers], dcoef (layout of coef)   outputs, overwritten (not added to)
 * A layer whose forward failed gets NaN gradients. d/d omega is taken at the clamped albedo
 * (omega <= 1 - 1e-12); d/d alpha1_0 is reported although alpha1_0 is fixed at 1 by the
 * normalisation. Errors: INVALID (null pointer, plan without the flag, no forward solve yet),
 * DEVICE. */
vbrdf_status vbrdf_backward(vbrdf_plan* plan, const double* tau, const double* omega, const double* coef,
                            const double* dF_r, double* dtau, double* domega, double* dcoef, void* stream);

/* Scheduling and tile choices of a plan: how the eigensolver's workgroups take the (layer, order)
 * problems, and the rows per tile of the FP64 right divisions. Results do not depend on them (every
 * problem is solved by the same arithmetic); only the time does. */
#define VBRDF_EIGEN_PLAN_ORDER 0    /* one workgroup per problem, in plan order (default) */
#define VBRDF_EIGEN_LONGEST_FIRST 1 /* one workgroup per problem, largest systems first */
#define VBRDF_EIGEN_PERSISTENT 2    /* one workgroup per compute unit taking problems from a queue,
                                       largest first, until none is left */
typedef struct vbrdf_tuning {
  int32_t eigen_schedule; /* VBRDF_EIGEN_* */
  int32_t trsm_rows;      /* 4, 8 or 16 (default) right-hand-side rows per right-division tile; 4 and 8
                             split each dot product over the lanes of one wave, 16 runs the blocked
                             solve on the matrix cores */
} vbrdf_tuning;

/* Current choices of the plan (host call). */
vbrdf_status vbrdf_plan_get_tuning(const vbrdf_plan* plan, vbrdf_tuning* out);

/* Set the choices (INVALID for values outside the lists above). A captured graph is recaptured at
 * the next solve. */
vbrdf_status vbrdf_plan_set_tuning(vbrdf_plan* plan, const vbrdf_tuning* tuning);

/* Autotuner: enqueues solves of the given inputs with each candidate schedule and tile shape,
 * times the eigensolver stage and the right-division stage with hipEvents on `stream` (waiting
 * for them), and keeps the fastest choice of each. Synchronous. Afterwards F_r and layer_status
 * hold the result of one more solve with the chosen configuration. `chosen` (host, may be NULL) receives the choice.
 * Errors as for vbrdf_solve, plus DEVICE. */
vbrdf_status vbrdf_plan_autotune(vbrdf_plan* plan, const double* tau, const double* omega, const double* coef,
                                 double* F_r, int32_t* layer_status, void* stream, vbrdf_tuning* chosen);

/* Stokes radiances of eq. 1: for a beam of Stokes vector I0 (host array of 4) incident on node q
 * at azimuth phi0 (radians), I_out[i][k][r] = mu_q sum_p F_r(i <- q, phi_k - phi0)[r][p] I0[p],
 * the upward radiance at the top towards (-mu_i, phi_k = 2 pi k / n_dphi). When phi0 lies on the
 * azimuth grid (a multiple of 2 pi / n_dphi within 1e-12 rad) the entries are read from the table
 * F_r (device pointer, as written by vbrdf_solve); otherwise the Fourier series of eq. 12 is summed
 * exactly at phi_k - phi0 from the per-order responses of the plan's last solve (valid until the
 * next vbrdf_solve on this plan; F_r is then not read). I_out is a device pointer of N*n_dphi*4
 * doubles. Enqueued on `stream`. */
vbrdf_status vbrdf_radiance(const vbrdf_plan* plan, const double* F_r, int32_t layer, int32_t q, double phi0,
                            const double I0[4], double* I_out, void* stream);

/* Allocation-free solve of ONE layer, for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc). The same computation as
 * a one-layer plan's vbrdf_solve, with the plan's tables and workspace replaced by a static device
 * array of VBRDF_NOALLOC_SCRATCH_BYTES held by the library on every GPU it runs on until the
 * process ends. Allocates nothing and copies nothing from the host: the tables, quadrature nodes
 * included, are written by a set-up kernel on `stream`.
 *   N, L, M, n_dphi          the layer's shape, as in vbrdf_plan_desc
 *   tau, omega               device pointers to one double each
 *   coef                     device doubles [6][L]
 *   F_r                      device doubles [N][N][n_dphi][4][4]
 *   layer_status             device int32 [1], written with VBRDF_OK or a negative code
 * Enqueued on `stream`; returns after enqueueing. Errors: INVALID (null pointer, bad shape),
 * UNSUPPORTED (N > VBRDF_MAX_N, M > 512, n_dphi > 1024), NOMEM (the layer's workspace, about
 * 8 M (4N)^2 doubles, does not fit the static array: e.g. N = 32 fits up to M = 74, N = 64 up to
 * M = 19), DEVICE. Every call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (other streams or threads) race and must be serialised by the caller. Data-dependent problems
 * are reported in layer_status exactly as by vbrdf_solve. */
#define VBRDF_NOALLOC_SCRATCH_BYTES (80ull << 20)
vbrdf_status vbrdf_solve_noalloc(int32_t N, int32_t L, int32_t M, int32_t n_dphi, const double* tau,
                                 const double* omega, const double* coef, double* F_r, int32_t* layer_status,
                                 void* stream);

#ifdef __cplusplus
}
#endif

#endif /* VBRDF_H */
