// Internal descriptors shared by the host planner and the gfx950 kernels.
//
// A work item is one (layer, Fourier order m) pair. Every per-order step of the solve runs on one
// item independently (Sec. 3: the homogeneous solution is computed once per order and serves all
// incident directions), so kernels are launched over the item table and index their workspace by
// the item's offset.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/vbrdf.h"

namespace vbrdf {

constexpr int kMaxN = 128;          // nodes per hemisphere
constexpr int kMaxn = 4 * kMaxN;     // Stokes system size 4N
constexpr int kEigenThreads = 512;  // k_eigen workgroup: 8 waves
constexpr int kLdsMaxn = 128;        // largest system kept whole in LDS (128 x 129 doubles)
constexpr double kOmegaMax = 1.0 - 1e-12;

// Buffers of n*n doubles inside an item's workspace block.
enum Buf : int {
  kBufE = 0,   // E~ = M^-1 (I - omega/2 S+ W); later the emergent response R^m
  kBufF = 1,   // F~ = M^-1 (I - omega/2 S- W)
  kBufG = 2,   // G = F~ E~ (eigen input; reduced in place when n > kLdsMaxn); then U' = Z X; later V = E~ U
  kBufZ = 3,   // Schur vectors (column-major); later S' = U + V D_s
  kBufX = 4,   // eigenvectors of the quasi-triangular factor; later T' = U + V D_t
  kBufU = 5,   // eigenvectors U of G (columns)
  kBufYS = 6,  // Householder vectors of the Hessenberg reduction; later U S'^-1
  kBufYT = 7,  // U T'^-1
  kNumBuf = 8
};

struct Layer {
  int32_t N, L, M, n_dphi;
  int64_t coef_off;  // doubles, into the caller's packed coefficient array
  int64_t out_off;   // doubles, into the caller's packed F_r array
  int64_t quad_off;  // doubles, into the plan's quadrature table (mu[N] then alpha[N])
  int64_t item0;     // index of this layer's m = 0 item
  int64_t beam_off;  // doubles, into the caller's packed off-node beam output (plans with beams)
};

struct Item {
  int32_t layer, m, N, L;
  int32_t n;         // 4N
  int32_t pad;
  int64_t ws;        // doubles, start of this item's workspace block
};

// Per-item extras after the kNumBuf matrices (n doubles each): lam_re, lam_im, balancing factors,
// Schur block sizes (int), two spare, then d_s (re, im) and d_t (re, im) of the boundary solve;
// followed by the Legendre table [L][N][3].
__host__ __device__ inline int64_t extras_off(int n) { return (int64_t)kNumBuf * n * n; }
__host__ __device__ inline int64_t leg_off(int n) { return extras_off(n) + 10 * (int64_t)n; }
__host__ __device__ inline int64_t item_doubles(int n, int N, int L) {
  return leg_off(n) + (int64_t)L * N * 3;
}

// Per-item block: the kNumBuf matrices, the extras, the Legendre table, then (plans that keep
// the state for the adjoint) kNumBwdBuf more n x n matrices. Buffer index b < kNumBuf addresses
// the first group, kNumBuf <= b < kNumBuf + kNumBwdBuf the second.
constexpr int kNumBwdBuf = 8;
enum BwdBuf : int {
  kBufSE = kNumBuf,  // E~ kept from the forward
  kBufSF,            // F~ kept from the forward
  kBufW,             // U^-T
  kBufT1, kBufT2, kBufT3, kBufT4, kBufT5  // adjoint temporaries
};
__host__ __device__ inline int64_t bwd_off(int n, int N, int L) { return (item_doubles(n, N, L) + 31) / 32 * 32; }
__host__ __device__ inline int64_t block_doubles_of(int n, int N, int L, bool save) {
  return bwd_off(n, N, L) + (save ? (int64_t)kNumBwdBuf * n * n : 0);
}
// Off-node incidence ("beams", a plan option exclusive with the adjoint state): eight n x n
// matrices in the second group's slots, then the Legendre tables at the incident cosines
// [L][n_mu0][3] and at the extra outgoing cosines [L][n_mu_out][3]. The beams of an order occupy
// the first 4 n_mu0 columns (column 4 j + p: unit Stokes p incident at mu0_j); the extra outgoing
// directions the first 4 n_mu_out rows of the reconstruction buffers (row 4 o + r).
constexpr int kNumBeamBuf = 8;
enum BeamBuf : int { kBufB0 = kNumBuf, kBufB1, kBufB2, kBufB3, kBufB4, kBufB5, kBufB6, kBufB7 };
static_assert(kNumBeamBuf <= kNumBwdBuf, "beam buffers use the adjoint's slots");
__host__ __device__ inline int64_t beam_leg_off(int n, int N, int L) {
  return bwd_off(n, N, L) + (int64_t)kNumBeamBuf * n * n;
}
__host__ __device__ inline int64_t beam_out_leg_off(int n, int N, int L, int n_mu0) {
  return beam_leg_off(n, N, L) + (int64_t)L * n_mu0 * 3;
}
__host__ __device__ inline int64_t block_doubles_beams(int n, int N, int L, int n_mu0, int n_mu_out) {
  return (beam_out_leg_off(n, N, L, n_mu0) + (int64_t)L * n_mu_out * 3 + 31) / 32 * 32;
}
constexpr int kMaxBeams = 64;  // incident directions per plan

struct BeamTask {  // one workgroup of the beam synthesis: (layer, outgoing node i, incident mu0_j)
  int32_t layer, i, j, pad;
};

struct SynthTask {
  int32_t layer, i, q, pad;
};

constexpr int kSynthMaxM = 512;     // Fourier orders per layer
constexpr int kSynthMaxPhi = 1024;  // azimuth samples per layer

__host__ __device__ inline double* buf_ptr(double* ws, const Item& it, int b) {
  const int64_t nn = (int64_t)it.n * it.n;
  return ws + it.ws + (b < kNumBuf ? b * nn : bwd_off(it.n, it.N, it.L) + (b - kNumBuf) * nn);
}

// ---- kernels (one translation unit each)
__global__ void k_validate(const Layer* layers, int n_layers, const double* tau, const double* omega,
                           const double* coef, int32_t* status);
constexpr int kLegThreads = 3 * 128;  // k_legendre: three recurrences x up to 128 nodes
__global__ void k_legendre(const Item* items, const Layer* layers, const double* quad, double* ws,
                           const int32_t* status);
__global__ void k_assemble(const Item* items, const Layer* layers, const double* quad, const double* omega,
                           const double* coef, double* ws, const int32_t* status);
// C = op(A) op(B) for buffers of one item; mode: OR of the bits below (C written transposed,
// negated, or added to the existing C)
constexpr int kGemmTransA = 1, kGemmTransB = 2, kGemmTransC = 4, kGemmNegate = 8, kGemmAccumulate = 16;
__global__ void k_gemm(const Item* items, double* ws, int bufA, int bufB, int bufC, int mode, const int32_t* status);
// sweep_cap: largest number of QR sweeps per problem (above it the layer is NUMERIC), 0 = default.
// order: item permutation (workgroup b solves items[order[b]]), or null for the plan order. The
// persistent form takes positions of `order` from the counter `queue` (reset to 0 before the
// launch) until n_items are taken.
constexpr int kEigenPlanOrder = 0, kEigenLongestFirst = 1, kEigenPersistent = 2;
// k_eigen and k_eigen_persistent solve the problems of at most kLdsMaxn rows (H in LDS);
// k_eigen_big the larger ones, over the first n_big positions of the longest-first order (which
// are exactly those), whatever the schedule.
__global__ void k_eigen(const Item* items, double* ws, int32_t* status, int sweep_cap, const int32_t* order);
__global__ void k_eigen_big(const Item* items, double* ws, int32_t* status, int sweep_cap, const int32_t* order);
__global__ void k_eigen_persistent(const Item* items, double* ws, int32_t* status, int sweep_cap,
                                   const int32_t* order, int32_t* queue, int n_items);
__global__ void k_reset_counter(int32_t* counter);
__global__ void k_vfix(const Item* items, double* ws, int32_t* status);
__global__ void k_colscal(const Item* items, const double* tau, double* ws, int32_t* status);
__global__ void k_bcbuild(const Item* items, double* ws, const int32_t* status);
constexpr int kHqCols = 4;  // columns per k_hqapply wave
// k_hqapply_mfma (16 columns per wave, panels of 16 reflectors on the matrix cores) takes the
// systems of at most kHqMfmaMaxN rows, k_hqapply the larger ones
constexpr int kHqMfmaMaxN = 256;
__global__ void k_hqapply(const Item* items, int n_items, int tiles, double* ws, const int32_t* status);
__global__ void k_hqapply_mfma(const Item* items, int n_items, int tiles, double* ws, const int32_t* status);
// Buffers of the factorisation and right-division kernels per side (blockIdx.y of k_lu, or the
// low digit of the matrix index of k_trsm): LU of src into the transposed factor dst; right
// division y = rhs a^-1 with a's factor in buffer a. The side also selects the pivot and 1 / Uu_kk
// slots of the extras block.
struct LuBufs {
  int32_t src[2], dst[2];
  int32_t only_flagged;  // factor only the sides whose FP32 refinement asked for the FP64 solve
};
struct TrsmBufs {
  int32_t a[2], rhs[2], y[2];
  int32_t sides;         // 1 or 2 matrices per item
  int32_t only_flagged;  // as in LuBufs
};

// State of the FP32-refined boundary solve per item, in the extras block at [3n, 3n + 4) (free
// at that stage): the largest residual entry of each side and of U (non-negative doubles compared
// through their bit patterns by atomicMax), and per side whether the FP64 solve must be redone.
struct BoundaryFlags {
  unsigned long long resmax[2];
  unsigned long long umax;
  int32_t fallback[2];
};
__host__ __device__ inline BoundaryFlags* boundary_flags(double* ex, int n) {
  return reinterpret_cast<BoundaryFlags*>(ex + 3 * (int64_t)n);
}
// Refined-path kernels: FP32 LU of S' and T' (factors as floats in the first half of the k_lu
// output buffers), FP32 right division (set or accumulate), FP64 residual U - Y A rounded to FP32
// into kBufE, and the end-of-refinement check (fallback flag, or NONCONVERGED when the FP64
// fallback is disabled).
constexpr int kLu32LdsMaxn = 192;  // largest n factored in LDS in FP32
__global__ void k_lu32(const Item* items, double* ws, int32_t* status);
__global__ void k_trsm32(const Item* items, int n_items, int tiles, double* ws, int32_t* status, int accumulate);
__global__ void k_resid(const Item* items, double* ws, const int32_t* status);
__global__ void k_bcheck(const Item* items, double* ws, int32_t* status, int no_fallback);
// k_lu runs twice per factorisation: with kLuThreadsLds threads over the systems held in LDS
// (n <= kLdsMaxn) and with kLuThreadsBig over the larger, blocked ones (a thread per row);
// launch_lu issues both (the second only when the plan has such systems).
constexpr int kLuThreadsLds = 1024, kLuThreadsBig = 512;
static_assert(kLuThreadsBig >= kMaxn && kLuThreadsBig % 64 == 0, "a thread per row in the blocked LU");
__global__ void k_lu(const Item* items, double* ws, int32_t* status, LuBufs b);
void launch_lu(dim3 grid, hipStream_t s, const Item* items, double* ws, int32_t* status, int max_n, LuBufs b);
// one kernel per tile shape (rows per tile 4, 8 or 16); launch_trsm picks it
template <int kRows>
__global__ void k_trsm(const Item* items, int n_items, int tiles, double* ws, int32_t* status, TrsmBufs b);
void launch_trsm(int rows, dim3 grid, size_t lds, hipStream_t s, const Item* items, int n_items, int tiles, double* ws,
                 int32_t* status, TrsmBufs b);
// the kernel instances, for attribute queries and settings
const void* trsm_kernel_ptr(int rows);
// Eigenpair refinement of the homogeneous step (between the eigenvector back-transformation and the
// mode vectors): transposed copy, per-column update of the eigenvalues, correction matrix, commit.
__global__ void k_transpose(const Item* items, double* ws, int src, int dst, const int32_t* status);
__global__ void k_refine_lam(const Item* items, double* ws, const int32_t* status);
__global__ void k_refine_close(const Item* items, double* ws, const int32_t* status);
__global__ void k_refine_pairs(const Item* items, double* ws, const int32_t* status);
__global__ void k_refine_delta(const Item* items, double* ws, const int32_t* status);
__global__ void k_refine_commit(const Item* items, double* ws, const int32_t* status);
// right-hand-side rows per right-division tile (one wave, 64 / kTrsmRows lanes per row; the tile takes
// n x (trsm_ldb(n) + 2) doubles of LDS). The FP32 right division and the allocation-free entry point
// use this shape; plans start from kTrsmRowsDefault, the 16-row tile whose products run on the
// matrix cores.
constexpr int kTrsmRows = 8;
constexpr int kTrsmRowsDefault = 16;
// LDS row stride of the right-division tile, in doubles. A 64-bit LDS access is served 16 lanes
// at a time over 32 banks: 8 parts x 2 rows at offsets 18 part + row = 2 part + row (mod 16) meet
// 16 distinct bank pairs. Above n = 128 the tile would then hold so much LDS that fewer tiles fit
// on a CU, which costs more than the conflicts, so those sizes keep the dense stride.
constexpr int kTrsmLdb = 18;
static_assert(kTrsmLdb > kTrsmRows, "the tile row holds kTrsmRows entries");
__host__ __device__ inline int trsm_ldb(int n) { return n <= kLdsMaxn ? kTrsmLdb : kTrsmRows + 1; }
// LDS row stride of the FP64 right-division tile for `rows` rows per tile (4, 8 or 16).
__host__ __device__ inline int trsm_ldb_rows(int n, int rows) { return rows == 8 ? trsm_ldb(n) : rows + 1; }
// Right-division tile geometry for `rows` rows per tile over systems up to max_n.
inline int trsm_tiles_for(int max_n, int rows) { return (max_n + rows - 1) / rows; }
inline size_t trsm_lds_for(int max_n, int rows) {
  // the 16-row tile keeps only itself in LDS (stride 17; the factor is read from the workspace)
  if (rows == 16) return sizeof(double) * (size_t)max_n * 17;
  return sizeof(double) * (size_t)max_n * (trsm_ldb_rows(max_n, rows) + 2);
}

// XCD-aware launch order: workgroups are dealt round-robin to the 8 XCDs (each with its own L2),
// so the `tiles` workgroups that read one matrix get linear ids that agree mod 8. For `groups`
// matrices the grid has xcd_grid(groups, tiles) workgroups; xcd_split recovers (group, tile) of a
// workgroup, group >= groups meaning an idle one.
constexpr int kXcds = 8;
__host__ __device__ inline int xcd_grid(int groups, int tiles) { return (groups + kXcds - 1) / kXcds * kXcds * tiles; }
__host__ __device__ inline void xcd_split(int id, int tiles, int& group, int& tile) {
  const int blk = id / (kXcds * tiles), rem = id % (kXcds * tiles);
  tile = rem / kXcds;
  group = blk * kXcds + rem % kXcds;
}
// R^m into kBufE; with transmission also T^m = (U S'^-1 - U T'^-1) R0 into kBufF. mode
// kResponseBrackets instead writes the unscaled operators R~ = U S'^-1 + U T'^-1 - I (kBufE) and
// T~ = U S'^-1 - U T'^-1 (kBufF) for the stack stage.
constexpr int kResponseTransmission = 1, kResponseBrackets = 2;
__global__ void k_response(const Item* items, const Layer* layers, const double* quad, double* ws,
                           const int32_t* status, int mode);
// ---- layer stacks and reflecting bases (k_stack.hip)
// One adding step per item of a level: the reflection beneath comes from the item below (its
// combined R~ in kBufE, at workspace offset src_ws) or, for src_ws < 0, from the base data at
// base_off (Lambertian: the layer's rho; Mueller: this order's block).
struct StackTask {
  int64_t src_ws;
  int64_t base_off;
  int32_t src_layer;  // the layer beneath (its status is inherited), or -1
  int32_t pad;
};
constexpr int kMaxStackLevels = 64;
__global__ void k_stack_validate(const Layer* layers, const int32_t* below, int base_kind, const double* base,
                                 const int64_t* base_off, int32_t* status);
__global__ void k_stack_status(int n_layers, const int32_t* below, int32_t* status);
__global__ void k_stack_x(const Item* items, const StackTask* tasks, const Layer* layers, const double* quad,
                          int base_kind, const double* base, double* ws, int32_t* status);
__global__ void k_stack_finish(const Item* items, const Layer* layers, const double* quad, double* ws,
                               const int32_t* status);
__global__ void k_synth_mfma(const SynthTask* tasks, const Layer* layers, const Item* items, const double* quad,
                        const double* ws, double* F, const int32_t* status);
// Device tables and launch shape of a solve: the plan's, or those of the allocation-free entry
// point (tables inside its static scratch array).
struct LaunchSet {
  const Layer* layers_d = nullptr;
  const Item* items_d = nullptr;
  const SynthTask* tasks_d = nullptr;
  const double* quad_d = nullptr;  // per layer mu[N] then alpha[N]
  double* ws_d = nullptr;          // per-item workspace blocks
  int n_layers = 0, n_items = 0, n_tasks = 0;
  int max_n = 0, max_N = 0;
  int trsm_rows = kTrsmRowsDefault;  // right-hand-side rows per FP64 right-division tile (4, 8, 16)
  int trsm_tiles = 0;         // row tiles of the FP64 right division (largest item)
  size_t trsm_lds = 0;        // its LDS bytes
  int trsm32_tiles = 0;       // row tiles of the FP32 right division (kTrsmRows rows each)
  int eigen_mode = 0;         // k_eigen scheduling: kEigenPlanOrder / kEigenLongestFirst / kEigenPersistent
  const int32_t* order_d = nullptr;  // items by decreasing size (longest first)
  int32_t* queue_d = nullptr;        // work counter of the persistent eigensolver
  int persist_groups = 256;          // workgroups of the persistent eigensolver (compute units)
  int n_big = 0;                     // items with n > kLdsMaxn (the first n_big positions of order_d)
  int qr_sweep_cap = 0;       // 0 = the eigensolver's default
  bool transmission = false;  // also write the per-order transmission T^m
  int precision = 0;          // VBRDF_PRECISION_*
  bool no_fallback = false;   // FP32-refined: NONCONVERGED instead of the FP64 redo
  int refine_steps = 0;       // FP32-refined: correction steps of the boundary solve
  bool save = false;          // keep the state the adjoint needs (E~, F~ copies, layer status)
  int32_t* status_d = nullptr;  // copy of the last forward's layer status (adjoint plans)
  // layer stacks and bases
  bool stacked = false;                     // below[] given or a reflecting base
  int base_kind = 0;                        // VBRDF_BASE_*
  const int32_t* below_d = nullptr;         // per layer: the layer beneath, or -1
  const int64_t* base_off_d = nullptr;      // per layer: offset of its base data (doubles)
  const Item* stack_items_d = nullptr;      // items that take an adding step, grouped by level
  const StackTask* stack_tasks_d = nullptr; // matching tasks
  int n_levels = 0;
  int lvl_off[kMaxStackLevels + 1] = {};    // level k: stack items [lvl_off[k], lvl_off[k + 1])
  // off-node incidence
  int n_mu0 = 0;                            // incident directions (0: none)
  const double* mu0_d = nullptr;            // their cosines
  int n_mu_out = 0;                         // extra outgoing directions of the beams (0: nodes only)
  const double* mu_out_d = nullptr;         // their cosines
  const BeamTask* btasks_d = nullptr;       // beam synthesis tasks
  int n_btasks = 0;
};
constexpr int kBoundaryRefineSteps = 2;  // FP32-refined boundary solve: correction steps

// Records the calling thread's error message (returned by vbrdf_last_error) and returns code.
int32_t vbrdf_fail(int32_t code, const char* fmt, ...);

// Stages of the launch sequence (events are recorded around and between them when requested).
constexpr int kNumSolveStages = 17;
void enqueue_solve(const LaunchSet& ls, const double* tau, const double* omega, const double* coef,
                   const double* base, double* F_r, double* F_beam, int32_t* layer_status, hipStream_t s,
                   hipEvent_t* evs);
// ---- off-node incidence (k_beam.hip): the half-size particular solution (eq. 46-48), before the
// boundary factorisation overwrites F~; the response through the boundary operators after the right
// divisions; the synthesis of the beam BRDF.
void enqueue_beam_particular(const LaunchSet& ls, const double* omega, const double* coef, int32_t* status,
                             hipStream_t s);
void enqueue_beam_response(const LaunchSet& ls, const double* tau, int32_t* status, hipStream_t s);
// the beams' radiance towards the extra outgoing directions by source-function integration (eq. 36-38),
// after enqueue_beam_response and before the response stage overwrites E~
void enqueue_beam_outgoing(const LaunchSet& ls, const double* tau, const double* omega, const double* coef,
                           int32_t* status, hipStream_t s);
void enqueue_beam_synth(const LaunchSet& ls, double* F_beam, const int32_t* status, hipStream_t s);
void enqueue_backward(const LaunchSet& ls, const double* tau, const double* omega, const double* dF, double* dtau,
                      double* domega, double* dcoef, hipStream_t s);

// ---- adjoint kernels (k_adjoint.hip)
__global__ void k_copy_buf(const Item* items, double* ws, int src, int dst, const int32_t* status);
__global__ void k_fill_identity(const Item* items, double* ws, int dst, const int32_t* status);
__global__ void k_copy_status(const int32_t* src, int32_t* dst, int n);
__global__ void k_bwd_q(const Item* items, const Layer* layers, const double* quad, const double* dF, double* ws,
                        const int32_t* status);
__global__ void k_bwd_dscale(const Item* items, double* ws, const int32_t* status);
__global__ void k_bwd_dk(const Item* items, const double* tau, double* ws, const int32_t* status);
__global__ void k_bwd_tau(const Item* items, const double* tau, double* ws, const int32_t* status);
__global__ void k_bwd_omega(const Item* items, const Layer* layers, const double* quad, const double* omega,
                            double* ws, const int32_t* status);
constexpr int kCoefThreads = 256;
__global__ void k_bwd_coef(const Item* items, const Layer* layers, const double* quad, const double* omega,
                           double* ws, const int32_t* status);
__global__ void k_bwd_reduce(const Layer* layers, const Item* items, const double* ws, const int32_t* status,
                             double* dtau, double* domega, double* dcoef);

// Radiance of eq. 1 from the F_r table, the incident azimuth being kshift grid steps
__global__ void k_radiance(const Layer* layers, int layer, int q, int kshift, const double* quad, const double* F,
                           double i0, double i1, double i2, double i3, double* I_out);
// The same at an arbitrary incident azimuth phi0, summing the Fourier series over the layer's
// per-order responses R^m kept in the workspace
__global__ void k_radiance_series(const Layer* layers, const Item* items, int layer, int q, double phi0,
                                  const double* ws, double i0, double i1, double i2, double i3, double* I_out);

}  // namespace vbrdf
