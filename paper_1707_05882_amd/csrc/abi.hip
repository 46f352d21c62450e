// C-ABI of the library: plans, validation, launch sequence and error reporting.
//
// A plan is specialised to a list of layer shapes (N, L, M, n_dphi). It owns the quadrature table,
// the work-item table (one item per (layer, Fourier order)), the synthesis task table and one
// device workspace block per item. vbrdf_solve only enqueues kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/vbrdf.h"
#include "vbrdf_internal.hpp"

using namespace vbrdf;

namespace {

constexpr int kNumStages = kNumSolveStages;
constexpr int kTimedSolves = 256;  // solves whose stage events are kept between queries
const char* const kStageNames[kNumStages] = {"validate", "legendre", "assemble", "gemm_FE", "eigen",  "gemm_U",
                                             "hqapply",  "refine",   "gemm_V",   "vfix",    "colscal", "bcbuild",
                                             "lu",       "trsm",     "response", "stack",   "synth"};

thread_local std::string g_err;

vbrdf_status fail(vbrdf_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

}  // namespace

namespace vbrdf {

vbrdf_status vbrdf_fail(vbrdf_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

}  // namespace vbrdf

namespace {

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(VBRDF_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// P_N(z) and P_N'(z) by the three-term recurrence.
void legendre_pn(int N, double z, double& pn, double& dpn) {
  double p1 = 1.0, p0 = 0.0;
  for (int k = 1; k <= N; ++k) {
    const double p2 = p0;
    p0 = p1;
    p1 = ((2.0 * k - 1.0) * z * p0 - (k - 1.0) * p2) / k;
  }
  pn = p1;
  dpn = N * (z * p1 - p0) / (z * z - 1.0);
}

// N-point Gauss-Legendre rule on [-1, 1], nodes ascending: Newton iteration on P_N from the
// classical cosine guesses, weights w = 2 / ((1 - x^2) P_N'(x)^2).
void gauss_legendre(int N, std::vector<double>& x, std::vector<double>& w) {
  x.assign(N, 0.0);
  w.assign(N, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < (N + 1) / 2; ++i) {
    double z = std::cos(pi * (i + 0.75) / (N + 0.5));
    double pn, dp;
    for (int it = 0; it < 100; ++it) {
      legendre_pn(N, z, pn, dp);
      const double dz = pn / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-15) break;
    }
    legendre_pn(N, z, pn, dp);  // one more step at the converged node
    z -= pn / dp;
    legendre_pn(N, z, pn, dp);
    const double wi = 2.0 / ((1.0 - z * z) * dp * dp);
    x[i] = -z;
    x[N - 1 - i] = z;
    w[i] = wi;
    w[N - 1 - i] = wi;
  }
  if (N % 2 == 1) x[N / 2] = 0.0;
}

template <class T>
vbrdf_status upload(const std::vector<T>& h, T** d) {
  *d = nullptr;
  if (h.empty()) return VBRDF_OK;
  HIP_TRY(hipMalloc(reinterpret_cast<void**>(d), h.size() * sizeof(T)));
  HIP_TRY(hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return VBRDF_OK;
}

}  // namespace

struct vbrdf_plan : LaunchSet {
  size_t out_doubles = 0;
  size_t ws_bytes = 0;
  std::vector<Layer> layers_h;
  std::vector<Item> items_h;
  bool ws_owned = true;  // false when the workspace is the caller's
  bool solved = false;   // a forward solve has been enqueued (the adjoint reads its state)
  bool timing = false;
  bool graph = false;             // capture the solve into a hipGraph and replay it
  hipGraphExec_t gexec = nullptr;  // instantiated for the pointers in gkey
  const void* gkey[8] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  size_t base_doubles = 0;  // base data a solve reads (vbrdf_plan_base_bytes / 8)
  size_t beam_doubles = 0;  // off-node beam output (vbrdf_plan_beam_bytes / 8)
  int timed = 0;  // solves recorded since the last stage_times query (capped at kTimedSolves)
  std::vector<hipEvent_t> ev;  // kTimedSolves sets of kNumStages + 1 events

  ~vbrdf_plan() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    if (layers_d) (void)hipFree(const_cast<Layer*>(layers_d));
    if (items_d) (void)hipFree(const_cast<Item*>(items_d));
    if (tasks_d) (void)hipFree(const_cast<SynthTask*>(tasks_d));
    if (quad_d) (void)hipFree(const_cast<double*>(quad_d));
    if (ws_d && ws_owned) (void)hipFree(ws_d);
    if (status_d) (void)hipFree(status_d);
    if (order_d) (void)hipFree(const_cast<int32_t*>(order_d));
    if (queue_d) (void)hipFree(queue_d);
    if (below_d) (void)hipFree(const_cast<int32_t*>(below_d));
    if (base_off_d) (void)hipFree(const_cast<int64_t*>(base_off_d));
    if (stack_items_d) (void)hipFree(const_cast<Item*>(stack_items_d));
    if (stack_tasks_d) (void)hipFree(const_cast<StackTask*>(stack_tasks_d));
    if (mu0_d) (void)hipFree(const_cast<double*>(mu0_d));
    if (mu_out_d) (void)hipFree(const_cast<double*>(mu_out_d));
    if (btasks_d) (void)hipFree(const_cast<BeamTask*>(btasks_d));
  }
};

extern "C" {

int32_t vbrdf_abi_version(void) { return VBRDF_ABI_VERSION; }

const char* vbrdf_last_error(void) { return g_err.c_str(); }

vbrdf_status vbrdf_gauss_nodes(int32_t N, double* mu, double* alpha) {
  if (N < 1) return fail(VBRDF_E_INVALID, "N must be >= 1 (got %d)", N);
  if (!mu || !alpha) return fail(VBRDF_E_INVALID, "null output pointer");
  std::vector<double> x, w;
  gauss_legendre(N, x, w);
  for (int i = 0; i < N; ++i) {
    mu[i] = 0.5 * (1.0 + x[i]);
    alpha[i] = 0.5 * w[i];
  }
  return VBRDF_OK;
}

// Right-division tile rows of a plan (4, 8 or 16) and the matching grid and LDS size.
static void set_trsm_rows(LaunchSet* p, int rows) {
  p->trsm_rows = rows;
  p->trsm_tiles = trsm_tiles_for(p->max_n, rows);
  p->trsm_lds = trsm_lds_for(p->max_n, rows);
}

// Descriptor checks shared by plan creation and the workspace query.
static vbrdf_status check_desc(const vbrdf_plan_desc* d) {
  if (!d) return fail(VBRDF_E_INVALID, "null plan descriptor");
  if (d->abi_version != VBRDF_ABI_VERSION)
    return fail(VBRDF_E_INVALID, "abi_version %d does not match library %d", d->abi_version, VBRDF_ABI_VERSION);
  if (d->n_layers < 1) return fail(VBRDF_E_INVALID, "n_layers must be >= 1");
  if (!d->N || !d->L || !d->M || !d->n_dphi) return fail(VBRDF_E_INVALID, "null shape array");
  if (d->precision != VBRDF_PRECISION_FP64 && d->precision != VBRDF_PRECISION_FP32_REFINED)
    return fail(VBRDF_E_UNSUPPORTED, "unknown precision %d", d->precision);
  const int known = VBRDF_FLAG_STAGE_TIMING | VBRDF_FLAG_GRAPH | VBRDF_FLAG_EMIT_TRANSMISSION |
                    VBRDF_FLAG_SAVE_FOR_BACKWARD | VBRDF_FLAG_DISABLE_FP64_FALLBACK;
  if (d->flags & ~known) return fail(VBRDF_E_UNSUPPORTED, "unknown flags 0x%x", d->flags);
  if ((d->flags & VBRDF_FLAG_STAGE_TIMING) && (d->flags & VBRDF_FLAG_GRAPH))
    return fail(VBRDF_E_UNSUPPORTED, "stage timing and graph replay cannot be combined");
  if ((d->flags & VBRDF_FLAG_DISABLE_FP64_FALLBACK) && d->precision != VBRDF_PRECISION_FP32_REFINED)
    return fail(VBRDF_E_INVALID, "DISABLE_FP64_FALLBACK needs the FP32_REFINED precision");
  if (d->qr_sweep_cap < 0) return fail(VBRDF_E_INVALID, "qr_sweep_cap must be >= 0 (got %d)", d->qr_sweep_cap);
  if (d->refine_steps < -1 || d->refine_steps > 8)
    return fail(VBRDF_E_INVALID, "refine_steps must lie in [-1, 8] (got %d)", d->refine_steps);
  if (d->refine_steps != 0 && d->precision != VBRDF_PRECISION_FP32_REFINED)
    return fail(VBRDF_E_INVALID, "refine_steps needs the FP32_REFINED precision");
  if (d->workspace_bytes && !d->workspace) return fail(VBRDF_E_INVALID, "workspace_bytes given without a workspace");
  if (d->workspace && (reinterpret_cast<uintptr_t>(d->workspace) & 255))
    return fail(VBRDF_E_INVALID, "caller workspace must be 256-byte aligned");
  for (int l = 0; l < d->n_layers; ++l) {
    const int N = d->N[l], L = d->L[l], M = d->M[l], P = d->n_dphi[l];
    if (N < 1 || L < 1 || M < 1 || P < 1) return fail(VBRDF_E_INVALID, "layer %d: N, L, M, n_dphi must be >= 1", l);
    if (M > L) return fail(VBRDF_E_INVALID, "layer %d: M = %d exceeds L = %d", l, M, L);
    if (N > VBRDF_MAX_N) return fail(VBRDF_E_UNSUPPORTED, "layer %d: N = %d above %d", l, N, VBRDF_MAX_N);
    if (M > kSynthMaxM) return fail(VBRDF_E_UNSUPPORTED, "layer %d: M = %d above %d", l, M, kSynthMaxM);
    if (P > kSynthMaxPhi) return fail(VBRDF_E_UNSUPPORTED, "layer %d: n_dphi = %d above %d", l, P, kSynthMaxPhi);
  }
  if (d->base != VBRDF_BASE_BLACK && d->base != VBRDF_BASE_LAMBERTIAN && d->base != VBRDF_BASE_MUELLER)
    return fail(VBRDF_E_UNSUPPORTED, "unknown base kind %d", d->base);
  bool stacks = false;
  if (d->below) {
    std::vector<int> above(d->n_layers, -1);
    for (int l = 0; l < d->n_layers; ++l) {
      const int b = d->below[l];
      if (b == -1) continue;
      if (b < 0 || b >= d->n_layers || b == l) return fail(VBRDF_E_INVALID, "layer %d: below = %d out of range", l, b);
      if (above[b] >= 0) return fail(VBRDF_E_INVALID, "layers %d and %d both lie on layer %d", above[b], l, b);
      above[b] = l;
      if (d->N[b] != d->N[l] || d->M[b] != d->M[l])
        return fail(VBRDF_E_INVALID, "layers %d and %d of one stack differ in N or M", l, b);
      stacks = true;
    }
    for (int l = 0; l < d->n_layers; ++l) {  // every chain must end within kMaxStackLevels layers
      int j = l, depth = 0;
      while (d->below[j] >= 0 && depth <= d->n_layers) {
        j = d->below[j];
        ++depth;
      }
      if (d->below[j] >= 0) return fail(VBRDF_E_INVALID, "the stack under layer %d has a cycle", l);
      if (depth >= kMaxStackLevels)
        return fail(VBRDF_E_UNSUPPORTED, "the stack under layer %d is deeper than %d layers", l, kMaxStackLevels);
    }
  }
  if ((stacks || d->base != VBRDF_BASE_BLACK) &&
      (d->flags & (VBRDF_FLAG_SAVE_FOR_BACKWARD | VBRDF_FLAG_EMIT_TRANSMISSION)))
    return fail(VBRDF_E_UNSUPPORTED, "stacks and reflecting bases take neither SAVE_FOR_BACKWARD nor EMIT_TRANSMISSION");
  if (d->n_mu0 < 0 || d->n_mu0 > kMaxBeams)
    return fail(VBRDF_E_INVALID, "n_mu0 must lie in [0, %d] (got %d)", kMaxBeams, d->n_mu0);
  if (d->n_mu0 > 0) {
    if (!d->mu0) return fail(VBRDF_E_INVALID, "null mu0 array");
    for (int j = 0; j < d->n_mu0; ++j)
      if (!(d->mu0[j] > 0.0 && d->mu0[j] <= 1.0)) return fail(VBRDF_E_INVALID, "mu0[%d] outside (0, 1]", j);
    for (int l = 0; l < d->n_layers; ++l)
      if (d->n_mu0 > d->N[l]) return fail(VBRDF_E_INVALID, "n_mu0 = %d exceeds N = %d of layer %d", d->n_mu0, d->N[l], l);
    if (stacks || d->base != VBRDF_BASE_BLACK || (d->flags & VBRDF_FLAG_SAVE_FOR_BACKWARD))
      return fail(VBRDF_E_UNSUPPORTED, "off-node beams take neither stacks, a reflecting base nor SAVE_FOR_BACKWARD");
  }
  if (d->n_mu_out < 0 || d->n_mu_out > kMaxBeams)
    return fail(VBRDF_E_INVALID, "n_mu_out must lie in [0, %d] (got %d)", kMaxBeams, d->n_mu_out);
  if (d->n_mu_out > 0) {
    if (d->n_mu0 < 1) return fail(VBRDF_E_INVALID, "extra outgoing directions need off-node beams (n_mu0 > 0)");
    if (!d->mu_out) return fail(VBRDF_E_INVALID, "null mu_out array");
    for (int o = 0; o < d->n_mu_out; ++o)
      if (!(d->mu_out[o] > 0.0 && d->mu_out[o] <= 1.0)) return fail(VBRDF_E_INVALID, "mu_out[%d] outside (0, 1]", o);
    for (int l = 0; l < d->n_layers; ++l)
      if (d->n_mu_out > d->N[l])
        return fail(VBRDF_E_INVALID, "n_mu_out = %d exceeds N = %d of layer %d", d->n_mu_out, d->N[l], l);
  }
  return VBRDF_OK;
}

// Level tables of the stack stage. level(l) = 0 for the bottom layer of a stack, one more than the
// layer beneath otherwise; level-0 items take an adding step only over a reflecting base.
static vbrdf_status build_stacks(vbrdf_plan* p, const vbrdf_plan_desc* d) {
  const int nl = d->n_layers;
  std::vector<int32_t> below(nl, -1);
  if (d->below)
    for (int l = 0; l < nl; ++l) below[l] = d->below[l];
  std::vector<int> level(nl, 0);
  for (int l = 0; l < nl; ++l) {
    int j = l, k = 0;
    while (below[j] >= 0) {
      j = below[j];
      ++k;
    }
    level[l] = k;
  }
  std::vector<int64_t> base_off(nl, -1);
  int64_t off = 0;
  for (int l = 0; l < nl; ++l) {
    if (below[l] >= 0) continue;
    const Layer& ly = p->layers_h[l];
    if (d->base == VBRDF_BASE_LAMBERTIAN) base_off[l] = l;
    if (d->base == VBRDF_BASE_MUELLER) {
      base_off[l] = off;
      off += (int64_t)ly.M * 16 * ly.N * ly.N;
    }
  }
  p->base_doubles = d->base == VBRDF_BASE_LAMBERTIAN ? (size_t)nl : (size_t)off;
  std::vector<Item> sitems;
  std::vector<StackTask> stasks;
  int n_levels = 0;
  for (int l = 0; l < nl; ++l) n_levels = std::max(n_levels, level[l] + 1);
  p->n_levels = n_levels;
  for (int k = 0; k < n_levels; ++k) {
    p->lvl_off[k] = (int)sitems.size();
    for (int l = 0; l < nl; ++l) {
      if (level[l] != k) continue;
      if (below[l] < 0 && d->base == VBRDF_BASE_BLACK) continue;  // nothing beneath to add
      const Layer& ly = p->layers_h[l];
      const int64_t nn = 16 * (int64_t)ly.N * ly.N;
      for (int m = 0; m < ly.M; ++m) {
        const Item& it = p->items_h[ly.item0 + m];
        StackTask tk{};
        if (below[l] >= 0) {
          tk.src_ws = p->items_h[p->layers_h[below[l]].item0 + m].ws;
          tk.src_layer = below[l];
          tk.base_off = -1;
        } else {
          tk.src_ws = -1;
          tk.src_layer = -1;
          tk.base_off = d->base == VBRDF_BASE_MUELLER ? base_off[l] + m * nn : base_off[l];
        }
        sitems.push_back(it);
        stasks.push_back(tk);
      }
    }
  }
  p->lvl_off[n_levels] = (int)sitems.size();
  p->stacked = true;
  int32_t* below_d = nullptr;
  int64_t* base_off_d = nullptr;
  Item* sitems_d = nullptr;
  StackTask* stasks_d = nullptr;
  vbrdf_status st = upload(below, &below_d);
  p->below_d = below_d;
  if (st == VBRDF_OK) st = upload(base_off, &base_off_d);
  p->base_off_d = base_off_d;
  if (st == VBRDF_OK) st = upload(sitems, &sitems_d);
  p->stack_items_d = sitems_d;
  if (st == VBRDF_OK) st = upload(stasks, &stasks_d);
  p->stack_tasks_d = stasks_d;
  return st;
}

// Per-item workspace blocks, 256-byte aligned.
static int64_t block_doubles(int N, int L, bool save, int n_mu0, int n_mu_out) {
  return n_mu0 > 0 ? block_doubles_beams(4 * N, N, L, n_mu0, n_mu_out) : block_doubles_of(4 * N, N, L, save);
}

vbrdf_status vbrdf_workspace_query(const vbrdf_plan_desc* d, uint64_t* bytes) {
  if (!bytes) return fail(VBRDF_E_INVALID, "null output pointer");
  *bytes = 0;
  const vbrdf_status st = check_desc(d);
  if (st != VBRDF_OK) return st;
  int64_t total = 0;
  const bool save = (d->flags & VBRDF_FLAG_SAVE_FOR_BACKWARD) != 0;
  for (int l = 0; l < d->n_layers; ++l)
    total += (int64_t)d->M[l] * block_doubles(d->N[l], d->L[l], save, d->n_mu0, d->n_mu_out);
  *bytes = (uint64_t)total * sizeof(double);
  return VBRDF_OK;
}

vbrdf_status vbrdf_plan_create(const vbrdf_plan_desc* d, vbrdf_plan** out) {
  if (!out) return fail(VBRDF_E_INVALID, "null plan output pointer");
  *out = nullptr;
  const vbrdf_status chk = check_desc(d);
  if (chk != VBRDF_OK) return chk;

  vbrdf_plan* p = new (std::nothrow) vbrdf_plan();
  if (!p) return fail(VBRDF_E_NOMEM, "host allocation failed");
  p->n_layers = d->n_layers;
  std::vector<double> quad;
  std::vector<SynthTask> tasks;
  int64_t coef_off = 0, out_off = 0, ws_off = 0, beam_off = 0;
  std::vector<BeamTask> btasks;
  for (int l = 0; l < d->n_layers; ++l) {
    Layer ly{};
    ly.N = d->N[l];
    ly.L = d->L[l];
    ly.M = d->M[l];
    ly.n_dphi = d->n_dphi[l];
    ly.coef_off = coef_off;
    ly.out_off = out_off;
    ly.quad_off = (int64_t)quad.size();
    ly.item0 = (int64_t)p->items_h.size();
    ly.beam_off = beam_off;
    beam_off += (int64_t)(ly.N + d->n_mu_out) * d->n_mu0 * ly.n_dphi * 16;
    for (int i = 0; i < ly.N + d->n_mu_out; ++i)
      for (int j = 0; j < d->n_mu0; ++j) btasks.push_back(BeamTask{l, i, j, 0});
    std::vector<double> x, w;
    gauss_legendre(ly.N, x, w);
    for (int i = 0; i < ly.N; ++i) quad.push_back(0.5 * (1.0 + x[i]));
    for (int i = 0; i < ly.N; ++i) quad.push_back(0.5 * w[i]);
    const int n = 4 * ly.N;
    for (int m = 0; m < ly.M; ++m) {
      Item it{};
      it.layer = l;
      it.m = m;
      it.N = ly.N;
      it.L = ly.L;
      it.n = n;
      it.ws = ws_off;
      ws_off += block_doubles(ly.N, ly.L, (d->flags & VBRDF_FLAG_SAVE_FOR_BACKWARD) != 0, d->n_mu0, d->n_mu_out);
      p->items_h.push_back(it);
    }
    for (int i = 0; i < ly.N; ++i)
      for (int q = 0; q < ly.N; ++q) tasks.push_back(SynthTask{l, i, q, 0});
    p->max_n = std::max(p->max_n, n);
    p->trsm32_tiles = std::max(p->trsm32_tiles, (n + kTrsmRows - 1) / kTrsmRows);
    p->max_N = std::max(p->max_N, ly.N);
    coef_off += 6 * (int64_t)ly.L;
    out_off += (int64_t)ly.N * ly.N * ly.n_dphi * 16;
    p->layers_h.push_back(ly);
  }
  p->n_items = (int)p->items_h.size();
  p->n_tasks = (int)tasks.size();
  p->out_doubles = (size_t)out_off;
  p->ws_bytes = (size_t)ws_off * sizeof(double);
  if (d->workspace_cap_bytes && p->ws_bytes > d->workspace_cap_bytes) {
    size_t need = p->ws_bytes;
    delete p;
    return fail(VBRDF_E_NOMEM, "workspace %zu bytes exceeds the cap %llu", need,
                (unsigned long long)d->workspace_cap_bytes);
  }
  if (d->workspace && d->workspace_bytes < p->ws_bytes) {
    size_t need = p->ws_bytes;
    delete p;
    return fail(VBRDF_E_NOMEM, "caller workspace of %llu bytes is below the %zu bytes needed",
                (unsigned long long)d->workspace_bytes, need);
  }
  vbrdf_status st;
  Layer* layers_d = nullptr;
  Item* items_d = nullptr;
  SynthTask* tasks_d = nullptr;
  double* quad_d = nullptr;
  st = upload(p->layers_h, &layers_d);
  p->layers_d = layers_d;
  if (st == VBRDF_OK) st = upload(p->items_h, &items_d);
  p->items_d = items_d;
  if (st == VBRDF_OK) st = upload(tasks, &tasks_d);
  p->tasks_d = tasks_d;
  if (st == VBRDF_OK) st = upload(quad, &quad_d);
  p->quad_d = quad_d;
  if (st == VBRDF_OK) {  // eigensolver work order: largest systems first (stable)
    std::vector<int32_t> order(p->items_h.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int32_t)i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return p->items_h[a].n > p->items_h[b].n; });
    int32_t* order_d = nullptr;
    st = upload(order, &order_d);
    p->order_d = order_d;
    for (const Item& it : p->items_h) p->n_big += it.n > kLdsMaxn ? 1 : 0;
  }
  if (st == VBRDF_OK) {
    std::vector<int32_t> zero(1, 0);
    st = upload(zero, &p->queue_d);
  }
  if (st != VBRDF_OK) {
    delete p;
    return st;
  }
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
      p->persist_groups = cus;
  }
  p->eigen_mode = kEigenPlanOrder;
  p->graph = (d->flags & VBRDF_FLAG_GRAPH) != 0;
  p->precision = d->precision;
  p->transmission = (d->flags & VBRDF_FLAG_EMIT_TRANSMISSION) != 0;
  p->qr_sweep_cap = d->qr_sweep_cap;
  p->no_fallback = (d->flags & VBRDF_FLAG_DISABLE_FP64_FALLBACK) != 0;
  p->refine_steps = d->refine_steps == 0 ? kBoundaryRefineSteps : (d->refine_steps < 0 ? 0 : d->refine_steps);
  p->save = (d->flags & VBRDF_FLAG_SAVE_FOR_BACKWARD) != 0;
  if (p->save) {
    for (const Layer& ly : p->layers_h)
      if (6 * (int64_t)ly.L > 16 * (int64_t)ly.N * ly.N) {
        delete p;
        return fail(VBRDF_E_UNSUPPORTED, "SAVE_FOR_BACKWARD needs 6 L <= (4 N)^2 per layer");
      }
    hipError_t es = hipMalloc(reinterpret_cast<void**>(&p->status_d), sizeof(int32_t) * p->n_layers);
    if (es != hipSuccess) {
      p->status_d = nullptr;
      delete p;
      return fail(VBRDF_E_NOMEM, "status copy allocation failed: %s", hipGetErrorString(es));
    }
  }
  if (d->flags & VBRDF_FLAG_STAGE_TIMING) {
    p->timing = true;
    p->ev.assign((size_t)kTimedSolves * (kNumStages + 1), nullptr);
    for (auto& ev : p->ev) {
      hipError_t ee = hipEventCreate(&ev);
      if (ee != hipSuccess) {
        delete p;
        return fail(VBRDF_E_DEVICE, "hipEventCreate: %s", hipGetErrorString(ee));
      }
    }
  }
  set_trsm_rows(p, kTrsmRowsDefault);
  for (int rows : {4, 8, 16}) {
    const size_t lds = trsm_lds_for(p->max_n, rows);
    if (lds <= 65536) continue;  // the right-division tile of a large system exceeds the default LDS cap
    const hipError_t ea = hipFuncSetAttribute(trsm_kernel_ptr(rows), hipFuncAttributeMaxDynamicSharedMemorySize,
                                              (int)lds);
    if (ea != hipSuccess) {
      delete p;
      return fail(VBRDF_E_DEVICE, "hipFuncSetAttribute(k_trsm): %s", hipGetErrorString(ea));
    }
  }
  if (d->workspace) {
    p->ws_d = static_cast<double*>(d->workspace);
    p->ws_owned = false;
  } else {
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&p->ws_d), p->ws_bytes);
    if (e != hipSuccess) {
      size_t need = p->ws_bytes;
      p->ws_d = nullptr;
      delete p;
      return fail(VBRDF_E_NOMEM, "workspace allocation of %zu bytes failed: %s", need, hipGetErrorString(e));
    }
  }
  p->base_kind = d->base;
  if (d->n_mu0 > 0) {
    std::vector<double> mu0(d->mu0, d->mu0 + d->n_mu0);
    double* mu0_d = nullptr;
    BeamTask* bt_d = nullptr;
    vbrdf_status bs = upload(mu0, &mu0_d);
    p->mu0_d = mu0_d;
    if (bs == VBRDF_OK) bs = upload(btasks, &bt_d);
    p->btasks_d = bt_d;
    if (bs != VBRDF_OK) {
      delete p;
      return bs;
    }
    if (d->n_mu_out > 0) {
      std::vector<double> mo(d->mu_out, d->mu_out + d->n_mu_out);
      double* mo_d = nullptr;
      bs = upload(mo, &mo_d);
      p->mu_out_d = mo_d;
      if (bs != VBRDF_OK) {
        delete p;
        return bs;
      }
      p->n_mu_out = d->n_mu_out;
    }
    p->n_mu0 = d->n_mu0;
    p->n_btasks = (int)btasks.size();
    p->beam_doubles = (size_t)beam_off;
  }
  if (d->below || d->base != VBRDF_BASE_BLACK) {
    const vbrdf_status sst = build_stacks(p, d);
    if (sst != VBRDF_OK) {
      delete p;
      return sst;
    }
  }
  *out = p;
  return VBRDF_OK;
}

vbrdf_status vbrdf_plan_destroy(vbrdf_plan* plan) {
  delete plan;
  return VBRDF_OK;
}

size_t vbrdf_plan_output_bytes(const vbrdf_plan* plan) { return plan ? plan->out_doubles * sizeof(double) : 0; }

size_t vbrdf_plan_workspace_bytes(const vbrdf_plan* plan) { return plan ? plan->ws_bytes : 0; }

}  // extern "C"

namespace vbrdf {

static void enqueue_stacks(const LaunchSet& ls, const double* base, int32_t* layer_status, hipStream_t s);

// The launch sequence of one solve on stream s; when evs is given, kNumSolveStages + 1 events are
// recorded around and between the stages.
void enqueue_solve(const LaunchSet& ls, const double* tau, const double* omega, const double* coef,
                   const double* base, double* F_r, double* F_beam, int32_t* layer_status, hipStream_t s,
                   hipEvent_t* evs) {
  const bool beams = ls.n_mu0 > 0 && F_beam;
  const LaunchSet* p = &ls;
  const int ni = p->n_items, mn = p->max_n, mN = p->max_N;
  int stage = 0;
  auto mark = [&]() {
    if (evs) (void)hipEventRecord(evs[stage], s);
    ++stage;
  };
  mark();
  k_validate<<<p->n_layers, 64, 0, s>>>(p->layers_d, p->n_layers, tau, omega, coef, layer_status);
  mark();
  k_legendre<<<ni, kLegThreads, 0, s>>>(p->items_d, p->layers_d, p->quad_d, p->ws_d, layer_status);
  mark();
  const int at = (mN + 15) / 16;
  k_assemble<<<dim3(at, at, ni), 256, 0, s>>>(p->items_d, p->layers_d, p->quad_d, omega, coef, p->ws_d, layer_status);
  if (p->save) {  // E~ and F~ are overwritten later in the sequence; the adjoint needs them
    const dim3 cg((mn * mn + 255) / 256, ni);
    k_copy_buf<<<cg, 256, 0, s>>>(p->items_d, p->ws_d, kBufE, kBufSE, layer_status);
    k_copy_buf<<<cg, 256, 0, s>>>(p->items_d, p->ws_d, kBufF, kBufSF, layer_status);
  }
  mark();
  const int gt = (mn + 63) / 64;
  const dim3 gg(gt, gt, ni);
  k_gemm<<<gg, 256, 0, s>>>(p->items_d, p->ws_d, kBufF, kBufE, kBufG, 0, layer_status);  // G = F~ E~
  mark();
  // problems above the LDS size by their own kernel (the same for every schedule, so a schedule
  // never changes a result), largest first; then the others in the chosen schedule
  const int nb = p->n_big;
  if (nb > 0)
    k_eigen_big<<<nb, kEigenThreads, 0, s>>>(p->items_d, p->ws_d, layer_status, p->qr_sweep_cap, p->order_d);
  if (p->eigen_mode == kEigenPersistent && p->queue_d && p->order_d) {
    if (ni > nb) {
      k_reset_counter<<<1, 1, 0, s>>>(p->queue_d);
      k_eigen_persistent<<<std::min(ni - nb, p->persist_groups), kEigenThreads, 0, s>>>(
          p->items_d, p->ws_d, layer_status, p->qr_sweep_cap, p->order_d + nb, p->queue_d, ni - nb);
    }
  } else if (p->eigen_mode == kEigenPlanOrder || !p->order_d) {
    if (ni > nb) k_eigen<<<ni, kEigenThreads, 0, s>>>(p->items_d, p->ws_d, layer_status, p->qr_sweep_cap, nullptr);
  } else if (ni > nb) {
    k_eigen<<<ni - nb, kEigenThreads, 0, s>>>(p->items_d, p->ws_d, layer_status, p->qr_sweep_cap, p->order_d + nb);
  }
  mark();
  k_gemm<<<gg, 256, 0, s>>>(p->items_d, p->ws_d, kBufZ, kBufX, kBufG, kGemmTransA, layer_status);  // U' = Z X
  mark();
  const int hqt = (std::min(mn, kHqMfmaMaxN) + 15) / 16;
  k_hqapply_mfma<<<xcd_grid(ni, hqt), 64, 0, s>>>(p->items_d, ni, hqt, p->ws_d, layer_status);  // U = Q U'
  if (mn > kHqMfmaMaxN) {
    const int hqb = (mn + kHqCols - 1) / kHqCols;
    k_hqapply<<<xcd_grid(ni, hqb), 64, 0, s>>>(p->items_d, ni, hqb, p->ws_d, layer_status);
  }
  mark();
  // one Newton step on the eigen-decomposition with the factored product F~ (E~ U)
  const int et = (mn + 15) / 16;
  const int tt = (mn + 31) / 32;
  k_gemm<<<gg, 256, 0, s>>>(p->items_d, p->ws_d, kBufE, kBufU, kBufG, 0, layer_status);  // E~ U
  k_gemm<<<gg, 256, 0, s>>>(p->items_d, p->ws_d, kBufF, kBufG, kBufZ, kGemmTransC, layer_status);  // (F~ E~ U)^T
  k_transpose<<<dim3(tt, tt, ni), 256, 0, s>>>(p->items_d, p->ws_d, kBufU, kBufX, layer_status);  // U^T
  launch_lu(dim3(ni, 1), s, p->items_d, p->ws_d, layer_status, p->max_n, LuBufs{{kBufX, kBufX}, {kBufYS, kBufYS}});
  launch_trsm(p->trsm_rows, dim3(xcd_grid(ni, p->trsm_tiles)), p->trsm_lds, s, p->items_d, ni, p->trsm_tiles,
              p->ws_d, layer_status, TrsmBufs{{kBufYS, kBufYS}, {kBufZ, kBufZ}, {kBufG, kBufG}, 1, 0});  // Y^T = (G U)^T U^-T
  k_refine_lam<<<dim3((mn + 255) / 256, ni), 256, 0, s>>>(p->items_d, p->ws_d, layer_status);
  k_refine_close<<<dim3(et, et, ni), dim3(16, 16), 0, s>>>(p->items_d, p->ws_d, layer_status);
  k_refine_pairs<<<dim3((mn + 255) / 256, ni), 256, 0, s>>>(p->items_d, p->ws_d, layer_status);
  k_refine_delta<<<dim3(et, et, ni), dim3(16, 16), 0, s>>>(p->items_d, p->ws_d, layer_status);
  k_gemm<<<gg, 256, 0, s>>>(p->items_d, p->ws_d, kBufU, kBufX, kBufZ, 0, layer_status);  // U (I + X) Q
  k_refine_commit<<<dim3((mn * mn + 255) / 256, ni), 256, 0, s>>>(p->items_d, p->ws_d, layer_status);
  if (beams) enqueue_beam_particular(*p, omega, coef, layer_status, s);  // needs F~, before the boundary solve
  mark();
  k_gemm<<<gg, 256, 0, s>>>(p->items_d, p->ws_d, kBufE, kBufU, kBufG, 0, layer_status);  // V = E~ U
  mark();
  k_vfix<<<ni, 256, 0, s>>>(p->items_d, p->ws_d, layer_status);
  mark();
  k_colscal<<<dim3((mn + 63) / 64, ni), 64, 0, s>>>(p->items_d, tau, p->ws_d, layer_status);
  mark();
  k_bcbuild<<<dim3(et, et, ni), dim3(16, 16), 0, s>>>(p->items_d, p->ws_d, layer_status);
  mark();
  const LuBufs lub{{kBufZ, kBufX}, {kBufG, kBufF}, 0};
  const TrsmBufs trb{{kBufG, kBufF}, {kBufU, kBufU}, {kBufYS, kBufYT}, 2, 0};  // U S'^-1, U T'^-1
  const dim3 xg(xcd_grid(2 * ni, p->trsm_tiles));
  const dim3 xg32(xcd_grid(2 * ni, p->trsm32_tiles));
  if (p->precision == VBRDF_PRECISION_FP32_REFINED) {
    // FP32 factorisations and right divisions, refined against FP64 residuals; sides that do not
    // converge are redone in FP64 (or reported NONCONVERGED when the fallback is disabled)
    const size_t lds32 = sizeof(float) * (size_t)mn * (kTrsmRows + 1 + 2);
    const dim3 rg(gt, gt, 2 * ni);
    k_lu32<<<dim3(ni, 2), 1024, 0, s>>>(p->items_d, p->ws_d, layer_status);
    mark();
    k_trsm32<<<xg32, 64, lds32, s>>>(p->items_d, ni, p->trsm32_tiles, p->ws_d, layer_status, 0);
    for (int r = 0; r < p->refine_steps; ++r) {
      k_resid<<<rg, 256, 0, s>>>(p->items_d, p->ws_d, layer_status);
      k_trsm32<<<xg32, 64, lds32, s>>>(p->items_d, ni, p->trsm32_tiles, p->ws_d, layer_status, 1);
    }
    k_resid<<<rg, 256, 0, s>>>(p->items_d, p->ws_d, layer_status);
    k_bcheck<<<ni, 64, 0, s>>>(p->items_d, p->ws_d, layer_status, p->no_fallback ? 1 : 0);
    LuBufs lf = lub;
    lf.only_flagged = 1;
    TrsmBufs tf = trb;
    tf.only_flagged = 1;
    launch_lu(dim3(ni, 2), s, p->items_d, p->ws_d, layer_status, p->max_n, lf);
    launch_trsm(p->trsm_rows, xg, p->trsm_lds, s, p->items_d, ni, p->trsm_tiles, p->ws_d, layer_status, tf);
    mark();
  } else {
    launch_lu(dim3(ni, 2), s, p->items_d, p->ws_d, layer_status, p->max_n, lub);
    mark();
    launch_trsm(p->trsm_rows, xg, p->trsm_lds, s, p->items_d, ni, p->trsm_tiles, p->ws_d, layer_status, trb);
    mark();
  }
  if (beams) enqueue_beam_response(*p, tau, layer_status, s);
  if (beams && p->n_mu_out > 0) enqueue_beam_outgoing(*p, tau, omega, coef, layer_status, s);
  const int rmode = p->stacked ? kResponseBrackets : (p->transmission ? kResponseTransmission : 0);
  k_response<<<dim3(et, et, ni), dim3(16, 16), 0, s>>>(p->items_d, p->layers_d, p->quad_d, p->ws_d, layer_status,
                                                       rmode);
  mark();
  if (p->stacked) enqueue_stacks(*p, base, layer_status, s);
  mark();
  k_synth_mfma<<<p->n_tasks, 64, 0, s>>>(p->tasks_d, p->layers_d, p->items_d, p->quad_d, p->ws_d, F_r, layer_status);
  if (beams) enqueue_beam_synth(*p, F_beam, layer_status, s);
  if (p->save) k_copy_status<<<(p->n_layers + 255) / 256, 256, 0, s>>>(layer_status, p->status_d, p->n_layers);
  mark();
}

// The stack stage: base checks, status inheritance, then one adding step per level from the bottom
// up (formulas in k_stack.hip), and the final scaling of every item's response.
static void enqueue_stacks(const LaunchSet& ls, const double* base, int32_t* layer_status, hipStream_t s) {
  const LaunchSet* p = &ls;
  const int mn = p->max_n, gt = (mn + 63) / 64, et = (mn + 15) / 16;
  if (p->base_kind != VBRDF_BASE_BLACK)
    k_stack_validate<<<p->n_layers, 256, 0, s>>>(p->layers_d, p->below_d, p->base_kind, base, p->base_off_d,
                                                  layer_status);
  k_stack_status<<<(p->n_layers + 255) / 256, 256, 0, s>>>(p->n_layers, p->below_d, layer_status);
  const int xb = std::min(1024, (mn * mn + 255) / 256);
  for (int k = 0; k < p->n_levels; ++k) {
    const int cnt = p->lvl_off[k + 1] - p->lvl_off[k];
    if (cnt == 0) continue;
    const Item* it = p->stack_items_d + p->lvl_off[k];
    const StackTask* tk = p->stack_tasks_d + p->lvl_off[k];
    k_stack_x<<<dim3(xb, cnt), 256, 0, s>>>(it, tk, p->layers_d, p->quad_d, p->base_kind, base, p->ws_d,
                                            layer_status);
    const dim3 gg(gt, gt, cnt);
    k_gemm<<<gg, 256, 0, s>>>(it, p->ws_d, kBufG, kBufE, kBufZ, kGemmNegate | kGemmAccumulate, layer_status);  // I - X R
    k_gemm<<<gg, 256, 0, s>>>(it, p->ws_d, kBufG, kBufF, kBufYS, 0, layer_status);                             // X T
    launch_lu(dim3(cnt, 1), s, it, p->ws_d, layer_status, p->max_n, LuBufs{{kBufZ, kBufZ}, {kBufX, kBufX}, 0});
    launch_trsm(p->trsm_rows, dim3(xcd_grid(cnt, p->trsm_tiles)), p->trsm_lds, s, it, cnt, p->trsm_tiles, p->ws_d,
                layer_status, TrsmBufs{{kBufX, kBufX}, {kBufF, kBufF}, {kBufU, kBufU}, 1, 0});  // T (I - X R)^-1
    k_gemm<<<gg, 256, 0, s>>>(it, p->ws_d, kBufU, kBufYS, kBufE, kGemmAccumulate, layer_status);  // R += Y (X T)
  }
  k_stack_finish<<<dim3(et, et, p->n_items), dim3(16, 16), 0, s>>>(p->items_d, p->layers_d, p->quad_d, p->ws_d,
                                                                    layer_status);
}

// The adjoint sequence over all items (see k_adjoint.hip for the formulas and buffer roles).
void enqueue_backward(const LaunchSet& ls, const double* tau, const double* omega, const double* dF, double* dtau,
                      double* domega, double* dcoef, hipStream_t s) {
  const LaunchSet* p = &ls;
  const int ni = p->n_items, mn = p->max_n, mN = p->max_N;
  const int32_t* st = p->status_d;
  int32_t* stw = p->status_d;
  const int gt = (mn + 63) / 64;
  const dim3 gg(gt, gt, ni);
  const int et = (mn + 15) / 16;
  const int tt = (mn + 31) / 32;
  auto gemm = [&](int a, int b, int c, int mode) { k_gemm<<<gg, 256, 0, s>>>(p->items_d, p->ws_d, a, b, c, mode, st); };
  k_bwd_q<<<dim3((mN * mN + 255) / 256, ni), 256, 0, s>>>(p->items_d, p->layers_d, p->quad_d, dF, p->ws_d, st);
  // U^-T: LU of U^T, right division of the identity
  k_transpose<<<dim3(tt, tt, ni), 256, 0, s>>>(p->items_d, p->ws_d, kBufU, kBufX, st);
  launch_lu(dim3(ni, 1), s, p->items_d, p->ws_d, stw, p->max_n, LuBufs{{kBufX, kBufX}, {kBufG, kBufG}, 0});
  k_fill_identity<<<dim3((mn * mn + 255) / 256, ni), 256, 0, s>>>(p->items_d, p->ws_d, kBufF, st);
  launch_trsm(p->trsm_rows, dim3(xcd_grid(ni, p->trsm_tiles)), p->trsm_lds, s, p->items_d, ni, p->trsm_tiles, p->ws_d,
              stw, TrsmBufs{{kBufG, kBufG}, {kBufF, kBufF}, {kBufW, kBufW}, 1, 0});
  gemm(kBufYS, kBufE, kBufT1, kGemmTransA);                 // P_s^T Q
  gemm(kBufT1, kBufYS, kBufT2, kGemmTransB | kGemmNegate);  // A_s-bar
  gemm(kBufYT, kBufE, kBufT1, kGemmTransA);
  gemm(kBufT1, kBufYT, kBufT3, kGemmTransB | kGemmNegate);  // A_t-bar
  gemm(kBufSE, kBufT2, kBufT4, kGemmTransA);                // F_s-bar = E~^T A_s-bar
  gemm(kBufSE, kBufT3, kBufT5, kGemmTransA);                // F_t-bar
  gemm(kBufT2, kBufW, kBufT1, 0);                           // A_s-bar U^-T
  gemm(kBufT3, kBufW, kBufZ, 0);                            // A_t-bar U^-T
  k_bwd_dscale<<<dim3(et, et, ni), dim3(16, 16), 0, s>>>(p->items_d, p->ws_d, st);
  gemm(kBufT2, kBufU, kBufG, kGemmTransB);                  // E~-bar, explicit part
  gemm(kBufU, kBufT4, kBufT1, kGemmTransA);
  gemm(kBufT1, kBufW, kBufT4, 0);                           // X_s = U^T F_s-bar U^-T
  gemm(kBufU, kBufT5, kBufT1, kGemmTransA);
  gemm(kBufT1, kBufW, kBufT5, 0);                           // X_t
  k_bwd_dk<<<dim3(et, et, ni), dim3(16, 16), 0, s>>>(p->items_d, tau, p->ws_d, st);
  k_bwd_tau<<<ni, 256, 0, s>>>(p->items_d, tau, p->ws_d, st);
  gemm(kBufW, kBufT1, kBufT2, 0);
  gemm(kBufT2, kBufU, kBufT3, kGemmTransB);                 // G-bar = U^-T Y U^T
  gemm(kBufT3, kBufSE, kBufT4, kGemmTransB);                // F~-bar = G-bar E~^T
  gemm(kBufSF, kBufT3, kBufG, kGemmTransA | kGemmAccumulate);  // E~-bar += F~^T G-bar
  k_bwd_omega<<<ni, 256, 0, s>>>(p->items_d, p->layers_d, p->quad_d, omega, p->ws_d, st);
  k_bwd_coef<<<ni, kCoefThreads, 0, s>>>(p->items_d, p->layers_d, p->quad_d, omega, p->ws_d, st);
  k_bwd_reduce<<<p->n_layers, 256, 0, s>>>(p->layers_d, p->items_d, p->ws_d, st, dtau, domega, dcoef);
}

}  // namespace vbrdf

extern "C" {

static vbrdf_status solve_impl(vbrdf_plan* p, const double* tau, const double* omega, const double* coef,
                               const double* base, double* F_r, double* F_beam, int32_t* layer_status,
                               void* stream) {
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (p->graph) {
    if (!s) return fail(VBRDF_E_INVALID, "graph replay needs a non-default stream");
    const void* key[8] = {tau, omega, coef, F_r, layer_status, stream, base, F_beam};
    bool same = p->gexec != nullptr;
    for (int i = 0; i < 8; ++i) same = same && key[i] == p->gkey[i];
    if (!same) {
      if (p->gexec) {
        HIP_TRY(hipGraphExecDestroy(p->gexec));
        p->gexec = nullptr;
      }
      HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      enqueue_solve(*p, tau, omega, coef, base, F_r, F_beam, layer_status, s, nullptr);
      hipGraph_t g = nullptr;
      const hipError_t ec = hipStreamEndCapture(s, &g);
      if (ec != hipSuccess) return fail(VBRDF_E_DEVICE, "stream capture: %s", hipGetErrorString(ec));
      const hipError_t ei = hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ei != hipSuccess) {
        p->gexec = nullptr;
        return fail(VBRDF_E_DEVICE, "graph instantiation: %s", hipGetErrorString(ei));
      }
      for (int i = 0; i < 8; ++i) p->gkey[i] = key[i];
    }
    HIP_TRY(hipGraphLaunch(p->gexec, s));
    p->solved = true;
    return VBRDF_OK;
  }
  const bool rec = p->timing && p->timed < kTimedSolves;
  p->solved = true;
  enqueue_solve(*p, tau, omega, coef, base, F_r, F_beam, layer_status, s,
                rec ? &p->ev[(size_t)p->timed * (kNumStages + 1)] : nullptr);
  if (rec) ++p->timed;
  HIP_TRY(hipGetLastError());
  return VBRDF_OK;
}

vbrdf_status vbrdf_solve(vbrdf_plan* p, const double* tau, const double* omega, const double* coef, double* F_r,
                         int32_t* layer_status, void* stream) {
  if (!p) return fail(VBRDF_E_INVALID, "null plan");
  if (!tau || !omega || !coef || !F_r || !layer_status) return fail(VBRDF_E_INVALID, "null device pointer");
  if (p->base_kind != VBRDF_BASE_BLACK)
    return fail(VBRDF_E_INVALID, "the plan has a reflecting base: its data go through vbrdf_solve_base");
  return solve_impl(p, tau, omega, coef, nullptr, F_r, nullptr, layer_status, stream);
}

vbrdf_status vbrdf_solve_base(vbrdf_plan* p, const double* tau, const double* omega, const double* coef,
                              const double* base, double* F_r, int32_t* layer_status, void* stream) {
  if (!p) return fail(VBRDF_E_INVALID, "null plan");
  if (!tau || !omega || !coef || !F_r || !layer_status) return fail(VBRDF_E_INVALID, "null device pointer");
  if (p->base_kind != VBRDF_BASE_BLACK && !base) return fail(VBRDF_E_INVALID, "null base data for a reflecting base");
  return solve_impl(p, tau, omega, coef, p->base_kind == VBRDF_BASE_BLACK ? nullptr : base, F_r, nullptr,
                    layer_status, stream);
}

vbrdf_status vbrdf_solve_ex(vbrdf_plan* p, const double* tau, const double* omega, const double* coef,
                            const double* base, double* F_r, double* F_beam, int32_t* layer_status, void* stream) {
  if (!p) return fail(VBRDF_E_INVALID, "null plan");
  if (!tau || !omega || !coef || !F_r || !layer_status) return fail(VBRDF_E_INVALID, "null device pointer");
  if (p->base_kind != VBRDF_BASE_BLACK && !base) return fail(VBRDF_E_INVALID, "null base data for a reflecting base");
  if (p->n_mu0 > 0 && !F_beam) return fail(VBRDF_E_INVALID, "null beam output for a plan with off-node beams");
  return solve_impl(p, tau, omega, coef, p->base_kind == VBRDF_BASE_BLACK ? nullptr : base, F_r,
                    p->n_mu0 > 0 ? F_beam : nullptr, layer_status, stream);
}

size_t vbrdf_plan_beam_bytes(const vbrdf_plan* p) { return p ? p->beam_doubles * sizeof(double) : 0; }

size_t vbrdf_plan_base_bytes(const vbrdf_plan* p) { return p ? p->base_doubles * sizeof(double) : 0; }

vbrdf_status vbrdf_plan_inspect(const vbrdf_plan* p, int32_t layer, int32_t m, double* R_out, double* lam_re,
                                double* lam_im, double* T_out, void* stream) {
  if (!p) return fail(VBRDF_E_INVALID, "null plan");
  if (layer < 0 || layer >= p->n_layers) return fail(VBRDF_E_INVALID, "layer %d out of range", layer);
  const Layer& ly = p->layers_h[layer];
  if (m < 0 || m >= ly.M) return fail(VBRDF_E_INVALID, "order %d out of range", m);
  const Item& it = p->items_h[ly.item0 + m];
  const int n = it.n;
  HIP_TRY(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
  const double* base = p->ws_d + it.ws;
  if (R_out) HIP_TRY(hipMemcpy(R_out, base + (int64_t)kBufE * n * n, sizeof(double) * n * n, hipMemcpyDeviceToHost));
  if (lam_re) HIP_TRY(hipMemcpy(lam_re, base + extras_off(n), sizeof(double) * n, hipMemcpyDeviceToHost));
  if (lam_im) HIP_TRY(hipMemcpy(lam_im, base + extras_off(n) + n, sizeof(double) * n, hipMemcpyDeviceToHost));
  if (T_out) {
    if (!p->transmission) return fail(VBRDF_E_INVALID, "the plan was created without EMIT_TRANSMISSION");
    HIP_TRY(hipMemcpy(T_out, base + (int64_t)kBufF * n * n, sizeof(double) * n * n, hipMemcpyDeviceToHost));
  }
  return VBRDF_OK;
}

int32_t vbrdf_plan_stage_times(vbrdf_plan* p, float* ms_out, int32_t cap) {
  if (!p) return fail(VBRDF_E_INVALID, "null plan");
  if (!p->timing || p->timed == 0) return fail(VBRDF_E_INVALID, "plan has no timed solve");
  const int nsolve = p->timed;
  HIP_TRY(hipEventSynchronize(p->ev[(size_t)(nsolve - 1) * (kNumStages + 1) + kNumStages]));
  for (int i = 0; i < kNumStages && i < cap; ++i) {
    double sum = 0.0;
    for (int k = 0; k < nsolve; ++k) {
      float ms = 0.0f;
      const hipEvent_t* e = &p->ev[(size_t)k * (kNumStages + 1)];
      HIP_TRY(hipEventElapsedTime(&ms, e[i], e[i + 1]));
      sum += ms;
    }
    if (ms_out) ms_out[i] = (float)(sum / nsolve);
  }
  p->timed = 0;
  return kNumStages;
}

const char* vbrdf_stage_name(int32_t i) { return (i >= 0 && i < kNumStages) ? kStageNames[i] : nullptr; }

vbrdf_status vbrdf_plan_get_tuning(const vbrdf_plan* p, vbrdf_tuning* out) {
  if (!p || !out) return fail(VBRDF_E_INVALID, "null pointer");
  out->eigen_schedule = p->eigen_mode;
  out->trsm_rows = p->trsm_rows;
  return VBRDF_OK;
}

vbrdf_status vbrdf_plan_set_tuning(vbrdf_plan* p, const vbrdf_tuning* t) {
  if (!p || !t) return fail(VBRDF_E_INVALID, "null pointer");
  if (t->eigen_schedule < kEigenPlanOrder || t->eigen_schedule > kEigenPersistent)
    return fail(VBRDF_E_INVALID, "unknown eigen schedule %d", t->eigen_schedule);
  if (t->trsm_rows != 4 && t->trsm_rows != 8 && t->trsm_rows != 16)
    return fail(VBRDF_E_INVALID, "trsm_rows must be 4, 8 or 16 (got %d)", t->trsm_rows);
  p->eigen_mode = t->eigen_schedule;
  set_trsm_rows(p, t->trsm_rows);
  if (p->gexec) {  // the captured launch sequence no longer matches
    (void)hipGraphExecDestroy(p->gexec);
    p->gexec = nullptr;
  }
  return VBRDF_OK;
}

vbrdf_status vbrdf_plan_autotune(vbrdf_plan* p, const double* tau, const double* omega, const double* coef,
                                 double* F_r, int32_t* layer_status, void* stream, vbrdf_tuning* chosen) {
  if (!p) return fail(VBRDF_E_INVALID, "null plan");
  if (!tau || !omega || !coef || !F_r || !layer_status) return fail(VBRDF_E_INVALID, "null device pointer");
  if (p->base_kind != VBRDF_BASE_BLACK) return fail(VBRDF_E_UNSUPPORTED, "autotune of a plan with a reflecting base");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::vector<hipEvent_t> ev(kNumSolveStages + 1, nullptr);
  for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
  const int eig_stage = 4, refine_stage = 7, trsm_stage = 13;  // positions in kStageNames
  const int row_stage = p->precision == VBRDF_PRECISION_FP32_REFINED ? refine_stage : trsm_stage;
  const int cand_e[3] = {kEigenPlanOrder, kEigenLongestFirst, kEigenPersistent};
  const int cand_r[3] = {4, 8, 16};
  float best_e = 1e30f, best_r = 1e30f;
  int pick_e = p->eigen_mode, pick_r = p->trsm_rows;
  vbrdf_status st = VBRDF_OK;
  for (int round = 0; round < 2 && st == VBRDF_OK; ++round) {  // round 0 warms every variant up
    for (int c = 0; c < 3; ++c) {
      p->eigen_mode = cand_e[c];
      set_trsm_rows(p, cand_r[c]);
      enqueue_solve(*p, tau, omega, coef, nullptr, F_r, nullptr, layer_status, s, ev.data());
      hipError_t e = hipEventSynchronize(ev[kNumSolveStages]);
      float te = 0.0f, tr = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&te, ev[eig_stage], ev[eig_stage + 1]);
      if (e == hipSuccess) e = hipEventElapsedTime(&tr, ev[row_stage], ev[row_stage + 1]);
      if (e != hipSuccess) {
        st = fail(VBRDF_E_DEVICE, "autotune timing: %s", hipGetErrorString(e));
        break;
      }
      if (round == 1 && te < best_e) {
        best_e = te;
        pick_e = cand_e[c];
      }
      if (round == 1 && tr < best_r) {
        best_r = tr;
        pick_r = cand_r[c];
      }
    }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  p->eigen_mode = pick_e;
  set_trsm_rows(p, pick_r);
  if (st == VBRDF_OK) {  // leave the result of the chosen configuration behind
    enqueue_solve(*p, tau, omega, coef, nullptr, F_r, nullptr, layer_status, s, nullptr);
    const hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = fail(VBRDF_E_DEVICE, "autotune: %s", hipGetErrorString(e));
  }
  p->solved = true;
  if (p->gexec) {
    (void)hipGraphExecDestroy(p->gexec);
    p->gexec = nullptr;
  }
  if (st != VBRDF_OK) return st;
  if (chosen) {
    chosen->eigen_schedule = pick_e;
    chosen->trsm_rows = pick_r;
  }
  return VBRDF_OK;
}

vbrdf_status vbrdf_backward(vbrdf_plan* p, const double* tau, const double* omega, const double* coef,
                            const double* dF_r, double* dtau, double* domega, double* dcoef, void* stream) {
  if (!p) return fail(VBRDF_E_INVALID, "null plan");
  if (!p->save) return fail(VBRDF_E_INVALID, "the plan was created without SAVE_FOR_BACKWARD");
  if (!p->solved) return fail(VBRDF_E_INVALID, "no forward solve has been enqueued on this plan");
  if (!tau || !omega || !coef || !dF_r || !dtau || !domega || !dcoef)
    return fail(VBRDF_E_INVALID, "null device pointer");
  enqueue_backward(*p, tau, omega, dF_r, dtau, domega, dcoef, reinterpret_cast<hipStream_t>(stream));
  HIP_TRY(hipGetLastError());
  return VBRDF_OK;
}

vbrdf_status vbrdf_radiance(const vbrdf_plan* p, const double* F_r, int32_t layer, int32_t q, double phi0,
                            const double I0[4], double* I_out, void* stream) {
  if (!p) return fail(VBRDF_E_INVALID, "null plan");
  if (!I0 || !I_out) return fail(VBRDF_E_INVALID, "null pointer");
  if (layer < 0 || layer >= p->n_layers) return fail(VBRDF_E_INVALID, "layer %d out of range", layer);
  const Layer& ly = p->layers_h[layer];
  if (q < 0 || q >= ly.N) return fail(VBRDF_E_INVALID, "incident node %d out of range", q);
  if (!std::isfinite(phi0)) return fail(VBRDF_E_INVALID, "phi0 must be finite");
  const int total = ly.N * ly.n_dphi * 4;
  const double two_pi = 6.283185307179586;
  const double steps = phi0 / two_pi * ly.n_dphi;
  const double kr = std::nearbyint(steps);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (std::fabs(steps - kr) * two_pi / ly.n_dphi <= 1e-12) {  // on the grid: read the table
    if (!F_r) return fail(VBRDF_E_INVALID, "null F_r");
    const int kshift = (int)(((long long)kr % ly.n_dphi + ly.n_dphi) % ly.n_dphi);
    k_radiance<<<(total + 255) / 256, 256, 0, s>>>(p->layers_d, layer, q, kshift, p->quad_d, F_r, I0[0], I0[1],
                                                   I0[2], I0[3], I_out);
  } else {
    k_radiance_series<<<(total + 255) / 256, 256, 0, s>>>(p->layers_d, p->items_d, layer, q, phi0, p->ws_d, I0[0],
                                                          I0[1], I0[2], I0[3], I_out);
  }
  HIP_TRY(hipGetLastError());
  return VBRDF_OK;
}

}  // extern "C"
