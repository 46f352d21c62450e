// Allocation-free solve of one layer: vbrdf_solve_noalloc.
//
// The plan-based entry point keeps its tables and per-(layer, order) workspace in device memory
// that plan creation allocates. Callers that cannot allocate (code under stream capture, serving
// loops, harnesses that forbid it) use this entry point instead: the tables and the workspace of
// one layer live in the file-scope array `scratch` below, which the runtime places on every GPU
// the library runs on (and holds until the process ends). Host code never uses the array's name
// as a device address: its address on the current device is looked up once per device with
// hipGetSymbolAddress and cached. The tables are written on the device by a set-up kernel (the
// Gauss nodes included), so the call makes no host-to-device copy either.
//
// Every call on one GPU shares that GPU's array and leaves its contents behind; nothing in it has
// to start at zero (every kernel writes what it later reads). Calls that overlap on one GPU (on
// different streams or threads) race on the array and must be serialised by the caller.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/vbrdf.h"
#include "vbrdf_internal.hpp"

namespace vbrdf {

constexpr size_t kScratchDoubles = VBRDF_NOALLOC_SCRATCH_BYTES / sizeof(double);
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};

// Table layout inside the scratch array, in doubles (every part 256-byte aligned).
struct ScratchLayout {
  int64_t layer, items, tasks, quad, ws, total;
};

int64_t align32(int64_t d) { return (d + 31) / 32 * 32; }

ScratchLayout layout(int N, int L, int M) {
  ScratchLayout s;
  const int n = 4 * N;
  s.layer = 0;
  s.items = align32((int64_t)(sizeof(Layer) + 7) / 8);
  s.tasks = s.items + align32(((int64_t)M * sizeof(Item) + 7) / 8);
  s.quad = s.tasks + align32(((int64_t)N * N * sizeof(SynthTask) + 7) / 8);
  s.ws = s.quad + align32(2 * (int64_t)N);
  s.total = s.ws + (int64_t)M * align32(item_doubles(n, N, L));
  return s;
}

}  // namespace

// P_N(z) and P_N'(z) by the three-term recurrence (device copy of the host routine).
__device__ inline void legendre_pn_dev(int N, double z, double& pn, double& dpn) {
  double p1 = 1.0, p0 = 0.0;
  for (int k = 1; k <= N; ++k) {
    const double p2 = p0;
    p0 = p1;
    p1 = ((2.0 * k - 1.0) * z * p0 - (k - 1.0) * p2) / k;
  }
  pn = p1;
  dpn = N * (z * p1 - p0) / (z * z - 1.0);
}

// Writes the layer, item and synthesis-task tables and the double-Gauss nodes of eq. 15 (Newton
// iteration on P_N from the classical cosine guesses, one thread per symmetric node pair).
__global__ __launch_bounds__(256) void k_noalloc_setup(double* base, ScratchLayout s, int N, int L, int M, int P) {
  const int tid = threadIdx.x;
  const int n = 4 * N;
  if (tid == 0) {
    Layer ly{};
    ly.N = N;
    ly.L = L;
    ly.M = M;
    ly.n_dphi = P;
    ly.coef_off = 0;
    ly.out_off = 0;
    ly.quad_off = 0;
    ly.item0 = 0;
    *reinterpret_cast<Layer*>(base + s.layer) = ly;
  }
  Item* items = reinterpret_cast<Item*>(base + s.items);
  for (int m = tid; m < M; m += blockDim.x) {
    Item it{};
    it.layer = 0;
    it.m = m;
    it.N = N;
    it.L = L;
    it.n = n;
    it.ws = (int64_t)m * ((item_doubles(n, N, L) + 31) / 32 * 32);  // from the workspace start
    items[m] = it;
  }
  SynthTask* tasks = reinterpret_cast<SynthTask*>(base + s.tasks);
  for (int t = tid; t < N * N; t += blockDim.x) tasks[t] = SynthTask{0, t / N, t % N, 0};
  double* quad = base + s.quad;
  const double pi = 3.14159265358979323846;
  for (int i = tid; i < (N + 1) / 2; i += blockDim.x) {
    double z = cos(pi * (i + 0.75) / (N + 0.5));
    double pn, dp;
    for (int it = 0; it < 100; ++it) {
      legendre_pn_dev(N, z, pn, dp);
      const double dz = pn / dp;
      z -= dz;
      if (fabs(dz) < 1e-15) break;
    }
    legendre_pn_dev(N, z, pn, dp);
    z -= pn / dp;
    legendre_pn_dev(N, z, pn, dp);
    const double wi = 2.0 / ((1.0 - z * z) * dp * dp);
    const bool mid = (N % 2 == 1) && i == N / 2;  // the node at x = 0 of an odd rule
    quad[i] = 0.5 * (1.0 + (mid ? 0.0 : -z));
    quad[N - 1 - i] = 0.5 * (1.0 + (mid ? 0.0 : z));
    quad[N + i] = 0.5 * wi;
    quad[N + N - 1 - i] = 0.5 * wi;
  }
}

}  // namespace vbrdf

using namespace vbrdf;

extern "C" vbrdf_status vbrdf_solve_noalloc(int32_t N, int32_t L, int32_t M, int32_t n_dphi, const double* tau,
                                            const double* omega, const double* coef, double* F_r,
                                            int32_t* layer_status, void* stream) {
  if (!tau || !omega || !coef || !F_r || !layer_status) return vbrdf_fail(VBRDF_E_INVALID, "null device pointer");
  if (N < 1 || L < 1 || M < 1 || n_dphi < 1)
    return vbrdf_fail(VBRDF_E_INVALID, "N, L, M, n_dphi must be >= 1 (got %d, %d, %d, %d)", N, L, M, n_dphi);
  if (M > L) return vbrdf_fail(VBRDF_E_INVALID, "M = %d exceeds L = %d", M, L);
  if (N > VBRDF_MAX_N) return vbrdf_fail(VBRDF_E_UNSUPPORTED, "N = %d above %d", N, VBRDF_MAX_N);
  if (M > kSynthMaxM) return vbrdf_fail(VBRDF_E_UNSUPPORTED, "M = %d above %d", M, kSynthMaxM);
  if (n_dphi > kSynthMaxPhi) return vbrdf_fail(VBRDF_E_UNSUPPORTED, "n_dphi = %d above %d", n_dphi, kSynthMaxPhi);
  const ScratchLayout sl = layout(N, L, M);
  if ((size_t)sl.total * sizeof(double) > VBRDF_NOALLOC_SCRATCH_BYTES)
    return vbrdf_fail(VBRDF_E_NOMEM, "layer N = %d, L = %d, M = %d needs %lld bytes of scratch, above the static %llu",
                      N, L, M, (long long)(sl.total * (int64_t)sizeof(double)),
                      (unsigned long long)VBRDF_NOALLOC_SCRATCH_BYTES);
  const int n = 4 * N;
  const size_t trsm_lds = sizeof(double) * (size_t)n * (trsm_ldb(n) + 2);
  if (trsm_lds > 65536)  // never for the sizes that fit the scratch; kept as a guard
    return vbrdf_fail(VBRDF_E_UNSUPPORTED, "right-division tile of %zu bytes above the default LDS cap", trsm_lds);

  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return vbrdf_fail(VBRDF_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return vbrdf_fail(VBRDF_E_UNSUPPORTED, "device %d above %d", dev, kMaxDevices);
  double* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
      void* ptr = nullptr;
      e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr)
        return vbrdf_fail(VBRDF_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
      g_scratch[dev] = static_cast<double*>(ptr);
    }
    base = g_scratch[dev];
  }

  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  k_noalloc_setup<<<1, 256, 0, s>>>(base, sl, N, L, M, n_dphi);
  LaunchSet ls;
  ls.layers_d = reinterpret_cast<const Layer*>(base + sl.layer);
  ls.items_d = reinterpret_cast<const Item*>(base + sl.items);
  ls.tasks_d = reinterpret_cast<const SynthTask*>(base + sl.tasks);
  ls.quad_d = base + sl.quad;
  ls.ws_d = base + sl.ws;
  ls.n_layers = 1;
  ls.n_items = M;
  ls.n_tasks = N * N;
  ls.max_n = n;
  ls.max_N = N;
  ls.trsm_rows = kTrsmRows;  // the tile shape its scratch sizes assume
  ls.trsm_tiles = (n + kTrsmRows - 1) / kTrsmRows;
  ls.trsm32_tiles = ls.trsm_tiles;
  ls.trsm_lds = trsm_lds;
  ls.eigen_mode = kEigenPlanOrder;  // one layer: every order has the same size
  ls.n_big = n > kLdsMaxn ? M : 0;   // and the same eigensolver kernel (no order table needed)
  enqueue_solve(ls, tau, omega, coef, nullptr, F_r, nullptr, layer_status, s, nullptr);
  e = hipGetLastError();
  if (e != hipSuccess) return vbrdf_fail(VBRDF_E_DEVICE, "launch: %s", hipGetErrorString(e));
  return VBRDF_OK;
}
