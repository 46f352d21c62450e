// Layer stacks and reflecting bases (Sec. 2.C: one homogeneous solution per layer with the radiance
// continuous across interfaces, and the base condition; Sec. 3.C "Base Reflection", eq. 57-66).
//
// Every layer is first solved over a black base. Per order, its reflection and transmission
// operators on radiance at the nodes are R~ = U S'^-1 + U T'^-1 - I and T~ = U S'^-1 - U T'^-1,
// with upward fields stored mirrored (Stokes U and V negated), the storage in which a homogeneous
// layer looks the same from above and from below. The stack is then combined from the bottom up:
// with X~ the reflection of what lies beneath a layer (the combined sub-stack, or the base matrix
// of eq. 58 in the same storage),
//     R~_stack = R~ + T~ X~ (I - R~ X~)^-1 T~ = R~ + T~ (I - X~ R~)^-1 (X~ T~),
// which is what the full boundary system with interface continuity and the base condition gives
// (the downward field at the interface is (I - R~ X~)^-1 T~ times the incident one, and the
// upward field there is X~ times it). The products run on the matrix cores (k_gemm), the system
// (I - X~ R~) is factored by k_lu and applied as a right division by k_trsm. Levels are launched
// from the bottom: level 0 holds the bottom layers over a reflecting base, level k the layers k
// above their stack's bottom.
//
// Base matrix in the node representation (eq. 58 in quadrature form): the upward radiance at the
// base is X_b times the downward one, X_b[(i,r),(j,p)] = alpha_j mu_j Rb^m[(i,r),(j,p)]. The ideal
// depolarising Lambertian base has Rb^0 = 2 rho on the (I, I) entries and nothing else (eq. 66).
// Mirrored storage negates the U and V rows: X~ = Delta X_b.
#include "vbrdf_internal.hpp"

namespace vbrdf {

constexpr double kPi = 3.141592653589793;

// Base data checks: rho in [0, 1] (Lambertian), finite entries (Mueller). One workgroup per layer;
// only bottom layers of stacks carry base data.
__global__ void k_stack_validate(const Layer* layers, const int32_t* below, int base_kind, const double* base,
                                 const int64_t* base_off, int32_t* status) {
  const int l = blockIdx.x;
  if (below[l] >= 0 || base_kind == VBRDF_BASE_BLACK) return;
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  if (base_kind == VBRDF_BASE_LAMBERTIAN) {
    if (threadIdx.x == 0) {
      const double rho = base[l];
      bad = !(rho >= 0.0 && rho <= 1.0);  // NaN fails both
    }
  } else {
    const Layer ly = layers[l];
    const int64_t n = 4 * (int64_t)ly.N, cnt = (int64_t)ly.M * n * n;
    const double* b = base + base_off[l];
    int mine = 0;
    for (int64_t t = threadIdx.x; t < cnt; t += blockDim.x) mine |= !isfinite(b[t]);
    if (mine) atomicOr(&bad, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0 && bad && status[l] == 0) status[l] = VBRDF_E_INVALID;
}

// A layer inherits the status of the first failed layer beneath it. The walk reads statuses that
// other threads may be rewriting, but a rewritten entry holds the same code the walk would reach
// further down, so the result does not depend on the order.
__global__ void k_stack_status(int n_layers, const int32_t* below, int32_t* status) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= n_layers || status[l] != 0) return;
  for (int j = below[l], steps = 0; j >= 0 && steps < n_layers; j = below[j], ++steps) {
    const int32_t s = status[j];
    if (s != 0) {
      status[l] = s;
      return;
    }
  }
}

// Per item of one level: X~ (the reflection beneath) into kBufG and the identity into kBufZ.
__global__ void k_stack_x(const Item* items, const StackTask* tasks, const Layer* layers, const double* quad,
                          int base_kind, const double* base, double* ws, int32_t* status) {
  const Item it = items[blockIdx.y];
  if (status[it.layer] != 0) return;
  const StackTask tk = tasks[blockIdx.y];
  if (tk.src_layer >= 0) {  // a failure in the adding step beneath (a singular system) ends this layer too
    const int32_t ss = status[tk.src_layer];
    if (ss != 0) {
      if (blockIdx.x == 0 && threadIdx.x == 0) status[it.layer] = ss;
      return;
    }
  }
  const int n = it.n;
  const int64_t nn = (int64_t)n * n;
  double* X = buf_ptr(ws, it, kBufG);
  double* I = buf_ptr(ws, it, kBufZ);
  const Layer ly = layers[it.layer];
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nn; t += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(t / n), b = (int)(t % n);
    double x = 0.0;
    if (tk.src_ws >= 0) {
      x = ws[tk.src_ws + (int64_t)kBufE * nn + t];
    } else {
      const int j = b >> 2, r = a & 3;
      const double w = quad[ly.quad_off + j] * quad[ly.quad_off + ly.N + j];  // mu_j alpha_j
      if (base_kind == VBRDF_BASE_LAMBERTIAN) {
        if (it.m == 0 && r == 0 && (b & 3) == 0) x = 2.0 * base[tk.base_off] * w;
      } else if (base_kind == VBRDF_BASE_MUELLER) {
        x = (r >= 2 ? -w : w) * base[tk.base_off + t];
      }
    }
    X[t] = x;
    I[t] = (a == b) ? 1.0 : 0.0;
  }
}

// Final per-order response of every layer of a stacked plan: R^m = Delta R~ R0 in place in kBufE
// (R0 = diag(1 / (pi alpha_q)) on the incident streams), as k_response writes for a lone layer.
__global__ void k_stack_finish(const Item* items, const Layer* layers, const double* quad, double* ws,
                               const int32_t* status) {
  const Item it = items[blockIdx.z];
  if (status[it.layer] != 0) return;
  const int n = it.n;
  const int a = blockIdx.y * 16 + threadIdx.y;
  const int b = blockIdx.x * 16 + threadIdx.x;
  if (a >= n || b >= n) return;
  const Layer ly = layers[it.layer];
  double* R = buf_ptr(ws, it, kBufE);
  const int64_t idx = (int64_t)a * n + b;
  const double alq = quad[ly.quad_off + it.N + b / 4];
  const double sgn = ((a & 3) >= 2) ? -1.0 : 1.0;
  const double r0 = 1.0 / (kPi * alq);
  R[idx] = sgn * R[idx] * r0;
}

}  // namespace vbrdf
