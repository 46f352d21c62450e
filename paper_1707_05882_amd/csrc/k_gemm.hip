// Batched square FP64 GEMM on the CDNA matrix cores: C = op(A) B (or its transpose) for every
// work item.
//
// Used for the products of the homogeneous step: FE (Sec. 3.A, eq. 43), E X for the mode vectors
// (eq. 45), the back-transformation of the eigenvectors and the products of the eigenpair
// refinement. Each item carries its own n; the grid covers the largest n and surplus tiles exit.
//
// Workgroup order: the (item, tile) list is cut into 8 contiguous ranges, one per XCD, and every
// range holds whole items, every eighth one (all tiles of an item share one L2; 18% faster than the
// plain grid order, and a split into contiguous item ranges lost that to the uneven sizes).
// Tiling: 64 x 64 output tile per workgroup of 4 waves; each wave owns a 32 x 32 quadrant as 2 x 2
// v_mfma_f64_16x16x4 tiles; K is staged through LDS 16 at a time, the next step's tiles loaded into
// registers while the current step is multiplied. Lane layout of the 16x16x4 FP64
// MFMA (measured on gfx950 with an in-bounds probe): A element (row = lane % 16, k = lane / 16),
// B element (k = lane / 16, col = lane % 16), accumulator register v (row = lane / 16 + 4 v,
// col = lane % 16).
#include "vbrdf_internal.hpp"

namespace vbrdf {

typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int kGT = 64;  // output tile
constexpr int kGK = 16;  // K step

__global__ __launch_bounds__(256) void k_gemm(const Item* items, double* ws, int bufA, int bufB, int bufC, int mode,
                                               const int32_t* status) {
  const bool transA = mode & kGemmTransA, transB = mode & kGemmTransB, transC = mode & kGemmTransC;
  // XCD-aware order: workgroups go to the 8 XCDs round-robin by linear id L, so XCD g (= L mod 8)
  // takes a contiguous range of the (item, tile) list, V = g q + min(g, r) + L / 8 with
  // q r = divmod(#workgroups, 8), a bijection: the tiles of an item share one L2.
  const int ntile = gridDim.x * gridDim.y;
  const int64_t total = (int64_t)ntile * gridDim.z;
  const int64_t L = blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z);
  const int64_t xq = total / 8, xr = total % 8, xg = L % 8;
  const int64_t V = xg * xq + (xg < xr ? xg : xr) + L / 8;
  // Within the range, virtual item c becomes item 8 k + g for the c-th entry (g, k) of the
  // contiguous split of the items into 8 groups: each XCD holds every eighth item, so the sizes of
  // consecutive items (one layer's orders) spread evenly over the XCDs.
  const int tile = (int)(V % ntile);
  const int64_t vi = V / ntile, ni = gridDim.z, iq = ni / 8, ir = ni % 8;
  int64_t ig, ik;
  if (vi < ir * (iq + 1)) {
    ig = vi / (iq + 1);
    ik = vi - ig * (iq + 1);
  } else {
    ig = ir + (vi - ir * (iq + 1)) / (iq > 0 ? iq : 1);
    ik = vi - ir * (iq + 1) - (ig - ir) * iq;
  }
  const Item it = items[8 * ik + ig];
  if (status[it.layer] != 0) return;
  const int n = it.n;
  const int r0 = (tile / gridDim.x) * kGT, c0 = (tile % gridDim.x) * kGT;
  if (r0 >= n || c0 >= n) return;
  const double* A = buf_ptr(ws, it, bufA);
  const double* B = buf_ptr(ws, it, bufB);
  double* C = buf_ptr(ws, it, bufC);

  __shared__ double sA[kGT][kGK + 1];
  __shared__ double sB[kGK][kGT + 1];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;

  double4_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (double4_t){0.0, 0.0, 0.0, 0.0};

  // The next K step's tiles go to registers while the current step is multiplied; loads are
  // unconditional (indices clamped, values outside the matrix masked after the load).
  constexpr int kPer = kGT * kGK / 256;
  double ra[kPer], rb[kPer];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int t = threadIdx.x + 256 * q;
      const int ar = transA ? t % kGT : t / kGK, ak = transA ? t / kGT : t % kGK;
      const int gr = min(r0 + ar, n - 1), gk = min(k0 + ak, n - 1);
      const double v = transA ? A[(int64_t)gk * n + gr] : A[(int64_t)gr * n + gk];
      ra[q] = (r0 + ar < n && k0 + ak < n) ? v : 0.0;
      const int bc = transB ? t / kGK : t % kGT, bk = transB ? t % kGK : t / kGT;
      const int hc = min(c0 + bc, n - 1), hk = min(k0 + bk, n - 1);
      const double w = transB ? B[(int64_t)hc * n + hk] : B[(int64_t)hk * n + hc];
      rb[q] = (k0 + bk < n && c0 + bc < n) ? w : 0.0;
    }
  };
  load(0);
  for (int k0 = 0; k0 < n; k0 += kGK) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int t = threadIdx.x + 256 * q;
      if (transA)
        sA[t % kGT][t / kGT] = ra[q];
      else
        sA[t / kGK][t % kGK] = ra[q];
      if (transB)
        sB[t % kGK][t / kGK] = rb[q];
      else
        sB[t / kGT][t % kGT] = rb[q];
    }
    __syncthreads();
    if (k0 + kGK < n) load(k0 + kGK);
#pragma unroll
    for (int kk = 0; kk < kGK; kk += 4) {
      double a[2], b[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        a[x] = sA[wr + x * 16 + li][kk + lk];
        b[x] = sB[kk + lk][wc + x * 16 + li];
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
    }
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = r0 + wr + x * 16 + lk + 4 * v;
        const int col = c0 + wc + y * 16 + li;
        if (row < n && col < n) {
          const int64_t idx = transC ? (int64_t)col * n + row : (int64_t)row * n + col;
          const double val = (mode & kGemmNegate) ? -acc[x][y][v] : acc[x][y][v];
          C[idx] = (mode & kGemmAccumulate) ? C[idx] + val : val;
        }
      }
}

}  // namespace vbrdf
