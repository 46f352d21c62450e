// Refinement of the eigen-decomposition of the homogeneous step (Sec. 3.A, eq. 43-45).
//
// G = F~ E~ is formed explicitly for the eigensolver, and forming it squares the grading of the
// problem (||G|| ~ 1/mu_min^2): eigenpairs of the small (diffusion-mode) eigenvalues, and pairs
// of nearly equal eigenvalues, come out with errors of eps ||G|| relative to their own scale. One
// step of Newton refinement of the whole decomposition brings them back to the accuracy of the
// factored product. With U the computed eigenvectors (a complex pair stored as the real and
// imaginary parts in columns j, j+1 with Im lambda_j > 0) and Lambda the matching block-diagonal
// matrix (1x1 blocks lambda, 2x2 blocks [[a, b], [-b, a]] for a +- i b):
//   Y = U^-1 F~ (E~ U)                  (the product is never formed: two GEMMs, then a solve),
//   Lambda_a X_ab - X_ab Lambda_b = -Y_ab     for every pair of blocks a != b,
//   U <- U (I + X) Q,   Lambda <- the blocks of Y rewritten in standard form by Q.
// The solve uses the LU of U^T and a right division: Y^T = (G U)^T U^-T. A block pair whose
// correction is not small (|X_ab| or |X_ba| > 0.1: nearly equal eigenvalues with a large coupling,
// where the first-order step would not hold) is "close" and gets no correction; a close pair of
// real eigenvalues that are close to nothing else is instead diagonalised exactly within its
// 2 x 2 block of Y. Q has at most two nonzeros per column: identity on the other real
// eigenvalues; for a complex pair the basis change that puts the pair's 2x2 block of Y back into
// the form [[a, b], [-b, a]] with b > 0 (Re w, Im w of the block's eigenvector w, scaled so that Q
// is close to the identity); for a close real pair the eigenvectors of its 2 x 2 block.
//
// Workspace during the step: kBufG = Y^T; per column j in the extras block, Q[j][j] at [6n),
// Q[p_j][j] at [7n) with p_j the partner column (or -1) in the ints at [3n), the close-partner
// count and the last close partner in the ints at [3.5n) and [5n), the new eigenvalues at [8n) and
// [9n) until the commit. All of these are overwritten later by the boundary solve.
#include "vbrdf_internal.hpp"

namespace vbrdf {

constexpr double kRefineMaxCorr = 0.1;

// dst = src^T for every item, 32 x 32 tiles through LDS (both sides coalesced).
__global__ __launch_bounds__(256) void k_transpose(const Item* items, double* ws, int src, int dst,
                                                   const int32_t* status) {
  const Item it = items[blockIdx.z];
  if (status[it.layer] != 0) return;
  const int n = it.n;
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  if (r0 >= n || c0 >= n) return;
  const double* S = buf_ptr(ws, it, src);
  double* D = buf_ptr(ws, it, dst);
  __shared__ double t[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8)
    if (r0 + r < n && c0 + tx < n) t[r][tx] = S[(int64_t)(r0 + r) * n + c0 + tx];
  __syncthreads();
  for (int c = ty; c < 32; c += 8)
    if (c0 + c < n && r0 + tx < n) D[(int64_t)(c0 + c) * n + r0 + tx] = t[tx][c];
}

__device__ inline double yel(const double* YT, int n, int i, int j) { return YT[(int64_t)j * n + i]; }

struct RefineCols {  // per-column state of the step, in the extras block
  double *qs, *qo, *nre, *nim;
  int *pt, *cnt, *cpart;
};
__device__ inline RefineCols refine_cols(double* ex, int n) {
  RefineCols c;
  c.qs = ex + 6 * n;
  c.qo = ex + 7 * n;
  c.nre = ex + 8 * n;
  c.nim = ex + 9 * n;
  c.pt = reinterpret_cast<int*>(ex + 3 * n);
  c.cnt = c.pt + n;
  c.cpart = reinterpret_cast<int*>(ex + 5 * n);
  return c;
}

// Per column j: the new eigenvalue (1x1: Y_jj; pair: the standard form of its 2x2 block of Y), the
// column's entries of Q, and a zero close-partner count.
__global__ __launch_bounds__(256) void k_refine_lam(const Item* items, double* ws, const int32_t* status) {
  const Item it = items[blockIdx.y];
  if (status[it.layer] != 0) return;
  const int n = it.n;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double* base = ws + it.ws;
  const double* YT = base + (int64_t)kBufG * n * n;
  double* ex = base + extras_off(n);
  const double* lre = ex;
  const double* lim = ex + n;
  const RefineCols rc = refine_cols(ex, n);
  rc.cnt[j] = 0;
  rc.cpart[j] = -1;
  const double li = lim[j];
  if (li == 0.0) {
    rc.qs[j] = 1.0;
    rc.qo[j] = 0.0;
    rc.pt[j] = -1;
    rc.nre[j] = yel(YT, n, j, j);
    rc.nim[j] = 0.0;
    return;
  }
  const int j0 = li > 0.0 ? j : j - 1;  // first column of the pair
  const bool first = j == j0;
  rc.pt[j] = first ? j0 + 1 : j0;
  const double y00 = yel(YT, n, j0, j0), y01 = yel(YT, n, j0, j0 + 1);
  const double y10 = yel(YT, n, j0 + 1, j0), y11 = yel(YT, n, j0 + 1, j0 + 1);
  const double a = 0.5 * (y00 + y11);
  const double h = 0.5 * (y00 - y11);
  const double disc = h * h + y01 * y10;
  if (!(disc < 0.0) || !isfinite(disc)) {  // no longer a complex pair: keep it as it was
    rc.qs[j] = 1.0;
    rc.qo[j] = 0.0;
    rc.nre[j] = lre[j];
    rc.nim[j] = li;
    return;
  }
  const double b = sqrt(-disc);
  // Q = [Re w, Im w] (rows j0, j0 + 1) for the eigenvector w of a + i b
  double q0r, q1r, q0i, q1i;
  if (fabs(y01) >= fabs(y10)) {  // w = (y01, a - y00 + i b) / y01
    q0r = 1.0;
    q1r = (a - y00) / y01;
    q0i = 0.0;
    q1i = b / y01;
  } else {  // w = -i (a - y11 + i b, y10) / b
    q0r = 1.0;
    q1r = 0.0;
    q0i = -(a - y11) / b;
    q1i = -y10 / b;
  }
  rc.qs[j] = first ? q0r : q1i;  // Q[j][j]
  rc.qo[j] = first ? q1r : q0i;  // Q[partner][j]
  rc.nre[j] = a;
  rc.nim[j] = first ? b : -b;
}

// The 1x1 or 2x2 block of Lambda that starts at column j0 (s = 1 or 2): lam = p (+ q J).
struct Blk {
  int j0, s;
  double p, q;
};

__device__ inline Blk block_of(const double* lre, const double* lim, int j) {
  Blk b;
  b.j0 = lim[j] < 0.0 ? j - 1 : j;
  b.s = lim[b.j0] > 0.0 ? 2 : 1;
  b.p = lre[b.j0];
  b.q = b.s == 2 ? lim[b.j0] : 0.0;
  return b;
}

// (p I + q J)^-1 C for a 2 x 2 C (row-major c[4]), J = [[0, 1], [-1, 0]]
__device__ inline void left_inv(double p, double q, const double* c, double* x) {
  const double d = 1.0 / (p * p + q * q);
  // (p I - q J) C
  x[0] = d * (p * c[0] - q * c[2]);
  x[1] = d * (p * c[1] - q * c[3]);
  x[2] = d * (q * c[0] + p * c[2]);
  x[3] = d * (q * c[1] + p * c[3]);
}

// X_ab (as a 2 x 2 array, unused entries zero) solving Lambda_a X - X Lambda_b = -Y_ab, and whether
// every entry is finite and at most kRefineMaxCorr in modulus.
__device__ inline bool sylvester(const double* YT, int n, const Blk& A, const Blk& B, double* x) {
  double c[4] = {0.0, 0.0, 0.0, 0.0};
  for (int r = 0; r < A.s; ++r)
    for (int k = 0; k < B.s; ++k) c[2 * r + k] = -yel(YT, n, A.j0 + r, B.j0 + k);
  for (int k = 0; k < 4; ++k) x[k] = 0.0;
  if (A.s == 1 && B.s == 1) {
    x[0] = c[0] / (A.p - B.p);
  } else if (A.s == 2 && B.s == 1) {  // (Lambda_a - lam_b I) x = c, x a column
    const double p = A.p - B.p, q = A.q, d = 1.0 / (p * p + q * q);
    x[0] = d * (p * c[0] - q * c[2]);
    x[2] = d * (q * c[0] + p * c[2]);
  } else if (A.s == 1 && B.s == 2) {  // x (lam_a I - Lambda_b) = c, x a row
    const double p = A.p - B.p, q = -B.q, d = 1.0 / (p * p + q * q);
    // x = c (p I + q J)^-1 = c (p I - q J) d,  (p I - q J) = [[p, -q], [q, p]]
    x[0] = d * (c[0] * p + c[1] * q);
    x[1] = d * (-c[0] * q + c[1] * p);
  } else {  // both 2 x 2: split C into the parts commuting and anticommuting with J
    double c1[4], c2[4], x1[4], x2[4];
    // J C J = [[-c3, c2], [c1, -c0]] (row-major)
    const double jcj[4] = {-c[3], c[2], c[1], -c[0]};
    for (int k = 0; k < 4; ++k) {
      c1[k] = 0.5 * (c[k] - jcj[k]);
      c2[k] = 0.5 * (c[k] + jcj[k]);
    }
    left_inv(A.p - B.p, A.q - B.q, c1, x1);
    left_inv(A.p - B.p, A.q + B.q, c2, x2);
    for (int k = 0; k < 4; ++k) x[k] = x1[k] + x2[k];
  }
  bool small = true;
  for (int k = 0; k < 4; ++k) small = small && isfinite(x[k]) && fabs(x[k]) <= kRefineMaxCorr;
  return small;
}

// Entry (i, k) of X (zero within a block and for close block pairs); *close tells whether the
// blocks of i and k differ and are close.
__device__ inline double corr_entry(const double* YT, int n, const double* lre, const double* lim, int i, int k,
                                    bool* close) {
  const Blk A = block_of(lre, lim, i), B = block_of(lre, lim, k);
  *close = false;
  if (A.j0 == B.j0) return 0.0;
  double xab[4], xba[4];
  const bool ok = sylvester(YT, n, A, B, xab) & sylvester(YT, n, B, A, xba);
  *close = !ok;
  return ok ? xab[2 * (i - A.j0) + (k - B.j0)] : 0.0;
}

// Close block pairs: one thread per (row block leader, column block leader) counts the column
// block's close partners of row block a, and records the last one.
__global__ void k_refine_close(const Item* items, double* ws, const int32_t* status) {
  const Item it = items[blockIdx.z];
  if (status[it.layer] != 0) return;
  const int n = it.n;
  const int i = blockIdx.y * 16 + threadIdx.y;
  const int k = blockIdx.x * 16 + threadIdx.x;
  if (i >= n || k >= n) return;
  double* base = ws + it.ws;
  const double* YT = base + (int64_t)kBufG * n * n;
  double* ex = base + extras_off(n);
  const double* lre = ex;
  const double* lim = ex + n;
  if (lim[i] < 0.0 || lim[k] < 0.0) return;  // not a block leader
  bool close;
  corr_entry(YT, n, lre, lim, i, k, &close);
  if (!close) return;
  const RefineCols rc = refine_cols(ex, n);
  atomicAdd(rc.cnt + i, 1);
  rc.cpart[i] = k;  // meaningful only when the count ends at 1 (a single writer)
}

// A close pair of real eigenvalues a, b, each close to nothing else: the eigenvectors of the 2 x 2
// block C = Y[{a, b}, {a, b}] (real eigenvalues; a pair that turned complex is left as it was).
__global__ __launch_bounds__(256) void k_refine_pairs(const Item* items, double* ws, const int32_t* status) {
  const Item it = items[blockIdx.y];
  if (status[it.layer] != 0) return;
  const int n = it.n;
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  double* base = ws + it.ws;
  const double* YT = base + (int64_t)kBufG * n * n;
  double* ex = base + extras_off(n);
  const double* lim = ex + n;
  const RefineCols rc = refine_cols(ex, n);
  if (lim[a] != 0.0 || rc.cnt[a] != 1) return;
  const int b = rc.cpart[a];
  if (b < 0 || lim[b] != 0.0 || rc.cnt[b] != 1 || rc.cpart[b] != a) return;
  const int lo = min(a, b), hi = max(a, b);
  const double c00 = yel(YT, n, lo, lo), c01 = yel(YT, n, lo, hi);
  const double c10 = yel(YT, n, hi, lo), c11 = yel(YT, n, hi, hi);
  const double h = 0.5 * (c00 - c11);
  const double disc = h * h + c01 * c10;
  if (!(disc >= 0.0) || !isfinite(disc)) return;
  const double sq = sqrt(disc);
  const double m1 = 0.5 * (c00 + c11) + (h >= 0.0 ? sq : -sq);  // the eigenvalue nearer c00
  const double m2 = (c00 + c11) - m1;
  // eigenvector of m1 as (1, x) and of m2 as (y, 1)
  const double d1 = m1 - c11, d2 = m2 - c00;
  const double x = d1 != 0.0 ? c10 / d1 : 0.0;
  const double y = d2 != 0.0 ? c01 / d2 : 0.0;
  if (!isfinite(x) || !isfinite(y) || fabs(x * y) > 0.5) return;  // nearly parallel: keep as it was
  if (a == lo) {
    rc.qs[a] = 1.0;
    rc.qo[a] = x;
    rc.nre[a] = m1;
  } else {
    rc.qs[a] = 1.0;
    rc.qo[a] = y;
    rc.nre[a] = m2;
  }
  rc.pt[a] = b;
}

// M = (I + X) Q entry by entry, into kBufX.
__global__ void k_refine_delta(const Item* items, double* ws, const int32_t* status) {
  const Item it = items[blockIdx.z];
  if (status[it.layer] != 0) return;
  const int n = it.n;
  const int i = blockIdx.y * 16 + threadIdx.y;
  const int j = blockIdx.x * 16 + threadIdx.x;
  if (i >= n || j >= n) return;
  double* base = ws + it.ws;
  const double* YT = base + (int64_t)kBufG * n * n;
  double* Mo = base + (int64_t)kBufX * n * n;
  double* ex = base + extras_off(n);
  const double* lre = ex;
  const double* lim = ex + n;
  const RefineCols rc = refine_cols(ex, n);
  bool close;
  double v = ((i == j) ? 1.0 : corr_entry(YT, n, lre, lim, i, j, &close)) * rc.qs[j];
  const int p = rc.pt[j];
  if (p >= 0) v += ((i == p) ? 1.0 : corr_entry(YT, n, lre, lim, i, p, &close)) * rc.qo[j];
  Mo[(int64_t)i * n + j] = v;
}

// U <- U M (computed into kBufZ by the GEMM before this kernel), eigenvalues <- the new ones.
__global__ __launch_bounds__(256) void k_refine_commit(const Item* items, double* ws, const int32_t* status) {
  const Item it = items[blockIdx.y];
  if (status[it.layer] != 0) return;
  const int n = it.n;
  double* base = ws + it.ws;
  const double* Z = base + (int64_t)kBufZ * n * n;
  double* U = base + (int64_t)kBufU * n * n;
  double* ex = base + extras_off(n);
  const int64_t nn = (int64_t)n * n;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nn; t += (int64_t)gridDim.x * blockDim.x) {
    U[t] = Z[t];
    if (t < n) {
      ex[t] = ex[8 * n + t];
      ex[n + t] = ex[9 * n + t];
    }
  }
}

}  // namespace vbrdf
