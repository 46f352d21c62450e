// Input validation, Legendre matrices and assembly of the half-size matrices E~ and F~.
//
// Per Fourier order m the phase-matrix coefficient A^m(mu, mu') is the sum over degrees l of
// P_l^m(mu) B_l P_l^m(mu') (Sec. 2.B, eq. 9), with the Legendre matrices
// P_l^m = [[Pb,0,0,0],[0,R,-T,0],[0,-T,R,0],[0,0,0,Pb]] (eq. 9-11) built from Wigner d-functions:
// Pb = d^l_{m0}, R = -(d^l_{m2} + d^l_{m,-2})/2, T = -(d^l_{m2} - d^l_{m,-2})/2. The half-size
// reduction (Sec. 3.A, eq. 41) needs S+- = sum_l Pi_l B_l [I4 +- (-1)^(l-m) D] Pi_l^T on the
// Gauss nodes. Since B_l (I4 + D) keeps the IQ columns of B_l and B_l (I4 - D) the UV columns,
// each 4x4 block of S+- is a sum of an "IQ part" and a "UV part" over the two parity classes of
// l - m. The kernel forms E~ = M^-1 (I - omega/2 S+ W) and F~ = M^-1 (I - omega/2 S- W), which
// are similar to the paper's E and F (E = M E~ M^-1) and have the same spectrum products.
#include "vbrdf_internal.hpp"

namespace vbrdf {

// Input checks per layer (one wave per layer, lanes striding over the coefficients): tau > 0 and
// finite, 0 < omega <= 1, alpha_1 of degree 0 equal to 1, every coefficient finite.
__global__ __launch_bounds__(64) void k_validate(const Layer* layers, int n_layers, const double* tau,
                                                 const double* omega, const double* coef, int32_t* status) {
  const int l = blockIdx.x;
  if (l >= n_layers) return;
  const Layer ly = layers[l];
  const double* c = coef + ly.coef_off;
  int bad = 0;
  for (int k = threadIdx.x; k < 6 * ly.L; k += 64)
    if (!isfinite(c[k])) bad = 1;
  for (int o = 1; o < 64; o <<= 1) bad |= __shfl_xor(bad, o);
  if (threadIdx.x != 0) return;
  const double t = tau[l], w = omega[l];
  int32_t st = bad ? -1 : 0;
  if (!(t > 0.0) || !isfinite(t)) st = -1;
  if (!(w > 0.0) || !(w <= 1.0)) st = -1;
  if (!(fabs(c[0] - 1.0) <= 1e-12)) st = -1;
  status[l] = st;
}

// Start value of d^l_{mn}(x) at l = lmin = max(|m|, |n|), computed in logarithms so that large
// orders neither overflow the prefactor nor lose the small power of (1 - x^2).
__device__ inline double wigner_start(int m, int n, double x, int lmin) {
  int amn = abs(m - n), apn = abs(m + n);
  double lg = 0.5 * (lgamma(2.0 * lmin + 1.0) - lgamma(amn + 1.0) - lgamma(apn + 1.0)) - lmin * 0.6931471805599453;
  if (amn) lg += 0.5 * amn * log1p(-x);
  if (apn) lg += 0.5 * apn * log1p(x);
  double v = exp(lg);
  if (n < m && ((m - n) & 1)) v = -v;
  return v;
}

// One upward step of the three-term recurrence of d^s_{mn} in s: returns d^{s+1}.
__device__ inline double wigner_step(int s, int m, int n, double x, double d_s, double d_sm1) {
  double a = (2.0 * s + 1.0) * (s * (s + 1.0) * x - (double)m * n);
  double b = (s + 1.0) * sqrt(((double)s * s - (double)m * m) * ((double)s * s - (double)n * n));
  double c = s * sqrt(((s + 1.0) * (s + 1.0) - (double)m * m) * ((s + 1.0) * (s + 1.0) - (double)n * n));
  return (a * d_s - b * d_sm1) / c;
}

struct WSeq {
  int m, n, lmin;
  double prev, cur;  // d^{l-1}, d^l at the current l
};

__device__ inline double wseq_value(WSeq& q, int l, double x) {
  // returns d^l_{mn}(x) for increasing l = 0, 1, 2, ... (called once per l in order)
  if (l < q.lmin) return 0.0;
  if (l == q.lmin) {
    q.prev = 0.0;
    q.cur = wigner_start(q.m, q.n, x, q.lmin);
    return q.cur;
  }
  double nxt;
  if (l - 1 == 0)
    nxt = x * q.cur;  // m = n = 0: d^1_00 = x
  else
    nxt = wigner_step(l - 1, q.m, q.n, x, q.cur, q.prev);
  q.prev = q.cur;
  q.cur = nxt;
  return nxt;
}

// Legendre table per item: leg[(l * N + i) * 3 + {0,1,2}] = (Pb, R, T) of order m at mu_i.
// The three recurrences d_{m0}, d_{m2}, d_{m,-2} of a node run on three threads (thread =
// 128 sequence + node, N <= 128): each writes its own slot, d_{m2} and d_{m,-2} into the R and T
// slots, and after a barrier R = -(d_{m2} + d_{m,-2})/2 and T = -(d_{m2} - d_{m,-2})/2 are formed
// in place. Launched with kLegThreads threads.
__global__ __launch_bounds__(kLegThreads) void k_legendre(const Item* items, const Layer* layers,
                                                          const double* quad, double* ws,
                                                          const int32_t* status) {
  const Item it = items[blockIdx.x];
  if (status[it.layer] != 0) return;
  const Layer ly = layers[it.layer];
  const int N = it.N, L = it.L, m = it.m;
  double* leg = ws + it.ws + leg_off(it.n);
  const int seq = threadIdx.x / 128, i = threadIdx.x % 128;
  if (i < N) {
    const double x = quad[ly.quad_off + i];
    const int nn = seq == 0 ? 0 : (seq == 1 ? 2 : -2);
    WSeq q{m, nn, seq == 0 ? m : (m > 2 ? m : 2), 0.0, 0.0};
    for (int l = 0; l < L; ++l) {
      const double d = wseq_value(q, l, x);
      leg[((int64_t)l * N + i) * 3 + seq] = (l < m) ? 0.0 : d;
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < L * N; t += blockDim.x) {
    double* o = leg + (int64_t)t * 3;
    const double dp = o[1], dm = o[2];
    o[1] = -0.5 * (dp + dm);
    o[2] = -0.5 * (dp - dm);
  }
}

constexpr int kAsmTile = 16;   // 16 x 16 node pairs (4x4 Stokes blocks) per workgroup
constexpr int kAsmChunk = 32;  // degrees staged per LDS pass
static_assert(kAsmChunk % 2 == 0, "degree parity within a chunk follows the degree index");

// One workgroup per (item, tile of output node i, tile of input node j); one thread per (i, j)
// Stokes block. Legendre values and coefficients of a chunk of degrees are staged in LDS and
// shared by the 256 blocks of the tile.
__global__ __launch_bounds__(256) void k_assemble(const Item* items, const Layer* layers, const double* quad,
                                                   const double* omega, const double* coef, double* ws,
                                                   const int32_t* status) {
  const Item it = items[blockIdx.z];
  if (status[it.layer] != 0) return;
  const int N = it.N, L = it.L, m = it.m, n = it.n;
  const int i0 = blockIdx.y * kAsmTile, j0 = blockIdx.x * kAsmTile;
  if (i0 >= N || j0 >= N) return;
  const Layer ly = layers[it.layer];
  const double* leg = ws + it.ws + leg_off(n);
  const double* cf = coef + ly.coef_off;

  __shared__ double sPi[kAsmChunk][kAsmTile][3];
  __shared__ double sPj[kAsmChunk][kAsmTile][3];
  __shared__ double sC[6][kAsmChunk];

  const int tid = threadIdx.x;
  const int ti = tid / kAsmTile, tj = tid % kAsmTile;
  const int i = i0 + ti, j = j0 + tj;

  // accumulators: [parity][9] for the IQ part and the UV part
  double q[2][9], u[2][9];
#pragma unroll
  for (int e = 0; e < 2; ++e)
#pragma unroll
    for (int k = 0; k < 9; ++k) { q[e][k] = 0.0; u[e][k] = 0.0; }

  for (int lc = m; lc < L; lc += kAsmChunk) {
    const int cnt = min(kAsmChunk, L - lc);
    __syncthreads();
    for (int t = tid; t < cnt * kAsmTile * 3; t += blockDim.x) {
      int l = t / (kAsmTile * 3), r = t % (kAsmTile * 3);
      int a = r / 3, c = r % 3;
      sPi[l][a][c] = (i0 + a < N) ? leg[((int64_t)(lc + l) * N + i0 + a) * 3 + c] : 0.0;
      sPj[l][a][c] = (j0 + a < N) ? leg[((int64_t)(lc + l) * N + j0 + a) * 3 + c] : 0.0;
    }
    for (int t = tid; t < 6 * cnt; t += blockDim.x) {
      int row = t / cnt, l = t % cnt;
      sC[row][l] = cf[(int64_t)row * L + lc + l];
    }
    __syncthreads();
    // Degree l of the chunk has parity (lc + l - m) & 1 = l & 1 (chunks start at even offsets
    // from m), so pairs of degrees keep every accumulator index constant (registers, no scratch).
    auto acc = [&](double* Q, double* U, int l) __attribute__((always_inline)) {
      const double pi_ = sPi[l][ti][0], ri = sPi[l][ti][1], tI = sPi[l][ti][2];
      const double pj = sPj[l][tj][0], rj = sPj[l][tj][1], tJ = sPj[l][tj][2];
      const double a1 = sC[0][l], a2 = sC[1][l], a3 = sC[2][l], a4 = sC[3][l];
      const double b1 = sC[4][l], b2 = sC[5][l];
      // IQ part: Pi B_l diag(1,1,0,0) Pj
      Q[0] += pi_ * a1 * pj;
      Q[1] += pi_ * b1 * rj;
      Q[2] += pi_ * b1 * tJ;
      Q[3] += ri * b1 * pj;
      Q[4] += ri * a2 * rj;
      Q[5] += ri * a2 * tJ;
      Q[6] += tI * b1 * pj;
      Q[7] += tI * a2 * rj;
      Q[8] += tI * a2 * tJ;
      // UV part: Pi B_l diag(0,0,1,1) Pj
      U[0] += tI * a3 * tJ;
      U[1] += tI * a3 * rj;
      U[2] += tI * b2 * pj;
      U[3] += ri * a3 * tJ;
      U[4] += ri * a3 * rj;
      U[5] += ri * b2 * pj;
      U[6] += pi_ * b2 * tJ;
      U[7] += pi_ * b2 * rj;
      U[8] += pi_ * a4 * pj;
    };
    int l = 0;
    for (; l + 1 < cnt; l += 2) {
      acc(q[0], u[0], l);
      acc(q[1], u[1], l + 1);
    }
    if (l < cnt) acc(q[0], u[0], l);
  }
  if (i >= N || j >= N) return;

  // Block matrices (4x4, row r, column c) of the two parts for parity e.
  auto iq = [&](int e, int r, int c) -> double {
    if (r == 3 || c == 3) return 0.0;
    const double* Q = q[e];
    const double v[3][3] = {{Q[0], Q[1], -Q[2]}, {Q[3], Q[4], -Q[5]}, {-Q[6], -Q[7], Q[8]}};
    return v[r][c];
  };
  auto uv = [&](int e, int r, int c) -> double {
    if (r == 0 || c == 0) return 0.0;
    const double* U = u[e];
    const double v[3][3] = {{U[0], -U[1], -U[2]}, {-U[3], U[4], U[5]}, {U[6], -U[7], U[8]}};
    return v[r - 1][c - 1];
  };

  const double w = fmin(omega[it.layer], kOmegaMax);
  const double mui = quad[ly.quad_off + i];
  const double alj = quad[ly.quad_off + N + j];
  double* E = ws + it.ws + (int64_t)kBufE * n * n;
  double* F = ws + it.ws + (int64_t)kBufF * n * n;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      // S+ = 2 (IQ_even + UV_odd), S- = 2 (UV_even + IQ_odd)
      const double sp = 2.0 * (iq(0, r, c) + uv(1, r, c));
      const double sm = 2.0 * (uv(0, r, c) + iq(1, r, c));
      const double dl = (i == j && r == c) ? 1.0 : 0.0;
      const int64_t idx = (int64_t)(4 * i + r) * n + 4 * j + c;
      E[idx] = (dl - 0.5 * w * sp * alj) / mui;
      F[idx] = (dl - 0.5 * w * sm * alj) / mui;
    }
  }
}

}  // namespace vbrdf

namespace vbrdf {

// ---- off-node incidence: Legendre table and source at the incident cosines mu0_j

// Legendre tables of order m at the incident cosines (which = 0: leg0[(l * n_mu0 + j) * 3 + c]) or
// at the extra outgoing cosines (which = 1: [(l * n_x + o) * 3 + c]), as k_legendre at the nodes.
__global__ __launch_bounds__(kLegThreads) void k_beam_legendre(const Item* items, const double* xs, int n_x,
                                                               int n_mu0, int which, double* ws,
                                                               const int32_t* status) {
  const Item it = items[blockIdx.x];
  if (status[it.layer] != 0) return;
  const int L = it.L, m = it.m;
  double* leg = ws + it.ws + (which ? beam_out_leg_off(it.n, it.N, it.L, n_mu0) : beam_leg_off(it.n, it.N, it.L));
  const int n_mu0_ = n_x;
  const int seq = threadIdx.x / 128, j = threadIdx.x % 128;
  if (j < n_mu0_) {
    const double x = xs[j];
    const int nn = seq == 0 ? 0 : (seq == 1 ? 2 : -2);
    WSeq q{m, nn, seq == 0 ? m : (m > 2 ? m : 2), 0.0, 0.0};
    for (int l = 0; l < L; ++l) {
      const double d = wseq_value(q, l, x);
      leg[((int64_t)l * n_mu0_ + j) * 3 + seq] = (l < m) ? 0.0 : d;
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < L * n_mu0_; t += blockDim.x) {
    double* o = leg + (int64_t)t * 3;
    const double dp = o[1], dm = o[2];
    o[1] = -0.5 * (dp + dm);
    o[2] = -0.5 * (dp - dm);
  }
}

// The order-m source of a unit Stokes beam e_p at mu0_j (Sec. 2.C, eq. 28; the per-order phase
// function normalisation of the rest of the solve): X(+-mu_i) = omega/(2 pi) A^m(+-mu_i, mu0_j) e_p.
// In the half-size form only the mirrored sum and difference enter, X_s = X+ + D X- and
// X_d = X+ - D X-, which are the blocks of S+ and S- with their second Legendre factor taken at
// mu0_j. Written scaled for the particular solve: kBufB0 = M^-1 X_s, kBufB1 = M^-1 X_d / mu0_j
// (column 4 j + p); the columns of the n x n buffers beyond the beams are zeroed. Grid as
// k_assemble, the column tiles running over the N node columns.
__global__ __launch_bounds__(256) void k_beam_source(const Item* items, const Layer* layers, const double* quad,
                                                     const double* omega, const double* coef, const double* mu0,
                                                     int n_mu0, double* ws, const int32_t* status) {
  const Item it = items[blockIdx.z];
  if (status[it.layer] != 0) return;
  const int N = it.N, L = it.L, m = it.m, n = it.n;
  const int i0 = blockIdx.y * kAsmTile, j0 = blockIdx.x * kAsmTile;
  if (i0 >= N || j0 >= N) return;
  const Layer ly = layers[it.layer];
  const double* leg = ws + it.ws + leg_off(n);
  const double* leg0 = ws + it.ws + beam_leg_off(n, N, L);
  const double* cf = coef + ly.coef_off;
  double* X0 = buf_ptr(ws, it, kBufB0);
  double* X1 = buf_ptr(ws, it, kBufB1);
  __shared__ double sPi[kAsmChunk][kAsmTile][3];
  __shared__ double sPj[kAsmChunk][kAsmTile][3];
  __shared__ double sC[6][kAsmChunk];
  const int tid = threadIdx.x;
  const int ti = tid / kAsmTile, tj = tid % kAsmTile;
  const int i = i0 + ti, j = j0 + tj;
  if (j0 >= n_mu0) {  // columns beyond the beams
    if (i < N && j < N)
      for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
          const int64_t idx = (int64_t)(4 * i + r) * n + 4 * j + c;
          X0[idx] = 0.0;
          X1[idx] = 0.0;
        }
    return;
  }
  double q[2][9], u[2][9];
#pragma unroll
  for (int e = 0; e < 2; ++e)
#pragma unroll
    for (int k = 0; k < 9; ++k) { q[e][k] = 0.0; u[e][k] = 0.0; }
  for (int lc = m; lc < L; lc += kAsmChunk) {
    const int cnt = min(kAsmChunk, L - lc);
    __syncthreads();
    for (int t = tid; t < cnt * kAsmTile * 3; t += blockDim.x) {
      int l = t / (kAsmTile * 3), r = t % (kAsmTile * 3);
      int a = r / 3, c = r % 3;
      sPi[l][a][c] = (i0 + a < N) ? leg[((int64_t)(lc + l) * N + i0 + a) * 3 + c] : 0.0;
      sPj[l][a][c] = (j0 + a < n_mu0) ? leg0[((int64_t)(lc + l) * n_mu0 + j0 + a) * 3 + c] : 0.0;
    }
    for (int t = tid; t < 6 * cnt; t += blockDim.x) {
      int row = t / cnt, l = t % cnt;
      sC[row][l] = cf[(int64_t)row * L + lc + l];
    }
    __syncthreads();
    auto acc = [&](double* Q, double* U, int l) __attribute__((always_inline)) {
      const double pi_ = sPi[l][ti][0], ri = sPi[l][ti][1], tI = sPi[l][ti][2];
      const double pj = sPj[l][tj][0], rj = sPj[l][tj][1], tJ = sPj[l][tj][2];
      const double a1 = sC[0][l], a2 = sC[1][l], a3 = sC[2][l], a4 = sC[3][l];
      const double b1 = sC[4][l], b2 = sC[5][l];
      Q[0] += pi_ * a1 * pj;
      Q[1] += pi_ * b1 * rj;
      Q[2] += pi_ * b1 * tJ;
      Q[3] += ri * b1 * pj;
      Q[4] += ri * a2 * rj;
      Q[5] += ri * a2 * tJ;
      Q[6] += tI * b1 * pj;
      Q[7] += tI * a2 * rj;
      Q[8] += tI * a2 * tJ;
      U[0] += tI * a3 * tJ;
      U[1] += tI * a3 * rj;
      U[2] += tI * b2 * pj;
      U[3] += ri * a3 * tJ;
      U[4] += ri * a3 * rj;
      U[5] += ri * b2 * pj;
      U[6] += pi_ * b2 * tJ;
      U[7] += pi_ * b2 * rj;
      U[8] += pi_ * a4 * pj;
    };
    int l = 0;
    for (; l + 1 < cnt; l += 2) {
      acc(q[0], u[0], l);
      acc(q[1], u[1], l + 1);
    }
    if (l < cnt) acc(q[0], u[0], l);
  }
  if (i >= N || j >= N) return;
  auto iq = [&](int e, int r, int c) -> double {
    if (r == 3 || c == 3) return 0.0;
    const double* Q = q[e];
    const double v[3][3] = {{Q[0], Q[1], -Q[2]}, {Q[3], Q[4], -Q[5]}, {-Q[6], -Q[7], Q[8]}};
    return v[r][c];
  };
  auto uv = [&](int e, int r, int c) -> double {
    if (r == 0 || c == 0) return 0.0;
    const double* U = u[e];
    const double v[3][3] = {{U[0], -U[1], -U[2]}, {-U[3], U[4], U[5]}, {U[6], -U[7], U[8]}};
    return v[r - 1][c - 1];
  };
  const bool beam = j < n_mu0;
  const double w = fmin(omega[it.layer], kOmegaMax);
  const double sc = w / (2.0 * 3.141592653589793) / quad[ly.quad_off + i];
  const double inv0 = beam ? 1.0 / mu0[j] : 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double sp = 2.0 * (iq(0, r, c) + uv(1, r, c));
      const double sm = 2.0 * (uv(0, r, c) + iq(1, r, c));
      const int64_t idx = (int64_t)(4 * i + r) * n + 4 * j + c;
      X0[idx] = beam ? sc * sp : 0.0;
      X1[idx] = beam ? sc * sm * inv0 : 0.0;
    }
  }
}

}  // namespace vbrdf

namespace vbrdf {

// Sums over degrees l of P_l^m(x) B_l P_l^m(y)^T split by parity of l - m into the IQ part and the UV
// part (as in k_assemble) for one pair of cosines, from Legendre rows li(l) and lj(l).
struct ParitySums {
  double q[2][9], u[2][9];
  __device__ void clear() {
    for (int e = 0; e < 2; ++e)
      for (int k = 0; k < 9; ++k) { q[e][k] = 0.0; u[e][k] = 0.0; }
  }
  __device__ void add(int e, const double* li, const double* lj, const double* c) {
    const double pi_ = li[0], ri = li[1], tI = li[2], pj = lj[0], rj = lj[1], tJ = lj[2];
    const double a1 = c[0], a2 = c[1], a3 = c[2], a4 = c[3], b1 = c[4], b2 = c[5];
    double* Q = q[e];
    double* U = u[e];
    Q[0] += pi_ * a1 * pj; Q[1] += pi_ * b1 * rj; Q[2] += pi_ * b1 * tJ;
    Q[3] += ri * b1 * pj;  Q[4] += ri * a2 * rj;  Q[5] += ri * a2 * tJ;
    Q[6] += tI * b1 * pj;  Q[7] += tI * a2 * rj;  Q[8] += tI * a2 * tJ;
    U[0] += tI * a3 * tJ;  U[1] += tI * a3 * rj;  U[2] += tI * b2 * pj;
    U[3] += ri * a3 * tJ;  U[4] += ri * a3 * rj;  U[5] += ri * b2 * pj;
    U[6] += pi_ * b2 * tJ; U[7] += pi_ * b2 * rj; U[8] += pi_ * a4 * pj;
  }
  __device__ double iq(int e, int r, int c) const {
    if (r == 3 || c == 3) return 0.0;
    const double* Q = q[e];
    const double v[3][3] = {{Q[0], Q[1], -Q[2]}, {Q[3], Q[4], -Q[5]}, {-Q[6], -Q[7], Q[8]}};
    return v[r][c];
  }
  __device__ double uv(int e, int r, int c) const {
    if (r == 0 || c == 0) return 0.0;
    const double* U = u[e];
    const double v[3][3] = {{U[0], -U[1], -U[2]}, {-U[3], U[4], U[5]}, {U[6], -U[7], U[8]}};
    return v[r - 1][c - 1];
  }
  // A^m(x, y) and A^m(x, -y) D, D = diag(1, 1, -1, -1)
  __device__ double same(int r, int c) const { return iq(0, r, c) + iq(1, r, c) + uv(0, r, c) + uv(1, r, c); }
  __device__ double cross(int r, int c) const { return iq(0, r, c) + uv(1, r, c) - uv(0, r, c) - iq(1, r, c); }
};

// Source rows of the reconstruction (eq. 38) at the extra outgoing cosines mu_o, mirrored storage:
// kBufB5 = P_cross, kBufB6 = P_same with P_same[(o, r), (j, p)] = omega/2 alpha_j A^m(mu_o, mu_j)[r, p]
// and P_cross = omega/2 alpha_j [A^m(mu_o, -mu_j) D][r, p]; rows beyond 4 n_out are zeroed. One thread
// per (o, j) block; grid over (node tiles, outgoing tiles, items).
__global__ __launch_bounds__(256) void k_recon_rows(const Item* items, const Layer* layers, const double* quad,
                                                    const double* omega, const double* coef, int n_mu0, int n_out,
                                                    double* ws, const int32_t* status) {
  const Item it = items[blockIdx.z];
  if (status[it.layer] != 0) return;
  const int N = it.N, L = it.L, m = it.m, n = it.n;
  const int o = blockIdx.y * 16 + threadIdx.x / 16, j = blockIdx.x * 16 + threadIdx.x % 16;
  if (o >= N || j >= N) return;
  double* Pc = buf_ptr(ws, it, kBufB5);
  double* Ps = buf_ptr(ws, it, kBufB6);
  if (o >= n_out) {
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c) {
        Pc[(int64_t)(4 * o + r) * n + 4 * j + c] = 0.0;
        Ps[(int64_t)(4 * o + r) * n + 4 * j + c] = 0.0;
      }
    return;
  }
  const Layer ly = layers[it.layer];
  const double* leg = ws + it.ws + leg_off(n);
  const double* lego = ws + it.ws + beam_out_leg_off(n, N, L, n_mu0);
  const double* cf = coef + ly.coef_off;
  ParitySums S;
  S.clear();
  for (int l = m; l < L; ++l) {
    const double c6[6] = {cf[l], cf[L + l], cf[2 * L + l], cf[3 * L + l], cf[4 * L + l], cf[5 * L + l]};
    S.add((l - m) & 1, lego + ((int64_t)l * n_out + o) * 3, leg + ((int64_t)l * N + j) * 3, c6);
  }
  const double w = 0.5 * fmin(omega[it.layer], kOmegaMax) * quad[ly.quad_off + N + j];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      const int64_t idx = (int64_t)(4 * o + r) * n + 4 * j + c;
      Pc[idx] = w * S.cross(r, c);
      Ps[idx] = w * S.same(r, c);
    }
}

// Reconstructed upward radiance at the top towards -mu_o per unit beam e_p at mu0_j (physical
// storage) into kBufB5: D [Omodes + (P_cross Z+ + P_same D Z- + D X(-mu_o)) f0], with Omodes in
// kBufB2, the particular part's rows in kBufB7, D X(-mu_o) = omega/(2 pi) A^m(mu_o, -mu0_j) D e_p and
// f0 = int_0^tau0 exp(-t/mu0) exp(-t/mu_o) dt / mu_o. One thread per (o, j).
__global__ void k_recon_out(const Item* items, const Layer* layers, const double* omega, const double* coef,
                            const double* tau, const double* mu0, int n_mu0, const double* mu_out, int n_out,
                            double* ws, const int32_t* status) {
  const Item it = items[blockIdx.y];
  if (status[it.layer] != 0) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_out * n_mu0) return;
  const int o = t / n_mu0, j = t % n_mu0;
  const int N = it.N, L = it.L, m = it.m, n = it.n;
  const Layer ly = layers[it.layer];
  const double* lego = ws + it.ws + beam_out_leg_off(n, N, L, n_mu0);
  const double* leg0 = ws + it.ws + beam_leg_off(n, N, L);
  const double* cf = coef + ly.coef_off;
  ParitySums S;
  S.clear();
  for (int l = m; l < L; ++l) {
    const double c6[6] = {cf[l], cf[L + l], cf[2 * L + l], cf[3 * L + l], cf[4 * L + l], cf[5 * L + l]};
    S.add((l - m) & 1, lego + ((int64_t)l * n_out + o) * 3, leg0 + ((int64_t)l * n_mu0 + j) * 3, c6);
  }
  const double sc = fmin(omega[it.layer], kOmegaMax) / (2.0 * 3.141592653589793);
  const double m0 = mu0[j], mo = mu_out[o], tau0 = tau[it.layer];
  const double f0 = m0 * (-expm1(-tau0 * (1.0 / m0 + 1.0 / mo))) / (m0 + mo);
  const double* Om = buf_ptr(ws, it, kBufB2);
  const double* Pz = buf_ptr(ws, it, kBufB7);
  double* out = buf_ptr(ws, it, kBufB5);
  for (int r = 0; r < 4; ++r)
    for (int p = 0; p < 4; ++p) {
      const int64_t idx = (int64_t)(4 * o + r) * n + 4 * j + p;
      const double v = Om[idx] + (Pz[idx] + sc * S.cross(r, p)) * f0;
      out[idx] = r >= 2 ? -v : v;
    }
}

}  // namespace vbrdf
