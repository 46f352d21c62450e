// Black-base boundary solve and emergent response for all incident (node, Stokes) pairs.
//
// With U the eigenvectors of G = F~ E~ (eigenvalues lambda_j = 1/nu_j^2, Re nu_j > 0) and
// V = E~ U, the mode vectors of eq. 45 are Phi+- = (U +- V diag(nu)) / 2, the downward field being
// Phi+ and the D-mirrored upward field Phi- (Sec. 2.C, eq. 24-25). Zero incoming diffuse light at
// the top and at the black base (Sec. 3.C, eq. 49-56) gives the block system
// [[Phi+, Phi- Ex], [Phi- Ex, Phi+]] [a; b] = [R0; 0] with Ex = diag(exp(-tau0/nu_j)). Its
// symmetric/antisymmetric halves decouple; scaling the columns by 1/(1 +- exp(-tau0/nu_j)) turns
// them into S' = U + V D_s and T' = U + V D_t with D_s = diag(nu tanh(tau0/(2 nu))) and
// D_t = diag(nu coth(tau0/(2 nu))). The upward radiance at the top is then
//     R^m = Delta [U S'^-1 + U T'^-1 - I] R0,
// Delta = I_N (x) diag(1, 1, -1, -1), R0 = diag(1 / (pi alpha_q)) (x) I4: one column per incident
// node q and unit Stokes vector e_p, the incident beam being carried as a discrete stream whose
// quadrature-weighted scattering equals the source of eq. 14. A complex pair (columns j, j+1 =
// real and imaginary parts) is mixed with the complex D of lambda_j, which is the same
// real-basis change on numerator and denominator.
#include "vbrdf_internal.hpp"

namespace vbrdf {

// complex tanh(z) for Re z > 0, written with exp(-2 Re z) so that it never overflows
__device__ inline void ctanh_pos(double x, double y, double& tr, double& ti) {
  const double e2 = exp(-2.0 * x), e4 = e2 * e2;
  const double c2 = cos(2.0 * y), s2 = sin(2.0 * y);
  const double den = 1.0 + e4 + 2.0 * e2 * c2;
  tr = (1.0 - e4) / den;
  ti = 2.0 * e2 * s2 / den;
}

// Per column: lam -> (d_s, d_t) real/imag parts, stored in extras [6n, 10n).
__global__ void k_colscal(const Item* items, const double* tau, double* ws, int32_t* status) {
  const Item it = items[blockIdx.y];
  if (status[it.layer] != 0) return;
  const int n = it.n;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double* ex = ws + it.ws + extras_off(n);
  const double lr = ex[j], li = ex[n + j];
  double* dsr = ex + 6 * n;
  double* dsi = ex + 7 * n;
  double* dtr = ex + 8 * n;
  double* dti = ex + 9 * n;
  const double t0 = tau[it.layer];
  if (li == 0.0) {
    if (!(lr > 0.0) || !isfinite(lr)) {
      status[it.layer] = -5;
      return;
    }
    const double sq = sqrt(lr);           // 1/nu
    const double z = 0.5 * t0 * sq;       // tau0 / (2 nu)
    const double th = -expm1(-2.0 * z) / (1.0 + exp(-2.0 * z));
    dsr[j] = th / sq;
    dtr[j] = 1.0 / (th * sq);
    dsi[j] = 0.0;
    dti[j] = 0.0;
  } else {
    // principal square root of lambda: Re > 0
    const double r = hypot(lr, li);
    double sr = sqrt(0.5 * (r + lr));
    double si = 0.5 * li / sr;
    if (!(sr > 0.0) || !isfinite(sr)) {
      status[it.layer] = -5;
      return;
    }
    double tr, ti;
    ctanh_pos(0.5 * t0 * sr, 0.5 * t0 * si, tr, ti);
    // d_s = tanh / sqrt(lambda), d_t = 1 / (tanh * sqrt(lambda))
    const double den = sr * sr + si * si;
    const double ir = sr / den, ii = -si / den;  // 1/sqrt(lambda)
    dsr[j] = tr * ir - ti * ii;
    dsi[j] = tr * ii + ti * ir;
    const double pr = tr * sr - ti * si, pi = tr * si + ti * sr;  // tanh * sqrt(lambda)
    const double pd = pr * pr + pi * pi;
    dtr[j] = pr / pd;
    dti[j] = -pi / pd;
  }
}

// S' (into kBufZ) and T' (into kBufX), element-wise over the n x n block of one item.
__global__ void k_bcbuild(const Item* items, double* ws, const int32_t* status) {
  const Item it = items[blockIdx.z];
  if (status[it.layer] != 0) return;
  const int n = it.n;
  const int i = blockIdx.y * 16 + threadIdx.y;
  const int j = blockIdx.x * 16 + threadIdx.x;
  if (i >= n || j >= n) return;
  double* base = ws + it.ws;
  const double* U = base + (int64_t)kBufU * n * n;
  const double* V = base + (int64_t)kBufF * n * n;
  double* S = base + (int64_t)kBufZ * n * n;
  double* T = base + (int64_t)kBufX * n * n;
  const double* ex = base + extras_off(n);
  const double li = ex[n + j];
  const int64_t idx = (int64_t)i * n + j;
  if (li == 0.0) {
    const double u = U[idx], v = V[idx];
    S[idx] = u + v * ex[6 * n + j];
    T[idx] = u + v * ex[8 * n + j];
  } else {
    const int jf = (li > 0.0) ? j : j - 1;  // first column of the pair
    const double vr = V[(int64_t)i * n + jf], vi = V[(int64_t)i * n + jf + 1];
    const double sr = ex[6 * n + jf], si = ex[7 * n + jf], tr = ex[8 * n + jf], ti = ex[9 * n + jf];
    if (j == jf) {
      S[idx] = U[idx] + vr * sr - vi * si;
      T[idx] = U[idx] + vr * tr - vi * ti;
    } else {
      S[idx] = U[idx] + vr * si + vi * sr;
      T[idx] = U[idx] + vr * ti + vi * tr;
    }
  }
}

constexpr int kRows = 16;  // right-hand-side rows per LDS pass

__device__ inline void block_argmax(double v, int idx, double* sv, int* si) {
  // leaves the winner in sv[0], si[0]; ties resolve to the smaller index
  for (int o = 32; o > 0; o >>= 1) {
    if (o < (int)blockDim.x) {
      const double ov = __shfl_xor(v, o);
      const int oi = __shfl_xor(idx, o);
      if (ov > v || (ov == v && oi < idx)) {
        v = ov;
        idx = oi;
      }
    }
  }
  if ((threadIdx.x & 63) == 0) {
    sv[threadIdx.x >> 6] = v;
    si[threadIdx.x >> 6] = idx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 1; w < nw; ++w)
      if (sv[w] > sv[0] || (sv[w] == sv[0] && si[w] < si[0])) {
        sv[0] = sv[w];
        si[0] = si[w];
      }
  }
  __syncthreads();
}

// LU factorisation with partial pivoting of A (S' or T') and the right division Y = U A^-1.
// blockIdx.y selects S' (0) or T' (1). With P^T A = L Uu (row perm[k] of A at position k),
// Y A = U becomes W L Uu = U for W = Y P, i.e. Y[:, perm[k]] = W[:, k].
__global__ __launch_bounds__(256) void k_rdiv(const Item* items, double* ws, int32_t* status) {
  const Item it = items[blockIdx.x];
  if (status[it.layer] != 0) return;
  const int n = it.n;
  const int which = blockIdx.y;
  double* base = ws + it.ws;
  double* Ag = base + (int64_t)(which == 0 ? kBufZ : kBufX) * n * n;
  const double* U = base + (int64_t)kBufU * n * n;
  double* Y = base + (int64_t)(which == 0 ? kBufYS : kBufYT) * n * n;

  __shared__ double smem[kLdsMaxn * (kLdsMaxn + 1) + kRows * (kLdsMaxn + 1) > kRows * (kMaxn + 1)
                            ? kLdsMaxn * (kLdsMaxn + 1) + kRows * (kLdsMaxn + 1)
                            : kRows * (kMaxn + 1)];
  __shared__ int perm[kMaxn];
  __shared__ double invd[kMaxn];
  __shared__ double redv[8];
  __shared__ int redi[8];
  __shared__ int sflag;

  const int tid = threadIdx.x, NT = blockDim.x;
  const bool in_lds = n <= kLdsMaxn;
  double* A = in_lds ? smem : Ag;
  const int64_t ld = in_lds ? n + 1 : n;
  const int ldb = n + 1;  // padded: rows of the right-hand-side tile fall in distinct LDS banks
  double* B = in_lds ? smem + kLdsMaxn * (kLdsMaxn + 1) : smem;  // [kRows][n + 1]
#define AA(r, c) A[(int64_t)(r) * ld + (c)]
#define BB(r, c) B[(int64_t)(r) * ldb + (c)]

  if (in_lds)
    for (int t = tid; t < n * n; t += NT) AA(t / n, t % n) = Ag[t];
  for (int i = tid; i < n; i += NT) perm[i] = i;
  if (tid == 0) sflag = 0;
  __syncthreads();

  for (int k = 0; k < n; ++k) {
    double best = -1.0;
    int bi = k;
    for (int i = k + tid; i < n; i += NT) {
      const double v = fabs(AA(i, k));
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    block_argmax(best, bi, redv, redi);
    const int p = redi[0];
    const double pv = redv[0];
    if (!(pv > 0.0) || !isfinite(pv)) {
      if (tid == 0) sflag = 1;
      break;  // uniform: every thread read the same pivot
    }
    if (p != k) {
      for (int c = tid; c < n; c += NT) {
        const double t = AA(k, c);
        AA(k, c) = AA(p, c);
        AA(p, c) = t;
      }
      if (tid == 0) {
        const int t = perm[k];
        perm[k] = perm[p];
        perm[p] = t;
      }
    }
    __syncthreads();
    const double inv = 1.0 / AA(k, k);
    for (int i = k + 1 + tid; i < n; i += NT) AA(i, k) *= inv;
    if (tid == 0) invd[k] = inv;
    __syncthreads();
    const int m = n - k - 1;
    for (int t = tid; t < m * m; t += NT) {
      const int i = k + 1 + t / m, c = k + 1 + t % m;
      AA(i, c) -= AA(i, k) * AA(k, c);
    }
    __syncthreads();
  }
  __syncthreads();
  if (sflag) {
    if (tid == 0) status[it.layer] = -5;
    return;
  }

  // right division, kRows rows of U per pass
  for (int r0 = 0; r0 < n; r0 += kRows) {
    const int nr = min(kRows, n - r0);
    for (int t = tid; t < kRows * n; t += NT) {
      const int r = t / n, c = t % n;
      BB(r, c) = (r < nr) ? U[(int64_t)(r0 + r) * n + c] : 0.0;
    }
    __syncthreads();
    // z Uu = u, column by column: z_j = u_j / Uu_jj, then u_c -= z_j Uu_jc for c > j
    for (int j = 0; j + 1 < n; ++j) {
      const int m = n - j - 1;
      const double ijj = invd[j];
      for (int t = tid; t < kRows * m; t += NT) {
        const int r = t % kRows, c = j + 1 + t / kRows;
        BB(r, c) -= BB(r, j) * ijj * AA(j, c);
      }
      __syncthreads();
    }
    for (int t = tid; t < kRows * n; t += NT) {
      const int r = t % kRows, c = t / kRows;
      BB(r, c) *= invd[c];
    }
    __syncthreads();
    // w L = z with unit lower L, from the last column: w_j = z_j, then z_c -= w_j L_jc for c < j
    for (int j = n - 1; j >= 1; --j) {
      for (int t = tid; t < kRows * j; t += NT) {
        const int r = t % kRows, c = t / kRows;
        BB(r, c) -= BB(r, j) * AA(j, c);
      }
      __syncthreads();
    }
    for (int t = tid; t < nr * n; t += NT) {
      const int r = t / n, k = t % n;
      Y[(int64_t)(r0 + r) * n + perm[k]] = BB(r, k);
    }
    __syncthreads();
  }
#undef BB
#undef AA
}

// R^m = Delta (Y_S + Y_T - I) R0, written over kBufE.
__global__ void k_response(const Item* items, const Layer* layers, const double* quad, double* ws,
                           const int32_t* status) {
  const Item it = items[blockIdx.z];
  if (status[it.layer] != 0) return;
  const int n = it.n;
  const int a = blockIdx.y * 16 + threadIdx.y;
  const int b = blockIdx.x * 16 + threadIdx.x;
  if (a >= n || b >= n) return;
  const Layer ly = layers[it.layer];
  double* base = ws + it.ws;
  const int64_t idx = (int64_t)a * n + b;
  const double y = base[(int64_t)kBufYS * n * n + idx] + base[(int64_t)kBufYT * n * n + idx] - (a == b ? 1.0 : 0.0);
  const double alq = quad[ly.quad_off + it.N + b / 4];
  const double sgn = ((a & 3) >= 2) ? -1.0 : 1.0;
  base[(int64_t)kBufE * n * n + idx] = sgn * y / (3.141592653589793 * alq);
}

}  // namespace vbrdf
