// Adjoint of the per-order solve: gradients of a loss on F_r with respect to the optical thickness,
// the albedo and the phase-matrix expansion coefficients.
//
// The forward pass of one order (Sec. 3.A-3.C) is written as a chain of matrix operations on the
// half-size matrices E~ = M^-1 (I - omega/2 S+ W), F~ = M^-1 (I - omega/2 S- W) (eq. 41-42):
//   G = F~ E~ = U Lambda U^-1                      (eq. 43-45; Lambda block diagonal, real basis)
//   F_s = f_s(G), F_t = f_t(G),  f_s(l) = nu tanh(tau0 / 2 nu), f_t(l) = nu coth(tau0 / 2 nu),
//         nu = l^-1/2, so that U S'^-1 = (I + E~ F_s)^-1 = P_s and U T'^-1 = P_t (eq. 49-56),
//   R^m = Delta (P_s + P_t - I) R0,    F_r = sum_m c_m tau(m dphi) R^m / (2 mu_q)   (eq. 12, 39).
// Reverse mode, per order, with X-bar the gradient of the loss with respect to X:
//   Q = Delta R-bar R0 (= P_s-bar = P_t-bar),   A_s-bar = -P_s^T Q P_s^T,
//   E~-bar = A_s-bar F_s^T + A_t-bar F_t^T + F~^T G-bar,   F_s-bar = E~^T A_s-bar,
//   G-bar = U^-T [L_s*(U^T F_s-bar U^-T) + L_t*(U^T F_t-bar U^-T)] U^T,   F~-bar = G-bar E~^T,
//   tau0-bar = <U^T F_s-bar U^-T, d f_s / d tau0 (Lambda)> + (same for t),
//   omega-bar = <E~-bar, (E~ - M^-1) / omega> + <F~-bar, (F~ - M^-1) / omega>,
//   S+-bar = -(omega/2) M^-1 E~-bar W,  S--bar likewise from F~-bar,
//   B_l-bar = sum_ij P_l(mu_i) S+-bar_ij P_l(mu_j) (I + s D) + (same for S-, I - s D), s = (-1)^(l-m).
// L_f* is the adjoint of the Frechet derivative of the matrix function f at Lambda (the
// Daleckii-Krein form): it is the Frechet derivative at Lambda^T. On a pair of blocks a != b of the
// block-diagonal Lambda it solves Lambda_a^T Y - Y Lambda_b^T = f(Lambda_a^T) X - X f(Lambda_b^T)
// (for two real eigenvalues: Y = X (f(l_a) - f(l_b)) / (l_a - l_b), the derivative at the midpoint
// when they nearly coincide); on a diagonal block it is f'(l) X for a real eigenvalue and, for a
// complex pair z = p + i q, f'(z) on the part of X that commutes with J = [[0, 1], [-1, 0]] and
// Im f(z) / q on the part that anticommutes. The GEMMs run on k_gemm; these kernels hold the
// element-wise, per-block and reduction steps.
#include "vbrdf_internal.hpp"

namespace vbrdf {

namespace {

struct Cz {
  double re, im;
};
__device__ inline Cz cz(double r, double i = 0.0) { return {r, i}; }
__device__ inline Cz operator+(Cz a, Cz b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline Cz operator-(Cz a, Cz b) { return {a.re - b.re, a.im - b.im}; }
__device__ inline Cz operator*(Cz a, Cz b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline Cz operator*(double s, Cz a) { return {s * a.re, s * a.im}; }
__device__ inline Cz cinv(Cz a) {
  const double d = a.re * a.re + a.im * a.im;
  return {a.re / d, -a.im / d};
}
__device__ inline Cz operator/(Cz a, Cz b) { return a * cinv(b); }
// principal square root (Re >= 0)
__device__ inline Cz csqrt_p(Cz z) {
  const double r = hypot(z.re, z.im);
  double sr = sqrt(0.5 * (r + z.re));
  double si = 0.5 * z.im / sr;
  if (z.re < 0.0) {  // avoid cancellation: take the imaginary part first
    si = copysign(sqrt(0.5 * (r - z.re)), z.im);
    sr = 0.5 * z.im / si;
  }
  return {sr, si};
}

// The boundary functions of one eigenvalue z: f_s = nu tanh x, f_t = nu coth x with
// nu = 1 / sqrt(z) and x = tau0 / (2 nu), their z-derivatives and their tau0-derivatives.
struct FVals {
  Cz fs, ft, dfs, dft, tfs, tft;
};
__device__ inline FVals boundary_functions(Cz z, double tau0) {
  const Cz w = csqrt_p(z);  // 1 / nu
  const Cz x = (0.5 * tau0) * w;
  // tanh x = (1 - e^-2x) / (1 + e^-2x), |e^-2x| < 1 since Re x > 0
  const double e = exp(-2.0 * x.re);
  double sn, cs;
  sincos(-2.0 * x.im, &sn, &cs);
  const Cz em = {e * cs, e * sn};
  const Cz t = (cz(1.0) - em) / (cz(1.0) + em);
  const Cz sech2 = cz(1.0) - t * t;
  const Cz t2 = t * t;
  const Cz w3 = w * w * w;
  FVals f;
  f.fs = t / w;
  f.ft = cinv(w * t);
  f.dfs = -0.5 * ((t - x * sech2) / w3);
  f.dft = -0.5 * ((t + x * sech2) / (w3 * t2));
  f.tfs = 0.5 * sech2;
  f.tft = -0.5 * (sech2 / t2);
  return f;
}

// A 1x1 or 2x2 block of Lambda: p (+ q J), starting at column j0 of size s.
struct Blk {
  int j0, s;
  double p, q;
};
__device__ inline Blk block_at(const double* lre, const double* lim, int j) {
  Blk b;
  b.j0 = lim[j] < 0.0 ? j - 1 : j;
  b.s = lim[b.j0] > 0.0 ? 2 : 1;
  b.p = lre[b.j0];
  b.q = b.s == 2 ? lim[b.j0] : 0.0;
  return b;
}

// 2 x 2 real matrices (row-major) of the form a I + b J and their products with general ones.
__device__ inline void aij_left(double a, double b, const double* X, double* out) {  // (aI + bJ) X
  out[0] = a * X[0] + b * X[2];
  out[1] = a * X[1] + b * X[3];
  out[2] = -b * X[0] + a * X[2];
  out[3] = -b * X[1] + a * X[3];
}
__device__ inline void aij_right(double a, double b, const double* X, double* out) {  // X (aI + bJ)
  out[0] = a * X[0] - b * X[1];
  out[1] = b * X[0] + a * X[1];
  out[2] = a * X[2] - b * X[3];
  out[3] = b * X[2] + a * X[3];
}
// (p I + q J)^-1 C from the left
__device__ inline void aij_solve_left(double p, double q, const double* C, double* X) {
  const double d = 1.0 / (p * p + q * q);
  aij_left(p * d, -q * d, C, X);
}

// Solve A Y - Y B = C for blocks A = pa I + qa J (sa x sa) and B = pb I + qb J (sb x sb); C, Y are
// 2 x 2 row-major with the unused entries zero.
__device__ inline void block_sylvester(double pa, double qa, int sa, double pb, double qb, int sb, const double* C,
                                       double* Y) {
  for (int k = 0; k < 4; ++k) Y[k] = 0.0;
  if (sa == 1 && sb == 1) {
    Y[0] = C[0] / (pa - pb);
  } else if (sa == 2 && sb == 1) {  // ((pa - pb) I + qa J) y = c, y a column (entries 0 and 2)
    const double p = pa - pb, q = qa, d = 1.0 / (p * p + q * q);
    Y[0] = d * (p * C[0] - q * C[2]);
    Y[2] = d * (q * C[0] + p * C[2]);
  } else if (sa == 1 && sb == 2) {  // y ((pa - pb) I - qb J) = c, y a row (entries 0 and 1)
    const double p = pa - pb, q = -qb, d = 1.0 / (p * p + q * q);
    Y[0] = d * (C[0] * p + C[1] * q);
    Y[1] = d * (-C[0] * q + C[1] * p);
  } else {  // parts commuting / anticommuting with J
    const double jcj[4] = {-C[3], C[2], C[1], -C[0]};
    double c1[4], c2[4], y1[4], y2[4];
    for (int k = 0; k < 4; ++k) {
      c1[k] = 0.5 * (C[k] - jcj[k]);
      c2[k] = 0.5 * (C[k] + jcj[k]);
    }
    aij_solve_left(pa - pb, qa - qb, c1, y1);
    aij_solve_left(pa - pb, qa + qb, c2, y2);
    for (int k = 0; k < 4; ++k) Y[k] = y1[k] + y2[k];
  }
}

constexpr double kCloseRel = 1e-6;  // divided differences of nearly equal real eigenvalues

}  // namespace

// dst = src for the items' n x n buffers.
__global__ __launch_bounds__(256) void k_copy_buf(const Item* items, double* ws, int src, int dst,
                                                  const int32_t* status) {
  const Item it = items[blockIdx.y];
  if (status[it.layer] != 0) return;
  const int64_t nn = (int64_t)it.n * it.n;
  const double* S = buf_ptr(ws, it, src);
  double* D = buf_ptr(ws, it, dst);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nn; t += (int64_t)gridDim.x * blockDim.x)
    D[t] = S[t];
}

__global__ void k_copy_status(const int32_t* src, int32_t* dst, int n) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) dst[t] = src[t];
}

// dst = I.
__global__ __launch_bounds__(256) void k_fill_identity(const Item* items, double* ws, int dst, const int32_t* status) {
  const Item it = items[blockIdx.y];
  if (status[it.layer] != 0) return;
  const int n = it.n;
  const int64_t nn = (int64_t)n * n;
  double* D = buf_ptr(ws, it, dst);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nn; t += (int64_t)gridDim.x * blockDim.x)
    D[t] = (t / n == t % n) ? 1.0 : 0.0;
}

// Q = Delta R-bar R0 into kBufE, with R-bar^m[(i,r),(q,p)] = c_m / (2 mu_q) sum_k tau_rp(m dphi_k)
// dF[i,q,k][r,p] (the adjoint of the synthesis of eq. 12 and 39). One thread per (i, q).
__global__ __launch_bounds__(256) void k_bwd_q(const Item* items, const Layer* layers, const double* quad,
                                               const double* dF, double* ws, const int32_t* status) {
  const Item it = items[blockIdx.y];
  if (status[it.layer] != 0) return;
  const Layer ly = layers[it.layer];
  const int N = it.N, n = it.n, P = ly.n_dphi, m = it.m;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * N) return;
  const int i = t / N, q = t % N;
  const double* g = dF + ly.out_off + ((int64_t)i * N + q) * P * 16;
  double acc_c[16], acc_s[16];
  for (int k = 0; k < 16; ++k) acc_c[k] = acc_s[k] = 0.0;
  for (int k = 0; k < P; ++k) {
    const int ph = (int)(((int64_t)m * k) % P);
    double sn, cs;
    sincospi(2.0 * ph / P, &sn, &cs);
    for (int e = 0; e < 16; ++e) {
      const double v = g[(int64_t)k * 16 + e];
      acc_c[e] += cs * v;
      acc_s[e] += sn * v;
    }
  }
  const double muq = quad[ly.quad_off + q], alq = quad[ly.quad_off + N + q];
  const double cm = (m == 0 ? 1.0 : 2.0) / (2.0 * muq);
  const double r0 = 1.0 / (3.141592653589793 * alq);
  double* Q = buf_ptr(ws, it, kBufE);
  for (int r = 0; r < 4; ++r)
    for (int p = 0; p < 4; ++p) {
      const bool riq = r < 2, piq = p < 2;
      const int e = r * 4 + p;
      const double tr = (riq == piq) ? acc_c[e] : (piq ? acc_s[e] : -acc_s[e]);
      const double sgn = riq ? 1.0 : -1.0;
      Q[(int64_t)(4 * i + r) * n + 4 * q + p] = sgn * r0 * cm * tr;
    }
}

// dst = X_s f_s(Lambda)^T + X_t f_t(Lambda)^T (the transposes of F_s = U f_s(Lambda) U^-1 enter
// E~-bar): a complex pair's block f = Re f I + Im f J is applied transposed, Re f I - Im f J.
// X_s in kBufT1, X_t in kBufZ, result in kBufT2.
__global__ void k_bwd_dscale(const Item* items, double* ws, const int32_t* status) {
  const Item it = items[blockIdx.z];
  if (status[it.layer] != 0) return;
  const int n = it.n;
  const int i = blockIdx.y * 16 + threadIdx.y;
  const int j = blockIdx.x * 16 + threadIdx.x;
  if (i >= n || j >= n) return;
  const double* Xs = buf_ptr(ws, it, kBufT1);
  const double* Xt = buf_ptr(ws, it, kBufZ);
  double* O = buf_ptr(ws, it, kBufT2);
  const double* ex = ws + it.ws + extras_off(n);
  const double li = ex[n + j];
  const int64_t idx = (int64_t)i * n + j;
  if (li == 0.0) {
    O[idx] = Xs[idx] * ex[6 * n + j] + Xt[idx] * ex[8 * n + j];
  } else {
    const int jf = li > 0.0 ? j : j - 1;
    const double sr = ex[6 * n + jf], si = ex[7 * n + jf], tr = ex[8 * n + jf], ti = ex[9 * n + jf];
    const double xs0 = Xs[(int64_t)i * n + jf], xs1 = Xs[(int64_t)i * n + jf + 1];
    const double xt0 = Xt[(int64_t)i * n + jf], xt1 = Xt[(int64_t)i * n + jf + 1];
    if (j == jf)
      O[idx] = xs0 * sr + xs1 * si + xt0 * tr + xt1 * ti;
    else
      O[idx] = -xs0 * si + xs1 * sr - xt0 * ti + xt1 * tr;
  }
}

// Y = L_s*(X_s) + L_t*(X_t) into kBufT1, X_s in kBufT4, X_t in kBufT5 (Daleckii-Krein adjoint on
// the blocks of Lambda, see the header).
__global__ void k_bwd_dk(const Item* items, const double* tau, double* ws, const int32_t* status) {
  const Item it = items[blockIdx.z];
  if (status[it.layer] != 0) return;
  const int n = it.n;
  const int i = blockIdx.y * 16 + threadIdx.y;
  const int j = blockIdx.x * 16 + threadIdx.x;
  if (i >= n || j >= n) return;
  const double* ex = ws + it.ws + extras_off(n);
  const double* lre = ex;
  const double* lim = ex + n;
  const double t0 = tau[it.layer];
  const Blk A = block_at(lre, lim, i), B = block_at(lre, lim, j);
  const int ri = i - A.j0, cj = j - B.j0;
  const double* XS = buf_ptr(ws, it, kBufT4);
  const double* XT = buf_ptr(ws, it, kBufT5);
  double y = 0.0;
  if (A.s == 1 && B.s == 1) {
    const double la = A.p, lb = B.p;
    const int64_t idx = (int64_t)i * n + j;
    if (A.j0 == B.j0 || fabs(la - lb) <= kCloseRel * fmax(fabs(la), fabs(lb))) {
      const FVals f = boundary_functions(cz(0.5 * (la + lb)), t0);
      y = f.dfs.re * XS[idx] + f.dft.re * XT[idx];
    } else {
      const double fsa = ex[6 * n + A.j0], fsb = ex[6 * n + B.j0];
      const double fta = ex[8 * n + A.j0], ftb = ex[8 * n + B.j0];
      y = (fsa - fsb) / (la - lb) * XS[idx] + (fta - ftb) / (la - lb) * XT[idx];
    }
  } else {
    // gather the block of each X (2 x 2, unused entries zero)
    for (int which = 0; which < 2; ++which) {
      const double* X = which == 0 ? XS : XT;
      double xb[4] = {0.0, 0.0, 0.0, 0.0};
      for (int r = 0; r < A.s; ++r)
        for (int c = 0; c < B.s; ++c) xb[2 * r + c] = X[(int64_t)(A.j0 + r) * n + B.j0 + c];
      double yb[4];
      if (A.j0 == B.j0) {  // 2 x 2 diagonal block of a complex pair
        const FVals f = boundary_functions(cz(A.p, A.q), t0);
        const Cz fz = which == 0 ? f.fs : f.ft;
        const Cz dz = which == 0 ? f.dfs : f.dft;
        const double jxj[4] = {-xb[3], xb[2], xb[1], -xb[0]};
        double x1[4], x2[4], y1[4];
        for (int k = 0; k < 4; ++k) {
          x1[k] = 0.5 * (xb[k] - jxj[k]);
          x2[k] = 0.5 * (xb[k] + jxj[k]);
        }
        aij_left(dz.re, -dz.im, x1, y1);  // f'(Lambda^T) = Re f' I - Im f' J
        // (f(z) - f(conj z)) / (z - conj z); for a pair that nearly merges, Im f(z) loses its digits
        // and the limit Re f'(z) is used instead
        const double dd = (A.q > kCloseRel * fabs(A.p)) ? fz.im / A.q : dz.re;
        for (int k = 0; k < 4; ++k) yb[k] = y1[k] + dd * x2[k];
      } else {  // off-diagonal pair with at least one complex block: Sylvester form at Lambda^T
        const double* fa = ex + (which == 0 ? 6 : 8) * n;
        const double fare = fa[A.j0], faim = A.s == 2 ? fa[n + A.j0] : 0.0;
        const double fbre = fa[B.j0], fbim = B.s == 2 ? fa[n + B.j0] : 0.0;
        double c1[4], c2[4], c[4];
        // f(Lambda_a^T) X - X f(Lambda_b^T), f(Lambda^T) = Re f I - Im f J
        if (A.s == 2) {
          aij_left(fare, -faim, xb, c1);
        } else {
          for (int k = 0; k < 4; ++k) c1[k] = fare * xb[k];
        }
        if (B.s == 2) {
          aij_right(fbre, -fbim, xb, c2);
        } else {
          for (int k = 0; k < 4; ++k) c2[k] = fbre * xb[k];
        }
        for (int k = 0; k < 4; ++k) c[k] = c1[k] - c2[k];
        if (A.s == 1) c[2] = c[3] = 0.0;
        if (B.s == 1) c[1] = c[3] = 0.0;
        block_sylvester(A.p, -A.q, A.s, B.p, -B.q, B.s, c, yb);
      }
      y += yb[2 * ri + cj];
    }
  }
  buf_ptr(ws, it, kBufT1)[(int64_t)i * n + j] = y;
}

// Per item: tau0-bar = <X_s, d f_s/d tau0 (Lambda)> + <X_t, d f_t/d tau0 (Lambda)> (diagonal
// blocks of X_s in kBufT4 and X_t in kBufT5), into extras slot 3n.
__global__ __launch_bounds__(256) void k_bwd_tau(const Item* items, const double* tau, double* ws,
                                                 const int32_t* status) {
  const Item it = items[blockIdx.x];
  if (status[it.layer] != 0) return;
  const int n = it.n;
  double* ex = ws + it.ws + extras_off(n);
  const double* XS = buf_ptr(ws, it, kBufT4);
  const double* XT = buf_ptr(ws, it, kBufT5);
  const double t0 = tau[it.layer];
  double part = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const double li = ex[n + j];
    if (li < 0.0) continue;  // second column of a pair: handled with the first
    if (li == 0.0) {
      const FVals f = boundary_functions(cz(ex[j]), t0);
      part += f.tfs.re * XS[(int64_t)j * n + j] + f.tft.re * XT[(int64_t)j * n + j];
    } else {
      const FVals f = boundary_functions(cz(ex[j], li), t0);
      for (int which = 0; which < 2; ++which) {
        const double* X = which == 0 ? XS : XT;
        const Cz g = which == 0 ? f.tfs : f.tft;
        const double x00 = X[(int64_t)j * n + j], x01 = X[(int64_t)j * n + j + 1];
        const double x10 = X[(int64_t)(j + 1) * n + j], x11 = X[(int64_t)(j + 1) * n + j + 1];
        part += g.re * (x00 + x11) + g.im * (x01 - x10);  // <X, Re g I + Im g J>
      }
    }
  }
  __shared__ double red[4];
  for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
  __syncthreads();
  if (threadIdx.x == 0) ex[3 * n] = red[0] + red[1] + red[2] + red[3];
}

// Per item: omega-bar = <E~-bar, (E~ - M^-1) / omega> + <F~-bar, (F~ - M^-1) / omega> with E~-bar in
// kBufG, F~-bar in kBufT4 and E~, F~ in kBufSE, kBufSF, into extras slot 3n + 1.
__global__ __launch_bounds__(256) void k_bwd_omega(const Item* items, const Layer* layers, const double* quad,
                                                   const double* omega, double* ws, const int32_t* status) {
  const Item it = items[blockIdx.x];
  if (status[it.layer] != 0) return;
  const int n = it.n;
  const Layer ly = layers[it.layer];
  const double om = fmin(omega[it.layer], kOmegaMax);
  const double* Eb = buf_ptr(ws, it, kBufG);
  const double* Fb = buf_ptr(ws, it, kBufT4);
  const double* E = buf_ptr(ws, it, kBufSE);
  const double* F = buf_ptr(ws, it, kBufSF);
  double part = 0.0;
  for (int64_t t = threadIdx.x; t < (int64_t)n * n; t += blockDim.x) {
    const int r = (int)(t / n), c = (int)(t % n);
    const double minv = (r == c) ? 1.0 / quad[ly.quad_off + r / 4] : 0.0;
    part += Eb[t] * (E[t] - minv) + Fb[t] * (F[t] - minv);
  }
  __shared__ double red[4];
  for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
  __syncthreads();
  if (threadIdx.x == 0) ws[it.ws + extras_off(n) + 3 * n + 1] = (red[0] + red[1] + red[2] + red[3]) / om;
}

// Per item: coefficient partials for degrees l = m..L-1 from B_l-bar (see the header), written as
// [6][L] doubles over kBufT5 (family order alpha1..alpha4, beta1, beta2; zero below l = m). One
// workgroup per item; the node-pair blocks of S+-bar and S--bar of one outgoing node i are staged
// in LDS and every thread accumulates its own degrees.
__global__ __launch_bounds__(kCoefThreads) void k_bwd_coef(const Item* items, const Layer* layers,
                                                           const double* quad, const double* omega, double* ws,
                                                           const int32_t* status) {
  const Item it = items[blockIdx.x];
  if (status[it.layer] != 0) return;
  const int n = it.n, N = it.N, L = it.L, m = it.m;
  const Layer ly = layers[it.layer];
  const double om = fmin(omega[it.layer], kOmegaMax);
  const double* Eb = buf_ptr(ws, it, kBufG);
  const double* Fb = buf_ptr(ws, it, kBufT4);
  const double* leg = ws + it.ws + leg_off(n);  // [(l N + i) 3 + {Pb, R, T}]
  double* out = buf_ptr(ws, it, kBufT5);
  __shared__ double sp[4 * kMaxn];  // S+-bar row strip of node i: [4][n]
  __shared__ double sm[4 * kMaxn];
  for (int l0 = 0; l0 < L; l0 += kCoefThreads) {
    const int l = l0 + threadIdx.x;
    const bool act = l >= m && l < L;
    double bp[16], bm[16];  // sum_ij P_i S+-bar_ij P_j and the same for S-
    for (int k = 0; k < 16; ++k) bp[k] = bm[k] = 0.0;
    for (int i = 0; i < N; ++i) {
      __syncthreads();
      const double mui = quad[ly.quad_off + i];
      for (int t = threadIdx.x; t < 4 * n; t += kCoefThreads) {
        const int a = t / n, c = t % n;
        const double w = -0.5 * om * quad[ly.quad_off + N + c / 4] / mui;
        sp[t] = w * Eb[(int64_t)(4 * i + a) * n + c];
        sm[t] = w * Fb[(int64_t)(4 * i + a) * n + c];
      }
      __syncthreads();
      if (!act) continue;
      // Z = sum_j S_ij P_j (4 x 4 per sign)
      double zp[16], zm[16];
      for (int k = 0; k < 16; ++k) zp[k] = zm[k] = 0.0;
      for (int j = 0; j < N; ++j) {
        const double pb = leg[((int64_t)l * N + j) * 3], rr = leg[((int64_t)l * N + j) * 3 + 1],
                     tt = leg[((int64_t)l * N + j) * 3 + 2];
        // P_j = [[pb,0,0,0],[0,rr,-tt,0],[0,-tt,rr,0],[0,0,0,pb]]
        for (int a = 0; a < 4; ++a) {
          const double* rp = sp + a * n + 4 * j;
          const double* rm = sm + a * n + 4 * j;
          zp[4 * a + 0] += rp[0] * pb;
          zp[4 * a + 1] += rp[1] * rr - rp[2] * tt;
          zp[4 * a + 2] += -rp[1] * tt + rp[2] * rr;
          zp[4 * a + 3] += rp[3] * pb;
          zm[4 * a + 0] += rm[0] * pb;
          zm[4 * a + 1] += rm[1] * rr - rm[2] * tt;
          zm[4 * a + 2] += -rm[1] * tt + rm[2] * rr;
          zm[4 * a + 3] += rm[3] * pb;
        }
      }
      const double pb = leg[((int64_t)l * N + i) * 3], rr = leg[((int64_t)l * N + i) * 3 + 1],
                   tt = leg[((int64_t)l * N + i) * 3 + 2];
      for (int b = 0; b < 4; ++b) {  // P_i Z, column b
        bp[0 * 4 + b] += pb * zp[0 * 4 + b];
        bp[1 * 4 + b] += rr * zp[1 * 4 + b] - tt * zp[2 * 4 + b];
        bp[2 * 4 + b] += -tt * zp[1 * 4 + b] + rr * zp[2 * 4 + b];
        bp[3 * 4 + b] += pb * zp[3 * 4 + b];
        bm[0 * 4 + b] += pb * zm[0 * 4 + b];
        bm[1 * 4 + b] += rr * zm[1 * 4 + b] - tt * zm[2 * 4 + b];
        bm[2 * 4 + b] += -tt * zm[1 * 4 + b] + rr * zm[2 * 4 + b];
        bm[3 * 4 + b] += pb * zm[3 * 4 + b];
      }
    }
    if (l < L) {
      double Bb[16];
      const double sg = ((l - m) & 1) ? -1.0 : 1.0;
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
          const double d = b < 2 ? 1.0 : -1.0;  // D = diag(1, 1, -1, -1)
          Bb[4 * a + b] = act ? bp[4 * a + b] * (1.0 + sg * d) + bm[4 * a + b] * (1.0 - sg * d) : 0.0;
        }
      out[0 * L + l] = Bb[0];
      out[1 * L + l] = Bb[5];
      out[2 * L + l] = Bb[10];
      out[3 * L + l] = Bb[15];
      out[4 * L + l] = Bb[1] + Bb[4];
      out[5 * L + l] = Bb[11] - Bb[14];
    }
  }
}

// Per layer: the sums over its orders, in order (deterministic), into the caller's arrays. A failed
// layer gets NaN gradients.
__global__ __launch_bounds__(256) void k_bwd_reduce(const Layer* layers, const Item* items, const double* ws,
                                                    const int32_t* status, double* dtau, double* domega,
                                                    double* dcoef) {
  const int lyi = blockIdx.x;
  const Layer ly = layers[lyi];
  const bool bad = status[lyi] != 0;
  const double nanv = __builtin_nan("");
  for (int t = threadIdx.x; t < 6 * ly.L + 2; t += blockDim.x) {
    double acc = 0.0;
    for (int m = 0; m < ly.M; ++m) {
      const Item it = items[ly.item0 + m];
      const double* ex = ws + it.ws + extras_off(it.n);
      if (t == 6 * ly.L)
        acc += ex[3 * it.n];
      else if (t == 6 * ly.L + 1)
        acc += ex[3 * it.n + 1];
      else
        acc += buf_ptr(const_cast<double*>(ws), it, kBufT5)[t];
    }
    if (bad) acc = nanv;
    if (t == 6 * ly.L)
      dtau[lyi] = acc;
    else if (t == 6 * ly.L + 1)
      domega[lyi] = acc;
    else
      dcoef[ly.coef_off + t] = acc;
  }
}

}  // namespace vbrdf
