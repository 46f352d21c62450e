// Off-node incidence: a collimated beam at an arbitrary incident cosine mu0 (not a Gauss node),
// reflected towards the Gauss nodes (Sec. 2.C particular solution, eq. 28-33; its half-size form,
// Sec. 3.B, eq. 46-48).
//
// For the order-m source X exp(-tau/mu0) (k_beam_source) the particular solution Z exp(-tau/mu0)
// splits, with upward fields stored mirrored (Z^- -> D Z^-, D = diag(1,1,-1,-1) per node), into
// the sum g = Z+ + D Z- and difference G- = Z+ - D Z-:
//     (F~ E~ - mu0^-2 I) g = F~ M^-1 X_s + M^-1 X_d / mu0,     G- = mu0 (E~ g - M^-1 X_s),
// solved with the eigen-decomposition of F~ E~ already at hand, g = U (Lambda - mu0^-2)^-1 U^-1 rhs
// (U^-1 through the LU of U^T and a right division; complex pairs through their 2 x 2 real
// blocks). The homogeneous part then cancels the particular solution's incoming diffuse light at
// the top (-Z+) and at the black base (-D Z- exp(-tau0/mu0)); through the layer's operators
// R~ = Y_S + Y_T - I and T~ = Y_S - Y_T (mirrored storage) the upward radiance at the top is
//     D [ D Z- + Z+ - (Y_S + Y_T) Z+ - exp(-tau0/mu0) (Y_S - Y_T) D Z- ].
// The beams of an order are the first 4 n_mu0 columns of n x n buffers, so the products run on the
// matrix cores (k_gemm) and the solves on the same kernels as the rest of the path.
//
// Resonance: g has the factor 1/(lambda_k - mu0^-2). A beam within a relative 1e-12 of an
// eigenvalue's resonance (mu0 = 1/sqrt(lambda_k); in weakly scattering orders these sit at the
// Gauss nodes, where the node path is exact) makes the layer NUMERIC rather than return a result
// dominated by rounding.
#include "vbrdf_internal.hpp"

namespace vbrdf {

__global__ void k_beam_legendre(const Item* items, const double* xs, int n_x, int n_mu0, int which, double* ws,
                                const int32_t* status);
__global__ void k_recon_rows(const Item* items, const Layer* layers, const double* quad, const double* omega,
                             const double* coef, int n_mu0, int n_out, double* ws, const int32_t* status);
__global__ void k_recon_out(const Item* items, const Layer* layers, const double* omega, const double* coef,
                            const double* tau, const double* mu0, int n_mu0, const double* mu_out, int n_out,
                            double* ws, const int32_t* status);
__global__ void k_beam_source(const Item* items, const Layer* layers, const double* quad, const double* omega,
                              const double* coef, const double* mu0, int n_mu0, double* ws, const int32_t* status);

constexpr double kResonanceRel = 1e-12;

// Rows c < 4 n_mu0 of kBufB2 hold (U^-1 rhs)^T: y = column c of U^-1 rhs over the modes k. Each
// mode (or complex pair) is divided by (Lambda_k - mu0^-2): a pair with Lambda block a I + b J
// (J = [[0, 1], [-1, 0]]) by ((a - s) I - b J) / ((a - s)^2 + b^2).
__global__ void k_beam_scale(const Item* items, const double* mu0, int n_mu0, double* ws, int32_t* status) {
  const Item it = items[blockIdx.z];
  if (status[it.layer] != 0) return;
  const int n = it.n;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (k >= n || c >= 4 * n_mu0) return;
  const double* ex = ws + it.ws + extras_off(n);
  const double* lre = ex;
  const double* lim = ex + n;
  if (lim[k] < 0.0) return;  // second column of a pair: done by the first
  double* y = buf_ptr(ws, it, kBufB2) + (int64_t)c * n;
  const double s = 1.0 / (mu0[c >> 2] * mu0[c >> 2]);
  const double a = lre[k] - s;
  if (lim[k] == 0.0) {
    if (!(fabs(a) > kResonanceRel * fmax(fabs(lre[k]), s))) {
      status[it.layer] = VBRDF_E_NUMERIC;
      return;
    }
    y[k] = y[k] / a;
    return;
  }
  const double b = lim[k];
  const double d = a * a + b * b;
  if (!(sqrt(d) > kResonanceRel * fmax(hypot(lre[k], b), s))) {
    status[it.layer] = VBRDF_E_NUMERIC;
    return;
  }
  const double y0 = y[k], y1 = y[k + 1];
  y[k] = (a * y0 - b * y1) / d;
  y[k + 1] = (a * y1 + b * y0) / d;
}

// kBufB4 = E~ g, kBufB1 = g, kBufB0 = M^-1 X_s: G- = mu0 (E~ g - M^-1 X_s), then Z+ = (g + G-)/2
// into kBufB0 and the mirrored Z- = (g - G-)/2 into kBufB1.
__global__ void k_beam_zpm(const Item* items, const double* mu0, int n_mu0, double* ws, const int32_t* status) {
  const Item it = items[blockIdx.y];
  if (status[it.layer] != 0) return;
  const int n = it.n;
  const int64_t nn = (int64_t)n * n;
  double* B0 = buf_ptr(ws, it, kBufB0);
  double* B1 = buf_ptr(ws, it, kBufB1);
  const double* B4 = buf_ptr(ws, it, kBufB4);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nn; t += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(t % n);
    if (c >= 4 * n_mu0) {
      B0[t] = 0.0;
      B1[t] = 0.0;
      continue;
    }
    const double g = B1[t];
    const double gm = mu0[c >> 2] * (B4[t] - B0[t]);
    B0[t] = 0.5 * (g + gm);
    B1[t] = 0.5 * (g - gm);
  }
}

// kBufB2 = (Y_S + Y_T) Z+, kBufB3 = (Y_S - Y_T) Z- (mirrored): the upward radiance at the top per
// unit beam, in physical storage, into kBufB4.
__global__ void k_beam_resp(const Item* items, const double* tau, const double* mu0, int n_mu0, double* ws,
                            const int32_t* status) {
  const Item it = items[blockIdx.z];
  if (status[it.layer] != 0) return;
  const int n = it.n;
  const int a = blockIdx.y * 16 + threadIdx.y;
  const int c = blockIdx.x * 16 + threadIdx.x;
  if (a >= n || c >= 4 * n_mu0) return;
  const int64_t idx = (int64_t)a * n + c;
  const double att = exp(-tau[it.layer] / mu0[c >> 2]);
  const double v = buf_ptr(ws, it, kBufB1)[idx] + buf_ptr(ws, it, kBufB0)[idx] - buf_ptr(ws, it, kBufB2)[idx] -
                   att * buf_ptr(ws, it, kBufB3)[idx];
  buf_ptr(ws, it, kBufB4)[idx] = ((a & 3) >= 2) ? -v : v;
}

// F_beam[i][j][k][r][p] = 1/(2 mu0_j) sum_m c_m tau_rp(m dphi_k) R_beam^m[(i, r), 4 j + p]: the
// synthesis of eq. 12 and 39 with the horizontal irradiance mu0_j I0 (as k_synth_mfma for the nodes).
// Outgoing index i < N: the Gauss nodes (kBufB4); N <= i < N + n_out: the extra outgoing
// directions (kBufB5, rows 4 (i - N) + r).
__global__ __launch_bounds__(256) void k_beam_synth(const BeamTask* tasks, const Layer* layers, const Item* items,
                                                    const double* mu0, int n_mu0, const double* ws, double* F,
                                                    const int32_t* status) {
  const BeamTask tk = tasks[blockIdx.x];
  const Layer ly = layers[tk.layer];
  const int N = ly.N, M = ly.M, nphi = ly.n_dphi, n = 4 * N;
  double* out = F + ly.beam_off + ((int64_t)tk.i * n_mu0 + tk.j) * nphi * 16;
  const int tid = threadIdx.x, NT = blockDim.x;
  if (status[tk.layer] != 0) {
    const double nanv = __builtin_nan("");
    for (int t = tid; t < nphi * 16; t += NT) out[t] = nanv;
    return;
  }
  __shared__ double sR[kSynthMaxM][16];
  __shared__ double sc[kSynthMaxPhi], ss[kSynthMaxPhi];
  for (int t = tid; t < M * 16; t += NT) {
    const int m = t / 16, rp = t % 16, r = rp / 4, p = rp % 4;
    const Item it = items[ly.item0 + m];
    const bool node = tk.i < N;
    const double* B = ws + it.ws + bwd_off(n, N, it.L) + (int64_t)((node ? kBufB4 : kBufB5) - kNumBuf) * n * n;
    sR[m][rp] = B[(int64_t)(4 * (node ? tk.i : tk.i - N) + r) * n + 4 * tk.j + p];
  }
  for (int t = tid; t < nphi; t += NT) {
    const double a = 6.283185307179586 * (double)t / (double)nphi;
    sc[t] = cos(a);
    ss[t] = sin(a);
  }
  __syncthreads();
  const double inv2mu = 0.5 / mu0[tk.j];
  for (int t = tid; t < nphi * 16; t += NT) {
    const int k = t / 16, rp = t % 16, r = rp / 4, p = rp % 4;
    const bool riq = r < 2, piq = p < 2;
    const int kind = (riq == piq) ? 0 : (piq ? 1 : 2);  // cos, +sin, -sin
    double acc = (kind == 0) ? sR[0][rp] : 0.0;
    int ph = 0;
    for (int m = 1; m < M; ++m) {
      ph += k;
      if (ph >= nphi) ph -= nphi;
      const double f = (kind == 0) ? sc[ph] : (kind == 1 ? ss[ph] : -ss[ph]);
      acc += 2.0 * f * sR[m][rp];
    }
    out[t] = acc * inv2mu;
  }
}

// ---- reconstruction towards the extra outgoing cosines (eq. 36-38), half-size form
//
// With Phi+- = (u +- nu v) / 2 the homogeneous field is I+(t) = Phi+ A e^(-t/nu) + Phi- B e^(-(tau0-t)/nu)
// and (mirrored) I-(t) = Phi- A e^(-t/nu) + Phi+ B e^(-(tau0-t)/nu). Its boundary values, the particular
// solution's incoming light with the sign changed (x_top = -Z+, x_bot = -D Z- exp(-tau0/mu0)), give
// the mode coefficients through the layer's operators: with E = exp(-tau0/nu),
//     A + B = 2 (I + E)^-1 U^-1 Y_S (x_top + x_bot),   A - B = 2 (I - E)^-1 U^-1 Y_T (x_top - x_bot).
// The source of eq. 38 towards -mu (mirrored) is P_cross I+ + P_same I- + D X(-mu) e^(-t/mu0), and each
// exponential integrates in closed form against exp(-t/mu) dt / mu:
//     f_A = nu (1 - exp(-tau0 (1/nu + 1/mu))) / (nu + mu),  f_B = nu (exp(-tau0/mu) - exp(-tau0/nu)) / (mu - nu),
// so the radiance is W_A A + W_B B + (P_cross Z+ + P_same D Z- + D X(-mu)) f0 with the rows
// W_A = (P_s U + P_d V nu) / 2 f_A, W_B = (P_s U - P_d V nu) / 2 f_B, P_s = P_cross + P_same,
// P_d = P_cross - P_same. A complex pair (columns k, k+1 holding Re, Im of its eigenvector u) takes
// the complex scalars nu, f_A, f_B of the eigenvalue with Im > 0: on rows as the column mix
// (c_k, c_k+1) -> (c_k z_r - c_k+1 z_i, c_k z_i + c_k+1 z_r), on coefficients (which encode
// (y_k - i y_k+1) / 2) as (y_k, y_k+1) -> (y_k z_r + y_k+1 z_i, -y_k z_i + y_k+1 z_r).

struct Cx2 {
  double re, im;
};
__device__ inline Cx2 cx_mul(Cx2 a, Cx2 b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline Cx2 cx_div(Cx2 a, Cx2 b) {
  const double d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
__device__ inline Cx2 cx_exp(Cx2 a) {
  const double e = exp(a.re);
  return {e * cos(a.im), e * sin(a.im)};
}
__device__ inline Cx2 cx_expm1(Cx2 a) {  // e^a - 1, by its series for small |a|
  if (fabs(a.re) + fabs(a.im) < 1e-4) {
    const Cx2 a2 = cx_mul(a, a), a3 = cx_mul(a2, a);
    return {a.re + a2.re / 2 + a3.re / 6, a.im + a2.im / 2 + a3.im / 6};
  }
  const Cx2 e = cx_exp(a);
  return {e.re - 1.0, e.im};
}
// nu = lambda^-1/2 with Re nu > 0 for the eigenvalue of column k (the one with Im > 0 for a pair)
__device__ inline Cx2 mode_nu(const double* lre, const double* lim, int k) {
  const double a = lre[k], b = lim[k];
  if (b == 0.0) return {1.0 / sqrt(a), 0.0};
  const double r = hypot(a, b);
  const Cx2 sq{sqrt(0.5 * (r + a)), copysign(sqrt(0.5 * (r - a)), b)};  // principal square root
  return cx_div(Cx2{1.0, 0.0}, sq);
}
__device__ inline Cx2 f_a(Cx2 nu, double mu, double tau0) {  // nu (1 - exp(-tau0 (1/nu + 1/mu))) / (nu + mu)
  const Cx2 inv = cx_div(Cx2{1.0, 0.0}, nu);
  const Cx2 e = cx_expm1(Cx2{-tau0 * (inv.re + 1.0 / mu), -tau0 * inv.im});
  return cx_div(cx_mul(nu, Cx2{-e.re, -e.im}), Cx2{nu.re + mu, nu.im});
}
__device__ inline Cx2 f_b(Cx2 nu, double mu, double tau0) {
  // (tau0 / mu) exp(-tau0/mu) expm1(x) / x with x = tau0 (1/mu - 1/nu); directly when |x| is not small
  const Cx2 inv = cx_div(Cx2{1.0, 0.0}, nu);
  const Cx2 x{tau0 * (1.0 / mu - inv.re), -tau0 * inv.im};
  const double em = exp(-tau0 / mu);
  if (fabs(x.re) + fabs(x.im) < 1e-3) {
    const Cx2 x2 = cx_mul(x, x), x3 = cx_mul(x2, x);
    const Cx2 q{1.0 + x.re / 2 + x2.re / 6 + x3.re / 24, x.im / 2 + x2.im / 6 + x3.im / 24};
    return {tau0 / mu * em * q.re, tau0 / mu * em * q.im};
  }
  const Cx2 en = cx_exp(Cx2{-tau0 * inv.re, -tau0 * inv.im});  // exp(-tau0/nu)
  return cx_div(cx_mul(nu, Cx2{em - en.re, -en.im}), Cx2{mu - nu.re, -nu.im});
}

// Rows a < 4 n_out: kBufZ = P_s U, kBufX = P_d V on entry; W_A into kBufZ, W_B into kBufX.
__global__ void k_recon_weights(const Item* items, const double* tau, const double* mu_out, int n_out, double* ws,
                                const int32_t* status) {
  const Item it = items[blockIdx.z];
  if (status[it.layer] != 0) return;
  const int n = it.n;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int a = blockIdx.y;
  if (k >= n || a >= 4 * n_out) return;
  const double* ex = ws + it.ws + extras_off(n);
  const double* lre = ex;
  const double* lim = ex + n;
  if (lim[k] < 0.0) return;
  double* WA = buf_ptr(ws, it, kBufZ) + (int64_t)a * n;
  double* WB = buf_ptr(ws, it, kBufX) + (int64_t)a * n;
  const double mu = mu_out[a >> 2], tau0 = tau[it.layer];
  const Cx2 nu = mode_nu(lre, lim, k);
  const Cx2 fa = f_a(nu, mu, tau0), fb = f_b(nu, mu, tau0);
  if (lim[k] == 0.0) {
    const double s = WA[k], d = WB[k] * nu.re;
    WA[k] = 0.5 * (s + d) * fa.re;
    WB[k] = 0.5 * (s - d) * fb.re;
    return;
  }
  const double s0 = WA[k], s1 = WA[k + 1], p0 = WB[k], p1 = WB[k + 1];
  const double d0 = p0 * nu.re - p1 * nu.im, d1 = p0 * nu.im + p1 * nu.re;  // P_d V nu
  const double a0 = 0.5 * (s0 + d0), a1 = 0.5 * (s1 + d1), b0 = 0.5 * (s0 - d0), b1 = 0.5 * (s1 - d1);
  WA[k] = a0 * fa.re - a1 * fa.im;
  WA[k + 1] = a0 * fa.im + a1 * fa.re;
  WB[k] = b0 * fb.re - b1 * fb.im;
  WB[k + 1] = b0 * fb.im + b1 * fb.re;
}

// x_top + x_bot into kBufB2 and x_top - x_bot into kBufB3 (beam columns; zero elsewhere), from
// kBufB0 = Z+ and kBufB1 = D Z-.
__global__ void k_recon_x(const Item* items, const double* tau, const double* mu0, int n_mu0, double* ws,
                          const int32_t* status) {
  const Item it = items[blockIdx.y];
  if (status[it.layer] != 0) return;
  const int n = it.n;
  const int64_t nn = (int64_t)n * n;
  const double* Zp = buf_ptr(ws, it, kBufB0);
  const double* Zm = buf_ptr(ws, it, kBufB1);
  double* Xs = buf_ptr(ws, it, kBufB2);
  double* Xd = buf_ptr(ws, it, kBufB3);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nn; t += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(t % n);
    if (c >= 4 * n_mu0) {
      Xs[t] = 0.0;
      Xd[t] = 0.0;
      continue;
    }
    const double xt = -Zp[t], xb = -Zm[t] * exp(-tau[it.layer] / mu0[c >> 2]);
    Xs[t] = xt + xb;
    Xd[t] = xt - xb;
  }
}

// Rows c < 4 n_mu0 of kBufF = (U^-1 Y_S x_s)^T and kBufG = (U^-1 Y_T x_d)^T: s = 2 (I + E)^-1 and
// d = 2 (I - E)^-1 of them, then A = (s + d) / 2 into kBufF and B = (s - d) / 2 into kBufG.
__global__ void k_recon_coef(const Item* items, const double* tau, int n_mu0, double* ws, const int32_t* status) {
  const Item it = items[blockIdx.z];
  if (status[it.layer] != 0) return;
  const int n = it.n;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (k >= n || c >= 4 * n_mu0) return;
  const double* ex = ws + it.ws + extras_off(n);
  const double* lre = ex;
  const double* lim = ex + n;
  if (lim[k] < 0.0) return;
  double* F = buf_ptr(ws, it, kBufF) + (int64_t)c * n;
  double* G = buf_ptr(ws, it, kBufG) + (int64_t)c * n;
  const Cx2 nu = mode_nu(lre, lim, k);
  const Cx2 inv = cx_div(Cx2{1.0, 0.0}, nu);
  const double tau0 = tau[it.layer];
  const Cx2 em1 = cx_expm1(Cx2{-tau0 * inv.re, -tau0 * inv.im});   // E - 1
  const Cx2 ws_ = cx_div(Cx2{2.0, 0.0}, Cx2{2.0 + em1.re, em1.im});  // 2 / (1 + E)
  const Cx2 wd = cx_div(Cx2{2.0, 0.0}, Cx2{-em1.re, -em1.im});       // 2 / (1 - E)
  if (lim[k] == 0.0) {
    const double s = F[k] * ws_.re, d = G[k] * wd.re;
    F[k] = 0.5 * (s + d);
    G[k] = 0.5 * (s - d);
    return;
  }
  const double y0 = F[k], y1 = F[k + 1], z0 = G[k], z1 = G[k + 1];
  const double s0 = y0 * ws_.re + y1 * ws_.im, s1 = -y0 * ws_.im + y1 * ws_.re;
  const double d0 = z0 * wd.re + z1 * wd.im, d1 = -z0 * wd.im + z1 * wd.re;
  F[k] = 0.5 * (s0 + d0);
  F[k + 1] = 0.5 * (s1 + d1);
  G[k] = 0.5 * (s0 - d0);
  G[k + 1] = 0.5 * (s1 - d1);
}

void enqueue_beam_outgoing(const LaunchSet& ls, const double* tau, const double* omega, const double* coef,
                           int32_t* st, hipStream_t s) {
  const LaunchSet* p = &ls;
  const int ni = p->n_items, mn = p->max_n, mN = p->max_N, nb = p->n_mu0, no = p->n_mu_out;
  const int gt = (mn + 63) / 64, tt = (mn + 31) / 32, at = (mN + 15) / 16;
  const dim3 gg(gt, gt, ni);
  auto gemm = [&](int a, int b, int c, int mode) { k_gemm<<<gg, 256, 0, s>>>(p->items_d, p->ws_d, a, b, c, mode, st); };
  auto trsm = [&](int a, int rhs, int y) {
    launch_trsm(p->trsm_rows, dim3(xcd_grid(ni, p->trsm_tiles)), p->trsm_lds, s, p->items_d, ni, p->trsm_tiles,
                p->ws_d, st, TrsmBufs{{a, a}, {rhs, rhs}, {y, y}, 1, 0});
  };
  auto transpose = [&](int a, int b) {
    k_transpose<<<dim3(tt, tt, ni), 256, 0, s>>>(p->items_d, p->ws_d, a, b, st);
  };
  k_beam_legendre<<<ni, kLegThreads, 0, s>>>(p->items_d, p->mu_out_d, no, nb, 1, p->ws_d, st);
  gemm(kBufE, kBufU, kBufG, 0);  // V = E~ U
  k_recon_rows<<<dim3(at, at, ni), 256, 0, s>>>(p->items_d, p->layers_d, p->quad_d, omega, coef, nb, no, p->ws_d, st);
  gemm(kBufB5, kBufB0, kBufB7, 0);
  gemm(kBufB6, kBufB1, kBufB7, kGemmAccumulate);                // P_cross Z+ + P_same D Z-
  gemm(kBufB5, kBufU, kBufZ, 0);
  gemm(kBufB6, kBufU, kBufZ, kGemmAccumulate);                  // P_s U
  gemm(kBufB5, kBufG, kBufX, 0);
  gemm(kBufB6, kBufG, kBufX, kGemmNegate | kGemmAccumulate);    // P_d V
  k_recon_weights<<<dim3((mn + 255) / 256, 4 * no, ni), 256, 0, s>>>(p->items_d, tau, p->mu_out_d, no, p->ws_d, st);
  k_recon_x<<<dim3(std::min(1024, (mn * mn + 255) / 256), ni), 256, 0, s>>>(p->items_d, tau, p->mu0_d, nb, p->ws_d,
                                                                            st);
  gemm(kBufYS, kBufB2, kBufF, 0);                               // Y_S (x_top + x_bot)
  gemm(kBufYT, kBufB3, kBufG, 0);                               // Y_T (x_top - x_bot)
  transpose(kBufU, kBufB2);
  launch_lu(dim3(ni, 1), s, p->items_d, p->ws_d, st, p->max_n, LuBufs{{kBufB2, kBufB2}, {kBufB3, kBufB3}, 0});
  transpose(kBufF, kBufB2);
  trsm(kBufB3, kBufB2, kBufF);                                  // (U^-1 Y_S x_s)^T
  transpose(kBufG, kBufB2);
  trsm(kBufB3, kBufB2, kBufG);                                  // (U^-1 Y_T x_d)^T
  k_recon_coef<<<dim3((mn + 255) / 256, 4 * nb, ni), 256, 0, s>>>(p->items_d, tau, nb, p->ws_d, st);
  gemm(kBufZ, kBufF, kBufB2, kGemmTransB);
  gemm(kBufX, kBufG, kBufB2, kGemmTransB | kGemmAccumulate);    // W_A A + W_B B
  k_recon_out<<<dim3((no * nb + 63) / 64, ni), 64, 0, s>>>(p->items_d, p->layers_d, omega, coef, tau, p->mu0_d, nb,
                                                          p->mu_out_d, no, p->ws_d, st);
}

void enqueue_beam_particular(const LaunchSet& ls, const double* omega, const double* coef, int32_t* st,
                             hipStream_t s) {
  const LaunchSet* p = &ls;
  const int ni = p->n_items, mn = p->max_n, mN = p->max_N, nb = p->n_mu0;
  const int at = (mN + 15) / 16, gt = (mn + 63) / 64, tt = (mn + 31) / 32;
  const dim3 gg(gt, gt, ni);
  k_beam_legendre<<<ni, kLegThreads, 0, s>>>(p->items_d, p->mu0_d, nb, nb, 0, p->ws_d, st);
  k_beam_source<<<dim3(at, at, ni), 256, 0, s>>>(p->items_d, p->layers_d, p->quad_d, omega, coef, p->mu0_d, nb,
                                                 p->ws_d, st);
  k_gemm<<<gg, 256, 0, s>>>(p->items_d, p->ws_d, kBufF, kBufB0, kBufB1, kGemmAccumulate, st);  // rhs
  k_transpose<<<dim3(tt, tt, ni), 256, 0, s>>>(p->items_d, p->ws_d, kBufU, kBufB2, st);        // U^T
  launch_lu(dim3(ni, 1), s, p->items_d, p->ws_d, st, p->max_n, LuBufs{{kBufB2, kBufB2}, {kBufB3, kBufB3}, 0});
  k_transpose<<<dim3(tt, tt, ni), 256, 0, s>>>(p->items_d, p->ws_d, kBufB1, kBufB4, st);       // rhs^T
  launch_trsm(p->trsm_rows, dim3(xcd_grid(ni, p->trsm_tiles)), p->trsm_lds, s, p->items_d, ni, p->trsm_tiles,
              p->ws_d, st, TrsmBufs{{kBufB3, kBufB3}, {kBufB4, kBufB4}, {kBufB2, kBufB2}, 1, 0});  // (U^-1 rhs)^T
  k_beam_scale<<<dim3((mn + 255) / 256, 4 * nb, ni), 256, 0, s>>>(p->items_d, p->mu0_d, nb, p->ws_d, st);
  k_gemm<<<gg, 256, 0, s>>>(p->items_d, p->ws_d, kBufU, kBufB2, kBufB1, kGemmTransB, st);  // g
  k_gemm<<<gg, 256, 0, s>>>(p->items_d, p->ws_d, kBufE, kBufB1, kBufB4, 0, st);            // E~ g
  k_beam_zpm<<<dim3(std::min(1024, (mn * mn + 255) / 256), ni), 256, 0, s>>>(p->items_d, p->mu0_d, nb, p->ws_d, st);
}

void enqueue_beam_response(const LaunchSet& ls, const double* tau, int32_t* st, hipStream_t s) {
  const LaunchSet* p = &ls;
  const int ni = p->n_items, mn = p->max_n, nb = p->n_mu0;
  const int gt = (mn + 63) / 64;
  const dim3 gg(gt, gt, ni);
  k_gemm<<<gg, 256, 0, s>>>(p->items_d, p->ws_d, kBufYS, kBufB0, kBufB2, 0, st);
  k_gemm<<<gg, 256, 0, s>>>(p->items_d, p->ws_d, kBufYT, kBufB0, kBufB2, kGemmAccumulate, st);  // (Y_S + Y_T) Z+
  k_gemm<<<gg, 256, 0, s>>>(p->items_d, p->ws_d, kBufYS, kBufB1, kBufB3, 0, st);
  k_gemm<<<gg, 256, 0, s>>>(p->items_d, p->ws_d, kBufYT, kBufB1, kBufB3, kGemmNegate | kGemmAccumulate, st);
  const int ct = (4 * nb + 15) / 16, rt = (mn + 15) / 16;
  k_beam_resp<<<dim3(ct, rt, ni), dim3(16, 16), 0, s>>>(p->items_d, tau, p->mu0_d, nb, p->ws_d, st);
}

void enqueue_beam_synth(const LaunchSet& ls, double* F_beam, const int32_t* st, hipStream_t s) {
  const LaunchSet* p = &ls;
  k_beam_synth<<<p->n_btasks, 256, 0, s>>>(p->btasks_d, p->layers_d, p->items_d, p->mu0_d, p->n_mu0, p->ws_d,
                                          F_beam, st);
}

}  // namespace vbrdf
