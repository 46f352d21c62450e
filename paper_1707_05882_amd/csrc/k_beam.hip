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

__global__ void k_beam_legendre(const Item* items, const double* mu0, int n_mu0, double* ws, const int32_t* status);
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
// synthesis of eq. 12 and 39 with the horizontal irradiance mu0_j I0 (as k_synth for the nodes).
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
    const double* B4 = ws + it.ws + bwd_off(n, N, it.L) + (int64_t)(kBufB4 - kNumBuf) * n * n;
    sR[m][rp] = B4[(int64_t)(4 * tk.i + r) * n + 4 * tk.j + p];
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

void enqueue_beam_particular(const LaunchSet& ls, const double* omega, const double* coef, int32_t* st,
                             hipStream_t s) {
  const LaunchSet* p = &ls;
  const int ni = p->n_items, mn = p->max_n, mN = p->max_N, nb = p->n_mu0;
  const int at = (mN + 15) / 16, gt = (mn + 63) / 64, tt = (mn + 31) / 32;
  const dim3 gg(gt, gt, ni);
  k_beam_legendre<<<ni, kLegThreads, 0, s>>>(p->items_d, p->mu0_d, nb, p->ws_d, st);
  k_beam_source<<<dim3(at, at, ni), 256, 0, s>>>(p->items_d, p->layers_d, p->quad_d, omega, coef, p->mu0_d, nb,
                                                 p->ws_d, st);
  k_gemm<<<gg, 256, 0, s>>>(p->items_d, p->ws_d, kBufF, kBufB0, kBufB1, kGemmAccumulate, st);  // rhs
  k_transpose<<<dim3(tt, tt, ni), 256, 0, s>>>(p->items_d, p->ws_d, kBufU, kBufB2, st);        // U^T
  k_lu<<<dim3(ni, 1), 1024, 0, s>>>(p->items_d, p->ws_d, st, LuBufs{{kBufB2, kBufB2}, {kBufB3, kBufB3}, 0});
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
