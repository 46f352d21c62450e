// Fourier synthesis of the BRDF Mueller matrix (Sec. 2.B, eq. 12; Sec. 2.D, eq. 1 and 39).
//
// F_r[i][q][k][r][p] = 1/(2 mu_q) sum_{m<M} c_m tau_rp(m dphi_k) R^m[(i,r),(q,p)], c_m = 2 - delta_m0,
// dphi_k = 2 pi k / n_dphi. tau_rp is cos on the IQ-IQ and UV-UV blocks, +sin on the UV<-IQ block
// and -sin on the IQ<-UV block (the diagonal of Phi_1^m for an IQ input, of Phi_2^m for a UV input).
// The 1/(2 mu_q) combines the 1/2 of the Stokes series with the horizontal irradiance mu_q I0 of the
// BRDF definition. One workgroup per (layer, i, q): the 16 M response values are staged in LDS and
// the n_dphi x 16 outputs are written contiguously. Angles are taken from a table indexed by
// (m k) mod n_dphi, so no phase is accumulated in floating point.
#include "vbrdf_internal.hpp"

namespace vbrdf {

__global__ __launch_bounds__(256) void k_synth(const SynthTask* tasks, const Layer* layers, const Item* items,
                                                const double* quad, const double* ws, double* F,
                                                const int32_t* status) {
  const SynthTask tk = tasks[blockIdx.x];
  const Layer ly = layers[tk.layer];
  const int N = ly.N, M = ly.M, nphi = ly.n_dphi, n = 4 * N;
  double* out = F + ly.out_off + ((int64_t)tk.i * N + tk.q) * nphi * 16;
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
    sR[m][rp] = ws[it.ws + (int64_t)kBufE * n * n + (int64_t)(4 * tk.i + r) * n + 4 * tk.q + p];
  }
  for (int t = tid; t < nphi; t += NT) {
    const double a = 6.283185307179586 * (double)t / (double)nphi;
    sc[t] = cos(a);
    ss[t] = sin(a);
  }
  __syncthreads();
  const double inv2mu = 0.5 / quad[ly.quad_off + tk.q];
  for (int t = tid; t < nphi * 16; t += NT) {
    const int k = t / 16, rp = t % 16, r = rp / 4, p = rp % 4;
    const bool riq = r < 2, piq = p < 2;
    const int kind = (riq == piq) ? 0 : (piq ? 1 : 2);  // cos, +sin, -sin
    double acc = (kind == 0) ? sR[0][rp] : 0.0;
    int ph = 0;  // (m k) mod nphi
    for (int m = 1; m < M; ++m) {
      ph += k;
      if (ph >= nphi) ph -= nphi;
      const double f = (kind == 0) ? sc[ph] : (kind == 1 ? ss[ph] : -ss[ph]);
      acc += 2.0 * f * sR[m][rp];
    }
    out[t] = acc * inv2mu;
  }
}

// I_out[i][k][r] = mu_q sum_p F_r[i][q][k][r][p] I0[p] (eq. 1 with E = mu_q I0).
__global__ void k_radiance(const Layer* layers, int layer, int q, int kshift, const double* quad, const double* F,
                           double i0, double i1, double i2, double i3, double* I_out) {
  const Layer ly = layers[layer];
  const int N = ly.N, nphi = ly.n_dphi;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * nphi * 4) return;
  const int i = t / (nphi * 4), k = (t / 4) % nphi, r = t % 4;
  const int kd = (k - kshift + nphi) % nphi;  // phi_k - phi0 on the grid
  const double* f = F + ly.out_off + (((int64_t)i * N + q) * nphi + kd) * 16 + r * 4;
  const double muq = quad[ly.quad_off + q];
  I_out[t] = muq * (f[0] * i0 + f[1] * i1 + f[2] * i2 + f[3] * i3);
}

// I(-mu_i, phi_k) = mu_q F_r(i <- q, phi_k - phi0) I0 with F_r summed from the per-order responses
// (eq. 12 with eq. 1 and 39): I_r = 1/2 sum_m c_m sum_p tau_rp(m (phi_k - phi0)) R^m[(i,r),(q,p)] I0_p.
__global__ void k_radiance_series(const Layer* layers, const Item* items, int layer, int q, double phi0,
                                  const double* ws, double i0, double i1, double i2, double i3, double* I_out) {
  const Layer ly = layers[layer];
  const int N = ly.N, nphi = ly.n_dphi, n = 4 * N;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * nphi * 4) return;
  const int i = t / (nphi * 4), k = (t / 4) % nphi, r = t % 4;
  const double d = 6.283185307179586 * k / nphi - phi0;
  const double in[4] = {i0, i1, i2, i3};
  const bool row_iq = r < 2;
  double acc = 0.0;
  for (int m = 0; m < ly.M; ++m) {
    const Item it = items[ly.item0 + m];
    const double* R = ws + it.ws + (int64_t)kBufE * n * n + (int64_t)(4 * i + r) * n + 4 * q;
    double sn, cs;
    sincos(m * d, &sn, &cs);
    double same = 0.0, mixed = 0.0;
    for (int p = 0; p < 4; ++p) {
      const double v = R[p] * in[p];
      if ((p < 2) == row_iq)
        same += v;
      else
        mixed += v;
    }
    // mixed blocks: +sin on UV <- IQ, -sin on IQ <- UV
    const double term = cs * same + (row_iq ? -sn : sn) * mixed;
    acc += (m == 0 ? 1.0 : 2.0) * term;
  }
  I_out[t] = 0.5 * acc;
}

}  // namespace vbrdf
