// Fourier synthesis of the BRDF Mueller matrix (Sec. 2.B, eq. 12; Sec. 2.D, eq. 1 and 39).
//
// F_r[i][q][k][r][p] = 1/(2 mu_q) sum_{m<M} c_m tau_rp(m dphi_k) R^m[(i,r),(q,p)], c_m = 2 - delta_m0,
// dphi_k = 2 pi k / n_dphi. tau_rp is cos on the IQ-IQ and UV-UV blocks, +sin on the UV<-IQ block
// and -sin on the IQ<-UV block (the diagonal of Phi_1^m for an IQ input, of Phi_2^m for a UV input).
// The 1/(2 mu_q) combines the 1/2 of the Stokes series with the horizontal irradiance mu_q I0 of the
// BRDF definition. Angles are taken from a table indexed by (m k) mod n_dphi, so no phase is
// accumulated in floating point.
#include "vbrdf_internal.hpp"

namespace vbrdf {

typedef double double4_t __attribute__((ext_vector_type(4)));

// The synthesis as a product on the matrix cores: for a fixed row block i and two input
// nodes q0, q0 + 1, out[k][e] = sum_m T[k][m] R^m[e] over the 16 entries e of one kind (the 8 cos
// entries of each node, or the 8 sin entries), with T[k][m] = c_m cos(2 pi m k / n_dphi) or
// c_m sin(...): one v_mfma_f64_16x16x4 per 16 azimuths, 4 orders and kind. A operand = T from LDS
// tables (row = azimuth lane % 16, k = order lane / 16 + 4 t), B operand = R^m[e] gathered from the
// items' workspaces (k = order, column = entry lane % 16), loaded one step ahead and shared by up to
// 8 azimuth tiles; the sign of the IQ <- UV block and 1 / (2 mu_q) come in when storing. One wave
// per task with even q (odd-q tasks are covered by their even neighbour and return at once).
constexpr int kSynthTiles = 8;  // azimuth tiles of 16 held in registers per pass over the orders

__global__ __launch_bounds__(64) void k_synth_mfma(const SynthTask* tasks, const Layer* layers, const Item* items,
                                                    const double* quad, const double* ws, double* F,
                                                    const int32_t* status) {
  const SynthTask tk = tasks[blockIdx.x];
  if (tk.q & 1) return;
  const Layer ly = layers[tk.layer];
  const int N = ly.N, M = ly.M, nphi = ly.n_dphi, n = 4 * N;
  const int lane = threadIdx.x, lr = lane & 15, kq = lane >> 4;
  const int nq = min(2, N - tk.q);  // input nodes of this task
  if (status[tk.layer] != 0) {
    const double nanv = __builtin_nan("");
    double* out = F + ly.out_off + ((int64_t)tk.i * N + tk.q) * nphi * 16;
    for (int t = lane; t < nq * nphi * 16; t += 64) out[t] = nanv;
    return;
  }
  __shared__ double sc[kSynthMaxPhi], ss[kSynthMaxPhi];
  __shared__ int64_t sws[kSynthMaxM];
  for (int t = lane; t < nphi; t += 64) {
    const double a = 6.283185307179586 * (double)t / (double)nphi;
    sc[t] = cos(a);
    ss[t] = sin(a);
  }
  for (int t = lane; t < M; t += 64) sws[t] = items[ly.item0 + t].ws + (int64_t)kBufE * n * n;
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  // entry of this lane's column: node q = q0 + lr / 8, (r, p) of the cos list or of the sin list
  const int e8 = lr & 7, qq = min(tk.q + (lr >> 3), N - 1);
  const int rc = (e8 < 4) ? (e8 >> 1) : 2 + ((e8 - 4) >> 1), pc = (e8 < 4) ? (e8 & 1) : 2 + (e8 & 1);
  const int rs = (e8 < 4) ? 2 + (e8 >> 1) : (e8 - 4) >> 1, ps = (e8 < 4) ? (e8 & 1) : 2 + (e8 & 1);
  const int64_t oc = (int64_t)(4 * tk.i + rc) * n + 4 * qq + pc;
  const int64_t os = (int64_t)(4 * tk.i + rs) * n + 4 * qq + ps;
  const int nsteps = (M + 3) >> 2;
  for (int kg = 0; kg * 16 * kSynthTiles < nphi; ++kg) {
    const int kt0 = kg * kSynthTiles, ntile = min(kSynthTiles, (nphi + 15) / 16 - kt0);
    double4_t acc_c[kSynthTiles], acc_s[kSynthTiles];
#pragma unroll
    for (int t = 0; t < kSynthTiles; ++t) {
      acc_c[t] = (double4_t){0.0, 0.0, 0.0, 0.0};
      acc_s[t] = (double4_t){0.0, 0.0, 0.0, 0.0};
    }
    auto gather = [&](int st, double& bcv, double& bsv) {
      const int m = min(4 * st + kq, M - 1);
      const double* R = ws + sws[m];
      bcv = R[oc];
      bsv = R[os];
    };
    double bc, bs, bcn, bsn;
    gather(0, bc, bs);
    for (int st = 0; st < nsteps; ++st) {
      gather(min(st + 1, nsteps - 1), bcn, bsn);
      const int m = 4 * st + kq;
      const bool mok = m < M;
      const double cm = (m == 0) ? 1.0 : 2.0;
#pragma unroll
      for (int t = 0; t < kSynthTiles; ++t) {
        if (t < ntile) {  // uniform
          const int k = min((kt0 + t) * 16 + lr, nphi - 1);
          const int ph = (int)(((int64_t)m * k) % nphi);
          const double ac = mok ? cm * sc[ph] : 0.0;
          const double as = (mok && m > 0) ? cm * ss[ph] : 0.0;
          acc_c[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ac, mok ? bc : 0.0, acc_c[t], 0, 0, 0);
          acc_s[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(as, mok ? bs : 0.0, acc_s[t], 0, 0, 0);
        }
      }
      bc = bcn;
      bs = bsn;
    }
    // store: accumulator row = azimuth kq + 4 v of the tile, column = entry lr
    if (tk.q + (lr >> 3) < N) {
      const double inv2mu = 0.5 / quad[ly.quad_off + qq];
      const double sgn = (rs < 2) ? -1.0 : 1.0;  // IQ <- UV: -sin; UV <- IQ: +sin
      double* outq = F + ly.out_off + ((int64_t)tk.i * N + qq) * nphi * 16;
#pragma unroll
      for (int t = 0; t < kSynthTiles; ++t) {
        if (t < ntile)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int k = (kt0 + t) * 16 + kq + 4 * v;
            if (k < nphi) {
              outq[(int64_t)k * 16 + rc * 4 + pc] = acc_c[t][v] * inv2mu;
              outq[(int64_t)k * 16 + rs * 4 + ps] = sgn * acc_s[t][v] * inv2mu;
            }
          }
      }
    }
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
