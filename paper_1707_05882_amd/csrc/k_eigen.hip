// Batched real non-symmetric eigensolver for the homogeneous step (Sec. 3.A, eq. 43-45).
//
// The half-size problem (F E) X = lambda X has real or complex-conjugate eigenvalues (the vector
// equation may produce complex pairs). The paper calls a library eigensolver once per order; here
// one workgroup solves one (layer, order) matrix and all orders of all layers run in one launch.
//
// Steps (all in FP64):
//   1. Householder reduction to upper Hessenberg form (the Householder vectors are kept in the
//      workspace; k_hqapply_mfma / k_hqapply apply them later, so the orthogonal factor is not
//      accumulated here; blocked, with matrix-core panel updates, for 128 < n <= 256),
//   2. implicit double-shift (Francis) QR to real Schur form T = Z^T H Z with deflation by the
//      Ahues-Tisseur criterion, exceptional shifts every 10 stagnant sweeps, a real shift pair
//      replaced by the eigenvalue closer to the corner used twice, and after 40 stagnant sweeps
//      (a cluster of nearly equal eigenvalues) a normwise deflation |h| <= ulp ||H||_F,
//   3. eigenvectors of the quasi-triangular T by back-substitution (complex arithmetic only for
//      complex pairs), normalised; all eigenvectors (n <= 128) or groups of them (n <= 256) advance
//      together with their columns in LDS.
// The matrix is not balanced: F E = M^-1 X- M^-1 X+ is graded by the 1/mu factors, and a diagonal
// power-of-two balancing loses about two digits on its smallest (diffusion-mode) eigenvalues,
// which dominate the response; without it the eigenpairs reach about 1e-11 relative.
// The caller then forms U' = Z X_T with a GEMM and U = Q U' with k_hqapply_mfma or k_hqapply (Q
// from the Hessenberg reduction). Output convention: for a complex pair stored at
// (j, j+1) with Im lambda_j > 0, U[:, j] + i U[:, j+1] is the eigenvector of lambda_j.
//
// H is kept in LDS (row stride n + 1) when n <= 128 and reduced in place in global memory
// otherwise (the body is instantiated for both, so LDS-resident H uses LDS instructions); larger
// systems chase their multi-bulge passes through an LDS window (windowed_multibulge). A QR
// sweep touches only a 3-row / 3-column window per bulge step, too little work for a workgroup
// barrier per step: wave 0 alone runs the deflation scan, the shift choice and the bulge chase,
// its lanes kept in step by wave-level ordering (every lane computes the reflector itself). The
// sweep's reflectors are kept in LDS and all waves then apply them to Z, each thread streaming
// along its own rows of Z with a three-element window.
#include "vbrdf_internal.hpp"

namespace vbrdf {

constexpr double kUlp = 2.220446049250313e-16;
constexpr double kSafeMin = 2.2250738585072014e-308;

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1)
    if (o < (int)blockDim.x) v += __shfl_xor(v, o);
  return v;
}
__device__ inline int wave_max(int v) {
  for (int o = 32; o > 0; o >>= 1)
    if (o < (int)blockDim.x) v = max(v, __shfl_xor(v, o));
  return v;
}
__device__ inline double block_sum(double v, double* sred) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
  const int nw = (blockDim.x + 63) >> 6;
  for (int w = 0; w < nw; ++w) r += sred[w];
  __syncthreads();
  return r;
}

struct Cx {
  double re, im;
};
__device__ inline Cx cmul(Cx a, Cx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline Cx csub(Cx a, Cx b) { return {a.re - b.re, a.im - b.im}; }
__device__ inline double cabs1(Cx a) { return fabs(a.re) + fabs(a.im); }
__device__ inline Cx cdiv(Cx a, Cx b) {
  // Smith's algorithm
  if (fabs(b.re) >= fabs(b.im)) {
    double r = b.im / b.re, d = b.re + b.im * r;
    return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  }
  double r = b.re / b.im, d = b.im + b.re * r;
  return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}
__device__ inline Cx cguard(Cx d, double smin) {
  if (cabs1(d) < smin) return {smin, 0.0};
  return d;
}

// Solve the 2x2 complex system [[a, b], [c, d]] x = r by Gaussian elimination with pivoting;
// tiny pivots are replaced by smin (perturbation in the style of LAPACK's eigenvector solver).
__device__ inline void csolve2(Cx a, Cx b, Cx c, Cx d, Cx r0, Cx r1, double smin, Cx& x0, Cx& x1) {
  if (cabs1(a) >= cabs1(c)) {
    a = cguard(a, smin);
    Cx f = cdiv(c, a);
    Cx d2 = cguard(csub(d, cmul(f, b)), smin);
    Cx s1 = csub(r1, cmul(f, r0));
    x1 = cdiv(s1, d2);
    x0 = cdiv(csub(r0, cmul(b, x1)), a);
  } else {
    Cx f = cdiv(a, c);
    Cx b2 = cguard(csub(b, cmul(f, d)), smin);
    Cx s0 = csub(r0, cmul(f, r1));
    x1 = cdiv(s0, b2);
    x0 = cdiv(csub(r1, cmul(d, x1)), c);
  }
}

// Orders LDS (and global) accesses of different lanes of one wave: a wave's memory operations
// execute in order, so a compiler scheduling barrier is all the hand-off needs.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Action codes of the QR driver (sctl[4]).
enum : int { kActDeflated = 0, kActSweep = 1, kActRotate = 2, kActStop = 3, kActMulti = 4 };

// Multi-bulge passes: with at least kMultiMin active rows and fewer than kMultiIts iterations since
// the last deflation, one pass chases one bulge per wave (up to kMaxBulges = 8 double shifts at
// once), the bulges kMultiGap rows apart. Otherwise a single double-shift sweep runs on wave 0.
constexpr int kMultiMin = 32;
constexpr int kMultiIts = 6;
// Systems that take the windowed pass keep to multi-bulge passes longer: there a pass costs less
// than the single-wave sweep in global memory it replaces (measured at n = 256: eigen stage -9%).
constexpr int kMultiItsWindowed = 20;
constexpr int kMultiGap = 4;
constexpr int kMaxBulges = kEigenThreads / 64;  // one bulge per wave

// Z-update descriptor of one QR iteration, produced by wave 0 and applied by the other waves
// during the next iteration (double-buffered): kind 0 none, 1 sweep (reflectors of steps lo..hh-1
// as (tau, u1, u2) triples in the slot's reflector buffer), 2 rotation of columns hh-1, hh by
// (cs, sn) stored at the start of the reflector buffer. `stop` ends the QR loop after this
// iteration; it lives in the double-buffered slot so that wave 0 cannot overwrite it (in the
// next iteration) before every wave has read it.
struct ZOp {
  int kind, lo, hh, stop, nb;  // nb > 0: multi-bulge pass over lo..hh with nb bulges (no Z op)
};

// Applies the reflectors of a sweep over lo..hh (rf[3 k .. 3 k + 2] = (tau, u1, u2) of step k; the
// last one has two elements) to the line e(k) = L[k st], k = lo..hh: a row of Z or of H from the
// right, or a column of H from the left (the reflectors are symmetric, so both read the same).
__device__ __forceinline__ void sweep_line(const double* rf, double* __restrict__ L, int64_t st, int lo, int hh) {
  double z0 = L[(int64_t)lo * st], z1 = L[(int64_t)(lo + 1) * st];
  for (int k0 = lo; k0 <= hh - 1; k0 += 8) {
    double zb[8];  // entries of the next 8 steps, loaded ahead (not yet written)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int c = k0 + 2 + j;
      zb[j] = (c <= hh) ? L[(int64_t)c * st] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = k0 + j;
      if (k <= hh - 1) {
        const bool three = k < hh - 1;
        double z2 = three ? zb[j] : 0.0;
        const double tau = rf[3 * k];
        if (tau != 0.0) {
          const double u1 = rf[3 * k + 1], u2 = rf[3 * k + 2];
          const double w = tau * (z0 + u1 * z1 + (three ? u2 * z2 : 0.0));
          z0 -= w;
          z1 -= w * u1;
          if (three) z2 -= w * u2;
        }
        L[(int64_t)k * st] = z0;
        z0 = z1;
        z1 = z2;
      }
    }
  }
  L[(int64_t)hh * st] = z0;
}

// Applies one ZOp to lines t0, t0 + nt, ... of the job list: the n rows of Z (Z(r, c) at
// ZT[c * n + r]) and, when Hd is given (H row-major in global memory, the QR driver's wave 0 having
// updated only the active block), the parts of H outside the block that the op's transformation
// reaches: rows 0..b-1 from the right and columns hh+1..n-1 from the left, b = lo (sweep) or
// hh - 1 (rotation of rows/columns hh - 1, hh).
__device__ __forceinline__ void apply_zop(const ZOp& op, const double* rf, double* __restrict__ ZT, double* Hd,
                                          int n, int t0, int nt) {
  if (op.kind != 1 && op.kind != 2) return;
  const int hh = op.hh, b = (op.kind == 1) ? op.lo : hh - 1;
  const int nj = n + (Hd ? b + (n - 1 - hh) : 0);
  for (int q = t0; q < nj; q += nt) {
    double* L;
    int64_t st;
    if (q < n) {
      L = ZT + q;
      st = n;
    } else if (q < n + b) {
      L = Hd + (int64_t)(q - n) * n;
      st = 1;
    } else {
      L = Hd + (hh + 1 + (q - n - b));
      st = n;
    }
    if (op.kind == 1) {
      sweep_line(rf, L, st, op.lo, hh);
    } else {
      const double cs = rf[0], sn = rf[1];
      const double zx = L[(int64_t)b * st], zy = L[(int64_t)hh * st];
      L[(int64_t)b * st] = cs * zx + sn * zy;
      L[(int64_t)hh * st] = -sn * zx + cs * zy;
    }
  }
}

// Line (row or column) of a thread in the two-sided Hessenberg update, where P adjacent lanes
// share a line and split its dot product (part = tid mod P, element i of the line taken by part
// i mod P). In LDS, element (r, c) sits in bank pair (r + c) mod 16 of the 32 banks (row stride
// 1 mod 16 doubles), and a 64-bit access is served 16 lanes at a time, so lines handled together
// must be P apart: half-wave h covers lines 32 (h / P) + P j + h mod P, j < 32 / P, and every 16
// lanes of it meet 16 distinct bank pairs. Blocks too small for that keep consecutive lines.
// Either way tid -> line is a bijection onto [0, NT / P).
__device__ inline int hess_line(int tid, int P, int NT) {
  if (NT % (32 * P) != 0) return tid / P;
  const int hw = tid >> 5, l32 = tid & 31;
  return 32 * (hw / P) + P * (l32 / P) + hw % P;
}

// ---- Windowed multi-bulge pass for systems kept in global memory (n > kLdsMaxn)
//
// Chasing the bulges through H in global memory costs, per chain step and bulge, a read and write
// of three rows and three columns of H and three columns of Z: the whole matrix streams through
// the caches once per few steps and, with one problem per compute unit, the L2 of an XCD cannot
// hold the working sets. Here the pass works on a kWin x kWin diagonal window of H held in LDS:
// the chain is chased inside the window (left updates limited to the window's columns, right
// updates to its rows), the reflectors are accumulated into an orthogonal U (kWin x kWin, LDS),
// and when the leading bulge reaches the window's end the parts outside the window take the
// window's whole transformation at once on the matrix cores:
//     H[a:b, b:n] <- U^T H[a:b, b:n],   H[0:a, a:b] <- H[0:a, a:b] U,   Z[:, a:b] <- Z[:, a:b] U.
// The next window starts one row above the trailing bulge, so every bulge's reflector input stays
// inside a window, and moves the chain kWin - 4 (bulges) rows further.
constexpr int kWin = 88;          // window rows and columns
constexpr int kWinLd = kWin + 1;  // LDS row stride of the window
// LDS row stride of U: at least the columns of whole 16-column MFMA tiles (96), and odd so that the
// lanes of a column update (one row each) fall in different banks (a stride of 96 doubles put
// all 64 lanes in one bank)
constexpr int kWinU = 97;
static_assert(kWin % 4 == 0 && kWinU >= (kWin + 15) / 16 * 16 && kWinU % 2 == 1, "MFMA tiling of the window update");
static_assert(kWin * kWinLd + kWin * kWinU <= kLdsMaxn * (kLdsMaxn + 1) + 3 * 64,
              "window and U fit the LDS buffer of the LDS-resident path");
static_assert(kWin > 4 * kMaxBulges + 4, "a window holds the whole bulge chain and lets it advance");
// Largest system that takes the windowed pass. Larger ones (n = 512) keep the pass that updates H
// and Z in global memory step by step: at N = 128 one nearly degenerate node cluster's per-order
// response depends on the rounding of the QR phase more than the eigenpair refinement can absorb
// (a close pair whose second-order coupling to the node's other Stokes eigenvalues it neglects),
// and that path is the one its per-order accuracy was established on.
constexpr int kWinMaxN = 256;

typedef double double4_t __attribute__((ext_vector_type(4)));

// Reflector (I - tau u u^T), u = (1, u1, u2), taking (x, y, z) to (beta, 0, 0),
// beta = -sign(x) ||(x, y, z)||; the identity (tau = 0, beta = x) when y = z = 0.
__device__ __forceinline__ void householder3(double x, double y, double z, double& tau, double& u1, double& u2,
                                             double& beta) {
  tau = 0.0;
  u1 = 0.0;
  u2 = 0.0;
  beta = x;
  if (y == 0.0 && z == 0.0) return;
  double xs = x, ys = y, zs = z, unscale = 1.0;
  double s2 = xs * xs + ys * ys + zs * zs;
  if (s2 < 0x1p-900) {  // keep the squares clear of the subnormal range
    xs *= 0x1p600;
    ys *= 0x1p600;
    zs *= 0x1p600;
    unscale = 0x1p-600;
    s2 = xs * xs + ys * ys + zs * zs;
  }
  double r = __builtin_amdgcn_rsq(s2);
  const double h2 = 0.5 * s2;
  r = r * fma(-h2 * r, r, 1.5);
  r = r * fma(-h2 * r, r, 1.5);
  const double nrm = s2 * r;
  const double ax = fabs(xs);
  tau = fma(ax, r, 1.0);
  const double dd = ax + nrm;
  double q = __builtin_amdgcn_rcp(dd);
  q = fma(q, fma(-dd, q, 1.0), q);
  q = fma(q, fma(-dd, q, 1.0), q);
  const double sc = copysign(q, xs);
  u1 = ys * sc;
  u2 = zs * sc;
  beta = -copysign(nrm, xs) * unscale;
}

// X <- X U for rows 16 rb .. 16 rb + 15 of an m x w block of global memory (X[r][j] at
// X0[r sr + j sj]), U in LDS (U[k][j] at sU[k kWinU + j], zero outside w x w). One wave: the 16 rows
// are loaded whole as the A operands of v_mfma_f64_16x16x4 (row = lane % 16, k = lane / 16 + 4 t)
// before any of them is stored; B = U (k = lane / 16, column = lane % 16); the accumulator holds
// row lane / 16 + 4 v, column lane % 16.
__device__ __forceinline__ void window_update_rows(double* __restrict__ X0, int64_t sr, int64_t sj, int m, int w,
                                                   const double* __restrict__ sU, int rb, int lane) {
  constexpr int kT = kWin / 4;
  const int lr = lane & 15, kq = lane >> 4;
  const int r = rb * 16 + lr;
  double a[kT];
#pragma unroll
  for (int t = 0; t < kT; ++t) {
    const int k = 4 * t + kq;
    a[t] = (r < m && k < w) ? X0[(int64_t)r * sr + (int64_t)k * sj] : 0.0;
  }
#pragma unroll 1
  for (int cb = 0; cb < kWinU / 16; ++cb) {
    if (cb * 16 >= w) break;
    double4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int t = 0; t < kT; ++t)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], sU[(4 * t + kq) * kWinU + cb * 16 + lr], acc, 0, 0, 0);
    const int col = cb * 16 + lr;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = rb * 16 + kq + 4 * v;
      if (row < m && col < w) X0[(int64_t)row * sr + (int64_t)col * sj] = acc[v];
    }
  }
}

// One multi-bulge pass over rows/columns lo..hh of H (global, row-major, n x n) with Z (global,
// Z(r, c) at ZT[c n + r]): wave b chases bulge b (shift pair sh[4 b .. 4 b + 3]) kMultiGap rows
// behind bulge b - 1, as in the LDS-resident pass, but window by window (see above). sbuf: LDS
// for the window and U. Called by every thread of the workgroup.
__device__ void windowed_multibulge(double* __restrict__ H, int n, double* __restrict__ ZT, int lo, int hh, int nb,
                                    const double* sh, double* sbuf) {
  const int tid = threadIdx.x, NT = blockDim.x, lane = tid & 63, wv = tid >> 6, nw = NT >> 6;
  double* sW = sbuf;
  double* sU = sbuf + kWin * kWinLd;
  const int nsteps = (hh - lo) + kMultiGap * (nb - 1);
  int t = 0, a = lo;
  while (t < nsteps) {
    const int bw = min(a + kWin, hh + 1);  // window rows/columns a..bw-1
    const int w = bw - a;
    const bool last = bw == hh + 1;
#define WW(r, c) sW[((r) - a) * kWinLd + ((c) - a)]
    for (int i = tid; i < w * w; i += NT) {
      const int r = i / w, c = i - (i / w) * w;
      sW[r * kWinLd + c] = H[(int64_t)(a + r) * n + a + c];
    }
    for (int i = tid; i < kWin * kWinU; i += NT) {
      const int r = i / kWinU, c = i - (i / kWinU) * kWinU;
      sU[i] = (r == c && r < w) ? 1.0 : 0.0;
    }
    __syncthreads();
    // steps while the leading bulge's rows k..k+3 stay inside the window (all of them in the last)
    const int t_end = last ? nsteps : min(nsteps, bw - 3 - lo);
    for (; t < t_end; ++t) {
      const int k = lo + t - kMultiGap * wv;
      const bool on = wv < nb && k >= lo && k <= hh - 1;
      const bool three = k < hh - 1;
      double tau = 0.0, u1 = 0.0, u2 = 0.0, beta = 0.0;
      if (on) {
        double x, y, z;
        if (k == lo) {  // the bulge enters: first column of (H - s1)(H - s2), product form (a == lo)
          const double s1r = sh[4 * wv], s1i = sh[4 * wv + 1], s2r = sh[4 * wv + 2], s2i = sh[4 * wv + 3];
          const double a0 = WW(lo, lo), a1 = WW(lo + 1, lo);
          const double sc = fabs(a0 - s2r) + fabs(s2i) + fabs(a1);
          const double a1s = a1 / sc;
          x = a1s * WW(lo, lo + 1) + (a0 - s1r) * ((a0 - s2r) / sc) - s1i * (s2i / sc);
          y = a1s * (a0 + WW(lo + 1, lo + 1) - s1r - s2r);
          z = a1s * WW(lo + 2, lo + 1);
        } else {
          x = WW(k, k - 1);
          y = WW(k + 1, k - 1);
          z = three ? WW(k + 2, k - 1) : 0.0;
        }
        wave_sync();  // every lane has read its input before the left phase overwrites it
        householder3(x, y, z, tau, u1, u2, beta);
        if (tau != 0.0) {
          if (lane == 0 && k > lo) {
            WW(k, k - 1) = beta;
            WW(k + 1, k - 1) = 0.0;
            if (three) WW(k + 2, k - 1) = 0.0;
          }
          if (three) {
            for (int c = k + lane; c < bw; c += 64) {
              const double h0 = WW(k, c), h1 = WW(k + 1, c), h2 = WW(k + 2, c);
              const double wl = tau * (h0 + u1 * h1 + u2 * h2);
              WW(k, c) = h0 - wl;
              WW(k + 1, c) = h1 - wl * u1;
              WW(k + 2, c) = h2 - wl * u2;
            }
          } else {
            for (int c = k + lane; c < bw; c += 64) {
              const double h0 = WW(k, c), h1 = WW(k + 1, c);
              const double wl = tau * (h0 + u1 * h1);
              WW(k, c) = h0 - wl;
              WW(k + 1, c) = h1 - wl * u1;
            }
          }
        }
      }
      __syncthreads();
      if (on && tau != 0.0) {
        const int rmax = min(k + 3, hh);
        const int j = k - a;  // window column of the reflector
        if (three) {
          for (int r = a + lane; r <= rmax; r += 64) {
            const double h0 = WW(r, k), h1 = WW(r, k + 1), h2 = WW(r, k + 2);
            const double wr = tau * (h0 + u1 * h1 + u2 * h2);
            WW(r, k) = h0 - wr;
            WW(r, k + 1) = h1 - wr * u1;
            WW(r, k + 2) = h2 - wr * u2;
          }
          for (int r = lane; r < w; r += 64) {
            double* ur = sU + r * kWinU + j;
            const double v0 = ur[0], v1 = ur[1], v2 = ur[2];
            const double wr = tau * (v0 + u1 * v1 + u2 * v2);
            ur[0] = v0 - wr;
            ur[1] = v1 - wr * u1;
            ur[2] = v2 - wr * u2;
          }
        } else {
          for (int r = a + lane; r <= rmax; r += 64) {
            const double h0 = WW(r, k), h1 = WW(r, k + 1);
            const double wr = tau * (h0 + u1 * h1);
            WW(r, k) = h0 - wr;
            WW(r, k + 1) = h1 - wr * u1;
          }
          for (int r = lane; r < w; r += 64) {
            double* ur = sU + r * kWinU + j;
            const double v0 = ur[0], v1 = ur[1];
            const double wr = tau * (v0 + u1 * v1);
            ur[0] = v0 - wr;
            ur[1] = v1 - wr * u1;
          }
        }
      }
      __syncthreads();
    }
#undef WW
    for (int i = tid; i < w * w; i += NT) {
      const int r = i / w, c = i - (i / w) * w;
      H[(int64_t)(a + r) * n + a + c] = sW[r * kWinLd + c];
    }
    // the window's transformation on Z (n rows), on the rows above the window and, transposed,
    // on the columns right of it: disjoint blocks, 16 rows per wave task
    const int bz = (n + 15) >> 4, ba = (a + 15) >> 4, br = (n - bw + 15) >> 4;
    for (int q = wv; q < bz + ba + br; q += nw) {
      if (q < bz)
        window_update_rows(ZT + (int64_t)a * n, 1, n, n, w, sU, q, lane);
      else if (q < bz + ba)
        window_update_rows(H + a, n, 1, a, w, sU, q - bz, lane);
      else
        window_update_rows(H + (int64_t)a * n + bw, 1, n, n - bw, w, sU, q - bz - ba, lane);
    }
    __syncthreads();
    // next window: one row above the trailing bulge's next reflector row
    a = max(lo, lo + t - kMultiGap * (nb - 1) - 1);
  }
}

// ---- Blocked Householder reduction to Hessenberg form for systems kept in global memory
//
// The step-by-step reduction reads and writes the whole trailing matrix twice per column (left and
// right update). Here the reflectors of a panel of nb columns are gathered in the compact WY form
// Q_j = H_0 ... H_{j-1} = I - V T V^T, with W = V T kept instead of T, and the panel's column c is
// brought up to date on its own: with A_0 the matrix at the panel start and Y = A_0 W,
//     column c of Q_j^T A_0 Q_j = b - V (W^T b),   b = a0_c - Y V[c, :]^T,
// on rows p+1..n-1 (the rows a reflector of the panel touches). Each new reflector v_j adds
//     z = V^T v_j,  W[:, j] = tau (v_j - W z),  Y[:, j] = tau (A_0 v_j - Y z),
// so the only pass over the matrix inside the panel is the product A_0 v_j (read only). After the
// panel the trailing columns take the whole transformation at once,
//     X = A_0 - Y V^T,   X <- X - V (W^T X)   (rows p+1..n-1, columns p+nb..n-1),
// and the rows above the panel (0..p) take the right update A_0 - (A_0 W) V^T, both on the matrix
// cores. The reflectors are
// those of the step-by-step reduction (same v_k, tau_k in QV), up to rounding.
// Used up to kWinMaxN rows, for the reason given there: at n = 512 the blocked form's rounding
// moves that node cluster's per-order error past what its refinement absorbs (measured 4.6e-9 of
// max |R| against about 5e-10 with the step-by-step reduction).
constexpr int kHessNb = 16;  // panel width: at most 16 (one 32-lane group per dot product)
constexpr int kHessChunks = kWinMaxN / 64;  // 64-column chunks of a row of the product A_0 v
constexpr int kHessBatch = 8;               // rows whose loads are issued together in the updates
constexpr int kHessLds = kWin * kWinLd + kWin * kWinU;  // LDS doubles available (k_eigen_big's buffer)

__device__ void blocked_hessenberg(double* __restrict__ H, int n, double* __restrict__ QV, double* sbuf,
                                   double* sred) {
  const int tid = threadIdx.x, NT = blockDim.x, lane = tid & 63, wv = tid >> 6, nw = NT >> 6;
  int nb = kHessNb;
  while (nb > 4 && 3 * nb * n + 2 * n + 64 + 8 * 16 * 17 > kHessLds) nb -= 4;
  double* Vs = sbuf;          // V[t][a] at Vs[a n + t] (row p + 1 + t)
  double* Ys = Vs + nb * n;   // Y[t][a] at Ys[a n + t]; after the panel, Y_top[r][a] at Ys[a n + r]
  double* Ws = Ys + nb * n;   // W[t][a] at Ws[a n + t]
  double* bs = Ws + nb * n;   // the panel column being reduced
  double* gs = bs + n;        // A_0 v_j
  double* us = gs + n;        // W^T b (16), then V^T v_j (16)
  double* zs = us + 16;
  const int djj = tid >> 5, dpart = tid & 31;  // 16 dot products, 32 lanes each
#define AH(r, c) H[(int64_t)(r) * n + (c)]
  for (int p = 0; p + 2 < n; p += nb) {
    const int nbp = min(nb, n - 2 - p);
    const int R = n - p - 1;  // rows p+1..n-1
    for (int j = 0; j < nbp; ++j) {
      const int c = p + j;
      // b = a0_c - Y V[c, :]^T (each thread its own rows t = tid + k NT, as in the Y update below)
      for (int t = tid; t < R; t += NT) {
        double x = AH(p + 1 + t, c);
        for (int a = 0; a < j; ++a) x -= Ys[a * n + t] * Vs[a * n + j - 1];
        bs[t] = x;
      }
      __syncthreads();
      if (j > 0) {  // u = W^T b
        double u = 0.0;
        if (djj < j)
          for (int t = dpart; t < R; t += 32) u += Ws[djj * n + t] * bs[t];
        for (int o = 16; o > 0; o >>= 1) u += __shfl_xor(u, o);
        if (dpart == 0 && djj < j) us[djj] = u;
        __syncthreads();
      }
      // b <- b - V u; the reflector's norm below row c+1
      double part = 0.0;
      for (int t = tid; t < R; t += NT) {
        double x = bs[t];
        for (int a = 0; a < j; ++a) x -= Vs[a * n + t] * us[a];
        bs[t] = x;
        if (t > j) part += x * x;
      }
      const double sigma = block_sum(part, sred);
      const double x0 = bs[j];
      double tau = 0.0, beta = x0, scal = 0.0;
      if (sigma != 0.0) {  // uniform
        const double nrm = sqrt(x0 * x0 + sigma);
        beta = (x0 >= 0.0) ? -nrm : nrm;
        tau = (beta - x0) / beta;
        scal = 1.0 / (x0 - beta);
      }
      for (int t = tid; t < R; t += NT) {
        const double v = (t < j) ? 0.0 : (t == j) ? 1.0 : bs[t] * scal;
        Vs[j * n + t] = v;
        if (t >= j) QV[(int64_t)c * n + (t - j)] = v;
        AH(p + 1 + t, c) = (t < j) ? bs[t] : (t == j) ? beta : 0.0;
      }
      if (tid == 0) QV[(int64_t)(n - 1) * n + c] = tau;
      __syncthreads();
      // z = V^T v_j (LDS only), then g = A_0 v_j on rows p+1..n-1, columns c+1..n-1
      if (j > 0) {
        double z = 0.0;
        if (djj < j)
          for (int t = j + dpart; t < R; t += 32) z += Vs[djj * n + t] * Vs[j * n + t];
        for (int o = 16; o > 0; o >>= 1) z += __shfl_xor(z, o);
        if (dpart == 0 && djj < j) zs[djj] = z;
      }
      for (int rb = wv * 8; rb < R; rb += nw * 8) {
        double acc[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) acc[r] = 0.0;
        // every column chunk of the row block at once (n <= kWinMaxN: at most kHessChunks chunks),
        // columns clamped and their v masked, so that no branch separates the loads from their use
        double hv[kHessChunks][8], vv[kHessChunks];
#pragma unroll
        for (int q = 0; q < kHessChunks; ++q) {
          const int col = c + 1 + lane + 64 * q, cc = min(col, n - 1);
          vv[q] = col < n ? Vs[j * n + cc - p - 1] : 0.0;
#pragma unroll
          for (int r = 0; r < 8; ++r) hv[q][r] = AH(p + 1 + min(rb + r, R - 1), cc);
        }
#pragma unroll
        for (int q = 0; q < kHessChunks; ++q)
#pragma unroll
          for (int r = 0; r < 8; ++r) acc[r] += hv[q][r] * vv[q];
        // 8 sums over 64 lanes: halve the set at each of the first three exchanges
        {
          const bool h = lane & 32;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const double snd = h ? acc[r] : acc[r + 4], kp = h ? acc[r + 4] : acc[r];
            acc[r] = kp + __shfl_xor(snd, 32);
          }
        }
        {
          const bool h = lane & 16;
#pragma unroll
          for (int r = 0; r < 2; ++r) {
            const double snd = h ? acc[r] : acc[r + 2], kp = h ? acc[r + 2] : acc[r];
            acc[r] = kp + __shfl_xor(snd, 16);
          }
        }
        {
          const bool h = lane & 8;
          const double snd = h ? acc[0] : acc[1], kp = h ? acc[1] : acc[0];
          acc[0] = kp + __shfl_xor(snd, 8);
        }
        acc[0] += __shfl_xor(acc[0], 4);
        acc[0] += __shfl_xor(acc[0], 2);
        acc[0] += __shfl_xor(acc[0], 1);
        const int row = rb + ((lane >> 5) & 1) * 4 + ((lane >> 4) & 1) * 2 + ((lane >> 3) & 1);
        if ((lane & 7) == 0 && row < R) gs[row] = acc[0];
      }
      __syncthreads();
      // W[:, j] = tau (v_j - W z), Y[:, j] = tau (g - Y z); the next column's update reads only
      // the rows each thread writes here, so no barrier follows
      for (int t = tid; t < R; t += NT) {
        double wy = Vs[j * n + t], yy = gs[t];
        for (int a = 0; a < j; ++a) {
          wy -= Ws[a * n + t] * zs[a];
          yy -= Ys[a * n + t] * zs[a];
        }
        Ws[j * n + t] = tau * wy;
        Ys[j * n + t] = tau * yy;
      }
    }
    __syncthreads();
    // The panel's update of the rest of the matrix, on the matrix cores (v_mfma_f64_16x16x4), as
    // tasks of one wave each:
    //  * a block of 16 trailing columns (p+nbp..n-1) on rows p+1..n-1: X = A_0 - Y V^T tile by tile
    //    while W^T X is summed over the row tiles (the accumulator layout of X is the B-operand
    //    layout), then a second pass X = A_0 - Y V^T - V (W^T X) stores the tiles;
    //  * a block of 16 rows above the panel (0..p) on columns p+1..n-1: Y_top = A_0 W (staged
    //    through LDS to serve as an A operand), then A_0 - Y_top V^T.
    // The two kinds touch disjoint parts of H and only read V, Y, W. Panel columns a >= nbp of
    // V, Y, W are masked (they hold an earlier panel's values); rows past the end are clamped and
    // masked. The next tile's loads are issued before the current tile's MFMAs.
    {
      const int lr = lane & 15, kq = lane >> 4;
      const int ct0 = p + nbp;                   // first trailing column
      const int ncb = (n - ct0 + 15) >> 4;       // trailing column blocks
      const int nrb = (R + 15) >> 4;             // row tiles of the trailing rows
      const int ntb = (p + 1 + 15) >> 4;         // row blocks above the panel
      double* Yt = zs + 48 + wv * (16 * 17);     // per wave: Y_top block [16][17]
      for (int task = wv; task < ncb + ntb; task += nw) {
        if (task < ncb) {
          const int col = ct0 + task * 16 + lr, colc = min(col, n - 1);
          double bv[4];  // B of Y V^T: V[col][a], a = 4 t + kq
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int a = 4 * t + kq;
            bv[t] = a < nbp ? Vs[a * n + colc - p - 1] : 0.0;
          }
          auto load_tile = [&](int rb, double4_t& x) {
#pragma unroll
            for (int v = 0; v < 4; ++v) x[v] = AH(p + 1 + min(16 * rb + kq + 4 * v, R - 1), colc);
          };
          auto minus_yv = [&](int rb, double4_t& x) {
            const int tr = 16 * rb + lr;  // A-operand row of this lane
#pragma unroll
            for (int t = 0; t < 4; ++t) {
              const int a = 4 * t + kq;
              const double y = Ys[a * n + min(tr, R - 1)];
              x = __builtin_amdgcn_mfma_f64_16x16x4f64((a < nbp && tr < R) ? -y : 0.0, bv[t], x, 0, 0, 0);
            }
          };
          double4_t wt = {0.0, 0.0, 0.0, 0.0};  // W^T X: rows a = kq + 4 v, column lr
          double4_t xc, xn;
          load_tile(0, xc);
          for (int rb = 0; rb < nrb; ++rb) {
            load_tile(min(rb + 1, nrb - 1), xn);
            minus_yv(rb, xc);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
              const int tk = 16 * rb + 4 * t + kq;  // row of X in this k-step
              const double w = Ws[lr * n + min(tk, R - 1)];
              wt = __builtin_amdgcn_mfma_f64_16x16x4f64((lr < nbp && tk < R) ? w : 0.0, xc[t], wt, 0, 0, 0);
            }
            xc = xn;
          }
          load_tile(0, xc);
          for (int rb = 0; rb < nrb; ++rb) {
            load_tile(min(rb + 1, nrb - 1), xn);
            minus_yv(rb, xc);
            const int tr = 16 * rb + lr;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
              const int a = 4 * t + kq;
              const double v = Vs[a * n + min(tr, R - 1)];
              xc = __builtin_amdgcn_mfma_f64_16x16x4f64((a < nbp && tr < R) ? -v : 0.0, wt[t], xc, 0, 0, 0);
            }
            if (col < n)
#pragma unroll
              for (int v = 0; v < 4; ++v) {
                const int t = 16 * rb + kq + 4 * v;
                if (t < R) AH(p + 1 + t, col) = xc[v];
              }
            xc = xn;
          }
        } else {
          const int r0 = (task - ncb) * 16;     // rows r0..r0+15 (those <= p)
          const int ra = min(r0 + lr, p);       // A-operand row of this lane
          // Y_top = A_0[rows, p+1..n-1] W: A = A_0 (row lr, column 4 t + kq), B = W[column][a]
          double4_t yt = {0.0, 0.0, 0.0, 0.0};
          constexpr int kC = 8;
          double ac[kC], an[kC];
#pragma unroll
          for (int u = 0; u < kC; ++u) ac[u] = AH(ra, p + 1 + min(4 * u + kq, R - 1));
          for (int k = 0; k < R; k += 4 * kC) {
#pragma unroll
            for (int u = 0; u < kC; ++u) an[u] = AH(ra, p + 1 + min(k + 4 * kC + 4 * u + kq, R - 1));
#pragma unroll
            for (int u = 0; u < kC; ++u) {
              const int tk = k + 4 * u + kq;
              const double w = Ws[lr * n + min(tk, R - 1)];
              yt = __builtin_amdgcn_mfma_f64_16x16x4f64(ac[u], (lr < nbp && tk < R) ? w : 0.0, yt, 0, 0, 0);
            }
#pragma unroll
            for (int u = 0; u < kC; ++u) ac[u] = an[u];
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) Yt[(kq + 4 * v) * 17 + lr] = yt[v];
          wave_sync();
          double ya[4];  // A of Y_top V^T: Y_top[row lr][a = 4 t + kq]
#pragma unroll
          for (int t = 0; t < 4; ++t) ya[t] = -Yt[lr * 17 + 4 * t + kq];
          for (int cb = 0; cb * 16 < R; ++cb) {
            const int col = p + 1 + cb * 16 + lr, colc = min(col, n - 1);
            double4_t x;
#pragma unroll
            for (int v = 0; v < 4; ++v) x[v] = AH(min(r0 + kq + 4 * v, p), colc);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
              const int a = 4 * t + kq;
              const double b = a < nbp ? Vs[a * n + colc - p - 1] : 0.0;
              x = __builtin_amdgcn_mfma_f64_16x16x4f64(ya[t], b, x, 0, 0, 0);
            }
            if (col < n)
#pragma unroll
              for (int v = 0; v < 4; ++v)
                if (r0 + kq + 4 * v <= p) AH(r0 + kq + 4 * v, col) = x[v];
          }
          wave_sync();  // Yt is read before the wave's next task rewrites it
        }
      }
    }
    __syncthreads();
  }
#undef AH
}

// One double-shift sweep over rows/columns lo..hh - 1 (the three-element steps; the final
// two-element step is left to the caller) of an n x n matrix held in LDS at row stride LD, run by
// one wave: x, y, z carry the reflector input from step to step, rf[3 k .. 3 k + 2] receives
// (tau, u1, u2) of step k, and dum is this lane's private three-double slot beyond the matrix.
template <int LD>
__device__ __forceinline__ void lds_chase(double* __restrict__ H, int n, int lo, int hh, double& x, double& y,
                                          double& z, double* rf, int lane, int W0, int dum) {
  // Off-block work as n - 3 uniform jobs of three elements each: job j < n - k - 3 is
  // column k + 3 + j (rows k..k+2, left update), the rest are rows 0..k-1 (columns
  // k..k+2, right update). Relative to the block origin k (ld + 1) a job starts at
  // 3 + j (stride ld) or at (j - n + 3) ld (stride 1). Each lane owns jobs lane and
  // lane + 64; an idle slot works on its private triple in the LDS tail.
  const int ja = lane, jb = lane + W0;
  for (int k = lo; k < hh - 1; ++k) {
    const int kb = k * (LD + 1);
    double b[4][3];  // rows k..k+3, columns k..k+2 (row k+3 is unused when k+3 > hh)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) b[i][j] = H[kb + i * LD + j];
    const bool cola = k < n - 3 - ja, colb = k < n - 3 - jb;
    int ia = cola ? kb + 3 + ja : kb + (ja - n + 3) * LD, sa = cola ? LD : 1;
    int ib = colb ? kb + 3 + jb : kb + (jb - n + 3) * LD, sb = colb ? LD : 1;
    if (ja >= n - 3) {
      ia = dum;
      sa = 1;
    }
    if (jb >= n - 3) {
      ib = dum;
      sb = 1;
    }
    double va[3], vb[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      va[i] = H[ia + i * sa];
      vb[i] = H[ib + i * sb];
    }
    wave_sync();  // all loads of the step precede its stores
    // Reflector (I - tau u u^T), u = (1, u1, u2), taking (x, y, z) to (beta, 0, 0)
    // with beta = -sign(x) ||(x, y, z)||. Then tau = 1 + |x| / ||.|| and
    // 1 / (x - beta) = sign(x) / (|x| + ||.||): one reciprocal square root and one
    // reciprocal, each refined by two Newton steps. With y = z = 0 the step is the
    // identity (tau = 0, beta = x) and the updates below rewrite the same values.
    double tau = 0.0, u1 = 0.0, u2 = 0.0, beta = x;
    if (y != 0.0 || z != 0.0) {
      double xs = x, ys = y, zs = z, unscale = 1.0;
      double s2 = xs * xs + ys * ys + zs * zs;
      if (s2 < 0x1p-900) {  // keep the squares clear of the subnormal range
        xs *= 0x1p600;
        ys *= 0x1p600;
        zs *= 0x1p600;
        unscale = 0x1p-600;
        s2 = xs * xs + ys * ys + zs * zs;
      }
      double r = __builtin_amdgcn_rsq(s2);
      const double h2 = 0.5 * s2;
      r = r * fma(-h2 * r, r, 1.5);
      r = r * fma(-h2 * r, r, 1.5);
      const double nrm = s2 * r;
      const double ax = fabs(xs);
      tau = fma(ax, r, 1.0);
      const double dd = ax + nrm;
      double q = __builtin_amdgcn_rcp(dd);
      q = fma(q, fma(-dd, q, 1.0), q);
      q = fma(q, fma(-dd, q, 1.0), q);
      const double sc = copysign(q, xs);
      u1 = ys * sc;
      u2 = zs * sc;
      beta = -copysign(nrm, xs) * unscale;
    }
    {
      const double w = tau * (va[0] + u1 * va[1] + u2 * va[2]);
      H[ia] = va[0] - w;
      H[ia + sa] = va[1] - w * u1;
      H[ia + 2 * sa] = va[2] - w * u2;
    }
    {
      const double w = tau * (vb[0] + u1 * vb[1] + u2 * vb[2]);
      H[ib] = vb[0] - w;
      H[ib + sb] = vb[1] - w * u1;
      H[ib + 2 * sb] = vb[2] - w * u2;
    }
    for (int j = lane + 2 * W0; j < n - 3; j += W0) {  // only with fewer than 64 lanes
      const int jj = (j < n - k - 3) ? kb + 3 + j : kb + (j - n + 3) * LD;
      const int st = (j < n - k - 3) ? LD : 1;
      const double w = tau * (H[jj] + u1 * H[jj + st] + u2 * H[jj + 2 * st]);
      H[jj] -= w;
      H[jj + st] -= w * u1;
      H[jj + 2 * st] -= w * u2;
    }
    // corner block: rows k..k+2 from the left, then rows k..k+3 from the right
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double w = tau * (b[0][j] + u1 * b[1][j] + u2 * b[2][j]);
      b[0][j] -= w;
      b[1][j] -= w * u1;
      b[2][j] -= w * u2;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double w = tau * (b[i][0] + u1 * b[i][1] + u2 * b[i][2]);
      b[i][0] -= w;
      b[i][1] -= w * u1;
      b[i][2] -= w * u2;
    }
    if (lane == 0) {
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) H[kb + i * LD + j] = b[i][j];
      if (k + 3 <= hh) {
#pragma unroll
        for (int j = 0; j < 3; ++j) H[kb + 3 * LD + j] = b[3][j];
      }
      if (k > lo) {
        H[kb - 1] = beta;
        H[kb - 1 + LD] = 0.0;
        H[kb - 1 + 2 * LD] = 0.0;
      }
      rf[3 * k] = tau;
      rf[3 * k + 1] = u1;
      rf[3 * k + 2] = u2;
    }
    wave_sync();
    x = b[1][0];
    y = b[2][0];
    z = b[3][0];
  }
}

template <bool kLds>
__device__ __forceinline__ void eigen_body(const Item& it, double* base, int32_t* status, double* sH, double* srefl,
                                           double* sred, int* sctl, double* sxyz, ZOp* zops, int sweep_cap) {
  const int n = it.n;
  double* G = base + (int64_t)kBufG * n * n;
  double* __restrict__ ZT = base + (int64_t)kBufZ * n * n;  // Z(r, c) = ZT[c * n + r]
  double* __restrict__ XT = base + (int64_t)kBufX * n * n;  // eigenvector j, component i at XT[i * n + j]
  double* ex = base + extras_off(n);
  double* lre = ex;
  double* lim = ex + n;
  int* blk = reinterpret_cast<int*>(ex + 3 * n);

  const int tid = threadIdx.x, NT = blockDim.x, lane = tid & 63;
  const bool wave0 = tid < 64;
  const int W0 = NT < 64 ? NT : 64;  // lanes of wave 0
  double* H = kLds ? sH : G;
  // In LDS the row stride is the fixed kLdsMaxn + 1 (offsets become immediates); the rows
  // beyond the matrix and a tail of 3 doubles per lane absorb loads and stores of idle lanes.
  const int64_t ld = kLds ? kLdsMaxn + 1 : n;
  double* sv = srefl;  // Householder vector of the reduction (the reflector buffers are free then)
#define HH(r, c) H[(kLds ? (int64_t)(int)((r) * (int)ld + (c)) : (int64_t)(r) * ld + (c))]
#define ZZ(r, c) ZT[(int64_t)(c) * n + (r)]

  // ---- load, Z = I
  if (kLds)
    for (int t = tid; t < n * n; t += NT) HH(t / n, t % n) = G[t];
  for (int t = tid; t < n * n; t += NT) ZT[t] = ((t / n) == (t % n)) ? 1.0 : 0.0;
  __syncthreads();

  // Frobenius norm (invariant under the orthogonal similarities that follow): backstop scale
  // for deflation in clusters of nearly equal eigenvalues where the local test cannot be met.
  {
    double part = 0.0;
    for (int t = tid; t < n * n; t += NT) {
      const double v = HH(t / n, t % n);
      part += v * v;
    }
    const double nrm2 = block_sum(part, sred);
    if (tid == 0) sxyz[0] = sqrt(nrm2);
    __syncthreads();
  }
  const double hnorm = sxyz[0];
  __syncthreads();

  // ---- 1. Householder reduction to Hessenberg form. Z is not accumulated here: v_k and tau_k
  // of every step go to the workspace (QV) and k_hqapply applies them to the eigenvectors, so the
  // QR phase starts from Z = I. Each dot product of the two-sided update is split over P adjacent
  // lanes (combined by lane exchange) so that all threads work although a step has at most n
  // columns and n rows. The column below the subdiagonal is kept raw in sv (v_0 = 1 and
  // v_i = sv[i] / (x0 - beta)), which lets its norm and its copy share one barrier. Systems kept
  // in global memory take the blocked form (blocked_hessenberg), which produces the same reflectors.
  double* __restrict__ QV = base + (int64_t)kBufYS * n * n;  // v_k at QV[k n + i], tau_k at QV[(n-1) n + k]
  if (!kLds && n <= kWinMaxN) {
    blocked_hessenberg(H, n, QV, sH, sred);
  } else {
    int Pr = 1;
    while (Pr < 4 && n * Pr * 2 <= NT) Pr *= 2;
    const int line_r = hess_line(tid, Pr, NT);
    for (int k = 0; k + 2 < n; ++k) {
      const int len = n - k - 1;
      double part = 0.0;
      for (int i = 1 + tid; i < len; i += NT) {
        const double v = HH(k + 1 + i, k);
        sv[i] = v;
        part += v * v;
      }
      const double x0 = HH(k + 1, k);
      part = wave_sum(part);
      double* red = sred + 8 * (k & 1);  // two reduction slots: no second barrier needed
      if ((tid & 63) == 0) red[tid >> 6] = part;
      __syncthreads();
      double sigma = 0.0;
      for (int w = 0; w < (NT + 63) / 64; ++w) sigma += red[w];
      if (sigma == 0.0) {  // column already reduced (uniform decision)
        if (tid == 0) QV[(int64_t)(n - 1) * n + k] = 0.0;
        continue;
      }
      const double nrm = sqrt(x0 * x0 + sigma);
      const double beta = (x0 >= 0.0) ? -nrm : nrm;
      const double tau = (beta - x0) / beta;
      const double dlt = x0 - beta;
      const double scal = 1.0 / dlt;
      for (int i = tid; i < len; i += NT) {
        QV[(int64_t)k * n + i] = (i == 0) ? 1.0 : sv[i] * scal;
        HH(k + 1 + i, k) = (i == 0) ? beta : 0.0;
      }
      if (tid == 0) QV[(int64_t)(n - 1) * n + k] = tau;
      // left: (I - tau v v^T) H on columns k+1..n-1
      int Pl = 1;
      while (Pl < 8 && len * Pl * 2 <= NT) Pl *= 2;
      const int part_l = tid & (Pl - 1);
      const int line_l = hess_line(tid, Pl, NT);
      for (int c0 = k + 1; c0 < n; c0 += NT / Pl) {
        const int c = c0 + line_l;
        double w = 0.0;
        if (c < n) {
          if (part_l == 0) w = HH(k + 1, c) * dlt;
  #pragma unroll 4
          for (int i = (part_l == 0 ? Pl : part_l); i < len; i += Pl) w += sv[i] * HH(k + 1 + i, c);
        }
        for (int o = 1; o < Pl; o <<= 1) w += __shfl_xor(w, o);
        w *= tau * scal;
        if (c < n) {
          if (part_l == 0) HH(k + 1, c) -= w;
  #pragma unroll 4
          for (int i = (part_l == 0 ? Pl : part_l); i < len; i += Pl) HH(k + 1 + i, c) -= sv[i] * scal * w;
        }
      }
      __syncthreads();
      // right: H (I - tau v v^T), rows 0..n-1
      const int part_r = tid & (Pr - 1);
      for (int r0 = 0; r0 < n; r0 += NT / Pr) {
        const int r = r0 + line_r;
        double y = 0.0;
        if (r < n) {
          if (part_r == 0) y = HH(r, k + 1);
  #pragma unroll 4
          for (int i = (part_r == 0 ? Pr : part_r); i < len; i += Pr) y += HH(r, k + 1 + i) * (sv[i] * scal);
        }
        for (int o = 1; o < Pr; o <<= 1) y += __shfl_xor(y, o);
        y *= tau;
        if (r < n) {
          if (part_r == 0) HH(r, k + 1) -= y;
  #pragma unroll 4
          for (int i = (part_r == 0 ? Pr : part_r); i < len; i += Pr) HH(r, k + 1 + i) -= y * (sv[i] * scal);
        }
      }
      __syncthreads();
    }
  }

  // ---- 2. Francis double-shift QR to real Schur form
  // Wave 0 runs the deflation scan, the shift choice, each sweep's bulge chase and the block
  // splitting on its own (lane-synchronous, no workgroup barrier inside an iteration). The
  // orthogonal factor is updated one iteration behind by the other waves, from the reflectors
  // wave 0 left in LDS, so the two overlap. With a single wave the update follows at once.
  const bool split = NT > 64;
  const int nwave = (NT % 64 == 0) ? NT / 64 : 0;  // waves available for multi-bulge passes
  // Systems in global memory that take the windowed multi-bulge pass also keep wave 0's sweeps and
  // rotations inside the active block [lo, hh] (a block of at most kWin rows is chased in LDS); the
  // parts of H the transformation reaches outside the block (rows above it, columns to its right)
  // are updated with Z by the other waves during the next iteration. Nothing wave 0 reads before
  // that lies there: the next block is the same block, a part of it, or lies above it, and the
  // deflation scan reads near-diagonal entries only (the one in those parts, H(lo - 1, lo), sits
  // beside the zero H(lo, lo - 1), which decides the test on its own).
  const bool dec = !kLds && n <= kWinMaxN && NT >= 64;
  if (tid == 0) {
    sctl[1] = n - 1;  // active bottom index hh
    sctl[2] = 0;      // iterations since last deflation
    sctl[3] = 0;      // total iterations
    sctl[5] = 0;      // failure flag
    zops[0] = zops[1] = ZOp{0, 0, 0, 0, 0};
  }
  __syncthreads();
  for (int iter = 0;; ++iter) {
    const int slot = iter & 1;
    double* rf = srefl + slot * 3 * kMaxn;
    if (wave0) {
      const int hh = __builtin_amdgcn_readfirstlane(sctl[1]);
      if (hh < 0) {
        if (lane == 0) zops[slot] = ZOp{0, 0, 0, 1, 0};
      } else {
        // scanned from the bottom, W0 rows at a time: the first group with a negligible
        // subdiagonal entry holds the lowest one
        int l = 0;
        for (int top = hh; top >= 1; top -= W0) {
          int cand = 0;
          const int k = top - lane;
          if (k >= 1) {
            const double hk = fabs(HH(k, k - 1));
            bool small = hk <= kSafeMin || (sctl[2] >= 40 && hk <= kUlp * hnorm);
            if (!small) {
              double tst = fabs(HH(k - 1, k - 1)) + fabs(HH(k, k));
              if (tst == 0.0) {
                if (k >= 2) tst += fabs(HH(k - 1, k - 2));
                if (k + 1 <= hh) tst += fabs(HH(k + 1, k));
              }
              if (hk <= kUlp * tst) {
                const double hu = fabs(HH(k - 1, k));
                const double ab = fmax(hk, hu), ba = fmin(hk, hu);
                const double dd = fabs(HH(k - 1, k - 1) - HH(k, k));
                const double aa = fmax(fabs(HH(k, k)), dd), bb = fmin(fabs(HH(k, k)), dd);
                const double s = aa + ab;
                small = ba * (ab / s) <= fmax(kSafeMin, kUlp * (bb * (aa / s)));
              }
            }
            if (small) cand = k;
          }
          l = __builtin_amdgcn_readfirstlane(wave_max(cand));
          if (l > 0) break;
        }
        if (lane == 0) {
          zops[slot] = ZOp{0, 0, 0, 0, 0};
          if (l > 0) HH(l, l - 1) = 0.0;
          if (l == hh) {  // 1x1 block
            lre[hh] = HH(hh, hh);
            lim[hh] = 0.0;
            blk[hh] = 1;
            sctl[1] = hh - 1;
            sctl[2] = 0;
            sctl[4] = kActDeflated;
          } else if (l == hh - 1) {  // 2x2 block
            const double a = HH(hh - 1, hh - 1), b = HH(hh - 1, hh), c = HH(hh, hh - 1), d = HH(hh, hh);
            const double p = 0.5 * (a - d), bc = b * c, disc = p * p + bc;
            if (disc >= 0.0) {
              // real pair: rotate the block to upper triangular form (first column = eigenvector
              // of the first eigenvalue) so that both become 1x1 blocks
              const double zz = p + copysign(sqrt(disc), p);
              const double l1 = d + zz;
              double v0 = b, v1 = l1 - a;
              const double w0 = l1 - d, w1 = c;
              if (fabs(w0) + fabs(w1) > fabs(v0) + fabs(v1)) {
                v0 = w0;
                v1 = w1;
              }
              const double nv = hypot(v0, v1);
              sxyz[0] = (nv > 0.0) ? v0 / nv : 1.0;
              sxyz[1] = (nv > 0.0) ? v1 / nv : 0.0;
              sctl[4] = kActRotate;
            } else {
              lre[hh - 1] = lre[hh] = 0.5 * (a + d);
              lim[hh - 1] = sqrt(-disc);
              lim[hh] = -sqrt(-disc);
              blk[hh - 1] = 2;
              blk[hh] = 0;
              sctl[1] = hh - 2;
              sctl[2] = 0;
              sctl[4] = kActDeflated;
            }
          } else {
            const int its = ++sctl[2];
            const int tot = ++sctl[3];
            if (its > 100 || tot > 60 * n || (sweep_cap > 0 && tot > sweep_cap)) {
              sctl[5] = 1;
              sctl[1] = -1;
              sctl[4] = kActStop;
              zops[slot].stop = 1;
            } else if (nwave >= 2 && its < (!kLds && n <= kWinMaxN ? kMultiItsWindowed : kMultiIts) && hh - l + 1 >= kMultiMin) {
              // one shift pair per bulge: the eigenvalues of the 2x2 diagonal blocks ending at
              // rows hh, hh - 2, ... (both roots of a real pair), stored in this slot's buffer
              const int nb = nwave < kMaxBulges ? nwave : kMaxBulges;
              for (int bq = 0; bq < nb; ++bq) {
                const int j = hh - 2 * bq;
                const double a = HH(j - 1, j - 1), b = HH(j - 1, j), c = HH(j, j - 1), d = HH(j, j);
                const double p = 0.5 * (a - d), bc = b * c, disc = p * p + bc;
                double s1r, s1i, s2r, s2i;
                if (disc >= 0.0) {
                  const double zz = p + copysign(sqrt(disc), p);
                  s1r = d + zz;
                  s2r = (zz != 0.0) ? d - bc / zz : d;
                  s1i = s2i = 0.0;
                } else {
                  s1r = s2r = d + p;
                  s1i = sqrt(-disc);
                  s2i = -s1i;
                }
                rf[4 * bq] = s1r;
                rf[4 * bq + 1] = s1i;
                rf[4 * bq + 2] = s2r;
                rf[4 * bq + 3] = s2i;
              }
              zops[slot] = ZOp{0, l, hh, 0, nb};
              sctl[4] = kActMulti;
            } else {
              double h11, h12, h21, h22;
              if (its % 20 == 10) {
                const double s = fabs(HH(l + 1, l)) + fabs(HH(l + 2, l + 1));
                h11 = 0.75 * s + HH(l, l);
                h12 = -0.4375 * s;
                h21 = s;
                h22 = h11;
              } else if (its % 20 == 0) {
                const double s = fabs(HH(hh, hh - 1)) + fabs(HH(hh - 1, hh - 2));
                h11 = 0.75 * s + HH(hh, hh);
                h12 = -0.4375 * s;
                h21 = s;
                h22 = h11;
              } else {
                h11 = HH(hh - 1, hh - 1);
                h12 = HH(hh - 1, hh);
                h21 = HH(hh, hh - 1);
                h22 = HH(hh, hh);
              }
              // shifts = eigenvalues of [[h11, h12], [h21, h22]]; a real pair is replaced by the
              // root closer to h22 used twice (keeps the iteration from stagnating on real clusters)
              double s1r, s1i, s2r, s2i;
              {
                const double hp = 0.5 * (h11 - h22), bc = h12 * h21, disc = hp * hp + bc;
                if (disc >= 0.0) {
                  const double zz = hp + copysign(sqrt(disc), hp);
                  const double d1 = zz, d2 = (zz != 0.0) ? -bc / zz : 0.0;  // root - h22
                  const double rt = h22 + ((fabs(d1) <= fabs(d2)) ? d1 : d2);
                  s1r = s2r = rt;
                  s1i = s2i = 0.0;
                } else {
                  s1r = s2r = h22 + hp;
                  s1i = sqrt(-disc);
                  s2i = -s1i;
                }
              }
              // first column of (H - s1)(H - s2) at row l, in product form (no cancellation)
              const double a0 = HH(l, l), a1 = HH(l + 1, l);
              const double sc = fabs(a0 - s2r) + fabs(s2i) + fabs(a1);
              const double a1s = a1 / sc;
              sxyz[0] = a1s * HH(l, l + 1) + (a0 - s1r) * ((a0 - s2r) / sc) - s1i * (s2i / sc);
              sxyz[1] = a1s * (a0 + HH(l + 1, l + 1) - s1r - s2r);
              sxyz[2] = a1s * HH(l + 2, l + 1);
              sctl[6] = l;
              sctl[4] = kActSweep;
            }
          }
        }
        wave_sync();
        const int act = __builtin_amdgcn_readfirstlane(sctl[4]);
        if (act == kActSweep) {
          // Bulge chase over rows/columns lo..hh. A three-element step k touches rows k..k+2
          // (columns >= k) and columns k..k+2 (rows <= k+3); every lane loads the 4 x 3 corner
          // block those share, updates it itself (left, then right) and so holds the next
          // step's reflector input, column k rows k+1..k+3, in registers. The loads of a step
          // are issued before its reflector is formed.
          const int lo = __builtin_amdgcn_readfirstlane(sctl[6]);
          double x = sxyz[0], y = sxyz[1], z = sxyz[2];
          const bool blk_lds = dec && hh - lo + 1 <= kWin;
          if constexpr (kLds) {
            lds_chase<kLdsMaxn + 1>(H, n, lo, hh, x, y, z, rf, lane, W0, kLdsMaxn * (kLdsMaxn + 1) + 3 * lane);
          } else if (blk_lds) {
            // The block rows/columns lo..hh moves to LDS (row stride kWinLd), is chased there as
            // a matrix of its own and goes back; a lane's private slots lie after row kWin.
            const int m = hh - lo + 1;
            double* __restrict__ B = sH;
            for (int r0 = 0; r0 < m; r0 += 4) {
              double v[4][2];  // loads of four rows in flight (clamped indexes, stores masked)
              const int c0 = min(lane, m - 1), c1 = min(lane + 64, m - 1);
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const int r = min(r0 + i, m - 1);
                v[i][0] = HH(lo + r, lo + c0);
                v[i][1] = HH(lo + r, lo + c1);
              }
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                if (r0 + i < m) {
                  if (lane < m) B[(r0 + i) * kWinLd + lane] = v[i][0];
                  if (lane + 64 < m) B[(r0 + i) * kWinLd + lane + 64] = v[i][1];
                }
              }
            }
            wave_sync();
            lds_chase<kWinLd>(B, m, 0, m - 1, x, y, z, rf + 3 * lo, lane, 64, kWin * kWinLd + 3 * lane);
            {  // final two-element step on block rows/columns m - 2, m - 1
              const int k = m - 2;
              const double nrm = sqrt(x * x + y * y);
              double tau = 0.0, u1 = 0.0, beta = 0.0;
              if (nrm != 0.0 && y != 0.0) {
                beta = (x >= 0.0) ? -nrm : nrm;
                tau = (beta - x) / beta;
                u1 = y / (x - beta);
              }
              if (tau != 0.0) {
                if (lane == 0) {
                  B[k * kWinLd + k - 1] = beta;
                  B[(k + 1) * kWinLd + k - 1] = 0.0;
                }
                if (lane < 2) {
                  const int c = k + lane;
                  const double w = tau * (B[k * kWinLd + c] + u1 * B[(k + 1) * kWinLd + c]);
                  B[k * kWinLd + c] -= w;
                  B[(k + 1) * kWinLd + c] -= w * u1;
                }
                wave_sync();
                for (int r = lane; r < m; r += 64) {
                  const double w = tau * (B[r * kWinLd + k] + u1 * B[r * kWinLd + k + 1]);
                  B[r * kWinLd + k] -= w;
                  B[r * kWinLd + k + 1] -= w * u1;
                }
              }
              if (lane == 0) {
                rf[3 * (hh - 1)] = tau;
                rf[3 * (hh - 1) + 1] = u1;
                rf[3 * (hh - 1) + 2] = 0.0;
                zops[slot] = ZOp{1, lo, hh, 0, 0};
              }
              wave_sync();
            }
            for (int r = 0; r < m; ++r) {
              if (lane < m) HH(lo + r, lo + lane) = B[r * kWinLd + lane];
              if (lane + 64 < m) HH(lo + r, lo + lane + 64) = B[r * kWinLd + lane + 64];
            }
            wave_sync();
          } else {
          for (int k = lo; k < hh - 1; ++k) {
            const bool row3 = k + 3 <= hh;
            double b[4][3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
              for (int j = 0; j < 3; ++j) b[i][j] = HH(k + i, k + j);
#pragma unroll
            for (int j = 0; j < 3; ++j) b[3][j] = row3 ? HH(k + 3, k + j) : 0.0;
            // Off-block work as uniform jobs of three elements each: job j < ncol is column
            // k + 3 + j (rows k..k+2, left update), the rest are rows rbeg..k-1 (columns
            // k..k+2, right update), over the whole matrix (rbeg = 0, cend = n) or, with the
            // block-local updates, the block (rbeg = lo, cend = hh + 1). The first two jobs of
            // each lane are loaded up front.
            const int cend = dec ? hh + 1 : n, rbeg = dec ? lo : 0;
            const int ncol = cend - k - 3, njob = cend - rbeg - 3;
            int64_t ja = 0, jb = 0, sa = 1, sb = 1;
            double va[3] = {0.0, 0.0, 0.0}, vb[3] = {0.0, 0.0, 0.0};
            const bool ha = lane < njob, hb = lane + W0 < njob;
            if (ha) {
              const int j = lane;
              ja = (j < ncol) ? (int64_t)k * ld + k + 3 + j : (int64_t)(rbeg + j - ncol) * ld + k;
              sa = (j < ncol) ? ld : 1;
#pragma unroll
              for (int i = 0; i < 3; ++i) va[i] = H[ja + i * sa];
            }
            if (hb) {
              const int j = lane + W0;
              jb = (j < ncol) ? (int64_t)k * ld + k + 3 + j : (int64_t)(rbeg + j - ncol) * ld + k;
              sb = (j < ncol) ? ld : 1;
#pragma unroll
              for (int i = 0; i < 3; ++i) vb[i] = H[jb + i * sb];
            }
            wave_sync();  // all loads of the step precede its stores
            // Reflector (I - tau u u^T), u = (1, u1, u2), taking (x, y, z) to (beta, 0, 0) with
            // beta = -sign(x) ||(x, y, z)||. Then tau = 1 + |x| / ||.|| and 1 / (x - beta) =
            // sign(x) / (|x| + ||.||): one reciprocal square root and one reciprocal, each
            // refined by two Newton steps.
            double tau = 0.0, u1 = 0.0, u2 = 0.0, beta = 0.0;
            if (y != 0.0 || z != 0.0) {
              double xs = x, ys = y, zs = z, unscale = 1.0;
              double s2 = xs * xs + ys * ys + zs * zs;
              if (s2 < 0x1p-900) {  // keep the squares clear of the subnormal range
                xs *= 0x1p600;
                ys *= 0x1p600;
                zs *= 0x1p600;
                unscale = 0x1p-600;
                s2 = xs * xs + ys * ys + zs * zs;
              }
              double r = __builtin_amdgcn_rsq(s2);
              const double h2 = 0.5 * s2;
              r = r * fma(-h2 * r, r, 1.5);
              r = r * fma(-h2 * r, r, 1.5);
              const double nrm = s2 * r;
              const double ax = fabs(xs);
              tau = fma(ax, r, 1.0);
              const double dd = ax + nrm;
              double q = __builtin_amdgcn_rcp(dd);
              q = fma(q, fma(-dd, q, 1.0), q);
              q = fma(q, fma(-dd, q, 1.0), q);
              const double sc = copysign(q, xs);
              u1 = ys * sc;
              u2 = zs * sc;
              beta = -copysign(nrm, xs) * unscale;
            }
            if (tau != 0.0) {
              if (ha) {
                const double w = tau * (va[0] + u1 * va[1] + u2 * va[2]);
                H[ja] = va[0] - w;
                H[ja + sa] = va[1] - w * u1;
                H[ja + 2 * sa] = va[2] - w * u2;
              }
              if (hb) {
                const double w = tau * (vb[0] + u1 * vb[1] + u2 * vb[2]);
                H[jb] = vb[0] - w;
                H[jb + sb] = vb[1] - w * u1;
                H[jb + 2 * sb] = vb[2] - w * u2;
              }
              for (int j = lane + 2 * W0; j < njob; j += W0) {
                const int64_t jj = (j < ncol) ? (int64_t)k * ld + k + 3 + j : (int64_t)(rbeg + j - ncol) * ld + k;
                const int64_t st = (j < ncol) ? ld : 1;
                const double w = tau * (H[jj] + u1 * H[jj + st] + u2 * H[jj + 2 * st]);
                H[jj] -= w;
                H[jj + st] -= w * u1;
                H[jj + 2 * st] -= w * u2;
              }
              // corner block: rows k..k+2 from the left, then rows k..k+3 from the right
#pragma unroll
              for (int j = 0; j < 3; ++j) {
                const double w = tau * (b[0][j] + u1 * b[1][j] + u2 * b[2][j]);
                b[0][j] -= w;
                b[1][j] -= w * u1;
                b[2][j] -= w * u2;
              }
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const double w = tau * (b[i][0] + u1 * b[i][1] + u2 * b[i][2]);
                b[i][0] -= w;
                b[i][1] -= w * u1;
                b[i][2] -= w * u2;
              }
              if (lane == 0) {
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                  for (int j = 0; j < 3; ++j) HH(k + i, k + j) = b[i][j];
                if (row3) {
#pragma unroll
                  for (int j = 0; j < 3; ++j) HH(k + 3, k + j) = b[3][j];
                }
                if (k > lo) {
                  HH(k, k - 1) = beta;
                  HH(k + 1, k - 1) = 0.0;
                  HH(k + 2, k - 1) = 0.0;
                }
              }
            }
            if (lane == 0) {
              rf[3 * k] = tau;
              rf[3 * k + 1] = u1;
              rf[3 * k + 2] = u2;
            }
            wave_sync();
            x = b[1][0];
            y = b[2][0];
            z = b[3][0];
          }
          }
          if (!blk_lds) {  // final two-element step k = hh - 1 on rows/columns hh-1, hh
            const int k = hh - 1;
            const double nrm = sqrt(x * x + y * y);
            double tau = 0.0, u1 = 0.0, beta = 0.0;
            if (nrm != 0.0 && y != 0.0) {
              beta = (x >= 0.0) ? -nrm : nrm;
              tau = (beta - x) / beta;
              u1 = y / (x - beta);
            }
            if (tau != 0.0) {
              if (lane == 0) {
                HH(k, k - 1) = beta;
                HH(k + 1, k - 1) = 0.0;
              }
              for (int c = k + lane; c < (dec ? hh + 1 : n); c += W0) {
                const double w = tau * (HH(k, c) + u1 * HH(k + 1, c));
                HH(k, c) -= w;
                HH(k + 1, c) -= w * u1;
              }
              wave_sync();
              for (int r = (dec ? lo : 0) + lane; r <= hh; r += W0) {
                const double w = tau * (HH(r, k) + u1 * HH(r, k + 1));
                HH(r, k) -= w;
                HH(r, k + 1) -= w * u1;
              }
            }
            if (lane == 0) {
              rf[3 * k] = tau;
              rf[3 * k + 1] = u1;
              rf[3 * k + 2] = 0.0;
              zops[slot] = ZOp{1, lo, hh, 0, 0};
            }
            wave_sync();
          }
        } else if (act == kActRotate) {  // split a real 2x2 block with [[cs, -sn], [sn, cs]]
          const int h1 = hh - 1;
          const double cs = sxyz[0], sn = sxyz[1];
          for (int c = h1 + lane; c < (dec ? hh + 1 : n); c += W0) {
            const double x = HH(h1, c), y = HH(hh, c);
            HH(h1, c) = cs * x + sn * y;
            HH(hh, c) = -sn * x + cs * y;
          }
          wave_sync();
          for (int r = (dec ? h1 : 0) + lane; r <= hh; r += W0) {
            const double x = HH(r, h1), y = HH(r, hh);
            HH(r, h1) = cs * x + sn * y;
            HH(r, hh) = -sn * x + cs * y;
          }
          wave_sync();
          if (lane == 0) {
            HH(hh, h1) = 0.0;
            lre[h1] = HH(h1, h1);
            lre[hh] = HH(hh, hh);
            lim[h1] = 0.0;
            lim[hh] = 0.0;
            blk[h1] = 1;
            blk[hh] = 1;
            sctl[1] = hh - 2;
            sctl[2] = 0;
            rf[0] = cs;
            rf[1] = sn;
            zops[slot] = ZOp{2, 0, hh, 0, 0};
          }
          wave_sync();
        }
      }
    }
    if (split) {
      if (!wave0 && iter > 0)
        apply_zop(zops[slot ^ 1], srefl + (slot ^ 1) * 3 * kMaxn, ZT, dec ? H : nullptr, n, tid - 64, NT - 64);
    } else {
      wave_sync();
      apply_zop(zops[slot], rf, ZT, dec ? H : nullptr, n, tid, NT);
    }
    __syncthreads();
    const ZOp op = zops[slot];  // not rewritten before the barrier of the next iteration
    if (!kLds && op.nb > 0 && n <= kWinMaxN) {
      windowed_multibulge(H, n, ZT, op.lo, op.hh, op.nb, srefl + slot * 3 * kMaxn, sH);
    } else if (op.nb > 0) {
      // Multi-bulge pass: wave b chases bulge b, kMultiGap rows behind bulge b - 1. A chain step
      // moves every bulge one row: each wave forms its reflector (from column k - 1, or from the
      // shift polynomial when it enters at row lo), applies it from the left to rows k..k+2,
      // then after a barrier from the right to columns k..k+2 of H and Z. Rows of different
      // bulges in a left phase and columns in a right phase are disjoint, and a bulge's
      // reflector input is not touched by the neighbours within a step (gap >= 4).
      // With H in LDS (n <= 128) the wave's three columns of Z (k..k+2, rows lane and lane + 64)
      // stay in registers from step to step: after a step, column k is final for this bulge and is
      // stored, the other two move down, and column k+3 is loaded for the next step (no bulge
      // touches it in this step: the one ahead works on k+4..k+6, and wrote k+3 in the previous
      // step). Larger systems update their columns of Z in global memory at every step.
      const int lo = op.lo, hh = op.hh, nb = op.nb, wv = tid >> 6;
      const double* sh = srefl + slot * 3 * kMaxn;
      const int nsteps = (hh - lo) + kMultiGap * (nb - 1);
      const int zr0 = lane, zr1 = min(lane + 64, n - 1);
      const bool zv1 = lane + 64 < n;
      double z00 = 0.0, z01 = 0.0, z02 = 0.0, z10 = 0.0, z11 = 0.0, z12 = 0.0;
      for (int t = 0; t < nsteps; ++t) {
        const int k = lo + t - kMultiGap * wv;
        const bool on = wv < nb && k >= lo && k <= hh - 1;
        const bool three = k < hh - 1;
        if (kLds && on && k == lo && lane < n) {  // the bulge enters: its first three columns
          z00 = ZZ(zr0, lo);
          z01 = ZZ(zr0, lo + 1);
          z02 = ZZ(zr0, lo + 2);
          z10 = ZZ(zr1, lo);
          z11 = ZZ(zr1, lo + 1);
          z12 = ZZ(zr1, lo + 2);
        }
        double tau = 0.0, u1 = 0.0, u2 = 0.0, beta = 0.0;
        if (on) {
          double x, y, z;
          if (k == lo) {
            const double s1r = sh[4 * wv], s1i = sh[4 * wv + 1], s2r = sh[4 * wv + 2], s2i = sh[4 * wv + 3];
            const double a0 = HH(lo, lo), a1 = HH(lo + 1, lo);
            const double sc = fabs(a0 - s2r) + fabs(s2i) + fabs(a1);
            const double a1s = a1 / sc;
            x = a1s * HH(lo, lo + 1) + (a0 - s1r) * ((a0 - s2r) / sc) - s1i * (s2i / sc);
            y = a1s * (a0 + HH(lo + 1, lo + 1) - s1r - s2r);
            z = a1s * HH(lo + 2, lo + 1);
          } else {
            x = HH(k, k - 1);
            y = HH(k + 1, k - 1);
            z = three ? HH(k + 2, k - 1) : 0.0;
          }
          wave_sync();  // every lane has read its input before the left phase overwrites it
          beta = x;
          if (y != 0.0 || z != 0.0) {
            double xs = x, ys = y, zs = z, unscale = 1.0;
            double s2 = xs * xs + ys * ys + zs * zs;
            if (s2 < 0x1p-900) {
              xs *= 0x1p600;
              ys *= 0x1p600;
              zs *= 0x1p600;
              unscale = 0x1p-600;
              s2 = xs * xs + ys * ys + zs * zs;
            }
            double r = __builtin_amdgcn_rsq(s2);
            const double h2 = 0.5 * s2;
            r = r * fma(-h2 * r, r, 1.5);
            r = r * fma(-h2 * r, r, 1.5);
            const double nrm = s2 * r;
            const double ax = fabs(xs);
            tau = fma(ax, r, 1.0);
            const double dd = ax + nrm;
            double q = __builtin_amdgcn_rcp(dd);
            q = fma(q, fma(-dd, q, 1.0), q);
            q = fma(q, fma(-dd, q, 1.0), q);
            const double sc = copysign(q, xs);
            u1 = ys * sc;
            u2 = zs * sc;
            beta = -copysign(nrm, xs) * unscale;
          }
          if (tau != 0.0) {
            if (lane == 0 && k > lo) {
              HH(k, k - 1) = beta;
              HH(k + 1, k - 1) = 0.0;
              if (three) HH(k + 2, k - 1) = 0.0;
            }
            if (three) {
              for (int c = k + lane; c < n; c += 64) {
                const double h0 = HH(k, c), h1 = HH(k + 1, c), h2 = HH(k + 2, c);
                const double w = tau * (h0 + u1 * h1 + u2 * h2);
                HH(k, c) = h0 - w;
                HH(k + 1, c) = h1 - w * u1;
                HH(k + 2, c) = h2 - w * u2;
              }
            } else {
              for (int c = k + lane; c < n; c += 64) {
                const double h0 = HH(k, c), h1 = HH(k + 1, c);
                const double w = tau * (h0 + u1 * h1);
                HH(k, c) = h0 - w;
                HH(k + 1, c) = h1 - w * u1;
              }
            }
          }
        }
        __syncthreads();
        if (on && tau != 0.0) {
          const int rmax = min(k + 3, hh);
          if (three) {
            for (int r = lane; r <= rmax; r += 64) {
              const double h0 = HH(r, k), h1 = HH(r, k + 1), h2 = HH(r, k + 2);
              const double w = tau * (h0 + u1 * h1 + u2 * h2);
              HH(r, k) = h0 - w;
              HH(r, k + 1) = h1 - w * u1;
              HH(r, k + 2) = h2 - w * u2;
            }
            if constexpr (kLds) {
              const double w0 = tau * (z00 + u1 * z01 + u2 * z02), w1 = tau * (z10 + u1 * z11 + u2 * z12);
              z00 -= w0;
              z01 -= w0 * u1;
              z02 -= w0 * u2;
              z10 -= w1;
              z11 -= w1 * u1;
              z12 -= w1 * u2;
            } else {
              for (int r = lane; r < n; r += 64) {
                const double z0 = ZZ(r, k), z1 = ZZ(r, k + 1), z2 = ZZ(r, k + 2);
                const double w = tau * (z0 + u1 * z1 + u2 * z2);
                ZZ(r, k) = z0 - w;
                ZZ(r, k + 1) = z1 - w * u1;
                ZZ(r, k + 2) = z2 - w * u2;
              }
            }
          } else {
            for (int r = lane; r <= rmax; r += 64) {
              const double h0 = HH(r, k), h1 = HH(r, k + 1);
              const double w = tau * (h0 + u1 * h1);
              HH(r, k) = h0 - w;
              HH(r, k + 1) = h1 - w * u1;
            }
            if constexpr (kLds) {
              const double w0 = tau * (z00 + u1 * z01), w1 = tau * (z10 + u1 * z11);
              z00 -= w0;
              z01 -= w0 * u1;
              z10 -= w1;
              z11 -= w1 * u1;
            } else {
              for (int r = lane; r < n; r += 64) {
                const double z0 = ZZ(r, k), z1 = ZZ(r, k + 1);
                const double w = tau * (z0 + u1 * z1);
                ZZ(r, k) = z0 - w;
                ZZ(r, k + 1) = z1 - w * u1;
              }
            }
          }
        }
        if (kLds && on && lane < n) {  // column k is final for this bulge; at its last step column k+1 too
          ZZ(zr0, k) = z00;
          if (zv1) ZZ(zr1, k) = z10;
          if (three) {
            z00 = z01;
            z01 = z02;
            z10 = z11;
            z11 = z12;
            if (k + 3 <= hh) {
              z02 = ZZ(zr0, k + 3);
              z12 = ZZ(zr1, k + 3);
            }
          } else {
            ZZ(zr0, k + 1) = z01;
            if (zv1) ZZ(zr1, k + 1) = z11;
          }
        }
        __syncthreads();
      }
    }
    if (op.stop) break;
  }
  if (sctl[5]) {
    if (tid == 0) status[it.layer] = -5;
    return;
  }

  // ---- 3. eigenvectors of the quasi-triangular factor T by back-substitution. Eigenvalues
  // closer than a few ulp ||G|| cannot be told apart: a diagonal entry (or 2x2 block) that close to
  // lambda is another copy of the same multiple eigenvalue of a diagonalisable matrix (e.g. the
  // unscattered Stokes components at one node, lambda = 1/mu^2), and its Schur coupling is
  // rounding noise. Its component is set to zero instead of dividing the noise by a guarded pivot,
  // which would make the copies' eigenvectors parallel.
  const double same = 8.0 * kUlp * hnorm;
  if constexpr (kLds) {
    // All eigenvectors advance together over T's diagonal blocks from the bottom: the block's
    // rows of T are staged in LDS (the same for every thread) and the eigenvector matrix X
    // replaces T in the LDS array, so every dependent read stays in LDS. T itself goes to the
    // workspace first.
    double* TG = base + (int64_t)kBufYT * n * n;
    for (int t = tid; t < n * n; t += NT) TG[t] = HH(t / n, t % n);
    __syncthreads();
    double* X = sH;  // X(i, j) at X[i * ld + j]
    double* trow = srefl;  // rows s and i of the current block: [2][n]
    for (int t = tid; t < n * ld; t += NT) X[t] = 0.0;
    __syncthreads();
    // own blocks (the rest of each column stays zero below them)
    for (int j = tid; j < n; j += NT) {
      const double wr = lre[j], wi = lim[j];
      if (wi < 0.0) continue;  // second member of a complex pair: written by j - 1
      const int b0 = (blk[j] == 0) ? j - 1 : j;
      const int bend = (blk[b0] == 2) ? b0 + 1 : b0;
      const bool cplx = wi > 0.0;
      const Cx lam{wr, wi};
      Cx xb0{0.0, 0.0}, xb1{0.0, 0.0};
      if (bend == b0) {
        xb0 = {1.0, 0.0};
      } else {
        const Cx a{TG[(int64_t)b0 * n + b0], 0.0}, bb{TG[(int64_t)b0 * n + b0 + 1], 0.0};
        const Cx c{TG[(int64_t)(b0 + 1) * n + b0], 0.0}, d{TG[(int64_t)(b0 + 1) * n + b0 + 1], 0.0};
        const Cx v0a = bb, v1a = csub(lam, a);  // (b, lambda - a)
        const Cx v0b = csub(lam, d), v1b = c;   // (lambda - d, c)
        if (cabs1(v0a) + cabs1(v1a) >= cabs1(v0b) + cabs1(v1b)) {
          xb0 = v0a;
          xb1 = v1a;
        } else {
          xb0 = v0b;
          xb1 = v1b;
        }
        if (cabs1(xb0) + cabs1(xb1) == 0.0) {
          if (j == b0) xb0 = {1.0, 0.0}; else xb1 = {1.0, 0.0};
        }
      }
      X[b0 * ld + j] = xb0.re;
      if (cplx) X[b0 * ld + j + 1] = xb0.im;
      if (bend > b0) {
        X[bend * ld + j] = xb1.re;
        if (cplx) X[bend * ld + j + 1] = xb1.im;
      }
    }
    // the next block's rows are loaded into registers while the current block is solved
    double ps[4], pi[4];
    auto fetch_rows = [&](int sbq, int iq) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = tid + q * NT;
        if (c < n) {
          ps[q] = TG[(int64_t)sbq * n + c];
          pi[q] = TG[(int64_t)iq * n + c];
        }
      }
    };
    fetch_rows((blk[n - 1] == 0) ? n - 2 : n - 1, n - 1);
    for (int i = n - 1; i >= 0;) {
      const int sb = (blk[i] == 0) ? i - 1 : i;  // block rows [sb, i]
      __syncthreads();  // previous block's rows are no longer read
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = tid + q * NT;
        if (c < n) {
          trow[c] = ps[q];
          trow[n + c] = pi[q];
        }
      }
      for (int c = tid + 4 * NT; c < n; c += NT) {  // only with fewer than n / 4 threads
        trow[c] = TG[(int64_t)sb * n + c];
        trow[n + c] = TG[(int64_t)i * n + c];
      }
      if (sb > 0) fetch_rows((blk[sb - 1] == 0) ? sb - 2 : sb - 1, sb - 1);
      __syncthreads();
      // four lanes per eigenvector: each sums every fourth term of the row products, combined by
      // two lane exchanges (outside any per-eigenvector branch), then lane 0 of the four solves
      const int lpv = (NT >= 64) ? 4 : 1;  // lanes per eigenvector (1 only for tiny test blocks)
      for (int j0 = 0; j0 < n; j0 += NT / lpv) {
        const int j = j0 + tid / lpv, part = tid % lpv;
        bool act = j < n;
        double wr = 0.0, wi = 0.0;
        int b0 = 0, bend = 0;
        if (act) {
          wr = lre[j];
          wi = lim[j];
          b0 = (blk[j] == 0) ? j - 1 : j;
          bend = (blk[b0] == 2) ? b0 + 1 : b0;
          act = !(wi < 0.0) && i < b0;  // second member of a pair, or not above the own block
        }
        const bool cplx = wi > 0.0;
        const double* ts = trow;
        const double* ti = trow + n;
        double p0r = 0.0, p0i = 0.0, p1r = 0.0, p1i = 0.0;
        if (act) {
          if (cplx) {
            for (int c = i + 1 + part; c <= bend; c += lpv) {
              const double xr = X[c * ld + j], xi = X[c * ld + j + 1];
              p0r -= ts[c] * xr;
              p0i -= ts[c] * xi;
              p1r -= ti[c] * xr;
              p1i -= ti[c] * xi;
            }
          } else {
            for (int c = i + 1 + part; c <= bend; c += lpv) {
              const double xc = X[c * ld + j];
              p0r -= ts[c] * xc;
              p1r -= ti[c] * xc;
            }
          }
        }
        if (lpv == 4) {
          p0r += __shfl_xor(p0r, 1);
          p0i += __shfl_xor(p0i, 1);
          p1r += __shfl_xor(p1r, 1);
          p1i += __shfl_xor(p1i, 1);
          p0r += __shfl_xor(p0r, 2);
          p0i += __shfl_xor(p0i, 2);
          p1r += __shfl_xor(p1r, 2);
          p1i += __shfl_xor(p1i, 2);
        }
        if (!act || part != 0) continue;
        const double smin = fmax(kUlp * (fabs(wr) + fabs(wi)), kSafeMin);
        const Cx lam{wr, wi};
        const Cx r0{p0r, p0i}, r1{p1r, p1i};
        if (sb == i) {
          const Cx d0 = csub(Cx{ti[i], 0.0}, lam);
          const Cx xi = (cabs1(d0) <= same) ? Cx{0.0, 0.0} : cdiv(r0, cguard(d0, smin));
          X[i * ld + j] = xi.re;
          if (cplx) X[i * ld + j + 1] = xi.im;
        } else if (cabs1(csub(Cx{lre[sb], lim[sb]}, lam)) <= same || cabs1(csub(Cx{lre[i], lim[i]}, lam)) <= same) {
          X[sb * ld + j] = 0.0;
          X[i * ld + j] = 0.0;
          if (cplx) {
            X[sb * ld + j + 1] = 0.0;
            X[i * ld + j + 1] = 0.0;
          }
        } else {
          Cx x0, x1;
          csolve2(csub(Cx{ts[sb], 0.0}, lam), Cx{ts[i], 0.0}, Cx{ti[sb], 0.0}, csub(Cx{ti[i], 0.0}, lam), r0, r1,
                  smin, x0, x1);
          X[sb * ld + j] = x0.re;
          X[i * ld + j] = x1.re;
          if (cplx) {
            X[sb * ld + j + 1] = x0.im;
            X[i * ld + j + 1] = x1.im;
          }
        }
      }
      i = sb - 1;
    }
    __syncthreads();
    // normalise (max modulus component -> 1) and write out
    for (int j = tid; j < n; j += NT) {
      const double wi = lim[j];
      if (wi < 0.0) continue;
      const bool cplx = wi > 0.0;
      double mx = 0.0;
      for (int q = 0; q < n; ++q) {
        double v = fabs(X[q * ld + j]);
        if (cplx) v += fabs(X[q * ld + j + 1]);
        mx = fmax(mx, v);
      }
      const double sc = (mx > 0.0) ? 1.0 / mx : 1.0;
      for (int q = 0; q < n; ++q) {
        X[q * ld + j] *= sc;
        if (cplx) X[q * ld + j + 1] *= sc;
      }
    }
    __syncthreads();
    for (int t = tid; t < n * n; t += NT) XT[t] = X[(t / n) * ld + (t % n)];
  } else if (n <= kWinMaxN) {
    // The same scheme for T in global memory, by groups of eigenvectors whose columns of X fit the
    // LDS buffer (a complex pair is kept in one group); each group runs over T's blocks from its
    // last column up.
    const double* TG = H;
    double* trow = srefl;  // rows s and i of the current block: [2][n]
    const int gmax = kHessLds / n - 2;
    const int ldx = gmax + 2;
    for (int g0 = 0; g0 < n;) {
    int g1 = min(n, g0 + gmax);
    if (g1 < n && lim[g1] < 0.0) ++g1;  // the second member of a pair joins its first
    double* X = sH;  // X(i, j) at X[i * ldx + j - g0]
    __syncthreads();  // the previous group's columns are written out
    for (int t = tid; t < n * ldx; t += NT) X[t] = 0.0;
    __syncthreads();
    // own blocks (the rest of each column stays zero below them)
    for (int j = g0 + tid; j < g1; j += NT) {
      const double wr = lre[j], wi = lim[j];
      if (wi < 0.0) continue;  // second member of a complex pair: written by j - 1
      const int b0 = (blk[j] == 0) ? j - 1 : j;
      const int bend = (blk[b0] == 2) ? b0 + 1 : b0;
      const bool cplx = wi > 0.0;
      const Cx lam{wr, wi};
      Cx xb0{0.0, 0.0}, xb1{0.0, 0.0};
      if (bend == b0) {
        xb0 = {1.0, 0.0};
      } else {
        const Cx a{TG[(int64_t)b0 * n + b0], 0.0}, bb{TG[(int64_t)b0 * n + b0 + 1], 0.0};
        const Cx c{TG[(int64_t)(b0 + 1) * n + b0], 0.0}, d{TG[(int64_t)(b0 + 1) * n + b0 + 1], 0.0};
        const Cx v0a = bb, v1a = csub(lam, a);  // (b, lambda - a)
        const Cx v0b = csub(lam, d), v1b = c;   // (lambda - d, c)
        if (cabs1(v0a) + cabs1(v1a) >= cabs1(v0b) + cabs1(v1b)) {
          xb0 = v0a;
          xb1 = v1a;
        } else {
          xb0 = v0b;
          xb1 = v1b;
        }
        if (cabs1(xb0) + cabs1(xb1) == 0.0) {
          if (j == b0) xb0 = {1.0, 0.0}; else xb1 = {1.0, 0.0};
        }
      }
      X[b0 * ldx + j - g0] = xb0.re;
      if (cplx) X[b0 * ldx + j + 1 - g0] = xb0.im;
      if (bend > b0) {
        X[bend * ldx + j - g0] = xb1.re;
        if (cplx) X[bend * ldx + j + 1 - g0] = xb1.im;
      }
    }
    // the next block's rows are loaded into registers while the current block is solved
    double ps[4], pi[4];
    auto fetch_rows = [&](int sbq, int iq) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = tid + q * NT;
        if (c < n) {
          ps[q] = TG[(int64_t)sbq * n + c];
          pi[q] = TG[(int64_t)iq * n + c];
        }
      }
    };
    fetch_rows((blk[g1 - 1] == 0) ? g1 - 2 : g1 - 1, g1 - 1);
    for (int i = g1 - 1; i >= 0;) {
      const int sb = (blk[i] == 0) ? i - 1 : i;  // block rows [sb, i]
      __syncthreads();  // previous block's rows are no longer read
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int c = tid + q * NT;
        if (c < n) {
          trow[c] = ps[q];
          trow[n + c] = pi[q];
        }
      }
      for (int c = tid + 4 * NT; c < n; c += NT) {  // only with fewer than n / 4 threads
        trow[c] = TG[(int64_t)sb * n + c];
        trow[n + c] = TG[(int64_t)i * n + c];
      }
      if (sb > 0) fetch_rows((blk[sb - 1] == 0) ? sb - 2 : sb - 1, sb - 1);
      __syncthreads();
      // eight lanes per eigenvector (a group has at most about 64 of them): each sums every eighth
      // term of the row products, combined by three lane exchanges, then lane 0 of the eight solves
      const int lpv = 8;
      for (int j0 = g0; j0 < g1; j0 += NT / lpv) {
        const int j = j0 + tid / lpv, part = tid % lpv;
        bool act = j < g1;
        double wr = 0.0, wi = 0.0;
        int b0 = 0, bend = 0;
        if (act) {
          wr = lre[j];
          wi = lim[j];
          b0 = (blk[j] == 0) ? j - 1 : j;
          bend = (blk[b0] == 2) ? b0 + 1 : b0;
          act = !(wi < 0.0) && i < b0;  // second member of a pair, or not above the own block
        }
        const bool cplx = wi > 0.0;
        const double* ts = trow;
        const double* ti = trow + n;
        double p0r = 0.0, p0i = 0.0, p1r = 0.0, p1i = 0.0;
        if (act) {
          if (cplx) {
            for (int c = i + 1 + part; c <= bend; c += lpv) {
              const double xr = X[c * ldx + j - g0], xi = X[c * ldx + j + 1 - g0];
              p0r -= ts[c] * xr;
              p0i -= ts[c] * xi;
              p1r -= ti[c] * xr;
              p1i -= ti[c] * xi;
            }
          } else {
            for (int c = i + 1 + part; c <= bend; c += lpv) {
              const double xc = X[c * ldx + j - g0];
              p0r -= ts[c] * xc;
              p1r -= ti[c] * xc;
            }
          }
        }
#pragma unroll
        for (int o = 1; o < 8; o <<= 1) {
          p0r += __shfl_xor(p0r, o);
          p0i += __shfl_xor(p0i, o);
          p1r += __shfl_xor(p1r, o);
          p1i += __shfl_xor(p1i, o);
        }
        if (!act || part != 0) continue;
        const double smin = fmax(kUlp * (fabs(wr) + fabs(wi)), kSafeMin);
        const Cx lam{wr, wi};
        const Cx r0{p0r, p0i}, r1{p1r, p1i};
        if (sb == i) {
          const Cx d0 = csub(Cx{ti[i], 0.0}, lam);
          const Cx xi = (cabs1(d0) <= same) ? Cx{0.0, 0.0} : cdiv(r0, cguard(d0, smin));
          X[i * ldx + j - g0] = xi.re;
          if (cplx) X[i * ldx + j + 1 - g0] = xi.im;
        } else if (cabs1(csub(Cx{lre[sb], lim[sb]}, lam)) <= same || cabs1(csub(Cx{lre[i], lim[i]}, lam)) <= same) {
          X[sb * ldx + j - g0] = 0.0;
          X[i * ldx + j - g0] = 0.0;
          if (cplx) {
            X[sb * ldx + j + 1 - g0] = 0.0;
            X[i * ldx + j + 1 - g0] = 0.0;
          }
        } else {
          Cx x0, x1;
          csolve2(csub(Cx{ts[sb], 0.0}, lam), Cx{ts[i], 0.0}, Cx{ti[sb], 0.0}, csub(Cx{ti[i], 0.0}, lam), r0, r1,
                  smin, x0, x1);
          X[sb * ldx + j - g0] = x0.re;
          X[i * ldx + j - g0] = x1.re;
          if (cplx) {
            X[sb * ldx + j + 1 - g0] = x0.im;
            X[i * ldx + j + 1 - g0] = x1.im;
          }
        }
      }
      i = sb - 1;
    }
    __syncthreads();
    // normalise (max modulus component -> 1) and write the group's columns out
    for (int j = g0 + tid; j < g1; j += NT) {
      const double wi = lim[j];
      if (wi < 0.0) continue;
      const bool cplx = wi > 0.0;
      double mx = 0.0;
      for (int q = 0; q < n; ++q) {
        double v = fabs(X[q * ldx + j - g0]);
        if (cplx) v += fabs(X[q * ldx + j + 1 - g0]);
        mx = fmax(mx, v);
      }
      const double sc = (mx > 0.0) ? 1.0 / mx : 1.0;
      for (int q = 0; q < n; ++q) {
        X[q * ldx + j - g0] *= sc;
        if (cplx) X[q * ldx + j + 1 - g0] *= sc;
      }
    }
    __syncthreads();
    const int gw = g1 - g0;
    for (int t = tid; t < n * gw; t += NT) {
      const int q = t / gw, jj = t - (t / gw) * gw;
      XT[(int64_t)q * n + g0 + jj] = X[q * ldx + jj];
    }
    g0 = g1;
    }
  } else {
#define TV(r, c) H[(int64_t)(r) * ld + (c)]
#define XV(r, c) XT[(int64_t)(r) * n + (c)]
  for (int j = tid; j < n; j += NT) {
    const double wr = lre[j], wi = lim[j];
    if (wi < 0.0) continue;  // second member of a complex pair: written by j - 1
    const int b0 = (blk[j] == 0) ? j - 1 : j;   // own block start
    const int bend = (blk[b0] == 2) ? b0 + 1 : b0;
    const double smin = fmax(kUlp * (fabs(wr) + fabs(wi)), kSafeMin);
    const bool cplx = wi > 0.0;
    const Cx lam{wr, wi};
    for (int i = bend + 1; i < n; ++i) {
      XV(i, j) = 0.0;
      if (cplx) XV(i, j + 1) = 0.0;
    }
    // own block
    Cx xb0{0.0, 0.0}, xb1{0.0, 0.0};
    if (bend == b0) {
      xb0 = {1.0, 0.0};
    } else {
      const Cx a{TV(b0, b0), 0.0}, bb{TV(b0, b0 + 1), 0.0}, c{TV(b0 + 1, b0), 0.0}, d{TV(b0 + 1, b0 + 1), 0.0};
      const Cx v0a = bb, v1a = csub(lam, a);   // (b, lambda - a)
      const Cx v0b = csub(lam, d), v1b = c;    // (lambda - d, c)
      if (cabs1(v0a) + cabs1(v1a) >= cabs1(v0b) + cabs1(v1b)) {
        xb0 = v0a;
        xb1 = v1a;
      } else {
        xb0 = v0b;
        xb1 = v1b;
      }
      if (cabs1(xb0) + cabs1(xb1) == 0.0) {
        if (j == b0) xb0 = {1.0, 0.0}; else xb1 = {1.0, 0.0};
      }
    }
    XV(b0, j) = xb0.re;
    if (cplx) XV(b0, j + 1) = xb0.im;
    if (bend > b0) {
      XV(bend, j) = xb1.re;
      if (cplx) XV(bend, j + 1) = xb1.im;
    }
    // blocks above, bottom to top
    int i = b0 - 1;
    while (i >= 0) {
      const int s = (blk[i] == 0) ? i - 1 : i;  // block [s, i]
      Cx r0{0.0, 0.0}, r1{0.0, 0.0};
      if (cplx) {
        for (int c = i + 1; c <= bend; ++c) {
          const double xr = XV(c, j), xi = XV(c, j + 1);
          const double t0 = TV(s, c);
          r0.re -= t0 * xr;
          r0.im -= t0 * xi;
          if (s < i) {
            const double t1 = TV(i, c);
            r1.re -= t1 * xr;
            r1.im -= t1 * xi;
          }
        }
      } else if (s == i) {
        double acc = 0.0;
#pragma unroll 8
        for (int c = i + 1; c <= bend; ++c) acc -= TV(s, c) * XV(c, j);
        r0.re = acc;
      } else {
        double a0 = 0.0, a1 = 0.0;
#pragma unroll 4
        for (int c = i + 1; c <= bend; ++c) {
          const double xc = XV(c, j);
          a0 -= TV(s, c) * xc;
          a1 -= TV(i, c) * xc;
        }
        r0.re = a0;
        r1.re = a1;
      }
      if (s == i) {
        const Cx d0 = csub(Cx{TV(i, i), 0.0}, lam);
        const Cx xi = (cabs1(d0) <= same) ? Cx{0.0, 0.0} : cdiv(r0, cguard(d0, smin));
        XV(i, j) = xi.re;
        if (cplx) XV(i, j + 1) = xi.im;
      } else if (cabs1(csub(Cx{lre[s], lim[s]}, lam)) <= same || cabs1(csub(Cx{lre[i], lim[i]}, lam)) <= same) {
        XV(s, j) = 0.0;
        XV(i, j) = 0.0;
        if (cplx) {
          XV(s, j + 1) = 0.0;
          XV(i, j + 1) = 0.0;
        }
      } else {
        Cx x0, x1;
        csolve2(csub(Cx{TV(s, s), 0.0}, lam), Cx{TV(s, i), 0.0}, Cx{TV(i, s), 0.0},
                csub(Cx{TV(i, i), 0.0}, lam), r0, r1, smin, x0, x1);
        XV(s, j) = x0.re;
        XV(i, j) = x1.re;
        if (cplx) {
          XV(s, j + 1) = x0.im;
          XV(i, j + 1) = x1.im;
        }
      }
      i = s - 1;
    }
    // normalise (max modulus component -> 1)
    double mx = 0.0;
    for (int q = 0; q <= bend; ++q) {
      double v = fabs(XV(q, j));
      if (cplx) v += fabs(XV(q, j + 1));
      mx = fmax(mx, v);
    }
    const double sc = (mx > 0.0) ? 1.0 / mx : 1.0;
    for (int q = 0; q <= bend; ++q) {
      XV(q, j) *= sc;
      if (cplx) XV(q, j + 1) *= sc;
    }
  }
#undef TV
#undef XV
  }
#undef HH
#undef ZZ
}

// One workgroup per problem of at most kLdsMaxn rows: workgroup b solves items[order[b]] (order
// null: items[b]); larger problems are left to k_eigen_big.
__global__ __launch_bounds__(kEigenThreads) void k_eigen(const Item* items, double* ws, int32_t* status,
                                                          int sweep_cap, const int32_t* order) {
  const Item it = items[order ? order[blockIdx.x] : blockIdx.x];
  if (status[it.layer] != 0 || it.n > kLdsMaxn) return;
  __shared__ double sH[kLdsMaxn * (kLdsMaxn + 1) + 3 * 64];
  __shared__ double srefl[2 * 3 * kMaxn];
  __shared__ double sred[16];
  __shared__ int sctl[8];
  __shared__ double sxyz[3];
  __shared__ ZOp zops[2];
  eigen_body<true>(it, ws + it.ws, status, sH, srefl, sred, sctl, sxyz, zops, sweep_cap);
}

// Problems larger than kLdsMaxn (H and Z in global memory, multi-bulge passes through an LDS
// window): workgroup b solves items[order[b]] (order null: items[b]). A kernel of its own so that
// its register allocation does not weigh on the LDS-resident path.
__global__ __launch_bounds__(kEigenThreads) void k_eigen_big(const Item* items, double* ws, int32_t* status,
                                                              int sweep_cap, const int32_t* order) {
  const Item it = items[order ? order[blockIdx.x] : blockIdx.x];
  if (status[it.layer] != 0 || it.n <= kLdsMaxn) return;
  __shared__ double sbuf[kWin * kWinLd + kWin * kWinU];
  __shared__ double srefl[2 * 3 * kMaxn];
  __shared__ double sred[16];
  __shared__ int sctl[8];
  __shared__ double sxyz[3];
  __shared__ ZOp zops[2];
  eigen_body<false>(it, ws + it.ws, status, sbuf, srefl, sred, sctl, sxyz, zops, sweep_cap);
}

// Persistent form: every workgroup takes the next position of `order` from the counter `queue`
// (reset to 0 before the launch) and solves that problem, until n_items are taken; every wave
// reaches the exit once the counter passes n_items.
__global__ __launch_bounds__(kEigenThreads) void k_eigen_persistent(const Item* items, double* ws, int32_t* status,
                                                                     int sweep_cap, const int32_t* order,
                                                                     int32_t* queue, int n_items) {
  __shared__ double sH[kLdsMaxn * (kLdsMaxn + 1) + 3 * 64];
  __shared__ double srefl[2 * 3 * kMaxn];
  __shared__ double sred[16];
  __shared__ int sctl[8];
  __shared__ double sxyz[3];
  __shared__ ZOp zops[2];
  __shared__ int snext;
  for (;;) {
    __syncthreads();  // the previous problem is done with the LDS
    if (threadIdx.x == 0) snext = atomicAdd(queue, 1);
    __syncthreads();
    const int pos = snext;
    if (pos >= n_items) return;
    const Item it = items[order[pos]];
    if (status[it.layer] != 0 || it.n > kLdsMaxn) continue;
    eigen_body<true>(it, ws + it.ws, status, sH, srefl, sred, sctl, sxyz, zops, sweep_cap);
  }
}

__global__ void k_reset_counter(int32_t* counter) { *counter = 0; }

// U = Q U' for the reflectors of the Hessenberg reduction, Q = H_0 H_1 ... H_{n-3} with
// H_k = I - tau_k v_k v_k^T on rows k+1..n-1 (v_k and tau_k left in the workspace by k_eigen):
// U' = Z X from the QR phase becomes the eigenvector matrix of G. One wave per kHqCols columns,
// the column blocks of one item on one XCD. The block stays in LDS (row stride kHqCols) while the
// reflectors are applied from the last to the first. Lane = kHqCols part + column: the 16 parts
// of a column split the dot product v^T u (rows i = part + 16 q, kPer of them per lane) and
// combine it by lane exchanges, so no workgroup barrier is needed; each lane's entries of a
// reflector are loaded a few steps before it is applied. 16 consecutive lanes touch 16
// consecutive doubles (no LDS bank conflict).
static_assert(64 % kHqCols == 0, "a wave holds whole columns");
template <int kPer>
__device__ __forceinline__ void hqapply_body(const Item& it, int tile, double* ws, double* sb, double* stau) {
  const int n = it.n;
  const int c0 = tile * kHqCols;
  if (c0 >= n) return;
  double* base = ws + it.ws;
  const double* __restrict__ QV = base + (int64_t)kBufYS * n * n;
  const double* __restrict__ Up = base + (int64_t)kBufG * n * n;
  double* __restrict__ U = base + (int64_t)kBufU * n * n;
  constexpr int kParts = 64 / kHqCols;
  const int lane = threadIdx.x, col = lane % kHqCols, part = lane / kHqCols;
  const int nc = min(kHqCols, n - c0);
  auto sync = [] {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  };
  for (int r = part; r < n; r += kParts) sb[r * kHqCols + col] = (col < nc) ? Up[(int64_t)r * n + c0 + col] : 0.0;
  // Reflector k (n - k - 1 entries) is loaded kDepth steps before it is applied: its data was
  // written by another workgroup, usually on another XCD, and a load takes about a step's time.
  // The loads are unconditional (index clamped to the row; entries past the reflector are never
  // used) so that the compiler can count them and wait only for the oldest; the taus are staged
  // in LDS once.
  constexpr int kDepth = kPer <= 16 ? 4 : 1;  // registers: (kDepth + 1) kPer doubles
  double va[kDepth][kPer];
  auto load = [&](int k, double* dst) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) dst[q] = QV[(int64_t)k * n + min(part + kParts * q, n - 1)];
  };
  for (int i = lane; i < n - 2; i += 64) stau[i] = QV[(int64_t)(n - 1) * n + i];
#pragma unroll
  for (int s = 0; s < kDepth; ++s) load(max(n - 3 - s, 0), va[s]);
  sync();
  for (int k0 = n - 3; k0 >= 0; k0 -= kDepth) {
#pragma unroll
    for (int s = 0; s < kDepth; ++s) {
      const int k = k0 - s;
      if (k < 0) break;
      double vc[kPer];
#pragma unroll
      for (int q = 0; q < kPer; ++q) vc[q] = va[s][q];
      load(max(k - kDepth, 0), va[s]);
      const double tau = stau[k];
      if (tau == 0.0) continue;  // uniform
      const int len = n - k - 1;
      double* u = sb + (k + 1) * kHqCols + col;
      double w = 0.0;
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const int i = part + kParts * q;
        if (i < len) w += vc[q] * u[i * kHqCols];
      }
      for (int o = kHqCols; o < 64; o <<= 1) w += __shfl_xor(w, o);
      w *= tau;
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const int i = part + kParts * q;
        if (i < len) u[i * kHqCols] -= vc[q] * w;
      }
      sync();  // the next reflector reads entries other lanes just wrote
    }
  }
  if (col < nc)
    for (int r = part; r < n; r += kParts) U[(int64_t)r * n + c0 + col] = sb[r * kHqCols + col];
}

// U = Q U' on the matrix cores, for systems of at most kHqMfmaMaxN rows (the larger ones keep
// k_hqapply: at n = 512 the large workload's per-order accuracy was established on its rounding). The reflectors are taken
// 16 at a time, Q_p = H_p ... H_{p+15} = I - V T V^T, and applied from the last panel to the first
// to a block of 16 columns of U' kept in LDS (row stride 17):
//   W = V^T U and G = V^T V  in one pass over the panel's rows (per 4-row step one V entry is the
//                            A operand of both products and the B operand of the second),
//   X = T W                  from T^-1 = diag(1 / tau) + the strictly upper part of G (the compact
//                            WY factor of an orthogonal product), by back substitution in the
//                            accumulator layout, row j handed to the other lanes by an exchange,
//   U -= V X                 (A = V from the workspace; the accumulator layout of X is the
//                            B-operand layout).
// A reflector with tau = 0 (a column already reduced) is the identity: its vector is taken as
// zero. Loads of V are unconditional (index clamped) and masked afterwards, so that the next
// chunk's loads stay in flight over the current chunk's MFMAs. One wave per 16 columns.
constexpr int kHqLd = 17;

__global__ __launch_bounds__(64) void k_hqapply_mfma(const Item* items, int n_items, int tiles, double* ws,
                                                      const int32_t* status) {
  int g, tile;
  xcd_split(blockIdx.x, tiles, g, tile);  // the column blocks of one item share an XCD
  if (g >= n_items) return;
  const Item it = items[g];
  if (status[it.layer] != 0 || it.n > kHqMfmaMaxN) return;
  const int n = it.n, c0 = tile * 16;
  if (c0 >= n) return;
  double* base = ws + it.ws;
  const double* __restrict__ QV = base + (int64_t)kBufYS * n * n;
  const double* __restrict__ tauv = QV + (int64_t)(n - 1) * n;
  const double* __restrict__ Up = base + (int64_t)kBufG * n * n;
  double* __restrict__ U = base + (int64_t)kBufU * n * n;
  __shared__ double sb[kHqMfmaMaxN * kHqLd];
  const int lane = threadIdx.x, lr = lane & 15, kq = lane >> 4;
  const int nc = min(16, n - c0);
  auto sync = [] {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  };
  for (int t = lane; t < n * 16; t += 64) {
    const int r = t >> 4, c = t & 15;
    sb[r * kHqLd + c] = c < nc ? Up[(int64_t)r * n + c0 + c] : 0.0;
  }
  sync();
  // V[row][j] (zero off the reflector's support or for tau_j = 0)
  auto vload = [&](int j, int row) { return QV[(int64_t)min(j, n - 2) * n + min(max(row - j - 1, 0), n - 1)]; };
  const int npan = (n - 2 + 15) / 16;
  for (int pi = npan - 1; pi >= 0; --pi) {
    const int p = 16 * pi, nbp = min(16, n - 2 - p);
    const int jw = p + lr;  // reflector of this lane in the W and G products
    const bool jok = lr < nbp && tauv[min(jw, n - 3)] != 0.0;
    double tr[4];  // tau of reflectors p + kq + 4 v (rows of X held by this lane)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = kq + 4 * v;
      tr[v] = j < nbp ? tauv[p + j] : 0.0;
    }
    double4_t accW = {0.0, 0.0, 0.0, 0.0}, accG = {0.0, 0.0, 0.0, 0.0};
    constexpr int kC = 8;
    double vc[kC], vn[kC];
#pragma unroll
    for (int u = 0; u < kC; ++u) vc[u] = vload(jw, p + 1 + 4 * u + kq);
    for (int k = p + 1; k < n; k += 4 * kC) {
#pragma unroll
      for (int u = 0; u < kC; ++u) vn[u] = vload(jw, k + 4 * kC + 4 * u + kq);
#pragma unroll
      for (int u = 0; u < kC; ++u) {
        const int row = k + 4 * u + kq;
        const bool ok = jok && row > jw && row < n;
        const double v = ok ? vc[u] : 0.0;
        const double x = row < n ? sb[min(row, n - 1) * kHqLd + lr] : 0.0;
        accW = __builtin_amdgcn_mfma_f64_16x16x4f64(v, x, accW, 0, 0, 0);
        accG = __builtin_amdgcn_mfma_f64_16x16x4f64(v, v, accG, 0, 0, 0);
      }
#pragma unroll
      for (int u = 0; u < kC; ++u) vc[u] = vn[u];
    }
    // X = T W: row j = kq + 4 v of W on this lane, column lr
#pragma unroll
    for (int j = 15; j >= 0; --j) {
      if ((j & 3) == kq) accW[j >> 2] *= tr[j >> 2];
      const double xj = __shfl(accW[j >> 2], ((j & 3) << 4) | lr);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double gij = __shfl(accG[v], (kq << 4) | j);
        if (kq + 4 * v < j) accW[v] -= gij * xj;
      }
    }
    // U -= V X on rows p+1..n-1, 16 at a time
    for (int r0 = p + 1; r0 < n; r0 += 16) {
      double4_t acc;
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[v] = sb[min(r0 + kq + 4 * v, n - 1) * kHqLd + lr];
      const int row = r0 + lr;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int j = p + 4 * t + kq;
        const double vr = vload(j, row);
        const double a = (tr[t] != 0.0 && row > j && row < n) ? -vr : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, accW[t], acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rr = r0 + kq + 4 * v;
        if (rr < n) sb[rr * kHqLd + lr] = acc[v];
      }
    }
    sync();
  }
  for (int t = lane; t < n * 16; t += 64) {
    const int r = t >> 4, c = t & 15;
    if (c < nc) U[(int64_t)r * n + c0 + c] = sb[r * kHqLd + c];
  }
}

__global__ __launch_bounds__(64) void k_hqapply(const Item* items, int n_items, int tiles, double* ws,
                                                 const int32_t* status) {
  int g, tile;
  xcd_split(blockIdx.x, tiles, g, tile);  // the column blocks of one item share an XCD
  if (g >= n_items) return;
  const Item it = items[g];
  if (status[it.layer] != 0 || it.n <= kHqMfmaMaxN) return;
  __shared__ double sb[kMaxn * kHqCols];  // rows x kHqCols columns
  __shared__ double stau[kMaxn];          // tau_k of every reflector
  if (it.n <= 128)
    hqapply_body<128 / (64 / kHqCols)>(it, tile, ws, sb, stau);
  else if (it.n <= 256)
    hqapply_body<256 / (64 / kHqCols)>(it, tile, ws, sb, stau);
  else
    hqapply_body<kMaxn / (64 / kHqCols)>(it, tile, ws, sb, stau);
}

}  // namespace vbrdf
