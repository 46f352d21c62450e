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
  const double* V = base + (int64_t)kBufG * n * n;
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

// LU factorisation with partial pivoting, P^T A = L Uu, in place and with the row exchanges kept
// logical: A keeps its original row order, perm[k] is the original row that holds position k of
// the factor, and so L(k', k) = A(perm[k'], k) for k' > k (unit diagonal), Uu(k, c) =
// A(perm[k], c) for c >= k, invd[k] = 1 / Uu_kk. A has row stride ld and lives in LDS or global
// memory (the caller passes a pointer derived from the __shared__ array so the accesses compile to
// LDS instructions). perm holds 2n ints (two position buffers); on return perm[0, n) is the final
// order. Returns false (uniformly) on a zero or non-finite pivot.
// Look-ahead by one column: while waves 1.. apply the rank-1 update of step k to columns k+2..,
// wave 0 updates column k+1 by step k, picks its pivot (largest modulus, ties to the smaller
// position) and scales it, lane-synchronous and in registers. One workgroup barrier per column.
// The block is a multiple of 64 threads and n <= 64 kPer.
template <int kPer, typename T = double>
__device__ __forceinline__ bool lu_factor(T* A, int64_t ld, int n, int* perm, T* invd, int* redi) {
  const int tid = threadIdx.x, NT = blockDim.x, lane = tid & 63, wv = tid >> 6, nw = NT >> 6;
  const bool upd = nw == 1 || wv > 0;  // waves taking the rank-1 updates
  const int uw = nw == 1 ? 0 : wv - 1, unw = nw == 1 ? 1 : nw - 1;
  // Column j at positions j..n-1 (src), after the update of step j-1 for j > 0; the new order goes
  // to dst.
  auto panel = [&](int j, const int* src, int* dst) {
    T u = 0;
    if (j > 0) u = A[(int64_t)src[j - 1] * ld + j];  // Uu(j-1, j)
    T v[kPer];
    int ph[kPer];
    T best = -1, bval = 0;
    int bi = n;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int i = j + lane + 64 * q;
      if (i < n) {
        ph[q] = src[i];
        T x = A[(int64_t)ph[q] * ld + j];
        if (j > 0) x -= A[(int64_t)ph[q] * ld + j - 1] * u;
        v[q] = x;
        if (fabs(x) > best) {  // positions ascend within a lane: ties keep the first
          best = fabs(x);
          bval = x;
          bi = i;
        }
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const T ob = __shfl_xor(best, o), ov = __shfl_xor(bval, o);
      const int oi = __shfl_xor(bi, o);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bval = ov;
        bi = oi;
      }
    }
    const bool ok = best > T(0) && isfinite(best);
    if (ok) {
      const T inv = T(1) / bval;
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const int i = j + lane + 64 * q;
        if (i < n) A[(int64_t)ph[q] * ld + j] = (i == bi) ? v[q] : v[q] * inv;
      }
      const int pj = src[j], pb = src[bi];
      for (int i = lane; i < n; i += 64) dst[i] = (i == j) ? pb : (i == bi ? pj : src[i]);
      if (lane == 0) invd[j] = inv;
    }
    if (lane == 0) redi[j & 1] = ok ? 1 : 0;
  };
  for (int i = tid; i < n; i += NT) perm[n + i] = i;
  __syncthreads();
  if (wv == 0) panel(0, perm + n, perm);
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (!redi[k & 1]) return false;
    if (k + 1 == n) break;
    const int* cur = perm + (k & 1) * n;
    if (wv == 0) panel(k + 1, cur, perm + ((k + 1) & 1) * n);
    if (upd) {
      // rank-1 update of step k on columns k+2..: lane l takes columns k+2+l, k+2+l+64, ..., and
      // the updating waves share the positions k+1.. (row multiplier read once per row)
      const int pk = cur[k];
      T akc[kPer];
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const int c = k + 2 + lane + 64 * q;
        akc[q] = c < n ? A[(int64_t)pk * ld + c] : T(0);
      }
      for (int i = k + 1 + uw; i < n; i += unw) {
        const int r = cur[i];
        const T l = A[(int64_t)r * ld + k];
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
          const int c = k + 2 + lane + 64 * q;
          if (c < n) A[(int64_t)r * ld + c] -= l * akc[q];
        }
      }
    }
    __syncthreads();
  }
  if ((n - 1) & 1) {  // the final order is in the second buffer
    for (int i = tid; i < n; i += NT) perm[i] = perm[n + i];
    __syncthreads();
  }
  return true;
}

typedef double double4_t __attribute__((ext_vector_type(4)));

// Blocked form of lu_factor for systems kept in global memory (same conventions: logical row
// exchanges through perm, L and Uu in place, invd = 1 / Uu_kk, pivot = largest modulus with ties
// to the smaller position). The rank-1 updates of the step-by-step form read and write the whole
// trailing matrix once per column; here a panel of kLuNb columns is factored in LDS, the panel's
// rows of Uu to its right follow from a unit-triangular solve (L11 U12 = A12), and the trailing
// matrix takes the panel's whole update A22 -= L21 U12 at once, on the matrix cores
// (v_mfma_f64_16x16x4, rows addressed through the pivot order). P: LDS of at least
// (n + 1) kLuNb doubles; sL: kLuNb (kLuNb + 1) doubles (L11 at a fixed stride with zeros on and
// above the diagonal, so that the forward substitution needs no predicate and addresses it by
// immediate offsets); rv, ri: 32 doubles and 16 ints of LDS. The block has at least as many
// threads as the matrix has rows (kLuThreadsBig).
constexpr int kLuNb = 32;
static_assert(kLuNb % 4 == 0 && kLuNb <= 64, "panel width: whole MFMA k-steps");

__device__ bool lu_blocked(double* __restrict__ A, int n, int* perm, double* invd, double* P, double* sL, double* rv,
                           int* ri) {
  const int tid = threadIdx.x, NT = blockDim.x, lane = tid & 63, wv = tid >> 6, nw = NT >> 6;
  for (int i = tid; i < n; i += NT) perm[i] = i;
  __syncthreads();
  for (int k0 = 0; k0 < n; k0 += kLuNb) {
    const int w = min(kLuNb, n - k0), m = n - k0;
    const int ldp = m | 1;  // odd stride: a row of the panel spreads over the LDS banks
    // panel P[q][i] = A(perm[k0 + i], k0 + q): 32 lanes along a row's panel columns
    for (int t = tid; t < m * kLuNb; t += NT) {
      const int i = t / kLuNb, q = t % kLuNb;
      if (q < w) P[q * ldp + i] = A[(int64_t)perm[k0 + i] * n + k0 + q];
    }
    __syncthreads();
    for (int q = 0; q < w; ++q) {
      // pivot: largest |P[q][i]| over i >= q, ties to the smaller position
      const int i = q + tid;
      double best = -1.0, bval = 0.0;
      int bi = m;
      if (i < m) {
        bval = P[q * ldp + i];
        best = fabs(bval);
        bi = i;
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o), ov = __shfl_xor(bval, o);
        const int oi = __shfl_xor(bi, o);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bval = ov;
          bi = oi;
        }
      }
      if (lane == 0) {
        rv[wv] = best;
        rv[16 + wv] = bval;
        ri[wv] = bi;
      }
      __syncthreads();
      best = rv[0];
      bval = rv[16];
      bi = ri[0];
      for (int v = 1; v < nw; ++v)
        if (rv[v] > best || (rv[v] == best && ri[v] < bi)) {
          best = rv[v];
          bval = rv[16 + v];
          bi = ri[v];
        }
      if (!(best > 0.0 && isfinite(best))) return false;  // uniform
      const double inv = 1.0 / bval;
      __syncthreads();  // every thread has read rv, ri
      if (bi != q) {
        if (tid < w) {
          const double x = P[tid * ldp + q];
          P[tid * ldp + q] = P[tid * ldp + bi];
          P[tid * ldp + bi] = x;
        }
        if (tid == 0) {
          const int x = perm[k0 + q];
          perm[k0 + q] = perm[k0 + bi];
          perm[k0 + bi] = x;
        }
      }
      if (tid == 0) invd[k0 + q] = inv;
      __syncthreads();
      // scale the column below the pivot and update the panel columns to its right (row per thread)
      if (i > q && i < m) {
        const double l = P[q * ldp + i] * inv;
        P[q * ldp + i] = l;
        for (int c = q + 1; c < w; ++c) P[c * ldp + i] -= l * P[c * ldp + q];
      }
      __syncthreads();
    }
    // panel back to global memory under the new order
    for (int t = tid; t < m * kLuNb; t += NT) {
      const int i = t / kLuNb, q = t % kLuNb;
      if (q < w) A[(int64_t)perm[k0 + i] * n + k0 + q] = P[q * ldp + i];
    }
    const int r0 = k0 + w;
    if (r0 >= n) break;  // from here on the panel is whole: w = kLuNb
    for (int t = tid; t < kLuNb * kLuNb; t += NT) {  // strictly lower part of L11, zeros elsewhere
      const int sc = t / kLuNb, r = t % kLuNb;
      sL[sc * (kLuNb + 1) + r] = r > sc ? P[sc * ldp + r] : 0.0;
    }
    __syncthreads();
    // A wave per block of 16 columns to the right of the panel: first U12 = L11^-1 A12 for those
    // columns by forward substitution, held in the B-operand layout of v_mfma_f64_16x16x4
    // (x[t] = row 4 t + lane / 16, column lane % 16; row s comes from its lane by an exchange),
    // then A22 -= L21 U12 in 16 x 16 tiles, A = -L21 from the LDS panel, the accumulator starting
    // from the tile of A22.
    {
      const int lr = lane & 15, kq = lane >> 4;
      const int nrest = n - r0;
      for (int cb = wv; cb * 16 < nrest; cb += nw) {
        const int col = r0 + cb * 16 + lr;
        const bool live = col < n;
        const int colc = live ? col : n - 1;
        double x[kLuNb / 4];
#pragma unroll
        for (int t = 0; t < kLuNb / 4; ++t) x[t] = A[(int64_t)perm[k0 + 4 * t + kq] * n + colc];
#pragma unroll
        for (int sr = 0; sr + 1 < kLuNb; ++sr) {
          const double xs = __shfl(x[sr >> 2], ((sr & 3) << 4) | lr);
#pragma unroll
          for (int t = sr >> 2; t < kLuNb / 4; ++t)
            x[t] -= sL[sr * (kLuNb + 1) + 4 * t + kq] * xs;
          __builtin_amdgcn_sched_barrier(0);  // keep each step's loads in their step (registers)
        }
        if (live)
#pragma unroll
          for (int t = 0; t < kLuNb / 4; ++t) A[(int64_t)perm[k0 + 4 * t + kq] * n + col] = x[t];
        for (int rb = 0; rb * 16 < nrest; ++rb) {
          double4_t acc;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int pos = r0 + rb * 16 + kq + 4 * v;
            acc[v] = (pos < n && live) ? A[(int64_t)perm[pos] * n + col] : 0.0;
          }
          const int pi = w + rb * 16 + lr;  // panel row of the A operand
#pragma unroll
          for (int t = 0; t < kLuNb / 4; ++t) {
            const double a = pi < m ? -P[(4 * t + kq) * ldp + pi] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, x[t], acc, 0, 0, 0);
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int pos = r0 + rb * 16 + kq + 4 * v;
            if (pos < n && live) A[(int64_t)perm[pos] * n + col] = acc[v];
          }
        }
      }
    }
    __syncthreads();
  }
  return true;
}

constexpr int kLuLds = kLdsMaxn * (kLdsMaxn + 1);  // LDS matrix
static_assert(kLuLds >= (kMaxn + 1) * kLuNb, "the panel of the blocked factorisation fits");
constexpr int kVfixLds = kLuLds + kLdsMaxn;          // LDS matrix and one work vector
static_assert(kVfixLds >= 2 * 256, "the column-maximum partials of a 256-thread block fit");

// Per-item scratch of the boundary solve, in the extras block: 1 / Uu_kk of S' and T'
// (2 x n doubles) and the two pivot orders (2 x n int32 in n doubles).
__device__ inline double* lu_invd(double* ex, int n, int which) { return ex + (4 + which) * (int64_t)n; }
__device__ inline int* lu_perm(double* ex, int n, int which) {
  return reinterpret_cast<int*>(ex + 2 * (int64_t)n) + which * n;
}

// LU factorisation with partial pivoting of buffer b.src[side] (side = blockIdx.y: S' and T' of the
// boundary solve, or U^T of the eigenpair refinement), P^T A = L Uu. The factor is written
// transposed into b.dst[side], AT[j n + c] = A(c, j), so that column j of Uu (c < j) and of L
// (c > j) are contiguous for the right division; pivots and 1 / Uu_kk go to the extras block.
// The source buffer is overwritten when n > kLdsMaxn (factored in place, in blocked form).
__global__ __launch_bounds__(kLuThreadsLds) void k_lu(const Item* items, double* ws, int32_t* status, LuBufs b) {
  const Item it = items[blockIdx.x];
  if (status[it.layer] != 0) return;
  if ((it.n > kLdsMaxn) != ((int)blockDim.x == kLuThreadsBig)) return;  // the other launch's systems
  const int n = it.n, tid = threadIdx.x, NT = blockDim.x;
  const int which = blockIdx.y;
  double* base = ws + it.ws;
  if (b.only_flagged && !boundary_flags(base + extras_off(n), n)->fallback[which]) return;
  double* Ag = buf_ptr(ws, it, b.src[which]);
  double* AT = buf_ptr(ws, it, b.dst[which]);
  double* ex = base + extras_off(n);
  __shared__ double smem[kLuLds];
  __shared__ int perm[2 * kMaxn];
  __shared__ double invd[kMaxn];
  __shared__ int redi[8];
  __shared__ double slu_rv[32];
  __shared__ double slu_l[kLuNb * (kLuNb + 1)];
  __shared__ int slu_ri[16];
  const bool in_lds = n <= kLdsMaxn;
  double* A = in_lds ? smem : Ag;
  const int64_t ld = in_lds ? n + 1 : n;
  bool ok;
  if (in_lds) {
    for (int t = tid; t < n * n; t += NT) smem[(t / n) * (n + 1) + (t % n)] = Ag[t];
    __syncthreads();
    ok = lu_factor<kLdsMaxn / 64>(smem, n + 1, n, perm, invd, redi);
  } else {
    ok = lu_blocked(Ag, n, perm, invd, smem, slu_l, slu_rv, slu_ri);
  }
  if (!ok) {
    if (tid == 0) status[it.layer] = -5;
    return;
  }
  for (int t = tid; t < n * n; t += NT) {
    const int j = t / n, c = t % n;
    AT[t] = A[(int64_t)perm[c] * ld + j];
  }
  double* id = lu_invd(ex, n, which);
  int* pm = lu_perm(ex, n, which);
  for (int i = tid; i < n; i += NT) {
    id[i] = invd[i];
    pm[i] = perm[i];
  }
}

void launch_lu(dim3 grid, hipStream_t s, const Item* items, double* ws, int32_t* status, int max_n, LuBufs b) {
  k_lu<<<grid, kLuThreadsLds, 0, s>>>(items, ws, status, b);
  if (max_n > kLdsMaxn) k_lu<<<grid, kLuThreadsBig, 0, s>>>(items, ws, status, b);
}

// Right division Y = B A^-1 with the factors of k_lu (S' and T' with B = U in the boundary solve,
// U^T with B = (G U)^T in the eigenpair refinement), for a tile of kTrsmRows rows of B (workgroups
// ordered so that the tiles of one matrix run on one XCD and share its L2). One wave:
// kLpr = 64 / kTrsmRows lanes share a row (lane = kLpr row + part), each taking every kLpr-th term
// of the row's dot products, combined by lane exchanges. The tile is kept in LDS as Bt[c][r] (row
// stride trsm_ldb(n)). No workgroup barrier. With W = Y P:
//   Z Uu = U :  Z_j = (U_j - sum_{c<j} Z_c Uu_cj) / Uu_jj      (j ascending)
//   W L = Z  :  W_j = Z_j - sum_{c>j} W_c L_cj                 (j descending, unit L)
// and Y[:, perm[j]] = W[:, j]. The factor column used at step j is the same for all rows: the
// wave stages it in LDS while the loads of the next column are in flight.
// TF: type of the factor and of the arithmetic (double, or float in the refined path); TB: type
// of the right-hand side rows (the FP64 U, or an FP32 residual); kAdd: accumulate into Y instead of
// overwriting it. The right-hand side of side `which` is read at rhs_off doubles from the item base.
// R: right-hand-side rows per tile (64 / R lanes per row).
template <int R, int ldb, typename TF, typename TB, bool kAdd>
__device__ __forceinline__ void trsm_tile(const Item& it, int which, int r0, double* ws, const TF* __restrict__ AT,
                                          const TB* __restrict__ U, double* __restrict__ Y) {
  const int n = it.n, lane = threadIdx.x;
  double* base = ws + it.ws;
  double* ex = base + extras_off(n);
  const double* __restrict__ id = lu_invd(ex, n, which);
  const int* __restrict__ pm = lu_perm(ex, n, which);
  // LDS: Bt [n][ldb], then two factor-column buffers [2][n]
  HIP_DYNAMIC_SHARED(double, smem_raw)
  TF* smem = reinterpret_cast<TF*>(smem_raw);
  TF* Bt = smem;
  TF* cb = smem + (int64_t)n * ldb;
  const int nr = min(R, n - r0);
  for (int t = lane; t < nr * n; t += 64) {
    const int rr = t / n, c = t % n;
    Bt[c * ldb + rr] = (TF)U[(int64_t)(r0 + rr) * n + c];
  }
  TF pre[kMaxn / 64];
  auto fetch = [&](int j) {
#pragma unroll
    for (int q = 0; q < kMaxn / 64; ++q) {
      const int c = lane + 64 * q;
      if (c < n) pre[q] = AT[(int64_t)j * n + c];
    }
  };
  auto stash = [&](TF* dst) {
#pragma unroll
    for (int q = 0; q < kMaxn / 64; ++q) {
      const int c = lane + 64 * q;
      if (c < n) dst[c] = pre[q];
    }
  };
  auto sync = [] {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  };
  constexpr int kLpr = 64 / R;  // lanes per right-hand-side row
  const int row = lane / kLpr, part = lane % kLpr;
  TF* b = Bt + row;
  const bool own = row < nr;
  // Z Uu = U, j ascending
  fetch(0);
  stash(cb);
  sync();
  for (int j = 0; j < n; ++j) {
    const TF* col = cb + (j & 1) * n;
    if (j + 1 < n) fetch(j + 1);
    TF a0 = 0, a1 = 0;
    int c = part;
    for (; c + kLpr < j; c += 2 * kLpr) {
      a0 -= b[c * ldb] * col[c];
      a1 -= b[(c + kLpr) * ldb] * col[c + kLpr];
    }
    if (c < j) a0 -= b[c * ldb] * col[c];
    TF acc = a0 + a1;
    for (int o = 1; o < kLpr; o <<= 1) acc += __shfl_xor(acc, o);
    if (own && part == 0) b[j * ldb] = (b[j * ldb] + acc) * (TF)id[j];
    sync();  // the new entry and every read of the buffer the next stash overwrites are done
    if (j + 1 < n) stash(cb + ((j + 1) & 1) * n);
    sync();
  }
  // W L = Z, j descending (unit diagonal)
  fetch(n - 1);
  stash(cb + ((n - 1) & 1) * n);
  sync();
  for (int j = n - 1; j >= 0; --j) {
    const TF* col = cb + (j & 1) * n;
    if (j > 0) fetch(j - 1);
    TF a0 = 0, a1 = 0;
    int c = j + 1 + part;
    for (; c + kLpr < n; c += 2 * kLpr) {
      a0 -= b[c * ldb] * col[c];
      a1 -= b[(c + kLpr) * ldb] * col[c + kLpr];
    }
    if (c < n) a0 -= b[c * ldb] * col[c];
    TF acc = a0 + a1;
    for (int o = 1; o < kLpr; o <<= 1) acc += __shfl_xor(acc, o);
    if (own && part == 0) b[j * ldb] += acc;
    sync();
    if (j > 0) stash(cb + ((j - 1) & 1) * n);
    sync();
  }
  for (int t = lane; t < nr * n; t += 64) {
    const int rr = t / n, c = t % n;
    if (kAdd)
      Y[(int64_t)(r0 + rr) * n + pm[c]] += (double)Bt[c * ldb + rr];
    else
      Y[(int64_t)(r0 + rr) * n + pm[c]] = (double)Bt[c * ldb + rr];
  }
}

// Right division Y = B A^-1 for a tile of 16 rows of B on the matrix cores (the kRows = 16 form of
// k_trsm; same factors, pivots and output convention as trsm_tile). One wave. The tile is kept in
// LDS column by column, Zt[c][r] (stride 17). Both triangular solves go by blocks of 16 columns:
//   Z Uu = B  (ascending):  Z_J = (B_J - Z_{<J} Uu_{<J,J}) Uu_JJ^-1,
//   W L = Z   (descending): W_J = Z_J - W_{>J} L_{>J,J}         (unit diagonal),
// the products with v_mfma_f64_16x16x4 (A = -Z or -W from LDS: row = lane % 16, k = lane / 16 +
// 4 t; B = the factor's columns, read from AT where they are contiguous; two accumulators so that
// consecutive MFMAs do not wait on each other), the 16 x 16 diagonal blocks by substitution in the
// accumulator layout (row lane / 16 + 4 v, column lane % 16), column c handed to the other lanes
// by an exchange.
constexpr int kTrsmLdz = 17;

// acc -= Zt[:, kb:ke] F[kb:ke, col] for the 16 rows of the tile (ke - kb a multiple of 4; fc a valid
// column of the factor also for padding lanes, whose results are discarded): chunks of 8 k-steps
// whose factor loads are issued one chunk ahead. Loads are unconditional (indices clamped) and the
// k-steps past ke get a zero A operand, so the code has no branches between a load and its use and
// the next chunk's loads stay in flight over the current chunk's MFMAs.
__device__ __forceinline__ void trsm_block_product(const double* Zt, const double* __restrict__ fc, int n, int kb,
                                                   int ke, int lr, int kq, double4_t& acc0, double4_t& acc1) {
  constexpr int kC = 8;
  double bc[kC], bn[kC];
#pragma unroll
  for (int u = 0; u < kC; ++u) bc[u] = fc[min(kb + 4 * u + kq, n - 1)];
  for (int k = kb; k < ke; k += 4 * kC) {
#pragma unroll
    for (int u = 0; u < kC; ++u) bn[u] = fc[min(k + 4 * kC + 4 * u + kq, n - 1)];
    double a[kC];
#pragma unroll
    for (int u = 0; u < kC; ++u) {
      const double z = Zt[min(k + 4 * u + kq, n - 1) * kTrsmLdz + lr];
      a[u] = (k + 4 * u < ke) ? -z : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kC; u += 2) {
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], bc[u], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u + 1], bc[u + 1], acc1, 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < kC; ++u) bc[u] = bn[u];
  }
}

__device__ __forceinline__ void trsm_tile_mfma(const Item& it, int which, int r0, double* ws,
                                               const double* __restrict__ AT, const double* __restrict__ U,
                                               double* __restrict__ Y) {
  const int n = it.n, lane = threadIdx.x;
  const int lr = lane & 15, kq = lane >> 4;
  double* base = ws + it.ws;
  double* ex = base + extras_off(n);
  const double* __restrict__ id = lu_invd(ex, n, which);
  const int* __restrict__ pm = lu_perm(ex, n, which);
  HIP_DYNAMIC_SHARED(double, Zt)
  const int nr = min(16, n - r0);
  // the tile's rows, 8 loads in flight per lane
  for (int t0 = 0; t0 < 16 * n; t0 += 8 * 64) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = min(t0 + 64 * u + lane, 16 * n - 1), rr = t / n;
      v[u] = U[(int64_t)min(r0 + rr, n - 1) * n + t % n];
      if (rr >= nr) v[u] = 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int t = t0 + 64 * u + lane;
      if (t < 16 * n) Zt[(t % n) * kTrsmLdz + t / n] = v[u];
    }
  }
  auto sync = [] {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  };
  sync();
  const int nblk = (n + 15) >> 4;
  // Z Uu = B
  for (int jb = 0; jb < nblk; ++jb) {
    const int j0 = jb * 16, col = j0 + lr, nv = min(16, n - j0);
    const bool cl = col < n;
    const double* __restrict__ fc = AT + (int64_t)(cl ? col : 0) * n;  // column col of the factor
    // the diagonal block's factor entries and this column's 1 / Uu_jj, loaded ahead of the product
    double fd[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) fd[c] = fc[min(j0 + c, n - 1)];
#pragma unroll
    for (int c = 0; c < 16; ++c) fd[c] = c < lr ? fd[c] : 0.0;  // Uu(j0 + c, col)
    const double dinv = id[min(col, n - 1)];
    double4_t acc0, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int v = 0; v < 4; ++v) acc0[v] = Zt[min(col, n - 1) * kTrsmLdz + kq + 4 * v];
    trsm_block_product(Zt, fc, n, 0, j0, lr, kq, acc0, acc1);
    acc0 += acc1;
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      if (c < nv) {  // uniform
        if (lr == c) acc0 *= dinv;
#pragma unroll
        for (int v = 0; v < 4; ++v) acc0[v] -= __shfl(acc0[v], (kq << 4) | c) * fd[c];
      }
    }
    if (cl)
#pragma unroll
      for (int v = 0; v < 4; ++v) Zt[col * kTrsmLdz + kq + 4 * v] = acc0[v];
    sync();
  }
  // W L = Z
  for (int jb = nblk - 1; jb >= 0; --jb) {
    const int j0 = jb * 16, col = j0 + lr, nv = min(16, n - j0);
    const bool cl = col < n;
    const double* __restrict__ fc = AT + (int64_t)(cl ? col : 0) * n;
    double fd[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) fd[c] = fc[min(j0 + c, n - 1)];
#pragma unroll
    for (int c = 0; c < 16; ++c) fd[c] = (c > lr && c < nv) ? fd[c] : 0.0;  // L(j0 + c, col)
    double4_t acc0, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int v = 0; v < 4; ++v) acc0[v] = Zt[min(col, n - 1) * kTrsmLdz + kq + 4 * v];
    trsm_block_product(Zt, fc, n, j0 + 16, n, lr, kq, acc0, acc1);
    acc0 += acc1;
#pragma unroll
    for (int c = 15; c > 0; --c) {
      if (c < nv)  // uniform
#pragma unroll
        for (int v = 0; v < 4; ++v) acc0[v] -= __shfl(acc0[v], (kq << 4) | c) * fd[c];
    }
    if (cl)
#pragma unroll
      for (int v = 0; v < 4; ++v) Zt[col * kTrsmLdz + kq + 4 * v] = acc0[v];
    sync();
  }
  // Y[:, perm[c]] = W[:, c]
  for (int c0 = 0; c0 < n; c0 += 64) {
    const int c = c0 + lane;
    if (c < n) {
      const int64_t pc = pm[c];
      for (int rr = 0; rr < nr; ++rr) Y[(int64_t)(r0 + rr) * n + pc] = Zt[c * kTrsmLdz + rr];
    }
  }
}

template <int kRows>
__global__ __launch_bounds__(64) void k_trsm(const Item* items, int n_items, int tiles, double* ws, int32_t* status,
                                             TrsmBufs b) {
  int g, tile;
  xcd_split(blockIdx.x, tiles, g, tile);  // g = sides item + side; the tiles of one matrix share an XCD
  if (g >= b.sides * n_items) return;
  const Item it = items[g / b.sides];
  if (status[it.layer] != 0) return;
  const int r0 = tile * kRows;
  if (r0 >= it.n) return;
  const int side = g % b.sides;
  const int n = it.n;
  double* base = ws + it.ws;
  if (b.only_flagged && !boundary_flags(base + extras_off(n), n)->fallback[side]) return;
  const double* AT = buf_ptr(ws, it, b.a[side]);
  const double* U = buf_ptr(ws, it, b.rhs[side]);
  double* Y = buf_ptr(ws, it, b.y[side]);
  // the tile shape and stride are compile-time constants so that LDS offsets fold into the
  // instructions
  if (kRows == 16)
    trsm_tile_mfma(it, side, r0, ws, AT, U, Y);
  else if (kRows != 8)
    trsm_tile<kRows, kRows + 1, double, double, false>(it, side, r0, ws, AT, U, Y);
  else if (trsm_ldb(n) == kTrsmLdb)
    trsm_tile<kTrsmRows, kTrsmLdb, double, double, false>(it, side, r0, ws, AT, U, Y);
  else
    trsm_tile<kTrsmRows, kTrsmRows + 1, double, double, false>(it, side, r0, ws, AT, U, Y);
}
template __global__ void k_trsm<4>(const Item*, int, int, double*, int32_t*, TrsmBufs);
template __global__ void k_trsm<8>(const Item*, int, int, double*, int32_t*, TrsmBufs);
template __global__ void k_trsm<16>(const Item*, int, int, double*, int32_t*, TrsmBufs);

void launch_trsm(int rows, dim3 grid, size_t lds, hipStream_t s, const Item* items, int n_items, int tiles, double* ws,
                 int32_t* status, TrsmBufs b) {
  if (rows == 4)
    k_trsm<4><<<grid, 64, lds, s>>>(items, n_items, tiles, ws, status, b);
  else if (rows == 16)
    k_trsm<16><<<grid, 64, lds, s>>>(items, n_items, tiles, ws, status, b);
  else
    k_trsm<8><<<grid, 64, lds, s>>>(items, n_items, tiles, ws, status, b);
}

const void* trsm_kernel_ptr(int rows) {
  if (rows == 4) return reinterpret_cast<const void*>(&k_trsm<4>);
  if (rows == 16) return reinterpret_cast<const void*>(&k_trsm<16>);
  return reinterpret_cast<const void*>(&k_trsm<8>);
}

// Columns of V = E~ U that lost more than ~7 digits to cancellation (the conservation mode of
// order 0 when omega is near 1: E~ u is then O(1 - omega) while its terms are O(||E~|| ||u||)) are
// recomputed from F~ E~ U = U Lambda as V = F~^-1 U Lambda, which has no such cancellation. For a
// complex pair the 2x2 real block of Lambda is applied.
constexpr double kVfixRatio = 1e-7;

template <bool kLds>
__device__ __forceinline__ void vfix_body(const Item& it, double* base, int32_t* status, double* smem, int* perm,
                                          double* invd, double* redv, int* redi, int* flag, double* enorm) {
  const int n = it.n;
  const int tid = threadIdx.x, NT = blockDim.x;
  const double* E = base + (int64_t)kBufE * n * n;
  double* Fg = base + (int64_t)kBufF * n * n;
  const double* U = base + (int64_t)kBufU * n * n;
  double* V = base + (int64_t)kBufG * n * n;
  const double* lre = base + extras_off(n);
  const double* lim = lre + n;
  // ||E~||_inf: 16 lanes per row (coalesced), rows spread over the block
  constexpr int kRowLanes = 16;
  double part = 0.0;
  for (int r0 = 0; r0 < n; r0 += NT / kRowLanes) {
    const int r = r0 + tid / kRowLanes;
    double s = 0.0;
    if (r < n)
      for (int c = tid % kRowLanes; c < n; c += kRowLanes) s += fabs(E[(int64_t)r * n + c]);
    for (int o = 1; o < kRowLanes; o <<= 1) s += __shfl_xor(s, o);
    part = fmax(part, s);
  }
  if (tid == 0) *enorm = 0.0;
  __syncthreads();
  for (int o = 32; o > 0; o >>= 1)
    if (o < (int)blockDim.x) part = fmax(part, __shfl_xor(part, o));
  if ((tid & 63) == 0) redv[tid >> 6] = part;
  __syncthreads();
  if (tid == 0) {
    double e = 0.0;
    for (int w = 0; w < (NT + 63) / 64; ++w) e = fmax(e, redv[w]);
    *enorm = e;
  }
  __syncthreads();
  const double en = *enorm;
  int any = 0;
  if (n <= NT) {
    // column maxima of |U| and |V|: NT / n threads per column split its rows, partials in smem
    const int pc = NT / n;
    double* pu = smem;
    double* pv = smem + pc * n;
    if (tid < pc * n) {
      const int j = tid % n, q = tid / n;
      double nu = 0.0, nv = 0.0;
      for (int r = q; r < n; r += pc) {
        nu = fmax(nu, fabs(U[(int64_t)r * n + j]));
        nv = fmax(nv, fabs(V[(int64_t)r * n + j]));
      }
      pu[q * n + j] = nu;
      pv[q * n + j] = nv;
    }
    __syncthreads();
    for (int j = tid; j < n; j += NT) {
      double nu = 0.0, nv = 0.0;
      for (int q = 0; q < pc; ++q) {
        nu = fmax(nu, pu[q * n + j]);
        nv = fmax(nv, pv[q * n + j]);
      }
      const int f = (nv < kVfixRatio * en * nu) ? 1 : 0;
      flag[j] = f;
      any |= f;
    }
  } else {
    for (int j = tid; j < n; j += NT) {
      double nu = 0.0, nv = 0.0;
      for (int r = 0; r < n; ++r) {
        nu = fmax(nu, fabs(U[(int64_t)r * n + j]));
        nv = fmax(nv, fabs(V[(int64_t)r * n + j]));
      }
      const int f = (nv < kVfixRatio * en * nu) ? 1 : 0;
      flag[j] = f;
      any |= f;
    }
  }
  __syncthreads();
  // pairs are flagged together
  for (int j = tid; j < n; j += NT) {
    if (lim[j] > 0.0 && j + 1 < n && (flag[j] | flag[j + 1])) any = 1;
  }
  for (int o = 32; o > 0; o >>= 1)
    if (o < (int)blockDim.x) any |= __shfl_xor(any, o);
  if ((tid & 63) == 0) redi[tid >> 6] = any;
  __syncthreads();
  int need = 0;
  for (int w = 0; w < (NT + 63) / 64; ++w) need |= redi[w];
  __syncthreads();
  if (!need) return;  // uniform
  for (int j = tid; j < n; j += NT) {
    if (lim[j] > 0.0 && j + 1 < n && (flag[j] | flag[j + 1])) {
      flag[j] = 1;
      flag[j + 1] = 1;
    }
  }
  __syncthreads();
  double* A = kLds ? smem : Fg;
  const int64_t ld = kLds ? n + 1 : n;
  if (kLds) {
    for (int t = tid; t < n * n; t += NT) A[(int64_t)(t / n) * ld + (t % n)] = Fg[t];
    __syncthreads();
  }
  if (!lu_factor<(kLds ? kLdsMaxn : kMaxn) / 64>(A, ld, n, perm, invd, redi)) {
    if (tid == 0) status[it.layer] = -5;
    return;
  }
  double* w = kLds ? smem + kLuLds : smem + 0;  // [n] work vector (global path: A is in Fg)
  double* w2 = w + kMaxn;
  for (int j = 0; j < n; ++j) {
    if (!flag[j]) continue;  // uniform: flag is shared
    if (lim[j] < 0.0) continue;  // second column of a pair: handled with the first
    const bool pair = lim[j] > 0.0;
    for (int col = 0; col < (pair ? 2 : 1); ++col) {
      double* x = col ? w2 : w;
      // x = P^T u
      for (int r = tid; r < n; r += NT) x[r] = U[(int64_t)perm[r] * n + j + col];
      __syncthreads();
      for (int k = 0; k + 1 < n; ++k) {  // L y = P^T u
        const double xk = x[k];
        for (int r = k + 1 + tid; r < n; r += NT) x[r] -= A[(int64_t)perm[r] * ld + k] * xk;
        __syncthreads();
      }
      for (int k = n - 1; k >= 0; --k) {  // Uu z = y
        if (tid == 0) x[k] *= invd[k];
        __syncthreads();
        const double xk = x[k];
        for (int r = tid; r < k; r += NT) x[r] -= A[(int64_t)perm[r] * ld + k] * xk;
        __syncthreads();
      }
    }
    const double a = lre[j], b = lim[j];
    for (int r = tid; r < n; r += NT) {
      if (pair) {
        V[(int64_t)r * n + j] = a * w[r] - b * w2[r];
        V[(int64_t)r * n + j + 1] = b * w[r] + a * w2[r];
      } else {
        V[(int64_t)r * n + j] = a * w[r];
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_vfix(const Item* items, double* ws, int32_t* status) {
  const Item it = items[blockIdx.x];
  if (status[it.layer] != 0) return;
  double* base = ws + it.ws;
  __shared__ double smem[kVfixLds];
  __shared__ int perm[2 * kMaxn];
  __shared__ double invd[kMaxn];
  __shared__ double redv[8];
  __shared__ int redi[8];
  __shared__ int flag[kMaxn];
  __shared__ double enorm;
  if (it.n <= kLdsMaxn)
    vfix_body<true>(it, base, status, smem, perm, invd, redv, redi, flag, &enorm);
  else
    vfix_body<false>(it, base, status, smem, perm, invd, redv, redi, flag, &enorm);
}

// R^m = Delta (Y_S + Y_T - I) R0, written over kBufE. With `transmission`, also the downward
// field at the base for the same inputs, T^m = (Y_S - Y_T) R0 (the attenuated incident stream
// included: in the stream form the total field is what the boundary solve returns), over kBufF.
__global__ void k_response(const Item* items, const Layer* layers, const double* quad, double* ws,
                           const int32_t* status, int mode) {
  const Item it = items[blockIdx.z];
  if (status[it.layer] != 0) return;
  const int n = it.n;
  const int a = blockIdx.y * 16 + threadIdx.y;
  const int b = blockIdx.x * 16 + threadIdx.x;
  if (a >= n || b >= n) return;
  const Layer ly = layers[it.layer];
  double* base = ws + it.ws;
  const int64_t idx = (int64_t)a * n + b;
  const double ys = base[(int64_t)kBufYS * n * n + idx], yt = base[(int64_t)kBufYT * n * n + idx];
  const double y = ys + yt - (a == b ? 1.0 : 0.0);
  if (mode & kResponseBrackets) {
    base[(int64_t)kBufE * n * n + idx] = y;
    base[(int64_t)kBufF * n * n + idx] = ys - yt;
    return;
  }
  const double alq = quad[ly.quad_off + it.N + b / 4];
  const double sgn = ((a & 3) >= 2) ? -1.0 : 1.0;
  const double r0 = 1.0 / (3.141592653589793 * alq);
  base[(int64_t)kBufE * n * n + idx] = sgn * y * r0;
  if (mode & kResponseTransmission) base[(int64_t)kBufF * n * n + idx] = (ys - yt) * r0;
}

// ---- FP32-refined boundary solve -------------------------------------------------------------
// S' and T' are factored in FP32 and every right division is done in FP32; the solutions are
// recovered to FP64 accuracy by iterative refinement: with the FP64 residual Res = U - Y A
// rounded to FP32, the FP32 correction Res A^-1 is added to Y (FP64). The boundary matrices are
// well conditioned (unit eigenvector columns), so each step gains about seven digits.

// FP32 LU of S' (side 0) and T' (side 1): the FP32 transposed factor goes to the first half of
// kBufG / kBufF (as floats), pivots and 1 / Uu_kk to the extras block; the FP64 matrices stay.
// Systems up to kLu32LdsMaxn are factored in LDS; larger ones in an FP32 copy in the second half
// of the same buffer.
__global__ __launch_bounds__(1024) void k_lu32(const Item* items, double* ws, int32_t* status) {
  const Item it = items[blockIdx.x];
  if (status[it.layer] != 0) return;
  const int n = it.n, tid = threadIdx.x, NT = blockDim.x;
  const int which = blockIdx.y;
  double* base = ws + it.ws;
  const double* Ag = base + (int64_t)(which == 0 ? kBufZ : kBufX) * n * n;
  float* AT = reinterpret_cast<float*>(base + (int64_t)(which == 0 ? kBufG : kBufF) * n * n);
  double* ex = base + extras_off(n);
  __shared__ float smem[kLu32LdsMaxn * (kLu32LdsMaxn + 1)];
  __shared__ int perm[2 * kMaxn];
  __shared__ float invd[kMaxn];
  __shared__ int redi[8];
  const bool in_lds = n <= kLu32LdsMaxn;
  float* A = in_lds ? smem : AT + (int64_t)n * n;  // working copy
  const int64_t ld = in_lds ? n + 1 : n;
  for (int t = tid; t < n * n; t += NT) A[(int64_t)(t / n) * ld + (t % n)] = (float)Ag[t];
  __syncthreads();
  bool ok;
  if (in_lds)
    ok = lu_factor<kLu32LdsMaxn / 64, float>(smem, n + 1, n, perm, invd, redi);
  else
    ok = lu_factor<kMaxn / 64, float>(A, n, n, perm, invd, redi);
  BoundaryFlags* bf = boundary_flags(ex, n);
  if (!ok) {  // an FP32 pivot vanished: leave this side to the FP64 solve
    if (tid == 0) bf->fallback[which] = 1;
    return;
  }
  for (int t = tid; t < n * n; t += NT) {
    const int j = t / n, c = t % n;
    AT[t] = A[(int64_t)perm[c] * ld + j];
  }
  double* id = lu_invd(ex, n, which);
  int* pm = lu_perm(ex, n, which);
  for (int i = tid; i < n; i += NT) {
    id[i] = invd[i];
    pm[i] = perm[i];
  }
  if (tid == 0) bf->fallback[which] = 0;
}

// FP32 right division for both sides: Y = U A^-1 (accumulate = 0) or Y += Res A^-1 with the FP32
// residual of k_resid (accumulate = 1). Sides whose FP32 factorisation failed are skipped. Tile 0
// of each side clears the side's residual maximum (and side 0 the maximum of U) for the k_resid
// that follows.
__global__ __launch_bounds__(64) void k_trsm32(const Item* items, int n_items, int tiles, double* ws,
                                               int32_t* status, int accumulate) {
  int g, tile;
  xcd_split(blockIdx.x, tiles, g, tile);
  if (g >= 2 * n_items) return;
  const Item it = items[g >> 1];
  if (status[it.layer] != 0) return;
  const int side = g & 1, n = it.n;
  double* base = ws + it.ws;
  BoundaryFlags* bf = boundary_flags(base + extras_off(n), n);
  if (tile == 0 && threadIdx.x == 0) {
    bf->resmax[side] = 0ull;
    if (side == 0) bf->umax = 0ull;
  }
  const int r0 = tile * kTrsmRows;
  if (r0 >= n || bf->fallback[side]) return;
  const float* AT = reinterpret_cast<const float*>(base + (int64_t)(side == 0 ? kBufG : kBufF) * n * n);
  double* Y = base + (int64_t)(side == 0 ? kBufYS : kBufYT) * n * n;
  if (accumulate) {
    const float* R = reinterpret_cast<const float*>(base + (int64_t)kBufE * n * n) + (int64_t)side * n * n;
    trsm_tile<kTrsmRows, kTrsmRows + 1, float, float, true>(it, side, r0, ws, AT, R, Y);
  } else {
    const double* U = base + (int64_t)kBufU * n * n;
    trsm_tile<kTrsmRows, kTrsmRows + 1, float, double, false>(it, side, r0, ws, AT, U, Y);
  }
}

typedef double double4_r __attribute__((ext_vector_type(4)));

// FP64 residual of both sides, Res = U - Y A (Y = U S'^-1 against A = S', Y = U T'^-1 against T'),
// on the matrix cores (64 x 64 tiles, v_mfma_f64_16x16x4 as in k_gemm), rounded to FP32 into
// kBufE (side s at float offset s n^2), with the running maxima of |Res| and |U|.
__global__ __launch_bounds__(256) void k_resid(const Item* items, double* ws, const int32_t* status) {
  const Item it = items[blockIdx.z >> 1];
  if (status[it.layer] != 0) return;
  const int side = blockIdx.z & 1;
  const int n = it.n;
  const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
  if (r0 >= n || c0 >= n) return;
  double* base = ws + it.ws;
  BoundaryFlags* bf = boundary_flags(base + extras_off(n), n);
  if (bf->fallback[side]) return;
  const double* Y = base + (int64_t)(side == 0 ? kBufYS : kBufYT) * n * n;
  const double* A = base + (int64_t)(side == 0 ? kBufZ : kBufX) * n * n;
  const double* U = base + (int64_t)kBufU * n * n;
  float* Res = reinterpret_cast<float*>(base + (int64_t)kBufE * n * n) + (int64_t)side * n * n;
  __shared__ double sA[64][17];
  __shared__ double sB[16][65];
  __shared__ double sred[8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  double4_r acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = (double4_r){0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < n; k0 += 16) {
    __syncthreads();
    for (int t = tid; t < 64 * 16; t += 256) {
      const int k = t % 16, r = t / 16;
      sA[r][k] = (r0 + r < n && k0 + k < n) ? Y[(int64_t)(r0 + r) * n + k0 + k] : 0.0;
    }
    for (int t = tid; t < 16 * 64; t += 256) {
      const int c = t % 64, k = t / 64;
      sB[k][c] = (k0 + k < n && c0 + c < n) ? A[(int64_t)(k0 + k) * n + c0 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      double a[2], b[2];
      for (int x = 0; x < 2; ++x) {
        a[x] = sA[wr + x * 16 + li][kk + lk];
        b[x] = sB[kk + lk][wc + x * 16 + li];
      }
      for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
    }
  }
  double rmax = 0.0, umax = 0.0;
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y)
      for (int v = 0; v < 4; ++v) {
        const int row = r0 + wr + x * 16 + lk + 4 * v;
        const int col = c0 + wc + y * 16 + li;
        if (row < n && col < n) {
          const int64_t idx = (int64_t)row * n + col;
          const double u = U[idx];
          const double r = u - acc[x][y][v];
          Res[idx] = (float)r;
          rmax = fmax(rmax, fabs(r));
          umax = fmax(umax, fabs(u));
        }
      }
  for (int o = 32; o > 0; o >>= 1) {
    rmax = fmax(rmax, __shfl_xor(rmax, o));
    umax = fmax(umax, __shfl_xor(umax, o));
  }
  if (lane == 0) {
    sred[wave] = rmax;
    sred[4 + wave] = umax;
  }
  __syncthreads();
  if (tid == 0) {
    const double rm = fmax(fmax(sred[0], sred[1]), fmax(sred[2], sred[3]));
    const double um = fmax(fmax(sred[4], sred[5]), fmax(sred[6], sred[7]));
    // non-negative doubles order like their bit patterns; NaN (all ones exponent) sorts high
    atomicMax(&bf->resmax[side], (unsigned long long)__double_as_longlong(isnan(rm) ? __builtin_inf() : rm));
    if (side == 0) atomicMax(&bf->umax, (unsigned long long)__double_as_longlong(um));
  }
}

// After the last refinement step: a side converged when max |Res| <= 1e-11 max |U| (the boundary
// matrices have condition numbers of order ten, so this bounds the solution's relative error near
// 1e-10). Otherwise the side is flagged for the FP64 solve, or the layer is reported NONCONVERGED.
__global__ void k_bcheck(const Item* items, double* ws, int32_t* status, int no_fallback) {
  const Item it = items[blockIdx.x];
  if (status[it.layer] != 0 || threadIdx.x > 1) return;
  const int side = threadIdx.x, n = it.n;
  BoundaryFlags* bf = boundary_flags(ws + it.ws + extras_off(n), n);
  if (bf->fallback[side]) {
    if (no_fallback) status[it.layer] = -6;
    return;
  }
  const double rm = __longlong_as_double((long long)bf->resmax[side]);
  const double um = __longlong_as_double((long long)bf->umax);
  if (!(rm <= 1e-11 * um)) {
    if (no_fallback)
      status[it.layer] = -6;
    else
      bf->fallback[side] = 1;
  }
}

}  // namespace vbrdf
