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
template <int kPer>
__device__ __forceinline__ bool lu_factor(double* A, int64_t ld, int n, int* perm, double* invd, int* redi) {
  const int tid = threadIdx.x, NT = blockDim.x, lane = tid & 63, wv = tid >> 6, nw = NT >> 6;
  const bool upd = nw == 1 || wv > 0;  // waves taking the rank-1 updates
  const int uw = nw == 1 ? 0 : wv - 1, unw = nw == 1 ? 1 : nw - 1;
  // Column j at positions j..n-1 (src), after the update of step j-1 for j > 0; the new order goes
  // to dst.
  auto panel = [&](int j, const int* src, int* dst) {
    double u = 0.0;
    if (j > 0) u = A[(int64_t)src[j - 1] * ld + j];  // Uu(j-1, j)
    double v[kPer];
    int ph[kPer];
    double best = -1.0, bval = 0.0;
    int bi = n;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int i = j + lane + 64 * q;
      if (i < n) {
        ph[q] = src[i];
        double x = A[(int64_t)ph[q] * ld + j];
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
      const double ob = __shfl_xor(best, o), ov = __shfl_xor(bval, o);
      const int oi = __shfl_xor(bi, o);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bval = ov;
        bi = oi;
      }
    }
    const bool ok = best > 0.0 && isfinite(best);
    if (ok) {
      const double inv = 1.0 / bval;
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
      double akc[kPer];
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const int c = k + 2 + lane + 64 * q;
        akc[q] = c < n ? A[(int64_t)pk * ld + c] : 0.0;
      }
      for (int i = k + 1 + uw; i < n; i += unw) {
        const int r = cur[i];
        const double l = A[(int64_t)r * ld + k];
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

constexpr int kLuLds = kLdsMaxn * (kLdsMaxn + 1);  // LDS matrix
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
// The source buffer is overwritten when n > kLdsMaxn (factored in place).
__global__ __launch_bounds__(1024) void k_lu(const Item* items, double* ws, int32_t* status, LuBufs b) {
  const Item it = items[blockIdx.x];
  if (status[it.layer] != 0) return;
  const int n = it.n, tid = threadIdx.x, NT = blockDim.x;
  const int which = blockIdx.y;
  double* base = ws + it.ws;
  double* Ag = base + (int64_t)b.src[which] * n * n;
  double* AT = base + (int64_t)b.dst[which] * n * n;
  double* ex = base + extras_off(n);
  __shared__ double smem[kLuLds];
  __shared__ int perm[2 * kMaxn];
  __shared__ double invd[kMaxn];
  __shared__ int redi[8];
  const bool in_lds = n <= kLdsMaxn;
  double* A = in_lds ? smem : Ag;
  const int64_t ld = in_lds ? n + 1 : n;
  bool ok;
  if (in_lds) {
    for (int t = tid; t < n * n; t += NT) smem[(t / n) * (n + 1) + (t % n)] = Ag[t];
    __syncthreads();
    ok = lu_factor<kLdsMaxn / 64>(smem, n + 1, n, perm, invd, redi);
  } else {
    ok = lu_factor<kMaxn / 64>(Ag, n, n, perm, invd, redi);
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
template <int ldb>
__device__ __forceinline__ void trsm_tile(const Item& it, int which, int r0, double* ws, const TrsmBufs& bf) {
  const int n = it.n, lane = threadIdx.x;
  constexpr int R = kTrsmRows;
  double* base = ws + it.ws;
  const double* __restrict__ AT = base + (int64_t)bf.a[which] * n * n;
  const double* __restrict__ U = base + (int64_t)bf.rhs[which] * n * n;
  double* __restrict__ Y = base + (int64_t)bf.y[which] * n * n;
  double* ex = base + extras_off(n);
  const double* __restrict__ id = lu_invd(ex, n, which);
  const int* __restrict__ pm = lu_perm(ex, n, which);
  // LDS: Bt [n][ldb], then two factor-column buffers [2][n]
  HIP_DYNAMIC_SHARED(double, smem)
  double* Bt = smem;
  double* cb = smem + (int64_t)n * ldb;
  const int nr = min(R, n - r0);
  for (int t = lane; t < nr * n; t += 64) {
    const int rr = t / n, c = t % n;
    Bt[c * ldb + rr] = U[(int64_t)(r0 + rr) * n + c];
  }
  double pre[kMaxn / 64];
  auto fetch = [&](int j) {
#pragma unroll
    for (int q = 0; q < kMaxn / 64; ++q) {
      const int c = lane + 64 * q;
      if (c < n) pre[q] = AT[(int64_t)j * n + c];
    }
  };
  auto stash = [&](double* dst) {
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
  double* b = Bt + row;
  const bool own = row < nr;
  // Z Uu = U, j ascending
  fetch(0);
  stash(cb);
  sync();
  for (int j = 0; j < n; ++j) {
    const double* col = cb + (j & 1) * n;
    if (j + 1 < n) fetch(j + 1);
    double a0 = 0.0, a1 = 0.0;
    int c = part;
    for (; c + kLpr < j; c += 2 * kLpr) {
      a0 -= b[c * ldb] * col[c];
      a1 -= b[(c + kLpr) * ldb] * col[c + kLpr];
    }
    if (c < j) a0 -= b[c * ldb] * col[c];
    double acc = a0 + a1;
    for (int o = 1; o < kLpr; o <<= 1) acc += __shfl_xor(acc, o);
    if (own && part == 0) b[j * ldb] = (b[j * ldb] + acc) * id[j];
    sync();  // the new entry and every read of the buffer the next stash overwrites are done
    if (j + 1 < n) stash(cb + ((j + 1) & 1) * n);
    sync();
  }
  // W L = Z, j descending (unit diagonal)
  fetch(n - 1);
  stash(cb + ((n - 1) & 1) * n);
  sync();
  for (int j = n - 1; j >= 0; --j) {
    const double* col = cb + (j & 1) * n;
    if (j > 0) fetch(j - 1);
    double a0 = 0.0, a1 = 0.0;
    int c = j + 1 + part;
    for (; c + kLpr < n; c += 2 * kLpr) {
      a0 -= b[c * ldb] * col[c];
      a1 -= b[(c + kLpr) * ldb] * col[c + kLpr];
    }
    if (c < n) a0 -= b[c * ldb] * col[c];
    double acc = a0 + a1;
    for (int o = 1; o < kLpr; o <<= 1) acc += __shfl_xor(acc, o);
    if (own && part == 0) b[j * ldb] += acc;
    sync();
    if (j > 0) stash(cb + ((j - 1) & 1) * n);
    sync();
  }
  for (int t = lane; t < nr * n; t += 64) {
    const int rr = t / n, c = t % n;
    Y[(int64_t)(r0 + rr) * n + pm[c]] = Bt[c * ldb + rr];
  }
}

__global__ __launch_bounds__(64) void k_trsm(const Item* items, int n_items, int tiles, double* ws, int32_t* status,
                                             TrsmBufs b) {
  int g, tile;
  xcd_split(blockIdx.x, tiles, g, tile);  // g = sides item + side; the tiles of one matrix share an XCD
  if (g >= b.sides * n_items) return;
  const Item it = items[g / b.sides];
  if (status[it.layer] != 0) return;
  const int r0 = tile * kTrsmRows;
  if (r0 >= it.n) return;
  const int side = g % b.sides;
  // the tile stride is a compile-time constant so that LDS offsets fold into the instructions
  if (trsm_ldb(it.n) == kTrsmLdb)
    trsm_tile<kTrsmLdb>(it, side, r0, ws, b);
  else
    trsm_tile<kTrsmRows + 1>(it, side, r0, ws, b);
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
                           const int32_t* status, int transmission) {
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
  const double alq = quad[ly.quad_off + it.N + b / 4];
  const double sgn = ((a & 3) >= 2) ? -1.0 : 1.0;
  const double r0 = 1.0 / (3.141592653589793 * alq);
  base[(int64_t)kBufE * n * n + idx] = sgn * y * r0;
  if (transmission) base[(int64_t)kBufF * n * n + idx] = (ys - yt) * r0;
}

}  // namespace vbrdf
