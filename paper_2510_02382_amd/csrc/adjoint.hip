// Reverse mode (adjoint) of the unrolled CTF-MNMF-ISS iterations followed by
// the source images, FP64.  Gradients follow the real-calculus convention
// g = dL/dRe + i dL/dIm for complex variables (L real), so that for w = u v,
// g_u += conj(v) g_w, and for s = |u|^2, g_u += 2 u g_s.
//
// Per iteration (state W, B, V -> W', B', V'), the forward is
//   lambda = B V, phi_(n,l)[t] = 1 / lambda[n, t - l];  ISS sweep on W and
//   Y = W xbar (Eqs. (11), (16));  P[n, s] = sum_l |y_(n,l)[s + l]|^2;
//   B^ = max(B sqrt(sum_s P v / lambda^2 / sum_s c v / lambda), floor)  (Eq. (17));
//   V^ = max(V sqrt(sum_f B^ P / lambda^2 / sum_f B^ c / lambda), floor) with
//   lambda = B^ V (all taps of a source, c[n, s] = #{l : s + l < T}; under
//   Eq. (18) as printed, the tap-0 rule, P0[n, s] = |y_(n,0)[s]|^2 and 1 in
//   place of P and c);
//   mu_r = sqrt(sum_{f,t} |y_r|^2 / (F T)), W' = W^s / mu, B' = B^ / mu_first^2,
//   V' = V^  (Eqs. (19)-(21)),
// and the images are c_n = H[:M, rows(n)] y_rows(n) with H = W^{-1} (Eq. (24)).
// The kernels below take these steps backwards, one launch per step and
// index space; the ISS sweep is reversed row by row, reconstructing the rows
// before each rank-one step from the ones after it (the step is invertible:
// 1 - z_r = d_r^{-1/2} > 0) with the coefficients recorded by a forward sweep
// in the same kernel.
#include <hip/hip_runtime.h>

#include <utility>

#include "common.hpp"
#include "launch.hpp"

namespace ctfiss {
namespace {


template <typename R>
__device__ __forceinline__ Cx<R> cconj(Cx<R> a) { return {a.x, -a.y}; }
__device__ __forceinline__ float sqrt_t(float v) { return sqrtf(v); }
__device__ __forceinline__ double sqrt_t(double v) { return sqrt(v); }
template <typename R>
__device__ __forceinline__ Cx<R> cscale(Cx<R> a, R s) { return {a.x * s, a.y * s}; }

template <typename R>
struct AdjArgs {
  // forward quantities of the iteration being reversed
  const Cx<R>* X;       // [M][F][T]
  const Cx<R>* Wk;      // [F][Mb][Mb] state at the start of the iteration
  const R* Bk;  // [N][F][K]
  const R* Vk;  // [N][K][T]
  const Cx<R>* Ws;      // [F][Mb][Mb] after the sweep, before the rescale
  const R* Bh;  // [N][F][K] after the basis update, before the rescale
  const R* Vh;  // [N][K][T] after the activation update
  const R* ilam;  // [N][F][T] 1 / (Bk Vk)
  const R* P;     // [N][F][T] tap-aligned powers of the swept rows
  const R* P0;    // [N][F][T] tap-0 powers (tap-0 activation rule) or null
  const R* mu;    // [Mb]
  // adjoints
  Cx<R>* gW;       // [F][Mb][Mb] in: of W', out: of Wk
  R* gB;   // [N][F][K]   in: of B', out: of Bk
  R* gV;   // [N][K][T]   in: of V', out: of Vk
  R* gBh;  // [N][F][K]
  R* gVh;  // [N][K][T]
  R* gP;   // [N][F][T]
  R* gP0;  // [N][F][T] of P0 (tap-0 activation rule) or null
  R* glam;   // [N][F][T] of lambda = Bk Vk
  R* glamh;  // [N][F][T] of lambda = B^ Vk
  R* lamh;   // [N][F][T] B^ Vk
  R* q1;     // [N][F][T] P / lamh^2 (P0 / lamh^2 under the tap-0 rule)
  R* q2;     // [N][F][T] c / lamh (1 / lamh under the tap-0 rule)
  R* G1;     // [N][K][T] adjoint of the activation update's numerator sum
  R* G2;     // [N][K][T] ... denominator sum
  R* H1;     // [N][F][K] adjoint of the basis update's numerator sum
  R* H2;     // [N][F][K] ... denominator sum
  R* part;   // [F][Mb + N] rescale partial sums
  R* gS;     // [Mb] adjoint of the row power sums
  Cx<R>* gX;         // [M][F][T] accumulated
  int* status;
  // per-bin scratch of the sweep
  Cx<R>* Y;        // [F][Mb][T]
  Cx<R>* gY;       // [F][Mb][T]
  R* gphi; // [F][Mb][T]
  Cx<R>* ztape;    // [F][Mb][Mb] z of row r's step, [f][r][p]
  R* dtape;  // [F][Mb][Mb] d_p of row r's step
  R floor;
  int F, T, M, D, N, K, Mb;
  int sweep_lds;  // 1: the sweep keeps gY and gphi in LDS
  RowMap rm;
};

template <typename R>
__device__ __forceinline__ R tapc(const RowMap& rm, int n, int s, int T) {
  const int c = T - s;
  return (R)(c < rm.L[n] ? c : rm.L[n]);
}

// xbar_c[t] = x[m][f][t - d] for c = d M + m (zero before frame 0)
template <typename R>
__device__ __forceinline__ Cx<R> xbar(const AdjArgs<R>& a, int f, int c, int t) {
  const int d = c / a.M, m = c - d * a.M;
  return t - d >= 0 ? a.X[((size_t)m * a.F + f) * a.T + t - d] : Cx<R>{R(0.0), R(0.0)};
}

// fn(integral_constant<int, R>) for R in the sequence, in order: every R is a
// compile-time constant in fn's body.
template <typename Fn, int... R>
__device__ __forceinline__ void static_for(Fn&& fn, std::integer_sequence<int, R...>) {
  (fn(std::integral_constant<int, R>{}), ...);
}

template <typename R>
__device__ __forceinline__ R wave_sum(R v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Wave sums of N values at once, transposed.  Level k pairs lanes that differ in lane
// bit 5 - k (across halves and rows of 16 with the gfx950 lane swaps, within a row with
// DPP mirrors and quad permutations, each an involution that flips that bit); the
// lane whose bit is 0 keeps the lower half of its values plus its partner's lower
// half, the other the upper halves, so the values per lane halve at every level (an
// odd count takes a zero into the upper half).  After six levels lane l holds the wave
// sum of value tsum_index<N>(l) (a padding zero where that index is N or more):
// ~3 operations per value pair and level instead of a six-level butterfly per value.
// The lane swaps of a (lower, upper) pair leave, in either half or row, that part's
// own value in one result and its partner's matching value in the other.
template <int W>
__device__ __forceinline__ float pair_swap_sum(float lo, float hi) {
  const auto r = W == 32 ? __builtin_amdgcn_permlane32_swap(__float_as_uint(lo), __float_as_uint(hi), false, false)
                         : __builtin_amdgcn_permlane16_swap(__float_as_uint(lo), __float_as_uint(hi), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
template <int W>
__device__ __forceinline__ double pair_swap_sum(double lo, double hi) {
  const unsigned l0 = (unsigned)__double2loint(lo), l1 = (unsigned)__double2hiint(lo);
  const unsigned h0 = (unsigned)__double2loint(hi), h1 = (unsigned)__double2hiint(hi);
  const auto a = W == 32 ? __builtin_amdgcn_permlane32_swap(l0, h0, false, false)
                         : __builtin_amdgcn_permlane16_swap(l0, h0, false, false);
  const auto b = W == 32 ? __builtin_amdgcn_permlane32_swap(l1, h1, false, false)
                         : __builtin_amdgcn_permlane16_swap(l1, h1, false, false);
  return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
}
template <int D>
constexpr int tsum_dpp() {  // within a row of 16: the involution that flips lane bit log2(D)
  return D == 8 ? 0x140 : D == 4 ? 0x141 : D == 2 ? 0x4E : 0xB1;  // row_mirror, row_half_mirror, xor 2, xor 1
}
template <typename R, int N, int LEVEL>
struct TSum {
  static __device__ __forceinline__ R run(const R (&v)[N], int lane) {
    constexpr int D = 32 >> LEVEL, H = (N + 1) / 2;
    const bool up = (lane & D) != 0;
    R w[H];
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const R lo = v[i], hi = H + i < N ? v[H + i] : R(0);
      if constexpr (D >= 16) {
        w[i] = pair_swap_sum<D == 32 ? 32 : 16>(lo, hi);
      } else {
        const R send = up ? lo : hi, keep = up ? hi : lo;
        w[i] = keep + dpp<tsum_dpp<D>()>(send);
      }
    }
    return TSum<R, H, LEVEL + 1>::run(w, lane);
  }
};
template <typename R, int N>
struct TSum<R, N, 6> {
  static __device__ __forceinline__ R run(const R (&v)[N], int) { return v[0]; }
};
// The value index lane `lane` ends with, or N where it holds only padding: the lane's
// window of real values shrinks to its lower or upper half at every level.
template <int N>
__device__ __forceinline__ int tsum_index(int lane) {
  int j = 0, n = N, real = N;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int h = (n + 1) / 2;
    if (lane & (32 >> k)) {
      j += h;
      real = real > h ? real - h : 0;
    } else {
      real = real < h ? real : h;
    }
    n = h;
  }
  return real > 0 ? j : N;
}
// dst[j] = the wave sum of v[j] for every j < N (written by the lane that holds it).
template <typename R, int N>
__device__ __forceinline__ void wave_sums(const R (&v)[N], R* dst) {
  static_assert(N >= 1 && N <= 64, "values per transposed wave sum");
  const int lane = threadIdx.x & 63;
  const R s = TSum<R, N, 0>::run(v, lane);
  const int j = tsum_index<N>(lane);
  if (j < N) dst[j] = s;
}

// ------------------------------------------------------------------ images
// gC [N][M][F][T]: H = W^{-1} (Gauss-Jordan, partial pivoting), then
// g_H = g_C Y^H, g_Y = H^H g_C (rows of each source), g_W = -H^H g_H H^H + g_Y xbar^H,
// g_xbar = W^H g_Y.  Writes gW and gX (the first contributions).
template <typename R>
__global__ void __launch_bounds__(256) k_adj_images(AdjArgs<R> a, const Cx<R>* __restrict__ W, const Cx<R>* __restrict__ gC) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int f = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  const int Mb = a.Mb, M = a.M, T = a.T, F = a.F;
  Cx<R>* Wl = reinterpret_cast<Cx<R>*>(smem);     // [Mb][Mb]
  Cx<R>* aug = Wl + Mb * Mb;                   // [Mb][2 Mb]
  Cx<R>* gH = aug + 2 * Mb * Mb;               // [M][Mb]
  Cx<R>* A = gH + M * Mb;                      // [M][Mb]  gH H^H
  Cx<R>* colk = A + M * Mb;                    // [Mb] pivot column
  int* piv = reinterpret_cast<int*>(colk + Mb);
  const Cx<R>* Wf = W + (size_t)f * Mb * Mb;
  for (int i = tid; i < Mb * Mb; i += nt) {
    Wl[i] = Wf[i];
    const int r = i / Mb, c = i - r * Mb;
    aug[r * 2 * Mb + c] = Wf[i];
    aug[r * 2 * Mb + Mb + c] = Cx<R>{r == c ? R(1.0) : R(0.0), R(0.0)};
  }
  __syncthreads();
  for (int k = 0; k < Mb; ++k) {
    if (tid == 0) {
      int best = k;
      R bv = cabs2(aug[k * 2 * Mb + k]);
      for (int i = k + 1; i < Mb; ++i) {
        const R v = cabs2(aug[i * 2 * Mb + k]);
        if (v > bv) { bv = v; best = i; }
      }
      piv[0] = best;
      if (!(bv > R(0.0))) latch(a.status, kFaultOutSingular);
    }
    __syncthreads();
    const int pr = piv[0];
    if (pr != k)
      for (int j = tid; j < 2 * Mb; j += nt) {
        const Cx<R> t0 = aug[k * 2 * Mb + j];
        aug[k * 2 * Mb + j] = aug[pr * 2 * Mb + j];
        aug[pr * 2 * Mb + j] = t0;
      }
    __syncthreads();
    const Cx<R> p = aug[k * 2 * Mb + k];
    const R den = cabs2(p);
    const Cx<R> pinv{p.x / den, -p.y / den};
    __syncthreads();
    for (int j = tid; j < 2 * Mb; j += nt) aug[k * 2 * Mb + j] = cmul(aug[k * 2 * Mb + j], pinv);
    for (int i = tid; i < Mb; i += nt) colk[i] = aug[i * 2 * Mb + k];
    __syncthreads();
    for (int e = tid; e < Mb * 2 * Mb; e += nt) {
      const int i = e / (2 * Mb), j = e - i * 2 * Mb;
      if (i != k) aug[e] = cfms(colk[i], aug[k * 2 * Mb + j], aug[e]);
    }
    __syncthreads();
  }
  // H[i][j] = aug[i][Mb + j]
  auto H = [&](int i, int j) { return aug[i * 2 * Mb + Mb + j]; };
  auto gc = [&](int r, int m, int t) { return gC[(((size_t)a.rm.src[r] * M + m) * F + f) * T + t]; };
  const int lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  // y_r[t] = sum_c W[r][c] xbar_c[t], once per bin, into the sweep scratch (unused at this stage),
  // and gY[r][t] = sum_m conj(H[m][r]) gC[n(r)][m][t]
  Cx<R>* Yb = a.Y + (size_t)f * Mb * T;
  Cx<R>* gY = a.gY + (size_t)f * Mb * T;
  for (int e = tid; e < Mb * T; e += nt) {
    const int r = e / T, t = e - r * T;
    Cx<R> s{R(0.0), R(0.0)};
    for (int c = 0; c < Mb; ++c) s = cfma(Wl[r * Mb + c], xbar(a, f, c, t), s);
    Yb[e] = s;
    Cx<R> g{R(0.0), R(0.0)};
    for (int m = 0; m < M; ++m) g = cfma(cconj(H(m, r)), gc(r, m, t), g);
    gY[e] = g;
  }
  __syncthreads();
  // gH[m][r] = sum_t gC[n(r)][m][t] conj(y_r[t]): one wave per entry, lanes over the frames
  for (int e = wave; e < M * Mb; e += nw) {
    const int m = e / Mb, r = e - m * Mb;
    R sx = R(0.0), sy = R(0.0);
    for (int t = lane; t < T; t += 64) {
      const Cx<R> q = cmulc(gc(r, m, t), Yb[r * T + t]);
      sx += q.x;
      sy += q.y;
    }
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    if (lane == 0) gH[e] = Cx<R>{sx, sy};
  }
  __syncthreads();
  // A = gH H^H: A[m][c] = sum_r gH[m][r] conj(H[c][r])
  for (int e = tid; e < M * Mb; e += nt) {
    const int m = e / Mb, c = e - m * Mb;
    Cx<R> s{R(0.0), R(0.0)};
    for (int r = 0; r < Mb; ++r) s = cfma(gH[m * Mb + r], cconj(H(c, r)), s);
    A[e] = s;
  }
  __syncthreads();
  // gW[r][c] = sum_t gY[r][t] conj(xbar_c[t]) - sum_m conj(H[m][r]) A[m][c]: one wave per entry
  for (int e = wave; e < Mb * Mb; e += nw) {
    const int r = e / Mb, c = e - r * Mb;
    R sx = R(0.0), sy = R(0.0);
    for (int t = lane; t < T; t += 64) {
      const Cx<R> q = cmulc(gY[r * T + t], xbar(a, f, c, t));
      sx += q.x;
      sy += q.y;
    }
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    if (lane == 0) {
      Cx<R> s{sx, sy};
      for (int m = 0; m < M; ++m) s = cfms(cconj(H(m, r)), A[m * Mb + c], s);
      a.gW[(size_t)f * Mb * Mb + e] = s;
    }
  }
  // gX[m][f][t] = sum_d sum_r conj(W[r][d M + m]) gY[r][t + d]
  for (int e = tid; e < M * T; e += nt) {
    const int m = e / T, t = e - m * T;
    Cx<R> s{R(0.0), R(0.0)};
    for (int d = 0; d < a.D && t + d < T; ++d)
      for (int r = 0; r < Mb; ++r) s = cfma(cconj(Wl[r * Mb + d * M + m]), gY[r * T + t + d], s);
    a.gX[((size_t)m * F + f) * T + t] = s;
  }
}

// ------------------------------------------------------------------ rescale
// part[f][r] = sum_c Re(conj(W'[r][c]) gW'[r][c]) with W' = W^s / mu_r;
// part[f][Mb + n] = sum_k gB'[n][f][k] B'[n][f][k] with B' = B^ / mu_first(n)^2.
template <typename R>
__global__ void __launch_bounds__(256) k_adj_rescale_part(AdjArgs<R> a) {
  const int f = blockIdx.x, tid = threadIdx.x;
  const int Mb = a.Mb;
  if (tid < Mb) {
    const int r = tid;
    R s = R(0.0);
    for (int c = 0; c < Mb; ++c) {
      const size_t o = ((size_t)f * Mb + r) * Mb + c;
      const Cx<R> w = a.Ws[o], g = a.gW[o];
      s += (w.x * g.x + w.y * g.y) / a.mu[r];
    }
    a.part[(size_t)f * (Mb + a.N) + r] = s;
  } else if (tid < Mb + a.N) {
    const int n = tid - Mb;
    const R m0 = a.mu[a.rm.r0[n]];
    R s = R(0.0);
    for (int k = 0; k < a.K; ++k) {
      const size_t o = ((size_t)n * a.F + f) * a.K + k;
      s += a.gB[o] * a.Bh[o] / (m0 * m0);
    }
    a.part[(size_t)f * (Mb + a.N) + tid] = s;
  }
}

// One wave per row r (lanes over f): g_mu_r = -sum_f part[f][r] / mu_r, minus
// 2 sum_f part[f][Mb + n] / mu_r for the first row of source n;
// gS_r = g_mu_r / (2 mu_r F T).
template <typename R>
__global__ void __launch_bounds__(64) k_adj_rescale_final(AdjArgs<R> a) {
  const int r = blockIdx.x, lane = threadIdx.x;
  const int W = a.Mb + a.N, n = a.rm.src[r];
  const bool first = a.rm.r0[n] == r;
  R s = R(0.0), sb = R(0.0);
  for (int f = lane; f < a.F; f += 64) {
    s += a.part[(size_t)f * W + r];
    if (first) sb += a.part[(size_t)f * W + a.Mb + n];
  }
  s = wave_sum(s);
  sb = wave_sum(sb);
  if (lane == 0) {
    const R g = -(s + R(2.0) * sb) / a.mu[r];
    a.gS[r] = g / (R(2.0) * a.mu[r] * (R)a.F * (R)a.T);
  }
}

// gW^s = gW' / mu_r (in place), gB^ = gB' / mu_first^2, gV^ = gV'.
template <typename R>
__global__ void __launch_bounds__(256) k_adj_rescale_apply(AdjArgs<R> a) {
  const size_t nW = (size_t)a.F * a.Mb * a.Mb, nB = (size_t)a.N * a.F * a.K, nV = (size_t)a.N * a.K * a.T;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nW) {
    const int r = (int)((i / a.Mb) % a.Mb);
    a.gW[i] = cscale(a.gW[i], R(1.0) / a.mu[r]);
  } else if (i < nW + nB) {
    const size_t j = i - nW;
    const int n = (int)(j / ((size_t)a.F * a.K));
    const R m0 = a.mu[a.rm.r0[n]];
    a.gBh[j] = a.gB[j] / (m0 * m0);
  } else if (i < nW + nB + nV) {
    const size_t j = i - nW - nB;
    a.gVh[j] = a.gV[j];
  }
}

// ------------------------------------------------------------------ activation update
// Per (n, f, s): lamh = B^ Vk, q1 = P / lamh^2, q2 = c / lamh (P0 and 1 under the tap-0 rule).
template <typename R>
__global__ void __launch_bounds__(256) k_adj_v0(AdjArgs<R> a) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)a.N * a.F * a.T) return;
  const int s = (int)(i % a.T), f = (int)((i / a.T) % a.F), n = (int)(i / ((size_t)a.F * a.T));
  const R* b = a.Bh + ((size_t)n * a.F + f) * a.K;
  R lam = R(0.0);
  for (int k = 0; k < a.K; ++k) lam += b[k] * a.Vk[((size_t)n * a.K + k) * a.T + s];
  a.lamh[i] = lam;
  a.q1[i] = (a.P0 ? a.P0[i] : a.P[i]) / (lam * lam);
  a.q2[i] = (a.P0 ? R(1.0) : tapc<R>(a.rm, n, s, a.T)) / lam;
}

// One wave per (n, k, s): num = sum_f B^ q1, den = sum_f B^ q2 (lanes over f);
// where V^ was not clamped: gV[n][k][s] = gV^ sqrt(num / den), G1 = gV^ V^ / (2 num),
// G2 = -gV^ V^ / (2 den); else all zero.
template <typename R>
__global__ void __launch_bounds__(256) k_adj_v1(AdjArgs<R> a) {
  const size_t i = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= (size_t)a.N * a.K * a.T) return;
  const int s = (int)(i % a.T), k = (int)((i / a.T) % a.K), n = (int)(i / ((size_t)a.K * a.T));
  R num = R(0.0), den = R(0.0);
  for (int f = lane; f < a.F; f += 64) {
    const R b = a.Bh[((size_t)n * a.F + f) * a.K + k];
    const size_t o = ((size_t)n * a.F + f) * a.T + s;
    num += b * a.q1[o];
    den += b * a.q2[o];
  }
  num = wave_sum(num);
  den = wave_sum(den);
  if (lane != 0) return;
  const R ratio = sqrt_t(num / den);
  const R val = a.Vk[i] * ratio;
  const R g = a.gVh[i];
  if (val >= a.floor) {
    a.gV[i] = g * ratio;
    a.G1[i] = g * val / (R(2.0) * num);
    a.G2[i] = -g * val / (R(2.0) * den);
  } else {
    a.gV[i] = R(0.0);
    a.G1[i] = R(0.0);
    a.G2[i] = R(0.0);
  }
}

// Per (n, f, s): lamh = B^ Vk; gP = sum_k G1 B^ / lamh^2 (first contribution);
// glamh = sum_k (-2 G1 B^ P / lamh^3 - G2 B^ c / lamh^2).  Under the tap-0 rule
// P0 and 1 stand for P and c, that sum is gP0, and gP starts at zero.
template <typename R>
__global__ void __launch_bounds__(256) k_adj_v2(AdjArgs<R> a) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)a.N * a.F * a.T) return;
  const int s = (int)(i % a.T), f = (int)((i / a.T) % a.F), n = (int)(i / ((size_t)a.F * a.T));
  const R* b = a.Bh + ((size_t)n * a.F + f) * a.K;
  const R lam = a.lamh[i];
  const R p = a.P0 ? a.P0[i] : a.P[i], c = a.P0 ? R(1.0) : tapc<R>(a.rm, n, s, a.T);
  R gp = R(0.0), gl = R(0.0);
  for (int k = 0; k < a.K; ++k) {
    const size_t o = ((size_t)n * a.K + k) * a.T + s;
    gp += a.G1[o] * b[k] / (lam * lam);
    gl += -R(2.0) * a.G1[o] * b[k] * p / (lam * lam * lam) - a.G2[o] * b[k] * c / (lam * lam);
  }
  if (a.P0) {
    a.gP0[i] = gp;
    a.gP[i] = R(0.0);
  } else {
    a.gP[i] = gp;
  }
  a.glamh[i] = gl;
}

// ------------------------------------------------------------------ basis update
// One wave per (n, f, k), lanes over s: first the rest of gB^ from the
// activation update, gB^ += sum_s (G1 q1 + G2 q2 + glamh Vk); then the basis
// update with lam = 1 / ilam: num = sum_s P Vk / lam^2, den = sum_s c Vk / lam;
// where B^ was not clamped: gB = gB^ sqrt(num / den), H1 = gB^ B^ / (2 num),
// H2 = -gB^ B^ / (2 den); else zero.
template <typename R>
__global__ void __launch_bounds__(256) k_adj_b1(AdjArgs<R> a) {
  const size_t i = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= (size_t)a.N * a.F * a.K) return;
  const int k = (int)(i % a.K), f = (int)((i / a.K) % a.F), n = (int)(i / ((size_t)a.F * a.K));
  const size_t fo = ((size_t)n * a.F + f) * a.T, ko = ((size_t)n * a.K + k) * a.T;
  R gbh = R(0.0), num = R(0.0), den = R(0.0);
  for (int s = lane; s < a.T; s += 64) {
    const R c = tapc<R>(a.rm, n, s, a.T), p = a.P[fo + s], v = a.Vk[ko + s];
    gbh += a.G1[ko + s] * a.q1[fo + s] + a.G2[ko + s] * a.q2[fo + s] + a.glamh[fo + s] * v;
    const R il = a.ilam[fo + s];
    num += p * v * il * il;
    den += c * v * il;
  }
  gbh = wave_sum(gbh) + a.gBh[i];
  num = wave_sum(num);
  den = wave_sum(den);
  if (lane != 0) return;
  const R ratio = sqrt_t(num / den);
  const R val = a.Bk[i] * ratio;
  if (val >= a.floor) {
    a.gB[i] = gbh * ratio;
    a.H1[i] = gbh * val / (R(2.0) * num);
    a.H2[i] = -gbh * val / (R(2.0) * den);
  } else {
    a.gB[i] = R(0.0);
    a.H1[i] = R(0.0);
    a.H2[i] = R(0.0);
  }
}

// Per (n, f, s): gP += sum_k H1 Vk / lam^2;  glam = sum_k (-2 H1 Vk P / lam^3 - H2 c Vk / lam^2).
template <typename R>
__global__ void __launch_bounds__(256) k_adj_b2(AdjArgs<R> a) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)a.N * a.F * a.T) return;
  const int s = (int)(i % a.T), f = (int)((i / a.T) % a.F), n = (int)(i / ((size_t)a.F * a.T));
  const R il = a.ilam[i], p = a.P[i], c = tapc<R>(a.rm, n, s, a.T);
  R gp = R(0.0), gl = R(0.0);
  for (int k = 0; k < a.K; ++k) {
    const R v = a.Vk[((size_t)n * a.K + k) * a.T + s];
    const size_t o = ((size_t)n * a.F + f) * a.K + k;
    gp += a.H1[o] * v * il * il;
    gl += -R(2.0) * a.H1[o] * v * p * il * il * il - a.H2[o] * c * v * il * il;
  }
  a.gP[i] += gp;
  a.glam[i] = gl;
}

// ------------------------------------------------------------------ ISS sweep
// One workgroup per bin.  Forward: Y = Wk xbar, the sweep with z and d_p
// recorded.  Backward from gW^s and gY^s = 2 y (tap-aligned gP) + 2 gS_r y_r
// (+ 2 y gP0 on the tap-0 rows under the tap-0 rule), rows r = Mb-1 .. 0.
// Then the demix (gW += gY xbar^H, gxbar = Wk^H gY) and
// glam += -sum_l gphi_(n,l)[s + l] / lam^2.
template <typename R>
__global__ void __launch_bounds__(256) k_adj_iss(AdjArgs<R> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int f = blockIdx.x, tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  const int Mb = a.Mb, T = a.T, F = a.F;
  const R invT = R(1.0) / T;
  Cx<R>* W = reinterpret_cast<Cx<R>*>(smem);   // [Mb][Mb]
  Cx<R>* gWl = W + Mb * Mb;                 // [Mb][Mb]
  Cx<R>* zl = gWl + Mb * Mb;                // [Mb]
  Cx<R>* ga = zl + Mb;                      // [Mb] adjoint of a_p
  Cx<R>* wr = ga + Mb;                      // [Mb] row r of W
  R* dl = reinterpret_cast<R*>(wr + Mb);  // [Mb]
  R* gd = dl + Mb;                  // [Mb] adjoint of d_p
  Cx<R>* yr = reinterpret_cast<Cx<R>*>(gd + Mb);  // [T]
  // the rows (read-mostly) stay in global memory; their adjoints and the
  // weight adjoints go to LDS when they fit (every step reads and writes them)
  Cx<R>* Y = a.Y + (size_t)f * Mb * T;
  Cx<R>* gY = a.sweep_lds ? yr + T : a.gY + (size_t)f * Mb * T;
  R* gphi = a.sweep_lds ? reinterpret_cast<R*>(gY + (size_t)Mb * T) : a.gphi + (size_t)f * Mb * T;
  Cx<R>* zt = a.ztape + (size_t)f * Mb * Mb;
  R* dt = a.dtape + (size_t)f * Mb * Mb;
  auto phi = [&](int p, int t) {
    const int l = a.rm.tap[p];
    return t >= l ? a.ilam[((size_t)a.rm.src[p] * F + f) * T + t - l] : R(0.0);
  };
  for (int i = tid; i < Mb * Mb; i += nt) W[i] = a.Wk[(size_t)f * Mb * Mb + i];
  __syncthreads();
  for (int e = tid; e < Mb * T; e += nt) {
    const int r = e / T, t = e - r * T;
    Cx<R> s{R(0.0), R(0.0)};
    for (int c = 0; c < Mb; ++c) s = cfma(W[r * Mb + c], xbar(a, f, c, t), s);
    Y[e] = s;
  }
  __syncthreads();
  // forward sweep, recording z and d
  for (int r = 0; r < Mb; ++r) {
    for (int t = tid; t < T; t += nt) yr[t] = Y[r * T + t];
    if (tid < Mb) wr[tid] = W[r * Mb + tid];
    __syncthreads();
    for (int p = wave; p < Mb; p += nw) {
      R d = R(0.0), ax = R(0.0), ay = R(0.0);
      for (int t = lane; t < T; t += 64) {
        const R ph = phi(p, t);
        const Cx<R> y = yr[t], yp = Y[p * T + t];
        d += ph * cabs2(y);
        const Cx<R> q = cmulc(yp, y);
        ax += ph * q.x;
        ay += ph * q.y;
      }
      d = wave_sum(d) * invT;
      ax = wave_sum(ax) * invT;
      ay = wave_sum(ay) * invT;
      if (lane == 0) {
        Cx<R> z{ax / d, ay / d};
        if (p == r) z = Cx<R>{R(1.0) - R(1.0) / sqrt_t(d), R(0.0)};
        zl[p] = z;
        dl[p] = d;
        zt[r * Mb + p] = z;
        dt[r * Mb + p] = d;
      }
    }
    __syncthreads();
    for (int e = tid; e < Mb * T; e += nt) {
      const int p = e / T, t = e - p * T;
      Y[e] = cfms(zl[p], yr[t], Y[e]);
    }
    for (int e = tid; e < Mb * Mb; e += nt) {
      const int p = e / Mb, c = e - p * Mb;
      W[e] = cfms(zl[p], wr[c], W[e]);
    }
    __syncthreads();
  }
  // adjoint seeds
  for (int i = tid; i < Mb * Mb; i += nt) gWl[i] = a.gW[(size_t)f * Mb * Mb + i];
  for (int e = tid; e < Mb * T; e += nt) {
    const int r = e / T, t = e - r * T;
    const int n = a.rm.src[r], l = a.rm.tap[r];
    R g = R(2.0) * a.gS[r];
    if (t >= l) g += R(2.0) * a.gP[((size_t)n * F + f) * T + t - l];
    if (a.gP0 && l == 0) g += R(2.0) * a.gP0[((size_t)n * F + f) * T + t];
    gY[e] = cscale(Y[e], g);
    gphi[e] = R(0.0);
  }
  __syncthreads();
  for (int r = Mb - 1; r >= 0; --r) {
    const Cx<R> zr = zt[r * Mb + r];
    const R sc = R(1.0) - zr.x;  // y_r' = sc y_r
    // rows before the step: y_r = y_r' / sc (the other rows after the reductions)
    for (int t = tid; t < T; t += nt) {
      const Cx<R> v = cscale(Y[r * T + t], R(1.0) / sc);
      Y[r * T + t] = v;
      yr[t] = v;
    }
    if (tid < Mb) {
      wr[tid] = cscale(W[r * Mb + tid], R(1.0) / sc);
      zl[tid] = zt[r * Mb + tid];
      dl[tid] = dt[r * Mb + tid];
    }
    __syncthreads();
    // g_z_p = -sum_c gW'[p][c] conj(w_r[c]) - sum_t gY'[p][t] conj(y_r[t])
    for (int p = wave; p < Mb; p += nw) {
      R gx = R(0.0), gy = R(0.0);
      for (int t = lane; t < T; t += 64) {
        const Cx<R> q = cmulc(gY[p * T + t], yr[t]);
        gx += q.x;
        gy += q.y;
      }
      for (int c = lane; c < Mb; c += 64) {
        const Cx<R> q = cmulc(gWl[p * Mb + c], wr[c]);
        gx += q.x;
        gy += q.y;
      }
      gx = -wave_sum(gx);
      gy = -wave_sum(gy);
      if (lane == 0) {
        const Cx<R> gz{gx, gy};
        const R d = dl[p];
        if (p == r) {
          ga[p] = Cx<R>{R(0.0), R(0.0)};
          gd[p] = R(0.5) * gz.x / (d * sqrt_t(d));  // d^{-3/2} / 2
        } else {
          const Cx<R> z = zl[p];
          ga[p] = cscale(gz, R(1.0) / d);
          gd[p] = -(z.x * gz.x + z.y * gz.y) / d;
        }
      }
    }
    __syncthreads();
    for (int t = tid; t < T; t += nt) {
      const Cx<R> y = yr[t];
      const R y2 = cabs2(y);
      Cx<R> gyr = cscale(gY[r * T + t], sc);
      for (int p = 0; p < Mb; ++p) {
        const R ph = phi(p, t) * invT;
        gyr = cfma(cscale(y, R(2.0) * ph), Cx<R>{gd[p], R(0.0)}, gyr);
        gphi[p * T + t] += y2 * gd[p] * invT;
        if (p == r) continue;
        const Cx<R> z = zl[p];
        const Cx<R> gp = gY[p * T + t];
        gyr = cfms(cconj(z), gp, gyr);
        const Cx<R> yp = cfma(z, y, Y[p * T + t]);  // row p before the step
        Y[p * T + t] = yp;
        gyr = cfma(cscale(yp, ph), cconj(ga[p]), gyr);
        gY[p * T + t] = cfma(cscale(y, ph), ga[p], gp);
        gphi[p * T + t] += cmul(cconj(yp), cmul(y, ga[p])).x * invT;
      }
      gY[r * T + t] = gyr;
    }
    if (tid < Mb) {
      const int c = tid;
      Cx<R> g = cscale(gWl[r * Mb + c], sc);
      for (int p = 0; p < Mb; ++p) {
        if (p == r) continue;
        g = cfms(cconj(zl[p]), gWl[p * Mb + c], g);
        W[p * Mb + c] = cfma(zl[p], wr[c], W[p * Mb + c]);
      }
      gWl[r * Mb + c] = g;
      W[r * Mb + c] = wr[c];
    }
    __syncthreads();
  }
  // demix: gW = gWl + gY xbar^H; gxbar = Wk^H gY
  const Cx<R>* Wk = a.Wk + (size_t)f * Mb * Mb;
  for (int e = tid; e < Mb * Mb; e += nt) {
    const int r = e / Mb, c = e - r * Mb;
    Cx<R> s = gWl[e];
    for (int t = 0; t < T; ++t) s = cfma(gY[r * T + t], cconj(xbar(a, f, c, t)), s);
    a.gW[(size_t)f * Mb * Mb + e] = s;
  }
  for (int e = tid; e < a.M * T; e += nt) {
    const int m = e / T, t = e - m * T;
    Cx<R> s{R(0.0), R(0.0)};
    for (int d = 0; d < a.D && t + d < T; ++d)
      for (int r = 0; r < Mb; ++r) s = cfma(cconj(Wk[r * Mb + d * a.M + m]), gY[r * T + t + d], s);
    const size_t o = ((size_t)m * F + f) * T + t;
    a.gX[o] = cadd(a.gX[o], s);
  }
  // phi_(n,l)[t] = 1 / lam[n][t - l]: glam[n][s] -= sum_l gphi_(n,l)[s + l] ilam[n][s]^2
  for (int e = tid; e < a.N * T; e += nt) {
    const int n = e / T, s = e - n * T;
    const size_t o = ((size_t)n * F + f) * T + s;
    const R il = a.ilam[o];
    R g = R(0.0);
    for (int l = 0; l < a.rm.L[n] && s + l < T; ++l) g += gphi[(a.rm.r0[n] + l) * T + s + l];
    a.glam[o] -= g * il * il;
  }
}

// Register-column form of k_adj_iss for Mbar <= MB <= 12 and T <= 512: thread t
// owns frame t and keeps that frame's column of the rows (y), of their
// adjoints (gy), of the weight adjoints (gph) and of the weights (ph) in
// registers, for every row; the row loops are unrolled over MB, so no register
// array is indexed at run time.  Only the frame sums of each step cross
// threads (wave sums, then LDS across waves).  The coefficients z and d_p of
// the forward sweep stay in LDS.  Same arithmetic as k_adj_iss.
template <typename R, int MB>
__global__ void __launch_bounds__(512) k_adj_iss_reg(AdjArgs<R> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int f = blockIdx.x, tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  const int Mb = a.Mb, T = a.T, F = a.F, t = tid;
  const bool own = t < T;
  const R invT = R(1.0) / T;
  Cx<R>* W = reinterpret_cast<Cx<R>*>(smem);  // [Mb][Mb]
  Cx<R>* gWl = W + MB * MB;                // [Mb][Mb]
  Cx<R>* zt = gWl + MB * MB;               // [MB][MB] z of step r, [r][p]
  Cx<R>* ga = zt + MB * MB;                // [MB]
  Cx<R>* wr = ga + MB;                     // [MB]
  R* dt = reinterpret_cast<R*>(wr + MB);  // [MB][MB]
  R* gd = dt + MB * MB;                        // [MB]
  R* red = gd + MB;                            // [nw][3 MB] partial frame sums
  for (int i = tid; i < Mb * Mb; i += nt) {
    const int r = i / Mb, c = i - r * Mb;
    W[r * MB + c] = a.Wk[(size_t)f * Mb * Mb + i];
  }
  __syncthreads();
  Cx<R> y[MB], gy[MB];
  R ph[MB], gph[MB];
#pragma unroll
  for (int p = 0; p < MB; ++p) {
    Cx<R> s{R(0.0), R(0.0)};
    R w = R(0.0);
    if (p < Mb && own) {
      for (int c = 0; c < Mb; ++c) s = cfma(W[p * MB + c], xbar(a, f, c, t), s);
      const int l = a.rm.tap[p];
      w = t >= l ? a.ilam[((size_t)a.rm.src[p] * F + f) * T + t - l] : R(0.0);
    }
    y[p] = s;
    ph[p] = w;
    gph[p] = R(0.0);
  }
  // the waves' frame sums go to their slots (wave_sums); block_finish adds the slots
  auto block_finish = [&](int nv) {
    __syncthreads();
    if (tid < nv) {
      R s = R(0.0);
      for (int w2 = 0; w2 < nw; ++w2) s += red[w2 * 3 * MB + tid];
      red[tid] = s;  // wave 0's slot: every wave has read its partial above
    }
    __syncthreads();
  };
  // forward sweep: record z and d_p
  auto fwd_step = [&](auto rc) {
    constexpr int r = decltype(rc)::value;
    if (r < Mb) {
    const Cx<R> yr = y[r];
    // the frame sums of rows p0 .. p0 + 3 (3 values each), transposed wave sums
    auto fwd_sums = [&](auto cc) {
      constexpr int p0 = 4 * decltype(cc)::value, NR = MB - p0 < 4 ? MB - p0 : 4;
      R v[3 * NR];
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        const int p = p0 + i;
        const Cx<R> q = cmulc(y[p], yr);
        const bool ok = p < Mb;
        v[3 * i] = ok ? ph[p] * cabs2(yr) : R(0.0);
        v[3 * i + 1] = ok ? ph[p] * q.x : R(0.0);
        v[3 * i + 2] = ok ? ph[p] * q.y : R(0.0);
      }
      wave_sums<R, 3 * NR>(v, red + wave * 3 * MB + 3 * p0);
    };
    static_for(fwd_sums, std::make_integer_sequence<int, (MB + 3) / 4>{});
    if (tid < Mb) wr[tid] = W[r * MB + tid];
    block_finish(3 * Mb);
    if (tid < Mb) {
      const int p = tid;
      const R d = red[3 * p] * invT;
      Cx<R> z{red[3 * p + 1] * invT / d, red[3 * p + 2] * invT / d};
      if (p == r) z = Cx<R>{R(1.0) - R(1.0) / sqrt_t(d), R(0.0)};
      zt[r * MB + p] = z;
      dt[r * MB + p] = d;
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < MB; ++p) y[p] = cfms(zt[r * MB + p], yr, y[p]);
    for (int e = tid; e < Mb * Mb; e += nt) {
      const int p = e / Mb, c = e - p * Mb;
      W[p * MB + c] = cfms(zt[r * MB + p], wr[c], W[p * MB + c]);
    }
    __syncthreads();
    }
  };
  static_for(fwd_step, std::make_integer_sequence<int, MB>{});
  // adjoint seeds
  for (int i = tid; i < Mb * Mb; i += nt) {
    const int r = i / Mb, c = i - r * Mb;
    gWl[r * MB + c] = a.gW[(size_t)f * Mb * Mb + i];
  }
#pragma unroll
  for (int p = 0; p < MB; ++p) {
    R g = R(0.0);
    if (p < Mb && own) {
      const int n = a.rm.src[p], l = a.rm.tap[p];
      g = R(2.0) * a.gS[p];
      if (t >= l) g += R(2.0) * a.gP[((size_t)n * F + f) * T + t - l];
      if (a.gP0 && l == 0) g += R(2.0) * a.gP0[((size_t)n * F + f) * T + t];
    }
    gy[p] = cscale(y[p], g);
  }
  __syncthreads();
  auto rev_step = [&](auto rc) {
    constexpr int r = MB - 1 - decltype(rc)::value;
    if (r < Mb) {
    const R sc = R(1.0) - zt[r * MB + r].x;
    y[r] = cscale(y[r], R(1.0) / sc);  // row r before the step
    const Cx<R> yr = y[r];
    if (tid < Mb) wr[tid] = cscale(W[r * MB + tid], R(1.0) / sc);
    // the frame sums of rows p0 .. p0 + 5 (2 values each), transposed wave sums
    auto rev_sums = [&](auto cc) {
      constexpr int p0 = 6 * decltype(cc)::value, NR = MB - p0 < 6 ? MB - p0 : 6;
      R v[2 * NR];
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        const int p = p0 + i;
        const Cx<R> q = cmulc(gy[p], yr);
        const bool ok = p < Mb;
        v[2 * i] = ok ? q.x : R(0.0);
        v[2 * i + 1] = ok ? q.y : R(0.0);
      }
      wave_sums<R, 2 * NR>(v, red + wave * 3 * MB + 2 * p0);
    };
    static_for(rev_sums, std::make_integer_sequence<int, (MB + 5) / 6>{});
    block_finish(2 * Mb);  // also completes wr
    if (tid < Mb) {
      const int p = tid;
      R gx = red[2 * p], gyv = red[2 * p + 1];
      for (int c = 0; c < Mb; ++c) {
        const Cx<R> q = cmulc(gWl[p * MB + c], wr[c]);
        gx += q.x;
        gyv += q.y;
      }
      const Cx<R> gz{-gx, -gyv};
      const R d = dt[r * MB + p];
      if (p == r) {
        ga[p] = Cx<R>{R(0.0), R(0.0)};
        gd[p] = R(0.5) * gz.x / (d * sqrt_t(d));  // d^{-3/2} / 2
      } else {
        const Cx<R> z = zt[r * MB + p];
        ga[p] = cscale(gz, R(1.0) / d);
        gd[p] = -(z.x * gz.x + z.y * gz.y) / d;
      }
    }
    __syncthreads();
    {
      const R y2 = cabs2(yr);
      Cx<R> gyr = cscale(gy[r], sc);
#pragma unroll
      for (int p = 0; p < MB; ++p) {
        if (p >= Mb) continue;
        const R phs = ph[p] * invT;
        gyr = cfma(cscale(yr, R(2.0) * phs), Cx<R>{gd[p], R(0.0)}, gyr);
        gph[p] += y2 * gd[p] * invT;
        if (p == r) continue;
        const Cx<R> z = zt[r * MB + p];
        gyr = cfms(cconj(z), gy[p], gyr);
        const Cx<R> yp = cfma(z, yr, y[p]);
        y[p] = yp;
        gyr = cfma(cscale(yp, phs), cconj(ga[p]), gyr);
        gy[p] = cfma(cscale(yr, phs), ga[p], gy[p]);
        gph[p] += cmul(cconj(yp), cmul(yr, ga[p])).x * invT;
      }
      gy[r] = gyr;
    }
    if (tid < Mb) {
      const int c = tid;
      Cx<R> g = cscale(gWl[r * MB + c], sc);
      for (int p = 0; p < Mb; ++p) {
        if (p == r) continue;
        g = cfms(cconj(zt[r * MB + p]), gWl[p * MB + c], g);
        W[p * MB + c] = cfma(zt[r * MB + p], wr[c], W[p * MB + c]);
      }
      gWl[r * MB + c] = g;
      W[r * MB + c] = wr[c];
    }
    __syncthreads();
    }
  };
  static_for(rev_step, std::make_integer_sequence<int, MB>{});
  // columns and the row adjoint of W to memory; the steps that mix frames
  // (demix and lambda adjoints) run as separate launches
  Cx<R>* gY = a.gY + (size_t)f * Mb * T;
  R* gphi = a.gphi + (size_t)f * Mb * T;
  if (own) {
#pragma unroll
    for (int p = 0; p < MB; ++p)
      if (p < Mb) {
        gY[p * T + t] = gy[p];
        gphi[p * T + t] = gph[p];
      }
  }
  for (int i = tid; i < Mb * Mb; i += nt) {
    const int r = i / Mb, c = i - r * Mb;
    a.gW[(size_t)f * Mb * Mb + i] = gWl[r * MB + c];
  }
}

// One wave per (f, r, c), lanes over frames: gW[f][r][c] += sum_t gY[r][t] conj(xbar_c[t]).
template <typename R>
__global__ void __launch_bounds__(256) k_adj_demix_w(AdjArgs<R> a) {
  const size_t i = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  const int Mb = a.Mb, T = a.T;
  if (i >= (size_t)a.F * Mb * Mb) return;
  const int c = (int)(i % Mb), r = (int)((i / Mb) % Mb), f = (int)(i / ((size_t)Mb * Mb));
  const Cx<R>* g = a.gY + ((size_t)f * Mb + r) * T;
  R sx = R(0.0), sy = R(0.0);
  for (int t = lane; t < T; t += 64) {
    const Cx<R> q = cmulc(g[t], xbar(a, f, c, t));
    sx += q.x;
    sy += q.y;
  }
  sx = group_sum<64>(sx);
  sy = group_sum<64>(sy);
  if (lane == 0) a.gW[i] = cadd(a.gW[i], Cx<R>{sx, sy});
}

// Per (m, f, t): gX[m][f][t] += sum_d sum_r conj(Wk[r][d M + m]) gY[r][t + d].
template <typename R>
__global__ void __launch_bounds__(256) k_adj_demix_x(AdjArgs<R> a) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int Mb = a.Mb, T = a.T, F = a.F;
  if (i >= (size_t)a.M * F * T) return;
  const int t = (int)(i % T), f = (int)((i / T) % F), m = (int)(i / ((size_t)F * T));
  const Cx<R>* Wk = a.Wk + (size_t)f * Mb * Mb;
  const Cx<R>* g = a.gY + (size_t)f * Mb * T;
  Cx<R> s{R(0.0), R(0.0)};
  for (int d = 0; d < a.D && t + d < T; ++d)
    for (int r = 0; r < Mb; ++r) s = cfma(cconj(Wk[r * Mb + d * a.M + m]), g[r * T + t + d], s);
  a.gX[i] = cadd(a.gX[i], s);
}

// Both demix adjoints of one bin per workgroup, from LDS: the bin's gY rows, its observation
// rows (xs[m][D - 1 + t] = x[m][f][t], zero before frame 0, so xbar_c[t] = xs[m][D - 1 + t - d]
// for c = d M + m) and Wk are loaded once; gW[r][c] += sum_t gY[r][t] conj(xbar_c[t]) with a
// wave per entry (lanes over frames, as k_adj_demix_w) and gX[m][f][t] += sum_d sum_r
// conj(Wk[r][d M + m]) gY[r][t + d] with a thread per output (as k_adj_demix_x): the same sums in
// the same order as those two kernels, which read every gY value 12 times (M D) from memory and
// take the shapes whose rows do not fit LDS.
template <typename R>
__global__ void __launch_bounds__(1024) k_adj_demix(AdjArgs<R> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int f = blockIdx.x, tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  const int Mb = a.Mb, T = a.T, F = a.F, M = a.M, D = a.D, LX = T + D - 1;
  Cx<R>* gy = reinterpret_cast<Cx<R>*>(smem);  // [Mb][T]
  Cx<R>* xs = gy + (size_t)Mb * T;              // [M][LX]
  Cx<R>* w = xs + (size_t)M * LX;               // [Mb][Mb]
  const Cx<R>* g = a.gY + (size_t)f * Mb * T;
  for (int e = tid; e < Mb * T; e += nt) gy[e] = g[e];
  for (int e = tid; e < M * LX; e += nt) {
    const int m = e / LX, t = e - m * LX - (D - 1);
    xs[e] = t >= 0 ? a.X[((size_t)m * F + f) * T + t] : Cx<R>{R(0.0), R(0.0)};
  }
  for (int e = tid; e < Mb * Mb; e += nt) w[e] = a.Wk[(size_t)f * Mb * Mb + e];
  __syncthreads();
  for (int e = wave; e < Mb * Mb; e += nw) {
    const int r = e / Mb, c = e - r * Mb, d = c / M, m = c - d * M;
    const Cx<R>* xr = xs + m * LX + (D - 1 - d);
    R sx = R(0.0), sy = R(0.0);
    for (int t = lane; t < T; t += 64) {
      const Cx<R> q = cmulc(gy[r * T + t], xr[t]);
      sx += q.x;
      sy += q.y;
    }
    sx = group_sum<64>(sx);
    sy = group_sum<64>(sy);
    if (lane == 0) {
      const size_t o = (size_t)f * Mb * Mb + e;
      a.gW[o] = cadd(a.gW[o], Cx<R>{sx, sy});
    }
  }
  for (int e = tid; e < M * T; e += nt) {
    const int m = e / T, t = e - m * T;
    Cx<R> acc{R(0.0), R(0.0)};
    for (int d = 0; d < D && t + d < T; ++d)
      for (int r = 0; r < Mb; ++r) acc = cfma(cconj(w[r * Mb + d * M + m]), gy[r * T + t + d], acc);
    const size_t o = ((size_t)m * F + f) * T + t;
    a.gX[o] = cadd(a.gX[o], acc);
  }
}

// Per (n, f, s): glam[n][f][s] -= sum_l gphi_(n,l)[s + l] / lam^2 (phi = 1 / lambda).
template <typename R>
__global__ void __launch_bounds__(256) k_adj_phi(AdjArgs<R> a) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int T = a.T, F = a.F;
  if (i >= (size_t)a.N * F * T) return;
  const int sv = (int)(i % T), f = (int)((i / T) % F), n = (int)(i / ((size_t)F * T));
  const R* gp = a.gphi + (size_t)f * a.Mb * T;
  const R il = a.ilam[i];
  R g = R(0.0);
  for (int l = 0; l < a.rm.L[n] && sv + l < T; ++l) g += gp[(a.rm.r0[n] + l) * T + sv + l];
  a.glam[i] -= g * il * il;
}

// Row bound of the register-column instance for Mbar (0: none; beyond 12 rows
// the columns no longer fit 256 VGPRs).
int adj_reg_rows(int Mb) { return Mb <= 4 ? 4 : Mb <= 8 ? 8 : Mb <= 12 ? 12 : 0; }
size_t adj_reg_lds(int MB, int nthr, int rs) {
  return (size_t)(3 * MB * MB + 2 * MB) * 2 * rs + (size_t)(MB * MB + MB) * rs + (size_t)(nthr / 64) * 3 * MB * rs;
}

// ------------------------------------------------------------------ lambda
// One wave per (n, f, k), lanes over s: gB += sum_s glam Vk.
template <typename R>
__global__ void __launch_bounds__(256) k_adj_l1(AdjArgs<R> a) {
  const size_t i = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (i >= (size_t)a.N * a.F * a.K) return;
  const int k = (int)(i % a.K), f = (int)((i / a.K) % a.F), n = (int)(i / ((size_t)a.F * a.K));
  const R* g = a.glam + ((size_t)n * a.F + f) * a.T;
  const R* v = a.Vk + ((size_t)n * a.K + k) * a.T;
  R s = R(0.0);
  for (int t = lane; t < a.T; t += 64) s += g[t] * v[t];
  s = wave_sum(s);
  if (lane == 0) a.gB[i] += s;
}

// gV[n][k][s] += sum_f (B^ glamh + H1 P / lam^2 + H2 c / lam + Bk glam).  One workgroup
// of 16 waves per (source n, 64 frames, 8 bases, chunk of bins): lane l takes frame 64 x + l
// (the (n, f, s) arrays are read along s, contiguously, once for all 8 bases), wave w the
// chunk's bins f = f0 + w, f0 + w + 16, ... (the (n, f, k) factors are the same for the whole
// wave); the waves' partial sums are added in wave order through LDS.  With one chunk the sum
// goes to gV; with several, each chunk's sum goes to chunk_sums[chunk][n][k][s] and
// k_adj_l2_sum adds them to gV in chunk order (the chunks spread the bins of a few (source,
// frames, bases) tiles over many workgroups).
constexpr int kL2Waves = 16, kL2Bases = 8;
template <typename R>
__global__ void __launch_bounds__(64 * kL2Waves) k_adj_l2(AdjArgs<R> a, R* chunk_sums, int fchunk) {
  __shared__ R part[kL2Waves][kL2Bases][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ntile = (a.T + 63) / 64, nkc = (a.K + kL2Bases - 1) / kL2Bases;
  const int tile = blockIdx.x % ntile, kc = (blockIdx.x / ntile) % nkc, n = blockIdx.x / (ntile * nkc);
  const int ch = blockIdx.y, f0 = ch * fchunk, f1 = min(a.F, f0 + fchunk);
  const int s = tile * 64 + lane, k0 = kc * kL2Bases;
  const bool ok = s < a.T;
  const R c = ok ? tapc<R>(a.rm, n, s, a.T) : R(0.0);
  R acc[kL2Bases];
#pragma unroll
  for (int kk = 0; kk < kL2Bases; ++kk) acc[kk] = R(0.0);
  if (ok) {
    for (int f = f0 + wave; f < f1; f += kL2Waves) {
      const size_t fs = ((size_t)n * a.F + f) * a.T + s, fk = ((size_t)n * a.F + f) * a.K + k0;
      const R il = a.ilam[fs], e1 = a.glamh[fs], e2 = a.P[fs] * il * il, e3 = c * il, e4 = a.glam[fs];
#pragma unroll
      for (int kk = 0; kk < kL2Bases; ++kk) {
        if (k0 + kk < a.K)
          acc[kk] += a.Bh[fk + kk] * e1 + a.H1[fk + kk] * e2 + a.H2[fk + kk] * e3 + a.Bk[fk + kk] * e4;
      }
    }
  }
#pragma unroll
  for (int kk = 0; kk < kL2Bases; ++kk) part[wave][kk][lane] = acc[kk];
  __syncthreads();
  if (wave < kL2Bases && ok && k0 + wave < a.K) {  // wave kk adds basis kk's partials
    R sum = R(0.0);
    for (int w = 0; w < kL2Waves; ++w) sum += part[w][wave][lane];
    const size_t o = ((size_t)n * a.K + k0 + wave) * a.T + s;
    if (chunk_sums)
      chunk_sums[(size_t)ch * a.N * a.K * a.T + o] = sum;
    else
      a.gV[o] += sum;
  }
}

// gV[n][k][s] += the chunk sums of k_adj_l2 in chunk order.
template <typename R>
__global__ void __launch_bounds__(256) k_adj_l2_sum(AdjArgs<R> a, const R* chunk_sums, int nch) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x, n = (size_t)a.N * a.K * a.T;
  if (i >= n) return;
  R sum = R(0.0);
  for (int c = 0; c < nch; ++c) sum += chunk_sums[(size_t)c * n + i];
  a.gV[i] += sum;
}

}  // namespace

// Chunks of bins of the activation adjoint's sums: 64 bins or more each, at most kAdjL2Chunks.
int adj_l2_chunks(int F) {
  const int c = (F + 63) / 64;
  return c < 1 ? 1 : (c > kAdjL2Chunks ? kAdjL2Chunks : c);
}

// LDS of the per-bin adjoint kernels for real size rs (complex 2 rs).
size_t adj_images_lds(int Mb, int M, int rs) { return (size_t)(3 * Mb * Mb + 2 * M * Mb + Mb) * 2 * rs + 64; }
size_t adj_iss_lds_base(int Mb, int T, int rs) {
  return (size_t)(2 * Mb * Mb + 3 * Mb) * 2 * rs + 2 * Mb * rs + (size_t)T * 2 * rs;
}
// gY and gphi in LDS only while three workgroups still fit a CU: a launch has
// one workgroup per bin, and with fewer per CU the bins of a typical F (513)
// need several rounds, which costs more than the global-memory traffic saved.
bool adj_sweep_in_lds(int Mb, int T, int rs) {
  return adj_iss_lds_base(Mb, T, rs) + (size_t)Mb * T * 3 * rs <= kMaxLdsBytes / 3;
}
size_t adj_iss_lds(int Mb, int T, int rs) {
  return adj_iss_lds_base(Mb, T, rs) + (adj_sweep_in_lds(Mb, T, rs) ? (size_t)Mb * T * 3 * rs : 0);
}

namespace {
template <typename R>
AdjArgs<R> make_adj(const AdjPtrs& p, const Dims& d, double floor) {
  AdjArgs<R> a{};
  a.X = static_cast<const Cx<R>*>(p.X);
  a.Wk = static_cast<const Cx<R>*>(p.Wk);
  a.Bk = static_cast<const R*>(p.Bk);
  a.Vk = static_cast<const R*>(p.Vk);
  a.Ws = static_cast<const Cx<R>*>(p.Ws);
  a.Bh = static_cast<const R*>(p.Bh);
  a.Vh = static_cast<const R*>(p.Vh);
  a.ilam = static_cast<const R*>(p.ilam);
  a.P = static_cast<const R*>(p.P);
  a.P0 = static_cast<const R*>(p.P0);
  a.mu = static_cast<const R*>(p.mu);
  a.gW = static_cast<Cx<R>*>(p.gW);
  a.gB = static_cast<R*>(p.gB);
  a.gV = static_cast<R*>(p.gV);
  a.gBh = static_cast<R*>(p.gBh);
  a.gVh = static_cast<R*>(p.gVh);
  a.gP = static_cast<R*>(p.gP);
  a.gP0 = static_cast<R*>(p.gP0);
  a.glam = static_cast<R*>(p.glam);
  a.glamh = static_cast<R*>(p.glamh);
  a.lamh = static_cast<R*>(p.lamh);
  a.q1 = static_cast<R*>(p.q1);
  a.q2 = static_cast<R*>(p.q2);
  a.G1 = static_cast<R*>(p.G1);
  a.G2 = static_cast<R*>(p.G2);
  a.H1 = static_cast<R*>(p.H1);
  a.H2 = static_cast<R*>(p.H2);
  a.part = static_cast<R*>(p.part);
  a.gS = static_cast<R*>(p.gS);
  a.gX = static_cast<Cx<R>*>(p.gX);
  a.status = p.status;
  a.Y = static_cast<Cx<R>*>(p.Y);
  a.gY = static_cast<Cx<R>*>(p.gY);
  a.gphi = static_cast<R*>(p.gphi);
  a.ztape = static_cast<Cx<R>*>(p.ztape);
  a.dtape = static_cast<R*>(p.dtape);
  a.floor = (R)floor;
  a.F = d.F;
  a.T = d.T;
  a.M = d.M;
  a.D = d.D;
  a.N = d.N;
  a.K = d.K;
  a.Mb = d.Mb;
  a.sweep_lds = adj_sweep_in_lds(d.Mb, d.T, (int)sizeof(R)) ? 1 : 0;
  a.rm = d.rm;
  return a;
}

template <typename R>
hipError_t adj_images_t(const AdjPtrs& p, const Dims& d, const void* W, const void* gC, hipStream_t s) {
  const AdjArgs<R> a = make_adj<R>(p, d, 0.0);
  const size_t lds = adj_images_lds(d.Mb, d.M, (int)sizeof(R));
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k_adj_images<R>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_adj_images<R>, dim3(d.F), dim3(256), lds, s, a, static_cast<const Cx<R>*>(W),
                     static_cast<const Cx<R>*>(gC));
  return hipGetLastError();
}

template <typename R>
hipError_t adj_iteration_t(const AdjPtrs& p, const Dims& d, double floor, hipStream_t s) {
  const AdjArgs<R> a = make_adj<R>(p, d, floor);
  const int rs = (int)sizeof(R);
  auto blocks = [](size_t n) { return dim3((unsigned)((n + 255) / 256)); };
  const size_t nkt = (size_t)d.N * d.K * d.T, nft = (size_t)d.N * d.F * d.T, nfk = (size_t)d.N * d.F * d.K;
  const size_t napply = (size_t)d.F * d.Mb * d.Mb + nfk + nkt;
  hipLaunchKernelGGL(k_adj_rescale_part<R>, dim3(d.F), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_adj_rescale_final<R>, dim3(d.Mb), dim3(64), 0, s, a);
  hipLaunchKernelGGL(k_adj_rescale_apply<R>, blocks(napply), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_adj_v0<R>, blocks(nft), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_adj_v1<R>, blocks(nkt * 64), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_adj_v2<R>, blocks(nft), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_adj_b1<R>, blocks(nfk * 64), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_adj_b2<R>, blocks(nft), dim3(256), 0, s, a);
  const int MB = adj_reg_rows(d.Mb);
  if (MB > 0 && d.T <= 512) {  // register columns: one thread per frame
    const int nthr = (d.T + 63) / 64 * 64;
    const size_t lds = adj_reg_lds(MB, nthr, rs);
    if (MB == 4) hipLaunchKernelGGL((k_adj_iss_reg<R, 4>), dim3(d.F), dim3(nthr), lds, s, a);
    if (MB == 8) hipLaunchKernelGGL((k_adj_iss_reg<R, 8>), dim3(d.F), dim3(nthr), lds, s, a);
    if (MB == 12) hipLaunchKernelGGL((k_adj_iss_reg<R, 12>), dim3(d.F), dim3(nthr), lds, s, a);
    const size_t dlds = ((size_t)d.Mb * d.T + (size_t)d.M * (d.T + d.D - 1) + (size_t)d.Mb * d.Mb) * 2 * rs;
    if (dlds <= kMaxLdsBytes) {
      if (dlds > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)k_adj_demix<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)dlds);
        if (e != hipSuccess) return e;
      }
      // 8 waves per bin (three such workgroups share a CU at the differentiation workload's
      // FP32 size), 16 in FP64 (one workgroup per CU there)
      hipLaunchKernelGGL(k_adj_demix<R>, dim3(d.F), dim3(rs == 8 ? 1024 : 512), dlds, s, a);
    } else {
      hipLaunchKernelGGL(k_adj_demix_w<R>, blocks((size_t)d.F * d.Mb * d.Mb * 64), dim3(256), 0, s, a);
      hipLaunchKernelGGL(k_adj_demix_x<R>, blocks((size_t)d.M * d.F * d.T), dim3(256), 0, s, a);
    }
    hipLaunchKernelGGL(k_adj_phi<R>, blocks(nft), dim3(256), 0, s, a);
  } else {
    const size_t lds = adj_iss_lds(d.Mb, d.T, rs);
    if (lds > 65536) {
      hipError_t e = hipFuncSetAttribute((const void*)k_adj_iss<R>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_adj_iss<R>, dim3(d.F), dim3(256), lds, s, a);
  }
  hipLaunchKernelGGL(k_adj_l1<R>, blocks(nfk * 64), dim3(256), 0, s, a);
  const int l2ch = adj_l2_chunks(d.F), l2fc = (d.F + l2ch - 1) / l2ch;
  R* l2sums = l2ch > 1 ? static_cast<R*>(p.l2sums) : nullptr;
  hipLaunchKernelGGL(k_adj_l2<R>, dim3((unsigned)(d.N * ((d.K + kL2Bases - 1) / kL2Bases) * ((d.T + 63) / 64)), l2ch),
                     dim3(64 * kL2Waves), 0, s, a, l2sums, l2fc);
  if (l2ch > 1) hipLaunchKernelGGL(k_adj_l2_sum<R>, blocks(nkt), dim3(256), 0, s, a, l2sums, l2ch);
  return hipGetLastError();
}
}  // namespace

// Host side: the images stage and one reverse iteration (rs = 4: FP32, 8: FP64);
// launches go to stream s.
hipError_t adj_images(const AdjPtrs& p, const Dims& d, const void* W, const void* gC, int rs, hipStream_t s) {
  return rs == 4 ? adj_images_t<float>(p, d, W, gC, s) : adj_images_t<double>(p, d, W, gC, s);
}

hipError_t adj_iteration(const AdjPtrs& p, const Dims& d, double floor, int rs, hipStream_t s) {
  return rs == 4 ? adj_iteration_t<float>(p, d, floor, s) : adj_iteration_t<double>(p, d, floor, s);
}

}  // namespace ctfiss
