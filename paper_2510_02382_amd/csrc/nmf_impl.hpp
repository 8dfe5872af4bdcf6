// Source-model kernels of one iteration: lambda = b v, basis update (Eq. (17)),
// activation update (Eq. (18) / ALL_TAPS) and the scale of Eq. (19).
//
// The scale of iteration i is applied lazily: b_n times 1/mu_{(n,0)}^2 where b is
// next read (k_lambda and k_nmf_b of iteration i+1, or the W update's own staging
// of b where it forms 1/lambda), W rows and carried Y rows times 1/mu in the next
// W update, and by k_apply_mu after the last iteration of a call.
#pragma once

#include "common.hpp"

namespace ctfiss {

template <typename R>
struct NmfArgs {
  R* B;              // [N][F][K] bases (in/out)
  R* V;              // [N][K][T] activations (in/out)
  R* ilam;           // [N][F][T] 1 / lambda (out of k_lambda)
  const R* P;        // [N][F][T] tap-aligned power
  const R* P0;       // [N][F][T] tap-0 power (PAPER_TAP0) or null
  R* vnum;           // [N][nch][K][T] partial numerators
  R* vden;           // [N][nch][K][T] partial denominators
  const R* musq;     // [Mb][F] row power sums
  R* mu;             // [Mb] scale of this iteration (out of k_vfinal or k_vupdate)
  const R* mu_prev;  // [Mb] pending scale of the previous iteration, or null
  int* status;
  int* work;         // bin counter of the W-update kernel, zeroed here by k_lambda
  int F, T, K, nch, fchunk, tap0;
  R floor;
  RowMap rm;
};


template <typename R>
__device__ __forceinline__ R pending_scale(const NmfArgs<R>& a, int n) {
  if (!a.mu_prev) return R(1);
  const R m = a.mu_prev[a.rm.r0[n]];
  return R(1) / (m * m);
}

// ------------------------------------------------------------------ MFMA
// 16x16x4 matrix-core tiles (one wave = 64 lanes).  Lane l = 16*lq + lr holds
// A[lr][lq] and B[lq][lr] of the 16x4 and 4x16 operands, and accumulator
// element v < 4 of the 16x16 result in row acc_row(lq, v), column lr: row
// 4*lq + v for the FP32 instruction, lq + 4*v for the FP64 one (measured on
// gfx950).
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
template <typename R>
struct Acc4;
template <>
struct Acc4<float> {
  typedef f32x4 type;
};
template <>
struct Acc4<double> {
  typedef f64x4 type;
};
__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma16(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
template <typename R>
__device__ __forceinline__ int acc_row(int lq, int v) {
  return sizeof(R) == 4 ? 4 * lq + v : lq + 4 * v;
}
template <typename R>
__device__ __forceinline__ typename Acc4<R>::type acc_zero() {
  typename Acc4<R>::type z;
  z[0] = z[1] = z[2] = z[3] = R(0);
  return z;
}

// Sums the 16x16 accumulator tiles (num, den per K tile) of the workgroup's
// first nwave waves in wave order into red[c][kt] (red[c][kt][v][l]: register
// v of lane l).  Each wave writes its tile of one (kt, c) to LDS once, then
// thread e adds element e of every wave's tile, wave 0 first: the same sums as
// adding the tiles wave after wave, with two barriers per tile instead of one
// per wave.  Every thread of the workgroup must call it.
template <typename R, int KT, int NW>
__device__ __forceinline__ void sum_wave_tiles(const typename Acc4<R>::type (&num)[KT],
                                               const typename Acc4<R>::type (&den)[KT], int nkt, int nwave,
                                               R (&tiles)[NW][4][64], R (&red)[2][KT][4][64]) {
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int kt = 0; kt < KT; ++kt) {
    if (kt >= nkt) break;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (wave < nwave) {
#pragma unroll
        for (int v = 0; v < 4; ++v) tiles[wave][v][l] = c ? den[kt][v] : num[kt][v];
      }
      __syncthreads();
      for (int e = threadIdx.x; e < 256; e += blockDim.x) {
        R acc = R(0);
        for (int w = 0; w < nwave; ++w) acc += tiles[w][e >> 6][e & 63];
        red[c][kt][e >> 6][e & 63] = acc;
      }
      __syncthreads();
    }
  }
}

// 1/lambda_{n,f,t} with lambda = (b / mu^2) v: one 16 (bins) x 16 (frames) tile
// per wave, K/4 MFMA steps.  Grid (ceil(T/64), ceil(F/16), N), 4 waves per
// workgroup covering 64 frames.
template <typename R>
__device__ __forceinline__ void lambda_block(const NmfArgs<R>& a, const int bx, const int by, const int bz) {
  constexpr int KS = kMaxK / 4;
  const int T = a.T, K = a.K, F = a.F;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, lr = l & 15, lq = l >> 4;
  const int n = bz, f0 = by * 16, t0 = bx * 64 + wave * 16;
  if (a.work && bx == 0 && by == 0 && bz == 0 && threadIdx.x == 0) *a.work = 0;
  if (t0 >= T) return;
  const int nks = (K + 3) / 4;
  const R sc = pending_scale(a, n);
  const R* Bn = a.B + (size_t)n * F * K;
  const R* Vn = a.V + (size_t)n * K * T;
  const int fa = f0 + lr, tb = t0 + lr;
  R av[KS], bv[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int k = 4 * s + lq;
    const bool ok = s < nks && k < K;
    av[s] = (ok && fa < F) ? Bn[(size_t)fa * K + k] : R(0);
    bv[s] = (ok && tb < T) ? Vn[(size_t)k * T + tb] : R(0);
  }
  typename Acc4<R>::type acc = acc_zero<R>();
#pragma unroll
  for (int s = 0; s < KS; ++s)
    if (s < nks) acc = mfma16(av[s] * sc, bv[s], acc);
  bool bad = false;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int f = f0 + acc_row<R>(lq, v);
    if (f < F && tb < T) {
      const R lam = acc[v];
      bad |= !finite_pos(lam);
      a.ilam[((size_t)n * F + f) * T + tb] = R(1) / lam;
    }
  }
  latch_wave(a.status, bad, kFaultMu);
}

template <typename R>
__global__ void __launch_bounds__(256) k_lambda(NmfArgs<R> a) { lambda_block<R>(a, blockIdx.x, blockIdx.y, blockIdx.z); }

// Basis update, Eq. (17), with t' = t - l:
//   num_{f,k} = sum_t' P_{f,t'} v_{k,t'} / lambda_{f,t'}^2,  den_{f,k} = sum_t' C_{t'} v_{k,t'} / lambda_{f,t'},
//   C_{t'} = #{l < L_n : t' + l < T};  b <- max((b / mu^2) sqrt(num / den), floor).
// (F x T)(T x K) contractions on MFMA: one workgroup per 16 bins, its waves
// split the frames, partial tiles are summed in LDS in wave order.
template <typename R>
__device__ __forceinline__ void nmfb_block(const NmfArgs<R>& a, const int bx, const int by, const int nwe) {
  constexpr int KT = kMaxK / 16;
  constexpr int ST = sizeof(R) == 4 ? 8 : 4;  // MFMA steps (4 frames each) per wave and round
  __shared__ R red[2][KT][4][64];
  __shared__ R tiles[kMaxNmfWaves][4][64];
  const int T = a.T, K = a.K, F = a.F;
  // nwe: waves that share the frames (a batched launch may carry more, which stay idle)
  const int wave = threadIdx.x >> 6, nwave = nwe, l = threadIdx.x & 63, lr = l & 15, lq = l >> 4;
  const int n = by, f0 = bx * 16;
  const int L = a.rm.L[n];
  const int nkt = (K + 15) / 16;
  const R* Pn = a.P + (size_t)n * F * T;
  const R* In = a.ilam + (size_t)n * F * T;
  const R* Vn = a.V + (size_t)n * K * T;
  const int fa = f0 + lr;
  typename Acc4<R>::type num[KT], den[KT];
#pragma unroll
  for (int kt = 0; kt < KT; ++kt) num[kt] = den[kt] = acc_zero<R>();
  // rounds of ST steps; every wave's operand loads of a round are issued before its MFMAs
  for (int base = wave * ST; wave < nwave && 4 * base < T; base += nwave * ST) {
    R e1[ST], e2[ST], bv[ST][KT];
#pragma unroll
    for (int st = 0; st < ST; ++st) {
      const int t = 4 * (base + st) + lq;
      e1[st] = e2[st] = R(0);
      if (fa < F && t < T) {
        const R il = In[(size_t)fa * T + t];
        e1[st] = Pn[(size_t)fa * T + t] * il * il;
        e2[st] = (R)min(L, T - t) * il;
      }
#pragma unroll
      for (int kt = 0; kt < KT; ++kt) {
        const int k = 16 * kt + lr;
        bv[st][kt] = (kt < nkt && k < K && t < T) ? Vn[(size_t)k * T + t] : R(0);
      }
    }
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
      if (kt < nkt) {
#pragma unroll
        for (int st = 0; st < ST; ++st) {
          num[kt] = mfma16(e1[st], bv[st][kt], num[kt]);
          den[kt] = mfma16(e2[st], bv[st][kt], den[kt]);
        }
      }
    }
  }
  sum_wave_tiles<R, KT, kMaxNmfWaves>(num, den, nkt, nwave, tiles, red);
  if (wave != 0) return;
  const R sc = pending_scale(a, n);
  bool bad = false;
#pragma unroll
  for (int kt = 0; kt < KT; ++kt) {
    if (kt >= nkt) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int f = f0 + acc_row<R>(lq, v), k = 16 * kt + lr;
      if (f < F && k < K) {
        const size_t o = ((size_t)n * F + f) * K + k;
        R b = a.B[o] * sc * sqrt(red[0][kt][v][l] / red[1][kt][v][l]);
        bad |= !isfinite(b);
        a.B[o] = b > a.floor ? b : a.floor;
      }
    }
  }
  latch_wave(a.status, bad, kFaultMu);  // one atomic per wave, not per lane
}

template <typename R>
__global__ void __launch_bounds__(1024) k_nmf_b(NmfArgs<R> a) { nmfb_block<R>(a, blockIdx.x, blockIdx.y, blockDim.x >> 6); }

// Scale of row r, Eq. (19): mu_r = sqrt(sum_f musq[r][f] / (F T)).  Thread i < 256 adds
// f = i, i + 256, ...; then a tree over those 256 threads: every caller gets the same
// value bit for bit.  Every thread of the workgroup (at least 256) calls it; red: 256
// values of LDS.
template <typename R>
__device__ __forceinline__ R row_scale(const NmfArgs<R>& a, int r, R* red) {
  const int tid = threadIdx.x;
  if (tid < 256) {
    R acc = 0;
    for (int f = tid; f < a.F; f += 256) acc += a.musq[(size_t)r * a.F + f];
    red[tid] = acc;
  }
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  const R m = sqrt(red[0] / (R(a.F) * R(a.T)));
  __syncthreads();  // red may be reused
  return m;
}

// v_{n,k,t} <- max(v sqrt(num / (C' den)), floor) from the chunk partials summed in
// chunk order; C' = #{l < L_n : t + l < T} (ALL_TAPS) or 1 (PAPER_TAP0).
template <typename R>
__device__ __forceinline__ R vfinal_value(const NmfArgs<R>& a, int n, int k, int t, bool& bad) {
  const int T = a.T, K = a.K;
  // up to 24 chunks' partials in flight at once (one round trip for F <= 1536 at 64 bins per
  // chunk), then added in chunk order
  constexpr int CB = 24;
  const size_t step = (size_t)K * T, o0 = ((size_t)n * a.nch * K + k) * T + t;
  R num = 0, den = 0;
  for (int c0 = 0; c0 < a.nch; c0 += CB) {
    R xn[CB], xd[CB];
#pragma unroll
    for (int u = 0; u < CB; ++u) {
      const bool ok = c0 + u < a.nch;
      xn[u] = ok ? a.vnum[o0 + (size_t)(c0 + u) * step] : R(0);
      xd[u] = ok ? a.vden[o0 + (size_t)(c0 + u) * step] : R(0);
    }
#pragma unroll
    for (int u = 0; u < CB; ++u) {
      if (c0 + u < a.nch) {
        num += xn[u];
        den += xd[u];
      }
    }
  }
  const R c = a.tap0 ? R(1) : (R)min(a.rm.L[n], T - t);
  const R v = a.V[((size_t)n * K + k) * T + t] * sqrt(num / (c * den));
  bad |= !isfinite(v);
  return v > a.floor ? v : a.floor;
}

// Partial sums over one chunk of bins of
//   num[k][t] = sum_f b_{f,k} P'_{f,t} / lambda_{f,t}^2,  den[k][t] = sum_f b_{f,k} / lambda_{f,t},
// with lambda = b v recomputed from the updated bases.  One wave per 16 frames
// of one chunk: per 16-bin sub-tile, lambda on MFMA (K/4 steps), the two
// weights in the accumulator layout, then b^T times them on MFMA (the bin
// index of the accumulator rows is the reduction index, 4 MFMA steps).
template <typename R>
__device__ __forceinline__ void vpart_block(const NmfArgs<R>& a, const int bx, const int by, const int bz) {
  constexpr int KT = kMaxK / 16;
  constexpr int KS = kMaxK / 4;
  __shared__ R red[2][KT][4][64];
  const int T = a.T, K = a.K, F = a.F;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, lr = l & 15, lq = l >> 4;
  const int n = bz, ch = by, t0 = bx * 16;
  const int f1 = min(F, ch * a.fchunk + a.fchunk);
  const int fs = ch * a.fchunk + 16 * wave;  // this wave's 16-bin sub-tile
  const int nkt = (K + 15) / 16, nks = (K + 3) / 4;
  const R* Bn = a.B + (size_t)n * F * K;
  const R* Vn = a.V + (size_t)n * K * T;
  const R* Pn = (a.tap0 ? a.P0 : a.P) + (size_t)n * F * T;
  const int tb = t0 + lr, fa = fs + lr;
  R av[KS], vop[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int k = 4 * s + lq;
    const bool ok = s < nks && k < K;
    vop[s] = (ok && tb < T) ? Vn[(size_t)k * T + tb] : R(0);
    av[s] = (ok && fa < f1) ? Bn[(size_t)fa * K + k] : R(0);
  }
  R pv[4], bt[KT][4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int f = fs + acc_row<R>(lq, v);
    pv[v] = (f < f1 && tb < T) ? Pn[(size_t)f * T + tb] : R(0);
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
      const int k = 16 * kt + lr;
      bt[kt][v] = (kt < nkt && f < f1 && k < K) ? Bn[(size_t)f * K + k] : R(0);
    }
  }
  typename Acc4<R>::type lam = acc_zero<R>();
#pragma unroll
  for (int s = 0; s < KS; ++s)
    if (s < nks) lam = mfma16(av[s], vop[s], lam);
  R e1[4], e2[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int f = fs + acc_row<R>(lq, v);
    e1[v] = e2[v] = R(0);
    if (f < f1 && tb < T) {
      const R il = R(1) / lam[v];
      e1[v] = pv[v] * il * il;
      e2[v] = il;
    }
  }
  typename Acc4<R>::type num[KT], den[KT];
#pragma unroll
  for (int kt = 0; kt < KT; ++kt) {
    num[kt] = den[kt] = acc_zero<R>();
    if (kt < nkt) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        num[kt] = mfma16(bt[kt][v], e1[v], num[kt]);
        den[kt] = mfma16(bt[kt][v], e2[v], den[kt]);
      }
    }
  }
  // the four waves' tiles in wave order (K tiles in use only)
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int kt = 0; kt < KT; ++kt) {
        if (kt >= nkt) break;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          red[0][kt][v][l] = (w == 0 ? R(0) : red[0][kt][v][l]) + num[kt][v];
          red[1][kt][v][l] = (w == 0 ? R(0) : red[1][kt][v][l]) + den[kt][v];
        }
      }
    }
    __syncthreads();
  }
  if (wave == 0 && tb < T) {
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
      if (kt >= nkt) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = 16 * kt + acc_row<R>(lq, v);
        if (k < K) {
          const size_t o = (((size_t)n * a.nch + ch) * K + k) * T + tb;
          a.vnum[o] = red[0][kt][v][l];
          a.vden[o] = red[1][kt][v][l];
        }
      }
    }
  }
}

template <typename R>
__global__ void __launch_bounds__(256) k_vpart(NmfArgs<R> a) { vpart_block<R>(a, blockIdx.x, blockIdx.y, blockIdx.z); }

// Activation update in one launch: one workgroup per (source n, 16 frames) whose waves
// take the 16-bin subtiles of the band in turn (subtile s to wave s mod waves), each
// accumulating
//   num[k][t] = sum_f b_{f,k} P'_{f,t} / lambda_{f,t}^2,  den[k][t] = sum_f b_{f,k} / lambda_{f,t}
// over its subtiles in its MFMA accumulators (lambda = b v recomputed on MFMA per subtile,
// as in k_vpart), the loads of its next subtile in flight while it computes one.  The waves'
// tiles are then added in wave order and the workgroup updates v at its frames,
// v <- max(v sqrt(num / (C' den)), floor).  No partial sums leave the workgroup, so no
// second launch adds them up.  The extra y slice (y = N) computes the row scales mu of
// Eq. (19).  NKT: 16-wide tiles of the bases (K <= 16 NKT).
template <typename R, int NKT>
constexpr int vupdate_threads() {
  return sizeof(R) == 4 ? (NKT <= 2 ? 1024 : 512) : (NKT <= 1 ? 1024 : NKT == 2 ? 512 : 256);
}
template <typename R, int NKT>
struct VSub {
  R av[4 * NKT];  // b_{f, 4s + lq} at f = fs + lr (lambda's A operand)
  R pv[4];        // P'_{f, t} at the accumulator rows f
  R bt[NKT][4];   // b_{f, 16 kt + lr} at the accumulator rows f
};
template <typename R, int NKT>
__global__ void __launch_bounds__((vupdate_threads<R, NKT>())) k_vupdate(NmfArgs<R> a) {
  constexpr int KS = 4 * NKT;
  constexpr int NW = vupdate_threads<R, NKT>() / 64;
  __shared__ R tiles[NW][2][NKT][4][64];
  if ((int)blockIdx.y == a.rm.N) {  // the row scales (workgroup-uniform branch)
    R* rs = &tiles[0][0][0][0][0];
    for (int r = blockIdx.x; r < a.rm.Mb; r += gridDim.x) {
      const R m = row_scale(a, r, rs);
      if (threadIdx.x == 0) {
        if (!finite_pos(m)) latch(a.status, kFaultScale);
        a.mu[r] = m;
      }
    }
    return;
  }
  const int T = a.T, K = a.K, F = a.F;
  const int wave = threadIdx.x >> 6, nwave = blockDim.x >> 6, l = threadIdx.x & 63, lr = l & 15, lq = l >> 4;
  const int n = blockIdx.y, tb = blockIdx.x * 16 + lr;
  const int nkt = (K + 15) / 16, nks = (K + 3) / 4;
  const R* Bn = a.B + (size_t)n * F * K;
  const R* Vn = a.V + (size_t)n * K * T;
  const R* Pn = (a.tap0 ? a.P0 : a.P) + (size_t)n * F * T;
  R vop[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int k = 4 * s + lq;
    vop[s] = (s < nks && k < K && tb < T) ? Vn[(size_t)k * T + tb] : R(0);
  }
  __shared__ R vt[16 * NKT][16];  // v of the workgroup's frames, for the final update
  if (wave == 0) {
#pragma unroll
    for (int s = 0; s < KS; ++s) vt[4 * s + lq][lr] = vop[s];
  }
  auto load = [&](int fs, VSub<R, NKT>& u) {
    const int fa = fs + lr;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int k = 4 * s + lq;
      u.av[s] = (s < nks && k < K && fa < F) ? Bn[(size_t)fa * K + k] : R(0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int f = fs + acc_row<R>(lq, v);
      u.pv[v] = (f < F && tb < T) ? Pn[(size_t)f * T + tb] : R(0);
#pragma unroll
      for (int kt = 0; kt < NKT; ++kt) {
        const int k = 16 * kt + lr;
        u.bt[kt][v] = (kt < nkt && f < F && k < K) ? Bn[(size_t)f * K + k] : R(0);
      }
    }
  };
  typename Acc4<R>::type num[NKT], den[NKT];
#pragma unroll
  for (int kt = 0; kt < NKT; ++kt) num[kt] = den[kt] = acc_zero<R>();
  const int step = 16 * nwave;
  VSub<R, NKT> cur;
  load(16 * wave, cur);
  for (int fs = 16 * wave; fs < F; fs += step) {
    VSub<R, NKT> nxt;
    load(fs + step, nxt);  // lanes past the band load nothing
    typename Acc4<R>::type lam = acc_zero<R>();
#pragma unroll
    for (int s = 0; s < KS; ++s)
      if (s < nks) lam = mfma16(cur.av[s], vop[s], lam);
    R e1[4], e2[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int f = fs + acc_row<R>(lq, v);
      e1[v] = e2[v] = R(0);
      if (f < F && tb < T) {
        const R il = R(1) / lam[v];
        e1[v] = cur.pv[v] * il * il;
        e2[v] = il;
      }
    }
#pragma unroll
    for (int kt = 0; kt < NKT; ++kt) {
      if (kt < nkt) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          num[kt] = mfma16(cur.bt[kt][v], e1[v], num[kt]);
          den[kt] = mfma16(cur.bt[kt][v], e2[v], den[kt]);
        }
      }
    }
    cur = nxt;
  }
  // every wave's tiles to LDS at once, then element e of the sums: waves added in order
#pragma unroll
  for (int kt = 0; kt < NKT; ++kt) {
    if (kt < nkt) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        tiles[wave][0][kt][v][l] = num[kt][v];
        tiles[wave][1][kt][v][l] = den[kt][v];
      }
    }
  }
  __syncthreads();
  const int nel = 2 * NKT * 256;
  for (int e = threadIdx.x; e < nel; e += blockDim.x) {
    R* col = &tiles[0][0][0][0][0] + e;
    R acc = R(0);
    for (int w = 0; w < nwave; ++w) acc += col[(size_t)w * nel];
    col[0] = acc;  // wave 0's slot: read by this thread alone above
  }
  __syncthreads();
  if (wave != 0) return;
  bool bad = false;
  if (tb < T) {
    const R c = a.tap0 ? R(1) : (R)min(a.rm.L[n], T - tb);
#pragma unroll
    for (int kt = 0; kt < NKT; ++kt) {
      if (kt >= nkt) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = 16 * kt + acc_row<R>(lq, v);
        if (k < K) {
          const size_t o = ((size_t)n * K + k) * T + tb;
          const R vv = vt[k][lr] * sqrt(tiles[0][0][kt][v][l] / (c * tiles[0][1][kt][v][l]));
          bad |= !isfinite(vv);
          a.V[o] = vv > a.floor ? vv : a.floor;
        }
      }
    }
  }
  latch_wave(a.status, bad, kFaultMu);
}

// v <- max(v sqrt(num / (C' den)), floor) with the chunk partials summed in
// chunk order; C' = #{l < L_n : t + l < T} (ALL_TAPS) or 1 (PAPER_TAP0).
// The last Mb workgroups compute mu_r = sqrt(sum_f musq[r][f] / (F T)), Eq. (19).
template <typename R>
__device__ __forceinline__ void vfinal_block(const NmfArgs<R>& a, const int nvblocks, const int bx) {
  const int T = a.T, K = a.K, N = a.rm.N;
  if (bx >= nvblocks) {
    __shared__ R red[256];
    const int r = bx - nvblocks;
    const R m = row_scale(a, r, red);
    if (threadIdx.x == 0) {
      if (!finite_pos(m)) latch(a.status, kFaultScale);
      a.mu[r] = m;
    }
    return;
  }
  const int i = bx * blockDim.x + threadIdx.x;
  if (i >= N * K * T) return;
  const int n = i / (K * T), k = (i / T) % K, t = i % T;
  bool bad = false;
  const R v = vfinal_value(a, n, k, t, bad);
  latch_wave(a.status, bad, kFaultMu);
  a.V[i] = v;
}

template <typename R>
__global__ void __launch_bounds__(256) k_vfinal(NmfArgs<R> a, int nvblocks) { vfinal_block<R>(a, nvblocks, blockIdx.x); }

// ------------------------------------------------------------------ batched
// One grid over the workgroups of many problems (mixtures): a workgroup finds
// its problem in start[] and runs that problem's workgroup (gx, gy: the
// problem's own grid extents; z follows).  The work of each problem is the one
// its single-problem launch does, in the same order.
template <typename R>
struct NmfDesc {
  NmfArgs<R> a;
  int gx, gy;
  int extra;  // k_nmf_b: waves sharing the frames; k_vfinal: activation workgroups
};

template <typename R>
__global__ void __launch_bounds__(256) k_lambda_batch(const NmfDesc<R>* d, const int* start, int nprob, int* zero,
                                                      int nzero) {
  if (blockIdx.x == 0 && (int)threadIdx.x < nzero) zero[threadIdx.x] = 0;  // bin counters of the next launch
  const int m = find_problem(start, nprob, blockIdx.x);
  const NmfDesc<R>& D = d[m];
  int b = blockIdx.x - start[m];
  const int bx = b % D.gx;
  b /= D.gx;
  lambda_block<R>(D.a, bx, b % D.gy, b / D.gy);
}

template <typename R>
__global__ void __launch_bounds__(1024) k_nmf_b_batch(const NmfDesc<R>* d, const int* start, int nprob) {
  const int m = find_problem(start, nprob, blockIdx.x);
  const NmfDesc<R>& D = d[m];
  const int b = blockIdx.x - start[m];
  nmfb_block<R>(D.a, b % D.gx, b / D.gx, D.extra);
}

template <typename R>
__global__ void __launch_bounds__(256) k_vpart_batch(const NmfDesc<R>* d, const int* start, int nprob) {
  const int m = find_problem(start, nprob, blockIdx.x);
  const NmfDesc<R>& D = d[m];
  int b = blockIdx.x - start[m];
  const int bx = b % D.gx;
  b /= D.gx;
  vpart_block<R>(D.a, bx, b % D.gy, b / D.gy);
}

template <typename R>
__global__ void __launch_bounds__(256) k_vfinal_batch(const NmfDesc<R>* d, const int* start, int nprob) {
  const int m = find_problem(start, nprob, blockIdx.x);
  const NmfDesc<R>& D = d[m];
  vfinal_block<R>(D.a, D.extra, blockIdx.x - start[m]);
}

// W row r /= mu_r and b_n /= mu_{(n,0)}^2, Eqs. (20)-(21) applied to W and b;
// row r of the carried Y (when given) /= mu_r, keeping Y = W xbar.
template <typename R>
__global__ void __launch_bounds__(256) k_apply_mu(Cx<R>* W, R* B, Cx<R>* Y, const R* mu, int F, int T, int K,
                                                  RowMap rm) {
  const int Mb = rm.Mb, N = rm.N;
  const size_t nw = (size_t)F * Mb * Mb, nb = (size_t)N * F * K, ny = Y ? (size_t)F * Mb * T : 0;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nw) {
    const R rm = R(1) / mu[(i / Mb) % Mb];  // the rounding of the lazy form in the W update
    Cx<R> w = W[i];
    W[i] = Cx<R>{w.x * rm, w.y * rm};
  } else if (i < nw + nb) {
    const size_t j = i - nw;
    const int n = (int)(j / ((size_t)F * K));
    const R m = mu[rm.r0[n]];
    B[j] = B[j] * (R(1) / (m * m));  // the same rounding as pending_scale
  } else if (i < nw + nb + ny) {
    const size_t j = i - nw - nb;
    const R rm = R(1) / mu[(j / T) % Mb];
    Cx<R> y = Y[j];
    Y[j] = Cx<R>{y.x * rm, y.y * rm};
  }
}

}  // namespace ctfiss
