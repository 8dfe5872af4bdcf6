// Source-model kernels of one iteration: lambda = b v, basis update (Eq. (17)),
// activation update (Eq. (18) / ALL_TAPS) and the scale of Eq. (19).
//
// The scale of iteration i is applied lazily: b_n /= mu_{(n,0)}^2 where b is
// next read (k_lambda and k_nmf_b of iteration i+1), W rows /= mu in the next
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
  R* mu;             // [Mb] scale of this iteration (out of k_vfinal)
  const R* mu_prev;  // [Mb] pending scale of the previous iteration, or null
  int* status;
  int F, T, K, nch, fchunk, tap0;
  R floor;
  RowMap rm;
};

constexpr int kTile = 64;   // frames per workgroup tile
constexpr int kFSub = 4;    // bins per LDS sub-tile (one per wave)

template <typename R>
__device__ __forceinline__ R pending_scale(const NmfArgs<R>& a, int n) {
  if (!a.mu_prev) return R(1);
  const R m = a.mu_prev[a.rm.r0[n]];
  return R(1) / (m * m);
}

// 1/lambda_{n,f,t} with lambda = (b / mu^2) v.  256 threads: 64 frames x 4 bin lanes,
// 16 bins per workgroup.
template <typename R>
__global__ void __launch_bounds__(256) k_lambda(NmfArgs<R> a) {
  __shared__ R sV[kMaxK][kTile];
  __shared__ R sB[16][kMaxK];
  const int T = a.T, K = a.K, F = a.F;
  const int t0 = blockIdx.x * kTile, f0 = blockIdx.y * 16, n = blockIdx.z;
  const int tl = threadIdx.x & (kTile - 1), fl = threadIdx.x / kTile;
  const R sc = pending_scale(a, n);
  for (int i = threadIdx.x; i < K * kTile; i += blockDim.x) {
    const int k = i / kTile, t = t0 + (i - k * kTile);
    sV[k][i - k * kTile] = t < T ? a.V[((size_t)n * K + k) * T + t] : R(0);
  }
  for (int i = threadIdx.x; i < 16 * K; i += blockDim.x) {
    const int fi = i / K, k = i - fi * K;
    sB[fi][k] = f0 + fi < F ? a.B[((size_t)n * F + f0 + fi) * K + k] * sc : R(0);
  }
  __syncthreads();
  const int t = t0 + tl;
  if (t >= T) return;
  for (int fi = fl; fi < 16 && f0 + fi < F; fi += 4) {
    R lam = 0;
    for (int k = 0; k < K; ++k) lam += sB[fi][k] * sV[k][tl];
    if (!finite_pos(lam)) latch(a.status, kFaultMu);
    a.ilam[((size_t)n * F + f0 + fi) * T + t] = R(1) / lam;
  }
}

// Basis update, Eq. (17), with t' = t - l:
//   num_k = sum_t' P_{t'} v_{k,t'} / lambda_{t'}^2,  den_k = sum_t' C_{t'} v_{k,t'} / lambda_{t'},
//   C_{t'} = #{l < L_n : t' + l < T};  b <- max((b / mu^2) sqrt(num / den), floor).
// 256 threads per workgroup, FB bins per workgroup, one (bin, k) pair per thread.
template <typename R>
__global__ void __launch_bounds__(256) k_nmf_b(NmfArgs<R> a, int FB) {
  __shared__ R sV[kMaxK][kTile];
  __shared__ R sE1[16][kTile];
  __shared__ R sE2[16][kTile];
  const int T = a.T, K = a.K, F = a.F;
  const int f0 = blockIdx.x * FB, n = blockIdx.y;
  const int L = a.rm.L[n];
  const int pair = threadIdx.x, fi = pair / K, k = pair - fi * K;
  const bool own = fi < FB && f0 + fi < F;
  R num = 0, den = 0;
  for (int t0 = 0; t0 < T; t0 += kTile) {
    __syncthreads();
    for (int i = threadIdx.x; i < K * kTile; i += blockDim.x) {
      const int kk = i / kTile, t = t0 + (i - kk * kTile);
      sV[kk][i - kk * kTile] = t < T ? a.V[((size_t)n * K + kk) * T + t] : R(0);
    }
    for (int i = threadIdx.x; i < FB * kTile; i += blockDim.x) {
      const int ff = i / kTile, t = t0 + (i - ff * kTile);
      R e1 = 0, e2 = 0;
      if (t < T && f0 + ff < F) {
        const size_t o = ((size_t)n * F + f0 + ff) * T + t;
        const R il = a.ilam[o];
        e1 = a.P[o] * il * il;
        e2 = (R)min(L, T - t) * il;
      }
      sE1[ff][i - ff * kTile] = e1;
      sE2[ff][i - ff * kTile] = e2;
    }
    __syncthreads();
    if (own) {
#pragma unroll 8
      for (int tl = 0; tl < kTile; ++tl) {
        num += sE1[fi][tl] * sV[k][tl];
        den += sE2[fi][tl] * sV[k][tl];
      }
    }
  }
  if (own) {
    const size_t o = ((size_t)n * F + f0 + fi) * K + k;
    R b = a.B[o] * pending_scale(a, n) * sqrt(num / den);
    if (!isfinite(b)) latch(a.status, kFaultMu);
    a.B[o] = b > a.floor ? b : a.floor;
  }
}

// Partial sums over one chunk of bins of
//   num[k][t] = sum_f b_{f,k} P'_{f,t} / lambda_{f,t}^2,  den[k][t] = sum_f b_{f,k} / lambda_{f,t},
// with lambda = b v recomputed from the updated bases.  256 threads:
// thread (kg, tl) owns frame t0 + tl and bases k = kg, kg + 4, ...
template <typename R>
__global__ void __launch_bounds__(256) k_vpart(NmfArgs<R> a) {
  __shared__ R sV[kMaxK][kTile];
  __shared__ R sB[kFSub][kMaxK];
  __shared__ R sE1[kFSub][kTile];
  __shared__ R sE2[kFSub][kTile];
  const int T = a.T, K = a.K, F = a.F;
  const int t0 = blockIdx.x * kTile, ch = blockIdx.y, n = blockIdx.z;
  const int f0 = ch * a.fchunk;
  const int f1 = min(F, f0 + a.fchunk);
  const int tl = threadIdx.x & (kTile - 1), kg = threadIdx.x / kTile;
  const int t = t0 + tl;
  const bool tin = t < T;
  const R* Pn = (a.tap0 ? a.P0 : a.P) + (size_t)n * F * T;
  for (int i = threadIdx.x; i < K * kTile; i += blockDim.x) {
    const int k = i / kTile, tt = t0 + (i - k * kTile);
    sV[k][i - k * kTile] = tt < T ? a.V[((size_t)n * K + k) * T + tt] : R(1);
  }
  constexpr int KPT = kMaxK / 4;
  R num[KPT], den[KPT];
#pragma unroll
  for (int i = 0; i < KPT; ++i) num[i] = den[i] = R(0);
  const R* Bn = a.B + (size_t)n * F * K;
  for (int fs = f0; fs < f1; fs += kFSub) {
    __syncthreads();
    for (int i = threadIdx.x; i < kFSub * K; i += blockDim.x) {
      const int fi = i / K, k = i - fi * K;
      sB[fi][k] = fs + fi < f1 ? Bn[(size_t)(fs + fi) * K + k] : R(0);
    }
    __syncthreads();
    {
      const int fi = kg, f = fs + fi;
      R e1 = 0, e2 = 0;
      if (f < f1 && tin) {
        R lam = 0;
        for (int k = 0; k < K; ++k) lam += sB[fi][k] * sV[k][tl];
        const R il = R(1) / lam;
        e1 = Pn[(size_t)f * T + t] * il * il;
        e2 = il;
      }
      sE1[fi][tl] = e1;
      sE2[fi][tl] = e2;
    }
    __syncthreads();
    const int nf = min(kFSub, f1 - fs);
    for (int fi = 0; fi < nf; ++fi) {
      const R e1 = sE1[fi][tl], e2 = sE2[fi][tl];
#pragma unroll
      for (int i = 0; i < KPT; ++i) {
        const int k = kg + 4 * i;
        if (k < K) {
          num[i] += sB[fi][k] * e1;
          den[i] += sB[fi][k] * e2;
        }
      }
    }
  }
  if (tin) {
#pragma unroll
    for (int i = 0; i < KPT; ++i) {
      const int k = kg + 4 * i;
      if (k < K) {
        const size_t o = (((size_t)n * a.nch + ch) * K + k) * T + t;
        a.vnum[o] = num[i];
        a.vden[o] = den[i];
      }
    }
  }
}

// v <- max(v sqrt(num / (C' den)), floor) with the chunk partials summed in
// chunk order; C' = #{l < L_n : t + l < T} (ALL_TAPS) or 1 (PAPER_TAP0).
// The last Mb workgroups compute mu_r = sqrt(sum_f musq[r][f] / (F T)), Eq. (19).
template <typename R>
__global__ void __launch_bounds__(256) k_vfinal(NmfArgs<R> a, int nvblocks) {
  const int T = a.T, K = a.K, N = a.rm.N;
  if ((int)blockIdx.x >= nvblocks) {
    __shared__ R red[256];
    const int r = blockIdx.x - nvblocks, F = a.F;
    R acc = 0;
    for (int f = threadIdx.x; f < F; f += blockDim.x) acc += a.musq[(size_t)r * F + f];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const R m = sqrt(red[0] / (R(F) * R(T)));
      if (!finite_pos(m)) latch(a.status, kFaultScale);
      a.mu[r] = m;
    }
    return;
  }
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * K * T) return;
  const int n = i / (K * T), k = (i / T) % K, t = i % T;
  R num = 0, den = 0;
  for (int ch = 0; ch < a.nch; ++ch) {
    const size_t o = (((size_t)n * a.nch + ch) * K + k) * T + t;
    num += a.vnum[o];
    den += a.vden[o];
  }
  const R c = a.tap0 ? R(1) : (R)min(a.rm.L[n], T - t);
  R v = a.V[i] * sqrt(num / (c * den));
  if (!isfinite(v)) latch(a.status, kFaultMu);
  a.V[i] = v > a.floor ? v : a.floor;
}

// W row r /= mu_r and b_n /= mu_{(n,0)}^2, Eqs. (20)-(21) applied to W and b.
template <typename R>
__global__ void __launch_bounds__(256) k_apply_mu(Cx<R>* W, R* B, const R* mu, int F, int K, RowMap rm) {
  const int Mb = rm.Mb, N = rm.N;
  const size_t nw = (size_t)F * Mb * Mb, nb = (size_t)N * F * K;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nw) {
    const R m = mu[(i / Mb) % Mb];
    Cx<R> w = W[i];
    W[i] = Cx<R>{w.x / m, w.y / m};
  } else if (i < nw + nb) {
    const size_t j = i - nw;
    const int n = (int)(j / ((size_t)F * K));
    const R m = mu[rm.r0[n]];
    B[j] = B[j] * (R(1) / (m * m));  // the same rounding as pending_scale
  }
}

}  // namespace ctfiss
