// Activation update (Eq. (18) / ALL_TAPS), scale normalisation (Eqs. (19)-(21)).
#pragma once

#include "common.hpp"

namespace ctfiss {

template <typename R>
struct VArgs {
  const R* B;        // [N][F][K] updated bases
  R* V;              // [N][K][T] activations (in/out)
  const R* P;        // [N][F][T] tap-aligned power (ALL_TAPS) or tap-0 power (PAPER_TAP0)
  R* vnum;           // [N][nch][K][T] partial numerators
  R* vden;           // [N][nch][K][T] partial denominators
  const R* musq;     // [F][Mb] row power sums
  R* mu;             // [Mb] scale of this iteration (out)
  int* status;
  int F, T, K, nch, fchunk, tap0;
  R floor;
  RowMap rm;
};

constexpr int kVTile = 64;   // frames per workgroup
constexpr int kVFSub = 4;    // bins per LDS sub-tile (one per wave)

// Partial sums over one chunk of bins of
//   num[k][t] = sum_f b_{f,k} P'_{f,t} / lambda_{f,t}^2,  den[k][t] = sum_f b_{f,k} / lambda_{f,t},
// with lambda = b v recomputed from the updated bases.  256 threads:
// thread (kg, tl) owns frame t0 + tl and bases k = kg, kg + 4, ...
template <typename R>
__global__ void __launch_bounds__(256) k_vpart(VArgs<R> a) {
  __shared__ R sV[kMaxK][kVTile];
  __shared__ R sB[kVFSub][kMaxK];
  __shared__ R sE1[kVFSub][kVTile];
  __shared__ R sE2[kVFSub][kVTile];
  const int T = a.T, K = a.K, F = a.F;
  const int t0 = blockIdx.x * kVTile, ch = blockIdx.y, n = blockIdx.z;
  const int f0 = ch * a.fchunk;
  const int f1 = min(F, f0 + a.fchunk);
  const int tl = threadIdx.x & (kVTile - 1), kg = threadIdx.x / kVTile;
  const int t = t0 + tl;
  const bool tin = t < T;
  for (int i = threadIdx.x; i < K * kVTile; i += blockDim.x) {
    const int k = i / kVTile, tt = t0 + (i - k * kVTile);
    sV[k][i - k * kVTile] = tt < T ? a.V[((size_t)n * K + k) * T + tt] : R(1);
  }
  constexpr int KPT = kMaxK / 4;
  R num[KPT], den[KPT];
#pragma unroll
  for (int i = 0; i < KPT; ++i) num[i] = den[i] = R(0);
  const R* Bn = a.B + (size_t)n * F * K;
  const R* Pn = a.P + (size_t)n * F * T;
  for (int fs = f0; fs < f1; fs += kVFSub) {
    __syncthreads();
    for (int i = threadIdx.x; i < kVFSub * K; i += blockDim.x) {
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
    const int nf = min(kVFSub, f1 - fs);
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
// The last workgroup computes mu_r = sqrt(sum_f musq[f][r] / (F T)), Eq. (19).
template <typename R>
__global__ void __launch_bounds__(256) k_vfinal(VArgs<R> a) {
  const int T = a.T, K = a.K, N = a.rm.N;
  if (blockIdx.x == gridDim.x - 1) {
    __shared__ R red[256];
    const int Mb = a.rm.Mb, F = a.F;
    for (int r = 0; r < Mb; ++r) {
      R acc = 0;
      for (int f = threadIdx.x; f < F; f += blockDim.x) acc += a.musq[(size_t)f * Mb + r];
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
      __syncthreads();
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
    B[j] = B[j] / (m * m);
  }
}

}  // namespace ctfiss
