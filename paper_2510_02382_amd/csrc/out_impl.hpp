// Source images (Sec. III-B, Eq. (24)) and the objective of Eq. (5), both in FP64.
#pragma once

#include "common.hpp"

namespace ctfiss {

// Gaussian elimination with partial pivoting on the n x (n + nrhs) row-major
// matrix A (LDS).  On return the first n columns hold U, the right-hand
// sides hold the solutions (back substitution by one thread per column),
// and *logdet (thread 0) holds sum log|U_kk|.  A zero pivot latches `code`.
__device__ inline void lu_solve_d(Cx<double>* A, int n, int nrhs, Cx<double>* fac, int* piv_slot,
                                  double* logdet, int* status, int code) {
  const int tid = threadIdx.x, nthr = blockDim.x, ld = n + nrhs;
  double ld_acc = 0;
  for (int k = 0; k < n; ++k) {
    if (tid == 0) {
      int piv = k;
      double best = cabs2(A[k * ld + k]);
      for (int i = k + 1; i < n; ++i) {
        const double v = cabs2(A[i * ld + k]);
        if (v > best) {
          best = v;
          piv = i;
        }
      }
      if (!finite_pos(best)) latch(status, code);
      ld_acc += 0.5 * log(best);
      *piv_slot = piv;
    }
    __syncthreads();
    const int piv = *piv_slot;
    if (piv != k) {
      for (int j = k + tid; j < ld; j += nthr) {
        const Cx<double> t = A[k * ld + j];
        A[k * ld + j] = A[piv * ld + j];
        A[piv * ld + j] = t;
      }
    }
    __syncthreads();
    const Cx<double> pv = A[k * ld + k];
    const double den = cabs2(pv);
    const Cx<double> inv{pv.x / den, -pv.y / den};
    for (int i = k + 1 + tid; i < n; i += nthr) fac[i] = cmul(A[i * ld + k], inv);
    __syncthreads();
    const int w = ld - k - 1;
    for (int e = tid; e < (n - k - 1) * w; e += nthr) {
      const int i = k + 1 + e / w, j = k + 1 + e % w;
      A[i * ld + j] = cfms(fac[i], A[k * ld + j], A[i * ld + j]);
    }
    __syncthreads();
  }
  for (int c = tid; c < nrhs; c += nthr) {
    for (int i = n - 1; i >= 0; --i) {
      Cx<double> acc = A[i * ld + n + c];
      for (int j = i + 1; j < n; ++j) acc = cfms(A[i * ld + j], A[j * ld + n + c], acc);
      const Cx<double> pv = A[i * ld + i];
      const double den = cabs2(pv);
      A[i * ld + n + c] = Cx<double>{(acc.x * pv.x + acc.y * pv.y) / den, (acc.y * pv.x - acc.x * pv.y) / den};
    }
  }
  if (tid == 0 && logdet) *logdet = ld_acc;
  __syncthreads();
}

template <typename R>
struct OutArgs {
  const Cx<R>* X;   // [M][F][T]
  const Cx<R>* W;   // [F][Mb][Mb]
  const R* B;       // [N][F][K]
  const R* V;       // [N][K][T]
  Cx<R>* C;         // [N][M][F][T] (images)
  double* part;     // [F] per-bin objective (nll)
  int* status;
  int F, T, M, D, K;
  RowMap rm;
};

// LDS: A [Mb][Mb+M] (W^T | E_M), then G [N][M][Mb] projection matrices.
__host__ __device__ inline size_t out_lds_bytes(int Mb, int M, int N) {
  return sizeof(Cx<double>) * ((size_t)Mb * (Mb + M) + (size_t)N * M * Mb + Mb) + 64;
}

// c_{n,m,f,t} = sum_c G_n[m][c] xbar_c[t] with G_n = H_f[:M, rows(n)] W_f[rows(n), :]
// and H_f = W_f^{-1}: the first M rows of H solve W^T h_m = e_m.
template <typename R>
__global__ void __launch_bounds__(256) k_images(OutArgs<R> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int f = blockIdx.x, tid = threadIdx.x, nthr = blockDim.x;
  const int Mb = a.rm.Mb, M = a.M, N = a.rm.N, T = a.T, F = a.F, D = a.D;
  Cx<double>* A = reinterpret_cast<Cx<double>*>(smem);
  Cx<double>* G = A + (size_t)Mb * (Mb + M);
  Cx<double>* fac = G + (size_t)N * M * Mb;
  int* piv = reinterpret_cast<int*>(fac + Mb);
  const int ld = Mb + M;
  const Cx<R>* Wf = a.W + (size_t)f * Mb * Mb;
  for (int e = tid; e < Mb * ld; e += nthr) {
    const int i = e / ld, j = e - (e / ld) * ld;
    Cx<double> v{0.0, 0.0};
    if (j < Mb) {
      const Cx<R> w = Wf[j * Mb + i];  // transpose
      v = Cx<double>{(double)w.x, (double)w.y};
    } else if (i == j - Mb) {
      v = Cx<double>{1.0, 0.0};
    }
    A[e] = v;
  }
  __syncthreads();
  lu_solve_d(A, Mb, M, fac, piv, nullptr, a.status, kFaultOutSingular);
  // H[m][r] = A[r][Mb + m]
  for (int e = tid; e < N * M * Mb; e += nthr) {
    const int n = e / (M * Mb), m = (e / Mb) % M, c = e % Mb;
    const int r0 = a.rm.r0[n], L = a.rm.L[n];
    Cx<double> acc{0.0, 0.0};
    for (int l = 0; l < L; ++l) {
      const Cx<R> w = Wf[(r0 + l) * Mb + c];
      acc = cfma(A[(r0 + l) * ld + Mb + m], Cx<double>{(double)w.x, (double)w.y}, acc);
    }
    G[e] = acc;
  }
  __syncthreads();
  for (int e = tid; e < N * M * T; e += nthr) {
    const int n = e / (M * T), m = (e / T) % M, t = e % T;
    const Cx<double>* g = G + ((size_t)n * M + m) * Mb;
    Cx<double> acc{0.0, 0.0};
    for (int d = 0; d < D && d <= t; ++d) {
      for (int mm = 0; mm < M; ++mm) {
        const Cx<R> x = a.X[((size_t)mm * F + f) * T + (t - d)];
        acc = cfma(g[d * M + mm], Cx<double>{(double)x.x, (double)x.y}, acc);
      }
    }
    a.C[(((size_t)n * M + m) * F + f) * T + t] = Cx<R>{(R)acc.x, (R)acc.y};
  }
}

// Per-bin part of Eq. (5): sum_{r, t >= l} (log lambda + |y|^2 / lambda) - 2T log|det W_f|.
template <typename R>
__global__ void __launch_bounds__(256) k_nll(OutArgs<R> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int f = blockIdx.x, tid = threadIdx.x, nthr = blockDim.x;
  const int Mb = a.rm.Mb, M = a.M, N = a.rm.N, T = a.T, F = a.F, D = a.D, K = a.K;
  Cx<double>* A = reinterpret_cast<Cx<double>*>(smem);
  Cx<double>* fac = A + (size_t)Mb * Mb;
  double* red = reinterpret_cast<double*>(fac + Mb);
  int* piv = reinterpret_cast<int*>(red + 256);
  const Cx<R>* Wf = a.W + (size_t)f * Mb * Mb;
  for (int e = tid; e < Mb * Mb; e += nthr) A[e] = Cx<double>{(double)Wf[e].x, (double)Wf[e].y};
  __syncthreads();
  double logdet = 0;
  lu_solve_d(A, Mb, 0, fac, piv, &logdet, a.status, kFaultOutSingular);
  double acc = 0;
  for (int e = tid; e < Mb * T; e += nthr) {
    const int r = e / T, t = e % T;
    const int n = a.rm.src[r], l = a.rm.tap[r];
    if (t < l) continue;
    double lam = 0;
    for (int k = 0; k < K; ++k)
      lam += (double)a.B[((size_t)n * F + f) * K + k] * (double)a.V[((size_t)n * K + k) * T + (t - l)];
    Cx<double> y{0.0, 0.0};
    for (int d = 0; d < D && d <= t; ++d) {
      for (int m = 0; m < M; ++m) {
        const Cx<R> w = Wf[r * Mb + d * M + m];
        const Cx<R> x = a.X[((size_t)m * F + f) * T + (t - d)];
        y = cfma(Cx<double>{(double)w.x, (double)w.y}, Cx<double>{(double)x.x, (double)x.y}, y);
      }
    }
    acc += log(lam) + cabs2(y) / lam;
  }
  red[tid] = acc;
  __syncthreads();
  for (int w = nthr / 2; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) a.part[f] = red[0] - 2.0 * T * logdet;
}

__host__ __device__ inline size_t nll_lds_bytes(int Mb) {
  return sizeof(Cx<double>) * ((size_t)Mb * Mb + Mb) + 256 * sizeof(double) + 64;
}

}  // namespace ctfiss
