// W-update kernels of one CTF-MNMF iteration: one workgroup per frequency bin.
//
// Each workgroup
//   1. applies the pending scale of the previous iteration to W_f and b_f
//      (Eqs. (19)-(21)), forms the source variances lambda_{n,f,t} = b v
//      and the stacked observation block on chip;
//   2. demixes, y = W_f xbar (Eq. (4)), into registers;
//   3. runs the W update: the ISS sweep (Eqs. (11), (16)) or the IP sweep
//      (Eqs. (9), (10));
//   4. writes W_f, the tap-aligned powers P_{n,f,t'} = sum_l |y_{(n,l),f,t'+l}|^2,
//      the row power sums used for the scale of Eq. (19), and the updated
//      bases b_f of Eq. (17) (a T-long reduction per (n, k), done here while
//      lambda and P of the bin are on chip).
//
// Register layout of the demixed signals: the block is split into groups of
// G lanes; group g owns row p = g of Y_f and lane q of the group holds the
// frames t = q + G*j, j < CPL.  A row's frame reductions are therefore
// G-lane DPP butterflies, and each ISS step needs one LDS broadcast of y_r
// and one barrier.
#pragma once

#include "common.hpp"

namespace ctfiss {

template <typename R>
struct IterArgs {
  const Cx<R>* X;  // [M][F][T] observation
  Cx<R>* W;        // [F][Mb][Mb] demixing matrices (in/out)
  R* B;            // [N][F][K] bases (in/out)
  const R* V;      // [N][K][T] activations
  R* P;            // [N][F][T] tap-aligned power (out)
  R* P0;           // [N][F][T] tap-0 power (out, activation rule PAPER_TAP0) or null
  R* musq;         // [F][Mb] row power sums (out)
  const R* mu;     // [Mb] scale of the previous iteration still to apply, or null
  int* status;
  int F, T, M, D, K;
  R floor;
  RowMap rm;
};

template <typename R>
struct BinLds {
  Cx<R>* x;    // [M][T]
  Cx<R>* w;    // [Mb][Mb]
  R* a;        // [Mb][T] |y|^2 (aliases x, w after the sweep)
  R* lam;      // [N][T]
  R* p;        // [N][T]
  R* b;        // [N][K]
  Cx<R>* yb;   // [2][T] broadcast of y_r
  Cx<R>* wb;   // [2][Mb] broadcast of w_r^H
  Cx<R>* q;    // [Mb][Mb]  (IP)
  Cx<R>* aug;  // [Mb][Mb+1] (IP)
  Cx<R>* u;    // [Mb] (IP)
  Cx<R>* fac;  // [Mb+1] (IP)
  int* misc;
};

template <typename R>
__device__ __forceinline__ BinLds<R> carve(unsigned char* base, const IterLds& L) {
  BinLds<R> s;
  s.x = reinterpret_cast<Cx<R>*>(base + L.x);
  s.w = reinterpret_cast<Cx<R>*>(base + L.w);
  s.a = reinterpret_cast<R*>(base + L.a);
  s.lam = reinterpret_cast<R*>(base + L.lam);
  s.p = reinterpret_cast<R*>(base + L.p);
  s.b = reinterpret_cast<R*>(base + L.b);
  s.yb = reinterpret_cast<Cx<R>*>(base + L.yb);
  s.wb = reinterpret_cast<Cx<R>*>(base + L.wb);
  s.q = reinterpret_cast<Cx<R>*>(base + L.q);
  s.aug = reinterpret_cast<Cx<R>*>(base + L.aug);
  s.u = reinterpret_cast<Cx<R>*>(base + L.u);
  s.fac = reinterpret_cast<Cx<R>*>(base + L.fac);
  s.misc = reinterpret_cast<int*>(base + L.misc);
  return s;
}

// Stage 1: scaled b_f and W_f, the observation block and lambda into LDS.
template <typename R>
__device__ void load_bin(const IterArgs<R>& a, const BinLds<R>& s, int f) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int T = a.T, M = a.M, K = a.K, F = a.F, Mb = a.rm.Mb, N = a.rm.N;
  for (int i = tid; i < N * K; i += nthr) {
    const int n = i / K, k = i - n * K;
    R b = a.B[((size_t)n * F + f) * K + k];
    if (a.mu) {
      const R m = a.mu[a.rm.r0[n]];
      b = b / (m * m);
    }
    s.b[i] = b;
  }
  const Cx<R>* Wf = a.W + (size_t)f * Mb * Mb;
  for (int i = tid; i < Mb * Mb; i += nthr) {
    Cx<R> w = Wf[i];
    if (a.mu) {
      const R m = a.mu[i / Mb];
      w.x = w.x / m;
      w.y = w.y / m;
    }
    s.w[i] = w;
  }
  for (int i = tid; i < M * T; i += nthr) {
    const int m = i / T, t = i - m * T;
    s.x[i] = a.X[((size_t)m * F + f) * T + t];
  }
  __syncthreads();
  for (int i = tid; i < N * T; i += nthr) {
    const int n = i / T, t = i - n * T;
    const R* Vn = a.V + (size_t)n * K * T + t;
    R acc = 0;
    for (int k = 0; k < K; ++k) acc += s.b[n * K + k] * Vn[(size_t)k * T];
    s.lam[i] = acc;
  }
  __syncthreads();
}

// Stage 2: y_p[t] = sum_c W[p][c] xbar_c[t] for the lane's frames, and the
// row weights phi_p[t] = 1 / lambda_{n(p), t - l(p)} (0 for t < l(p)).
template <typename R, int G, int CPL>
__device__ __forceinline__ void demix_lane(const IterArgs<R>& a, const BinLds<R>& s, int p, int q,
                                           Cx<R> (&y)[CPL], R (&ph)[CPL]) {
  const int T = a.T, M = a.M, D = a.D, Mb = a.rm.Mb;
#pragma unroll
  for (int j = 0; j < CPL; ++j) y[j] = Cx<R>{R(0), R(0)};
  const Cx<R>* wrow = s.w + p * Mb;
  for (int d = 0; d < D; ++d) {
    for (int m = 0; m < M; ++m) {
      const Cx<R> w = wrow[d * M + m];
      const Cx<R>* xm = s.x + m * T;
#pragma unroll
      for (int j = 0; j < CPL; ++j) {
        const int t = q + G * j;
        if (t >= d && t < T) y[j] = cfma(w, xm[t - d], y[j]);
      }
    }
  }
  const int n = a.rm.src[p], l = a.rm.tap[p];
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    const int t = q + G * j;
    ph[j] = (t >= l && t < T) ? R(1) / s.lam[n * T + (t - l)] : R(0);
  }
}

// Stage 4: W_f out, |y|^2 -> LDS, row powers, tap-aligned powers, bases.
template <typename R, int G, int CPL>
__device__ void epilogue(const IterArgs<R>& a, const BinLds<R>& s, int f, int g, int q, const Cx<R> (&y)[CPL]) {
  const int T = a.T, Mb = a.rm.Mb, N = a.rm.N, K = a.K, F = a.F;
  const int tid = threadIdx.x, nthr = blockDim.x;
  __syncthreads();  // every read of the x / w region is over before |y|^2 overwrites it
  if (g < Mb) {
    R rs = 0;
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
      const int t = q + G * j;
      if (t < T) {
        const R v = cabs2(y[j]);
        s.a[g * T + t] = v;
        rs += v;
      }
    }
    rs = group_sum<G>(rs);
    if (q == 0) a.musq[(size_t)f * Mb + g] = rs;
  }
  __syncthreads();
  for (int i = tid; i < N * T; i += nthr) {
    const int n = i / T, t = i - n * T;
    const int r0 = a.rm.r0[n], L = a.rm.L[n];
    R acc = 0;
    for (int l = 0; l < L && t + l < T; ++l) acc += s.a[(r0 + l) * T + t + l];
    s.p[i] = acc;
    a.P[((size_t)n * F + f) * T + t] = acc;
    if (a.P0) a.P0[((size_t)n * F + f) * T + t] = s.a[r0 * T + t];
  }
  __syncthreads();
  // Eq. (17) with t' = t - l: num = sum_t' P v / lambda^2, den = sum_t' C v / lambda,
  // C_{n,t'} = #{l < L_n : t' + l < T}.  One (n, k) pair per group.
  const int ngroups = nthr / G;
  for (int nk = tid / G; nk < N * K; nk += ngroups) {
    const int n = nk / K, k = nk - n * K;
    const R* Vk = a.V + ((size_t)n * K + k) * T;
    const int L = a.rm.L[n];
    R num = 0, den = 0;
    for (int t = q; t < T; t += G) {
      const R il = R(1) / s.lam[n * T + t];
      const R v = Vk[t];
      const R c = (R)min(L, T - t);
      num += s.p[n * T + t] * v * il * il;
      den += c * v * il;
    }
    num = group_sum<G>(num);
    den = group_sum<G>(den);
    if (q == 0) {
      R bn = s.b[nk] * sqrt(num / den);
      if (!isfinite(bn)) latch(a.status, kFaultMu);
      bn = bn > a.floor ? bn : a.floor;
      a.B[((size_t)n * F + f) * K + k] = bn;
    }
  }
}

// ------------------------------------------------------------------ ISS
template <typename R, int G, int CPL>
__global__ void __launch_bounds__(iter_max_threads(sizeof(R), CPL)) k_iss(IterArgs<R> a, IterLds L) {
  extern __shared__ __align__(16) unsigned char smem[];
  const BinLds<R> s = carve<R>(smem, L);
  const int f = blockIdx.x, tid = threadIdx.x;
  const int g = tid / G, q = tid - g * G;
  const int T = a.T, Mb = a.rm.Mb;
  constexpr int WPL = (kMaxRows + G - 1) / G;

  load_bin(a, s, f);

  Cx<R> y[CPL];
  R ph[CPL];
  Cx<R> wreg[WPL];
  const bool active = g < Mb;
  if (active) {
    demix_lane<R, G, CPL>(a, s, g, q, y, ph);
#pragma unroll
    for (int i = 0; i < WPL; ++i) {
      const int c = q + G * i;
      wreg[i] = c < Mb ? s.w[g * Mb + c] : Cx<R>{R(0), R(0)};
    }
  } else {
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
      y[j] = Cx<R>{R(0), R(0)};
      ph[j] = R(0);
    }
#pragma unroll
    for (int i = 0; i < WPL; ++i) wreg[i] = Cx<R>{R(0), R(0)};
  }

  // ISS sweep: for each r, a_p = sum_t phi_p y_p conj(y_r), d_p = sum_t phi_p |y_r|^2
  // (the common 1/T cancels in a_p / d_p), z_p = a_p / d_p, z_r = 1 - (d_r / T)^{-1/2};
  // then y_p -= z_p y_r and W[p, :] -= z_p W[r, :] with the pre-update row r.
  const R invT = R(1) / R(T);
  for (int r = 0; r < Mb; ++r) {
    Cx<R>* yb = s.yb + (r & 1) * T;
    Cx<R>* wb = s.wb + (r & 1) * Mb;
    if (g == r) {
#pragma unroll
      for (int j = 0; j < CPL; ++j) {
        const int t = q + G * j;
        if (t < T) yb[t] = y[j];
      }
#pragma unroll
      for (int i = 0; i < WPL; ++i) {
        const int c = q + G * i;
        if (c < Mb) wb[c] = wreg[i];
      }
    }
    __syncthreads();
    if (active) {
      Cx<R> yr[CPL];
      R ar = 0, ai = 0, dd = 0;
#pragma unroll
      for (int j = 0; j < CPL; ++j) {
        const int t = q + G * j;
        yr[j] = t < T ? yb[t] : Cx<R>{R(0), R(0)};
        const Cx<R> sv = cmulc(y[j], yr[j]);
        ar += ph[j] * sv.x;
        ai += ph[j] * sv.y;
        dd += ph[j] * cabs2(yr[j]);
      }
      ar = group_sum<G>(ar);
      ai = group_sum<G>(ai);
      dd = group_sum<G>(dd);
      Cx<R> z;
      if (g == r) {
        const R dr = dd * invT;
        if (!finite_pos(dr)) latch(a.status, kFaultIssDenominator);
        z = Cx<R>{R(1) - R(1) / sqrt(dr), R(0)};
      } else {
        if (!finite_pos(dd)) latch(a.status, kFaultIssDenominator);
        z = Cx<R>{ar / dd, ai / dd};
      }
#pragma unroll
      for (int j = 0; j < CPL; ++j) y[j] = cfms(z, yr[j], y[j]);
#pragma unroll
      for (int i = 0; i < WPL; ++i) {
        const int c = q + G * i;
        if (c < Mb) wreg[i] = cfms(z, wb[c], wreg[i]);
      }
    }
  }

  if (active) {
#pragma unroll
    for (int i = 0; i < WPL; ++i) {
      const int c = q + G * i;
      if (c < Mb) a.W[((size_t)f * Mb + g) * Mb + c] = wreg[i];
    }
  }
  epilogue<R, G, CPL>(a, s, f, g, q, y);
}

// ------------------------------------------------------------------ IP
// Solves A u = rhs for the n x n system stored as the n x (n+1) augmented
// matrix A (row-major, LDS) by Gaussian elimination with partial pivoting.
template <typename R>
__device__ void solve_augmented(Cx<R>* A, Cx<R>* u, Cx<R>* fac, int* misc, int n, int* status) {
  const int tid = threadIdx.x, nthr = blockDim.x, ld = n + 1;
  for (int k = 0; k < n; ++k) {
    if (tid == 0) {
      int piv = k;
      R best = cabs2(A[k * ld + k]);
      for (int i = k + 1; i < n; ++i) {
        const R v = cabs2(A[i * ld + k]);
        if (v > best) {
          best = v;
          piv = i;
        }
      }
      if (!finite_pos(best)) latch(status, kFaultIpSingular);
      misc[0] = piv;
    }
    __syncthreads();
    const int piv = misc[0];
    if (piv != k) {
      for (int j = k + tid; j <= n; j += nthr) {
        const Cx<R> t = A[k * ld + j];
        A[k * ld + j] = A[piv * ld + j];
        A[piv * ld + j] = t;
      }
    }
    __syncthreads();
    const Cx<R> pv = A[k * ld + k];
    const R den = cabs2(pv);
    const Cx<R> inv{pv.x / den, -pv.y / den};
    for (int i = k + 1 + tid; i < n; i += nthr) fac[i] = cmul(A[i * ld + k], inv);
    __syncthreads();
    const int w = n - k;  // columns k+1 .. n
    for (int e = tid; e < (n - k - 1) * w; e += nthr) {
      const int i = k + 1 + e / w, j = k + 1 + e % w;
      A[i * ld + j] = cfms(fac[i], A[k * ld + j], A[i * ld + j]);
    }
    __syncthreads();
  }
  if (tid == 0) {
    for (int i = n - 1; i >= 0; --i) {
      Cx<R> acc = A[i * ld + n];
      for (int j = i + 1; j < n; ++j) acc = cfms(A[i * ld + j], u[j], acc);
      const Cx<R> pv = A[i * ld + i];
      const R den = cabs2(pv);
      u[i] = Cx<R>{(acc.x * pv.x + acc.y * pv.y) / den, (acc.y * pv.x - acc.x * pv.y) / den};
    }
  }
  __syncthreads();
}

template <typename R, int G, int CPL>
__global__ void __launch_bounds__(iter_max_threads(sizeof(R), CPL)) k_ip(IterArgs<R> a, IterLds L) {
  extern __shared__ __align__(16) unsigned char smem[];
  const BinLds<R> s = carve<R>(smem, L);
  const int f = blockIdx.x, tid = threadIdx.x, nthr = blockDim.x;
  const int g = tid / G, q = tid - g * G;
  const int T = a.T, M = a.M, Mb = a.rm.Mb;
  const R invT = R(1) / R(T);

  load_bin(a, s, f);

  for (int r = 0; r < Mb; ++r) {
    const int n = a.rm.src[r], l = a.rm.tap[r];
    // weights of row r (s.p is free until the epilogue)
    for (int t = tid; t < T; t += nthr) s.p[t] = t >= l ? R(1) / s.lam[n * T + (t - l)] : R(0);
    __syncthreads();
    // Q_r = (1/T) sum_t phi_r xbar xbar^H, Eq. (8): upper triangle, mirrored.
    for (int e = tid; e < Mb * Mb; e += nthr) {
      const int i = e / Mb, j = e - (e / Mb) * Mb;
      if (i > j) continue;
      const int di = i / M, mi = i - di * M, dj = j / M, mj = j - dj * M;
      int t0 = di > dj ? di : dj;
      t0 = t0 > l ? t0 : l;
      R accx = 0, accy = 0;
      const Cx<R>* xi = s.x + mi * T - di;
      const Cx<R>* xj = s.x + mj * T - dj;
      for (int t = t0; t < T; ++t) {
        const Cx<R> pr = cmulc(xi[t], xj[t]);
        accx += s.p[t] * pr.x;
        accy += s.p[t] * pr.y;
      }
      s.q[i * Mb + j] = Cx<R>{accx * invT, accy * invT};
      if (i != j) s.q[j * Mb + i] = Cx<R>{accx * invT, -accy * invT};
    }
    __syncthreads();
    // [W Q_r | e_r]
    for (int e = tid; e < Mb * Mb; e += nthr) {
      const int i = e / Mb, j = e - (e / Mb) * Mb;
      Cx<R> acc{R(0), R(0)};
      for (int k = 0; k < Mb; ++k) acc = cfma(s.w[i * Mb + k], s.q[k * Mb + j], acc);
      s.aug[i * (Mb + 1) + j] = acc;
    }
    for (int i = tid; i < Mb; i += nthr) s.aug[i * (Mb + 1) + Mb] = Cx<R>{R(i == r ? 1 : 0), R(0)};
    __syncthreads();
    // u = (W Q_r)^{-1} e_r, Eq. (9)
    solve_augmented(s.aug, s.u, s.fac, s.misc, Mb, a.status);
    // u <- u (u^H Q_r u)^{-1/2}, Eq. (10); row r of W becomes u^H
    for (int i = tid; i < Mb; i += nthr) {
      Cx<R> acc{R(0), R(0)};
      for (int j = 0; j < Mb; ++j) acc = cfma(s.q[i * Mb + j], s.u[j], acc);
      s.fac[i] = cmulc(acc, s.u[i]);  // conj(u_i) (Q u)_i
    }
    __syncthreads();
    if (tid == 0) {
      R sum = 0;
      for (int i = 0; i < Mb; ++i) sum += s.fac[i].x;
      if (!finite_pos(sum)) latch(a.status, kFaultIpSingular);
      s.fac[Mb].x = R(1) / sqrt(sum);
    }
    __syncthreads();
    const R sc = s.fac[Mb].x;
    for (int c = tid; c < Mb; c += nthr) s.w[r * Mb + c] = Cx<R>{s.u[c].x * sc, -s.u[c].y * sc};
    __syncthreads();
  }

  // W_f out, then y = W xbar of the final W for the shared epilogue.
  for (int i = tid; i < Mb * Mb; i += nthr) a.W[(size_t)f * Mb * Mb + i] = s.w[i];
  Cx<R> y[CPL];
  R ph[CPL];
  if (g < Mb) {
    demix_lane<R, G, CPL>(a, s, g, q, y, ph);
  } else {
#pragma unroll
    for (int j = 0; j < CPL; ++j) y[j] = Cx<R>{R(0), R(0)};
  }
  epilogue<R, G, CPL>(a, s, f, g, q, y);
}

}  // namespace ctfiss
