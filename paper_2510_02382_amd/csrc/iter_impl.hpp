// W-update kernels of one CTF-MNMF iteration: one workgroup per frequency bin.
//
// Each workgroup
//   1. applies the pending scale of the previous iteration to W_f (Eqs. (19)-(21)),
//      stages the observation block (zero-padded so that stacked delayed frames
//      need no bounds tests) and the inverse source variances 1/lambda_{n,f,t}
//      (precomputed by k_lambda) in LDS;
//   2. demixes, y = W_f xbar (Eq. (4)), into registers;
//   3. runs the W update: the ISS sweep (Eqs. (11), (16)) or the IP sweep
//      (Eqs. (9), (10));
//   4. writes W_f, the tap-aligned powers P_{n,f,t'} = sum_l |y_{(n,l),f,t'+l}|^2
//      (and the tap-0 power for the PAPER_TAP0 rule), and the row power sums
//      used by the scale of Eq. (19).
//
// Register layout of the demixed signals: the workgroup is split into groups
// of G lanes; group g owns rows p = g*RPL + i (i < RPL) and lane q of the group
// holds frames t = q + G*j (j < CPL) of each.  Frame reductions are G-lane DPP
// butterflies; each ISS step needs one LDS broadcast of y_r and one barrier.
// The weight of row p = (n, l) at frame t is phi[n][t - l], read from the
// per-source inverse-variance row in LDS (zero before the first frame).
#pragma once

#include "common.hpp"

namespace ctfiss {

template <typename R>
struct IterArgs {
  const Cx<R>* X;   // [M][F][T] observation
  Cx<R>* W;         // [F][Mb][Mb] demixing matrices (in/out)
  const R* ilam;    // [N][F][T] 1 / lambda
  R* P;             // [N][F][T] tap-aligned power (out)
  R* P0;            // [N][F][T] tap-0 power (out, PAPER_TAP0) or null
  R* musq;          // [Mb][F] row power sums (out)
  const R* mu;      // [Mb] scale of the previous iteration still to apply to W, or null
  int* status;
  int* work;        // bin counter of the persistent workgroups (zeroed before the launch)
  Cx<R>* Y;         // [F][Mb][T] demixed rows carried between iterations (ISS), or null
  int yload;        // 1: start from the carried Y (rows scaled by the pending mu), 0: Y = W xbar
  unsigned long long* xch;  // team launches: [F][team_words] exchange words, else null
  unsigned epoch;           // team launches: tag base of this launch's exchange words
  // Kernels with the NMF steps folded in (single-workgroup ISS): 1/lambda formed per
  // bin from b and v instead of read from ilam, and the basis update of Eq. (17) done
  // per bin after the sweep
  R* B;             // [N][F][K] bases (in/out there)
  const R* V;       // [N][K][T] activations (read there)
  R floor;          // factor floor of the basis update
  int F, T, M, D, K;
  RowMap rm;
};

template <typename R>
struct BinLds {
  Cx<R>* x;    // [M][LX]  x[m][D-1 + t] = X[m][f][t], zero elsewhere
  Cx<R>* w;    // [Mb][Mb]
  R* phi;      // [N][LP]  phi[n][Lmax-1 + t] = 1/lambda_{n,f,t} for t < T, zero elsewhere
  Cx<R>* yb;   // [2][TP]  broadcast of y_r
  Cx<R>* wb;   // [2][Mb]  broadcast of w_r^H
  Cx<R>* q;    // [Mb][Mb]  (IP)
  Cx<R>* aug;  // [Mb][Mb+1] (IP)
  Cx<R>* u;    // [Mb] (IP)
  Cx<R>* fac;  // [Mb+1] (IP)
  R* a;        // [Mb][TA] |y|^2 after the sweep (reuses the bytes above)
  unsigned* xv;  // team: gathered exchange payloads
  R* bs;       // fused: [N][K] b_{n,f,k} of the bin with the pending scale applied
  R* pw;       // fused: [N][T] tap-aligned powers of the bin
  R* vl;       // fused: [N][K][T] the activations (loaded once per launch)
  int* misc;
};

template <typename R>
__device__ __forceinline__ BinLds<R> carve(unsigned char* base, const IterLds& L) {
  BinLds<R> s;
  s.x = reinterpret_cast<Cx<R>*>(base + L.x);
  s.w = reinterpret_cast<Cx<R>*>(base + L.w);
  s.phi = reinterpret_cast<R*>(base + L.phi);
  s.yb = reinterpret_cast<Cx<R>*>(base + L.yb);
  s.wb = reinterpret_cast<Cx<R>*>(base + L.wb);
  s.q = reinterpret_cast<Cx<R>*>(base + L.q);
  s.aug = reinterpret_cast<Cx<R>*>(base + L.aug);
  s.u = reinterpret_cast<Cx<R>*>(base + L.u);
  s.fac = reinterpret_cast<Cx<R>*>(base + L.fac);
  s.a = reinterpret_cast<R*>(base + L.a);
  s.xv = reinterpret_cast<unsigned*>(base + L.xv);
  s.bs = reinterpret_cast<R*>(base + L.bs);
  s.pw = reinterpret_cast<R*>(base + L.pw);
  s.vl = reinterpret_cast<R*>(base + L.vl);
  s.misc = reinterpret_cast<int*>(base + L.misc);
  return s;
}

// Fast reciprocal / reciprocal square root: hardware v_rcp / v_rsq (1 ulp) in
// FP32, IEEE division and square root in FP64.
__device__ __forceinline__ float fast_rcp(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double fast_rcp(double v) { return 1.0 / v; }
__device__ __forceinline__ float fast_rsqrt(float v) { return __builtin_amdgcn_rsqf(v); }
__device__ __forceinline__ double fast_rsqrt(double v) { return 1.0 / sqrt(v); }

// Lane index hidden from the optimiser: values derived from it (frame and
// row masks, LDS offsets) are then recomputed per bin instead of being hoisted
// out of the persistent bin loop and held in registers across it.
__device__ __forceinline__ int lane_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}
// Same for a workgroup-uniform size used as a divisor: the division's
// reciprocal is then formed per bin rather than kept live across the loop.
__device__ __forceinline__ int per_bin(int v) {
  v = __builtin_amdgcn_readfirstlane(v);  // uniform by construction
  asm volatile("" : "+s"(v));
  return v;
}

// Copies n elements from global memory into LDS.  Where a thread has several
// elements, U loads are in flight per thread before their stores: a workgroup
// then waits for one memory round trip per U elements per thread instead of
// one per element, which is what bounds a bin's start-up when a workgroup
// holds few rows and long weight rows.  (n and nthr are uniform.)
template <int U, typename V, typename Ld, typename St>
__device__ __forceinline__ void stage_lds(int n, int tid, int nthr, Ld ld, St st) {
  if (U > 1 && n > nthr) {
    for (int i0 = tid; i0 < n; i0 += nthr * U) {
      V v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + u * nthr;
        if (i < n) v[u] = ld(i);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + u * nthr;
        if (i < n) st(i, v[u]);
      }
    }
  } else {
    for (int i = tid; i < n; i += nthr) st(i, ld(i));
  }
}

// Stage 1: scaled W_f, zero-padded observation block and inverse variances into LDS.
// The frames staged start at t0 (a team member's first frame; 0 otherwise).
// U: loads in flight per thread (1 where the caller's registers are scarce).
template <int U, typename R, bool NMF = false>
__device__ void load_bin(const IterArgs<R>& a, const BinLds<R>& s, const IterLds& L, int f, int tid,
                         bool need_x, int t0 = 0) {
  const int nthr = blockDim.x;
  const int T = a.T, M = a.M, F = a.F, Mb = per_bin(a.rm.Mb), N = a.rm.N;
  const int LX = per_bin(L.lx), LP = per_bin(L.lp), Dm1 = a.D - 1, Lm1 = L.lmax - 1;
  const Cx<R>* Wf = a.W + (size_t)f * Mb * Mb;
  stage_lds<U, Cx<R>>(
      Mb * Mb, tid, nthr,
      [&](int i) {
        Cx<R> w = Wf[i];
        if (a.mu) {  // rows times 1/mu (as k_apply_mu scales them)
          const R rm = R(1) / a.mu[i / Mb];
          w.x = w.x * rm;
          w.y = w.y * rm;
        }
        return w;
      },
      [&](int i, Cx<R> w) { s.w[i] = w; });
  stage_lds<U, Cx<R>>(
      need_x ? M * LX : 0, tid, nthr,
      [&](int i) {
        const int m = i / LX, t = i - m * LX - Dm1 + t0;
        return (t >= 0 && t < T) ? a.X[((size_t)m * F + f) * T + t] : Cx<R>{R(0), R(0)};
      },
      [&](int i, Cx<R> v) { s.x[i] = v; });
  if constexpr (NMF) {
    // b of the bin with the pending scale applied (as the basis update and lambda = b v
    // apply it); phi's frames are formed after the barrier, its padding cleared here
    const int K = a.K;
    for (int i = tid; i < N * K; i += nthr) {
      const int n = i / K;
      R sc = R(1);
      if (a.mu) {
        const R m = a.mu[a.rm.r0[n]];
        sc = R(1) / (m * m);
      }
      s.bs[i] = a.B[((size_t)n * F + f) * K + (i - n * K)] * sc;
    }
    for (int i = tid; i < N * LP; i += nthr) {
      const int n = i / LP, t = i - n * LP - Lm1;
      if (t < 0 || t >= T) s.phi[i] = R(0);
    }
  } else {
    stage_lds<U, R>(
        N * LP, tid, nthr,
        [&](int i) {
          const int n = i / LP, t = i - n * LP - Lm1 + t0;
          return (t >= 0 && t < T) ? a.ilam[((size_t)n * F + f) * T + t] : R(0);
        },
        [&](int i, R v) { s.phi[i] = v; });
  }
  __syncthreads();
}

// Fused: phi[n][Lmax-1 + t] = 1 / lambda_{n,f,t}, lambda = sum_k b v (Sec. II), from the
// staged b and the activations (the same for every bin): held in LDS, or read from
// device memory (VG; the launch's L2 keeps them).  Ends with a barrier.
template <typename R, bool VG>
__device__ __forceinline__ void form_phi_v(const IterArgs<R>& a, const BinLds<R>& s, const IterLds& L, int tid) {
  const int T = a.T, K = a.K, N = a.rm.N, nthr = blockDim.x, LP = L.lp, Lm1 = L.lmax - 1;
  bool bad = false;
  for (int i = tid; i < N * T; i += nthr) {
    const int n = i / T, t = i - n * T;
    const R* b = s.bs + n * K;
    R lam = R(0);
    if constexpr (VG) {
      const R* v = a.V + (size_t)n * K * T + t;
#pragma unroll 8
      for (int k = 0; k < K; ++k) lam += b[k] * v[(size_t)k * T];
    } else {
      const R* v = s.vl + (size_t)n * K * T + t;
      for (int k = 0; k < K; ++k) lam += b[k] * v[k * T];
    }
    bad |= !finite_pos(lam);
    s.phi[n * LP + Lm1 + t] = R(1) / lam;
  }
  latch_wave(a.status, bad, kFaultMu);
  __syncthreads();
}
template <typename R>
__device__ void form_phi(const IterArgs<R>& a, const BinLds<R>& s, const IterLds& L, int tid) {
  if (L.vg)
    form_phi_v<R, true>(a, s, L, tid);
  else
    form_phi_v<R, false>(a, s, L, tid);
}

// Fused: the basis update of Eq. (17) for bin f with t' = t - l,
//   num_k = sum_t' P_{t'} v_{k,t'} / lambda_{t'}^2,  den_k = sum_t' C_{t'} v_{k,t'} / lambda_{t'},
//   C_{t'} = #{l < L_n : t' + l < T};  b <- max(b sqrt(num / den), floor)
// (b with the pending scale, as staged).  Each (n, k) takes a group of S = 64, 32
// or 16 lanes (the largest with every pair in one pass where possible); lane j adds
// frames j, j + S, ..., and the group's sums are one DPP butterfly.  Starts with a
// barrier (pw written).
template <typename R, int S, bool VG>
__device__ __forceinline__ bool b_update_groups(const IterArgs<R>& a, const BinLds<R>& s, const IterLds& L, int f,
                                                int tid) {
  const int T = a.T, K = a.K, N = a.rm.N, F = a.F, nthr = blockDim.x, LP = L.lp, Lm1 = L.lmax - 1;
  const int NK = N * K, total = NK * S;
  bool bad = false;
  for (int o0 = 0; o0 < total; o0 += nthr) {  // the same trip count for every thread
    const int o = o0 + tid, nk = o / S, j = o - nk * S;
    const bool act = o < total;
    R num = R(0), den = R(0);
    if (act) {
      const int n = nk / K, Ln = a.rm.L[n];
      const R* ph = s.phi + n * LP + Lm1;
      const R* pw = s.pw + n * T;
      auto frame = [&](int t, R vv) {
        const R il = ph[t];
        num += pw[t] * il * il * vv;
        den += (R)(Ln < T - t ? Ln : T - t) * il * vv;
      };
      if constexpr (VG) {  // device-memory loads: several in flight (the sums keep their order)
        const R* v = a.V + (size_t)nk * T;
#pragma unroll 8
        for (int t = j; t < T; t += S) frame(t, v[t]);
      } else {
        const R* v = s.vl + (size_t)nk * T;
        for (int t = j; t < T; t += S) frame(t, v[t]);
      }
    }
    num = group_sum<S>(num);
    den = group_sum<S>(den);
    if (act && j == 0) {
      const int n = nk / K;
      const R b = s.bs[nk] * sqrt(num / den);
      bad |= !isfinite(b);
      a.B[((size_t)n * F + f) * K + (nk - n * K)] = b > a.floor ? b : a.floor;
    }
  }
  return bad;
}

template <typename R, bool VG>
__device__ __forceinline__ bool b_update_v(const IterArgs<R>& a, const BinLds<R>& s, const IterLds& L, int f,
                                           int tid) {
  const int NK = a.rm.N * a.K, nthr = blockDim.x;
  if (NK * 64 <= nthr) return b_update_groups<R, 64, VG>(a, s, L, f, tid);
  if (NK * 32 <= nthr) return b_update_groups<R, 32, VG>(a, s, L, f, tid);
  return b_update_groups<R, 16, VG>(a, s, L, f, tid);
}
template <typename R>
__device__ void b_update(const IterArgs<R>& a, const BinLds<R>& s, const IterLds& L, int f, int tid) {
  __syncthreads();
  const bool bad = L.vg ? b_update_v<R, true>(a, s, L, f, tid) : b_update_v<R, false>(a, s, L, f, tid);
  latch_wave(a.status, bad, kFaultMu);
}

// Stage 2: y_p[t] = sum_c W[p][c] xbar_c[t] for the lane's rows and frames.
template <typename R, int G, int CPL, int RPL>
__device__ __forceinline__ void demix_lane(const IterArgs<R>& a, const BinLds<R>& s, const IterLds& L, int g,
                                           int q, Cx<R> (&y)[RPL][CPL], int nloc) {
  const int M = per_bin(a.M), D = a.D, Mb = a.rm.Mb, LX = L.lx, Dm1 = D - 1;
#pragma unroll
  for (int i = 0; i < RPL; ++i)
#pragma unroll
    for (int j = 0; j < CPL; ++j) y[i][j] = Cx<R>{R(0), R(0)};
  // xbar_c[t] = x[m][D-1 + t - d] for c = d*M + m; two columns per trip so the
  // LDS loads of one overlap the FMAs of the other.
  const int nc = D * M;
#pragma unroll 2
  for (int c = 0; c < nc; ++c) {
    const int d = c / M, m = c - d * M;
    Cx<R> w[RPL];
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int p = g * RPL + i;
      w[i] = p < Mb ? s.w[p * Mb + c] : Cx<R>{R(0), R(0)};
    }
    const Cx<R>* xm = s.x + m * LX + Dm1 - d + q;
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
      const Cx<R> xv = xm[G * j];
#pragma unroll
      for (int i = 0; i < RPL; ++i) y[i][j] = cfma(w[i], xv, y[i][j]);
    }
  }
  // Padded frames (past T, or past a team member's slice): a delayed block
  // still reads real frames there, so clear them; the rank-1 updates keep them
  // zero and they add nothing to the frame sums.
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    if (q + G * j >= nloc) {
#pragma unroll
      for (int i = 0; i < RPL; ++i) y[i][j] = Cx<R>{R(0), R(0)};
    }
  }
}

// Stage 2 (carried): the lane's rows and frames of the stored Y, times the reciprocal
// of the pending row scale exactly as W is in load_bin; zero for t >= T.
template <typename R, int G, int CPL, int RPL>
__device__ __forceinline__ void load_rows(const IterArgs<R>& a, int f, int g, int q, Cx<R> (&y)[RPL][CPL],
                                          int t0, int nloc) {
  const int T = a.T, Mb = a.rm.Mb;
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int p = g * RPL + i;
    const bool ok = p < Mb;
    const R rm = (ok && a.mu) ? R(1) / a.mu[p] : R(1);  // one reciprocal per row
    const Cx<R>* yr = a.Y + ((size_t)f * Mb + (ok ? p : 0)) * T + t0 + q;
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
      Cx<R> v = (ok && q + G * j < nloc) ? yr[G * j] : Cx<R>{R(0), R(0)};
      if (a.mu) {
        v.x = v.x * rm;
        v.y = v.y * rm;
      }
      y[i][j] = v;
    }
  }
}

// Stage 4: |y|^2 row sums and rows into LDS, then the tap-aligned powers
// P_n[t] = sum_{l < L_n, t + l < T} |y_{(n,l)}[t + l]|^2 summed in tap order
// (bitwise reproducible), P / P0 out.  Starts with a barrier: the |y|^2 rows
// overwrite the sweep's LDS buffers.
template <typename R, int G, int CPL, int RPL, bool NMF = false>
__device__ void epilogue(const IterArgs<R>& a, const BinLds<R>& s, const IterLds& L, int f, int tid, int g,
                         int q, const Cx<R> (&y)[RPL][CPL]) {
  const int T = per_bin(a.T), Mb = a.rm.Mb, N = a.rm.N, F = a.F, TP = L.tp;
  const int nthr = blockDim.x;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int p = g * RPL + i;
    R rs = 0;
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
      const R v = cabs2(y[i][j]);
      rs += v;
      if (p < Mb) s.a[p * TP + q + G * j] = v;
    }
    rs = group_sum<G>(rs);
    if (p < Mb && q == 0) a.musq[(size_t)p * F + f] = rs;
  }
  __syncthreads();
  for (int i = tid; i < N * T; i += nthr) {
    const int n = i / T, t = i - n * T;
    const int r0 = a.rm.r0[n], Ln = a.rm.L[n];
    const R* ar = s.a + r0 * TP + t;
    R acc = 0;
    for (int l = 0; l < Ln && t + l < T; ++l) acc += ar[l * TP + l];
    const size_t o = ((size_t)n * F + f) * T + t;
    a.P[o] = acc;
    if (a.P0) a.P0[o] = ar[0];
    if constexpr (NMF) s.pw[i] = acc;
  }
}

// Orders the LDS accesses of one wave (its lanes then see each other's writes).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------ teams
// A bin whose Mbar rows x T frames do not fit the registers of one workgroup
// is split by frames over a team of P workgroups: member j holds frames
// [j S, min(T, (j + 1) S)) of every row and its own copy of W_f.  The frame
// sums of an ISS step are then partial per member: each member publishes the
// partial sums of its rows in exchange words of its bin and gathers those of
// all members, adding them in member order, so that every member takes the
// same steps bit for bit.  An exchange word holds a 32-bit tag (launch epoch
// and step) and a 32-bit payload, stored and loaded as one relaxed
// device-scope 64-bit atomic: a reader that sees the expected tag has the
// matching payload, and no fences are needed.  The words of consecutive steps
// alternate between two slots; no member gets two steps ahead of another,
// since it waits for that member's sums of the step in between.
//
// Members claim (bin, member) items in order from the work counter, so the
// members of a bin are all running once P workgroups are resident, and every
// wait ends.  Each wait is bounded all the same: past kTeamSpin polls, or once
// another fault is latched, it stops and the launch completes with
// kFaultTeamWait latched.
constexpr int kTeamSpin = 1 << 20;

__device__ __forceinline__ void xput(unsigned long long* w, unsigned tag, unsigned payload) {
  __hip_atomic_store(w, ((unsigned long long)tag << 32) | payload, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename R>
__device__ __forceinline__ void xput_val(unsigned long long* w, unsigned tag, R v) {
  if constexpr (sizeof(R) == 4) {
    xput(w, tag, __float_as_uint(v));
  } else {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    xput(w, tag, (unsigned)b);
    xput(w + 1, tag, (unsigned)(b >> 32));
  }
}
// Value k of gathered payloads (an FP64 value spans two words, low half first).
template <typename R>
__device__ __forceinline__ R xval(const unsigned* v, int k) {
  if constexpr (sizeof(R) == 4)
    return __uint_as_float(v[k]);
  else
    return __hiloint2double((int)v[2 * k + 1], (int)v[2 * k]);
}

// Wave-wide wait: word k (< KW) of a lane is src[idx[k]] (idx < 0: none);
// once it carries `tag`, its payload goes to *dst[k].  Every lane of the wave
// must call it.  Returns false if it stopped before all words arrived: past
// kTeamSpin polls (then it latches kFaultTeamWait itself) or once another
// fault is latched.
template <int KW>
__device__ bool xgather(const unsigned long long* src, const int (&idx)[KW], unsigned* const (&dst)[KW],
                        unsigned tag, int* status) {
  unsigned pend = 0;
#pragma unroll
  for (int k = 0; k < KW; ++k)
    if (idx[k] >= 0) pend |= 1u << k;
  for (int spin = 0;; ++spin) {
#pragma unroll
    for (int k = 0; k < KW; ++k) {
      if (pend & (1u << k)) {
        const unsigned long long w = __hip_atomic_load(src + idx[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((unsigned)(w >> 32) == tag) {
          *dst[k] = (unsigned)w;
          pend &= ~(1u << k);
        }
      }
    }
    if (!__any(pend != 0)) return true;
    if (spin >= kTeamSpin) {  // latched at once: the team's other waits then stop within 64 polls
      if ((threadIdx.x & 63) == 0) latch(status, kFaultTeamWait);
      return false;
    }
    if ((spin & 63) == 63 && __hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    __builtin_amdgcn_s_sleep(2);
  }
}

// One ISS step's exchange: publish this member's partial (a_p, d_p) of the
// group's rows, gather every member's and replace the partials by the totals.
template <typename R, int G, int RPL>
__device__ __forceinline__ bool team_step_sums(const IterArgs<R>& a, const BinLds<R>& s, const IterLds& L,
                                               unsigned long long* xb, int mem, int r, int g, int q, R (&ar)[RPL],
                                               R (&ai)[RPL], R (&dd)[RPL]) {
  constexpr int WPV = sizeof(R) / 4;
  constexpr int KW = (RPL * 3 * kMaxTeam * WPV + G - 1) / G;
  const int Mb = a.rm.Mb, P = L.team;
  const unsigned tag = a.epoch * 128u + (unsigned)r;
  unsigned long long* xs = xb + (size_t)(r & 1) * (team_step_words(Mb, P, sizeof(R)) / 2);
  if (q < 3 * RPL) {
    const int i = q / 3, c = q - 3 * i;
    R v = R(0);
#pragma unroll
    for (int ii = 0; ii < RPL; ++ii)
      if (ii == i) v = c == 0 ? ar[ii] : (c == 1 ? ai[ii] : dd[ii]);
    const int p = g * RPL + i;
    if (p < Mb) xput_val<R>(xs + ((size_t)(p * 3 + c) * P + mem) * WPV, tag, v);
  }
  const int per_row = 3 * P * WPV, w0 = g * RPL * per_row;
  int idx[KW];
  unsigned* dst[KW];
#pragma unroll
  for (int k = 0; k < KW; ++k) {
    const int e = q + G * k;
    const bool ok = e < RPL * per_row && g * RPL + e / per_row < Mb;
    idx[k] = ok ? w0 + e : -1;
    dst[k] = s.xv + (ok ? w0 + e : 0);
  }
  const bool ok = xgather<KW>(xs, idx, dst, tag, a.status);
  wave_sync();  // a group's lanes lie in one wave
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int p = g * RPL + i;
    R t[3] = {R(0), R(0), R(0)};
    if (p < Mb) {
      for (int c = 0; c < 3; ++c)
        for (int m = 0; m < P; ++m) t[c] += xval<R>(s.xv, (p * 3 + c) * P + m);
    }
    ar[i] = t[0];
    ai[i] = t[1];
    dd[i] = t[2];
  }
  return ok;
}

// Stage 4 of a team member: as epilogue(), with the tap-aligned powers of the
// member's last frames taking |y|^2 of the next member's first Lmax - 1 frames
// (exchanged), and the row powers summed over members in member order (by
// member 0).
template <typename R, int G, int CPL, int RPL>
__device__ bool epilogue_team(const IterArgs<R>& a, const BinLds<R>& s, const IterLds& L, int f, int mem, int t0,
                              int nloc, int tid, int g, int q, const Cx<R> (&y)[RPL][CPL], unsigned long long* xb) {
  constexpr int WPV = sizeof(R) / 4;
  constexpr int KW = 4;
  const int T = per_bin(a.T), Mb = a.rm.Mb, N = a.rm.N, F = a.F, TA = L.ta, P = L.team, S = L.slice;
  const int H = L.lmax - 1, nthr = blockDim.x;
  const unsigned tag = a.epoch * 128u + 127u;
  unsigned long long* xh = xb + team_step_words(Mb, P, sizeof(R));
  unsigned long long* xm = xh + team_halo_words(Mb, L.lmax, P, sizeof(R));
  bool ok = true;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int p = g * RPL + i;
    R rs = 0;
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
      const R v = cabs2(y[i][j]);
      rs += v;
      if (p < Mb) s.a[p * TA + q + G * j] = v;
    }
    rs = group_sum<G>(rs);
    if (p < Mb && q == 0) xput_val<R>(xm + ((size_t)p * P + mem) * WPV, tag, rs);
  }
  __syncthreads();
  if (mem > 0) {  // my first H frames: the halo of the previous member
    for (int e = tid; e < Mb * H; e += nthr) {
      const int p = e / H, h = e - p * H;
      xput_val<R>(xh + ((size_t)(mem * Mb + p) * H + h) * WPV, tag, s.a[p * TA + h]);
    }
  }
  if (mem + 1 < P) {  // the next member's first H frames follow my S frames
    const int nw = Mb * H * WPV;
    const unsigned long long* src = xh + (size_t)(mem + 1) * Mb * H * WPV;
    for (int e0 = 0; e0 < nw; e0 += nthr * KW) {
      int idx[KW];
      unsigned* dst[KW];
#pragma unroll
      for (int k = 0; k < KW; ++k) {
        const int e = e0 + tid + nthr * k;
        const bool in = e < nw;
        const int v = e / WPV, half = e - v * WPV, p = v / (H > 0 ? H : 1), h = v - p * H;
        idx[k] = in ? e : -1;
        dst[k] = reinterpret_cast<unsigned*>(s.a + (in ? p * TA + S + h : 0)) + (in ? half : 0);
      }
      ok &= xgather<KW>(src, idx, dst, tag, a.status);
    }
  }
  if (mem == 0) {  // every member's row powers
    const int nw = Mb * P * WPV;
    for (int e0 = 0; e0 < nw; e0 += nthr * KW) {
      int idx[KW];
      unsigned* dst[KW];
#pragma unroll
      for (int k = 0; k < KW; ++k) {
        const int e = e0 + tid + nthr * k;
        idx[k] = e < nw ? e : -1;
        dst[k] = s.xv + (e < nw ? e : 0);
      }
      ok &= xgather<KW>(xm, idx, dst, tag, a.status);
    }
  }
  __syncthreads();
  if (mem == 0) {
    for (int p = tid; p < Mb; p += nthr) {
      R acc = 0;
      for (int m = 0; m < P; ++m) acc += xval<R>(s.xv, p * P + m);
      a.musq[(size_t)p * F + f] = acc;
    }
  }
  for (int i = tid; i < N * nloc; i += nthr) {
    const int n = i / nloc, tl = i - n * nloc, t = t0 + tl;
    const int r0 = a.rm.r0[n], Ln = a.rm.L[n];
    const R* ar = s.a + r0 * TA + tl;
    R acc = 0;
    for (int l = 0; l < Ln && t + l < T; ++l) acc += ar[l * TA + l];
    const size_t o = ((size_t)n * F + f) * T + t;
    a.P[o] = acc;
    if (a.P0) a.P0[o] = ar[0];
  }
  return ok;
}

// ------------------------------------------------------------------ ISS
// TEAM: the workgroup is member `mem` of the bin's team (frames
// [t0, t0 + nloc)); otherwise it holds all T frames.
// WX: the rows of W are updated in FP64 registers during the sweep (R =
// float): its 64 rank-1 updates per iteration then add no FP32 rounding to W,
// which is loaded from and stored to the FP32 state once per iteration.
template <typename R, int G, int CPL, int RPL, bool TEAM = false, bool WX = false, bool NMF = false>
__device__ void iss_bin(const IterArgs<R>& a, const BinLds<R>& s, const IterLds& L, int f, int mem = 0) {
  using WR = typename std::conditional<WX, double, R>::type;
  const int tid = lane_tid();
  const int g = tid / G, q = tid - g * G;
  const int T = a.T, Mb = a.rm.Mb, TP = L.tp, LP = L.lp, Lm1 = L.lmax - 1;
  constexpr int WPL = (kMaxRows + G - 1) / G;
  const int t0 = TEAM ? mem * L.slice : 0;
  const int nloc = TEAM ? (T - t0 < L.slice ? T - t0 : L.slice) : T;
  unsigned long long* xb = TEAM ? a.xch + (size_t)f * team_words(Mb, L.lmax, L.team, sizeof(R)) : nullptr;
  bool wait_ok = true;

  // Y = W xbar equals the previous iteration's Y with rows divided by mu: the
  // sweep applies the same rank-1 steps to W and Y, and the rescale divides the
  // rows of both.  Carrying it replaces the demix contraction (Mbar^2 complex
  // MACs per frame) by one read and one write of Y.  A workgroup of at most
  // four waves (a few rows: its bin's latency is not hidden by other waves)
  // requests its rows before the staging loads, so that both share one round
  // trip, where the rows are short enough to stay in registers meanwhile.
  constexpr bool kRowsFirst = CPL * RPL * sizeof(R) <= 80;
  const bool rows_first = kRowsFirst && a.yload && blockDim.x <= 256;
  Cx<R> y[RPL][CPL];
  if (rows_first) load_rows<R, G, CPL, RPL>(a, f, g, q, y, t0, nloc);
  load_bin<kRowsFirst ? 32 / sizeof(R) : 1, R, NMF>(a, s, L, f, tid, !a.yload, t0);
  if constexpr (NMF) form_phi<R>(a, s, L, tid);
  if (a.yload && !rows_first) load_rows<R, G, CPL, RPL>(a, f, g, q, y, t0, nloc);
  if (!a.yload) demix_lane<R, G, CPL, RPL>(a, s, L, g, q, y, nloc);

  Cx<WR> wreg[RPL][WPL];
  // Weights of the lane's rows and frames, phi[n][t - l]: held in registers, or, for
  // long rows (>= 24 frames per lane, whose registers the demixed rows need), read
  // from LDS in every step (rows past Mbar then read row 0's weights: their y stays
  // zero and nothing of them is stored).
  constexpr bool kPhiLds = CPL >= 24;
  R ph[RPL][kPhiLds ? 1 : CPL];
  const R* phl[RPL];
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int p = g * RPL + i;
    const bool ok = p < Mb;
    const R* phr = s.phi + (ok ? a.rm.src[p] * LP + Lm1 - a.rm.tap[p] : Lm1) + q;
    phl[i] = phr;
    if constexpr (!kPhiLds) {
#pragma unroll
      for (int j = 0; j < CPL; ++j) ph[i][j] = ok ? phr[G * j] : R(0);
    }
#pragma unroll
    for (int k = 0; k < WPL; ++k) {
      const int c = q + G * k;
      const Cx<R> w0 = (ok && c < Mb) ? s.w[p * Mb + c] : Cx<R>{R(0), R(0)};
      wreg[i][k] = Cx<WR>{WR(w0.x), WR(w0.y)};
    }
  }

  // ISS sweep over r: a_p = sum_t phi_p y_p conj(y_r), d_p = sum_t phi_p |y_r|^2
  // (the common 1/T cancels in a_p / d_p), z_p = a_p / d_p, z_r = 1 - (d_r / T)^{-1/2};
  // then y_p -= z_p y_r and W[p, :] -= z_p W[r, :] with the pre-update row r.
  const R invT = R(1) / R(per_bin(T));
  bool bad = false;
  for (int r = 0; r < Mb; ++r) {
    Cx<R>* yb = s.yb + (r & 1) * TP;
    Cx<WR>* wb = reinterpret_cast<Cx<WR>*>(s.wb) + (r & 1) * Mb;
    if (g == r / RPL) {
      const int io = r - g * RPL;
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        if (i == io) {
#pragma unroll
          for (int j = 0; j < CPL; ++j) yb[q + G * j] = y[i][j];
#pragma unroll
          for (int k = 0; k < WPL; ++k) {
            const int c = q + G * k;
            if (c < Mb) wb[c] = wreg[i][k];
          }
        }
      }
    }
    __syncthreads();
    R ar[RPL], ai[RPL], dd[RPL];
#pragma unroll
    for (int i = 0; i < RPL; ++i) ar[i] = ai[i] = dd[i] = R(0);
    Cx<R> yr[CPL];
#pragma unroll
    for (int j = 0; j < CPL; ++j) yr[j] = yb[q + G * j];
    // With t = phi_p y_r: a_p += y_p conj(t) and d_p += Re(t conj(y_r)), eight
    // FMA-class operations per row and frame.
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const R phv = kPhiLds ? phl[i][G * j] : ph[i][kPhiLds ? 0 : j];
        const R tx = phv * yr[j].x, ty = phv * yr[j].y;
        ar[i] += y[i][j].x * tx;
        ar[i] += y[i][j].y * ty;
        ai[i] += y[i][j].y * tx;
        ai[i] -= y[i][j].x * ty;
        dd[i] += tx * yr[j].x;
        dd[i] += ty * yr[j].y;
      }
    }
    // z_p from the row's frame sums
    auto coef = [&](int i) {
      const int p = g * RPL + i;
      if (p == r) {
        const R dr = dd[i] * invT;
        bad |= !finite_pos(dr);
        return Cx<R>{R(1) - fast_rsqrt(dr), R(0)};
      }
      bad |= p < Mb && !finite_pos(dd[i]);
      const R inv = fast_rcp(dd[i]);
      return Cx<R>{ar[i] * inv, ai[i] * inv};
    };
    Cx<R> z[RPL];
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      ar[i] = group_sum<G>(ar[i]);
      ai[i] = group_sum<G>(ai[i]);
      dd[i] = group_sum<G>(dd[i]);
      if constexpr (!TEAM) z[i] = coef(i);
    }
    if constexpr (TEAM) {  // the partial sums of every member, added in member order
      wait_ok &= team_step_sums<R, G, RPL>(a, s, L, xb, mem, r, g, q, ar, ai, dd);
#pragma unroll
      for (int i = 0; i < RPL; ++i) z[i] = coef(i);
    }
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
#pragma unroll
      for (int i = 0; i < RPL; ++i) y[i][j] = cfms(z[i], yr[j], y[i][j]);
    }
#pragma unroll
    for (int k = 0; k < WPL; ++k) {
      const int c = q + G * k;
      if (c < Mb) {
        const Cx<WR> wr = wb[c];
#pragma unroll
        for (int i = 0; i < RPL; ++i) wreg[i][k] = cfms(Cx<WR>{WR(z[i].x), WR(z[i].y)}, wr, wreg[i][k]);
      }
    }
  }

  latch_wave(a.status, bad, kFaultIssDenominator);
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int p = g * RPL + i;
#pragma unroll
    for (int k = 0; k < WPL; ++k) {
      const int c = q + G * k;
      if (p < Mb && c < Mb && (!TEAM || mem == 0))
        a.W[((size_t)f * Mb + p) * Mb + c] = Cx<R>{R(wreg[i][k].x), R(wreg[i][k].y)};
    }
    if (a.Y && p < Mb) {
      Cx<R>* yr = a.Y + ((size_t)f * Mb + p) * T + t0 + q;
#pragma unroll
      for (int j = 0; j < CPL; ++j)
        if (q + G * j < nloc) yr[G * j] = y[i][j];
    }
  }
  if constexpr (TEAM) {
    wait_ok &= epilogue_team<R, G, CPL, RPL>(a, s, L, f, mem, t0, nloc, tid, g, q, y, xb);
    latch_wave(a.status, !wait_ok, kFaultTeamWait);
  } else {
    epilogue<R, G, CPL, RPL, NMF>(a, s, L, f, tid, g, q, y);
    if constexpr (NMF) b_update<R>(a, s, L, f, tid);
  }
}

// Work counter of the persistent launches that claim their items in order:
// the team launch (a bin's members must be claimed together) and the IP
// sweep.  (k_iss deals its bins round-robin; the batched launch has its own
// counter.)
template <typename R>
__device__ __forceinline__ int next_bin(const IterArgs<R>& a, const BinLds<R>& s) {
  __syncthreads();  // the previous bin's LDS traffic is over
  if (threadIdx.x == 0) s.misc[0] = atomicAdd(a.work, 1);
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(s.misc[0]);  // uniform: bin addressing stays scalar
}

// NMF: the bins also form 1/lambda and update b (single-workgroup plans that fit).
template <typename R, int G, int CPL, int RPL, bool WX = false, bool NMF = false>
__global__ void __launch_bounds__(iter_max_threads(sizeof(R), CPL, RPL), iter_min_waves(sizeof(R), CPL, RPL))
    k_iss(IterArgs<R> a, IterLds L) {
  extern __shared__ __align__(16) unsigned char smem[];
  const BinLds<R> s = carve<R>(smem, L);
  // fused: the activations, the same for every bin, into LDS once (the first bin's
  // staging barrier orders these stores before their first use), unless read from
  // device memory where they are used (L.vg)
  if constexpr (NMF)
    stage_lds<32 / sizeof(R), R>(
        L.vg ? 0 : a.rm.N * a.K * a.T, threadIdx.x, blockDim.x, [&](int i) { return a.V[i]; },
        [&](int i, R v) { s.vl[i] = v; });
  // Bins dealt out round-robin over the resident workgroups: every bin costs
  // the same, so this balances as well as a shared counter would, without a
  // device-scope atomic round trip per bin.
  for (int f = blockIdx.x; f < a.F; f += gridDim.x) {
    if (f != (int)blockIdx.x) __syncthreads();  // the previous bin's LDS traffic is over
    iss_bin<R, G, CPL, RPL, false, WX, NMF>(a, s, L, f);
  }
}

// Team launch: the persistent workgroups take (bin, member) items in order,
// item = bin * P + member.
template <typename R, int G, int CPL, int RPL, bool WX = false>
__global__ void __launch_bounds__(iter_max_threads(sizeof(R), CPL, RPL)) k_iss_team(IterArgs<R> a, IterLds L) {
  extern __shared__ __align__(16) unsigned char smem[];
  const BinLds<R> s = carve<R>(smem, L);
  const int P = L.team;
  for (int it = next_bin(a, s); it < a.F * P; it = next_bin(a, s)) {
    const int f = it / P;
    iss_bin<R, G, CPL, RPL, true, WX>(a, s, L, f, it - f * P);
  }
}

// Batched ISS: the persistent workgroups take (problem, bin) items from one
// counter over the bins of every problem of the launch (same launch shape);
// each bin is processed exactly as in the single-problem kernel.
template <typename R>
struct WDesc {
  IterArgs<R> a;
  IterLds L;
};

template <typename R, int G, int CPL, int RPL>
__global__ void __launch_bounds__(iter_max_threads(sizeof(R), CPL, RPL), iter_min_waves(sizeof(R), CPL, RPL))
    k_iss_batch(const WDesc<R>* __restrict__ d, const int* __restrict__ start, int nprob, int* work) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int claim;
  const int total = start[nprob];
  for (;;) {
    __syncthreads();  // the previous bin's LDS traffic is over
    if (threadIdx.x == 0) claim = atomicAdd(work, 1);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(claim);
    if (item >= total) break;
    const int m = __builtin_amdgcn_readfirstlane(find_problem(start, nprob, item));
    const WDesc<R>& D = d[m];
    iss_bin<R, G, CPL, RPL>(D.a, carve<R>(smem, D.L), D.L, item - start[m]);
  }
}

// ------------------------------------------------------------------ IP
// The update of Eqs. (9)-(10) for row r, u = (W Q_r)^{-1} e_r normalised by
// (u^H Q_r u)^{-1/2}, is evaluated as u = Q_r^{-1} h_r with h_r = W^{-1} e_r,
// and u^H Q_r u = h_r^H u (the same quantities in exact arithmetic).  Q_r
// does not depend on W, so the inverse weighted covariances of a run of rows
// of one source are formed and inverted together (one matrix per wave); H =
// W^{-1} is inverted once per bin and kept current across the sweep by the
// Sherman-Morrison update for a changed row of W.


template <typename R>
__device__ __forceinline__ Cx<R> crecip(Cx<R> v) {
  const R d = cabs2(v);
  return Cx<R>{v.x / d, -v.y / d};
}

// In-place Gauss-Jordan inversion of the n x n matrix A (LDS, row-major) by
// one wave; col is an n-vector of LDS scratch.  pivot: partial pivoting by
// row exchanges, undone as column exchanges at the end (perm: n ints of LDS);
// without it the matrix must be Hermitian positive definite (then every pivot
// is real and positive up to rounding).  Returns false on a non-positive or
// non-finite pivot.
template <typename R, bool PIVOT>
__device__ bool wave_invert(Cx<R>* A, Cx<R>* col, int* perm, int n) {
  const int lane = threadIdx.x & 63;
  bool ok = true;
  for (int k = 0; k < n; ++k) {
    if (PIVOT) {
      // argmax_{i >= k} |A[i][k]|^2, lowest index on ties
      R best = R(-1);
      int arg = k;
      for (int i0 = k; i0 < n; i0 += 64) {
        const int i = i0 + lane;
        R v = i < n ? cabs2(A[i * n + k]) : R(-1);
        int idx = i;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          const R ov = __shfl_xor(v, off);
          const int oi = __shfl_xor(idx, off);
          if (ov > v || (ov == v && oi < idx)) {
            v = ov;
            idx = oi;
          }
        }
        if (v > best) {
          best = v;
          arg = idx;
        }
      }
      ok &= finite_pos(best);
      if (lane == 0) perm[k] = arg;
      if (arg != k) {
        for (int j = lane; j < n; j += 64) {
          const Cx<R> t = A[k * n + j];
          A[k * n + j] = A[arg * n + j];
          A[arg * n + j] = t;
        }
      }
      wave_sync();
    }
    const Cx<R> piv = A[k * n + k];
    if (PIVOT)
      ok &= finite_pos(cabs2(piv));
    else
      ok &= finite_pos(piv.x);
    const Cx<R> p = crecip(piv);
    for (int i = lane; i < n; i += 64) col[i] = A[i * n + k];
    wave_sync();
    for (int j = lane; j < n; j += 64) A[k * n + j] = cmul(j == k ? Cx<R>{R(1), R(0)} : A[k * n + j], p);
    wave_sync();
    // lane: column j, rows [ib, ie) (two lanes per column when n <= 32); the
    // loads of 4 rows are issued before their stores, so a lane waits for LDS
    // once per 4 rows instead of once per entry.
    {
      const bool two = n <= 32;
      const int j = two ? (lane & 31) : lane, hn = two ? (n + 1) / 2 : n;
      const int ib = two ? (lane >> 5) * hn : 0, ie = ib + hn < n ? ib + hn : n;
      if (j < n) {
        const Cx<R> pr = A[k * n + j];
        for (int i0 = ib; i0 < ie; i0 += 4) {
          Cx<R> av[4], cv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int i = i0 + u < ie ? i0 + u : ie - 1;
            av[u] = A[i * n + j];
            cv[u] = col[i];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int i = i0 + u;
            if (i < ie && i != k) A[i * n + j] = cfms(cv[u], pr, j == k ? Cx<R>{R(0), R(0)} : av[u]);
          }
        }
      }
    }
    wave_sync();
  }
  if (PIVOT) {
    for (int k = n - 1; k >= 0; --k) {
      const int q = perm[k];
      if (q != k)
        for (int i = lane; i < n; i += 64) {
          const Cx<R> t = A[i * n + k];
          A[i * n + k] = A[i * n + q];
          A[i * n + q] = t;
        }
      wave_sync();
    }
  }
  return ok;
}

// Entry e (row-major upper triangle, i <= j) of the weighted covariances of
// rows c0 .. c0 + rc - 1 (taps) of source n, summed over frames [t0, t1):
// acc[c] = sum_t phi_n[t - (c0 + c)] xbar_i[t] conj(xbar_j[t]) (phi is zero for t < tap).
template <typename R>
__device__ __forceinline__ void ip_cov_entry(const IterArgs<R>& a, const BinLds<R>& s, const IterLds& L, int n,
                                             int c0, int rc, int e, int t0, int t1, int& i, int& j,
                                             Cx<R> (&acc)[ip_max_chunk(sizeof(R))]) {
  const int Mb = a.rm.Mb, M = a.M, LX = L.lx, Dm1 = a.D - 1;
  i = 0;
  while (e >= Mb - i) {
    e -= Mb - i;
    ++i;
  }
  j = i + e;
  const int di = i / M, mi = i - di * M, dj = j / M, mj = j - dj * M;
  const Cx<R>* xi = s.x + mi * LX + Dm1 - di;
  const Cx<R>* xj = s.x + mj * LX + Dm1 - dj;
  const R* ph = s.phi + n * L.lp + L.lmax - 1 - c0;  // ph[t - c] = phi_n[t - (c0 + c)]
#pragma unroll
  for (int c = 0; c < ip_max_chunk(sizeof(R)); ++c) acc[c] = Cx<R>{R(0), R(0)};
  constexpr int CM = ip_max_chunk(sizeof(R));
  if (rc == CM) {  // full run: constant offsets, no selects
    for (int t = t0; t < t1; ++t) {
      const Cx<R> pr = cmulc(xi[t], xj[t]);
      R w[CM];
#pragma unroll
      for (int c = 0; c < CM; ++c) w[c] = ph[t - c];
#pragma unroll
      for (int c = 0; c < CM; ++c) {
        acc[c].x += w[c] * pr.x;
        acc[c].y += w[c] * pr.y;
      }
    }
    return;
  }
  // Branch-free over the run: rows c >= rc read row rc - 1's weight (in range)
  // and add it times 0, so the weight loads of a frame are issued together.
  for (int t = t0; t < t1; ++t) {
    const Cx<R> pr = cmulc(xi[t], xj[t]);
    R w[ip_max_chunk(sizeof(R))];
#pragma unroll
    for (int c = 0; c < ip_max_chunk(sizeof(R)); ++c) w[c] = ph[t - (c < rc ? c : rc - 1)];
#pragma unroll
    for (int c = 0; c < ip_max_chunk(sizeof(R)); ++c) {
      const R wc = c < rc ? w[c] : R(0);
      acc[c].x += wc * pr.x;
      acc[c].y += wc * pr.y;
    }
  }
}

// Writes (add: adds to) entries (i, j) and (j, i) of the rc covariances, scaled by 1/T.
template <typename R>
__device__ __forceinline__ void ip_cov_store(const BinLds<R>& s, int Mb, int rc, int i, int j, bool add, R invT,
                                             const Cx<R> (&acc)[ip_max_chunk(sizeof(R))]) {
#pragma unroll
  for (int c = 0; c < ip_max_chunk(sizeof(R)); ++c) {
    if (c < rc) {
      Cx<R>* Q = s.q + (size_t)c * Mb * Mb;
      Cx<R> v{acc[c].x * invT, acc[c].y * invT};
      if (add) v = cadd(Q[i * Mb + j], v);  // frame ranges added in order
      Q[i * Mb + j] = v;
      if (i != j) Q[j * Mb + i] = Cx<R>{v.x, -v.y};
    }
  }
}

template <typename R, int G, int CPL, int RPL>
__device__ void ip_bin(const IterArgs<R>& a, const BinLds<R>& s, const IterLds& L, int f) {
  const int tid = lane_tid(), nthr = blockDim.x, wave = tid >> 6, lane = tid & 63, nwave = (nthr + 63) >> 6;
  const int g = tid / G, q = tid - g * G;
  const int T = per_bin(a.T), M = per_bin(a.M), Mb = per_bin(a.rm.Mb), LX = L.lx, LP = L.lp;
  const int Dm1 = a.D - 1, Lm1 = L.lmax - 1;
  const R invT = R(1) / R(T);
  Cx<R>* H = s.aug;                 // [Mb][Mb] W^{-1}
  Cx<R>* hv = s.u;                  // column r of H before its update
  Cx<R>* dv = s.u + Mb;             // new row r of W minus the old one
  Cx<R>* gv = s.u + 2 * Mb;         // dv^T H
  Cx<R>* colw = s.fac + wave * Mb;  // this wave's column scratch
  bool bad = false;

  load_bin<1>(a, s, L, f, tid, true);
  // H = W^{-1} (one wave, partial pivoting); the pivot order goes to the q region
  if (wave == 0) {
    for (int e = lane; e < Mb * Mb; e += 64) H[e] = s.w[e];
    wave_sync();
    bad |= !wave_invert<R, true>(H, colw, reinterpret_cast<int*>(s.q), Mb);
  }
  __syncthreads();

  const int U = Mb * (Mb + 1) / 2;
  int ts_n = nthr / U;
  ts_n = ts_n < 1 ? 1 : (ts_n > 4 ? 4 : ts_n);
  for (int n = 0; n < a.rm.N; ++n) {
    const int Ln = a.rm.L[n];
    for (int c0 = 0; c0 < Ln; c0 += L.rc) {
      const int rc = Ln - c0 < L.rc ? Ln - c0 : L.rc;
      // Q_{(n, c0 + c)}[i][j] = (1/T) sum_{t >= l} phi_n[t - l] xbar_i[t] conj(xbar_j[t]), l = c0 + c,
      // Eq. (8): one product xbar_i conj(xbar_j) per frame serves every row of the run.
      // ts_n > 1: thread tid < U ts_n takes entry tid % U over frame range tid / U, and
      // the ranges are added in order (every thread passes the same barriers);
      // ts_n = 1: threads loop over the entries.
      if (ts_n > 1) {
        const bool act = tid < U * ts_n;
        const int ts = act ? tid / U : 0, e = act ? tid - ts * U : 0;
        Cx<R> acc[ip_max_chunk(sizeof(R))];
        int i = 0, j = 0;
        if (act) ip_cov_entry<R>(a, s, L, n, c0, rc, e, ts * T / ts_n, (ts + 1) * T / ts_n, i, j, acc);
        for (int s2 = 0; s2 < ts_n; ++s2) {
          if (act && ts == s2) ip_cov_store<R>(s, Mb, rc, i, j, s2 > 0, invT, acc);
          __syncthreads();
        }
      } else {
        for (int e = tid; e < U; e += nthr) {
          Cx<R> acc[ip_max_chunk(sizeof(R))];
          int i = 0, j = 0;
          ip_cov_entry<R>(a, s, L, n, c0, rc, e, 0, T, i, j, acc);
          ip_cov_store<R>(s, Mb, rc, i, j, false, invT, acc);
        }
      }
      __syncthreads();
      // invert the rc weighted covariances, one per wave
      for (int c = wave; c < rc; c += nwave) bad |= !wave_invert<R, false>(s.q + (size_t)c * Mb * Mb, colw, nullptr, Mb);
      __syncthreads();

      for (int c = 0; c < rc; ++c) {
        const int r = a.rm.r0[n] + c0 + c;
        const Cx<R>* Qi = s.q + (size_t)c * Mb * Mb;
        if (wave == 0) {
          // u = Q_r^{-1} h_r, s = h_r^H u, new row r = conj(u) / sqrt(s)
          Cx<R> u{R(0), R(0)}, hr{R(0), R(0)};
          if (lane < Mb) {
            hr = H[lane * Mb + r];
            for (int k = 0; k < Mb; ++k) u = cfma(Qi[lane * Mb + k], H[k * Mb + r], u);
          }
          const R sp = lane < Mb ? hr.x * u.x + hr.y * u.y : R(0);  // Re(conj(h) u)
          const R sv = group_sum<64>(sp);
          bad |= !finite_pos(sv);
          const R rs = R(1) / sqrt(sv);
          if (lane < Mb) {
            const Cx<R> wn{u.x * rs, -u.y * rs};
            dv[lane] = csub(wn, s.w[r * Mb + lane]);
            hv[lane] = hr;
            s.w[r * Mb + lane] = wn;
          }
          wave_sync();
          // g = d^T H and the denominator 1 + g_r of the rank-one update of H
          if (lane < Mb) {
            Cx<R> gj{R(0), R(0)};
            for (int k = 0; k < Mb; ++k) gj = cfma(dv[k], H[k * Mb + lane], gj);
            gv[lane] = gj;
          }
          wave_sync();
        }
        __syncthreads();
        // H <- H - h_r g^T / (1 + g_r)
        const Cx<R> den = cadd(Cx<R>{R(1), R(0)}, gv[r]);
        bad |= !finite_pos(cabs2(den));
        const Cx<R> rden = crecip(den);
        for (int e = tid; e < Mb * Mb; e += nthr) {
          const int i = e / Mb, j = e - (e / Mb) * Mb;
          H[e] = cfms(cmul(hv[i], rden), gv[j], H[e]);
        }
        __syncthreads();
      }
    }
  }
  latch_wave(a.status, bad, kFaultIpSingular);

  // W_f out, then y = W xbar of the final W for the shared epilogue.
  for (int i = tid; i < Mb * Mb; i += nthr) a.W[(size_t)f * Mb * Mb + i] = s.w[i];
  Cx<R> y[RPL][CPL];
  demix_lane<R, G, CPL, RPL>(a, s, L, g, q, y, a.T);
  epilogue<R, G, CPL, RPL>(a, s, L, f, tid, g, q, y);
}

template <typename R, int G, int CPL, int RPL>
__global__ void __launch_bounds__(iter_max_threads(sizeof(R), CPL, RPL)) k_ip(IterArgs<R> a, IterLds L) {
  extern __shared__ __align__(16) unsigned char smem[];
  const BinLds<R> s = carve<R>(smem, L);
  for (int f = next_bin(a, s); f < a.F; f = next_bin(a, s)) ip_bin<R, G, CPL, RPL>(a, s, L, f);
}

}  // namespace ctfiss
