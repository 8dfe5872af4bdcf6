// NMF contractions on bfloat16 matrix cores (gfx950 v_mfma_f32_16x16x32_bf16):
// lambda = b v, the basis update of Eq. (17) and the activation partial sums of
// Eq. (18) / ALL_TAPS, with their operands rounded to bfloat16 (round to nearest
// even) and the products accumulated in FP32.  Everything around the
// contractions (1/lambda, the weights P / lambda^2 and C / lambda, the square
// roots, floors and faults) stays FP32, as in the FP32 kernels of nmf_impl.hpp,
// whose launch shapes these follow.
//
// Operand layout of the 16x16x32 instruction: lane l = 16 lq + lr holds
// A[lr][8 lq + i] and B[8 lq + i][lr] for i < 8, and the 16x16 FP32 result at
// rows 4 lq + v, column lr (as the 16x16x4 FP32 instruction).  A contraction
// only needs A's and B's slot i of lane block lq to carry the same index of the
// summed dimension; which index that is, is the kernel's choice.
#include "launch.hpp"
#include "nmf_impl.hpp"

namespace ctfiss {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x4 mfma_bf16(const float (&a)[8], const float (&b)[8], f32x4 c) {
  bf16x8 av, bv;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    av[i] = (__bf16)a[i];
    bv[i] = (__bf16)b[i];
  }
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
}

constexpr int kKB = kMaxK / 32;  // 32-wide steps over the bases

// 1/lambda with lambda = (b / mu^2) v: one 16 (bins) x 16 (frames) tile per wave, K/32
// steps.  Grid (ceil(T/64), ceil(F/16), N), 4 waves covering 64 frames.
__global__ void __launch_bounds__(256) k_lambda_bf16(NmfArgs<float> a) {
  const int T = a.T, K = a.K, F = a.F;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, lr = l & 15, lq = l >> 4;
  const int n = blockIdx.z, f0 = blockIdx.y * 16, t0 = blockIdx.x * 64 + wave * 16;
  if (a.work && blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0) *a.work = 0;
  if (t0 >= T) return;
  const float sc = pending_scale(a, n);
  const float* Bn = a.B + (size_t)n * F * K;
  const float* Vn = a.V + (size_t)n * K * T;
  const int fa = f0 + lr, tb = t0 + lr;
  f32x4 acc = acc_zero<float>();
#pragma unroll
  for (int s = 0; s < kKB; ++s) {
    if (32 * s >= K) break;
    float av[8], bv[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int k = 32 * s + 8 * lq + i;
      av[i] = (k < K && fa < F) ? Bn[(size_t)fa * K + k] * sc : 0.f;
      bv[i] = (k < K && tb < T) ? Vn[(size_t)k * T + tb] : 0.f;
    }
    acc = mfma_bf16(av, bv, acc);
  }
  bool bad = false;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int f = f0 + 4 * lq + v;
    if (f < F && tb < T) {
      const float lam = acc[v];
      bad |= !finite_pos(lam);
      a.ilam[((size_t)n * F + f) * T + tb] = 1.f / lam;
    }
  }
  latch_wave(a.status, bad, kFaultMu);
}

// Basis update, Eq. (17): num_{f,k} = sum_t' P v / lambda^2, den_{f,k} = sum_t' C v / lambda
// over frames, 32 frames per instruction; one workgroup per 16 bins, its waves split the
// frames and their tiles are summed in wave order.
__global__ void __launch_bounds__(1024) k_nmf_b_bf16(NmfArgs<float> a) {
  constexpr int KT = kMaxK / 16;
  __shared__ float red[2][KT][4][64];
  __shared__ float tiles[kMaxNmfWaves][4][64];
  const int T = a.T, K = a.K, F = a.F;
  const int wave = threadIdx.x >> 6, nwave = blockDim.x >> 6, l = threadIdx.x & 63, lr = l & 15, lq = l >> 4;
  const int n = blockIdx.y, f0 = blockIdx.x * 16;
  const int L = a.rm.L[n];
  const int nkt = (K + 15) / 16;
  const float* Pn = a.P + (size_t)n * F * T;
  const float* In = a.ilam + (size_t)n * F * T;
  const float* Vn = a.V + (size_t)n * K * T;
  const int fa = f0 + lr;
  f32x4 num[KT], den[KT];
#pragma unroll
  for (int kt = 0; kt < KT; ++kt) num[kt] = den[kt] = acc_zero<float>();
  for (int step = wave; 32 * step < T; step += nwave) {
    float e1[8], e2[8], bv[KT][8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int t = 32 * step + 8 * lq + i;
      e1[i] = e2[i] = 0.f;
      if (fa < F && t < T) {
        const float il = In[(size_t)fa * T + t];
        e1[i] = Pn[(size_t)fa * T + t] * il * il;
        e2[i] = (float)min(L, T - t) * il;
      }
#pragma unroll
      for (int kt = 0; kt < KT; ++kt) {
        const int k = 16 * kt + lr;
        bv[kt][i] = (kt < nkt && k < K && t < T) ? Vn[(size_t)k * T + t] : 0.f;
      }
    }
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) {
      if (kt < nkt) {
        num[kt] = mfma_bf16(e1, bv[kt], num[kt]);
        den[kt] = mfma_bf16(e2, bv[kt], den[kt]);
      }
    }
  }
  sum_wave_tiles<float, KT, kMaxNmfWaves>(num, den, nkt, nwave, tiles, red);
  if (wave != 0) return;
  const float sc = pending_scale(a, n);
  bool bad = false;
#pragma unroll
  for (int kt = 0; kt < KT; ++kt) {
    if (kt >= nkt) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int f = f0 + 4 * lq + v, k = 16 * kt + lr;
      if (f < F && k < K) {
        const size_t o = ((size_t)n * F + f) * K + k;
        const float b = a.B[o] * sc * sqrtf(red[0][kt][v][l] / red[1][kt][v][l]);
        bad |= !isfinite(b);
        a.B[o] = b > a.floor ? b : a.floor;
      }
    }
  }
  latch_wave(a.status, bad, kFaultMu);
}

// Activation partial sums over one chunk of 128 bins (4 waves x 32 bins):
//   num[k][t] = sum_f b P' / lambda^2,  den[k][t] = sum_f b / lambda,
// lambda = b v of the updated bases.  A wave forms lambda for its two 16-bin halves,
// the weights in the accumulator layout (lane: bins 4 lq + v of each half at frame lr),
// and contracts them with b over its 32 bins: slot i of lane block lq is bin 4 lq + i of
// the first half (i < 4) or 4 lq + i - 4 of the second, in both operands.
__global__ void __launch_bounds__(256) k_vpart_bf16(NmfArgs<float> a) {
  constexpr int KT = kMaxK / 16;
  __shared__ float red[2][KT][4][64];
  const int T = a.T, K = a.K, F = a.F;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, lr = l & 15, lq = l >> 4;
  const int n = blockIdx.z, ch = blockIdx.y, t0 = blockIdx.x * 16;
  const int f1 = min(F, ch * a.fchunk + a.fchunk);
  const int fs = ch * a.fchunk + 32 * wave;  // this wave's 32-bin subtile
  const int nkt = (K + 15) / 16;
  const float* Bn = a.B + (size_t)n * F * K;
  const float* Vn = a.V + (size_t)n * K * T;
  const float* Pn = (a.tap0 ? a.P0 : a.P) + (size_t)n * F * T;
  const int tb = t0 + lr;
  float e1[8], e2[8];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int fa = fs + 16 * h + lr;
    f32x4 lam = acc_zero<float>();
#pragma unroll
    for (int s = 0; s < kKB; ++s) {
      if (32 * s >= K) break;
      float av[8], vop[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int k = 32 * s + 8 * lq + i;
        av[i] = (k < K && fa < f1) ? Bn[(size_t)fa * K + k] : 0.f;
        vop[i] = (k < K && tb < T) ? Vn[(size_t)k * T + tb] : 0.f;
      }
      lam = mfma_bf16(av, vop, lam);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int f = fs + 16 * h + 4 * lq + v;
      float x1 = 0.f, x2 = 0.f;
      if (f < f1 && tb < T) {
        const float il = 1.f / lam[v];
        x1 = Pn[(size_t)f * T + tb] * il * il;
        x2 = il;
      }
      e1[4 * h + v] = x1;
      e2[4 * h + v] = x2;
    }
  }
  f32x4 num[KT], den[KT];
#pragma unroll
  for (int kt = 0; kt < KT; ++kt) {
    num[kt] = den[kt] = acc_zero<float>();
    if (kt < nkt) {
      float bt[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int f = fs + (i < 4 ? 4 * lq + i : 16 + 4 * lq + i - 4), k = 16 * kt + lr;
        bt[i] = (f < f1 && k < K) ? Bn[(size_t)f * K + k] : 0.f;
      }
      num[kt] = mfma_bf16(bt, e1, num[kt]);
      den[kt] = mfma_bf16(bt, e2, den[kt]);
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
          red[0][kt][v][l] = (w == 0 ? 0.f : red[0][kt][v][l]) + num[kt][v];
          red[1][kt][v][l] = (w == 0 ? 0.f : red[1][kt][v][l]) + den[kt][v];
        }
      }
    }
    __syncthreads();
  }
  if (wave != 0 || tb >= T) return;
#pragma unroll
  for (int kt = 0; kt < KT; ++kt) {
    if (kt >= nkt) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int k = 16 * kt + 4 * lq + v;
      if (k < K) {
        const size_t o = (((size_t)n * a.nch + ch) * K + k) * T + tb;
        a.vnum[o] = red[0][kt][v][l];
        a.vden[o] = red[1][kt][v][l];
      }
    }
  }
}

NmfArgs<float> make_nargs_f(const Dims& d, const VSplit& vs, const Ptrs& ptr, double floor, bool tap0,
                            bool apply_mu) {
  NmfArgs<float> a;
  a.B = static_cast<float*>(ptr.B);
  a.V = static_cast<float*>(ptr.V);
  a.ilam = static_cast<float*>(ptr.ilam);
  a.P = static_cast<const float*>(ptr.P);
  a.P0 = static_cast<const float*>(ptr.P0);
  a.vnum = static_cast<float*>(ptr.vnum);
  a.vden = static_cast<float*>(ptr.vden);
  a.musq = static_cast<const float*>(ptr.musq);
  a.mu = static_cast<float*>(ptr.mu);
  a.mu_prev = apply_mu ? static_cast<const float*>(ptr.mu) : nullptr;
  a.status = ptr.status;
  a.work = ptr.work;
  a.F = d.F;
  a.T = d.T;
  a.K = d.K;
  a.nch = vs.nch;
  a.fchunk = vs.fchunk;
  a.tap0 = tap0 ? 1 : 0;
  a.floor = (float)floor;
  a.rm = d.rm;
  return a;
}

hipError_t lambda_bf16_t(const Dims& d, const Ptrs& ptr, bool apply_mu, hipStream_t s) {
  NmfArgs<float> a = make_nargs_f(d, VSplit{1, d.F}, ptr, 0.0, false, apply_mu);
  dim3 grid((d.T + 63) / 64, (d.F + 15) / 16, d.N);
  hipLaunchKernelGGL(k_lambda_bf16, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t nmfb_bf16_t(const Dims& d, const Ptrs& ptr, double floor, bool apply_mu, hipStream_t s) {
  NmfArgs<float> a = make_nargs_f(d, VSplit{1, d.F}, ptr, floor, false, apply_mu);
  int waves = (d.T + 31) / 32;  // one wave per 32 frames, at most 16 (they loop over longer signals)
  if (waves > kMaxNmfWaves) waves = kMaxNmfWaves;
  dim3 grid((d.F + 15) / 16, d.N);
  hipLaunchKernelGGL(k_nmf_b_bf16, grid, dim3(64 * waves), 0, s, a);
  return hipGetLastError();
}

hipError_t vpart_bf16_t(const Dims& d, const VSplit& vs, const Ptrs& ptr, bool tap0, hipStream_t s) {
  if (vs.fchunk != 128) return hipErrorInvalidValue;  // 4 waves x 32 bins
  NmfArgs<float> a = make_nargs_f(d, vs, ptr, 0.0, tap0, false);
  dim3 grid((d.T + 15) / 16, vs.nch, d.N);
  hipLaunchKernelGGL(k_vpart_bf16, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace ctfiss
