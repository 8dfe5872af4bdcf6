// Device-side building blocks shared by the CTF-MNMF kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <type_traits>

namespace ctfiss {

constexpr int kMaxRows = 64;   // Mbar
constexpr int kMaxSrc = 8;     // N
constexpr int kMaxK = 64;      // K
constexpr int kMaxNmfWaves = 16;  // waves of a basis-update workgroup
constexpr int kMaxTeam = 8;    // workgroups sharing the frames of one bin

// Device fault codes latched in the status word (first one wins).
enum Fault : int {
  kFaultNone = 0,
  kFaultIssDenominator = 1,  // ISS weighted power d_p not positive / not finite
  kFaultIpSingular = 2,      // IP system (W Q_r) singular or u^H Q u not positive
  kFaultMu = 3,              // multiplicative update produced a non-finite factor
  kFaultOutSingular = 4,     // W_f singular in the source-image stage
  kFaultScale = 5,           // zero or non-finite row power in the rescale
  kFaultTeamWait = 6,        // the workgroups of a bin did not all publish their sums in time
};

template <typename R>
struct alignas(2 * sizeof(R)) Cx {  // aligned to its size: one 64/128-bit access
  R x, y;
};

template <typename R>
__device__ __forceinline__ Cx<R> cadd(Cx<R> a, Cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ Cx<R> csub(Cx<R> a, Cx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ Cx<R> cmul(Cx<R> a, Cx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename R>
__device__ __forceinline__ Cx<R> cmulc(Cx<R> a, Cx<R> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
// acc + a * b
template <typename R>
__device__ __forceinline__ Cx<R> cfma(Cx<R> a, Cx<R> b, Cx<R> acc) {
  return {acc.x + a.x * b.x - a.y * b.y, acc.y + a.x * b.y + a.y * b.x};
}
// acc - a * b
template <typename R>
__device__ __forceinline__ Cx<R> cfms(Cx<R> a, Cx<R> b, Cx<R> acc) {
  return {acc.x - a.x * b.x + a.y * b.y, acc.y - a.x * b.y - a.y * b.x};
}
template <typename R>
__device__ __forceinline__ R cabs2(Cx<R> a) { return a.x * a.x + a.y * a.y; }

// Row map of the extended demixing matrix: row r is tap tap[r] of source src[r].
struct RowMap {
  int Mb, N;
  int r0[kMaxSrc];   // first row of each source
  int L[kMaxSrc];    // taps per source
  uint8_t src[kMaxRows];
  uint8_t tap[kMaxRows];
};

// ------------------------------------------------------------------ reductions
// Sum over aligned groups of G lanes (G = 16, 32 or 64); every lane of the
// group receives the total.  Within 16 lanes the butterfly uses DPP
// (quad_perm xor1, quad_perm xor2, row_half_mirror, row_mirror); across rows
// the gfx950 lane swaps (v_permlane16_swap: rows 0<->1 and 2<->3;
// v_permlane32_swap: the two halves of the wave), plain VALU operations with
// no trip through the LDS crossbar.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float v) { return dpp_f<CTRL>(v); }
template <int CTRL>
__device__ __forceinline__ double dpp(double v) { return dpp_d<CTRL>(v); }

// v of this lane plus v of the same lane in the partner row (W = 16: the other
// row of the row pair) or half (W = 32).  Swapping a register with itself
// leaves the lower row's (half's) value in the first result and the upper
// one's in the second on both sides, so both lanes form the same sum.
template <int W>
__device__ __forceinline__ unsigned swap_rows(unsigned& hi, unsigned v) {
  if constexpr (W == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    hi = r[1];
    return r[0];
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    hi = r[1];
    return r[0];
  }
}
template <int W>
__device__ __forceinline__ float add_rows(float v) {
  unsigned hi;
  const unsigned lo = swap_rows<W>(hi, __float_as_uint(v));
  return __uint_as_float(lo) + __uint_as_float(hi);
}
template <int W>
__device__ __forceinline__ double add_rows(double v) {
  unsigned hl, hh;
  const unsigned ll = swap_rows<W>(hl, (unsigned)__double2loint(v));
  const unsigned lh = swap_rows<W>(hh, (unsigned)__double2hiint(v));
  return __hiloint2double((int)lh, (int)ll) + __hiloint2double((int)hh, (int)hl);
}

template <int G, typename R>
__device__ __forceinline__ R group_sum(R v) {
  static_assert(G == 16 || G == 32 || G == 64, "group size");
  v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp<0x141>(v);  // row_half_mirror
  v += dpp<0x140>(v);  // row_mirror
  if constexpr (G >= 32) v = add_rows<16>(v);
  if constexpr (G >= 64) v = add_rows<32>(v);
  return v;
}

__device__ __forceinline__ void latch(int* status, int code) {
  if (status) atomicCAS(status, 0, code);
}

// One atomic per wave: the lowest lane whose flag is set latches the code.
__device__ __forceinline__ void latch_wave(int* status, bool bad, int code) {
  const unsigned long long m = __ballot(bad ? 1 : 0);
  if (m && (int)(threadIdx.x & 63) == __ffsll((long long)m) - 1) latch(status, code);
}

template <typename R>
__device__ __forceinline__ bool finite_pos(R v) {
  return v > R(0) && isfinite(v);  // false for NaN, 0, negatives, +inf
}

// Largest workgroup the W-update kernels are compiled for.  A lane holds RPL
// rows of CPL frames of y plus RPL rows of its W slice (2 reals per complex,
// doubled for FP64) and ~40 registers of addressing and scalars; a SIMD has
// 512 VGPRs per lane, so at most floor(512 / need) waves of the workgroup may
// share it, i.e. 256 * that many threads (4 SIMDs per CU).
__host__ __device__ constexpr int iter_need_vgprs(int rsize, int cpl, int rpl) {
  return rpl * (2 * cpl + 8) * (rsize / 4) + 40;
}
// Occupancy target of the ISS kernel (minimum waves per SIMD): FP32 with one
// row per lane group and at most 10 frames per lane fits in 80 VGPRs, so two
// 12-wave workgroups (G = 32) share a CU; elsewhere the launch bound decides.
__host__ __device__ constexpr int iter_min_waves(int rsize, int cpl, int rpl) {
  return (rsize == 4 && rpl == 1 && cpl <= 10) ? 6 : 1;
}
__host__ __device__ constexpr int iter_max_threads(int rsize, int cpl, int rpl) {
  return (512 / iter_need_vgprs(rsize, cpl, rpl)) * 256 > 1024 ? 1024
                                                                : (512 / iter_need_vgprs(rsize, cpl, rpl)) * 256;
}

// Batched launches: start[m] is the first work item (block or bin) of problem
// m, start[nprob] the total; an item finds its problem by binary search.
__device__ __forceinline__ int find_problem(const int* start, int nprob, int item) {
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= item)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------------------ LDS layout
// Per-bin on-chip layout of the W-update kernels (TP = G * CPL padded frames).
// During the sweep: x, w, phi, yb, wb (+ q, aug, u, fac for IP).  After it the
// per-row powers |y|^2, a[Mb][TP], reuse the same bytes from offset 0.
struct IterLds {
  size_t x, w, phi, yb, wb, q, aug, u, fac, a, xv, bs, pw, vl, misc, total;
  int lx, lp, tp, lmax;
  int rc;     // IP: rows whose inverse weighted covariances are held at once
  int team;   // workgroups per bin (1: a bin is one workgroup)
  int slice;  // frames per team member (T for a single workgroup)
  int ta;     // row stride of a (TP, plus the Lmax - 1 frames of the next member in a team)
  int kb;     // K when the kernel also forms 1/lambda and updates b per bin (0: it does not)
  int vg;     // kb > 0: the activations are read from device memory, not staged in vl
};

// Exchange words of one bin in a team launch (64-bit words, one 32-bit
// payload each, so an FP64 value takes two): the partial frame sums of the
// ISS steps, [2 (step parity)][Mb][3][P][wpv]; the |y|^2 of the first Lmax - 1
// frames of every member, [P][Mb][Lmax - 1][wpv]; the partial row powers,
// [Mb][P][wpv].
__host__ __device__ constexpr int team_step_words(int Mb, int P, int rsize) { return 2 * Mb * 3 * P * (rsize / 4); }
__host__ __device__ constexpr int team_halo_words(int Mb, int lmax, int P, int rsize) {
  return P * Mb * (lmax - 1) * (rsize / 4);
}
__host__ __device__ constexpr int team_words(int Mb, int lmax, int P, int rsize) {
  return team_step_words(Mb, P, rsize) + team_halo_words(Mb, lmax, P, rsize) + Mb * P * (rsize / 4);
}

// LDS one workgroup may use on gfx950.
constexpr size_t kMaxLdsBytes = 163840;
// Rows per run of inverse weighted covariances: their accumulators live in
// registers (6 complex doubles or 12 complex floats).
__host__ __device__ constexpr int ip_max_chunk(int rsize) { return rsize == 8 ? 6 : 12; }

__host__ __device__ inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// team > 1: the bin's frames are split over `team` workgroups of `slice`
// frames each (slice <= G * cpl); the layout is that of one member.
// kb > 0 (single-workgroup ISS): the kernel also forms 1/lambda from b and v and
// updates b per bin; then phi, the scaled bases bs [N][kb], the tap-aligned
// powers pw [N][T] and the activations vl [N][kb][T] (loaded once per launch;
// not with vg, where the kernel reads them from device memory) outlive the sweep
// (placed after the shared region).
__host__ __device__ inline IterLds iter_lds_layout(int M, int T, int D, int Mb, int N, int lmax, int G, int cpl,
                                                   int rsize, bool ip, int team = 1, int slice = 0, int kb = 0,
                                                   bool vg = false) {
  IterLds L{};
  const size_t cs = 2 * (size_t)rsize;
  L.tp = G * cpl;
  L.lx = D - 1 + L.tp;
  L.lp = lmax - 1 + L.tp;
  L.lmax = lmax;
  L.team = team > 1 ? team : 1;
  L.slice = team > 1 ? slice : T;
  L.ta = team > 1 ? L.tp + lmax - 1 : L.tp;
  L.kb = (!ip && L.team == 1) ? kb : 0;
  L.vg = (L.kb && vg) ? 1 : 0;
  size_t off = 0;
  L.x = off; off += align_up((size_t)M * L.lx * cs, 16);
  L.w = off; off += align_up((size_t)Mb * Mb * cs, 16);
  if (!L.kb) {
    L.phi = off; off += align_up((size_t)N * L.lp * rsize, 16);
  }
  if (!ip) {  // the ISS broadcasts of y_r and w_r (w_r held in FP64 by the mixed-precision sweep)
    L.yb = off; off += align_up((size_t)2 * L.tp * cs, 16);
    L.wb = off; off += align_up((size_t)2 * Mb * 16, 16);
  } else {
    L.yb = L.wb = 0;
  }
  if (ip) {
    // aug: H = W^{-1} [Mb][Mb]; u: four Mb-vectors; fac: one Mb column per
    // wave; q: rc matrices [Mb][Mb] (the inverse weighted covariances, and
    // the scratch of the first inversion), rc as large as LDS allows.
    const int waves = (Mb * G + 63) / 64;
    L.aug = off; off += align_up((size_t)Mb * Mb * cs, 16);
    L.u = off; off += align_up((size_t)4 * Mb * cs, 16);
    L.fac = off; off += align_up((size_t)waves * Mb * cs, 16);
    L.q = off;
    const size_t mat = align_up((size_t)Mb * Mb * cs, 16);
    const size_t room = kMaxLdsBytes > off + 64 ? kMaxLdsBytes - off - 64 : 0;  // 64: misc
    int rc = (int)(room / mat);
    if (rc > lmax) rc = lmax;
    if (rc > ip_max_chunk(rsize)) rc = ip_max_chunk(rsize);
    L.rc = rc < 1 ? 1 : rc;
    off += (size_t)L.rc * mat;
  } else {
    L.q = L.aug = L.u = L.fac = 0;
    L.rc = 0;
  }
  L.a = 0;
  const size_t asz = align_up((size_t)Mb * L.ta * rsize, 16);
  if (asz > off) off = asz;
  L.bs = L.pw = L.vl = 0;
  if (L.kb) {
    L.phi = off; off += align_up((size_t)N * L.lp * rsize, 16);
    L.bs = off; off += align_up((size_t)N * L.kb * rsize, 16);
    L.pw = off; off += align_up((size_t)N * T * rsize, 16);
    if (!L.vg) {
      L.vl = off;
      off += align_up((size_t)N * L.kb * T * rsize, 16);
    }
  }
  // team: 32-bit payloads of the exchange words a wave gathers (one step's
  // partial sums of every row; also the row powers of the epilogue)
  L.xv = off;
  if (L.team > 1) off += align_up((size_t)Mb * 3 * L.team * (rsize / 4) * 4, 16);
  L.misc = off; off += 64;
  L.total = off;
  return L;
}

}  // namespace ctfiss
