// Typed kernel launchers; included by exactly one translation unit per precision.
#pragma once

#include <cstring>

#include "iter_impl.hpp"
#include "launch.hpp"
#include "nmf_impl.hpp"
#include "out_impl.hpp"

namespace ctfiss {

template <typename R>
using WFn = void (*)(IterArgs<R>, IterLds);

// WX: ISS kernels with FP64 W rows (mixed precision, R = float; no IP kernels).
// nmf: the ISS kernel with the NMF steps folded in, instantiated for one row per
// lane group and at most 16 frames per lane (the plans of small Mbar and T ~ 250-500).
template <typename R, bool WX, int G, int CPL, int RPL>
WFn<R> wfn(int rule, bool nmf) {
  if (rule == 0) {
    if constexpr (RPL == 1 && CPL <= 16) {
      if (nmf) return &k_iss<R, G, CPL, RPL, WX, true>;
    }
    return nmf ? nullptr : &k_iss<R, G, CPL, RPL, WX>;
  }
  if constexpr (RPL == 1 && !WX) {
    if (!nmf) return &k_ip<R, G, CPL, 1>;
  }
  return nullptr;
}

template <typename R, bool WX, int G, int RPL>
WFn<R> pick_cpl(int rule, int cpl, bool nmf) {
  if constexpr (sizeof(R) == 4) {
    switch (cpl) {
      case 4: return wfn<R, WX, G, 4, RPL>(rule, nmf);
      case 8: return wfn<R, WX, G, 8, RPL>(rule, nmf);
      case 10: return wfn<R, WX, G, 10, RPL>(rule, nmf);
      case 12: return wfn<R, WX, G, 12, RPL>(rule, nmf);
      case 16: return wfn<R, WX, G, 16, RPL>(rule, nmf);
      case 20: return wfn<R, WX, G, 20, RPL>(rule, nmf);
      case 24: return wfn<R, WX, G, 24, RPL>(rule, nmf);
      case 28: return wfn<R, WX, G, 28, RPL>(rule, nmf);
      case 32: return wfn<R, WX, G, 32, RPL>(rule, nmf);
      default: return nullptr;
    }
  } else {
    switch (cpl) {
      case 4: return wfn<R, WX, G, 4, RPL>(rule, nmf);
      case 6: return wfn<R, WX, G, 6, RPL>(rule, nmf);
      case 8: return wfn<R, WX, G, 8, RPL>(rule, nmf);
      case 10: return wfn<R, WX, G, 10, RPL>(rule, nmf);
      case 12: return wfn<R, WX, G, 12, RPL>(rule, nmf);
      case 16: return wfn<R, WX, G, 16, RPL>(rule, nmf);
      default: return nullptr;
    }
  }
}

template <typename R, bool WX, int G>
WFn<R> pick_rpl(int rule, int cpl, int rpl, bool nmf) {
  if (rpl == 1) return pick_cpl<R, WX, G, 1>(rule, cpl, nmf);
  if (rpl == 2) return pick_cpl<R, WX, G, 2>(rule, cpl, nmf);
  return nullptr;
}

template <typename R, bool WX>
WFn<R> pick(int rule, int G, int cpl, int rpl, bool nmf = false) {
  if constexpr (WX && sizeof(R) != 4) return nullptr;
  if (G == 16) return pick_rpl<R, WX, 16>(rule, cpl, rpl, nmf);
  if (G == 32) return pick_rpl<R, WX, 32>(rule, cpl, rpl, nmf);
  if constexpr (sizeof(R) == 4) {
    if (G == 64 && rpl == 1) return pick_cpl<R, WX, 64, 1>(rule, cpl, nmf);  // long frames, Mbar <= 16
  }
  if constexpr (sizeof(R) == 8) {
    if (G == 64) return pick_rpl<R, WX, 64>(rule, cpl, rpl, nmf);
  }
  return nullptr;
}

template <typename R, bool WX>
bool have_wkernel(int rule, int G, int cpl, int rpl) {
  return pick<R, WX>(rule, G, cpl, rpl) != nullptr;
}

// Team (frame-split) ISS kernels: Mbar up to 64 with long signals.
template <typename R, bool WX>
WFn<R> pickt(int G, int cpl, int rpl) {
  if constexpr (sizeof(R) == 4) {
    if (G == 16 && rpl == 1 && cpl == 16) return &k_iss_team<R, 16, 16, 1, WX>;
    if (G == 16 && rpl == 1 && cpl == 8) return &k_iss_team<R, 16, 8, 1, WX>;
    if (G == 16 && rpl == 2 && cpl == 8) return &k_iss_team<R, 16, 8, 2, WX>;
    if (G == 32 && rpl == 2 && cpl == 8) return &k_iss_team<R, 32, 8, 2, WX>;
    if (G == 32 && rpl == 2 && cpl == 4) return &k_iss_team<R, 32, 4, 2, WX>;
  } else if constexpr (!WX) {
    if (G == 16 && rpl == 1 && cpl == 8) return &k_iss_team<R, 16, 8, 1>;
    if (G == 16 && rpl == 1 && cpl == 4) return &k_iss_team<R, 16, 4, 1>;
    if (G == 16 && rpl == 2 && cpl == 4) return &k_iss_team<R, 16, 4, 2>;
  }
  return nullptr;
}

template <typename R, bool WX>
bool have_tkernel(int G, int cpl, int rpl) {
  return pickt<R, WX>(G, cpl, rpl) != nullptr;
}

// FP64 ISS W update of 10-16 frames per lane in workgroups of at most 768 threads (e.g. 24
// rows of 32 lanes): the k_iss bin loop under a 768-thread launch bound, which lets the
// compiler keep the rows in up to 168 VGPRs where the 1024-thread bound of k_iss caps them
// at 128 and spills inside the ISS step loop; three waves per SIMD still fit, as under the
// 1024-thread bound.  Same arithmetic in the same order as k_iss.
template <typename R, int G, int CPL>
__global__ void __launch_bounds__(768) k_iss768(IterArgs<R> a, IterLds L) {
  extern __shared__ __align__(16) unsigned char smem[];
  const BinLds<R> s = carve<R>(smem, L);
  for (int f = blockIdx.x; f < a.F; f += gridDim.x) {
    if (f != (int)blockIdx.x) __syncthreads();  // the previous bin's LDS traffic is over
    iss_bin<R, G, CPL, 1>(a, s, L, f);
  }
}

template <typename R, bool WX>
WFn<R> pick_plan(int rule, const Plan& p) {
  if (p.team > 1) return (rule == 0 && !p.nmf) ? pickt<R, WX>(p.G, p.CPL, p.RPL) : nullptr;
  if constexpr (sizeof(R) == 8 && !WX) {
    if (rule == 0 && !p.nmf && p.RPL == 1 && p.threads <= 768 && (p.G == 32 || p.G == 64)) {
      const bool g32 = p.G == 32;
      if (p.CPL == 10) return g32 ? &k_iss768<R, 32, 10> : &k_iss768<R, 64, 10>;
      if (p.CPL == 12) return g32 ? &k_iss768<R, 32, 12> : &k_iss768<R, 64, 12>;
      if (p.CPL == 16) return g32 ? &k_iss768<R, 32, 16> : &k_iss768<R, 64, 16>;
    }
  }
  return pick<R, WX>(rule, p.G, p.CPL, p.RPL, p.nmf != 0);
}

// Workgroups of the W-update kernel that fit on the device at once.
template <typename R, bool WX>
int resident_wblocks(int rule, const Plan& p, const Dims& d) {
  WFn<R> fn = pick_plan<R, WX>(rule, p);
  int dev = 0, cus = 0, per_cu = 0;
  if (!fn || hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (p.lds > 65536 &&
      hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)fn, p.threads, p.lds) != hipSuccess) return 0;
  const long long n = (long long)per_cu * cus, items = (long long)d.F * (p.team > 1 ? p.team : 1);
  return n < 1 ? 0 : (int)(n < items ? n : items);
}

template <typename R>
IterArgs<R> make_iargs(int rule, const Dims& d, const Ptrs& ptr, bool apply_mu, bool yload, double floor = 0.0) {
  IterArgs<R> a;
  a.B = static_cast<R*>(ptr.B);
  a.V = static_cast<const R*>(ptr.V);
  a.floor = (R)floor;
  a.X = static_cast<const Cx<R>*>(ptr.X);
  a.W = static_cast<Cx<R>*>(ptr.W);
  a.ilam = static_cast<const R*>(ptr.ilam);
  a.P = static_cast<R*>(ptr.P);
  a.P0 = static_cast<R*>(ptr.P0);
  a.musq = static_cast<R*>(ptr.musq);
  a.mu = apply_mu ? static_cast<const R*>(ptr.mu) : nullptr;
  a.status = ptr.status;
  a.work = ptr.work;
  a.Y = rule == 0 ? static_cast<Cx<R>*>(ptr.Y) : nullptr;
  a.yload = (rule == 0 && yload) ? 1 : 0;
  a.xch = static_cast<unsigned long long*>(ptr.xch);
  a.epoch = 0;
  a.F = d.F;
  a.T = d.T;
  a.M = d.M;
  a.D = d.D;
  a.K = d.K;
  a.rm = d.rm;
  return a;
}

inline IterLds wlayout(int rule, const Plan& p, const Dims& d, int rsize) {
  const bool nmf = p.nmf && rule == 0 && p.team <= 1;
  return iter_lds_layout(d.M, d.T, d.D, d.Mb, d.N, d.lmax, p.G, p.CPL, rsize, rule != 0, p.team, p.slice,
                         nmf ? d.K : 0, nmf && p.nmf == 2);
}

template <typename R, bool WX>
hipError_t wupdate_t(int rule, const Plan& p, const Dims& d, const Ptrs& ptr, bool apply_mu, bool yload,
                     unsigned epoch, double floor, hipStream_t s) {
  WFn<R> fn = pick_plan<R, WX>(rule, p);
  if (!fn || (p.team > 1 && !ptr.xch)) return hipErrorInvalidValue;
  IterArgs<R> a = make_iargs<R>(rule, d, ptr, apply_mu, yload, floor);
  a.epoch = epoch;
  const IterLds L = wlayout(rule, p, d, (int)sizeof(R));
  if (L.total > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.total);
    if (e != hipSuccess) return e;
  }
  const int items = d.F * (p.team > 1 ? p.team : 1);
  hipLaunchKernelGGL(fn, dim3(p.blocks > 0 ? p.blocks : items), dim3(p.threads), L.total, s, a, L);
  return hipGetLastError();
}

template <typename R>
NmfArgs<R> make_nargs(const Dims& d, const VSplit& vs, const Ptrs& ptr, double floor, bool tap0, bool apply_mu) {
  NmfArgs<R> a;
  a.B = static_cast<R*>(ptr.B);
  a.V = static_cast<R*>(ptr.V);
  a.ilam = static_cast<R*>(ptr.ilam);
  a.P = static_cast<const R*>(ptr.P);
  a.P0 = static_cast<const R*>(ptr.P0);
  a.vnum = static_cast<R*>(ptr.vnum);
  a.vden = static_cast<R*>(ptr.vden);
  a.musq = static_cast<const R*>(ptr.musq);
  a.mu = static_cast<R*>(ptr.mu);
  a.mu_prev = apply_mu ? static_cast<const R*>(ptr.mu) : nullptr;
  a.status = ptr.status;
  a.work = ptr.work;
  a.F = d.F;
  a.T = d.T;
  a.K = d.K;
  a.nch = vs.nch;
  a.fchunk = vs.fchunk;
  a.tap0 = tap0 ? 1 : 0;
  a.floor = (R)floor;
  a.rm = d.rm;
  return a;
}

template <typename R>
hipError_t lambda_t(const Dims& d, const Ptrs& ptr, bool apply_mu, hipStream_t s) {
  NmfArgs<R> a = make_nargs<R>(d, VSplit{1, d.F}, ptr, 0.0, false, apply_mu);
  dim3 grid((d.T + 63) / 64, (d.F + 15) / 16, d.N);
  hipLaunchKernelGGL(k_lambda<R>, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename R>
hipError_t nmfb_t(const Dims& d, const Ptrs& ptr, double floor, bool apply_mu, hipStream_t s) {
  NmfArgs<R> a = make_nargs<R>(d, VSplit{1, d.F}, ptr, floor, false, apply_mu);
  // one wave per 32 (FP32) or 16 (FP64) frames, at most 16 waves (they loop over longer signals)
  const int fpw = sizeof(R) == 4 ? 32 : 16;
  int waves = (d.T + fpw - 1) / fpw;
  if (waves > kMaxNmfWaves) waves = kMaxNmfWaves;
  dim3 grid((d.F + 15) / 16, d.N);
  hipLaunchKernelGGL(k_nmf_b<R>, grid, dim3(64 * waves), 0, s, a);
  return hipGetLastError();
}

template <typename R>
hipError_t vpart_t(const Dims& d, const VSplit& vs, const Ptrs& ptr, bool tap0, hipStream_t s) {
  NmfArgs<R> a = make_nargs<R>(d, vs, ptr, 0.0, tap0, false);
  dim3 grid((d.T + 15) / 16, vs.nch, d.N);
  hipLaunchKernelGGL(k_vpart<R>, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename R>
hipError_t vfinal_t(const Dims& d, const VSplit& vs, const Ptrs& ptr, double floor, bool tap0, hipStream_t s) {
  NmfArgs<R> a = make_nargs<R>(d, vs, ptr, floor, tap0, false);
  const int nv = (d.N * d.K * d.T + 255) / 256;
  hipLaunchKernelGGL(k_vfinal<R>, dim3(nv + d.Mb), dim3(256), 0, s, a, nv);
  return hipGetLastError();
}

// One launch for the activation update and the row scales: (ceil(T/16), N + 1) workgroups,
// as many waves as there are 16-bin subtiles up to the kernel's bound (at least four: the
// scale slice reduces over 256 threads).
template <typename R, int NKT>
hipError_t vupdate_n(const Dims& d, const Ptrs& ptr, double floor, bool tap0, hipStream_t s) {
  NmfArgs<R> a = make_nargs<R>(d, VSplit{1, d.F}, ptr, floor, tap0, false);
  int waves = (d.F + 15) / 16;
  const int wmax = vupdate_threads<R, NKT>() / 64;
  waves = waves < 4 ? 4 : waves > wmax ? wmax : waves;
  dim3 grid((d.T + 15) / 16, d.N + 1);
  hipLaunchKernelGGL((k_vupdate<R, NKT>), grid, dim3(64 * waves), 0, s, a);
  return hipGetLastError();
}
template <typename R>
hipError_t vupdate_t(const Dims& d, const Ptrs& ptr, double floor, bool tap0, hipStream_t s) {
  switch ((d.K + 15) / 16) {
    case 1: return vupdate_n<R, 1>(d, ptr, floor, tap0, s);
    case 2: return vupdate_n<R, 2>(d, ptr, floor, tap0, s);
    case 3: return vupdate_n<R, 3>(d, ptr, floor, tap0, s);
    case 4: return vupdate_n<R, 4>(d, ptr, floor, tap0, s);
  }
  return hipErrorInvalidValue;
}

template <typename R>
hipError_t apply_mu_t(const Dims& d, const Ptrs& ptr, bool scale_y, hipStream_t s) {
  const size_t n = (size_t)d.F * d.Mb * d.Mb + (size_t)d.N * d.F * d.K + (scale_y ? (size_t)d.F * d.Mb * d.T : 0);
  hipLaunchKernelGGL(k_apply_mu<R>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     static_cast<Cx<R>*>(ptr.W), static_cast<R*>(ptr.B),
                     scale_y ? static_cast<Cx<R>*>(ptr.Y) : nullptr, static_cast<const R*>(ptr.mu), d.F, d.T, d.K,
                     d.rm);
  return hipGetLastError();
}

// ------------------------------------------------------------------ batched
template <typename R>
using WBFn = void (*)(const WDesc<R>* __restrict__, const int* __restrict__, int, int*);

template <typename R, int G, int RPL>
WBFn<R> pickb_cpl(int cpl) {
  if constexpr (sizeof(R) == 4) {
    switch (cpl) {
      case 4: return &k_iss_batch<R, G, 4, RPL>;
      case 8: return &k_iss_batch<R, G, 8, RPL>;
      case 10: return &k_iss_batch<R, G, 10, RPL>;
      case 12: return &k_iss_batch<R, G, 12, RPL>;
      case 16: return &k_iss_batch<R, G, 16, RPL>;
      case 20: return &k_iss_batch<R, G, 20, RPL>;
      case 24: return &k_iss_batch<R, G, 24, RPL>;
      case 28: return &k_iss_batch<R, G, 28, RPL>;
      case 32: return &k_iss_batch<R, G, 32, RPL>;
      default: return nullptr;
    }
  } else {
    switch (cpl) {
      case 4: return &k_iss_batch<R, G, 4, RPL>;
      case 6: return &k_iss_batch<R, G, 6, RPL>;
      case 8: return &k_iss_batch<R, G, 8, RPL>;
      case 10: return &k_iss_batch<R, G, 10, RPL>;
      case 12: return &k_iss_batch<R, G, 12, RPL>;
      case 16: return &k_iss_batch<R, G, 16, RPL>;
      default: return nullptr;
    }
  }
}

template <typename R>
WBFn<R> pickb(const Plan& p) {
  if (p.RPL == 1) {
    if (p.G == 16) return pickb_cpl<R, 16, 1>(p.CPL);
    if (p.G == 32) return pickb_cpl<R, 32, 1>(p.CPL);
    if (p.G == 64) return pickb_cpl<R, 64, 1>(p.CPL);
  } else if (p.RPL == 2) {
    if (p.G == 16) return pickb_cpl<R, 16, 2>(p.CPL);
    if (p.G == 32) return pickb_cpl<R, 32, 2>(p.CPL);
  }
  return nullptr;
}

template <typename R>
size_t wdesc_bytes() {
  return sizeof(WDesc<R>);
}

template <typename R>
void fill_wdesc(void* dst, const Plan& p, const Dims& d, const Ptrs& ptr, bool apply_mu, bool yload) {
  WDesc<R> w;
  w.a = make_iargs<R>(0, d, ptr, apply_mu, yload);  // batched bins keep the separate NMF launches
  w.a.xch = nullptr;
  Plan q = p;
  q.nmf = 0;
  w.L = wlayout(0, q, d, (int)sizeof(R));
  std::memcpy(dst, &w, sizeof(w));
}

// Workgroups of the batched ISS kernel resident at once for a dynamic LDS size.
template <typename R>
int resident_wblocks_batch(const Plan& p, size_t lds) {
  WBFn<R> fn = pickb<R>(p);
  int dev = 0, cus = 0, per_cu = 0;
  if (!fn || hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (lds > 65536 &&
      hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)fn, p.threads, lds) != hipSuccess) return 0;
  return per_cu * cus;
}

template <typename R>
hipError_t wupdate_batch_t(const Plan& p, const void* desc, const int* start, int nprob, int* work, size_t lds,
                           int blocks, hipStream_t s) {
  WBFn<R> fn = pickb<R>(p);
  if (!fn || blocks < 1) return hipErrorInvalidValue;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fn, dim3(blocks), dim3(p.threads), lds, s, static_cast<const WDesc<R>*>(desc), start, nprob, work);
  return hipGetLastError();
}

template <typename R>
size_t ndesc_bytes() {
  return sizeof(NmfDesc<R>);
}

// Descriptor of one problem for batched NMF kernel `kind` (0 lambda, 1 basis
// update, 2 activation partials, 3 activation update); returns its workgroup
// count (the same grid its single-problem launch uses) and, for kind 1, the
// threads it needs in *threads.
template <typename R>
int fill_ndesc(void* dst, int kind, const Dims& d, const VSplit& vs, const Ptrs& ptr, double floor, bool tap0,
               bool apply_mu, int* threads) {
  NmfDesc<R> n;
  int blocks = 0;
  if (kind == 0) {
    n.a = make_nargs<R>(d, VSplit{1, d.F}, ptr, 0.0, false, apply_mu);
    n.gx = (d.T + 63) / 64;
    n.gy = (d.F + 15) / 16;
    n.extra = 0;
    blocks = n.gx * n.gy * d.N;
  } else if (kind == 1) {
    n.a = make_nargs<R>(d, VSplit{1, d.F}, ptr, floor, false, apply_mu);
    const int fpw = sizeof(R) == 4 ? 32 : 16;
    int waves = (d.T + fpw - 1) / fpw;
    if (waves > kMaxNmfWaves) waves = kMaxNmfWaves;
    n.gx = (d.F + 15) / 16;
    n.gy = d.N;
    n.extra = waves;
    blocks = n.gx * d.N;
    if (threads) *threads = 64 * waves;
  } else if (kind == 2) {
    n.a = make_nargs<R>(d, vs, ptr, 0.0, tap0, false);
    n.gx = (d.T + 15) / 16;
    n.gy = vs.nch;
    n.extra = 0;
    blocks = n.gx * n.gy * d.N;
  } else {
    n.a = make_nargs<R>(d, vs, ptr, floor, tap0, false);
    const int nv = (d.N * d.K * d.T + 255) / 256;
    n.gx = nv + d.Mb;
    n.gy = 1;
    n.extra = nv;
    blocks = nv + d.Mb;
  }
  std::memcpy(dst, &n, sizeof(n));
  return blocks;
}

template <typename R>
hipError_t nmf_batch_t(int kind, const void* desc, const int* start, int nprob, int blocks, int threads, int* zero,
                       int nzero, hipStream_t s) {
  const NmfDesc<R>* d = static_cast<const NmfDesc<R>*>(desc);
  if (kind == 0)
    hipLaunchKernelGGL(k_lambda_batch<R>, dim3(blocks), dim3(256), 0, s, d, start, nprob, zero, nzero);
  else if (kind == 1)
    hipLaunchKernelGGL(k_nmf_b_batch<R>, dim3(blocks), dim3(threads), 0, s, d, start, nprob);
  else if (kind == 2)
    hipLaunchKernelGGL(k_vpart_batch<R>, dim3(blocks), dim3(256), 0, s, d, start, nprob);
  else
    hipLaunchKernelGGL(k_vfinal_batch<R>, dim3(blocks), dim3(256), 0, s, d, start, nprob);
  return hipGetLastError();
}

template <typename R>
OutArgs<R> make_oargs(const Dims& d, const Ptrs& ptr, void* C) {
  OutArgs<R> a;
  a.X = static_cast<const Cx<R>*>(ptr.X);
  a.W = static_cast<const Cx<R>*>(ptr.W);
  a.B = static_cast<const R*>(ptr.B);
  a.V = static_cast<const R*>(ptr.V);
  a.C = static_cast<Cx<R>*>(C);
  a.part = ptr.nllpart;
  a.status = ptr.status;
  a.F = d.F;
  a.T = d.T;
  a.M = d.M;
  a.D = d.D;
  a.K = d.K;
  a.rm = d.rm;
  return a;
}

template <typename R>
hipError_t images_t(const Dims& d, const Ptrs& ptr, void* C, hipStream_t s) {
  OutArgs<R> a = make_oargs<R>(d, ptr, C);
  const size_t lds = out_lds_bytes(d.Mb, d.M, d.N);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k_images<R>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_images<R>, dim3(d.F), dim3(256), lds, s, a);
  return hipGetLastError();
}

template <typename R>
hipError_t nll_t(const Dims& d, const Ptrs& ptr, hipStream_t s) {
  OutArgs<R> a = make_oargs<R>(d, ptr, nullptr);
  const size_t lds = nll_lds_bytes(d.Mb);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k_nll<R>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_nll<R>, dim3(d.F), dim3(256), lds, s, a);
  return hipGetLastError();
}

template <typename R>
__global__ void __launch_bounds__(256) k_identity(Cx<R>* W, int F, int Mb) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t n = (size_t)F * Mb * Mb;
  if (i >= n) return;
  const int c = (int)(i % Mb), r = (int)((i / Mb) % Mb);
  W[i] = Cx<R>{R(r == c ? 1 : 0), R(0)};
}

template <typename R>
hipError_t identity_t(const Dims& d, void* W, hipStream_t s) {
  const size_t n = (size_t)d.F * d.Mb * d.Mb;
  hipLaunchKernelGGL(k_identity<R>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, static_cast<Cx<R>*>(W), d.F,
                     d.Mb);
  return hipGetLastError();
}

// The launchers of the W update for one arithmetic of the W rows (WX).
#define CTFISS_INSTANTIATE_W(R, WX)                                                                            \
  template hipError_t wupdate_t<R, WX>(int, const Plan&, const Dims&, const Ptrs&, bool, bool, unsigned,       \
                                       double, hipStream_t);                                                   \
  template bool have_wkernel<R, WX>(int, int, int, int);                                                      \
  template bool have_tkernel<R, WX>(int, int, int);                                                           \
  template int resident_wblocks<R, WX>(int, const Plan&, const Dims&);

#define CTFISS_INSTANTIATE(R)                                                                                  \
  CTFISS_INSTANTIATE_W(R, false)                                                                              \
  template hipError_t lambda_t<R>(const Dims&, const Ptrs&, bool, hipStream_t);                               \
  template hipError_t nmfb_t<R>(const Dims&, const Ptrs&, double, bool, hipStream_t);                         \
  template hipError_t vpart_t<R>(const Dims&, const VSplit&, const Ptrs&, bool, hipStream_t);                 \
  template hipError_t vfinal_t<R>(const Dims&, const VSplit&, const Ptrs&, double, bool, hipStream_t);        \
  template hipError_t vupdate_t<R>(const Dims&, const Ptrs&, double, bool, hipStream_t);                     \
  template hipError_t apply_mu_t<R>(const Dims&, const Ptrs&, bool, hipStream_t);                            \
  template hipError_t images_t<R>(const Dims&, const Ptrs&, void*, hipStream_t);                             \
  template hipError_t nll_t<R>(const Dims&, const Ptrs&, hipStream_t);                                       \
  template hipError_t identity_t<R>(const Dims&, void*, hipStream_t);                                        \
  template size_t wdesc_bytes<R>();                                                                           \
  template void fill_wdesc<R>(void*, const Plan&, const Dims&, const Ptrs&, bool, bool);                      \
  template int resident_wblocks_batch<R>(const Plan&, size_t);                                                \
  template hipError_t wupdate_batch_t<R>(const Plan&, const void*, const int*, int, int*, size_t, int,          \
                                         hipStream_t);                                                        \
  template size_t ndesc_bytes<R>();                                                                           \
  template int fill_ndesc<R>(void*, int, const Dims&, const VSplit&, const Ptrs&, double, bool, bool, int*);  \
  template hipError_t nmf_batch_t<R>(int, const void*, const int*, int, int, int, int*, int, hipStream_t);

}  // namespace ctfiss
