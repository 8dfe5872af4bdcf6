// Host-side launch interface between the C ABI and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace ctfiss {

struct Dims {
  int F, T, M, D, N, K, Mb;
  RowMap rm;
};

// Launch shape of the W-update kernels: groups of G lanes, CPL frames per lane.
struct Plan {
  int G, CPL, threads;
  size_t lds;
};

// Type-erased device pointers of one context.
struct Ptrs {
  const void* X;
  void* W;
  void* B;
  void* V;
  void* P;
  void* P0;
  void* musq;
  void* mu;
  void* vnum;
  void* vden;
  double* nllpart;
  int* status;
};

struct VSplit {
  int nch, fchunk;
};

// Group sizes G and frames per lane CPL instantiated for each precision.
constexpr int kG32[] = {16, 32};
constexpr int kCpl32[] = {4, 8, 12, 16, 20, 24, 28, 32};
constexpr int kG64[] = {32, 64, 16};
constexpr int kCpl64[] = {4, 6, 8, 10, 12, 16};

bool choose_plan(int prec, int rule, const Dims& d, size_t max_lds, Plan* out);
VSplit choose_vsplit(const Dims& d);

// Kernel launchers (prec 0 = FP32, 1 = FP64).  All are asynchronous on s.
// Typed launchers, defined once per precision.
template <typename R>
hipError_t wupdate_t(int rule, const Plan& p, const Dims& d, const Ptrs& ptr, double floor, bool apply_mu,
                     hipStream_t s);
template <typename R>
hipError_t vpart_t(const Dims& d, const VSplit& vs, const Ptrs& ptr, bool tap0, hipStream_t s);
template <typename R>
hipError_t vfinal_t(const Dims& d, const VSplit& vs, const Ptrs& ptr, double floor, bool tap0, hipStream_t s);
template <typename R>
hipError_t apply_mu_t(const Dims& d, const Ptrs& ptr, hipStream_t s);
template <typename R>
hipError_t images_t(const Dims& d, const Ptrs& ptr, void* C, hipStream_t s);
template <typename R>
hipError_t nll_t(const Dims& d, const Ptrs& ptr, hipStream_t s);
template <typename R>
hipError_t identity_t(const Dims& d, void* W, hipStream_t s);

hipError_t launch_wupdate(int prec, int rule, const Plan& p, const Dims& d, const Ptrs& ptr, double floor,
                          bool apply_mu, hipStream_t s);
hipError_t launch_vpart(int prec, const Dims& d, const VSplit& vs, const Ptrs& ptr, bool tap0, hipStream_t s);
hipError_t launch_vfinal(int prec, const Dims& d, const VSplit& vs, const Ptrs& ptr, double floor, bool tap0,
                         hipStream_t s);
hipError_t launch_apply_mu(int prec, const Dims& d, const Ptrs& ptr, hipStream_t s);
hipError_t launch_images(int prec, const Dims& d, const Ptrs& ptr, void* C, hipStream_t s);
hipError_t launch_nll(int prec, const Dims& d, const Ptrs& ptr, hipStream_t s);
hipError_t launch_identity(int prec, const Dims& d, void* W, hipStream_t s);
hipError_t launch_zero_status(int* status, hipStream_t s);
size_t images_lds(const Dims& d);
size_t nll_lds(const Dims& d);

}  // namespace ctfiss
