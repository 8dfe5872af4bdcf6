// Host-side launch interface between the C ABI and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace ctfiss {

struct Dims {
  int F, T, M, D, N, K, Mb, lmax;
  RowMap rm;
};

// Launch shape of the W-update kernels: groups of G lanes, CPL frames per lane,
// RPL rows per lane; team > 1: each bin's frames are split over `team`
// workgroups of `slice` frames (ISS only).
struct Plan {
  int G, CPL, RPL, threads;
  size_t lds;
  int blocks;  // persistent workgroups launched (resident ones; at most F items)
  int team = 1;
  int slice = 0;
  int nmf = 0;  // single-workgroup ISS: also forms 1/lambda and updates b per bin (lds sized for it),
                // with the activations in LDS (1) or read from device memory (2)
};

// Type-erased device pointers of one context.
struct Ptrs {
  const void* X;
  void* W;
  void* B;
  void* V;
  void* ilam;
  void* P;
  void* P0;
  void* musq;
  void* mu;
  void* vnum;
  void* vden;
  double* nllpart;
  int* status;
  int* work;
  void* Y;  // [F][Mb][T] carried demixed rows (ISS)
  void* xch;  // [F][team_words] exchange words of team launches, or null
};

struct VSplit {
  int nch, fchunk;
};

// Instantiated launch shapes.
constexpr int kCpl32[] = {4, 8, 10, 12, 16, 20, 24, 28, 32};
constexpr int kCpl64[] = {4, 6, 8, 10, 12, 16};

bool choose_plan(int prec, int rule, const Dims& d, size_t max_lds, Plan* out);
int plan_string_team(const char* spec);
bool plan_from_string(const char* spec, int prec, int rule, const Dims& d, size_t max_lds, Plan* out);
VSplit choose_vsplit(const Dims& d, int prec);

// Typed launchers, defined once per precision.  WX (R = float only): the
// ISS sweep updates the rows of W in FP64 registers (mixed precision).
template <typename R, bool WX = false>
hipError_t wupdate_t(int rule, const Plan& p, const Dims& d, const Ptrs& ptr, bool apply_mu, bool yload,
                     unsigned epoch, double floor, hipStream_t s);
// LDS of the W-update kernel for a plan (p.nmf included).
size_t wupdate_lds(int rule, const Plan& p, const Dims& d, int rsize);
template <typename R>
hipError_t lambda_t(const Dims& d, const Ptrs& ptr, bool apply_mu, hipStream_t s);
template <typename R>
hipError_t nmfb_t(const Dims& d, const Ptrs& ptr, double floor, bool apply_mu, hipStream_t s);
template <typename R>
hipError_t vpart_t(const Dims& d, const VSplit& vs, const Ptrs& ptr, bool tap0, hipStream_t s);
template <typename R>
hipError_t vfinal_t(const Dims& d, const VSplit& vs, const Ptrs& ptr, double floor, bool tap0, hipStream_t s);
// Activation update and row scales in one launch (replaces vpart_t + vfinal_t).
template <typename R>
hipError_t vupdate_t(const Dims& d, const Ptrs& ptr, double floor, bool tap0, hipStream_t s);
template <typename R>
hipError_t apply_mu_t(const Dims& d, const Ptrs& ptr, bool scale_y, hipStream_t s);
// bfloat16 matrix-core variants of the NMF contractions (FP32 data; nmf_bf16.hip).
hipError_t lambda_bf16_t(const Dims& d, const Ptrs& ptr, bool apply_mu, hipStream_t s);
hipError_t nmfb_bf16_t(const Dims& d, const Ptrs& ptr, double floor, bool apply_mu, hipStream_t s);
hipError_t vpart_bf16_t(const Dims& d, const VSplit& vs, const Ptrs& ptr, bool tap0, hipStream_t s);
template <typename R>
hipError_t images_t(const Dims& d, const Ptrs& ptr, void* C, hipStream_t s);
template <typename R>
hipError_t nll_t(const Dims& d, const Ptrs& ptr, hipStream_t s);
template <typename R>
hipError_t identity_t(const Dims& d, void* W, hipStream_t s);
template <typename R, bool WX = false>
bool have_wkernel(int rule, int G, int cpl, int rpl);
template <typename R, bool WX = false>
bool have_tkernel(int G, int cpl, int rpl);
template <typename R, bool WX = false>
int resident_wblocks(int rule, const Plan& p, const Dims& d);

// Batched launches (many problems of one launch shape per W-update launch).
template <typename R>
size_t wdesc_bytes();
template <typename R>
void fill_wdesc(void* dst, const Plan& p, const Dims& d, const Ptrs& ptr, bool apply_mu, bool yload);
template <typename R>
int resident_wblocks_batch(const Plan& p, size_t lds);
template <typename R>
hipError_t wupdate_batch_t(const Plan& p, const void* desc, const int* start, int nprob, int* work, size_t lds,
                           int blocks, hipStream_t s);
template <typename R>
size_t ndesc_bytes();
template <typename R>
int fill_ndesc(void* dst, int kind, const Dims& d, const VSplit& vs, const Ptrs& ptr, double floor, bool tap0,
               bool apply_mu, int* threads);
template <typename R>
hipError_t nmf_batch_t(int kind, const void* desc, const int* start, int nprob, int blocks, int threads, int* zero,
                       int nzero, hipStream_t s);
hipError_t launch_zero_status(int* status, hipStream_t s);

// Reverse mode of the unrolled iterations (FP32 or FP64; see adjoint.hip).
// Real arrays are of the context's real type, complex ones of its complex type.
struct AdjPtrs {
  const void* X;                     // [M][F][T]
  const void* Wk;                    // state at the start of the iteration being reversed
  const void* Bk;
  const void* Vk;
  const void* Ws;                    // W after the sweep (before the rescale)
  const void* Bh;                    // B after the basis update (before the rescale)
  const void* Vh;                    // V after the activation update
  const void* ilam;                  // 1 / (Bk Vk)
  const void* P;                     // tap-aligned powers of the swept rows
  const void* P0;                    // tap-0 powers (tap-0 activation rule) or null
  const void* mu;                    // row scales of the iteration
  void* gW;                          // adjoints of the state: in, of the next state; out, of this one
  void* gB;
  void* gV;
  void* gP0;                         // adjoint of P0 (tap-0 activation rule) or null
  void *gBh, *gVh, *gP, *glam, *glamh, *lamh, *q1, *q2, *G1, *G2, *H1, *H2, *part, *gS;  // scratch
  void* gX;                          // [M][F][T] accumulated
  int* status;
  void* Y;                           // [F][Mb][T] sweep scratch
  void* gY;
  void* gphi;
  void* ztape;                       // [F][Mb][Mb]
  void* dtape;
  void* l2sums;                      // [adj_l2_chunks(F)][N][K][T] chunk sums of the activation adjoint
};
constexpr int kAdjL2Chunks = 8;
int adj_l2_chunks(int F);
size_t adj_images_lds(int Mb, int M, int rs);
size_t adj_iss_lds(int Mb, int T, int rs);
hipError_t adj_images(const AdjPtrs& p, const Dims& d, const void* W, const void* gC, int rs, hipStream_t s);
hipError_t adj_iteration(const AdjPtrs& p, const Dims& d, double floor, int rs, hipStream_t s);
size_t images_lds(const Dims& d);
size_t nll_lds(const Dims& d);

}  // namespace ctfiss
