// C ABI of the CTF-MNMF-ISS library: validation, workspace layout, launch order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/ctfiss.h"
#include "launch.hpp"
#include "out_impl.hpp"

namespace ctfiss {

bool choose_plan(int prec, int rule, const Dims& d, size_t max_lds, Plan* out) {
  (void)rule;
  const int* gs = prec == 0 ? kG32 : kG64;
  const int ng = prec == 0 ? (int)(sizeof(kG32) / sizeof(int)) : (int)(sizeof(kG64) / sizeof(int));
  const int* cpls = prec == 0 ? kCpl32 : kCpl64;
  const int ncpl = prec == 0 ? (int)(sizeof(kCpl32) / sizeof(int)) : (int)(sizeof(kCpl64) / sizeof(int));
  const size_t lds = iter_lds_layout(d.M, d.T, d.Mb, d.N, d.K, prec == 0 ? 4 : 8, rule != 0).total;
  if (lds > max_lds) return false;
  for (int gi = 0; gi < ng; ++gi) {
    const int G = gs[gi];
    const int threads = (d.Mb * G + 63) / 64 * 64;
    const int need = (d.T + G - 1) / G;
    for (int ci = 0; ci < ncpl; ++ci) {
      if (cpls[ci] >= need) {
        if (threads > iter_max_threads(prec == 0 ? 4 : 8, cpls[ci])) break;
        out->G = G;
        out->CPL = cpls[ci];
        out->threads = threads;
        out->lds = lds;
        return true;
      }
    }
  }
  return false;
}

// Split of the bins for the activation partial sums: enough workgroups to
// cover the chip twice, bins per chunk a multiple of 4.
VSplit choose_vsplit(const Dims& d) {
  const int tiles = (d.T + 63) / 64;
  int nch = (512 + d.N * tiles - 1) / (d.N * tiles);
  if (nch < 1) nch = 1;
  int fchunk = (d.F + nch - 1) / nch;
  fchunk = (fchunk + 3) / 4 * 4;
  if (fchunk < 4) fchunk = 4;
  nch = (d.F + fchunk - 1) / fchunk;
  return VSplit{nch, fchunk};
}

hipError_t launch_wupdate(int prec, int rule, const Plan& p, const Dims& d, const Ptrs& ptr, double floor,
                          bool apply_mu, hipStream_t s) {
  return prec == 0 ? wupdate_t<float>(rule, p, d, ptr, floor, apply_mu, s)
                   : wupdate_t<double>(rule, p, d, ptr, floor, apply_mu, s);
}
hipError_t launch_vpart(int prec, const Dims& d, const VSplit& vs, const Ptrs& ptr, bool tap0, hipStream_t s) {
  return prec == 0 ? vpart_t<float>(d, vs, ptr, tap0, s) : vpart_t<double>(d, vs, ptr, tap0, s);
}
hipError_t launch_vfinal(int prec, const Dims& d, const VSplit& vs, const Ptrs& ptr, double floor, bool tap0,
                         hipStream_t s) {
  return prec == 0 ? vfinal_t<float>(d, vs, ptr, floor, tap0, s) : vfinal_t<double>(d, vs, ptr, floor, tap0, s);
}
hipError_t launch_apply_mu(int prec, const Dims& d, const Ptrs& ptr, hipStream_t s) {
  return prec == 0 ? apply_mu_t<float>(d, ptr, s) : apply_mu_t<double>(d, ptr, s);
}
hipError_t launch_images(int prec, const Dims& d, const Ptrs& ptr, void* C, hipStream_t s) {
  return prec == 0 ? images_t<float>(d, ptr, C, s) : images_t<double>(d, ptr, C, s);
}
hipError_t launch_nll(int prec, const Dims& d, const Ptrs& ptr, hipStream_t s) {
  return prec == 0 ? nll_t<float>(d, ptr, s) : nll_t<double>(d, ptr, s);
}
hipError_t launch_identity(int prec, const Dims& d, void* W, hipStream_t s) {
  return prec == 0 ? identity_t<float>(d, W, s) : identity_t<double>(d, W, s);
}

__global__ void k_zero_status(int* status) {
  if (threadIdx.x == 0) status[0] = 0;
}
hipError_t launch_zero_status(int* status, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_status, dim3(1), dim3(64), 0, s, status);
  return hipGetLastError();
}
size_t images_lds(const Dims& d) { return out_lds_bytes(d.Mb, d.M, d.N); }
size_t nll_lds(const Dims& d) { return nll_lds_bytes(d.Mb); }

}  // namespace ctfiss

using namespace ctfiss;

namespace {

constexpr size_t kAlign = 256;
constexpr int kClasses = 5;

struct Layout {
  size_t W, B, V, P, P0, musq, mu, vnum, vden, nllpart, status, total;
};

struct TimedLaunch {
  int cls;
  hipEvent_t a, b;
};

int validate_shape(const ctfiss_shape* sh, int precision, Dims* d) {
  if (!sh || !d) return CTFISS_E_ARG;
  if (precision != CTFISS_FP32 && precision != CTFISS_FP64) return CTFISS_E_ARG;
  if (sh->F < 1 || sh->T < 1 || sh->M < 1 || sh->D < 1 || sh->N < 1 || sh->K < 1) return CTFISS_E_SHAPE;
  if (!sh->taps) return CTFISS_E_ARG;
  if (sh->N > CTFISS_MAX_SOURCES || sh->K > CTFISS_MAX_BASES) return CTFISS_E_UNSUPPORTED;
  const long long mb = (long long)sh->M * sh->D;
  long long sum = 0;
  for (int n = 0; n < sh->N; ++n) {
    if (sh->taps[n] < 1) return CTFISS_E_SHAPE;
    sum += sh->taps[n];
  }
  if (sum != mb) return CTFISS_E_SHAPE;
  if (mb > CTFISS_MAX_ROWS) return CTFISS_E_UNSUPPORTED;
  if ((long long)sh->F * sh->T > (1LL << 31) / 8) return CTFISS_E_UNSUPPORTED;
  std::memset(d, 0, sizeof(*d));
  d->F = sh->F;
  d->T = sh->T;
  d->M = sh->M;
  d->D = sh->D;
  d->N = sh->N;
  d->K = sh->K;
  d->Mb = (int)mb;
  d->rm.Mb = (int)mb;
  d->rm.N = sh->N;
  int r = 0;
  for (int n = 0; n < sh->N; ++n) {
    d->rm.r0[n] = r;
    d->rm.L[n] = sh->taps[n];
    for (int l = 0; l < sh->taps[n]; ++l, ++r) {
      d->rm.src[r] = (uint8_t)n;
      d->rm.tap[r] = (uint8_t)l;
    }
  }
  return CTFISS_OK;
}

Layout make_layout(const Dims& d, int precision) {
  const size_t rs = precision == CTFISS_FP32 ? 4 : 8, cs = 2 * rs;
  const VSplit vs = choose_vsplit(d);
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, kAlign);
    return o;
  };
  L.W = take((size_t)d.F * d.Mb * d.Mb * cs);
  L.B = take((size_t)d.N * d.F * d.K * rs);
  L.V = take((size_t)d.N * d.K * d.T * rs);
  L.P = take((size_t)d.N * d.F * d.T * rs);
  L.P0 = take((size_t)d.N * d.F * d.T * rs);
  L.musq = take((size_t)d.F * d.Mb * rs);
  L.mu = take((size_t)d.Mb * rs);
  L.vnum = take((size_t)d.N * vs.nch * d.K * d.T * rs);
  L.vden = take((size_t)d.N * vs.nch * d.K * d.T * rs);
  L.nllpart = take((size_t)d.F * sizeof(double));
  L.status = take(kAlign);
  L.total = off;
  return L;
}

}  // namespace

struct ctfiss_ctx {
  Dims d;
  int prec, rule, vrule;
  double floor;
  hipStream_t stream;
  char* ws;
  Layout lay;
  Ptrs ptr;
  Plan plan;
  VSplit vs;
  bool have_input, have_state;
  bool prof;
  std::vector<TimedLaunch> timed;
  std::vector<hipEvent_t> pool;
  int64_t launches[kClasses];
  double ms[kClasses];
};

namespace {

hipError_t ev_get(ctfiss_ctx* c, hipEvent_t* e) {
  if (!c->pool.empty()) {
    *e = c->pool.back();
    c->pool.pop_back();
    return hipSuccess;
  }
  return hipEventCreate(e);
}

// Runs one launch, bracketed by events when profiling is on.
template <typename Fn>
hipError_t timed(ctfiss_ctx* c, int cls, Fn&& fn) {
  if (!c->prof) return fn();
  TimedLaunch t{cls, nullptr, nullptr};
  hipError_t e = ev_get(c, &t.a);
  if (e == hipSuccess) e = ev_get(c, &t.b);
  if (e == hipSuccess) e = hipEventRecord(t.a, c->stream);
  if (e == hipSuccess) e = fn();
  if (e == hipSuccess) e = hipEventRecord(t.b, c->stream);
  if (t.a && t.b) c->timed.push_back(t);
  return e;
}

hipError_t drain_timing(ctfiss_ctx* c) {
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return e;
  for (const TimedLaunch& t : c->timed) {
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, t.a, t.b);
    if (e != hipSuccess) return e;
    c->launches[t.cls] += 1;
    c->ms[t.cls] += ms;
    c->pool.push_back(t.a);
    c->pool.push_back(t.b);
  }
  c->timed.clear();
  return hipSuccess;
}

}  // namespace

extern "C" {

int ctfiss_workspace_size(const ctfiss_shape* shape, int precision, size_t* bytes) {
  if (!bytes) return CTFISS_E_ARG;
  Dims d;
  const int st = validate_shape(shape, precision, &d);
  if (st != CTFISS_OK) return st;
  *bytes = make_layout(d, precision).total;
  return CTFISS_OK;
}

int ctfiss_create(const ctfiss_shape* shape, int precision, int rule, int vrule, double floor, void* workspace,
                  size_t workspace_bytes, void* stream, ctfiss_ctx** out) {
  if (!out || !workspace) return CTFISS_E_ARG;
  if (rule != CTFISS_RULE_ISS && rule != CTFISS_RULE_IP) return CTFISS_E_ARG;
  if (vrule != CTFISS_VRULE_ALL_TAPS && vrule != CTFISS_VRULE_PAPER_TAP0) return CTFISS_E_ARG;
  if (!(floor >= 0.0) || !std::isfinite(floor)) return CTFISS_E_ARG;
  Dims d;
  int st = validate_shape(shape, precision, &d);
  if (st != CTFISS_OK) return st;
  const Layout lay = make_layout(d, precision);
  if (workspace_bytes < lay.total || (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0)
    return CTFISS_E_WORKSPACE;
  int dev = 0, max_lds = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CTFISS_E_HIP;
  if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return CTFISS_E_HIP;
  Plan plan;
  if (!choose_plan(precision, rule, d, (size_t)max_lds, &plan)) return CTFISS_E_UNSUPPORTED;
  if (images_lds(d) > (size_t)max_lds || nll_lds(d) > (size_t)max_lds) return CTFISS_E_UNSUPPORTED;
  ctfiss_ctx* c = new (std::nothrow) ctfiss_ctx();
  if (!c) return CTFISS_E_ARG;
  c->d = d;
  c->prec = precision;
  c->rule = rule;
  c->vrule = vrule;
  c->floor = floor;
  c->stream = static_cast<hipStream_t>(stream);
  c->ws = static_cast<char*>(workspace);
  c->lay = lay;
  c->plan = plan;
  c->vs = choose_vsplit(d);
  c->ptr.X = nullptr;
  c->ptr.W = c->ws + lay.W;
  c->ptr.B = c->ws + lay.B;
  c->ptr.V = c->ws + lay.V;
  c->ptr.P = c->ws + lay.P;
  c->ptr.P0 = vrule == CTFISS_VRULE_PAPER_TAP0 ? static_cast<void*>(c->ws + lay.P0) : nullptr;
  c->ptr.musq = c->ws + lay.musq;
  c->ptr.mu = c->ws + lay.mu;
  c->ptr.vnum = c->ws + lay.vnum;
  c->ptr.vden = c->ws + lay.vden;
  c->ptr.nllpart = reinterpret_cast<double*>(c->ws + lay.nllpart);
  c->ptr.status = reinterpret_cast<int*>(c->ws + lay.status);
  c->have_input = c->have_state = false;
  c->prof = false;
  for (int i = 0; i < kClasses; ++i) {
    c->launches[i] = 0;
    c->ms[i] = 0.0;
  }
  if (launch_zero_status(c->ptr.status, c->stream) != hipSuccess) {
    delete c;
    return CTFISS_E_HIP;
  }
  *out = c;
  return CTFISS_OK;
}

int ctfiss_set_input(ctfiss_ctx* c, const void* X) {
  if (!c || !X) return CTFISS_E_ARG;
  c->ptr.X = X;
  c->have_input = true;
  return CTFISS_OK;
}

int ctfiss_set_state(ctfiss_ctx* c, const void* W, const void* B, const void* V) {
  if (!c || !B || !V) return CTFISS_E_ARG;
  const Dims& d = c->d;
  const size_t rs = c->prec == CTFISS_FP32 ? 4 : 8;
  hipError_t e;
  if (W)
    e = hipMemcpyAsync(c->ptr.W, W, (size_t)d.F * d.Mb * d.Mb * 2 * rs, hipMemcpyDeviceToDevice, c->stream);
  else
    e = launch_identity(c->prec, d, c->ptr.W, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->ptr.B, B, (size_t)d.N * d.F * d.K * rs, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->ptr.V, V, (size_t)d.N * d.K * d.T * rs, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = launch_zero_status(c->ptr.status, c->stream);
  if (e != hipSuccess) return CTFISS_E_HIP;
  c->have_state = true;
  return CTFISS_OK;
}

int ctfiss_iterate(ctfiss_ctx* c, int32_t n_iter) {
  if (!c || n_iter < 0) return CTFISS_E_ARG;
  if (!c->have_input || !c->have_state) return CTFISS_E_ORDER;
  const bool tap0 = c->vrule == CTFISS_VRULE_PAPER_TAP0;
  for (int it = 0; it < n_iter; ++it) {
    hipError_t e = timed(c, 0, [&] {
      return launch_wupdate(c->prec, c->rule, c->plan, c->d, c->ptr, c->floor, it > 0, c->stream);
    });
    if (e == hipSuccess)
      e = timed(c, 1, [&] { return launch_vpart(c->prec, c->d, c->vs, c->ptr, tap0, c->stream); });
    if (e == hipSuccess)
      e = timed(c, 2, [&] { return launch_vfinal(c->prec, c->d, c->vs, c->ptr, c->floor, tap0, c->stream); });
    if (e != hipSuccess) return CTFISS_E_HIP;
  }
  if (n_iter > 0) {
    hipError_t e = timed(c, 3, [&] { return launch_apply_mu(c->prec, c->d, c->ptr, c->stream); });
    if (e != hipSuccess) return CTFISS_E_HIP;
  }
  return CTFISS_OK;
}

int ctfiss_get_state(ctfiss_ctx* c, void* W, void* B, void* V) {
  if (!c) return CTFISS_E_ARG;
  if (!c->have_state) return CTFISS_E_ORDER;
  const Dims& d = c->d;
  const size_t rs = c->prec == CTFISS_FP32 ? 4 : 8;
  hipError_t e = hipSuccess;
  if (W) e = hipMemcpyAsync(W, c->ptr.W, (size_t)d.F * d.Mb * d.Mb * 2 * rs, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess && B)
    e = hipMemcpyAsync(B, c->ptr.B, (size_t)d.N * d.F * d.K * rs, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess && V)
    e = hipMemcpyAsync(V, c->ptr.V, (size_t)d.N * d.K * d.T * rs, hipMemcpyDeviceToDevice, c->stream);
  return e == hipSuccess ? CTFISS_OK : CTFISS_E_HIP;
}

int ctfiss_source_images(ctfiss_ctx* c, void* C) {
  if (!c || !C) return CTFISS_E_ARG;
  if (!c->have_input || !c->have_state) return CTFISS_E_ORDER;
  hipError_t e = timed(c, 4, [&] { return launch_images(c->prec, c->d, c->ptr, C, c->stream); });
  return e == hipSuccess ? CTFISS_OK : CTFISS_E_HIP;
}

int ctfiss_nll(ctfiss_ctx* c, double* out) {
  if (!c || !out) return CTFISS_E_ARG;
  if (!c->have_input || !c->have_state) return CTFISS_E_ORDER;
  std::vector<double> part((size_t)c->d.F);
  hipError_t e = launch_nll(c->prec, c->d, c->ptr, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(part.data(), c->ptr.nllpart, part.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return CTFISS_E_HIP;
  double s = 0.0;
  for (double v : part) s += v;
  *out = s;
  return CTFISS_OK;
}

int ctfiss_sync_status(ctfiss_ctx* c, int32_t* fault_code) {
  if (!c) return CTFISS_E_ARG;
  int code = 0;
  hipError_t e = hipMemcpyAsync(&code, c->ptr.status, sizeof(int), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return CTFISS_E_HIP;
  if (fault_code) *fault_code = code;
  return code == 0 ? CTFISS_OK : CTFISS_E_NUMERIC;
}

int ctfiss_destroy(ctfiss_ctx* c) {
  if (!c) return CTFISS_E_ARG;
  (void)hipStreamSynchronize(c->stream);
  for (const TimedLaunch& t : c->timed) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (hipEvent_t ev : c->pool) (void)hipEventDestroy(ev);
  delete c;
  return CTFISS_OK;
}

const char* ctfiss_status_string(int status) {
  switch (status) {
    case CTFISS_OK: return "ok";
    case CTFISS_E_ARG: return "invalid argument (null pointer, bad enum or count)";
    case CTFISS_E_SHAPE: return "inconsistent shape (dimensions < 1 or sum of taps != M*D)";
    case CTFISS_E_UNSUPPORTED: return "shape beyond this build's kernel limits";
    case CTFISS_E_WORKSPACE: return "workspace too small or not 256-byte aligned";
    case CTFISS_E_ORDER: return "input or state not set";
    case CTFISS_E_HIP: return "HIP runtime error";
    case CTFISS_E_NUMERIC: return "device numeric fault latched";
    default: return "unknown status";
  }
}

int ctfiss_set_profiling(ctfiss_ctx* c, int enable) {
  if (!c) return CTFISS_E_ARG;
  if (drain_timing(c) != hipSuccess) return CTFISS_E_HIP;
  c->prof = enable != 0;
  for (int i = 0; i < kClasses; ++i) {
    c->launches[i] = 0;
    c->ms[i] = 0.0;
  }
  return CTFISS_OK;
}

int ctfiss_kernel_stats(ctfiss_ctx* c, int which, int64_t* launches, double* total_ms) {
  if (!c || which < 0 || which >= kClasses) return CTFISS_E_ARG;
  if (drain_timing(c) != hipSuccess) return CTFISS_E_HIP;
  if (launches) *launches = c->launches[which];
  if (total_ms) *total_ms = c->ms[which];
  return CTFISS_OK;
}

}  // extern "C"
