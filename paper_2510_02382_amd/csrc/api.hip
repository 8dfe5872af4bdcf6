// C ABI of the CTF-MNMF-ISS library: validation, workspace layout, launch order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "ctfiss.h"
#include "launch.hpp"
#include "out_impl.hpp"

namespace ctfiss {

// Candidate (G, RPL) orders per precision and rule; the first that fits wins.
// For each, CPL is the smallest instantiated value with G * CPL >= T.
namespace {
struct GR {
  int G, RPL;
};
constexpr GR kIss32[] = {{16, 1}, {32, 1}, {16, 2}, {32, 2}};
constexpr GR kIss64[] = {{32, 1}, {64, 1}, {16, 1}, {16, 2}, {32, 2}};
constexpr GR kIp32[] = {{16, 1}, {32, 1}};
constexpr GR kIp64[] = {{32, 1}, {64, 1}, {16, 1}};

// Precision codes: CTFISS_FP32 (0), CTFISS_FP64 (1), CTFISS_MIXED (2: FP32 data and
// kernels, FP64 W rows in the ISS sweep), CTFISS_MIXED_BF16 (3: CTFISS_MIXED with the
// NMF contractions on bfloat16 matrix cores).  wx(): the W update keeps FP64 W rows.
inline bool wx(int prec) { return prec == CTFISS_MIXED || prec == CTFISS_MIXED_BF16; }
bool have_w(int prec, int rule, int G, int cpl, int rpl) {
  if (wx(prec)) return have_wkernel<float, true>(rule, G, cpl, rpl);
  return prec == CTFISS_FP32 ? have_wkernel<float>(rule, G, cpl, rpl) : have_wkernel<double>(rule, G, cpl, rpl);
}
bool have_t(int prec, int G, int cpl, int rpl) {
  if (wx(prec)) return have_tkernel<float, true>(G, cpl, rpl);
  return prec == CTFISS_FP32 ? have_tkernel<float>(G, cpl, rpl) : have_tkernel<double>(G, cpl, rpl);
}

bool plan_for(int prec, int rule, const Dims& d, size_t max_lds, int G, int RPL, int cpl_req, Plan* out) {
  const bool f32 = prec != CTFISS_FP64;
  const int* cpls = f32 ? kCpl32 : kCpl64;
  const int ncpl = f32 ? (int)(sizeof(kCpl32) / sizeof(int)) : (int)(sizeof(kCpl64) / sizeof(int));
  const int rs = f32 ? 4 : 8;
  const int need = (d.T + G - 1) / G;
  for (int ci = 0; ci < ncpl; ++ci) {
    const int cpl = cpls[ci];
    if (cpl < need || (cpl_req > 0 && cpl != cpl_req)) continue;
    const int groups = (d.Mb + RPL - 1) / RPL;
    const int threads = (groups * G + 63) / 64 * 64;
    if (threads > iter_max_threads(rs, cpl, RPL)) return false;
    const bool ok = have_w(prec, rule, G, cpl, RPL);
    if (!ok) return false;
    const size_t lds = iter_lds_layout(d.M, d.T, d.D, d.Mb, d.N, d.lmax, G, cpl, rs, rule != 0).total;
    if (lds > max_lds) return false;
    *out = Plan{G, cpl, RPL, threads, lds, 0};
    return true;
  }
  return false;
}

// Team plan (ISS): the frames of each bin split over P workgroups of S =
// ceil(T / P) frames (fewer members if the last ones would be empty).  A
// member's slice must cover the Lmax - 1 frames its predecessor's tap-aligned
// powers read from it.
bool plan_for_team(int prec, const Dims& d, size_t max_lds, int G, int RPL, int P, int cpl_req, Plan* out) {
  if (P < 2 || P > kMaxTeam) return false;
  const int S = (d.T + P - 1) / P;
  const int Pe = (d.T + S - 1) / S;
  if (Pe < 2 || S < d.lmax - 1) return false;
  const bool f32 = prec != CTFISS_FP64;
  const int* cpls = f32 ? kCpl32 : kCpl64;
  const int ncpl = f32 ? (int)(sizeof(kCpl32) / sizeof(int)) : (int)(sizeof(kCpl64) / sizeof(int));
  const int rs = f32 ? 4 : 8;
  const int need = (S + G - 1) / G;
  for (int ci = 0; ci < ncpl; ++ci) {
    const int cpl = cpls[ci];
    if (cpl < need || (cpl_req > 0 && cpl != cpl_req)) continue;
    const bool ok = have_t(prec, G, cpl, RPL);
    if (!ok) continue;
    const int groups = (d.Mb + RPL - 1) / RPL;
    const int threads = (groups * G + 63) / 64 * 64;
    if (threads > iter_max_threads(rs, cpl, RPL)) return false;
    const size_t lds = iter_lds_layout(d.M, d.T, d.D, d.Mb, d.N, d.lmax, G, cpl, rs, false, Pe, S).total;
    if (lds > max_lds) return false;
    *out = Plan{G, cpl, RPL, threads, lds, 0, Pe, S};
    return true;
  }
  return false;
}

// Team shapes tried in order, each with the fewest members that fit.
constexpr GR kTeam32[] = {{16, 1}, {16, 2}, {32, 2}};
constexpr GR kTeam64[] = {{16, 1}, {16, 2}};
}  // namespace

// Plans measured by ctfiss_autotune, per (precision, rule, Mbar, M, D, N, Lmax,
// T rounded up to a multiple of 32): later contexts of such a shape take them.
namespace {
struct TuneKey {
  int prec, rule, Mb, M, D, N, lmax, tb;
  bool operator==(const TuneKey& o) const {
    return prec == o.prec && rule == o.rule && Mb == o.Mb && M == o.M && D == o.D && N == o.N && lmax == o.lmax &&
           tb == o.tb;
  }
};
struct TuneEntry {
  TuneKey key;
  Plan plan;
};
std::vector<TuneEntry>& tune_cache() {
  static std::vector<TuneEntry> cache;
  return cache;
}
std::mutex& tune_mutex() {
  static std::mutex m;
  return m;
}
TuneKey tune_key(int prec, int rule, const Dims& d) {
  return TuneKey{prec, rule, d.Mb, d.M, d.D, d.N, d.lmax, (d.T + 31) / 32 * 32};
}
}  // namespace

bool tuned_plan(int prec, int rule, const Dims& d, size_t max_lds, Plan* out) {
  const TuneKey k = tune_key(prec, rule, d);
  std::lock_guard<std::mutex> lock(tune_mutex());
  for (const auto& e : tune_cache()) {
    if (!(e.key == k)) continue;
    // re-derive for this T (the bucket may hold a slightly shorter signal)
    Plan p;
    if (e.plan.team > 1) {
      if (plan_for_team(prec, d, max_lds, e.plan.G, e.plan.RPL, e.plan.team, 0, &p)) { *out = p; return true; }
    } else if (plan_for(prec, rule, d, max_lds, e.plan.G, e.plan.RPL, 0, &p)) {
      *out = p;
      return true;
    }
  }
  return false;
}

bool choose_plan(int prec, int rule, const Dims& d, size_t max_lds, Plan* out) {
  if (tuned_plan(prec, rule, d, max_lds, out)) return true;
  const GR* list;
  int n;
  const bool f32 = prec != CTFISS_FP64;
  if (rule == 0) {
    list = f32 ? kIss32 : kIss64;
    n = f32 ? (int)(sizeof(kIss32) / sizeof(GR)) : (int)(sizeof(kIss64) / sizeof(GR));
  } else {
    if (wx(prec)) return false;  // the mixed paths are ISS paths
    list = f32 ? kIp32 : kIp64;
    n = f32 ? (int)(sizeof(kIp32) / sizeof(GR)) : (int)(sizeof(kIp64) / sizeof(GR));
  }
  // FP32 ISS: 32-lane groups whenever the workgroup fits (Mbar <= 32) and
  // needs at most 20 frames per lane (no spills); past that, 64-lane groups if
  // they fit (Mbar <= 16), else 32-lane groups with more frames per lane.
  // Against a 16-lane group: half the frames per lane (fewer registers), and
  // for Mbar = 24 three waves per SIMD (a 16-lane group has 2 on two SIMDs and
  // 1 on the others); at <= 10 frames per lane two such workgroups share a CU.
  // Mbar <= 8 (no or little frame stacking): 64-lane groups, a workgroup of at
  // most 8 waves whose bin latency is the frame loop of each ISS step; half
  // the frames per lane of a 32-lane group shortens it (measured at Mbar =
  // 4, 6, 8 with T = 501: 25-30 us per launch against 30-33 us).
  if (rule == 0 && f32) {
    Plan p;
    if (d.Mb <= 8 && plan_for(prec, rule, d, max_lds, 64, 1, 0, &p)) {
      *out = p;
      return true;
    }
    if (plan_for(prec, rule, d, max_lds, 32, 1, 0, &p) && p.CPL <= 20) {
      *out = p;
      return true;
    }
    if (plan_for(prec, rule, d, max_lds, 64, 1, 0, &p) || plan_for(prec, rule, d, max_lds, 32, 1, 0, &p)) {
      *out = p;
      return true;
    }
  }
  // Mbar <= 8 in FP64 (ISS and IP) and FP32 IP: the bin's latency is again the frame
  // loop of each step, so the wider groups that fit win (measured at Mbar = 4, 6, 8,
  // T = 501, W update per launch: FP64 ISS 64-lane 20.7 / 26.8 / 54.4 us against
  // 73.3 / 102.5 / 175.7 us for 32-lane groups; FP64 IP 64-lane 76 / 154 / 181 us against
  // 85 / 169 / 198; FP32 IP 32-lane 91 / 104 / 127 us against 124 / 134 / 174 us for
  // 16-lane groups and 85 / 172 / 198 us for 64-lane ones).
  if (d.Mb <= 8 && !(rule == 0 && f32)) {
    Plan p;
    if (plan_for(prec, rule, d, max_lds, f32 ? 32 : 64, 1, 0, &p)) {
      *out = p;
      return true;
    }
  }
  for (int i = 0; i < n; ++i)
    if (plan_for(prec, rule, d, max_lds, list[i].G, list[i].RPL, 0, out)) return true;
  // ISS bins too long for one workgroup: teams of workgroups
  if (rule == 0) {
    const GR* tl = f32 ? kTeam32 : kTeam64;
    const int tn = f32 ? (int)(sizeof(kTeam32) / sizeof(GR)) : (int)(sizeof(kTeam64) / sizeof(GR));
    for (int P = 2; P <= kMaxTeam; ++P)
      for (int i = 0; i < tn; ++i)
        if (plan_for_team(prec, d, max_lds, tl[i].G, tl[i].RPL, P, 0, out)) return true;
  }
  return false;
}

// "G,CPL,RPL" or "G,CPL,RPL,P" with P > 1 for a team of P workgroups per bin
// (used to tune launch shapes; CTFISS_PLAN in the environment).
bool plan_from_string(const char* spec, int prec, int rule, const Dims& d, size_t max_lds, Plan* out) {
  int G = 0, cpl = 0, rpl = 0, P = 1;
  if (!spec) return false;
  const int n = std::sscanf(spec, "%d,%d,%d,%d", &G, &cpl, &rpl, &P);
  if (n < 3) return false;
  if (n == 4 && P > 1) return rule == 0 && plan_for_team(prec, d, max_lds, G, rpl, P, cpl, out);
  return plan_for(prec, rule, d, max_lds, G, rpl, cpl, out);
}

// Members per bin a plan string asks for (1 if none).
int plan_string_team(const char* spec) {
  int G = 0, cpl = 0, rpl = 0, P = 1;
  if (!spec || std::sscanf(spec, "%d,%d,%d,%d", &G, &cpl, &rpl, &P) != 4) return 1;
  return P > 1 ? (P < kMaxTeam ? P : kMaxTeam) : 1;
}

// Split of the bins for the activation partial sums: chunks of 64 bins (four
// 16-bin MFMA sub-tiles per wave).
VSplit choose_vsplit(const Dims& d, int prec) {
  // bfloat16 activation partials take 32 bins per wave (the instruction sums 32 values)
  const int fchunk = prec == CTFISS_MIXED_BF16 ? 128 : 64;
  return VSplit{(d.F + fchunk - 1) / fchunk, fchunk};
}

__global__ void k_zero_status(int* status) {
  if (threadIdx.x == 0) status[0] = 0;
}
hipError_t launch_zero_status(int* status, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_status, dim3(1), dim3(64), 0, s, status);
  return hipGetLastError();
}
__global__ void __launch_bounds__(256) k_zero_words(unsigned long long* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}
// Three device-to-device copies of 32-bit words in one launch (the per-iteration
// saves and restores of W, B and V in the reverse pass are launch-bound copies).
struct Copy3 {
  unsigned* dst[3];
  const unsigned* src[3];
  size_t words[3];
};
__global__ void __launch_bounds__(256) k_copy3(Copy3 c) {
  const size_t n0 = c.words[0], n1 = n0 + c.words[1], n = n1 + c.words[2];
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int r = i < n0 ? 0 : (i < n1 ? 1 : 2);
    const size_t j = i - (r == 0 ? 0 : (r == 1 ? n0 : n1));
    c.dst[r][j] = c.src[r][j];
  }
}
// bytes: multiples of 4 (every state array here is).
hipError_t launch_copy3(void* d0, const void* s0, size_t b0, void* d1, const void* s1, size_t b1, void* d2,
                        const void* s2, size_t b2, hipStream_t s) {
  Copy3 c{{static_cast<unsigned*>(d0), static_cast<unsigned*>(d1), static_cast<unsigned*>(d2)},
          {static_cast<const unsigned*>(s0), static_cast<const unsigned*>(s1), static_cast<const unsigned*>(s2)},
          {b0 / 4, b1 / 4, b2 / 4}};
  const size_t n = c.words[0] + c.words[1] + c.words[2];
  if (n == 0) return hipSuccess;
  const size_t blocks = (n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024;
  hipLaunchKernelGGL(k_copy3, dim3((unsigned)blocks), dim3(256), 0, s, c);
  return hipGetLastError();
}
hipError_t launch_zero_words(unsigned long long* p, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const size_t blocks = (n + 255) / 256 < 2048 ? (n + 255) / 256 : 2048;
  hipLaunchKernelGGL(k_zero_words, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}
// Sum of n per-bin partials into *out by one workgroup in a fixed order
// (thread i adds elements i, i + 256, ...; then a tree over the threads).
__global__ void __launch_bounds__(256) k_sum_parts(const double* part, int n, double* out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += part[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}
hipError_t launch_sum_parts(const double* part, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, part, n, out);
  return hipGetLastError();
}
size_t images_lds(const Dims& d) { return out_lds_bytes(d.Mb, d.M, d.N); }
size_t wupdate_lds(int rule, const Plan& p, const Dims& d, int rsize) {
  const bool nmf = p.nmf && rule == 0 && p.team <= 1;
  return iter_lds_layout(d.M, d.T, d.D, d.Mb, d.N, d.lmax, p.G, p.CPL, rsize, rule != 0, p.team, p.slice,
                         nmf ? d.K : 0, nmf && p.nmf == 2)
      .total;
}
size_t nll_lds(const Dims& d) { return nll_lds_bytes(d.Mb); }

}  // namespace ctfiss

using namespace ctfiss;

namespace {

constexpr size_t kAlign = 256;
constexpr int kClasses = 7;
constexpr int kTraceCap = 256;  // NLL values one readback of ctfiss_iterate carries

struct Layout {
  size_t W, B, V, ilam, P, P0, musq, mu, vnum, vden, nllpart, trace, status, work, Y, xch, total;
  int team;  // members per bin the exchange words are sized for (0: none)
};

struct TimedLaunch {
  int cls;
  hipEvent_t a, b;
};

int validate_shape(const ctfiss_shape* sh, int precision, Dims* d) {
  if (!sh || !d) return CTFISS_E_ARG;
  if (precision != CTFISS_FP32 && precision != CTFISS_FP64 && precision != CTFISS_MIXED &&
      precision != CTFISS_MIXED_BF16)
    return CTFISS_E_ARG;
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
  d->lmax = 0;
  int r = 0;
  for (int n = 0; n < sh->N; ++n) {
    if (sh->taps[n] > d->lmax) d->lmax = sh->taps[n];
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
  const size_t rs = precision != CTFISS_FP64 ? 4 : 8, cs = 2 * rs;
  const VSplit vs = choose_vsplit(d, precision);
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
  L.ilam = take((size_t)d.N * d.F * d.T * rs);
  L.P = take((size_t)d.N * d.F * d.T * rs);
  L.P0 = take((size_t)d.N * d.F * d.T * rs);
  L.musq = take((size_t)d.F * d.Mb * rs);
  L.mu = take((size_t)d.Mb * rs);
  L.vnum = take((size_t)d.N * vs.nch * d.K * d.T * rs);
  L.vden = take((size_t)d.N * vs.nch * d.K * d.T * rs);
  L.nllpart = take((size_t)d.F * sizeof(double));
  L.trace = take((size_t)kTraceCap * sizeof(double));
  L.status = take(kAlign);
  L.work = take(kAlign);
  L.Y = take((size_t)d.F * d.Mb * d.T * cs);
  // Exchange words for team launches: sized for the plan an ISS context of
  // this shape takes on gfx950 (or the one CTFISS_PLAN asks for).
  Plan p;
  L.team = 0;
  if (choose_plan(precision, CTFISS_RULE_ISS, d, kMaxLdsBytes, &p) && p.team > 1) L.team = p.team;
  const int forced = plan_string_team(std::getenv("CTFISS_PLAN"));
  if (forced > 1 && forced > L.team) L.team = forced;
  L.xch = L.team > 1 ? take((size_t)d.F * team_words(d.Mb, d.lmax, L.team, (int)rs) * 8) : 0;
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
  double* trace;  // [kTraceCap] NLL after each iteration of a traced call
  Plan plan;
  VSplit vs;
  bool vone;  // activation update and row scales in one launch (else partials + final sum)
  bool have_input, have_state;
  bool y_valid;    // the carried Y holds W xbar of the current W (ISS)
  unsigned epoch;  // tag base of the last team launch's exchange words
  bool graph;      // ctfiss_iterate replays captured HIP graphs
  struct GraphEntry {
    int n;
    bool y_valid;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  int prof;  // bit mask of timed kernel classes
  std::vector<TimedLaunch> timed;
  std::vector<hipEvent_t> pool;
  int64_t launches[kClasses];
  double ms[kClasses];
};

namespace {

void drop_graphs(ctfiss_ctx* c) {
  for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
  c->graphs.clear();
}

// Timing events: read only through hipEventElapsedTime after drain_timing has
// synchronised the stream, so they record without the system-scope fence (a cache
// writeback and invalidation per record that would also slow the timed launches).
hipError_t ev_get(ctfiss_ctx* c, hipEvent_t* e) {
  if (!c->pool.empty()) {
    *e = c->pool.back();
    c->pool.pop_back();
    return hipSuccess;
  }
  return hipEventCreateWithFlags(e, hipEventDisableSystemFence);
}

// Runs one launch, bracketed by events when profiling is on.
template <typename Fn>
hipError_t timed(ctfiss_ctx* c, int cls, Fn&& fn) {
  if (!(c->prof & (1 << cls))) return fn();
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

namespace {

// Argument and shape checks of a context (no HIP call).
int check_create_args(const ctfiss_shape* shape, int precision, int rule, int vrule, double floor, Dims* d,
                      Layout* lay) {
  if (rule != CTFISS_RULE_ISS && rule != CTFISS_RULE_IP) return CTFISS_E_ARG;
  if (vrule != CTFISS_VRULE_ALL_TAPS && vrule != CTFISS_VRULE_PAPER_TAP0) return CTFISS_E_ARG;
  if (!(floor >= 0.0) || !std::isfinite(floor)) return CTFISS_E_ARG;
  const int st = validate_shape(shape, precision, d);
  if (st != CTFISS_OK) return st;
  *lay = make_layout(*d, precision);
  return CTFISS_OK;
}

// The single-launch activation update keeps each (source, 16 frames) in one workgroup,
// so the matrix-core work of each of its SIMDs grows with the band and with K: it
// beats the partial sums over bin chunks plus their final sum where a wave takes few
// 16-bin subtiles (measured on MI355X: F = 513, K = 3, one launch 7.7 us against
// 5.2 + 4.4 us; F = 1025, K = 20, 19.6 us against 6.9 + 4.9 us).  Cost: subtiles per
// wave times MFMA steps per subtile (K/4 for lambda, 8 per 16-wide K tile).
bool vupdate_pays(const Dims& d, int precision) {
  const int nkt = (d.K + 15) / 16, nks = (d.K + 3) / 4;
  const int waves = precision != CTFISS_FP64 ? (nkt <= 2 ? 16 : 8) : (nkt <= 1 ? 16 : nkt == 2 ? 8 : 4);
  const int sub = ((d.F + 15) / 16 + waves - 1) / waves;
  return sub * (nks + 8 * nkt) <= 48;
}

// Fills a context over `workspace` (checked by the caller): launch plan, pointers into the
// workspace, cleared status word and exchange words.
int init_ctx(ctfiss_ctx* c, const Dims& d, const Layout& lay, int precision, int rule, int vrule, double floor,
             void* workspace, void* stream) {
  int dev = 0, max_lds = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CTFISS_E_HIP;
  if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return CTFISS_E_HIP;
  Plan plan;
  const char* spec = std::getenv("CTFISS_PLAN");
  if (spec && *spec) {
    if (!plan_from_string(spec, precision, rule, d, (size_t)max_lds, &plan)) return CTFISS_E_UNSUPPORTED;
  } else if (!choose_plan(precision, rule, d, (size_t)max_lds, &plan)) {
    return CTFISS_E_UNSUPPORTED;
  }
  if (images_lds(d) > (size_t)max_lds || nll_lds(d) > (size_t)max_lds) return CTFISS_E_UNSUPPORTED;
  if (plan.team > 1 && plan.team > lay.team) return CTFISS_E_UNSUPPORTED;
  // Persistent W-update workgroups: as many as fit on the device at once
  // (CTFISS_WBLOCKS in the environment overrides it, for tuning); any count
  // >= 1 gives the same result, since the workgroups share out the bins.
  auto resident = [&](const Plan& p) {
    return wx(precision) ? resident_wblocks<float, true>(rule, p, d)
           : precision == CTFISS_FP32 ? resident_wblocks<float>(rule, p, d)
                                      : resident_wblocks<double>(rule, p, d);
  };
  plan.blocks = resident(plan);
  // Single-workgroup ISS bins form 1/lambda and update b themselves (no separate
  // lambda and basis-update launches) where the layout fits without fewer
  // workgroups in flight: with the activations in LDS (e.g. Mbar <= 8, K = 3, where
  // an iteration is bound by launch latency), else, in FP32 and mixed precision,
  // reading them from device memory (e.g. Mbar = 24, K = 20, where their 50 KB in LDS
  // would halve the workgroups per CU; measured on MI355X, 13.3 against 13.6 ms per
  // 100 FP32 iterations, while FP64, whose sweep is slower per bin, lost 31 against
  // 27 ms).  CTFISS_UNFUSED_NMF in the environment keeps the separate launches;
  // CTFISS_NMF_FROM_DEVICE reads the activations from device memory wherever the bins
  // fuse (the same arithmetic in the same order as from LDS).
  const bool unfused = std::getenv("CTFISS_UNFUSED_NMF") != nullptr;
  if (rule == CTFISS_RULE_ISS && plan.team <= 1 && !unfused && precision != CTFISS_MIXED_BF16) {
    const int need = plan.blocks < d.F ? plan.blocks : d.F;
    const bool dev_v = std::getenv("CTFISS_NMF_FROM_DEVICE") != nullptr;
    // FP64 reads the activations from device memory only at Mbar <= 8, where each bin is its
    // workgroup's only one (Mbar = 4, T = 501, K = 3: 33.5 us per iteration against 41.2 us for
    // the W update, lambda and basis-update launches; at Mbar = 24, T = 313, K = 20 the separate
    // launches win, 27.5 against 30.9 ms per 100 iterations)
    const int last = (dev_v || precision != CTFISS_FP64 || d.Mb <= 8) ? 2 : 1;
    for (int kind = dev_v ? 2 : 1; kind <= last; ++kind) {
      Plan q = plan;
      q.nmf = kind;
      q.lds = wupdate_lds(rule, q, d, precision != CTFISS_FP64 ? 4 : 8);
      if (q.lds > (size_t)max_lds) continue;
      q.blocks = resident(q);
      if (q.blocks >= need) {
        plan = q;
        break;
      }
    }
  }
  // A team's waits end only once all its members run together: a team plan
  // needs at least `team` resident workgroups.
  const int items = d.F * (plan.team > 1 ? plan.team : 1);
  if (const char* wb = std::getenv("CTFISS_WBLOCKS")) {
    int n = std::atoi(wb);
    if (n > 0) {
      if (n < plan.team) n = plan.team;
      plan.blocks = n < items ? n : items;
    }
  }
  if (plan.team > 1 && plan.blocks < plan.team) return CTFISS_E_UNSUPPORTED;
  c->d = d;
  c->prec = precision;
  c->rule = rule;
  c->vrule = vrule;
  c->floor = floor;
  c->stream = static_cast<hipStream_t>(stream);
  c->ws = static_cast<char*>(workspace);
  c->lay = lay;
  c->plan = plan;
  c->vs = choose_vsplit(d, precision);
  // The bfloat16 activation partials keep their own launch; CTFISS_UNFUSED_NMF keeps the
  // separate partial-sum and final launches that batches run.
  c->vone = !unfused && precision != CTFISS_MIXED_BF16 && vupdate_pays(d, precision);
  c->ptr.X = nullptr;
  c->ptr.W = c->ws + lay.W;
  c->ptr.B = c->ws + lay.B;
  c->ptr.V = c->ws + lay.V;
  c->ptr.ilam = c->ws + lay.ilam;
  c->ptr.P = c->ws + lay.P;
  c->ptr.P0 = vrule == CTFISS_VRULE_PAPER_TAP0 ? static_cast<void*>(c->ws + lay.P0) : nullptr;
  c->ptr.musq = c->ws + lay.musq;
  c->ptr.mu = c->ws + lay.mu;
  c->ptr.vnum = c->ws + lay.vnum;
  c->ptr.vden = c->ws + lay.vden;
  c->ptr.nllpart = reinterpret_cast<double*>(c->ws + lay.nllpart);
  c->trace = reinterpret_cast<double*>(c->ws + lay.trace);
  c->ptr.status = reinterpret_cast<int*>(c->ws + lay.status);
  c->ptr.work = reinterpret_cast<int*>(c->ws + lay.work);
  c->ptr.Y = c->ws + lay.Y;
  c->ptr.xch = lay.team > 1 ? static_cast<void*>(c->ws + lay.xch) : nullptr;
  c->have_input = c->have_state = c->y_valid = false;
  c->epoch = 0;
  c->graph = false;
  c->prof = 0;
  for (int i = 0; i < kClasses; ++i) {
    c->launches[i] = 0;
    c->ms[i] = 0.0;
  }
  hipError_t ze = launch_zero_status(c->ptr.status, c->stream);
  // exchange words start untagged (every launch's tags are nonzero); cleared by a
  // kernel rather than a memset node, so that a caller may capture the call
  if (ze == hipSuccess && c->ptr.xch)
    ze = launch_zero_words(static_cast<unsigned long long*>(c->ptr.xch),
                           (size_t)d.F * team_words(d.Mb, d.lmax, lay.team, precision != CTFISS_FP64 ? 4 : 8), c->stream);
  return ze == hipSuccess ? CTFISS_OK : CTFISS_E_HIP;
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
  Dims d;
  Layout lay;
  int st = check_create_args(shape, precision, rule, vrule, floor, &d, &lay);
  if (st != CTFISS_OK) return st;
  if (workspace_bytes < lay.total || (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0)
    return CTFISS_E_WORKSPACE;
  ctfiss_ctx* c = new (std::nothrow) ctfiss_ctx();
  if (!c) return CTFISS_E_ARG;
  st = init_ctx(c, d, lay, precision, rule, vrule, floor, workspace, stream);
  if (st != CTFISS_OK) {
    delete c;
    return st;
  }
  *out = c;
  return CTFISS_OK;
}

int ctfiss_set_input(ctfiss_ctx* c, const void* X) {
  if (!c || !X) return CTFISS_E_ARG;
  if (X != c->ptr.X && !c->graphs.empty()) {  // captured launches hold the old pointer
    if (hipStreamSynchronize(c->stream) != hipSuccess) return CTFISS_E_HIP;
    drop_graphs(c);
  }
  c->ptr.X = X;
  c->have_input = true;
  c->y_valid = false;
  return CTFISS_OK;
}

int ctfiss_set_state(ctfiss_ctx* c, const void* W, const void* B, const void* V) {
  if (!c || !B || !V) return CTFISS_E_ARG;
  const Dims& d = c->d;
  const size_t rs = c->prec != CTFISS_FP64 ? 4 : 8;
  hipError_t e;
  if (W)
    e = hipMemcpyAsync(c->ptr.W, W, (size_t)d.F * d.Mb * d.Mb * 2 * rs, hipMemcpyDeviceToDevice, c->stream);
  else
    e = c->prec != CTFISS_FP64 ? identity_t<float>(d, c->ptr.W, c->stream) : identity_t<double>(d, c->ptr.W, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->ptr.B, B, (size_t)d.N * d.F * d.K * rs, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->ptr.V, V, (size_t)d.N * d.K * d.T * rs, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = launch_zero_status(c->ptr.status, c->stream);
  if (e != hipSuccess) return CTFISS_E_HIP;
  c->have_state = true;
  c->y_valid = false;
  return CTFISS_OK;
}

}  // extern "C"

namespace {

// The launches of n_iter iterations on the context's stream (updates the
// host-side state as the launches will leave the device state).
int enqueue_iterations(ctfiss_ctx* c, int32_t n_iter) {
  const bool tap0 = c->vrule == CTFISS_VRULE_PAPER_TAP0;
  const bool f32 = c->prec != CTFISS_FP64;
  const Dims& d = c->d;
  const Ptrs& p = c->ptr;
  hipStream_t s = c->stream;
  for (int it = 0; it < n_iter; ++it) {
    const bool mu = it > 0;  // the previous iteration's scale is still to be applied
    // 1/lambda: formed per bin by the W update itself (plan.nmf), else by its own launch
    const bool nmf = c->plan.nmf != 0;
    hipError_t e = hipSuccess;
    const bool bf = c->prec == CTFISS_MIXED_BF16;
    if (!nmf)
      e = timed(c, 5, [&] {
        return bf ? lambda_bf16_t(d, p, mu, s) : f32 ? lambda_t<float>(d, p, mu, s) : lambda_t<double>(d, p, mu, s);
      });
    c->epoch = c->epoch % 0x1FFFFFFu + 1u;  // tags epoch * 128 + step stay within 32 bits
    if (e == hipSuccess)
      e = timed(c, 0, [&] {
        if (wx(c->prec))
          return wupdate_t<float, true>(c->rule, c->plan, d, p, mu, c->y_valid, c->epoch, c->floor, s);
        return f32 ? wupdate_t<float>(c->rule, c->plan, d, p, mu, c->y_valid, c->epoch, c->floor, s)
                   : wupdate_t<double>(c->rule, c->plan, d, p, mu, c->y_valid, c->epoch, c->floor, s);
      });
    if (e == hipSuccess && c->rule == CTFISS_RULE_ISS) c->y_valid = true;
    if (e == hipSuccess && !nmf)
      e = timed(c, 6, [&] {
        return bf ? nmfb_bf16_t(d, p, c->floor, mu, s)
               : f32 ? nmfb_t<float>(d, p, c->floor, mu, s) : nmfb_t<double>(d, p, c->floor, mu, s);
      });
    if (e == hipSuccess && c->vone)
      e = timed(c, 2, [&] {
        return f32 ? vupdate_t<float>(d, p, c->floor, tap0, s) : vupdate_t<double>(d, p, c->floor, tap0, s);
      });
    if (e == hipSuccess && !c->vone)
      e = timed(c, 1, [&] {
        return bf ? vpart_bf16_t(d, c->vs, p, tap0, s)
               : f32 ? vpart_t<float>(d, c->vs, p, tap0, s) : vpart_t<double>(d, c->vs, p, tap0, s);
      });
    if (e == hipSuccess && !c->vone)
      e = timed(c, 2, [&] {
        return f32 ? vfinal_t<float>(d, c->vs, p, c->floor, tap0, s) : vfinal_t<double>(d, c->vs, p, c->floor, tap0, s);
      });
    if (e != hipSuccess) return CTFISS_E_HIP;
  }
  if (n_iter > 0) {
    const bool sy = c->y_valid;
    hipError_t e = timed(c, 3, [&] { return f32 ? apply_mu_t<float>(d, p, sy, s) : apply_mu_t<double>(d, p, sy, s); });
    if (e != hipSuccess) return CTFISS_E_HIP;
  }
  return CTFISS_OK;
}

// Iterations one at a time, each followed by the objective of Eq. (5) at the
// state it leaves (its rescale applied, as at the end of any call): per-bin
// parts by k_nll, summed on the device into the trace; read back every
// kTraceCap iterations.  A run of one-iteration calls gives the same state,
// bit for bit, as one call of n_iter iterations.
int iterate_traced(ctfiss_ctx* c, int32_t n_iter, double* out) {
  const bool f32 = c->prec != CTFISS_FP64;
  for (int done = 0; done < n_iter;) {
    const int chunk = n_iter - done < kTraceCap ? n_iter - done : kTraceCap;
    for (int i = 0; i < chunk; ++i) {
      const int st = enqueue_iterations(c, 1);
      if (st != CTFISS_OK) return st;
      hipError_t e = f32 ? nll_t<float>(c->d, c->ptr, c->stream) : nll_t<double>(c->d, c->ptr, c->stream);
      if (e == hipSuccess) e = launch_sum_parts(c->ptr.nllpart, c->d.F, c->trace + i, c->stream);
      if (e != hipSuccess) return CTFISS_E_HIP;
    }
    hipError_t e = hipMemcpyAsync(out + done, c->trace, (size_t)chunk * sizeof(double), hipMemcpyDeviceToHost,
                                  c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return CTFISS_E_HIP;
    done += chunk;
  }
  return CTFISS_OK;
}

}  // namespace

extern "C" {

int ctfiss_iterate(ctfiss_ctx* c, int32_t n_iter, double* nll_host) {
  if (!c || n_iter < 0) return CTFISS_E_ARG;
  if (!c->have_input || !c->have_state) return CTFISS_E_ORDER;
  if (nll_host) return iterate_traced(c, n_iter, nll_host);
  if (!c->graph || n_iter == 0 || c->prof != 0) return enqueue_iterations(c, n_iter);
  // graph mode: one captured graph per (n_iter, carried Y valid at the start);
  // every argument of the launches is fixed per context, so a replay is the
  // same work as the launches it was captured from
  const bool yv = c->y_valid;
  for (auto& g : c->graphs) {
    if (g.n == n_iter && g.y_valid == yv) {
      if (hipGraphLaunch(g.exec, c->stream) != hipSuccess) return CTFISS_E_HIP;
      if (c->rule == CTFISS_RULE_ISS) c->y_valid = true;
      return CTFISS_OK;
    }
  }
  if (c->graphs.size() >= 8) drop_graphs(c);
  hipGraph_t graph = nullptr;
  if (hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return CTFISS_E_HIP;
  const int st = enqueue_iterations(c, n_iter);
  const hipError_t ee = hipStreamEndCapture(c->stream, &graph);
  if (st != CTFISS_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (ee != hipSuccess || !graph) return CTFISS_E_HIP;
  hipGraphExec_t exec = nullptr;
  const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) return CTFISS_E_HIP;
  c->graphs.push_back({n_iter, yv, exec});
  return hipGraphLaunch(exec, c->stream) == hipSuccess ? CTFISS_OK : CTFISS_E_HIP;
}

int ctfiss_set_graph(ctfiss_ctx* c, int enable) {
  if (!c) return CTFISS_E_ARG;
  if (enable) {
    // team launches take a new tag base per launch; capture needs a created stream
    if (c->plan.team > 1 || c->stream == nullptr) return CTFISS_E_UNSUPPORTED;
  } else if (!c->graphs.empty()) {
    if (hipStreamSynchronize(c->stream) != hipSuccess) return CTFISS_E_HIP;
    drop_graphs(c);
  }
  c->graph = enable != 0;
  return CTFISS_OK;
}

int ctfiss_get_state(ctfiss_ctx* c, void* W, void* B, void* V) {
  if (!c) return CTFISS_E_ARG;
  if (!c->have_state) return CTFISS_E_ORDER;
  const Dims& d = c->d;
  const size_t rs = c->prec != CTFISS_FP64 ? 4 : 8;
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
  hipError_t e = timed(c, 4, [&] {
    return c->prec != CTFISS_FP64 ? images_t<float>(c->d, c->ptr, C, c->stream) : images_t<double>(c->d, c->ptr, C, c->stream);
  });
  return e == hipSuccess ? CTFISS_OK : CTFISS_E_HIP;
}

int ctfiss_nll(ctfiss_ctx* c, double* out) {
  if (!c || !out) return CTFISS_E_ARG;
  if (!c->have_input || !c->have_state) return CTFISS_E_ORDER;
  std::vector<double> part((size_t)c->d.F);
  hipError_t e = c->prec != CTFISS_FP64 ? nll_t<float>(c->d, c->ptr, c->stream) : nll_t<double>(c->d, c->ptr, c->stream);
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
  // enqueued work keeps running (kernels hold no pointer to the context);
  // only pending timing events and captured graphs are waited for
  if (!c->timed.empty() || !c->graphs.empty()) (void)hipStreamSynchronize(c->stream);
  drop_graphs(c);
  for (const TimedLaunch& t : c->timed) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (hipEvent_t ev : c->pool) (void)hipEventDestroy(ev);
  delete c;
  return CTFISS_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ static scratch
// The workspace of ctfiss_separate_noalloc: a fixed device array, one copy per
// GPU the library runs on, held until the process ends.  Host code never
// passes `scratch` itself to the device (on the host the name stands for a
// host-side shadow); it uses the device address hipGetSymbolAddress returns,
// looked up once per device with that device current.
namespace {
constexpr size_t kStaticScratchBytes = (size_t)96 << 20;
constexpr int kMaxScratchDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

std::mutex& scratch_mutex() {
  static std::mutex m;
  return m;
}

// Device address of the current device's copy of `scratch`.
int static_scratch(void** out) {
  static void* addr[kMaxScratchDevices] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CTFISS_E_HIP;
  if (dev < 0 || dev >= kMaxScratchDevices) return CTFISS_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(scratch_mutex());
  if (!addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CTFISS_E_HIP;
    addr[dev] = p;
  }
  *out = addr[dev];
  return CTFISS_OK;
}

}  // namespace

extern "C" {

int ctfiss_separate_noalloc(const ctfiss_shape* shape, int precision, int rule, int vrule, double floor,
                            const void* X, const void* W0, const void* B0, const void* V0, int32_t n_iter, void* C,
                            void* W, void* B, void* V, int32_t* status, void* stream) {
  if (!X || !B0 || !V0 || n_iter < 0) return CTFISS_E_ARG;
  Dims d;
  Layout lay;
  int st = check_create_args(shape, precision, rule, vrule, floor, &d, &lay);
  if (st != CTFISS_OK) return st;
  if (lay.total > kStaticScratchBytes) return CTFISS_E_TOO_LARGE;
  void* ws = nullptr;
  st = static_scratch(&ws);
  if (st != CTFISS_OK) return st;
  // the calls a caller with its own workspace makes, on a context held on the stack
  // (no graphs, no profiling events: it owns no resources)
  ctfiss_ctx c{};
  st = init_ctx(&c, d, lay, precision, rule, vrule, floor, ws, stream);
  if (st == CTFISS_OK) st = ctfiss_set_input(&c, X);
  if (st == CTFISS_OK) st = ctfiss_set_state(&c, W0, B0, V0);
  if (st == CTFISS_OK) st = ctfiss_iterate(&c, n_iter, nullptr);
  if (st == CTFISS_OK && C) st = ctfiss_source_images(&c, C);
  if (st == CTFISS_OK) st = ctfiss_get_state(&c, W, B, V);
  if (st == CTFISS_OK && status &&
      hipMemcpyAsync(status, c.ptr.status, sizeof(int32_t), hipMemcpyDeviceToDevice, c.stream) != hipSuccess)
    st = CTFISS_E_HIP;
  return st;
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
    case CTFISS_E_TOO_LARGE: return "workspace of this shape exceeds the library's static scratch";
    default: return "unknown status";
  }
}

// ------------------------------------------------------------------ reverse mode
}  // extern "C"

namespace {

struct AdjLayout {
  size_t ckW, ckB, ckV, gW, gB, gBh, gV, gVh, gP, gP0, glam, glamh, lamh, q1, q2, G1, G2, H1, H2, part, gS, Y, gY, gphi,
      zt, dt, l2sums, total;
};

AdjLayout adj_layout(const Dims& d, int n_iter, size_t rs) {
  AdjLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, kAlign);
    return o;
  };
  const size_t cs = 2 * rs;
  const size_t w = (size_t)d.F * d.Mb * d.Mb * cs, b = (size_t)d.N * d.F * d.K * rs, v = (size_t)d.N * d.K * d.T * rs;
  const size_t ft = (size_t)d.N * d.F * d.T * rs, yt = (size_t)d.F * d.Mb * d.T;
  L.ckW = take((n_iter + 1) * w);
  L.ckB = take((n_iter + 1) * b);
  L.ckV = take((n_iter + 1) * v);
  L.gW = take(w);
  L.gB = take(b);
  L.gBh = take(b);
  L.gV = take(v);
  L.gVh = take(v);
  L.gP = take(ft);
  L.gP0 = take(ft);
  L.glam = take(ft);
  L.glamh = take(ft);
  L.lamh = take(ft);
  L.q1 = take(ft);
  L.q2 = take(ft);
  L.G1 = take(v);
  L.G2 = take(v);
  L.H1 = take(b);
  L.H2 = take(b);
  L.part = take((size_t)d.F * (d.Mb + d.N) * rs);
  L.gS = take((size_t)d.Mb * rs);
  L.Y = take(yt * cs);
  L.gY = take(yt * cs);
  L.gphi = take(yt * rs);
  L.zt = take(w);
  L.dt = take((size_t)d.F * d.Mb * d.Mb * rs);
  L.l2sums = take((size_t)adj_l2_chunks(d.F) * d.N * d.K * d.T * rs);
  L.total = off;
  return L;
}

// Reverse mode is built for FP32, FP64 and mixed ISS contexts (either
// activation rule) whose per-bin adjoint kernels fit LDS: every Mbar in FP32
// and mixed precision, Mbar <= 56 in FP64 (the images adjoint holds W, its
// augmented inverse and the image gradients of a bin, 3 Mbar^2 + 2 M Mbar + Mbar
// complex values).
bool adj_supported(const Dims& d, int rs) {
  return adj_iss_lds(d.Mb, d.T, rs) <= kMaxLdsBytes && adj_images_lds(d.Mb, d.M, rs) <= kMaxLdsBytes;
}

}  // namespace

extern "C" {

int ctfiss_adjoint_workspace_size(const ctfiss_shape* shape, int precision, int32_t n_iter, size_t* bytes) {
  if (!bytes || n_iter < 1) return CTFISS_E_ARG;
  if (precision != CTFISS_FP32 && precision != CTFISS_FP64 && precision != CTFISS_MIXED) return CTFISS_E_UNSUPPORTED;
  Dims d;
  const int st = validate_shape(shape, precision, &d);
  if (st != CTFISS_OK) return st;
  const int rs = precision == CTFISS_FP64 ? 8 : 4;
  if (!adj_supported(d, rs)) return CTFISS_E_UNSUPPORTED;
  *bytes = adj_layout(d, n_iter, rs).total;
  return CTFISS_OK;
}

int ctfiss_backward(ctfiss_ctx* c, int32_t n_iter, const void* B0, const void* V0, const void* gC, void* gX,
                    void* gB0, void* gV0, void* aws, size_t aws_bytes) {
  if (!c || !B0 || !V0 || !gC || !gX || !aws || n_iter < 1) return CTFISS_E_ARG;
  if (c->prec == CTFISS_MIXED_BF16 || c->rule != CTFISS_RULE_ISS) return CTFISS_E_UNSUPPORTED;
  const Dims& d = c->d;
  const bool f32 = c->prec != CTFISS_FP64;  // FP32, or mixed: FP32 data and adjoint kernels
  const bool tap0 = c->vrule == CTFISS_VRULE_PAPER_TAP0;
  const int rs = f32 ? 4 : 8;
  if (!adj_supported(d, rs)) return CTFISS_E_UNSUPPORTED;
  if (!c->have_input) return CTFISS_E_ORDER;
  const AdjLayout L = adj_layout(d, n_iter, (size_t)rs);
  if (aws_bytes < L.total || (reinterpret_cast<uintptr_t>(aws) % kAlign) != 0) return CTFISS_E_WORKSPACE;
  char* ws = static_cast<char*>(aws);
  hipStream_t s = c->stream;
  const size_t wb = (size_t)d.F * d.Mb * d.Mb * 2 * rs, bb = (size_t)d.N * d.F * d.K * rs,
               vb = (size_t)d.N * d.K * d.T * rs;
  auto cp = [&](void* dst, const void* src, size_t n) { return hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToDevice, s); };
  // forward from (I, B0, V0) with the state saved before every iteration and after the last
  hipError_t e = f32 ? identity_t<float>(d, c->ptr.W, s) : identity_t<double>(d, c->ptr.W, s);
  if (e == hipSuccess) e = cp(c->ptr.B, B0, bb);
  if (e == hipSuccess) e = cp(c->ptr.V, V0, vb);
  if (e == hipSuccess) e = launch_zero_status(c->ptr.status, s);
  if (e != hipSuccess) return CTFISS_E_HIP;
  c->have_state = true;
  c->y_valid = false;
  for (int k = 0; k <= n_iter; ++k) {
    e = launch_copy3(ws + L.ckW + k * wb, c->ptr.W, wb, ws + L.ckB + k * bb, c->ptr.B, bb, ws + L.ckV + k * vb,
                     c->ptr.V, vb, s);
    if (e != hipSuccess) return CTFISS_E_HIP;
    if (k < n_iter) {
      const int st = ctfiss_iterate(c, 1, nullptr);
      if (st != CTFISS_OK) return st;
    }
  }
  AdjPtrs p{};
  p.X = c->ptr.X;
  p.gW = ws + L.gW;
  p.gB = ws + L.gB;
  p.gV = ws + L.gV;
  p.gBh = ws + L.gBh;
  p.gVh = ws + L.gVh;
  p.gP = ws + L.gP;
  p.gP0 = tap0 ? ws + L.gP0 : nullptr;
  p.glam = ws + L.glam;
  p.glamh = ws + L.glamh;
  p.lamh = ws + L.lamh;
  p.q1 = ws + L.q1;
  p.q2 = ws + L.q2;
  p.G1 = ws + L.G1;
  p.G2 = ws + L.G2;
  p.H1 = ws + L.H1;
  p.H2 = ws + L.H2;
  p.part = ws + L.part;
  p.gS = ws + L.gS;
  p.gX = gX;
  p.status = c->ptr.status;
  p.Y = ws + L.Y;
  p.gY = ws + L.gY;
  p.gphi = ws + L.gphi;
  p.ztape = ws + L.zt;
  p.dtape = ws + L.dt;
  p.l2sums = ws + L.l2sums;
  // the iterations re-run below stop before the rescale and need lambda, the basis
  // update and the activation update from their own launches
  Plan sep = c->plan;
  if (sep.nmf) {
    sep.nmf = 0;
    sep.lds = wupdate_lds(c->rule, sep, d, rs);
  }
  // images: the first contributions to gW and gX
  e = adj_images(p, d, c->ptr.W, gC, rs, s);
  if (e == hipSuccess) e = hipMemsetAsync(p.gB, 0, bb, s);
  if (e == hipSuccess) e = hipMemsetAsync(p.gV, 0, vb, s);
  for (int k = n_iter - 1; k >= 0 && e == hipSuccess; --k) {
    // iteration k again from its saved state, stopping before the rescale is
    // applied: W = W^s, B = B^, V = V^, mu, P and 1/lambda of iteration k
    e = launch_copy3(c->ptr.W, ws + L.ckW + k * wb, wb, c->ptr.B, ws + L.ckB + k * bb, bb, c->ptr.V,
                     ws + L.ckV + k * vb, vb, s);
    c->epoch = c->epoch % 0x1FFFFFFu + 1u;
    if (f32) {
      if (e == hipSuccess) e = lambda_t<float>(d, c->ptr, false, s);
      if (e == hipSuccess)
        e = wx(c->prec) ? wupdate_t<float, true>(c->rule, sep, d, c->ptr, false, false, c->epoch, c->floor, s)
                        : wupdate_t<float>(c->rule, sep, d, c->ptr, false, false, c->epoch, c->floor, s);
      if (e == hipSuccess) e = nmfb_t<float>(d, c->ptr, c->floor, false, s);
      if (e == hipSuccess && c->vone) e = vupdate_t<float>(d, c->ptr, c->floor, tap0, s);
      if (e == hipSuccess && !c->vone) e = vpart_t<float>(d, c->vs, c->ptr, tap0, s);
      if (e == hipSuccess && !c->vone) e = vfinal_t<float>(d, c->vs, c->ptr, c->floor, tap0, s);
    } else {
      if (e == hipSuccess) e = lambda_t<double>(d, c->ptr, false, s);
      if (e == hipSuccess) e = wupdate_t<double>(c->rule, sep, d, c->ptr, false, false, c->epoch, c->floor, s);
      if (e == hipSuccess) e = nmfb_t<double>(d, c->ptr, c->floor, false, s);
      if (e == hipSuccess && c->vone) e = vupdate_t<double>(d, c->ptr, c->floor, tap0, s);
      if (e == hipSuccess && !c->vone) e = vpart_t<double>(d, c->vs, c->ptr, tap0, s);
      if (e == hipSuccess && !c->vone) e = vfinal_t<double>(d, c->vs, c->ptr, c->floor, tap0, s);
    }
    if (e != hipSuccess) break;
    p.Wk = ws + L.ckW + k * wb;
    p.Bk = ws + L.ckB + k * bb;
    p.Vk = ws + L.ckV + k * vb;
    p.Ws = c->ptr.W;
    p.Bh = c->ptr.B;
    p.Vh = c->ptr.V;
    p.ilam = c->ptr.ilam;
    p.P = c->ptr.P;
    p.P0 = c->ptr.P0;
    p.mu = c->ptr.mu;
    e = adj_iteration(p, d, c->floor, rs, s);
  }
  if (e == hipSuccess && gB0) e = cp(gB0, p.gB, bb);
  if (e == hipSuccess && gV0) e = cp(gV0, p.gV, vb);
  // the context ends in the forward's final state
  if (e == hipSuccess)
    e = launch_copy3(c->ptr.W, ws + L.ckW + n_iter * wb, wb, c->ptr.B, ws + L.ckB + n_iter * bb, bb, c->ptr.V,
                     ws + L.ckV + n_iter * vb, vb, s);
  c->y_valid = false;
  return e == hipSuccess ? CTFISS_OK : CTFISS_E_HIP;
}

int ctfiss_get_plan(ctfiss_ctx* c, int32_t* G, int32_t* cpl, int32_t* rpl, int32_t* team) {
  if (!c) return CTFISS_E_ARG;
  if (G) *G = c->plan.G;
  if (cpl) *cpl = c->plan.CPL;
  if (rpl) *rpl = c->plan.RPL;
  if (team) *team = c->plan.team;
  return CTFISS_OK;
}

int ctfiss_get_nmf_path(ctfiss_ctx* c, int32_t* fused, int32_t* v_one_launch) {
  if (!c) return CTFISS_E_ARG;
  if (fused) *fused = c->plan.nmf;
  if (v_one_launch) *v_one_launch = c->vone ? 1 : 0;
  return CTFISS_OK;
}

int ctfiss_clear_tuned_plans(void) {
  std::lock_guard<std::mutex> lock(tune_mutex());
  tune_cache().clear();
  return CTFISS_OK;
}

int ctfiss_autotune_scratch_size(ctfiss_ctx* c, size_t* bytes) {
  if (!c || !bytes) return CTFISS_E_ARG;
  const Dims& d = c->d;
  const size_t rs = c->prec != CTFISS_FP64 ? 4 : 8;
  *bytes = align_up((size_t)d.F * d.Mb * d.Mb * 2 * rs, kAlign) + align_up((size_t)d.N * d.F * d.K * rs, kAlign) +
           align_up((size_t)d.N * d.K * d.T * rs, kAlign);
  return CTFISS_OK;
}

}  // extern "C"

namespace {

// Device status word of a context (synchronises the stream).
hipError_t read_status(ctfiss_ctx* c, int* code) {
  hipError_t e = hipMemcpyAsync(code, c->ptr.status, sizeof(int), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return e;
}

}  // namespace

extern "C" {

int ctfiss_autotune(ctfiss_ctx* c, int32_t trials, void* scratch, size_t scratch_bytes) {
  if (!c || trials < 1 || !scratch) return CTFISS_E_ARG;
  if (!c->have_input || !c->have_state) return CTFISS_E_ORDER;
  if (c->graph) return CTFISS_E_UNSUPPORTED;  // captured graphs hold the current plan
  size_t need = 0;
  (void)ctfiss_autotune_scratch_size(c, &need);
  if (scratch_bytes < need || (reinterpret_cast<uintptr_t>(scratch) % kAlign) != 0) return CTFISS_E_WORKSPACE;
  const Dims& d = c->d;
  int dev = 0, max_lds = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return CTFISS_E_HIP;
  // a fault latched before the call stays latched (and nothing is timed on faulted data)
  int code = 0;
  if (read_status(c, &code) != hipSuccess) return CTFISS_E_HIP;
  if (code != 0) return CTFISS_E_NUMERIC;
  // candidates: every instantiated (G, RPL) with its smallest fitting frames per lane; team
  // shapes only where the default plan is a team plan (the workspace holds their exchange words)
  std::vector<Plan> cand;
  const int Gs[] = {16, 32, 64};
  for (int G : Gs)
    for (int rpl = 1; rpl <= 2; ++rpl) {
      Plan p;
      if (c->plan.team > 1) {
        for (int P = 2; P <= c->lay.team; ++P)
          if (plan_for_team(c->prec, d, (size_t)max_lds, G, rpl, P, 0, &p)) cand.push_back(p);
      } else if (plan_for(c->prec, c->rule, d, (size_t)max_lds, G, rpl, 0, &p)) {
        cand.push_back(p);
      }
    }
  if (cand.empty()) return CTFISS_OK;
  // time the W update on the context's own data; the state is restored from
  // the caller's scratch afterwards
  const size_t rs = c->prec != CTFISS_FP64 ? 4 : 8;
  const size_t wb = (size_t)d.F * d.Mb * d.Mb * 2 * rs, bb = (size_t)d.N * d.F * d.K * rs, vb = (size_t)d.N * d.K * d.T * rs;
  char* save = static_cast<char*>(scratch);
  char* saveB = save + align_up(wb, kAlign);
  char* saveV = saveB + align_up(bb, kAlign);
  hipError_t e = hipMemcpyAsync(save, c->ptr.W, wb, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(saveB, c->ptr.B, bb, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(saveV, c->ptr.V, vb, hipMemcpyDeviceToDevice, c->stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  const Plan keep = c->plan;
  Plan best = keep;
  float best_ms = -1.f;
  const bool f32 = c->prec != CTFISS_FP64;
  for (size_t i = 0; i < cand.size() && e == hipSuccess; ++i) {
    Plan p = cand[i];
    if (c->plan.nmf && p.team <= 1) {  // the fused form the context took, activations in LDS if they fit
      p.nmf = c->plan.nmf;
      p.lds = wupdate_lds(c->rule, p, d, (int)rs);
      if (p.lds > (size_t)max_lds && p.nmf == 1) {
        p.nmf = 2;
        p.lds = wupdate_lds(c->rule, p, d, (int)rs);
      }
      if (p.lds > (size_t)max_lds) continue;
    }
    p.blocks = wx(c->prec) ? resident_wblocks<float, true>(c->rule, p, d)
               : f32                   ? resident_wblocks<float>(c->rule, p, d)
                                       : resident_wblocks<double>(c->rule, p, d);
    if (p.blocks < 1 || (p.team > 1 && p.blocks < p.team)) continue;
    float total = 0.f;
    for (int t = 0; t <= trials && e == hipSuccess; ++t) {  // the first run warms up
      e = f32 ? lambda_t<float>(d, c->ptr, false, c->stream) : lambda_t<double>(d, c->ptr, false, c->stream);
      c->epoch = c->epoch % 0x1FFFFFFu + 1u;
      if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
      if (e == hipSuccess) {
        if (wx(c->prec))
          e = wupdate_t<float, true>(c->rule, p, d, c->ptr, false, false, c->epoch, c->floor, c->stream);
        else if (f32)
          e = wupdate_t<float>(c->rule, p, d, c->ptr, false, false, c->epoch, c->floor, c->stream);
        else
          e = wupdate_t<double>(c->rule, p, d, c->ptr, false, false, c->epoch, c->floor, c->stream);
      }
      if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (t > 0) total += ms;
      // back to the saved state for the next run (a W update with the basis update
      // folded in also changes B)
      if (e == hipSuccess) e = hipMemcpyAsync(c->ptr.W, save, wb, hipMemcpyDeviceToDevice, c->stream);
      if (e == hipSuccess && p.nmf) e = hipMemcpyAsync(c->ptr.B, saveB, bb, hipMemcpyDeviceToDevice, c->stream);
    }
    // a candidate whose runs latched a fault (e.g. a team wait that ran out) is not taken
    int fc = 0;
    if (e == hipSuccess) e = read_status(c, &fc);
    if (e == hipSuccess && fc != 0) {
      e = launch_zero_status(c->ptr.status, c->stream);
      continue;
    }
    if (e == hipSuccess && (best_ms < 0.f || total < best_ms)) {
      best_ms = total;
      best = p;
    }
  }
  if (e == hipSuccess) e = hipMemcpyAsync(c->ptr.W, save, wb, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(c->ptr.B, saveB, bb, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(c->ptr.V, saveV, vb, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);  // the scratch is the caller's again on return
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  c->y_valid = false;
  if (e != hipSuccess) {
    c->plan = keep;
    return CTFISS_E_HIP;
  }
  c->plan = best;
  {
    std::lock_guard<std::mutex> lock(tune_mutex());
    const TuneKey k = tune_key(c->prec, c->rule, d);
    bool found = false;
    for (auto& te : tune_cache())
      if (te.key == k) {
        te.plan = best;
        found = true;
      }
    if (!found) tune_cache().push_back({k, best});
  }
  return CTFISS_OK;
}

int ctfiss_set_profiling(ctfiss_ctx* c, int mask) {
  if (!c) return CTFISS_E_ARG;
  if (drain_timing(c) != hipSuccess) return CTFISS_E_HIP;
  c->prof = mask;
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


// ------------------------------------------------------------------ batches
}  // extern "C"

struct ctfiss_batch {
  int n, prec, rule;
  hipStream_t stream;
  char* ws;
  std::vector<ctfiss_ctx*> ctx;
  struct Bucket {
    Plan plan;
    std::vector<int> mix;  // mixture indices, in table order
    int wbase;             // first descriptor slot of the bucket in each variant table
    int sbase;             // first int of the bucket's start[] in the start region
    size_t lds;
    int blocks;
  };
  std::vector<Bucket> buckets;
  // W updates of different launch shapes overlap: bucket k runs on lane[k] (0: the batch's
  // stream, j > 0: side[j - 1]), forked from and joined to the batch's stream by events
  std::vector<hipStream_t> side;
  std::vector<int> lane;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  // device tables (offsets into ws) and their host images
  size_t off_w, off_ws, off_cnt, off_n, off_ns, tab_bytes, wsz, nsz;
  int nblocks[4], nmfb_threads;
  std::vector<unsigned char> host;
  bool have_input, have_state, y_valid;
  bool graph;  // ctfiss_batch_iterate replays captured HIP graphs
  struct GraphEntry {
    int n;
    bool y_valid;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
};

namespace {

size_t batch_tables_bytes(int n, size_t wsz, size_t nsz) {
  // W descriptors: 3 variants x n; W starts: 2n + 2 ints; counters: n ints;
  // NMF descriptors: (2 + 2 + 1 + 1) x n; NMF starts: 4 (n + 1) ints
  size_t b = 0;
  b = align_up(b + 3 * (size_t)n * wsz, kAlign);
  b = align_up(b + (2 * (size_t)n + 2) * sizeof(int), kAlign);
  b = align_up(b + (size_t)n * sizeof(int), kAlign);
  b = align_up(b + 6 * (size_t)n * nsz, kAlign);
  b = align_up(b + 4 * ((size_t)n + 1) * sizeof(int), kAlign);
  return b;
}

size_t desc_w_bytes(int prec) { return prec != CTFISS_FP64 ? wdesc_bytes<float>() : wdesc_bytes<double>(); }
size_t desc_n_bytes(int prec) { return prec != CTFISS_FP64 ? ndesc_bytes<float>() : ndesc_bytes<double>(); }

}  // namespace

extern "C" {

int ctfiss_batch_workspace_size(const ctfiss_shape* shapes, int32_t n, int precision, size_t* bytes) {
  if (!shapes || !bytes || n < 1) return CTFISS_E_ARG;
  size_t total = 0;
  for (int i = 0; i < n; ++i) {
    size_t b = 0;
    const int st = ctfiss_workspace_size(&shapes[i], precision, &b);
    if (st != CTFISS_OK) return st;
    total = align_up(total + b, kAlign);
  }
  *bytes = total + batch_tables_bytes(n, desc_w_bytes(precision), desc_n_bytes(precision));
  return CTFISS_OK;
}

int ctfiss_batch_destroy(ctfiss_batch* b) {
  if (!b) return CTFISS_E_ARG;
  if (!b->graphs.empty() || !b->side.empty()) (void)hipStreamSynchronize(b->stream);
  for (auto& g : b->graphs) (void)hipGraphExecDestroy(g.exec);
  b->graphs.clear();
  for (hipStream_t x : b->side) {
    (void)hipStreamSynchronize(x);
    (void)hipStreamDestroy(x);
  }
  for (hipEvent_t x : b->join) (void)hipEventDestroy(x);
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (ctfiss_ctx* c : b->ctx)
    if (c) ctfiss_destroy(c);
  delete b;
  return CTFISS_OK;
}

int ctfiss_batch_create(const ctfiss_shape* shapes, int32_t n, int precision, int rule, int vrule, double floor,
                        void* workspace, size_t workspace_bytes, void* stream, ctfiss_batch** out) {
  if (!out || !workspace) return CTFISS_E_ARG;
  size_t need = 0;
  int st = ctfiss_batch_workspace_size(shapes, n, precision, &need);
  if (st != CTFISS_OK) return st;
  if (workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0) return CTFISS_E_WORKSPACE;
  if (wx(precision)) return CTFISS_E_UNSUPPORTED;  // batched W updates run FP32 or FP64 rows
  ctfiss_batch* b = new (std::nothrow) ctfiss_batch();
  if (!b) return CTFISS_E_ARG;
  b->n = n;
  b->prec = precision;
  b->rule = rule;
  b->stream = static_cast<hipStream_t>(stream);
  b->ws = static_cast<char*>(workspace);
  b->have_input = b->have_state = b->y_valid = false;
  b->graph = false;
  size_t off = 0;
  for (int i = 0; i < n; ++i) {
    size_t wb = 0;
    ctfiss_workspace_size(&shapes[i], precision, &wb);
    ctfiss_ctx* c = nullptr;
    st = ctfiss_create(&shapes[i], precision, rule, vrule, floor, b->ws + off, wb, stream, &c);
    if (st != CTFISS_OK) {
      ctfiss_batch_destroy(b);
      return st;
    }
    b->ctx.push_back(c);
    off = align_up(off + wb, kAlign);
    if (c->plan.team > 1) {  // batched launches take one workgroup per bin
      ctfiss_batch_destroy(b);
      return CTFISS_E_UNSUPPORTED;
    }
  }
  b->wsz = desc_w_bytes(precision);
  b->nsz = desc_n_bytes(precision);
  b->off_w = off;
  b->off_ws = align_up(b->off_w + 3 * (size_t)n * b->wsz, kAlign);
  b->off_cnt = align_up(b->off_ws + (2 * (size_t)n + 2) * sizeof(int), kAlign);
  b->off_n = align_up(b->off_cnt + (size_t)n * sizeof(int), kAlign);
  b->off_ns = align_up(b->off_n + 6 * (size_t)n * b->nsz, kAlign);
  b->tab_bytes = align_up(b->off_ns + 4 * ((size_t)n + 1) * sizeof(int), kAlign) - b->off_w;
  // bucket the mixtures by launch shape of their W update
  int wbase = 0, sbase = 0;
  for (int i = 0; i < n; ++i) {
    const Plan& p = b->ctx[i]->plan;
    ctfiss_batch::Bucket* bk = nullptr;
    for (auto& x : b->buckets)
      if (x.plan.G == p.G && x.plan.CPL == p.CPL && x.plan.RPL == p.RPL && x.plan.threads == p.threads) bk = &x;
    if (!bk) {
      b->buckets.push_back(ctfiss_batch::Bucket{p, {}, 0, 0, 0, 0});
      bk = &b->buckets.back();
    }
    bk->mix.push_back(i);
    const size_t lds = iter_lds_layout(b->ctx[i]->d.M, b->ctx[i]->d.T, b->ctx[i]->d.D, b->ctx[i]->d.Mb,
                                       b->ctx[i]->d.N, b->ctx[i]->d.lmax, p.G, p.CPL,
                                       precision != CTFISS_FP64 ? 4 : 8, rule != 0)
                           .total;
    if (lds > bk->lds) bk->lds = lds;
  }
  if (b->buckets.size() > 256) {  // the lambda launch resets one counter per thread
    ctfiss_batch_destroy(b);
    return CTFISS_E_UNSUPPORTED;
  }
  for (auto& bk : b->buckets) {
    bk.wbase = wbase;
    bk.sbase = sbase;
    wbase += (int)bk.mix.size();
    sbase += (int)bk.mix.size() + 1;
    int bins = 0;
    for (int i : bk.mix) bins += b->ctx[i]->d.F;
    const int res = rule == CTFISS_RULE_ISS ? (precision != CTFISS_FP64 ? resident_wblocks_batch<float>(bk.plan, bk.lds)
                                                                        : resident_wblocks_batch<double>(bk.plan, bk.lds))
                                            : 1;
    if (res < 1) {
      ctfiss_batch_destroy(b);
      return CTFISS_E_UNSUPPORTED;
    }
    bk.blocks = res < bins ? res : bins;
  }
  // Streams for the W updates of the launch shapes: the buckets, largest first (by
  // sum of F T Mbar^2, the sweep's work), each to the least loaded of up to four
  // streams (the batch's and three side streams of default priority; a process has
  // four hardware queues), so that one launch's last round overlaps the next one's.
  // The persistent workgroups of concurrent launches take their items from separate
  // counters; a bin's arithmetic does not depend on which launch shares the device.
  if (rule == CTFISS_RULE_ISS && b->buckets.size() > 1) {
    const int nl = b->buckets.size() < 4 ? (int)b->buckets.size() : 4;
    std::vector<double> work(b->buckets.size(), 0.0), load(nl, 0.0);
    std::vector<int> order(b->buckets.size());
    for (size_t k = 0; k < b->buckets.size(); ++k) {
      order[k] = (int)k;
      for (int i : b->buckets[k].mix) {
        const Dims& d = b->ctx[i]->d;
        work[k] += (double)d.F * d.T * d.Mb * d.Mb;
      }
    }
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });
    b->lane.assign(b->buckets.size(), 0);
    for (int k : order) {
      int best = 0;
      for (int j = 1; j < nl; ++j)
        if (load[j] < load[best]) best = j;
      b->lane[k] = best;
      load[best] += work[k];
    }
    hipError_t e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    for (int j = 1; j < nl && e == hipSuccess; ++j) {
      hipStream_t x = nullptr;
      hipEvent_t ev = nullptr;
      e = hipStreamCreateWithFlags(&x, hipStreamNonBlocking);
      if (e == hipSuccess) b->side.push_back(x);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (e == hipSuccess) b->join.push_back(ev);
    }
    if (e != hipSuccess) {
      ctfiss_batch_destroy(b);
      return CTFISS_E_HIP;
    }
  }
  b->host.assign(b->tab_bytes, 0);
  *out = b;
  return CTFISS_OK;
}

int ctfiss_batch_set_input(ctfiss_batch* b, const void* const* X) {
  if (!b || !X) return CTFISS_E_ARG;
  for (int i = 0; i < b->n; ++i) {
    const int st = ctfiss_set_input(b->ctx[i], X[i]);
    if (st != CTFISS_OK) return st;
  }
  const bool f32 = b->prec != CTFISS_FP64;
  unsigned char* h = b->host.data();
  auto at = [&](size_t off) { return h + (off - b->off_w); };
  // W-update tables: per bucket, variants (no pending scale, demix), (pending scale, carried Y),
  // (no pending scale, carried Y)
  for (const auto& bk : b->buckets) {
    int* start = reinterpret_cast<int*>(at(b->off_ws)) + bk.sbase;
    int acc = 0;
    for (size_t j = 0; j < bk.mix.size(); ++j) {
      const ctfiss_ctx* c = b->ctx[bk.mix[j]];
      start[j] = acc;
      acc += c->d.F;
      for (int v = 0; v < 3; ++v) {
        void* dst = at(b->off_w + ((size_t)v * b->n + bk.wbase + j) * b->wsz);
        if (f32)
          fill_wdesc<float>(dst, c->plan, c->d, c->ptr, v == 1, v != 0);
        else
          fill_wdesc<double>(dst, c->plan, c->d, c->ptr, v == 1, v != 0);
      }
    }
    start[bk.mix.size()] = acc;
  }
  // NMF tables: lambda [2][n], basis [2][n], partials [n], update [n]
  const int slot[4] = {0, 2, 4, 5};
  b->nmfb_threads = 64;
  for (int kind = 0; kind < 4; ++kind) {
    int* start = reinterpret_cast<int*>(at(b->off_ns)) + kind * (b->n + 1);
    int acc = 0;
    for (int i = 0; i < b->n; ++i) {
      const ctfiss_ctx* c = b->ctx[i];
      const bool tap0 = c->vrule == CTFISS_VRULE_PAPER_TAP0;
      start[i] = acc;
      int blocks = 0, thr = 0;
      for (int v = 0; v < (kind < 2 ? 2 : 1); ++v) {
        void* dst = at(b->off_n + ((size_t)(slot[kind] + v) * b->n + i) * b->nsz);
        blocks = f32 ? fill_ndesc<float>(dst, kind, c->d, c->vs, c->ptr, c->floor, tap0, v == 1, &thr)
                     : fill_ndesc<double>(dst, kind, c->d, c->vs, c->ptr, c->floor, tap0, v == 1, &thr);
      }
      if (kind == 1 && thr > b->nmfb_threads) b->nmfb_threads = thr;
      acc += blocks;
    }
    start[b->n] = acc;
    b->nblocks[kind] = acc;
  }
  hipError_t e = hipMemcpyAsync(b->ws + b->off_w, h, b->tab_bytes, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return CTFISS_E_HIP;
  b->have_input = true;
  b->y_valid = false;
  return CTFISS_OK;
}

int ctfiss_batch_set_state(ctfiss_batch* b, const void* const* W, const void* const* B, const void* const* V) {
  if (!b || !B || !V) return CTFISS_E_ARG;
  for (int i = 0; i < b->n; ++i) {
    const int st = ctfiss_set_state(b->ctx[i], W ? W[i] : nullptr, B[i], V[i]);
    if (st != CTFISS_OK) return st;
  }
  b->have_state = true;
  b->y_valid = false;
  return CTFISS_OK;
}

}  // extern "C"

namespace {

// The launches of n_iter batched ISS iterations on the batch's stream.
int batch_enqueue(ctfiss_batch* b, int32_t n_iter) {
  const bool f32 = b->prec != CTFISS_FP64;
  char* w = b->ws;
  const int* nst = reinterpret_cast<const int*>(w + b->off_ns);
  int* cnt = reinterpret_cast<int*>(w + b->off_cnt);
  const int nb = (int)b->buckets.size();
  hipStream_t s = b->stream;
  auto ndesc = [&](int slot) { return static_cast<const void*>(w + b->off_n + (size_t)slot * b->n * b->nsz); };
  auto nmf = [&](int kind, int slot, int threads) {
    const int* start = nst + kind * (b->n + 1);
    return f32 ? nmf_batch_t<float>(kind, ndesc(slot), start, b->n, b->nblocks[kind], threads, cnt, nb, s)
               : nmf_batch_t<double>(kind, ndesc(slot), start, b->n, b->nblocks[kind], threads, cnt, nb, s);
  };
  for (int it = 0; it < n_iter; ++it) {
    const bool mu = it > 0;
    hipError_t e = nmf(0, mu ? 1 : 0, 256);  // lambda; also zeroes the bucket counters
    const int v = mu ? 1 : (b->y_valid ? 2 : 0);
    const int ns = (int)b->side.size();
    if (e == hipSuccess && ns > 0) {  // fork: the side streams start after lambda
      e = hipEventRecord(b->fork, s);
      for (int j = 0; j < ns && e == hipSuccess; ++j) e = hipStreamWaitEvent(b->side[j], b->fork, 0);
    }
    for (int k = 0; e == hipSuccess && k < nb; ++k) {
      const auto& bk = b->buckets[k];
      const void* desc = w + b->off_w + ((size_t)v * b->n + bk.wbase) * b->wsz;
      const int* start = reinterpret_cast<const int*>(w + b->off_ws) + bk.sbase;
      hipStream_t sk = (ns > 0 && b->lane[k] > 0) ? b->side[b->lane[k] - 1] : s;
      e = f32 ? wupdate_batch_t<float>(bk.plan, desc, start, (int)bk.mix.size(), cnt + k, bk.lds, bk.blocks, sk)
              : wupdate_batch_t<double>(bk.plan, desc, start, (int)bk.mix.size(), cnt + k, bk.lds, bk.blocks, sk);
    }
    for (int j = 0; e == hipSuccess && j < ns; ++j) {  // join before the basis update
      e = hipEventRecord(b->join[j], b->side[j]);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, b->join[j], 0);
    }
    if (e == hipSuccess) b->y_valid = true;
    if (e == hipSuccess) e = nmf(1, mu ? 3 : 2, b->nmfb_threads);
    if (e == hipSuccess) e = nmf(2, 4, 256);
    if (e == hipSuccess) e = nmf(3, 5, 256);
    if (e != hipSuccess) return CTFISS_E_HIP;
  }
  if (n_iter > 0) {
    for (ctfiss_ctx* c : b->ctx) {
      const hipError_t e = f32 ? apply_mu_t<float>(c->d, c->ptr, b->y_valid, s) : apply_mu_t<double>(c->d, c->ptr, b->y_valid, s);
      if (e != hipSuccess) return CTFISS_E_HIP;
    }
  }
  return CTFISS_OK;
}

void batch_drop_graphs(ctfiss_batch* b) {
  for (auto& g : b->graphs) (void)hipGraphExecDestroy(g.exec);
  b->graphs.clear();
}

}  // namespace

extern "C" {

int ctfiss_batch_iterate(ctfiss_batch* b, int32_t n_iter) {
  if (!b || n_iter < 0) return CTFISS_E_ARG;
  if (!b->have_input || !b->have_state) return CTFISS_E_ORDER;
  if (b->rule != CTFISS_RULE_ISS) {
    for (ctfiss_ctx* c : b->ctx) {
      const int st = ctfiss_iterate(c, n_iter, nullptr);
      if (st != CTFISS_OK) return st;
    }
    return CTFISS_OK;
  }
  if (!b->graph || n_iter == 0) return batch_enqueue(b, n_iter);
  // graph mode: one captured graph per (n_iter, carried Y valid at the start).  The
  // launches read the mixtures' buffers through the device work tables, so a graph
  // stays valid across set_input and set_state.
  const bool yv = b->y_valid;
  for (auto& g : b->graphs) {
    if (g.n == n_iter && g.y_valid == yv) {
      if (hipGraphLaunch(g.exec, b->stream) != hipSuccess) return CTFISS_E_HIP;
      b->y_valid = true;
      return CTFISS_OK;
    }
  }
  if (b->graphs.size() >= 8) {
    if (hipStreamSynchronize(b->stream) != hipSuccess) return CTFISS_E_HIP;
    batch_drop_graphs(b);
  }
  hipGraph_t graph = nullptr;
  if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return CTFISS_E_HIP;
  const int st = batch_enqueue(b, n_iter);
  const hipError_t ee = hipStreamEndCapture(b->stream, &graph);
  if (st != CTFISS_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    b->y_valid = yv;
    return st;
  }
  if (ee != hipSuccess || !graph) return CTFISS_E_HIP;
  hipGraphExec_t exec = nullptr;
  const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) return CTFISS_E_HIP;
  b->graphs.push_back({n_iter, yv, exec});
  return hipGraphLaunch(exec, b->stream) == hipSuccess ? CTFISS_OK : CTFISS_E_HIP;
}

int ctfiss_batch_set_graph(ctfiss_batch* b, int enable) {
  if (!b) return CTFISS_E_ARG;
  if (enable) {
    if (b->stream == nullptr) return CTFISS_E_UNSUPPORTED;  // capture needs a created stream
  } else if (!b->graphs.empty()) {
    if (hipStreamSynchronize(b->stream) != hipSuccess) return CTFISS_E_HIP;
    batch_drop_graphs(b);
  }
  b->graph = enable != 0;
  return CTFISS_OK;
}

int ctfiss_batch_source_images(ctfiss_batch* b, void* const* C) {
  if (!b || !C) return CTFISS_E_ARG;
  for (int i = 0; i < b->n; ++i) {
    const int st = ctfiss_source_images(b->ctx[i], C[i]);
    if (st != CTFISS_OK) return st;
  }
  return CTFISS_OK;
}

int ctfiss_batch_sync_status(ctfiss_batch* b, int32_t* mixture, int32_t* fault_code) {
  if (!b) return CTFISS_E_ARG;
  if (mixture) *mixture = -1;
  if (fault_code) *fault_code = 0;
  for (int i = 0; i < b->n; ++i) {
    int32_t code = 0;
    const int st = ctfiss_sync_status(b->ctx[i], &code);
    if (st == CTFISS_E_NUMERIC) {
      if (mixture) *mixture = i;
      if (fault_code) *fault_code = code;
      return st;
    }
    if (st != CTFISS_OK) return st;
  }
  return CTFISS_OK;
}

}  // extern "C"
