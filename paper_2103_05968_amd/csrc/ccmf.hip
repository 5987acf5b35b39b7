// Host runtime of the CCMF solver: plan, buffers, launch sequence, C ABI.
// Kernels: ccmf_kernels.h (stencil, fused update, reductions), ccmf_dht.h
// (spectral Laplacian solve).  See include/ccmf.h for the interface contract.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <string>
#include <vector>

#include "ccmf.h"
#include "ccmf_dht.h"
#include "ccmf_kernels.h"

using namespace ccmf;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(e_ == hipErrorOutOfMemory ? CCMF_ENOMEM : CCMF_EDEVICE, "%s: %s (%s:%d)", \
                  #expr, hipGetErrorString(e_), __FILE__, __LINE__);                    \
  } while (0)

#define HIP_LAUNCH_CHECK() HIP_TRY(hipGetLastError())

struct Axis {
  int n = 1;
  std::vector<int> radix;
  void* tw[2] = {nullptr, nullptr};  // complex twiddles exp(-2 pi i t / n), t < n: [0] double, [1] float
  void* tws[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};  // stage-major, per plan variant
  void* s[2] = {nullptr, nullptr};   // 4 sin^2(pi q / n), q < n: [0] double, [1] float
};

template <typename T>
constexpr int prec_index() { return sizeof(T) == 8 ? 0 : 1; }

std::vector<int> factor_radices(int n) {
  std::vector<int> r;
  int m = n;
  while (m % 8 == 0 && m > 4) {
    r.push_back(8);
    m /= 8;
  }
  if (m % 4 == 0) {
    r.push_back(4);
    m /= 4;
  }
  if (m % 2 == 0) {
    r.push_back(2);
    m /= 2;
  }
  for (int p = 3; m > 1; p += 2) {
    while (m % p == 0) {
      r.push_back(p);
      m /= p;
    }
    if (p * p > m && m > 1) {
      r.push_back(m);
      m = 1;
    }
  }
  return r;
}

}  // namespace

struct ccmf_plan_s {
  int dt = CCMF_F64;
  size_t esz = 8;
  int n[3] = {1, 1, 1};
  uint32_t N = 1;
  int64_t nfields = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;  // created by the plan when the caller passes the null stream
  int device = 0;
  void* kap = nullptr;
  std::vector<double> kmin, kmax;  // per field: smallest positive, largest
  Axis ax[3];

  // solve state
  int64_t B = 0, nloads = 0;
  void* z[2] = {nullptr, nullptr};
  void* a[2] = {nullptr, nullptr};
  void* r = nullptr;       // r = div^- A* w in the plan dtype (aliases phi in FP64 mode)
  double* phi = nullptr;   // node potential, FP64 in both modes
  double* partials = nullptr;
  Prob* prob = nullptr;    // device
  Prob* probh = nullptr;   // pinned host
  bool solved = false;
  double* hist = nullptr;    // [B][hist_len][4] convergence history (record_history)
  int hist_len = 0;
  bool hist_valid = false;
  bool state_ready = false;  // z[.]/a[.] and probh hold a state a warm start can resume
  int upd_blocks = 0;        // blocks per problem of the stencil kernels (k_div, k_update)
  int tiles_per_blk = 0, tpp = 0;  // tile walk of the stencil kernels (see tile_of)

  // autotuned tile widths (complex lines per block) of the five Hartley passes
  // (0 forward k, 1 forward j, 2 fused i, 3 inverse j, 4 inverse k); 0 = rule of thumb
  // kind 5: r = div^- A* w fused with the forward k pass
  int nlc_hint[6] = {0, 0, 0, 0, 0, 0};
  int walk_hint[5] = {0, 0, 0, 0, 0};     // tiles walked per block of passes 0-4; 0 = one
  int planes_hint = 0;                    // planes walked per block by the fused kernel
  int64_t tuned_B = 0;
  bool tuned_off = false;

  // captured chunk of iterations (HIP graph), valid for the current state buffers
  hipGraphExec_t gexec = nullptr;
  int graph_iters = 0;
  const double* graph_hist = nullptr;  // history buffer baked into the captured graph
  Prob* flagsh[2] = {nullptr, nullptr};  // pinned copies of the scalars, one per chunk in flight
  hipEvent_t fev[2] = {nullptr, nullptr};

  // kernel timing
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
  double kt_sum = 0.0;
  int64_t kt_count = 0;

  ~ccmf_plan_s() {
    hipFree(kap);
    for (int c = 0; c < 3; ++c) {
      for (int q = 0; q < 2; ++q) {
        hipFree(ax[c].tw[q]);
        for (int v = 0; v < 3; ++v) hipFree(ax[c].tws[q][v]);
        hipFree(ax[c].s[q]);
      }
    }
    free_state();
    for (auto e : ev) hipEventDestroy(e);
    for (int q = 0; q < 2; ++q)
      if (fev[q]) hipEventDestroy(fev[q]);
    if (own_stream) hipStreamDestroy(stream);
  }
  void drop_graph() {
    if (gexec) hipGraphExecDestroy(gexec);
    gexec = nullptr;
    graph_iters = 0;
    graph_hist = nullptr;
  }
  void free_state() {
    drop_graph();
    for (int q = 0; q < 2; ++q) {
      if (flagsh[q]) hipHostFree(flagsh[q]);
      flagsh[q] = nullptr;
    }
    for (int p = 0; p < 2; ++p) {
      hipFree(z[p]);
      hipFree(a[p]);
      z[p] = a[p] = nullptr;
    }
    if (r != (void*)phi) hipFree(r);
    hipFree(phi);
    r = nullptr;
    phi = nullptr;
    hipFree(partials);
    hipFree(hist);
    hist = nullptr;
    hist_len = 0;
    hist_valid = false;
    hipFree(prob);
    if (probh) hipHostFree(probh);
    r = nullptr;
    partials = nullptr;
    prob = nullptr;
    probh = nullptr;
    B = 0;
  }
};

namespace {

Geo make_geo(const ccmf_plan_s* p) {
  Geo g;
  g.n1 = p->n[0];
  g.n2 = p->n[1];
  g.n3 = p->n[2];
  g.n23 = p->n[1] * p->n[2];
  g.N = p->N;
  g.nloads = (int32_t)p->nloads;
  g.tiles = (int32_t)((p->N + kUpd - 1) / kUpd);
  g.tiles_per_blk = p->tiles_per_blk;
  g.tpp = p->tpp;
  return g;
}

bool is_pow2_len(int n);

template <int V>
bool stage_twiddles_v(int n, const double* w, double* out) {
  switch (n) {
    case 2: pow2::stage_twiddles<2, V>(w, out); return true;
    case 4: pow2::stage_twiddles<4, V>(w, out); return true;
    case 8: pow2::stage_twiddles<8, V>(w, out); return true;
    case 16: pow2::stage_twiddles<16, V>(w, out); return true;
    case 32: pow2::stage_twiddles<32, V>(w, out); return true;
    case 64: pow2::stage_twiddles<64, V>(w, out); return true;
    case 128: pow2::stage_twiddles<128, V>(w, out); return true;
    case 256: pow2::stage_twiddles<256, V>(w, out); return true;
    case 512: pow2::stage_twiddles<512, V>(w, out); return true;
    case 1024: pow2::stage_twiddles<1024, V>(w, out); return true;
    case 2048: pow2::stage_twiddles<2048, V>(w, out); return true;
    default: return false;
  }
}

bool stage_twiddles_of(int n, int v, const double* w, double* out) {
  return v == 0 ? stage_twiddles_v<0>(n, w, out) : v == 1 ? stage_twiddles_v<1>(n, w, out)
                                                          : stage_twiddles_v<2>(n, w, out);
}

int upload_axis(Axis& ax, int n) {
  ax.n = n;
  ax.radix = factor_radices(n);
  std::vector<double> tw(2 * (size_t)n), sv(n);
  for (int t = 0; t < n; ++t) {
    // angles from exact integer ratios, evaluated in long double, rounded once
    const long double pi = 3.14159265358979323846264338327950288L;
    const long double ang = -2.0L * pi * (long double)t / (long double)n;
    tw[2 * t] = (double)cosl(ang);
    tw[2 * t + 1] = (double)sinl(ang);
    const long double sn = sinl(pi * (long double)t / (long double)n);
    sv[t] = (double)(4.0L * sn * sn);
  }
  std::vector<float> tw32(tw.begin(), tw.end()), sv32(sv.begin(), sv.end());
  HIP_TRY(hipMalloc(&ax.tw[0], tw.size() * sizeof(double)));
  HIP_TRY(hipMalloc(&ax.s[0], sv.size() * sizeof(double)));
  HIP_TRY(hipMalloc(&ax.tw[1], tw32.size() * sizeof(float)));
  HIP_TRY(hipMalloc(&ax.s[1], sv32.size() * sizeof(float)));
  HIP_TRY(hipMemcpy(ax.tw[0], tw.data(), tw.size() * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(ax.s[0], sv.data(), sv.size() * sizeof(double), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(ax.tw[1], tw32.data(), tw32.size() * sizeof(float), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(ax.s[1], sv32.data(), sv32.size() * sizeof(float), hipMemcpyHostToDevice));
  if (is_pow2_len(n)) {
    // the same values, reordered stage-major for each register-blocked plan variant
    std::vector<double> st(2 * (size_t)n);
    for (int v = 0; v < 3; ++v) {
      if (!stage_twiddles_of(n, v, tw.data(), st.data())) return fail(CCMF_EINVAL, "no FFT plan for length %d", n);
      std::vector<float> st32(st.begin(), st.end());
      HIP_TRY(hipMalloc(&ax.tws[0][v], st.size() * sizeof(double)));
      HIP_TRY(hipMalloc(&ax.tws[1][v], st32.size() * sizeof(float)));
      HIP_TRY(hipMemcpy(ax.tws[0][v], st.data(), st.size() * sizeof(double), hipMemcpyHostToDevice));
      HIP_TRY(hipMemcpy(ax.tws[1][v], st32.data(), st32.size() * sizeof(float), hipMemcpyHostToDevice));
    }
  }
  return CCMF_OK;
}

// lines per LDS tile: ping-pong complex buffers within 64 KiB
int lines_per_tile(int n, size_t esz, int lines_total) {
  int nl = 32;
  while (nl > 2 && (size_t)2 * nl * n * esz > 65536) nl >>= 1;
  if (lines_total < nl) nl = std::max(2, lines_total + (lines_total & 1));
  return nl;
}

bool is_pow2_len(int n) { return n >= 2 && n <= 2048 && (n & (n - 1)) == 0; }

// Launch the power-of-two Hartley kernel: NLC complex lines (2 NLC real lines) per
// block, NLC * TPL <= 512 threads, padded LDS tile within 64 KiB.
// gfx950 gives a workgroup up to 160 KiB of LDS; above 64 KiB the kernel has to
// opt in (once per kernel).
constexpr size_t kMaxLds = 163840;

int allow_lds(const void* kernel, size_t lds) {
  if (lds <= 65536) return CCMF_OK;
  static std::mutex mu;
  static std::vector<const void*> done;
  std::lock_guard<std::mutex> lk(mu);
  for (const void* k : done)
    if (k == kernel) return CCMF_OK;
  HIP_TRY(hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds));
  done.push_back(kernel);
  return CCMF_OK;
}

template <typename TI, typename TO, typename TC, int N, int V>
int launch_p2v(ccmf_plan_s* p, const TI* in, TO* out, int64_t count, DhtArgs A, int outers, bool contig,
               bool middle, const void* twp, const void* twp32, const TC* s1, const TC* s2, const TC* s3,
               const Prob* prob, int kind) {
  constexpr int E = pow2::Plan<N, V>::E, TPL = N / E;
  constexpr int LP = line_pitch<N, V>();
  // the middle pass of FP32 fields also stages the FP32 twiddles of its forward transform
  const size_t tw32_bytes = (middle && sizeof(TI) == 4 && sizeof(TC) == 8) ? (size_t)N * 2 * sizeof(float) : 0;
  int nlc = 16;
  if (kind >= 0 && p->nlc_hint[kind] > 0) {
    nlc = p->nlc_hint[kind];
  } else {
    while (nlc > 1 && (nlc * TPL > 512 || (size_t)(nlc * LP + N) * 2 * sizeof(TC) + tw32_bytes > 65536)) nlc >>= 1;
    while (nlc > 1 && 2 * (nlc >> 1) >= A.lines_total) nlc >>= 1;  // do not pad tiny line counts
  }
  const int nl = 2 * nlc;
  int lognl = 0;
  while ((1 << lognl) < nl) ++lognl;
  A.nl = nl;
  A.lognl = lognl;
  A.tiles_per_outer = (A.lines_total + nl - 1) / nl;
  // vector loads/stores: rows need n3 % (16 / element size) == 0, columns an even n3
  if (contig)
    A.vec = (p->n[2] % (int)(16 / sizeof(TI)) == 0 && p->n[2] % (int)(16 / sizeof(TO)) == 0 && N >= 4) ? 1 : 0;
  else
    A.vec = (p->n[2] % 2 == 0) ? 1 : 0;
  if ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15) A.vec = 0;
  const size_t lds = (size_t)(nlc * LP + N) * 2 * sizeof(TC) + tw32_bytes;
  if (lds > kMaxLds || nlc * TPL > 512) return fail(CCMF_EINVAL, "transform length %d too large for the LDS tile", N);
  // tiles walked per block (the next tile's loads overlap the current transforms);
  // the arithmetic of a tile does not depend on it
  A.outers = outers;
  A.walk = (kind >= 0 && kind < 5 && p->walk_hint[kind] > 0) ? p->walk_hint[kind] : 1;
  if (const char* env = std::getenv("CCMF_TILE_WALK")) {  // diagnostic override (tests)
    const int w = std::atoi(env);
    if (w >= 1 && w <= 64) A.walk = w;
  }
  const int ntiles = outers * A.tiles_per_outer;
  dim3 grid((unsigned)((ntiles + A.walk - 1) / A.walk), (unsigned)count);
  dim3 block((unsigned)(nlc * TPL));
  const pow2::CX<TC>* tw = reinterpret_cast<const pow2::CX<TC>*>(twp);
  const pow2::CX<float>* tw32 = reinterpret_cast<const pow2::CX<float>*>(twp32);
  int rc;
  if (middle) {
    if ((rc = allow_lds((const void*)k_hartley_p2<TI, TO, TC, N, V, false, true>, lds))) return rc;
    hipLaunchKernelGGL((k_hartley_p2<TI, TO, TC, N, V, false, true>), grid, block, lds, p->stream, in, out, tw, tw32,
                       A, s1, s2, s3, prob);
  } else if (contig) {
    if ((rc = allow_lds((const void*)k_hartley_p2<TI, TO, TC, N, V, true, false>, lds))) return rc;
    hipLaunchKernelGGL((k_hartley_p2<TI, TO, TC, N, V, true, false>), grid, block, lds, p->stream, in, out, tw, tw32,
                       A, s1, s2, s3, prob);
  } else {
    if ((rc = allow_lds((const void*)k_hartley_p2<TI, TO, TC, N, V, false, false>, lds))) return rc;
    hipLaunchKernelGGL((k_hartley_p2<TI, TO, TC, N, V, false, false>), grid, block, lds, p->stream, in, out, tw, tw32,
                       A, s1, s2, s3, prob);
  }
  HIP_LAUNCH_CHECK();
  return CCMF_OK;
}

// Plan variant of a pass.  The variant changes the radix decomposition, hence
// the rounding, so it is a fixed function of the pass and the line length (never
// timed): results are reproducible and a batched solve equals the single solves
// bit for bit.  Chosen from per-pass timings of every variant on MI355X at 128,
// 256 and 512 points: FP64 lines radix-8/4 (variant 1) up to 256 and radix-8 (0)
// from 512; FP32 lines radix-8/4 below 256 and radix-16/8 (0) from 256; the
// fused i pass radix-16/8 (0) from 128 (its forward half runs in FP32 for FP32
// fields); the fused divergence pass radix-4 (2) in FP32 up to 256, else radix-8
// (0), and in FP64 radix-8 (0) up to 256, radix-16 (1) from 512.  The diagnostic
// environment variable CCMF_FFT_VARIANT (0, 1 or 2) overrides it.
int variant_of(int kind, bool fp64, int n) {
  const char* env = std::getenv("CCMF_FFT_VARIANT");
  if (env != nullptr && env[0] >= '0' && env[0] <= '2' && env[1] == '\0') return env[0] - '0';
  if (kind == 5) return fp64 ? (n >= 512 ? 1 : 0) : (n >= 512 ? 0 : 2);
  if (kind == 2 && n >= 128) return 0;
  if (fp64) return n >= 512 ? 0 : 1;
  return n >= 256 ? 0 : 1;
}

template <typename TI, typename TO, typename TC, int N>
int launch_p2(ccmf_plan_s* p, const TI* in, TO* out, int64_t count, DhtArgs A, int outers, bool contig,
              bool middle, void* const* tws, void* const* tws32, const TC* s1, const TC* s2, const TC* s3,
              const Prob* prob, int kind) {
  // tws, tws32: the stage-major twiddle tables of the three plan variants in the
  // compute precision and in FP32
  const int var = variant_of(kind, sizeof(TC) == 8, N);
  if (var == 1)
    return launch_p2v<TI, TO, TC, N, 1>(p, in, out, count, A, outers, contig, middle, tws[1], tws32[1], s1, s2, s3,
                                        prob, kind);
  if (var == 2)
    return launch_p2v<TI, TO, TC, N, 2>(p, in, out, count, A, outers, contig, middle, tws[2], tws32[2], s1, s2, s3,
                                        prob, kind);
  return launch_p2v<TI, TO, TC, N, 0>(p, in, out, count, A, outers, contig, middle, tws[0], tws32[0], s1, s2, s3,
                                      prob, kind);
}

// Launch one Hartley pass along `axis` over `count` fields: load TI from `in`,
// compute in TC, store TO to `out` (same layout, may alias).
template <typename TI, typename TO, typename TC>
int launch_hartley(ccmf_plan_s* p, const TI* in, TO* out, int64_t count, int axis, bool middle,
                   const Prob* prob, int kind = -1) {
  const int n1 = p->n[0], n2 = p->n[1], n3 = p->n[2];
  const Axis& ax = p->ax[axis];
  DhtArgs A;
  std::memset(&A, 0, sizeof(A));
  A.n = ax.n;
  A.nstages = (int)ax.radix.size();
  if (A.nstages > kMaxStages) return fail(CCMF_EINVAL, "transform length %d has too many factors", ax.n);
  for (int i = 0; i < A.nstages; ++i) A.radix[i] = ax.radix[i];
  A.field_stride = p->N;
  A.scale = 1.0 / (double)p->N;
  A.n2 = n2;
  A.n3 = n3;
  int outers;
  bool contig;
  if (axis == 2) {  // rows along k, contiguous samples
    contig = true;
    A.lines_total = n1 * n2;
    A.ss = 1;
    A.ls = n3;
    A.os = 0;
    outers = 1;
  } else if (axis == 1) {
    contig = false;
    A.lines_total = n3;
    A.ss = n3;
    A.ls = 1;
    A.os = (int64_t)n2 * n3;
    outers = n1;
  } else {
    contig = false;
    A.lines_total = n3;
    A.ss = (int64_t)n2 * n3;
    A.ls = 1;
    A.os = n3;
    outers = n2;
  }
  constexpr int q = prec_index<TC>();
  const TC* s1 = reinterpret_cast<const TC*>(p->ax[0].s[q]);
  const TC* s2 = reinterpret_cast<const TC*>(p->ax[1].s[q]);
  const TC* s3 = reinterpret_cast<const TC*>(p->ax[2].s[q]);
  if (is_pow2_len(A.n)) {
    switch (A.n) {
      case 2: return launch_p2<TI, TO, TC, 2>(p, in, out, count, A, outers, contig, middle, ax.tws[q], ax.tws[prec_index<float>()], s1, s2, s3, prob, kind);
      case 4: return launch_p2<TI, TO, TC, 4>(p, in, out, count, A, outers, contig, middle, ax.tws[q], ax.tws[prec_index<float>()], s1, s2, s3, prob, kind);
      case 8: return launch_p2<TI, TO, TC, 8>(p, in, out, count, A, outers, contig, middle, ax.tws[q], ax.tws[prec_index<float>()], s1, s2, s3, prob, kind);
      case 16: return launch_p2<TI, TO, TC, 16>(p, in, out, count, A, outers, contig, middle, ax.tws[q], ax.tws[prec_index<float>()], s1, s2, s3, prob, kind);
      case 32: return launch_p2<TI, TO, TC, 32>(p, in, out, count, A, outers, contig, middle, ax.tws[q], ax.tws[prec_index<float>()], s1, s2, s3, prob, kind);
      case 64: return launch_p2<TI, TO, TC, 64>(p, in, out, count, A, outers, contig, middle, ax.tws[q], ax.tws[prec_index<float>()], s1, s2, s3, prob, kind);
      case 128: return launch_p2<TI, TO, TC, 128>(p, in, out, count, A, outers, contig, middle, ax.tws[q], ax.tws[prec_index<float>()], s1, s2, s3, prob, kind);
      case 256: return launch_p2<TI, TO, TC, 256>(p, in, out, count, A, outers, contig, middle, ax.tws[q], ax.tws[prec_index<float>()], s1, s2, s3, prob, kind);
      case 512: return launch_p2<TI, TO, TC, 512>(p, in, out, count, A, outers, contig, middle, ax.tws[q], ax.tws[prec_index<float>()], s1, s2, s3, prob, kind);
      case 1024: return launch_p2<TI, TO, TC, 1024>(p, in, out, count, A, outers, contig, middle, ax.tws[q], ax.tws[prec_index<float>()], s1, s2, s3, prob, kind);
      case 2048: return launch_p2<TI, TO, TC, 2048>(p, in, out, count, A, outers, contig, middle, ax.tws[q], ax.tws[prec_index<float>()], s1, s2, s3, prob, kind);
      default: break;
    }
  }
  A.nl = lines_per_tile(A.n, sizeof(TC), A.lines_total);
  A.tiles_per_outer = (A.lines_total + A.nl - 1) / A.nl;
  const size_t lds = (size_t)2 * A.nl * A.n * sizeof(TC);
  if (lds > 65536) return fail(CCMF_EINVAL, "transform length %d too large for the LDS tile", A.n);
  dim3 grid((unsigned)(outers * A.tiles_per_outer), (unsigned)count);
  const C2<TC>* tw = reinterpret_cast<const C2<TC>*>(ax.tw[q]);
  if (middle) {
    hipLaunchKernelGGL((k_hartley<TI, TO, TC, false, true>), grid, dim3(kThreads), lds, p->stream, in, out, tw,
                       A, s1, s2, s3, prob);
  } else if (contig) {
    hipLaunchKernelGGL((k_hartley<TI, TO, TC, true, false>), grid, dim3(kThreads), lds, p->stream, in, out, tw,
                       A, s1, s2, s3, prob);
  } else {
    hipLaunchKernelGGL((k_hartley<TI, TO, TC, false, false>), grid, dim3(kThreads), lds, p->stream, in, out, tw,
                       A, s1, s2, s3, prob);
  }
  HIP_LAUNCH_CHECK();
  return CCMF_OK;
}

// r = div^- A* w fused with the forward k pass (power-of-two n3 >= 4)
bool fused_div_ok(const ccmf_plan_s* p) { return p->n[2] >= 4 && is_pow2_len(p->n[2]); }

template <typename T, int N, int V>
int launch_div_p2v(ccmf_plan_s* p, const T* z, const T* a, T* r, int64_t count, const Prob* prob) {
  constexpr int E = pow2::Plan<N, V>::E, TPL = N / E;
  constexpr int LP = line_pitch<N, V>();
  int nlc = p->nlc_hint[5] > 0 ? p->nlc_hint[5] : 16;
  if (p->nlc_hint[5] <= 0)
    while (nlc > 1 && (nlc * TPL > 512 || (size_t)(nlc * LP + N) * 2 * sizeof(T) > 65536)) nlc >>= 1;
  const size_t lds = (size_t)(nlc * LP + N) * 2 * sizeof(T);
  if (lds > kMaxLds || nlc * TPL > 512) return fail(CCMF_EINVAL, "fused tile of %d lines does not fit", 2 * nlc);
  int rc;
  if ((rc = allow_lds((const void*)k_div_hartley_p2<T, N, V>, lds))) return rc;
  DivArgs D;
  D.n1 = p->n[0];
  D.n2 = p->n[1];
  D.n3 = p->n[2];
  D.nl = 2 * nlc;
  D.lognl = 0;
  while ((1 << D.lognl) < D.nl) ++D.lognl;
  D.jtiles = (D.n2 + D.nl - 1) / D.nl;
  int planes = p->planes_hint;
  if (planes <= 0) planes = std::max(1, (D.jtiles * D.n1) / 2048);
  planes = std::min(planes, D.n1);
  D.planes = planes;
  D.ichunks = (D.n1 + planes - 1) / planes;
  D.vec = ((reinterpret_cast<uintptr_t>(r) & 15) == 0 && N * (int)sizeof(T) >= 16) ? 1 : 0;
  dim3 grid((unsigned)(D.jtiles * D.ichunks), (unsigned)count);
  const pow2::CX<T>* tw = reinterpret_cast<const pow2::CX<T>*>(p->ax[2].tws[prec_index<T>()][V]);
  hipLaunchKernelGGL((k_div_hartley_p2<T, N, V>), grid, dim3((unsigned)(nlc * TPL)), lds, p->stream, z, a, r, tw,
                     D, prob);
  HIP_LAUNCH_CHECK();
  return CCMF_OK;
}

template <typename T, int N>
int launch_div_p2(ccmf_plan_s* p, const T* z, const T* a, T* r, int64_t count, const Prob* prob) {
  const int var = variant_of(5, sizeof(T) == 8, N);
  if (var == 1) return launch_div_p2v<T, N, 1>(p, z, a, r, count, prob);
  if (var == 2) return launch_div_p2v<T, N, 2>(p, z, a, r, count, prob);
  return launch_div_p2v<T, N, 0>(p, z, a, r, count, prob);
}

template <typename T>
int launch_div_fused(ccmf_plan_s* p, const T* z, const T* a, T* r, int64_t count, const Prob* prob) {
  switch (p->n[2]) {
    case 4: return launch_div_p2<T, 4>(p, z, a, r, count, prob);
    case 8: return launch_div_p2<T, 8>(p, z, a, r, count, prob);
    case 16: return launch_div_p2<T, 16>(p, z, a, r, count, prob);
    case 32: return launch_div_p2<T, 32>(p, z, a, r, count, prob);
    case 64: return launch_div_p2<T, 64>(p, z, a, r, count, prob);
    case 128: return launch_div_p2<T, 128>(p, z, a, r, count, prob);
    case 256: return launch_div_p2<T, 256>(p, z, a, r, count, prob);
    case 512: return launch_div_p2<T, 512>(p, z, a, r, count, prob);
    case 1024: return launch_div_p2<T, 1024>(p, z, a, r, count, prob);
    case 2048: return launch_div_p2<T, 2048>(p, z, a, r, count, prob);
    default: return fail(CCMF_EINVAL, "fused divergence needs a power-of-two n3");
  }
}

// phi = (div^- grad^+)^dagger r: forward passes along k and j in place on r (the
// plan dtype), the fused axis-i pass reads r and writes phi in FP64, the inverse
// passes along j and k run in FP64 in place on phi.
template <typename T>
int launch_laplace(ccmf_plan_s* p, T* r, double* phi, int64_t count, const Prob* prob, bool k_done = false) {
  int rc;
  if (!k_done && p->n[2] > 1 && (rc = launch_hartley<T, T, T>(p, r, r, count, 2, false, prob, 0))) return rc;
  if (p->n[1] > 1 && (rc = launch_hartley<T, T, T>(p, r, r, count, 1, false, prob, 1))) return rc;
  if ((rc = launch_hartley<T, double, double>(p, r, phi, count, 0, true, prob, 2))) return rc;
  if (p->n[1] > 1 && (rc = launch_hartley<double, double, double>(p, phi, phi, count, 1, false, prob, 3)))
    return rc;
  if (p->n[2] > 1 && (rc = launch_hartley<double, double, double>(p, phi, phi, count, 2, false, prob, 4)))
    return rc;
  return CCMF_OK;
}

template <typename T>
int kappa_stats(ccmf_plan_s* p) {
  const int blocks = (int)std::min<uint64_t>(1024, (p->N + kThreads - 1) / kThreads);
  double* d = nullptr;
  const size_t cnt = (size_t)p->nfields * blocks * 3;
  HIP_TRY(hipMalloc(&d, cnt * sizeof(double)));
  hipLaunchKernelGGL((k_kappa_stats<T>), dim3(blocks, (unsigned)p->nfields), dim3(kThreads), 0, p->stream,
                     reinterpret_cast<const T*>(p->kap), p->N, d);
  hipError_t e = hipGetLastError();
  std::vector<double> h(cnt);
  if (e == hipSuccess) e = hipMemcpyAsync(h.data(), d, cnt * sizeof(double), hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  hipFree(d);
  if (e != hipSuccess) return fail(CCMF_EDEVICE, "kappa statistics: %s", hipGetErrorString(e));
  p->kmin.assign(p->nfields, INFINITY);
  p->kmax.assign(p->nfields, 0.0);
  for (int64_t f = 0; f < p->nfields; ++f) {
    double bad = 0.0;
    for (int bl = 0; bl < blocks; ++bl) {
      const double* o = &h[((size_t)f * blocks + bl) * 3];
      p->kmin[f] = std::min(p->kmin[f], o[0]);
      p->kmax[f] = std::max(p->kmax[f], o[1]);
      bad += o[2];
    }
    if (bad > 0.0)
      return fail(CCMF_EINVAL, "kappa field %lld has %.0f negative or non-finite entries", (long long)f, bad);
  }
  return CCMF_OK;
}

int ensure_state(ccmf_plan_s* p, int64_t nloads) {
  const int64_t B = p->nfields * nloads;
  p->nloads = nloads;
  // stencil kernels: up to kUpdBlocks blocks per problem walking tiles (with
  // whole tiles per i-plane a block walks planes, see tile_of); one FP64 partial
  // row per block and problem.  The reduction order depends on the grid only, so
  // every result is the same batched or alone.
  const int tiles = (int)((p->N + kUpd - 1) / kUpd);
  const int64_t n23 = (int64_t)p->n[1] * p->n[2];
  p->tpp = 0;
  if (n23 % kUpd == 0) {
    const int tpp = (int)(n23 / kUpd);
    int want = std::min(tiles, kUpdBlocks);
    int cpb = std::max(1, (want + tpp - 1) / tpp);          // i-chunks per problem
    cpb = std::min(cpb, p->n[0]);
    p->tiles_per_blk = (p->n[0] + cpb - 1) / cpb;            // planes per block
    cpb = (p->n[0] + p->tiles_per_blk - 1) / p->tiles_per_blk;
    p->upd_blocks = cpb * tpp;
    p->tpp = tpp;
  } else {
    int want = std::min(tiles, kUpdBlocks);
    if (want > 8) want &= ~7;
    p->tiles_per_blk = (tiles + want - 1) / want;
    p->upd_blocks = (tiles + p->tiles_per_blk - 1) / p->tiles_per_blk;
  }
  if (B == p->B && p->z[0] != nullptr) return CCMF_OK;
  p->free_state();
  const size_t N = p->N;
  for (int q = 0; q < 2; ++q) {
    HIP_TRY(hipMalloc(&p->z[q], (size_t)B * 6 * N * p->esz));
    HIP_TRY(hipMalloc(&p->a[q], (size_t)B * N * p->esz));
  }
  HIP_TRY(hipMalloc(&p->phi, (size_t)B * N * sizeof(double)));
  if (p->dt == CCMF_F64) {
    p->r = p->phi;
  } else {
    HIP_TRY(hipMalloc(&p->r, (size_t)B * N * p->esz));
  }
  HIP_TRY(hipMalloc(&p->partials, (size_t)B * p->upd_blocks * kNQ * sizeof(double)));
  HIP_TRY(hipMalloc(&p->prob, (size_t)B * sizeof(Prob)));
  HIP_TRY(hipHostMalloc((void**)&p->probh, (size_t)B * sizeof(Prob), hipHostMallocDefault));
  for (int q = 0; q < 2; ++q) {
    HIP_TRY(hipHostMalloc((void**)&p->flagsh[q], (size_t)B * sizeof(Prob), hipHostMallocDefault));
    if (!p->fev[q]) HIP_TRY(hipEventCreateWithFlags(&p->fev[q], hipEventDisableTiming));
  }
  p->B = B;
  return CCMF_OK;
}

int record_event(ccmf_plan_s* p, hipEvent_t* out) {
  if (p->ev_used == p->ev.size()) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    p->ev.push_back(e);
  }
  *out = p->ev[p->ev_used++];
  HIP_TRY(hipEventRecord(*out, p->stream));
  return CCMF_OK;
}

int harvest_events(ccmf_plan_s* p) {
  if (p->ev_used == 0) return CCMF_OK;
  HIP_TRY(hipEventSynchronize(p->ev[p->ev_used - 1]));
  for (size_t i = 0; i + 1 < p->ev_used; i += 2) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, p->ev[i], p->ev[i + 1]));
    p->kt_sum += ms;
    p->kt_count += 1;
  }
  p->ev_used = 0;
  return CCMF_OK;
}

template <typename T>
int run_iteration(ccmf_plan_s* p, int it, bool timed) {
  const Geo g = make_geo(p);
  const int cur = it & 1, nxt = cur ^ 1;
  T* z0 = reinterpret_cast<T*>(p->z[cur]);
  T* a0 = reinterpret_cast<T*>(p->a[cur]);
  T* z1 = reinterpret_cast<T*>(p->z[nxt]);
  T* a1 = reinterpret_cast<T*>(p->a[nxt]);
  T* r = reinterpret_cast<T*>(p->r);
  const T* kap = reinterpret_cast<const T*>(p->kap);
  int rc;
  const bool fused = fused_div_ok(p);
  if (fused) {
    if ((rc = launch_div_fused<T>(p, z0, a0, r, p->B, p->prob))) return rc;
  } else {
    hipLaunchKernelGGL((k_div<T>), dim3((unsigned)p->upd_blocks, (unsigned)p->B), dim3(kUpd), 0, p->stream, g,
                       z0, a0, r, p->prob);
    HIP_LAUNCH_CHECK();
  }
  if ((rc = launch_laplace<T>(p, r, p->phi, p->B, p->prob, fused))) return rc;
  hipEvent_t e0, e1;
  if (timed && (rc = record_event(p, &e0))) return rc;
  const dim3 ugrid((unsigned)p->upd_blocks, (unsigned)p->B);
  hipLaunchKernelGGL((k_update<T>), ugrid, dim3(kUpd), 0, p->stream, g, kap, z0, a0, p->phi, z1, a1,
                     p->partials, p->prob);
  HIP_LAUNCH_CHECK();
  if (timed && (rc = record_event(p, &e1))) return rc;
  hipLaunchKernelGGL(k_finish, dim3((unsigned)p->B), dim3(kFinishThreads), 0, p->stream, p->N, p->upd_blocks,
                     p->partials, p->prob, p->hist_valid ? p->hist : (double*)nullptr,
                     p->hist_valid ? p->hist_len : 0);
  HIP_LAUNCH_CHECK();
  return CCMF_OK;
}

// Autotuner of the Hartley tile widths: for each of the five passes, time every
// feasible width (1..16 complex lines per block) on the plan's own buffers for
// the current batch and keep the fastest.  The width only changes how lines are
// grouped into blocks, never the arithmetic of a line, so results do not depend
// on it.  Winners are cached per (grid, dtype, batch) for the process.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int, int64_t>, std::array<int, 13>> g_tune_cache;

template <typename T>
int run_pass(ccmf_plan_s* p, int kind) {
  T* r = reinterpret_cast<T*>(p->r);
  double* phi = p->phi;
  switch (kind) {
    case 0: return launch_hartley<T, T, T>(p, r, r, p->B, 2, false, nullptr, 0);
    case 1: return launch_hartley<T, T, T>(p, r, r, p->B, 1, false, nullptr, 1);
    case 2: return launch_hartley<T, double, double>(p, r, phi, p->B, 0, true, nullptr, 2);
    case 3: return launch_hartley<double, double, double>(p, phi, phi, p->B, 1, false, nullptr, 3);
    case 4: return launch_hartley<double, double, double>(p, phi, phi, p->B, 2, false, nullptr, 4);
    default:
      return launch_div_fused<T>(p, reinterpret_cast<const T*>(p->z[0]), reinterpret_cast<const T*>(p->a[0]), r,
                                 p->B, p->prob);
  }
}

template <typename T>
int autotune(ccmf_plan_s* p) {
  const auto key = std::make_tuple(p->n[0], p->n[1], p->n[2], p->dt, p->B);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      for (int k = 0; k < 6; ++k) {
        p->nlc_hint[k] = it->second[k];
      }
      for (int k = 0; k < 5; ++k) p->walk_hint[k] = it->second[6 + k];
      p->planes_hint = it->second[12];
      p->tuned_B = p->B;
      return CCMF_OK;
    }
  }
  HIP_TRY(hipMemsetAsync(p->phi, 0, (size_t)p->B * p->N * sizeof(double), p->stream));
  if (p->r != (void*)p->phi) HIP_TRY(hipMemsetAsync(p->r, 0, (size_t)p->B * p->N * sizeof(T), p->stream));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  std::array<int, 13> best{};
  const bool log = std::getenv("CCMF_TUNE_LOG") != nullptr;  // per-candidate timings on stderr
  const bool present[6] = {p->n[2] > 1, p->n[1] > 1, true, p->n[1] > 1, p->n[2] > 1, fused_div_ok(p)};
  p->planes_hint = 0;
  for (int k = 0; k < 5; ++k) p->walk_hint[k] = 0;
  for (int kind = 0; kind < 6; ++kind) {
    best[kind] = 0;
    if (!present[kind] || !is_pow2_len(p->ax[kind == 2 ? 0 : (kind == 1 || kind == 3) ? 1 : 2].n)) continue;
    float best_ms = 1e30f;
    for (int nlc = 1; nlc <= 32; nlc <<= 1) {
      p->nlc_hint[kind] = nlc;
      if (run_pass<T>(p, kind) != CCMF_OK) continue;  // infeasible width (LDS or threads)
      hipEventRecord(e0, p->stream);
      for (int rep = 0; rep < 3; ++rep) run_pass<T>(p, kind);
      hipEventRecord(e1, p->stream);
      if (hipEventSynchronize(e1) != hipSuccess) break;
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      if (log) std::fprintf(stderr, "[ccmf tune] pass %d lines %d: %.1f us\n", kind, 2 * nlc, ms / 3 * 1e3);
      if (ms < best_ms) {
        best_ms = ms;
        best[kind] = nlc;
      }
    }
    p->nlc_hint[kind] = best[kind];
    // tiles walked per block at the chosen width
    if (kind < 5 && best[kind] > 0) {
      best[6 + kind] = 1;
      for (int walk = 2; walk <= 8; walk <<= 1) {
        p->walk_hint[kind] = walk;
        if (run_pass<T>(p, kind) != CCMF_OK) break;
        hipEventRecord(e0, p->stream);
        for (int rep = 0; rep < 3; ++rep) run_pass<T>(p, kind);
        hipEventRecord(e1, p->stream);
        if (hipEventSynchronize(e1) != hipSuccess) break;
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        if (log) std::fprintf(stderr, "[ccmf tune] pass %d lines %d, %d tiles per block: %.1f us\n", kind,
                              2 * best[kind], walk, ms / 3 * 1e3);
        if (ms < best_ms) {
          best_ms = ms;
          best[6 + kind] = walk;
        }
      }
      p->walk_hint[kind] = best[6 + kind];
    }
  }
  // planes walked per block by the fused divergence kernel
  best[12] = 0;
  if (present[5]) {
    float best_ms = 1e30f;
    for (int planes = 1; planes <= 8 && planes <= p->n[0]; planes <<= 1) {
      p->planes_hint = planes;
      if (run_pass<T>(p, 5) != CCMF_OK) continue;
      hipEventRecord(e0, p->stream);
      for (int rep = 0; rep < 3; ++rep) run_pass<T>(p, 5);
      hipEventRecord(e1, p->stream);
      if (hipEventSynchronize(e1) != hipSuccess) break;
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      if (log) std::fprintf(stderr, "[ccmf tune] fused divergence, %d planes per block: %.1f us\n", planes, ms / 3 * 1e3);
      if (ms < best_ms) {
        best_ms = ms;
        best[12] = planes;
      }
    }
    p->planes_hint = best[12];
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(CCMF_EDEVICE, "autotune: %s", hipGetErrorString(e));
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = best;
  }
  p->tuned_B = p->B;
  return CCMF_OK;
}

template <typename T>
int solve_impl(ccmf_plan_s* p, const double* xi, int64_t nloads, double tol, const ccmf_options* o,
               double* geff, int32_t* iters, double* residual, double* dual_est, void* phi_dev,
               void* flux_dev) {
  ccmf_options opt;
  std::memset(&opt, 0, sizeof(opt));
  if (o) opt = *o;
  if (opt.delta == 0.0) opt.delta = 0.25;
  if (opt.max_iter == 0) opt.max_iter = 20000;
  if (opt.check_every == 0) opt.check_every = 32;
  if (opt.bb_min_corr == 0.0) opt.bb_min_corr = 0.2;
  if (opt.eta0 == 0.0) opt.eta0 = 1.0;
  if (opt.k0 == 0.0) opt.k0 = 100.0;
  if (!(opt.bb_min_corr >= 0.0 && opt.bb_min_corr <= 1.0)) return fail(CCMF_EINVAL, "bb_min_corr must lie in [0,1]");
  if (!(opt.eta0 > 0.0) || !std::isfinite(opt.eta0)) return fail(CCMF_EINVAL, "eta0 must be positive");
  if (!(opt.k0 > 0.0) || !std::isfinite(opt.k0)) return fail(CCMF_EINVAL, "k0 must be positive");
  if (!(opt.delta > 0.0 && opt.delta < 1.0)) return fail(CCMF_EINVAL, "delta must lie in (0,1)");
  if (opt.max_iter < 1) return fail(CCMF_EINVAL, "max_iter must be >= 1");
  if (opt.check_every < 1) return fail(CCMF_EINVAL, "check_every must be >= 1");
  if (opt.rule < 0 || opt.rule > 2) return fail(CCMF_EINVAL, "unknown penalty rule %d", opt.rule);
  if (!(opt.rho0 >= 0.0) || !std::isfinite(opt.rho0)) return fail(CCMF_EINVAL, "rho0 must be >= 0 and finite");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(CCMF_EINVAL, "tol must be positive and finite");
  if (nloads < 1 || !xi) return fail(CCMF_EINVAL, "need at least one load direction");
  if (!geff || !iters) return fail(CCMF_EINVAL, "geff and iters outputs are required");
  for (int64_t l = 0; l < nloads; ++l) {
    const double nr = std::sqrt(xi[3 * l] * xi[3 * l] + xi[3 * l + 1] * xi[3 * l + 1] + xi[3 * l + 2] * xi[3 * l + 2]);
    if (!(nr > 0.0) || !std::isfinite(nr)) return fail(CCMF_EINVAL, "load %lld is zero or not finite", (long long)l);
  }
  if (p->nfields * nloads > 65535) return fail(CCMF_EINVAL, "at most 65535 problems per solve");
  const bool warm = opt.warm_start != 0;
  if (warm && !(p->state_ready && p->B == p->nfields * nloads))
    return fail(CCMF_ESTATE, "warm start needs a preceding solve or ccmf_set_state with the same number of loads");
  int rc = ensure_state(p, nloads);
  if (rc) return rc;
  p->solved = false;
  p->state_ready = false;
  p->hist_valid = false;
  if (opt.record_history) {
    if (p->hist == nullptr || p->hist_len != opt.max_iter) {
      hipFree(p->hist);
      p->hist = nullptr;
      p->hist_len = 0;
      HIP_TRY(hipMalloc(&p->hist, (size_t)p->B * opt.max_iter * 4 * sizeof(double)));
      p->hist_len = opt.max_iter;
    }
    p->hist_valid = true;
  }

  for (int64_t b = 0; b < p->B; ++b) {
    const int64_t f = b / nloads, l = b % nloads;
    Prob& P = p->probh[b];
    const Prob kept = P;
    std::memset(&P, 0, sizeof(P));
    const double nr = std::sqrt(xi[3 * l] * xi[3 * l] + xi[3 * l + 1] * xi[3 * l + 1] + xi[3 * l + 2] * xi[3 * l + 2]);
    for (int c = 0; c < 3; ++c) P.xibar[c] = xi[3 * l + c] / nr;
    const bool any_pos = p->kmax[f] > 0.0;
    P.rho0 = opt.rho0 > 0.0 ? opt.rho0 : (any_pos ? p->kmin[f] : 1.0);
    P.lo = P.rho0 * 1e-6;   // hard limits of the adaptive penalty
    P.hi = P.rho0 * 1e6;
    P.bb_corr = opt.bb_min_corr;
    P.eta0 = opt.eta0;
    P.k0 = opt.k0;
    P.rho = P.rho0;
    P.rho_prev = P.rho0;
    P.tol = tol;
    P.delta = opt.delta;
    P.rule = opt.rule;
    P.max_iter = opt.max_iter;
    P.all_zero = any_pos ? 0 : 1;
    P.field = (int32_t)f;
    if (warm) {
      // resume the kept state k: penalties and iteration index carry over; the
      // state moves to ping-pong slot 0, where the iteration sequence starts
      P.rho = kept.rho;
      P.rho_prev = kept.rho_prev;
      P.k_off = kept.k_off + kept.k;
      if (kept.k & 1) {
        HIP_TRY(hipMemcpyAsync(static_cast<char*>(p->z[0]) + (size_t)b * 6 * p->N * p->esz,
                               static_cast<const char*>(p->z[1]) + (size_t)b * 6 * p->N * p->esz,
                               6 * p->N * p->esz, hipMemcpyDeviceToDevice, p->stream));
        HIP_TRY(hipMemcpyAsync(static_cast<char*>(p->a[0]) + (size_t)b * p->N * p->esz,
                               static_cast<const char*>(p->a[1]) + (size_t)b * p->N * p->esz,
                               p->N * p->esz, hipMemcpyDeviceToDevice, p->stream));
      }
    }
  }
  HIP_TRY(hipMemcpyAsync(p->prob, p->probh, (size_t)p->B * sizeof(Prob), hipMemcpyHostToDevice, p->stream));
  const Geo g = make_geo(p);
  if (!warm) {
    const int blocks = (int)std::min<uint64_t>(4096, (p->N + kThreads - 1) / kThreads);
    hipLaunchKernelGGL((k_init<T>), dim3(blocks, (unsigned)p->B), dim3(kThreads), 0, p->stream, g,
                       reinterpret_cast<const T*>(p->kap), reinterpret_cast<T*>(p->z[0]),
                       reinterpret_cast<T*>(p->a[0]), p->prob);
    HIP_LAUNCH_CHECK();
  }
  // tile widths of the spectral passes, timed on the initial state (results do
  // not depend on them); the graph below is captured with the chosen widths
  if (p->tuned_B != p->B || (opt.no_autotune != 0) != p->tuned_off) {
    p->drop_graph();
    if (opt.no_autotune) {
      for (int k = 0; k < 6; ++k) p->nlc_hint[k] = 0;
      for (int k = 0; k < 5; ++k) p->walk_hint[k] = 0;
      p->planes_hint = 0;
      p->tuned_B = p->B;
    } else if ((rc = autotune<T>(p))) {
      return rc;
    }
    p->tuned_off = opt.no_autotune != 0;
  }
  p->ev_used = 0;
  // HIP events recorded by graph nodes cannot be timed, so timed solves launch eagerly
  const bool timed = opt.time_kernels != 0;
  const bool eager = opt.eager != 0 || timed;
  if (eager) {
    bool all_done = false;
    for (int it = 0; it < opt.max_iter && !all_done; ++it) {
      if ((rc = run_iteration<T>(p, it, timed))) return rc;
      if ((it + 1) % opt.check_every == 0 || it + 1 == opt.max_iter) {
        HIP_TRY(hipMemcpyAsync(p->probh, p->prob, (size_t)p->B * sizeof(Prob), hipMemcpyDeviceToHost, p->stream));
        HIP_TRY(hipStreamSynchronize(p->stream));
        all_done = true;
        for (int64_t b = 0; b < p->B; ++b) all_done = all_done && p->probh[b].done != 0;
        if (timed && (rc = harvest_events(p))) return rc;
      }
    }
  } else {
    // One chunk of K iterations (K even, so the ping-pong parity repeats) is
    // captured once into a HIP graph and replayed; the kernels read the iteration
    // index from the device and finished problems return at once.  The host
    // keeps one chunk in flight and inspects the flags of the previous one.
    const int K = (opt.check_every + 1) & ~1;
    const double* hist_now = p->hist_valid ? p->hist : nullptr;
    if (!p->gexec || p->graph_iters != K || p->graph_hist != hist_now) {
      p->drop_graph();
      hipGraph_t graph = nullptr;
      HIP_TRY(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
      int crc = CCMF_OK;
      for (int j = 0; j < K && crc == CCMF_OK; ++j) crc = run_iteration<T>(p, j, false);
      hipError_t ce = hipStreamEndCapture(p->stream, &graph);
      if (crc) {
        if (graph) hipGraphDestroy(graph);
        return crc;
      }
      if (ce != hipSuccess) return fail(CCMF_EDEVICE, "graph capture: %s", hipGetErrorString(ce));
      ce = hipGraphInstantiate(&p->gexec, graph, nullptr, nullptr, 0);
      hipGraphDestroy(graph);
      if (ce != hipSuccess) {
        p->gexec = nullptr;
        return fail(CCMF_EDEVICE, "graph instantiate: %s", hipGetErrorString(ce));
      }
      p->graph_iters = K;
      p->graph_hist = hist_now;
    }
    const int chunks = (opt.max_iter + K - 1) / K;
    for (int c = 0; c < chunks; ++c) {
      HIP_TRY(hipGraphLaunch(p->gexec, p->stream));
      const int slot = c & 1;
      HIP_TRY(hipMemcpyAsync(p->flagsh[slot], p->prob, (size_t)p->B * sizeof(Prob), hipMemcpyDeviceToHost,
                             p->stream));
      HIP_TRY(hipEventRecord(p->fev[slot], p->stream));
      if (c >= 1) {
        HIP_TRY(hipEventSynchronize(p->fev[slot ^ 1]));
        bool all_done = true;
        for (int64_t b = 0; b < p->B; ++b) all_done = all_done && p->flagsh[slot ^ 1][b].done != 0;
        if (all_done) break;
      }
    }
  }
  HIP_TRY(hipMemcpyAsync(p->probh, p->prob, (size_t)p->B * sizeof(Prob), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (timed && (rc = harvest_events(p))) return rc;
  int status = CCMF_OK;
  for (int64_t b = 0; b < p->B; ++b) {
    const Prob& P = p->probh[b];
    if (P.done == 0) return fail(CCMF_EDEVICE, "problem %lld did not finish", (long long)b);
    if (P.done == 2) status = CCMF_NOT_CONVERGED;
    geff[b] = P.geff;
    iters[b] = P.k + 1;
    if (residual) residual[b] = P.res;
    if (dual_est) dual_est[b] = P.dual;
  }
  p->solved = true;
  p->state_ready = true;
  if (phi_dev) {
    HIP_TRY(hipMemcpyAsync(phi_dev, p->phi, (size_t)p->B * p->N * sizeof(double), hipMemcpyDeviceToDevice,
                           p->stream));
  }
  if (flux_dev) {
    const int blocks = (int)std::min<uint64_t>(4096, (p->N + kThreads - 1) / kThreads);
    hipLaunchKernelGGL((k_flux<T>), dim3(blocks, (unsigned)p->B), dim3(kThreads), 0, p->stream, g,
                       reinterpret_cast<const T*>(p->z[0]), reinterpret_cast<const T*>(p->z[1]),
                       reinterpret_cast<const T*>(p->a[0]), reinterpret_cast<const T*>(p->a[1]),
                       reinterpret_cast<T*>(flux_dev), p->prob);
    HIP_LAUNCH_CHECK();
  }
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (status == CCMF_NOT_CONVERGED) fail(CCMF_NOT_CONVERGED, "max_iter reached before the tolerance");
  return status;
}

template <typename T>
int grad_impl(ccmf_plan_s* p, const double* dl, void* dkap) {
  if (!p->solved) return fail(CCMF_ESTATE, "ccmf_grad_kappa needs a preceding ccmf_solve");
  if (!dl || !dkap) return fail(CCMF_EINVAL, "null argument");
  double* ddl = nullptr;
  HIP_TRY(hipMalloc(&ddl, (size_t)p->B * sizeof(double)));
  hipError_t e = hipMemcpyAsync(ddl, dl, (size_t)p->B * sizeof(double), hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) {
    const Geo g = make_geo(p);
    const int blocks = (int)std::min<uint64_t>(4096, (p->N + kThreads - 1) / kThreads);
    hipLaunchKernelGGL((k_grad<T>), dim3(blocks, (unsigned)p->nfields), dim3(kThreads), 0, p->stream, g,
                       reinterpret_cast<const T*>(p->z[0]), reinterpret_cast<const T*>(p->z[1]),
                       reinterpret_cast<const T*>(p->a[0]), reinterpret_cast<const T*>(p->a[1]),
                       p->phi, ddl, reinterpret_cast<T*>(dkap), p->prob);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  hipFree(ddl);
  if (e != hipSuccess) return fail(CCMF_EDEVICE, "gradient: %s", hipGetErrorString(e));
  return CCMF_OK;
}

template <typename T>
int certificate_impl(ccmf_plan_s* p, double* cert, double* sigma) {
  if (!p->solved) return fail(CCMF_ESTATE, "ccmf_certificate needs a preceding ccmf_solve");
  if (!cert) return fail(CCMF_EINVAL, "null argument");
  const Geo g = make_geo(p);
  const size_t n = (size_t)p->B * p->N;
  double* phic = nullptr;
  T* rc = nullptr;
  double* part = nullptr;
  const int blocks = (int)std::min<uint64_t>(1024, (p->N + kThreads - 1) / kThreads);
  hipError_t e = hipMalloc(&phic, n * sizeof(double));
  if (e == hipSuccess) {
    if (sizeof(T) == 8)
      rc = reinterpret_cast<T*>(phic);
    else
      e = hipMalloc(&rc, n * sizeof(T));
  }
  if (e == hipSuccess) e = hipMalloc(&part, (size_t)p->B * blocks * 3 * sizeof(double));
  int rc_status = CCMF_OK;
  std::vector<double> h((size_t)p->B * blocks * 3);
  if (e == hipSuccess) {
    hipLaunchKernelGGL((k_cert_r<T>), dim3(blocks, (unsigned)p->B), dim3(kThreads), 0, p->stream, g,
                       reinterpret_cast<const T*>(p->z[0]), reinterpret_cast<const T*>(p->z[1]),
                       reinterpret_cast<const T*>(p->a[0]), reinterpret_cast<const T*>(p->a[1]), rc, p->prob);
    e = hipGetLastError();
  }
  if (e == hipSuccess) rc_status = launch_laplace<T>(p, rc, phic, p->B, nullptr);
  if (e == hipSuccess && rc_status == CCMF_OK) {
    hipLaunchKernelGGL((k_cert_sigma<T>), dim3(blocks, (unsigned)p->B), dim3(kThreads), 0, p->stream, g,
                       reinterpret_cast<const T*>(p->kap), reinterpret_cast<const T*>(p->z[0]),
                       reinterpret_cast<const T*>(p->z[1]), reinterpret_cast<const T*>(p->a[0]),
                       reinterpret_cast<const T*>(p->a[1]), phic, part, p->prob);
    e = hipGetLastError();
    if (e == hipSuccess)
      e = hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  }
  if ((void*)rc != (void*)phic) hipFree(rc);
  hipFree(phic);
  hipFree(part);
  if (rc_status) return rc_status;
  if (e != hipSuccess) return fail(CCMF_EDEVICE, "certificate: %s", hipGetErrorString(e));
  for (int64_t b = 0; b < p->B; ++b) {
    double mx = 0.0, bad = 0.0, yn = 0.0;
    for (int bl = 0; bl < blocks; ++bl) {
      const double* o = &h[((size_t)b * blocks + bl) * 3];
      mx = std::max(mx, o[0]);
      bad = std::max(bad, o[1]);
      yn = std::max(yn, o[2]);
    }
    const double dual = p->probh[b].dual;
    // a pore carrying flux (beyond rounding) leaves no feasible scaling
    const bool undefined = bad > 1e-9 * std::max(1.0, yn);
    cert[b] = undefined ? -INFINITY : dual / std::max(1.0, mx);
    if (sigma) sigma[b] = undefined ? INFINITY : mx;
  }
  return CCMF_OK;
}

}  // namespace

extern "C" {

int ccmf_setup(ccmf_plan* out, const int64_t dims[3], int64_t n_fields, int32_t dtype, const void* kappa_dev,
               void* stream) {
  if (!out || !dims || !kappa_dev) return fail(CCMF_EINVAL, "null argument");
  *out = nullptr;
  if (dtype != CCMF_F64 && dtype != CCMF_F32) return fail(CCMF_EINVAL, "unknown dtype %d", dtype);
  if (n_fields < 1) return fail(CCMF_EINVAL, "n_fields must be >= 1");
  int64_t N = 1;
  for (int c = 0; c < 3; ++c) {
    if (dims[c] < 1) return fail(CCMF_EINVAL, "dims[%d] = %lld must be >= 1", c, (long long)dims[c]);
    N *= dims[c];
    if (N >= (int64_t)1 << 31) return fail(CCMF_EINVAL, "grid too large (N must be < 2^31)");
  }
  ccmf_plan_s* p = new (std::nothrow) ccmf_plan_s();
  if (!p) return fail(CCMF_ENOMEM, "host allocation failed");
  p->dt = dtype;
  p->esz = dtype == CCMF_F64 ? 8 : 4;
  for (int c = 0; c < 3; ++c) p->n[c] = (int)dims[c];
  p->N = (uint32_t)N;
  p->nfields = n_fields;
  p->stream = reinterpret_cast<hipStream_t>(stream);
  if (p->stream == nullptr) {
    // the null stream cannot be captured into a graph: use a blocking stream of
    // our own (default priority), ordered with the null stream by its semantics
    hipError_t se = hipStreamCreate(&p->stream);
    if (se != hipSuccess) {
      delete p;
      return fail(CCMF_EDEVICE, "stream creation: %s", hipGetErrorString(se));
    }
    p->own_stream = true;
  }
  for (int c = 0; c < 3; ++c) {
    if ((size_t)2 * 2 * p->n[c] * p->esz > 65536) {
      delete p;
      return fail(CCMF_EINVAL, "dims[%d] = %d exceeds the transform tile limit", c, p->n[c]);
    }
  }
  int rc;
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) {
    delete p;
    return fail(CCMF_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  }
  e = hipMalloc(&p->kap, (size_t)n_fields * N * p->esz);
  if (e != hipSuccess) {
    delete p;
    return fail(CCMF_ENOMEM, "kappa allocation: %s", hipGetErrorString(e));
  }
  e = hipMemcpyAsync(p->kap, kappa_dev, (size_t)n_fields * N * p->esz, hipMemcpyDeviceToDevice, p->stream);
  if (e != hipSuccess) {
    delete p;
    return fail(CCMF_EDEVICE, "kappa copy: %s", hipGetErrorString(e));
  }
  for (int c = 0; c < 3; ++c) {
    rc = upload_axis(p->ax[c], p->n[c]);
    if (rc) {
      delete p;
      return rc;
    }
  }
  rc = p->dt == CCMF_F64 ? kappa_stats<double>(p) : kappa_stats<float>(p);
  if (rc) {
    delete p;
    return rc;
  }
  *out = p;
  return CCMF_OK;
}

int ccmf_solve(ccmf_plan p, const double* xi, int64_t n_loads, double tol, const ccmf_options* opt, double* geff,
               int32_t* iters, double* residual, double* dual_est, void* phi_dev, void* flux_dev) {
  if (!p) return fail(CCMF_EINVAL, "null plan");
  return p->dt == CCMF_F64
             ? solve_impl<double>(p, xi, n_loads, tol, opt, geff, iters, residual, dual_est, phi_dev, flux_dev)
             : solve_impl<float>(p, xi, n_loads, tol, opt, geff, iters, residual, dual_est, phi_dev, flux_dev);
}

int ccmf_grad_kappa(ccmf_plan p, const double* dL_dgeff, void* dkappa_dev) {
  if (!p) return fail(CCMF_EINVAL, "null plan");
  return p->dt == CCMF_F64 ? grad_impl<double>(p, dL_dgeff, dkappa_dev) : grad_impl<float>(p, dL_dgeff, dkappa_dev);
}

int ccmf_certificate(ccmf_plan p, double* cert, double* sigma) {
  if (!p) return fail(CCMF_EINVAL, "null plan");
  return p->dt == CCMF_F64 ? certificate_impl<double>(p, cert, sigma) : certificate_impl<float>(p, cert, sigma);
}

int ccmf_mean_flux(ccmf_plan p, double* mflux) {
  if (!p || !mflux) return fail(CCMF_EINVAL, "null argument");
  if (!p->solved) return fail(CCMF_ESTATE, "ccmf_mean_flux needs a preceding ccmf_solve");
  for (int64_t b = 0; b < p->B; ++b)
    for (int c = 0; c < 3; ++c) mflux[3 * b + c] = p->probh[b].mflux[c];
  return CCMF_OK;
}

int ccmf_history(ccmf_plan p, int32_t max_len, double* out) {
  if (!p || !out || max_len < 1) return fail(CCMF_EINVAL, "bad argument");
  if (!p->solved || !p->hist_valid) return fail(CCMF_ESTATE, "the last solve recorded no history");
  const int rows = std::min<int>(max_len, p->hist_len);
  std::vector<double> h((size_t)p->B * p->hist_len * 4);
  HIP_TRY(hipMemcpyAsync(h.data(), p->hist, h.size() * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  for (int64_t b = 0; b < p->B; ++b) {
    const int n = p->probh[b].k + 1;  // iterations taken by problem b
    for (int i = 0; i < max_len; ++i)
      for (int q = 0; q < 4; ++q)
        out[((size_t)b * max_len + i) * 4 + q] =
            (i < rows && i < n) ? h[((size_t)b * p->hist_len + i) * 4 + q] : std::nan("");
  }
  return CCMF_OK;
}

int ccmf_get_state(ccmf_plan p, void* v_dev, void* e_dev, double* rho, int32_t* k) {
  if (!p) return fail(CCMF_EINVAL, "null plan");
  if (!p->state_ready) return fail(CCMF_ESTATE, "ccmf_get_state needs a preceding ccmf_solve");
  if (v_dev || e_dev) {
    const Geo g = make_geo(p);
    const int blocks = (int)std::min<uint64_t>(4096, (p->N + kThreads - 1) / kThreads);
    if (p->dt == CCMF_F64) {
      hipLaunchKernelGGL((k_get_state<double>), dim3(blocks, (unsigned)p->B), dim3(kThreads), 0, p->stream, g,
                         static_cast<const double*>(p->z[0]), static_cast<const double*>(p->z[1]),
                         static_cast<const double*>(p->a[0]), static_cast<const double*>(p->a[1]),
                         static_cast<double*>(v_dev), static_cast<double*>(e_dev), p->prob);
    } else {
      hipLaunchKernelGGL((k_get_state<float>), dim3(blocks, (unsigned)p->B), dim3(kThreads), 0, p->stream, g,
                         static_cast<const float*>(p->z[0]), static_cast<const float*>(p->z[1]),
                         static_cast<const float*>(p->a[0]), static_cast<const float*>(p->a[1]),
                         static_cast<float*>(v_dev), static_cast<float*>(e_dev), p->prob);
    }
    HIP_LAUNCH_CHECK();
    HIP_TRY(hipStreamSynchronize(p->stream));
  }
  for (int64_t b = 0; b < p->B; ++b) {
    if (rho) rho[b] = p->probh[b].rho;
    if (k) k[b] = p->probh[b].k_off + p->probh[b].k;
  }
  return CCMF_OK;
}

int ccmf_set_state(ccmf_plan p, int64_t n_loads, const void* v_dev, const void* e_dev, const double* rho,
                   const int32_t* k) {
  if (!p || !v_dev || !e_dev || !rho || !k) return fail(CCMF_EINVAL, "null argument");
  if (n_loads < 1 || p->nfields * n_loads > 65535) return fail(CCMF_EINVAL, "n_loads out of range");
  const int64_t B = p->nfields * n_loads;
  for (int64_t b = 0; b < B; ++b) {
    if (!(rho[b] > 0.0) || !std::isfinite(rho[b])) return fail(CCMF_EINVAL, "rho[%lld] must be positive", (long long)b);
    if (k[b] < 0) return fail(CCMF_EINVAL, "k[%lld] must be >= 0", (long long)b);
  }
  int rc = ensure_state(p, n_loads);
  if (rc) return rc;
  p->solved = false;
  p->state_ready = false;
  for (int64_t b = 0; b < B; ++b) {
    Prob& P = p->probh[b];
    std::memset(&P, 0, sizeof(P));
    P.rho = rho[b];
    P.rho_prev = rho[b];
    P.k_off = k[b];
    P.field = (int32_t)(b / n_loads);
  }
  HIP_TRY(hipMemcpyAsync(p->prob, p->probh, (size_t)B * sizeof(Prob), hipMemcpyHostToDevice, p->stream));
  const Geo g = make_geo(p);
  const int blocks = p->upd_blocks;  // one count per block in the partials buffer
  if (p->dt == CCMF_F64) {
    hipLaunchKernelGGL((k_set_state<double>), dim3(blocks, (unsigned)B), dim3(kThreads), 0, p->stream, g,
                       static_cast<const double*>(v_dev), static_cast<const double*>(e_dev),
                       static_cast<double*>(p->z[0]), static_cast<double*>(p->a[0]), p->partials, p->prob);
  } else {
    hipLaunchKernelGGL((k_set_state<float>), dim3(blocks, (unsigned)B), dim3(kThreads), 0, p->stream, g,
                       static_cast<const float*>(v_dev), static_cast<const float*>(e_dev),
                       static_cast<float*>(p->z[0]), static_cast<float*>(p->a[0]), p->partials, p->prob);
  }
  HIP_LAUNCH_CHECK();
  std::vector<double> cnt((size_t)B * blocks);
  HIP_TRY(hipMemcpy2DAsync(cnt.data(), sizeof(double), p->partials, kNQ * sizeof(double), sizeof(double),
                           (size_t)B * blocks, hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  double bad = 0.0;
  for (double c : cnt) bad += c;
  if (bad > 0.0)
    return fail(CCMF_EINVAL, "v and e are not non-negative multiples of one vector at %.0f voxels", bad);
  p->state_ready = true;
  return CCMF_OK;
}

int ccmf_kernel_times(ccmf_plan p, double* avg_ms, int64_t* count, double* bytes_per_launch) {
  if (!p) return fail(CCMF_EINVAL, "null plan");
  if (avg_ms) *avg_ms = p->kt_count ? p->kt_sum / (double)p->kt_count : 0.0;
  if (count) *count = p->kt_count;
  // fused update per voxel: read z (6), alpha, gamma (plan dtype) and phi (FP64);
  // write z (6), alpha (plan dtype)
  if (bytes_per_launch) *bytes_per_launch = (15.0 * (double)p->esz + 8.0) * (double)p->N;
  p->kt_sum = 0.0;
  p->kt_count = 0;
  return CCMF_OK;
}

int ccmf_laplace_pinv(ccmf_plan p, const void* r_dev, void* phi_dev, int64_t count) {
  if (!p || !r_dev || !phi_dev || count < 1) return fail(CCMF_EINVAL, "bad argument");
  const size_t n = (size_t)count * p->N;
  void* tmp = nullptr;
  if (p->dt == CCMF_F64) {
    if (r_dev != phi_dev) HIP_TRY(hipMemcpyAsync(phi_dev, r_dev, n * 8, hipMemcpyDeviceToDevice, p->stream));
    tmp = phi_dev;
  } else {
    HIP_TRY(hipMalloc(&tmp, n * 4));
    HIP_TRY(hipMemcpyAsync(tmp, r_dev, n * 4, hipMemcpyDeviceToDevice, p->stream));
  }
  int rc = p->dt == CCMF_F64
               ? launch_laplace<double>(p, reinterpret_cast<double*>(tmp), reinterpret_cast<double*>(phi_dev),
                                        count, nullptr)
               : launch_laplace<float>(p, reinterpret_cast<float*>(tmp), reinterpret_cast<double*>(phi_dev),
                                       count, nullptr);
  hipError_t e = hipStreamSynchronize(p->stream);
  if (tmp != phi_dev) hipFree(tmp);
  if (rc) return rc;
  if (e != hipSuccess) return fail(CCMF_EDEVICE, "laplace: %s", hipGetErrorString(e));
  return CCMF_OK;
}

int ccmf_hartley_axis(ccmf_plan p, void* data_dev, int64_t count, int32_t axis) {
  if (!p || !data_dev || count < 1 || axis < 0 || axis > 2) return fail(CCMF_EINVAL, "bad argument");
  if (p->n[axis] == 1) return CCMF_OK;
  int rc;
  if (p->dt == CCMF_F64) {
    double* d = reinterpret_cast<double*>(data_dev);
    rc = launch_hartley<double, double, double>(p, d, d, count, axis, false, nullptr);
  } else {
    float* d = reinterpret_cast<float*>(data_dev);
    rc = launch_hartley<float, float, float>(p, d, d, count, axis, false, nullptr);
  }
  if (rc) return rc;
  HIP_TRY(hipStreamSynchronize(p->stream));
  return CCMF_OK;
}

int ccmf_stream_copy(void* dst_dev, const void* src_dev, int64_t nbytes, void* stream) {
  if (!dst_dev || !src_dev || nbytes < 0 || (nbytes % 16) != 0) return fail(CCMF_EINVAL, "bad argument");
  const size_t n16 = (size_t)nbytes / 16;
  if (n16 == 0) return CCMF_OK;
  // one 16-byte element per thread over a grid that covers the buffer: blocks are
  // dispatched in address order, which keeps the set of open DRAM pages small (a
  // grid-stride loop over a few thousand blocks measured ~25 % slower on MI355X)
  const unsigned blocks = (unsigned)std::min<size_t>(size_t(1) << 30, (n16 + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(k_copy16, dim3(blocks), dim3(kThreads), 0, reinterpret_cast<hipStream_t>(stream),
                     reinterpret_cast<const uint4*>(src_dev), reinterpret_cast<uint4*>(dst_dev), n16);
  HIP_LAUNCH_CHECK();
  return CCMF_OK;
}

void ccmf_destroy(ccmf_plan p) { delete p; }

const char* ccmf_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
