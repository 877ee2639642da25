// The extern "C" entry points of libttm: argument validation on the host,
// workspace carving, and the launch sequence of each call (all asynchronous on
// the caller's stream).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <utility>
#include <vector>

#include "ttm_internal.h"

namespace ttm {

// Bump allocator over the caller's workspace; with base == nullptr it only
// measures.  Every block is 256-byte aligned.
struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(void* b) : base(static_cast<char*>(b)) {}
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
  size_t size() const { return (off + 255) & ~size_t(255); }
};

static bool dims_ok(const ttm_dims& d) { return d.n0 > 0 && d.n1 > 0 && d.n2 > 0; }
static bool image_dims_ok(const ttm_dims& N) {
  return supported_len(N.n0) && supported_len(N.n1) && supported_len(N.n2);
}
static bool fits(const ttm_dims& L, const ttm_dims& N) {
  return L.n0 <= N.n0 && L.n1 <= N.n1 && L.n2 <= N.n2;
}

static Geo make_geo(const ttm_dims& N, const ttm_dims& L) {
  Geo g;
  g.n0 = N.n0; g.n1 = N.n1; g.n2 = N.n2; g.h2 = N.n2 / 2 + 1; g.p2 = row_pitch(N.n2);
  g.L0 = L.n0; g.L1 = L.n1; g.L2 = L.n2;
  g.c0 = L.n0 / 2; g.c1 = L.n1 / 2; g.c2 = L.n2 / 2;
  return g;
}

#define TTM_TRY(expr)                         \
  do {                                        \
    if ((expr) != hipSuccess) return TTM_E_HIP; \
  } while (0)

// ---- optional event-pair instrumentation --------------------------------------
enum ProfClass { PC_STATS = 0, PC_ROWS, PC_PEN_FWD, PC_PASS1, PC_PEN_INV, PC_PASS3, PC_PEAKS, PC_POSE,
                 PC_BUILD, PC_EPI, PC_RMAP_SCAN, PC_RMAP_POLISH, PC_SNORM, PC_COUNT };
static const char* kProfNames[PC_COUNT] = {"image_moments", "r2c_rows", "pencils_fwd", "pass1_fanout",
                                           "pencils_inv", "pass3_c2r_reduce", "peaks", "pose",
                                           "tensor_build", "classical_epilogue", "rmap_scan", "rmap_polish",
                                           "snorm"};
struct Prof {
  std::mutex mu;
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
  std::vector<std::pair<int, int>> used;   // (class, pool index)
};
static Prof& prof() {
  static Prof p;
  return p;
}
// set on this thread while a call that must create nothing runs (the
// profiler's event pairs are created lazily)
static bool& prof_suppressed() {
  static thread_local bool off = false;
  return off;
}
struct ProfSuppress {
  ProfSuppress() { prof_suppressed() = true; }
  ~ProfSuppress() { prof_suppressed() = false; }
};
// RAII: records the start event on construction and the stop event on
// destruction (both on stream s) when profiling is on.
struct ProfScope {
  int idx = -1;
  hipStream_t s;
  ProfScope(int cls, hipStream_t st) : s(st) {
    if (prof_suppressed()) return;
    Prof& p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    if (!p.on) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    if (p.used.size() == p.pool.size()) {
      hipEvent_t a, b;
      if (hipEventCreate(&a) != hipSuccess) return;
      if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return; }
      p.pool.emplace_back(a, b);
    }
    idx = (int)p.used.size();
    p.used.emplace_back(cls, idx);
    (void)hipEventRecord(p.pool[idx].first, s);
  }
  ~ProfScope() {
    if (idx < 0) return;
    Prof& p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    (void)hipEventRecord(p.pool[idx].second, s);
  }
};
#define TTM_PROF(cls, expr)                  \
  do {                                       \
    ProfScope _ps(cls, stream);              \
    TTM_TRY(expr);                           \
  } while (0)

// ---- layouts ----------------------------------------------------------------
struct BuildWs {
  float* quats; double* weights; double* rstats; double* coef; float* rtab;
};
static BuildWs build_layout(Carve& c, int nrot, int K) {
  BuildWs w;
  w.rtab = c.take<float>((size_t)nrot * 9);
  w.quats = c.take<float>((size_t)nrot * 4);
  w.weights = c.take<double>((size_t)nrot);
  w.rstats = c.take<double>((size_t)nrot * 2);
  w.coef = c.take<double>((size_t)nrot * K);
  return w;
}

struct CorrWs {
  float2* Xf; float2* Xg; float2* H; double* stats; double* partials; float* mu;
  float* wtmp;   // w when the caller passes none (the two-pass inverse reads it back)
};
static CorrWs corr_layout(Carve& c, const Geo& g, int K) {
  CorrWs w;
  w.Xf = c.take<float2>(g.half());
  w.Xg = c.take<float2>(g.half());
  w.H = c.take<float2>(g.half() * (size_t)(K + 2));
  w.stats = c.take<double>(4);
  w.partials = c.take<double>(3 * kStatPartials);
  w.mu = c.take<float>(kMaxK);
  w.wtmp = two_pass_supported(g) ? c.take<float>((size_t)g.vol()) : nullptr;
  return w;
}

struct PoseWs {
  unsigned* hist; unsigned* ctrl; unsigned long long* allc; unsigned long long* cand; double* stats;
  double* partials; int* cand_pos; double* seeds; PoseScratch ps;
  // refine 3: two sets of per-candidate moved flags; a round reads the
  // previous round's set as its active mask and writes the other
  int* moved[2];
};
// peaks = false: only the pose part (poses at given positions, no peak
// search buffers)
static PoseWs pose_layout(Carve& c, const Geo& g, int max_peaks, int K, int refine, int n_seeds,
                          bool peaks = true) {
  PoseWs w;
  const size_t nb = (size_t)max_peaks * (refine ? 27 : 1);
  w.hist = peaks ? c.take<unsigned>(kHistBins) : nullptr;
  w.ctrl = peaks ? c.take<unsigned>(kPeakCtrlWords) : nullptr;
  w.allc = peaks ? c.take<unsigned long long>((size_t)peaks_bigcap(g)) : nullptr;
  w.cand = peaks ? c.take<unsigned long long>(kCandCap) : nullptr;
  w.seeds = c.take<double>((size_t)n_seeds * 4);
  w.ps.seeds = w.seeds;
  w.stats = c.take<double>(4);
  w.partials = c.take<double>(3 * kStatPartials);
  w.cand_pos = peaks ? c.take<int>((size_t)max_peaks * 3) : nullptr;
  w.ps.C = c.take<double>(nb * (size_t)K);
  w.ps.w = c.take<double>(nb);
  w.ps.ok = c.take<int>(nb);
  w.ps.q = c.take<float>(nb * 4);
  w.ps.lam = c.take<double>(nb);
  w.ps.flags = c.take<int>(nb);
  w.ps.ncc = c.take<double>(nb);
  w.ps.mlist = c.take<unsigned>((size_t)g.L0 * g.L1 * g.L2);
  w.ps.mval = c.take<float>((size_t)g.L0 * g.L1 * g.L2);
  w.ps.mcount = c.take<int>(2);
  w.ps.mom = c.take<double>(nb * 3);
  w.ps.mbits = c.take<unsigned long long>((size_t)mask_bricks(g.L0, g.L1, g.L2));
  w.ps.active = nullptr;
  w.moved[0] = w.moved[1] = nullptr;
  if (refine == 3)
    for (int i = 0; i < 2; ++i) w.moved[i] = c.take<int>((size_t)max_peaks);
  return w;
}

// refine 3: after the first round (the refinement of refine 2 from the
// start positions, already written to the outputs, with w.moved[0] set for
// the candidates that moved), rounds on the candidates whose position
// changed in the round before, until none moves or kRefineRounds rounds in
// all; each round starts from the candidates' rows of out_pos and writes its
// results to the same rows.  Most candidates move in the first round, so the
// second spreads each candidate's neighbours over 9 blocks as the first
// does; the later rounds, with few candidates left, over 27.  tensor(pos,
// count_dev, count_host, ps) fills the pose scratch ps with C_n at the 27
// neighbours of the candidates that ps.active marks.
template <class TensorFn>
static ttm_status refine_rounds(const Geo& g, const float* score, int order_n, const ttm_options* opt,
                                int max_peaks, const int* count_dev, int count_host, const float* image,
                                const float* tmpl, const float* mask, int32_t* out_pos, float* out_quat,
                                double* out_lambda, float* out_score, int32_t* out_flags, double* out_C, PoseWs& w,
                                TensorFn tensor, hipStream_t stream) {
  for (int r = 1; r < kRefineRounds; ++r) {
    PoseScratch ps = w.ps;
    ps.active = w.moved[(r - 1) & 1];
    TTM_PROF(PC_POSE, tensor(out_pos, count_dev, count_host, ps));
    TTM_PROF(PC_POSE, launch_pose_solve(g, score, order_n, opt->n_seeds, opt->hopm_max_iter, opt->hopm_tol,
                                        max_peaks, 2, out_pos, count_dev, count_host, image, tmpl, mask, out_pos,
                                        out_quat, out_lambda, out_score, out_flags, out_C, ps, stream, true,
                                        r == 1 ? 9 : 27, w.moved[r & 1]));
  }
  return TTM_OK;
}

constexpr int kClassicalBatch = 32;
struct ClassWs {
  float* quats; double* rstats; float2* Xf; float2* Xg; float2* H; float* tbatch; float2* bbank;
  float* w; double* stats; double* partials;
};
static ClassWs class_layout(Carve& c, const Geo& g, int nrot) {
  ClassWs w;
  const int B = nrot < kClassicalBatch ? nrot : kClassicalBatch;
  const int nH = B > 2 ? B : 2;
  const size_t L3 = (size_t)g.L0 * g.L1 * g.L2;
  w.quats = c.take<float>((size_t)nrot * 4);
  w.rstats = c.take<double>((size_t)nrot * 2);
  w.Xf = c.take<float2>(g.half());
  w.Xg = c.take<float2>(g.half());
  w.H = c.take<float2>(g.half() * (size_t)nH);
  w.tbatch = c.take<float>(L3 * (size_t)(B > 1 ? B : 1));
  w.bbank = c.take<float2>(g.bank_slab() * (size_t)(B > 1 ? B : 1));
  w.w = c.take<float>(g.vol());
  w.stats = c.take<double>(4);
  w.partials = c.take<double>(3 * kStatPartials);
  return w;
}

// forward axis-2 and axis-1 transforms of the image and of its square
// stats_in (optional): the image statistics (mean, variance, mask sum) taken
// elsewhere (the whole image of a tile); otherwise they are computed here,
// with the multiplicities of order mu_order into mu if mu is given
static ttm_status image_forward(const Geo& g, const float* image, float2* Xf, float2* Xg,
                                double* stats, double* partials, const float* mask, hipStream_t stream,
                                const double* stats_in = nullptr, int mu_order = 0, float* mu = nullptr) {
  const long L3 = (long)g.L0 * g.L1 * g.L2;
  const long rows = (long)g.n0 * g.n1;
  if (!stats_in)
    TTM_PROF(PC_STATS, launch_image_stats(image, g.vol(), mask, L3, partials, stats, stream, mu_order, mu));
  const double* st = stats_in ? stats_in : stats;
  TTM_PROF(PC_ROWS, launch_r2c_rows(g.n2, image, g.n2, g.n2, rows, Xf, Xg, rows, 0, 1, st, stream));
  TTM_PROF(PC_PEN_FWD, launch_pencils(g.n1, false, Xf, (long)g.n0 * g.p2, g.p2, (long)g.n1 * g.p2, g.p2, g.n1, 0,
                                      0, g.n1 - 1, 2, (long)(Xg - Xf), stream));
  return TTM_OK;
}

// bank entries for nent real [L0][L1][L2] blocks: rows R2C then axis-1 forward
static ttm_status bank_forward(const Geo& g, const float* src, int nent, float2* bank, hipStream_t stream) {
  const long rows = (long)nent * g.L0 * g.L1;
  TTM_PROF(PC_ROWS, launch_r2c_rows(g.n2, src, g.L2, g.L2, rows, bank, nullptr, g.L1, g.n1, 0, nullptr, stream));
  TTM_PROF(PC_PEN_FWD, launch_pencils(g.n1, false, bank, (long)nent * g.L0 * g.p2, g.p2, (long)g.n1 * g.p2, g.p2,
                                      g.L1, 0, 0, g.n1 - 1, 1, 0, stream));
  return TTM_OK;
}

// axis-1 inverse of nb arrays (half elements apart) after pass 1: only the
// planes x0 of the valid region hold data, only rows x1 of the valid region
// are stored (with the axis-1 centre shift)
static hipError_t pencils_inverse_valid(const Geo& g, float2* H, int nb, long half, hipStream_t stream) {
  const long plane = (long)g.n1 * g.p2;
  return launch_pencils(g.n1, true, H + (long)g.lo0() * plane, (long)(g.hi0() - g.lo0() + 1) * g.p2, g.p2, plane,
                        g.p2, g.n1, g.c1, g.lo1(), g.hi1(), nb, half, stream);
}

#define TTM_CALL(expr)                     \
  do {                                     \
    const ttm_status _st = (expr);         \
    if (_st != TTM_OK) return _st;         \
  } while (0)

// ---- the static scratch of ttm_pose_at_noalloc -------------------------------------
// Device memory that no call allocates: one array per GPU in the library's
// code object, held until the process ends.  In host code `scratch` names a
// host-side stand-in; its device address on the current GPU comes from
// hipGetSymbolAddress, taken once per device and kept.
constexpr size_t kStaticScratchBytes = size_t(8) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;

// the device address of `scratch` on the GPU of `stream` (which must be the
// current device: the symbol is resolved there)
static ttm_status static_scratch(hipStream_t stream, void** out) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int cur = 0;
  TTM_TRY(hipGetDevice(&cur));
  if (stream) {
    hipDevice_t sd = 0;
    TTM_TRY(hipStreamGetDevice(stream, &sd));
    if ((int)sd != cur) return TTM_E_ARG;
  }
  if (cur < 0 || cur >= kMaxDevices) return TTM_E_ARG;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[cur]) {
    void* p = nullptr;
    TTM_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return TTM_E_HIP;
    addr[cur] = p;
  }
  *out = addr[cur];
  return TTM_OK;
}

// the finiteness check of ttm_options.check_finite: the float64 moments
// (sum f, sum f^2 as mean and variance, and sum m) are finite exactly when no
// input value is a NaN or an infinity; they are copied to the host and waited
// for
static ttm_status moments_finite(const double* stats_dev, hipStream_t stream) {
  double h[3] = {0.0, 0.0, 0.0};
  TTM_TRY(hipMemcpyAsync(h, stats_dev, sizeof(h), hipMemcpyDeviceToHost, stream));
  TTM_TRY(hipStreamSynchronize(stream));
  for (double v : h)
    if (!std::isfinite(v)) return TTM_E_NONFINITE;
  return TTM_OK;
}

}  // namespace ttm

using namespace ttm;

extern "C" {

void ttm_default_options(ttm_options* o) {
  if (!o) return;
  o->eps_v = 1e-5f;
  o->threshold = 0.0f;
  o->min_dist = 8.0f;
  o->max_peaks = 64;
  o->n_seeds = 4096;
  o->hopm_max_iter = 1000;
  o->hopm_tol = 1e-12;
  o->refine = 0;
  o->check_finite = 0;
}

int32_t ttm_num_components(int32_t n) {
  if (n < 2 || n > kMaxOrder || (n & 1)) return TTM_E_ARG;
  return num_components(n);
}

int32_t ttm_supported_length(int32_t n) { return supported_len(n) ? 1 : 0; }

const char* ttm_status_string(int32_t s) {
  switch (s) {
    case TTM_OK: return "TTM_OK";
    case TTM_E_ARG: return "TTM_E_ARG: invalid argument";
    case TTM_E_SIZE: return "TTM_E_SIZE: unsupported or inconsistent size";
    case TTM_E_WORKSPACE: return "TTM_E_WORKSPACE: workspace missing or too small";
    case TTM_E_HIP: return "TTM_E_HIP: HIP launch failed";
    case TTM_E_NONFINITE: return "TTM_E_NONFINITE: non-finite input";
    default: return "unknown status";
  }
}

size_t ttm_bank_bytes(ttm_dims N, ttm_dims L, int32_t K) {
  if (!dims_ok(N) || !dims_ok(L) || K < 1) return 0;
  return (size_t)(K + 1) * L.n0 * N.n1 * row_pitch(N.n2) * sizeof(float2);
}

size_t ttm_build_workspace_bytes(ttm_dims L, int32_t order_n, int32_t n_rot, ttm_dims N) {
  (void)L; (void)N;
  const int K = ttm_num_components(order_n);
  if (K < 0 || n_rot < 1) return 0;
  Carve c(nullptr);
  build_layout(c, n_rot, K);
  return c.size();
}

ttm_status ttm_build_tensor_template(const float* tmpl, const float* mask, ttm_dims L, int32_t order_n,
                                     const float* quats_host, const double* weights_host, int32_t n_rot,
                                     float* out_components, ttm_dims N, void* out_bank, void* ws,
                                     size_t ws_bytes, hipStream_t stream) {
  if (!tmpl || !mask || !quats_host || !weights_host || !out_components) return TTM_E_ARG;
  const int K = ttm_num_components(order_n);
  if (K < 0 || n_rot < 1) return TTM_E_ARG;
  if (!dims_ok(L) || L.n2 > 512) return TTM_E_SIZE;
  if ((long)L.n0 * L.n1 * L.n2 > (1L << 24)) return TTM_E_SIZE;
  double wsum = 0.0;
  for (int j = 0; j < n_rot; ++j) {
    const float* q = quats_host + 4 * j;
    const double nq = (double)q[0] * q[0] + (double)q[1] * q[1] + (double)q[2] * q[2] + (double)q[3] * q[3];
    if (!std::isfinite(nq) || nq <= 0.0) return TTM_E_ARG;
    if (!std::isfinite(weights_host[j])) return TTM_E_ARG;
    wsum += weights_host[j];
  }
  if (std::fabs(wsum - 1.0) > 1e-6) return TTM_E_ARG;
  if (out_bank) {
    if (!image_dims_ok(N)) return TTM_E_SIZE;
    if (!fits(L, N)) return TTM_E_SIZE;
  }
  if (!ws || ws_bytes < ttm_build_workspace_bytes(L, order_n, n_rot, N)) return TTM_E_WORKSPACE;
  Carve c(ws);
  BuildWs w = build_layout(c, n_rot, K);
  TTM_TRY(hipMemcpyAsync(w.quats, quats_host, sizeof(float) * 4 * (size_t)n_rot, hipMemcpyHostToDevice, stream));
  TTM_TRY(hipMemcpyAsync(w.weights, weights_host, sizeof(double) * (size_t)n_rot, hipMemcpyHostToDevice, stream));
  // the host arrays are read before this call returns, so the caller may
  // free or reuse them at once: an asynchronous copy from pageable memory may
  // otherwise be staged after the caller has released it
  TTM_TRY(hipStreamSynchronize(stream));
  TTM_PROF(PC_BUILD, launch_rot_stats(tmpl, mask, L.n0, L.n1, L.n2, w.quats, n_rot, w.rstats, stream));
  TTM_PROF(PC_BUILD, launch_build_coef(w.quats, w.weights, w.rstats, n_rot, order_n, w.coef, stream));
  TTM_PROF(PC_BUILD, launch_build_accum(tmpl, mask, L.n0, L.n1, L.n2, w.quats, w.rstats, w.coef, n_rot, K, out_components,
                             w.rtab, stream));
  if (out_bank) {
    const Geo g = make_geo(N, L);
    float2* bank = static_cast<float2*>(out_bank);
    TTM_CALL(bank_forward(g, out_components, K, bank, stream));
    TTM_CALL(bank_forward(g, mask, 1, bank + (long)K * g.bank_slab(), stream));
  }
  return TTM_OK;
}

size_t ttm_correlate_workspace_bytes(ttm_dims N, ttm_dims L, int32_t K) {
  if (!dims_ok(N) || !dims_ok(L) || K < 1) return 0;
  Carve c(nullptr);
  corr_layout(c, make_geo(N, L), K);
  return c.size();
}

// out_C (optional): C_alpha over the valid box, [K][W0][W1][W2]; then only w
// is written here (out_score is not touched).  stats_in (optional): image
// statistics taken elsewhere (see image_forward).
// planar: the K = n + 1 components of a planar tensor (multiplicities C(n, k))
// two_pass: the two-pass inverse (k_pass1x, k_pass3x) where the shape allows
// it and only the score and w are wanted; its arrays are then not laid out
// for k_field_at
static ttm_status correlate_into(const Geo& g, int order_n, int K, const float* image, const float2* bk,
                                 const float* mask, float eps_v, float* out_score, float* out_w, CorrWs& w,
                                 hipStream_t stream, float* out_C = nullptr, const double* stats_in = nullptr,
                                 bool planar = false, bool check_finite = false, bool two_pass = true) {
  const long half = g.half();
  if (check_finite && !stats_in) {
    // the image moments first, checked before anything else is enqueued
    TTM_PROF(PC_STATS, launch_image_stats(image, g.vol(), mask, (long)g.L0 * g.L1 * g.L2, w.partials, w.stats,
                                          stream));
    TTM_CALL(moments_finite(w.stats, stream));
    stats_in = w.stats;
  }
  // the multiplicities: with the image statistics where those are taken here
  const bool mu_with_stats = !planar && !stats_in;
  if (planar)
    TTM_PROF(PC_STATS, launch_planar_mu(order_n, w.mu, stream));
  else if (!mu_with_stats)
    TTM_PROF(PC_STATS, launch_multiplicities(order_n, w.mu, stream));
  TTM_CALL(image_forward(g, image, w.Xf, w.Xg, w.stats, w.partials, mask, stream, stats_in, order_n,
                         mu_with_stats ? w.mu : nullptr));
  // K components and the mask against f, then the mask against f^2
  const Pass1Args p1{w.Xf, bk, K + 1, w.Xg, bk + (long)K * g.bank_slab(), 1, g.bank_slab(), w.H, half};
  if (two_pass && !out_C && !planar && two_pass_supported(g)) {
    Pass3Args a;
    std::memset(&a, 0, sizeof(a));
    a.H = w.H;
    a.pstride = half;
    a.npairs = K;
    a.mode = P3_SCORE;
    a.mu = w.mu;
    a.stats = stats_in ? stats_in : w.stats;
    a.eps_v = eps_v;
    a.out_score = out_score;
    a.out_w = out_w ? out_w : w.wtmp;
    TTM_PROF(PC_PASS1, launch_pass1x(g, p1, stream));
    TTM_PROF(PC_PASS3, launch_pass3x(g, a, stream));
    return TTM_OK;
  }
  TTM_PROF(PC_PASS1, launch_pass1(g, p1, stream));
  TTM_PROF(PC_PEN_INV, pencils_inverse_valid(g, w.H, K + 2, half, stream));
  Pass3Args a;
  std::memset(&a, 0, sizeof(a));
  a.H = w.H;
  a.pstride = half;
  a.npairs = K;
  a.mode = out_C ? P3_FIELD : P3_SCORE;
  a.out_C = out_C;
  a.c_plane = (long)(g.hi0() - g.lo0() + 1) * (g.hi1() - g.lo1() + 1) * (g.n2 - g.L2 + 1);
  a.mu = w.mu;
  a.stats = stats_in ? stats_in : w.stats;
  a.eps_v = eps_v;
  a.out_score = out_score;
  a.out_w = out_w;
  TTM_PROF(PC_PASS3, launch_pass3(g, a, stream));
  return TTM_OK;
}

ttm_status ttm_correlate(const float* image, ttm_dims N, const void* bank, ttm_dims L, int32_t order_n,
                         const float* mask, const ttm_options* opt, float* out_score, float* out_w, void* ws,
                         size_t ws_bytes, hipStream_t stream) {
  if (!image || !bank || !mask || !opt || !out_score) return TTM_E_ARG;
  const int K = ttm_num_components(order_n);
  if (K < 0) return TTM_E_ARG;
  if (!(opt->eps_v >= 0.0f)) return TTM_E_ARG;
  if (!dims_ok(L) || !image_dims_ok(N) || !fits(L, N)) return TTM_E_SIZE;
  if (!ws || ws_bytes < ttm_correlate_workspace_bytes(N, L, K)) return TTM_E_WORKSPACE;
  const Geo g = make_geo(N, L);
  Carve c(ws);
  CorrWs w = corr_layout(c, g, K);
  return correlate_into(g, order_n, K, image, static_cast<const float2*>(bank), mask, opt->eps_v, out_score,
                        out_w, w, stream, nullptr, nullptr, false, opt->check_finite != 0);
}

static bool pose_opts_ok(const ttm_options* opt) {
  if (opt->max_peaks < 1 || opt->max_peaks > 4096) return false;
  if (opt->n_seeds < 64 || opt->n_seeds > 65536) return false;
  if (opt->hopm_max_iter < 1 || !(opt->hopm_tol > 0.0)) return false;
  if (!(opt->threshold >= 0.0f) || !(opt->min_dist >= 0.0f) || !(opt->eps_v >= 0.0f)) return false;
  if (opt->refine < 0 || opt->refine > 3) return false;
  return true;
}

size_t ttm_pose_workspace_bytes(ttm_dims N, ttm_dims L, int32_t order_n, const ttm_options* opt) {
  (void)N; (void)L;
  const int K = ttm_num_components(order_n);
  if (K < 0 || !opt || !pose_opts_ok(opt)) return 0;
  Carve c(nullptr);
  pose_layout(c, make_geo(N, L), opt->max_peaks, K, opt->refine, opt->n_seeds);
  return c.size();
}

static ttm_status recover_pose_into(const Geo& g, const float* score, const float* image, const float* components,
                                    const float* mask, const float* tmpl, int order_n, int K, const ttm_options* opt,
                                    int32_t* out_pos, float* out_quat, double* out_lambda, float* out_peak_score,
                                    int32_t* out_flags, double* out_C, int32_t* out_count, PoseWs& w,
                                    hipStream_t stream) {
  TTM_PROF(PC_STATS, launch_image_stats(image, g.vol(), nullptr, 0, w.partials, w.stats, stream));
  PeakWs pw{w.hist, w.ctrl, w.allc, w.cand};
  float* cand_score = reinterpret_cast<float*>(w.ps.w);   // overwritten later by the pose scratch
  TTM_PROF(PC_PEAKS, launch_peaks(g, score, opt->threshold, opt->min_dist, opt->max_peaks, pw, w.cand_pos,
                                  cand_score, out_count, stream));
  const int rf = opt->refine == 3 ? 2 : opt->refine;   // each round of refine 3 is a refine-2 round
  TTM_PROF(PC_POSE, launch_pose_tensor(g, image, components, mask, order_n, w.stats, opt->eps_v,
                                       opt->max_peaks, rf, w.cand_pos, out_count, 0, w.ps, stream));
  TTM_PROF(PC_POSE, launch_pose_solve(g, score, order_n, opt->n_seeds, opt->hopm_max_iter, opt->hopm_tol,
                                      opt->max_peaks, rf, w.cand_pos, out_count, 0, image, tmpl, mask,
                                      out_pos, out_quat, out_lambda, out_peak_score, out_flags, out_C, w.ps,
                                      stream, false, 9, w.moved[0]));
  if (opt->refine == 3) {
    auto tensor = [&](const int* pos, const int* cnt, int cnt_host, const PoseScratch& ps) {
      return launch_pose_tensor(g, image, components, mask, order_n, w.stats, opt->eps_v, opt->max_peaks, 2, pos,
                                cnt, cnt_host, ps, stream);
    };
    TTM_CALL(refine_rounds(g, score, order_n, opt, opt->max_peaks, out_count, 0, image, tmpl, mask, out_pos,
                           out_quat, out_lambda, out_peak_score, out_flags, out_C, w, tensor, stream));
  }
  return TTM_OK;
}

// extents of images that are not transformed as a whole (pose, tiled
// correlation): any size >= 1 with a volume below 2^31 (peak keys hold a
// 32-bit linear index)
static bool any_dims_ok(const ttm_dims& N) {
  return dims_ok(N) && N.n0 <= 8192 && N.n1 <= 8192 && N.n2 <= 8192 && (long)N.n0 * N.n1 * N.n2 < (1L << 31);
}

ttm_status ttm_recover_pose(const float* score, const float* image, const float* components, const float* mask,
                            const float* tmpl, ttm_dims N, ttm_dims L, int32_t order_n, const ttm_options* opt,
                            int32_t* out_pos, float* out_quat, double* out_lambda, float* out_peak_score,
                            int32_t* out_flags, double* out_C, int32_t* out_count, void* ws, size_t ws_bytes,
                            hipStream_t stream) {
  if (!score || !image || !components || !mask || !opt || !out_pos || !out_quat || !out_lambda ||
      !out_peak_score || !out_flags || !out_count)
    return TTM_E_ARG;
  if (opt->refine >= 2 && !tmpl) return TTM_E_ARG;
  const int K = ttm_num_components(order_n);
  if (K < 0 || !pose_opts_ok(opt)) return TTM_E_ARG;
  if (!dims_ok(L) || !any_dims_ok(N) || !fits(L, N)) return TTM_E_SIZE;
  if (!ws || ws_bytes < ttm_pose_workspace_bytes(N, L, order_n, opt)) return TTM_E_WORKSPACE;
  const Geo g = make_geo(N, L);
  Carve c(ws);
  PoseWs w = pose_layout(c, g, opt->max_peaks, K, opt->refine, opt->n_seeds);
  return recover_pose_into(g, score, image, components, mask, tmpl, order_n, K, opt, out_pos, out_quat, out_lambda,
                           out_peak_score, out_flags, out_C, out_count, w, stream);
}

// host-side checks of a pose_at call (every argument but the workspace)
static ttm_status pose_at_check(const float* image, const float* components, const float* mask, const float* tmpl,
                                const ttm_dims& N, const ttm_dims& L, int32_t order_n, const ttm_options* opt,
                                const int32_t* positions, int32_t n_pos, int32_t* out_pos, float* out_quat,
                                double* out_lambda, int32_t* out_flags) {
  if (!image || !components || !mask || !opt || !positions || !out_pos || !out_quat || !out_lambda ||
      !out_flags)
    return TTM_E_ARG;
  if (opt->refine >= 2 && !tmpl) return TTM_E_ARG;
  const int K = ttm_num_components(order_n);
  if (K < 0 || !pose_opts_ok(opt)) return TTM_E_ARG;
  if (n_pos < 0 || n_pos > opt->max_peaks) return TTM_E_ARG;
  if (!dims_ok(L) || !any_dims_ok(N) || !fits(L, N)) return TTM_E_SIZE;
  return TTM_OK;
}

// the launch sequence of a pose_at call on a carved workspace
static ttm_status pose_at_into(const Geo& g, const float* image, const float* components, const float* mask,
                               const float* tmpl, int32_t order_n, int K, const ttm_options* opt,
                               const int32_t* positions, int32_t n_pos, int32_t* out_pos, float* out_quat,
                               double* out_lambda, int32_t* out_flags, double* out_C, PoseWs& w,
                               hipStream_t stream) {
  TTM_PROF(PC_STATS, launch_image_stats(image, g.vol(), nullptr, 0, w.partials, w.stats, stream));
  const int rf = opt->refine == 3 ? 2 : opt->refine;
  TTM_PROF(PC_POSE, launch_pose_tensor(g, image, components, mask, order_n, w.stats, opt->eps_v, n_pos,
                                       rf, positions, nullptr, n_pos, w.ps, stream));
  TTM_PROF(PC_POSE, launch_pose_solve(g, nullptr, order_n, opt->n_seeds, opt->hopm_max_iter, opt->hopm_tol, n_pos,
                                      rf, positions, nullptr, n_pos, image, tmpl, mask, out_pos, out_quat,
                                      out_lambda, nullptr, out_flags, out_C, w.ps, stream, false, 9, w.moved[0]));
  if (opt->refine == 3) {
    auto tensor = [&](const int* pos, const int* cnt, int cnt_host, const PoseScratch& ps) {
      return launch_pose_tensor(g, image, components, mask, order_n, w.stats, opt->eps_v, n_pos, 2, pos, cnt,
                                cnt_host, ps, stream);
    };
    TTM_CALL(refine_rounds(g, nullptr, order_n, opt, n_pos, nullptr, n_pos, image, tmpl, mask, out_pos, out_quat,
                           out_lambda, nullptr, out_flags, out_C, w, tensor, stream));
  }
  return TTM_OK;
}

ttm_status ttm_pose_at(const float* image, const float* components, const float* mask, const float* tmpl,
                       ttm_dims N, ttm_dims L, int32_t order_n, const ttm_options* opt, const int32_t* positions,
                       int32_t n_pos, int32_t* out_pos, float* out_quat, double* out_lambda, int32_t* out_flags,
                       double* out_C, void* ws, size_t ws_bytes, hipStream_t stream) {
  TTM_CALL(pose_at_check(image, components, mask, tmpl, N, L, order_n, opt, positions, n_pos, out_pos, out_quat,
                         out_lambda, out_flags));
  if (!ws || ws_bytes < ttm_pose_workspace_bytes(N, L, order_n, opt)) return TTM_E_WORKSPACE;
  if (n_pos == 0) return TTM_OK;
  const int K = ttm_num_components(order_n);
  const Geo g = make_geo(N, L);
  Carve c(ws);
  PoseWs w = pose_layout(c, g, opt->max_peaks, K, opt->refine, opt->n_seeds);
  return pose_at_into(g, image, components, mask, tmpl, order_n, K, opt, positions, n_pos, out_pos, out_quat,
                      out_lambda, out_flags, out_C, w, stream);
}

ttm_status ttm_pose_at_noalloc(const float* image, const float* components, const float* mask, const float* tmpl,
                               ttm_dims N, ttm_dims L, int32_t order_n, const ttm_options* opt,
                               const int32_t* positions, int32_t n_pos, int32_t* out_pos, float* out_quat,
                               double* out_lambda, int32_t* out_flags, double* out_C, hipStream_t stream) {
  TTM_CALL(pose_at_check(image, components, mask, tmpl, N, L, order_n, opt, positions, n_pos, out_pos, out_quat,
                         out_lambda, out_flags));
  const int K = ttm_num_components(order_n);
  const Geo g = make_geo(N, L);
  Carve need(nullptr);
  pose_layout(need, g, opt->max_peaks, K, opt->refine, opt->n_seeds, false);
  if (need.size() > kStaticScratchBytes) return TTM_E_WORKSPACE;
  void* base = nullptr;
  TTM_CALL(static_scratch(stream, &base));
  if (n_pos == 0) return TTM_OK;
  const ProfSuppress quiet;
  Carve c(base);
  PoseWs w = pose_layout(c, g, opt->max_peaks, K, opt->refine, opt->n_seeds, false);
  return pose_at_into(g, image, components, mask, tmpl, order_n, K, opt, positions, n_pos, out_pos, out_quat,
                      out_lambda, out_flags, out_C, w, stream);
}

size_t ttm_match_workspace_bytes(ttm_dims N, ttm_dims L, int32_t order_n, const ttm_options* opt) {
  const int K = ttm_num_components(order_n);
  if (K < 0 || !opt || !pose_opts_ok(opt) || !dims_ok(N) || !dims_ok(L)) return 0;
  const Geo g = make_geo(N, L);
  Carve c(nullptr);
  corr_layout(c, g, K);
  pose_layout(c, make_geo(N, L), opt->max_peaks, K, opt->refine, opt->n_seeds);
  c.take<float>(g.vol());
  return c.size();
}

ttm_status ttm_match(const float* image, ttm_dims N, const void* bank, ttm_dims L, int32_t order_n,
                     const float* mask, const float* tmpl, const ttm_options* opt, float* out_score, float* out_w,
                     int32_t* out_pos, float* out_quat, double* out_lambda, float* out_peak_score,
                     int32_t* out_flags, double* out_C, int32_t* out_count, void* ws, size_t ws_bytes,
                     hipStream_t stream) {
  if (!image || !bank || !mask || !opt || !out_score || !out_pos || !out_quat || !out_lambda ||
      !out_peak_score || !out_flags || !out_count)
    return TTM_E_ARG;
  if (opt->refine >= 2 && !tmpl) return TTM_E_ARG;
  const int K = ttm_num_components(order_n);
  if (K < 0 || !pose_opts_ok(opt)) return TTM_E_ARG;
  if (!dims_ok(L) || !image_dims_ok(N) || !fits(L, N)) return TTM_E_SIZE;
  if (!ws || ws_bytes < ttm_match_workspace_bytes(N, L, order_n, opt)) return TTM_E_WORKSPACE;
  const Geo g = make_geo(N, L);
  Carve c(ws);
  CorrWs cw = corr_layout(c, g, K);
  PoseWs pw = pose_layout(c, g, opt->max_peaks, K, opt->refine, opt->n_seeds);
  float* wmap = c.take<float>(g.vol());
  float* wout = out_w ? out_w : wmap;
  TTM_CALL(correlate_into(g, order_n, K, image, static_cast<const float2*>(bank), mask, opt->eps_v, out_score,
                          wout, cw, stream, nullptr, nullptr, false, opt->check_finite != 0, false));
  PeakWs pk{pw.hist, pw.ctrl, pw.allc, pw.cand};
  float* cand_score = reinterpret_cast<float*>(pw.ps.w);
  TTM_PROF(PC_PEAKS, launch_peaks(g, out_score, opt->threshold, opt->min_dist, opt->max_peaks, pk, pw.cand_pos,
                                  cand_score, out_count, stream));
  const int rf = opt->refine == 3 ? 2 : opt->refine;
  TTM_PROF(PC_POSE, launch_field_at(g, cw.H, g.half(), K, wout, opt->max_peaks, rf, pw.cand_pos,
                                    out_count, 0, pw.ps, stream));
  TTM_PROF(PC_POSE, launch_pose_solve(g, out_score, order_n, opt->n_seeds, opt->hopm_max_iter, opt->hopm_tol,
                                      opt->max_peaks, rf, pw.cand_pos, out_count, 0, image, tmpl, mask,
                                      out_pos, out_quat, out_lambda, out_peak_score, out_flags, out_C, pw.ps,
                                      stream, false, 9, pw.moved[0]));
  if (opt->refine == 3) {
    auto tensor = [&](const int* pos, const int* cnt, int cnt_host, const PoseScratch& ps) {
      return launch_field_at(g, cw.H, g.half(), K, wout, opt->max_peaks, 2, pos, cnt, cnt_host, ps, stream);
    };
    TTM_CALL(refine_rounds(g, out_score, order_n, opt, opt->max_peaks, out_count, 0, image, tmpl, mask, out_pos,
                           out_quat, out_lambda, out_peak_score, out_flags, out_C, pw, tensor, stream));
  }
  return TTM_OK;
}

// --- overlap-save tiled correlation, batches, graphs ---------------------------------
static bool tile_ok(int T, const ttm_dims& L) {
  return supported_len(T) && T >= L.n0 && T >= L.n1 && T >= L.n2;
}
static long tiles_along(int n, int l, int T) {
  const long W = (long)n - l + 1, WT = (long)T - l + 1;
  return (W + WT - 1) / WT;
}

struct TiledWs {
  float* tile; float* tscore; float* tw; double* stats; double* partials; CorrWs corr;
};
static TiledWs tiled_layout(Carve& c, int T, const ttm_dims& L, int K) {
  TiledWs w;
  const Geo gT = make_geo(ttm_dims{T, T, T}, L);
  const size_t T3 = (size_t)T * T * T;
  w.tile = c.take<float>(T3);
  w.tscore = c.take<float>(T3);
  w.tw = c.take<float>(T3);
  w.stats = c.take<double>(4);
  w.partials = c.take<double>(3 * kStatPartials);
  w.corr = corr_layout(c, gT, K);
  return w;
}

// the whole image's statistics once, then per tile: gather, correlate (with
// those statistics), scatter of the tile's valid part
static ttm_status correlate_tiled_into(const float* image, const ttm_dims& N, const float2* bank, const ttm_dims& L,
                                       int order_n, int K, int T, const float* mask, float eps_v, float* out_score,
                                       float* out_w, TiledWs& w, hipStream_t stream, bool check_finite = false) {
  const Geo gT = make_geo(ttm_dims{T, T, T}, L);
  const long vol = (long)N.n0 * N.n1 * N.n2;
  TTM_PROF(PC_STATS, launch_image_stats(image, vol, mask, (long)L.n0 * L.n1 * L.n2, w.partials, w.stats, stream));
  if (check_finite) TTM_CALL(moments_finite(w.stats, stream));
  TTM_PROF(PC_EPI, launch_fill_f32(out_score, vol, 0.0f, stream));
  if (out_w) TTM_PROF(PC_EPI, launch_fill_f32(out_w, vol, 0.0f, stream));
  TileGeo tg;
  tg.n0 = N.n0; tg.n1 = N.n1; tg.n2 = N.n2;
  tg.T = T;
  tg.L0 = L.n0; tg.L1 = L.n1; tg.L2 = L.n2;
  tg.c0 = L.n0 / 2; tg.c1 = L.n1 / 2; tg.c2 = L.n2 / 2;
  const long k0n = tiles_along(N.n0, L.n0, T), k1n = tiles_along(N.n1, L.n1, T), k2n = tiles_along(N.n2, L.n2, T);
  for (long k0 = 0; k0 < k0n; ++k0)
    for (long k1 = 0; k1 < k1n; ++k1)
      for (long k2 = 0; k2 < k2n; ++k2) {
        tg.o0 = (int)(k0 * (T - L.n0 + 1));
        tg.o1 = (int)(k1 * (T - L.n1 + 1));
        tg.o2 = (int)(k2 * (T - L.n2 + 1));
        TTM_PROF(PC_EPI, launch_tile_gather(image, tg, w.tile, stream));
        TTM_CALL(correlate_into(gT, order_n, K, w.tile, bank, mask, eps_v, w.tscore, w.tw, w.corr, stream, nullptr,
                                w.stats));
        TTM_PROF(PC_EPI, launch_tile_scatter(w.tscore, w.tw, tg, out_score, out_w, stream));
      }
  return TTM_OK;
}

int32_t ttm_tile_count(ttm_dims N, ttm_dims L, int32_t T) {
  if (!any_dims_ok(N) || !dims_ok(L) || !fits(L, N) || !tile_ok(T, L)) return TTM_E_SIZE;
  const long n = tiles_along(N.n0, L.n0, T) * tiles_along(N.n1, L.n1, T) * tiles_along(N.n2, L.n2, T);
  return n > 0x7fffffffL ? TTM_E_SIZE : (int32_t)n;
}

int32_t ttm_choose_tile(ttm_dims N, ttm_dims L, const int32_t* tiles_host, const float* ms_host, int32_t n) {
  if (!tiles_host || !ms_host || n < 1) return TTM_E_ARG;
  int best = TTM_E_SIZE;
  double best_cost = 0.0;
  for (int i = 0; i < n; ++i) {
    const int cnt = ttm_tile_count(N, L, tiles_host[i]);
    if (cnt <= 0 || !(ms_host[i] > 0.0f)) continue;
    const double cost = (double)cnt * ms_host[i];
    // the cheaper plan; the larger tile on equal cost
    if (best < 0 || cost < best_cost || (cost == best_cost && tiles_host[i] > best)) {
      best = tiles_host[i];
      best_cost = cost;
    }
  }
  return best;
}

size_t ttm_correlate_tiled_workspace_bytes(ttm_dims L, int32_t order_n, int32_t T) {
  const int K = ttm_num_components(order_n);
  if (K < 0 || !dims_ok(L) || !tile_ok(T, L)) return 0;
  Carve c(nullptr);
  tiled_layout(c, T, L, K);
  return c.size();
}

ttm_status ttm_correlate_tiled(const float* image, ttm_dims N, const void* bank, ttm_dims L, int32_t order_n,
                               int32_t T, const float* mask, const ttm_options* opt, float* out_score, float* out_w,
                               void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!image || !bank || !mask || !opt || !out_score) return TTM_E_ARG;
  const int K = ttm_num_components(order_n);
  if (K < 0 || !(opt->eps_v >= 0.0f)) return TTM_E_ARG;
  if (!dims_ok(L) || !any_dims_ok(N) || !fits(L, N) || !tile_ok(T, L)) return TTM_E_SIZE;
  if (!ws || ws_bytes < ttm_correlate_tiled_workspace_bytes(L, order_n, T)) return TTM_E_WORKSPACE;
  Carve c(ws);
  TiledWs w = tiled_layout(c, T, L, K);
  return correlate_tiled_into(image, N, static_cast<const float2*>(bank), L, order_n, K, T, mask, opt->eps_v,
                              out_score, out_w, w, stream, opt->check_finite != 0);
}

size_t ttm_autotune_workspace_bytes(ttm_dims L, int32_t order_n, const int32_t* tiles_host, int32_t n) {
  const int K = ttm_num_components(order_n);
  if (K < 0 || !dims_ok(L) || !tiles_host || n < 1) return 0;
  size_t need = 0;
  for (int i = 0; i < n; ++i) {
    if (!tile_ok(tiles_host[i], L)) return 0;
    Carve c(nullptr);
    tiled_layout(c, tiles_host[i], L, K);
    const size_t T3 = (size_t)tiles_host[i] * tiles_host[i] * tiles_host[i];
    c.take<float>(T3);
    c.take<float>(T3);
    need = std::max(need, c.size());
  }
  return need;
}

ttm_status ttm_autotune_tiles(const void* const* banks_host, const int32_t* tiles_host, int32_t n, ttm_dims L,
                              int32_t order_n, const float* mask, const ttm_options* opt, int32_t repeats,
                              float* ms_host, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!banks_host || !tiles_host || !mask || !opt || !ms_host || n < 1 || repeats < 1) return TTM_E_ARG;
  const int K = ttm_num_components(order_n);
  if (K < 0) return TTM_E_ARG;
  if (!dims_ok(L)) return TTM_E_SIZE;
  for (int i = 0; i < n; ++i) {
    if (!banks_host[i]) return TTM_E_ARG;
    if (!tile_ok(tiles_host[i], L)) return TTM_E_SIZE;
  }
  if (!ws || ws_bytes < ttm_autotune_workspace_bytes(L, order_n, tiles_host, n)) return TTM_E_WORKSPACE;
  hipEvent_t e0, e1;
  TTM_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return TTM_E_HIP;
  }
  ttm_status st = TTM_OK;
  for (int i = 0; i < n && st == TTM_OK; ++i) {
    const int T = tiles_host[i];
    Carve c(ws);
    TiledWs w = tiled_layout(c, T, L, K);
    const long T3 = (long)T * T * T;
    float* img = c.take<float>((size_t)T3);
    float* out = c.take<float>((size_t)T3);
    const ttm_dims NT{T, T, T};
    // an image of one tile (zeros: the passes do the same work for any
    // values), timed `repeats` times after one untimed run; the median is kept
    std::vector<float> ms;
    if (launch_fill_f32(img, T3, 0.0f, stream) != hipSuccess) st = TTM_E_HIP;
    for (int r = 0; r <= repeats && st == TTM_OK; ++r) {
      if (hipEventRecord(e0, stream) != hipSuccess) {
        st = TTM_E_HIP;
        break;
      }
      st = correlate_tiled_into(img, NT, static_cast<const float2*>(banks_host[i]), L, order_n, K, T, mask,
                                opt->eps_v, out, nullptr, w, stream);
      if (st != TTM_OK) break;
      float t = 0.0f;
      if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
        st = TTM_E_HIP;
        break;
      }
      if (r > 0) ms.push_back(t);
    }
    if (st == TTM_OK) {
      std::sort(ms.begin(), ms.end());
      ms_host[i] = ms[ms.size() / 2];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}

static bool job_ok(const ttm_batch_job& j, int order_n, const ttm_options* opt) {
  if (!j.image || !j.bank || !j.components || !j.mask || !j.out_score || !j.out_pos || !j.out_quat ||
      !j.out_lambda || !j.out_peak_score || !j.out_flags || !j.out_count)
    return false;
  if (opt->refine >= 2 && !j.tmpl) return false;
  (void)order_n;
  return true;
}
static ttm_status job_sizes(const ttm_batch_job& j) {
  if (!dims_ok(j.L) || !any_dims_ok(j.N) || !fits(j.L, j.N) || !tile_ok(j.tile, j.L)) return TTM_E_SIZE;
  return TTM_OK;
}

// workspace of one stream of a batch: the largest job's tiled and pose layouts
static size_t batch_stream_bytes(const ttm_batch_job* jobs_host, int32_t n_jobs, int32_t order_n,
                                 const ttm_options* opt) {
  const int K = ttm_num_components(order_n);
  if (!jobs_host || n_jobs < 1 || K < 0 || !opt || !pose_opts_ok(opt)) return 0;
  size_t need = 0;
  for (int i = 0; i < n_jobs; ++i) {
    const ttm_batch_job& j = jobs_host[i];
    if (job_sizes(j) != TTM_OK) return 0;
    Carve c(nullptr);
    tiled_layout(c, j.tile, j.L, K);
    pose_layout(c, make_geo(j.N, j.L), opt->max_peaks, K, opt->refine, opt->n_seeds);
    need = std::max(need, c.size());
  }
  return need;
}

size_t ttm_batch_workspace_bytes(const ttm_batch_job* jobs_host, int32_t n_jobs, int32_t order_n,
                                 const ttm_options* opt, int32_t n_streams) {
  if (n_streams < 1 || n_streams > kBatchMaxStreams) return 0;
  const size_t per = batch_stream_bytes(jobs_host, n_jobs, order_n, opt);
  // the slices, plus one 256-byte block for the graph's root and sink nodes
  return per == 0 ? 0 : per * (size_t)n_streams + 256;
}

static ttm_status batch_check(const ttm_batch_job* jobs_host, int32_t n_jobs, int32_t order_n,
                              const ttm_options* opt, int32_t n_streams, void* ws, size_t ws_bytes) {
  if (n_streams < 1 || n_streams > kBatchMaxStreams) return TTM_E_ARG;
  if (!jobs_host || n_jobs < 1 || !opt) return TTM_E_ARG;
  const int K = ttm_num_components(order_n);
  if (K < 0 || !pose_opts_ok(opt)) return TTM_E_ARG;
  if (opt->check_finite) return TTM_E_ARG;   // the check waits on the stream: not in a batch or graph
  for (int i = 0; i < n_jobs; ++i) {
    if (!job_ok(jobs_host[i], order_n, opt)) return TTM_E_ARG;
    const ttm_status st = job_sizes(jobs_host[i]);
    if (st != TTM_OK) return st;
  }
  if (!ws || ws_bytes < ttm_batch_workspace_bytes(jobs_host, n_jobs, order_n, opt, n_streams))
    return TTM_E_WORKSPACE;
  return TTM_OK;
}

// the listed jobs one after another on `stream`, sharing the workspace
static ttm_status batch_run(const ttm_batch_job* jobs_host, const int* idx, int n_idx, int32_t order_n,
                            const ttm_options* opt, void* ws, hipStream_t stream) {
  const int K = ttm_num_components(order_n);
  for (int ii = 0; ii < n_idx; ++ii) {
    const ttm_batch_job& j = jobs_host[idx[ii]];
    Carve c(ws);
    TiledWs tw = tiled_layout(c, j.tile, j.L, K);
    PoseWs pw = pose_layout(c, make_geo(j.N, j.L), opt->max_peaks, K, opt->refine, opt->n_seeds);
    TTM_CALL(correlate_tiled_into(j.image, j.N, static_cast<const float2*>(j.bank), j.L, order_n, K, j.tile, j.mask,
                                  opt->eps_v, j.out_score, j.out_w, tw, stream));
    TTM_CALL(recover_pose_into(make_geo(j.N, j.L), j.out_score, j.image, j.components, j.mask, j.tmpl, order_n, K,
                               opt, j.out_pos, j.out_quat, j.out_lambda, j.out_peak_score, j.out_flags, nullptr,
                               j.out_count, pw, stream));
  }
  return TTM_OK;
}

// jobs split over n streams: longest first onto the least loaded stream,
// with a job's cost estimated as its tiles times the tile volume
static std::vector<std::vector<int>> batch_split(const ttm_batch_job* jobs_host, int n_jobs, int n) {
  std::vector<std::pair<double, int>> cost(n_jobs);
  for (int i = 0; i < n_jobs; ++i) {
    const ttm_batch_job& j = jobs_host[i];
    const double T = j.tile;
    cost[i] = {(double)ttm_tile_count(j.N, j.L, j.tile) * T * T * T, i};
  }
  std::stable_sort(cost.begin(), cost.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
  std::vector<std::vector<int>> parts(n);
  std::vector<double> load(n, 0.0);
  for (const auto& c : cost) {
    const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    parts[b].push_back(c.second);
    load[b] += c.first;
  }
  for (auto& p : parts) std::sort(p.begin(), p.end());   // each stream keeps the caller's order
  return parts;
}

struct ttm_graph_s {
  hipGraphExec_t exec;
};

// the jobs split over n_streams branches on `stream` and side streams forked
// from it and joined back to it (recorded into a graph when `capture`)
static ttm_status batch_dispatch(const ttm_batch_job* jobs_host, int32_t n_jobs, int32_t order_n,
                                 const ttm_options* opt, int32_t n_streams, void* ws, hipStream_t stream,
                                 bool capture, hipGraph_t* graph_out) {
  const size_t per = batch_stream_bytes(jobs_host, n_jobs, order_n, opt);
  const std::vector<std::vector<int>> parts = batch_split(jobs_host, n_jobs, n_streams);
  // side streams (default priority) and the fork / join events, created and
  // destroyed by this call: a captured graph does not refer to them
  std::vector<hipStream_t> side(n_streams, nullptr);
  std::vector<hipEvent_t> ev(n_streams, nullptr);
  ttm_status st = TTM_OK;
  for (int b = 0; b < n_streams && st == TTM_OK; ++b) {
    if (hipEventCreateWithFlags(&ev[b], hipEventDisableTiming) != hipSuccess) st = TTM_E_HIP;
    if (b > 0 && st == TTM_OK && hipStreamCreateWithFlags(&side[b], hipStreamNonBlocking) != hipSuccess)
      st = TTM_E_HIP;
  }
  bool capturing = false;
  if (st == TTM_OK && capture) {
    if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess) st = TTM_E_HIP;
    else capturing = true;
  }
  int* marker = reinterpret_cast<int*>(static_cast<char*>(ws) + per * (size_t)n_streams);
  // fork: every side stream waits on the start, one kernel node that all
  // branches descend from
  if (st == TTM_OK && n_streams > 1) {
    if (launch_fill_i32(marker, 1, 0, stream) != hipSuccess || hipEventRecord(ev[0], stream) != hipSuccess)
      st = TTM_E_HIP;
    for (int b = 1; b < n_streams && st == TTM_OK; ++b)
      if (hipStreamWaitEvent(side[b], ev[0], 0) != hipSuccess) st = TTM_E_HIP;
  }
  for (int b = 0; b < n_streams && st == TTM_OK; ++b) {
    if (parts[b].empty()) continue;
    st = batch_run(jobs_host, parts[b].data(), (int)parts[b].size(), order_n, opt,
                   static_cast<char*>(ws) + per * (size_t)b, b == 0 ? stream : side[b]);
  }
  // join: `stream` waits on every side stream's end, then one kernel node
  for (int b = 1; b < n_streams && st == TTM_OK; ++b) {
    if (hipEventRecord(ev[b], side[b]) != hipSuccess || hipStreamWaitEvent(stream, ev[b], 0) != hipSuccess)
      st = TTM_E_HIP;
  }
  if (st == TTM_OK && n_streams > 1 && launch_fill_i32(marker, 1, 0, stream) != hipSuccess) st = TTM_E_HIP;
  if (capturing) {
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(stream, &graph);
    if (st == TTM_OK && (ec != hipSuccess || !graph)) st = TTM_E_HIP;
    if (st == TTM_OK) *graph_out = graph;
    else if (graph) (void)hipGraphDestroy(graph);
  }
  // an eager dispatch's side streams are destroyed only after their work is
  // ordered before `stream`'s later work (the join above); destroying a
  // stream with pending work is allowed and does not wait for it
  for (int b = 0; b < n_streams; ++b) {
    if (ev[b]) (void)hipEventDestroy(ev[b]);
    if (side[b]) (void)hipStreamDestroy(side[b]);
  }
  return st;
}

ttm_status ttm_batch_match(const ttm_batch_job* jobs_host, int32_t n_jobs, int32_t order_n, const ttm_options* opt,
                           int32_t n_streams, void* ws, size_t ws_bytes, hipStream_t stream) {
  TTM_CALL(batch_check(jobs_host, n_jobs, order_n, opt, n_streams, ws, ws_bytes));
  if (n_streams == 1) {
    std::vector<int> idx(n_jobs);
    for (int i = 0; i < n_jobs; ++i) idx[i] = i;
    return batch_run(jobs_host, idx.data(), n_jobs, order_n, opt, ws, stream);
  }
  return batch_dispatch(jobs_host, n_jobs, order_n, opt, n_streams, ws, stream, false, nullptr);
}

ttm_status ttm_batch_graph_create(const ttm_batch_job* jobs_host, int32_t n_jobs, int32_t order_n,
                                  const ttm_options* opt, int32_t n_streams, void* ws, size_t ws_bytes,
                                  hipStream_t stream, ttm_graph* out_graph) {
  if (!out_graph) return TTM_E_ARG;
  *out_graph = nullptr;
  TTM_CALL(batch_check(jobs_host, n_jobs, order_n, opt, n_streams, ws, ws_bytes));
  if (!stream) return TTM_E_ARG;   // the legacy default stream cannot be captured
  hipGraph_t graph = nullptr;
  TTM_CALL(batch_dispatch(jobs_host, n_jobs, order_n, opt, n_streams, ws, stream, true, &graph));
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) return TTM_E_HIP;
  *out_graph = new ttm_graph_s{exec};
  return TTM_OK;
}

ttm_status ttm_graph_launch(ttm_graph graph, hipStream_t stream) {
  if (!graph) return TTM_E_ARG;
  TTM_TRY(hipGraphLaunch(graph->exec, stream));
  return TTM_OK;
}

void ttm_graph_destroy(ttm_graph graph) {
  if (!graph) return;
  (void)hipGraphExecDestroy(graph->exec);
  delete graph;
}

// --- all-voxel rotation map --------------------------------------------------------
static long valid_voxels(const Geo& g) {
  return (long)(g.hi0() - g.lo0() + 1) * (g.hi1() - g.lo1() + 1) * (g.n2 - g.L2 + 1);
}
static bool rmap_seeds_ok(int n_seeds) { return n_seeds >= 32 && n_seeds <= kRmapMaxSeeds && n_seeds % 32 == 0; }

struct RmapWs {
  float* planes; uint4* table; int* group; float* wmap;
};
static RmapWs rmap_layout(Carve& c, const Geo& g, int order_n, int K, int n_seeds) {
  RmapWs w;
  const long V = valid_voxels(g);
  w.planes = c.take<float>((size_t)K * V);
  w.table = c.take<uint4>((size_t)rmap_table_uint4(order_n, n_seeds));
  w.group = c.take<int>((size_t)V);
  w.wmap = c.take<float>(g.vol());
  return w;
}

size_t ttm_rotation_map_workspace_bytes(ttm_dims N, ttm_dims L, int32_t order_n, int32_t n_seeds) {
  const int K = ttm_num_components(order_n);
  if (K < 0 || !dims_ok(N) || !dims_ok(L) || !fits(L, N) || !rmap_seeds_ok(n_seeds)) return 0;
  const Geo g = make_geo(N, L);
  Carve c(nullptr);
  corr_layout(c, g, K);
  rmap_layout(c, g, order_n, K, n_seeds);
  return c.size();
}

ttm_status ttm_rotation_map(const float* image, ttm_dims N, const void* bank, ttm_dims L, int32_t order_n,
                            const float* mask, const ttm_options* opt, const float* seeds, int32_t n_seeds,
                            float* out_score, float* out_w, float* out_quat, float* out_lambda,
                            int32_t* out_unconverged, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!image || !bank || !mask || !opt || !seeds || !out_score || !out_quat || !out_lambda) return TTM_E_ARG;
  const int K = ttm_num_components(order_n);
  if (K < 0 || !rmap_seeds_ok(n_seeds)) return TTM_E_ARG;
  if (!(opt->eps_v >= 0.0f) || opt->hopm_max_iter < 1 || !(opt->hopm_tol > 0.0)) return TTM_E_ARG;
  if (!dims_ok(L) || !image_dims_ok(N) || !fits(L, N)) return TTM_E_SIZE;
  if (!ws || ws_bytes < ttm_rotation_map_workspace_bytes(N, L, order_n, n_seeds)) return TTM_E_WORKSPACE;
  const Geo g = make_geo(N, L);
  Carve c(ws);
  CorrWs cw = corr_layout(c, g, K);
  RmapWs rw = rmap_layout(c, g, order_n, K, n_seeds);
  float* wout = out_w ? out_w : rw.wmap;
  TTM_CALL(correlate_into(g, order_n, K, image, static_cast<const float2*>(bank), mask, opt->eps_v, out_score,
                          wout, cw, stream, rw.planes, nullptr, false, opt->check_finite != 0));
  TTM_PROF(PC_RMAP_POLISH, launch_rmap_table(order_n, seeds, n_seeds, rw.table, stream));
  TTM_PROF(PC_RMAP_SCAN, launch_rmap_scan(g, order_n, rw.planes, rw.table, n_seeds, rw.group, stream));
  TTM_PROF(PC_RMAP_POLISH, launch_fill_f32(out_score, g.vol(), 0.0f, stream));
  TTM_PROF(PC_RMAP_POLISH, launch_fill_f32(out_quat, 4 * g.vol(), 0.0f, stream));
  TTM_PROF(PC_RMAP_POLISH, launch_fill_f32(out_lambda, g.vol(), 0.0f, stream));
  if (out_unconverged) TTM_PROF(PC_RMAP_POLISH, launch_fill_i32(out_unconverged, 1, 0, stream));
  TTM_PROF(PC_RMAP_POLISH, launch_rmap_polish(g, order_n, rw.planes, seeds, rw.group, opt->hopm_max_iter,
                                              opt->hopm_tol, out_score, out_quat, out_lambda, out_unconverged,
                                              stream));
  return TTM_OK;
}

// --- two-dimensional TTM -----------------------------------------------------------
// volume index of each planar multi-index (n - k, k, 0, 0), in the packed order
// (alpha_1 from n down, then alpha_2, then alpha_3)
static PlanarIdx planar_idx(int n) {
  PlanarIdx p{};
  int idx = 0;
  for (int a1 = n; a1 >= 0; --a1)
    for (int a2 = n - a1; a2 >= 0; --a2)
      for (int a3 = n - a1 - a2; a3 >= 0; --a3) {
        if (a3 == 0 && a1 + a2 == n) p.k3[a2] = idx;
        ++idx;
      }
  return p;
}

static bool planar_box_ok(int L1, int L2) {
  return L1 >= 1 && L2 >= 1 && L1 <= 1023 && L2 <= 512;
}

static bool planar_quadrature_ok(const float* z, const double* w, int n_rot) {
  double wsum = 0.0;
  for (int j = 0; j < n_rot; ++j) {
    const double nz = (double)z[2 * j] * z[2 * j] + (double)z[2 * j + 1] * z[2 * j + 1];
    if (!std::isfinite(nz) || nz <= 0.0 || !std::isfinite(w[j])) return false;
    wsum += w[j];
  }
  return std::fabs(wsum - 1.0) <= 1e-6;
}

size_t ttm_bank_bytes_2d(int32_t B, int32_t n1, int32_t n2, int32_t L1, int32_t L2, int32_t order_n) {
  if (ttm_num_components(order_n) < 0 || order_n > kPlanarMaxOrder) return 0;
  return ttm_bank_bytes(ttm_dims{B, n1, n2}, ttm_dims{1, L1, L2}, order_n + 1);
}

size_t ttm_build_workspace_bytes_2d(int32_t L1, int32_t L2, int32_t order_n, int32_t n_rot) {
  const int K3 = ttm_num_components(order_n);
  if (K3 < 0 || order_n > kPlanarMaxOrder || n_rot < 1 || !planar_box_ok(L1, L2)) return 0;
  Carve c(nullptr);
  build_layout(c, n_rot, K3);
  c.take<float>(2 * (size_t)n_rot);
  c.take<float>((size_t)K3 * L1 * L2);
  return c.size();
}

ttm_status ttm_build_tensor_template_2d(const float* tmpl, const float* mask, int32_t L1, int32_t L2,
                                        int32_t order_n, const float* z_host, const double* weights_host,
                                        int32_t n_rot, float* out_components, int32_t B, int32_t n1, int32_t n2,
                                        void* out_bank, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!tmpl || !mask || !z_host || !weights_host || !out_components) return TTM_E_ARG;
  const int K3 = ttm_num_components(order_n);
  if (K3 < 0 || order_n > kPlanarMaxOrder || n_rot < 1) return TTM_E_ARG;
  if (!planar_quadrature_ok(z_host, weights_host, n_rot)) return TTM_E_ARG;
  if (!planar_box_ok(L1, L2)) return TTM_E_SIZE;
  const ttm_dims N{B, n1, n2}, L{1, L1, L2};
  if (out_bank && (!image_dims_ok(N) || !fits(L, N))) return TTM_E_SIZE;
  if (!ws || ws_bytes < ttm_build_workspace_bytes_2d(L1, L2, order_n, n_rot)) return TTM_E_WORKSPACE;
  Carve c(ws);
  BuildWs w = build_layout(c, n_rot, K3);
  float* zd = c.take<float>(2 * (size_t)n_rot);
  float* comps3 = c.take<float>((size_t)K3 * L1 * L2);
  TTM_TRY(hipMemcpyAsync(zd, z_host, sizeof(float) * 2 * (size_t)n_rot, hipMemcpyHostToDevice, stream));
  TTM_TRY(hipMemcpyAsync(w.weights, weights_host, sizeof(double) * (size_t)n_rot, hipMemcpyHostToDevice, stream));
  // the host arrays are read before this call returns, so the caller may
  // free or reuse them at once: an asynchronous copy from pageable memory may
  // otherwise be staged after the caller has released it
  TTM_TRY(hipStreamSynchronize(stream));
  TTM_PROF(PC_BUILD, launch_planar_quats(zd, n_rot, w.quats, stream));
  TTM_PROF(PC_BUILD, launch_rot_stats(tmpl, mask, 1, L1, L2, w.quats, n_rot, w.rstats, stream));
  TTM_PROF(PC_BUILD, launch_build_coef(w.quats, w.weights, w.rstats, n_rot, order_n, w.coef, stream));
  TTM_PROF(PC_BUILD, launch_build_accum(tmpl, mask, 1, L1, L2, w.quats, w.rstats, w.coef, n_rot, K3, comps3,
                                        w.rtab, stream));
  TTM_PROF(PC_BUILD, launch_planar_gather(comps3, planar_idx(order_n), order_n + 1, (long)L1 * L2, out_components,
                                          stream));
  if (out_bank) {
    const int K2 = order_n + 1;
    const Geo g = make_geo(N, L);
    float2* bank = static_cast<float2*>(out_bank);
    TTM_CALL(bank_forward(g, out_components, K2, bank, stream));
    TTM_CALL(bank_forward(g, mask, 1, bank + (long)K2 * g.bank_slab(), stream));
  }
  return TTM_OK;
}

struct Match2dWs {
  CorrWs cw; PoseWs pw; PeakWs pk; float* comps3; int* cand; float* cand_score; int* list; int* idx; int* total;
  int* pos3; float* quat3; double* lam3; float* score3; int* flags3;
};
// the pose scratch serves all B P candidates of the stack at once; the peak
// search of every plane runs at once on B copies of the peak scratch
static Match2dWs match2d_layout(Carve& c, const Geo& gs, const Geo& gp, int B, int order_n,
                                const ttm_options* opt) {
  const int K3 = ttm_num_components(order_n);
  const size_t P = (size_t)opt->max_peaks, BP = (size_t)B * P;
  Match2dWs m;
  m.cw = corr_layout(c, gs, order_n + 1);
  m.pw = pose_layout(c, gs, (int)BP, K3, opt->refine, opt->n_seeds);
  m.pk.hist = c.take<unsigned>((size_t)kHistBins * B);
  m.pk.ctrl = c.take<unsigned>((size_t)kPeakCtrlWords * B);
  m.pk.allc = c.take<unsigned long long>((size_t)peaks_bigcap(gp) * B);
  m.pk.cand = c.take<unsigned long long>((size_t)kCandCap * B);
  m.comps3 = c.take<float>((size_t)K3 * gs.L1 * gs.L2);
  m.cand = c.take<int>(BP * 3);
  m.cand_score = c.take<float>(BP);
  m.list = c.take<int>(BP * 3);
  m.idx = c.take<int>(BP);
  m.total = c.take<int>(1);
  m.pos3 = c.take<int>(BP * 3);
  m.quat3 = c.take<float>(BP * 4);
  m.lam3 = c.take<double>(BP);
  m.score3 = c.take<float>(BP);
  m.flags3 = c.take<int>(BP);
  return m;
}

constexpr long kPlanarMaxCandidates = 65536;

size_t ttm_match_2d_workspace_bytes(int32_t B, int32_t n1, int32_t n2, int32_t L1, int32_t L2, int32_t order_n,
                                    const ttm_options* opt) {
  if (ttm_num_components(order_n) < 0 || order_n > kPlanarMaxOrder || !opt || !pose_opts_ok(opt)) return 0;
  const ttm_dims N{B, n1, n2}, L{1, L1, L2};
  if (!planar_box_ok(L1, L2) || !image_dims_ok(N) || !fits(L, N)) return 0;
  if ((long)B * opt->max_peaks > kPlanarMaxCandidates) return 0;
  Carve c(nullptr);
  match2d_layout(c, make_geo(N, L), make_geo(ttm_dims{1, n1, n2}, L), B, order_n, opt);
  return c.size();
}

ttm_status ttm_match_2d(const float* images, int32_t B, int32_t n1, int32_t n2, const void* bank,
                        const float* components, const float* tmpl, const float* mask, int32_t L1, int32_t L2,
                        int32_t order_n, const ttm_options* opt, float* out_score, float* out_w, int32_t* out_pos,
                        float* out_z, double* out_lambda, float* out_peak_score, int32_t* out_flags,
                        int32_t* out_count, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!images || !bank || !components || !mask || !opt || !out_score || !out_pos || !out_z || !out_lambda ||
      !out_peak_score || !out_flags || !out_count)
    return TTM_E_ARG;
  if (opt->refine >= 2 && !tmpl) return TTM_E_ARG;
  const int K3 = ttm_num_components(order_n);
  if (K3 < 0 || order_n > kPlanarMaxOrder || !pose_opts_ok(opt)) return TTM_E_ARG;
  const ttm_dims N{B, n1, n2}, L{1, L1, L2};
  if (!planar_box_ok(L1, L2) || !image_dims_ok(N) || !fits(L, N)) return TTM_E_SIZE;
  if ((long)B * opt->max_peaks > kPlanarMaxCandidates) return TTM_E_SIZE;
  if (!ws || ws_bytes < ttm_match_2d_workspace_bytes(B, n1, n2, L1, L2, order_n, opt)) return TTM_E_WORKSPACE;
  Geo gs = make_geo(N, L);
  const Geo gp = make_geo(ttm_dims{1, n1, n2}, L);
  Carve c(ws);
  Match2dWs m = match2d_layout(c, gs, gp, B, order_n, opt);
  PoseWs& w = m.pw;
  const int K2 = order_n + 1;
  TTM_CALL(correlate_into(gs, order_n, K2, images, static_cast<const float2*>(bank), mask, opt->eps_v, out_score,
                          out_w, m.cw, stream, nullptr, nullptr, true));
  TTM_PROF(PC_POSE, launch_planar_embed(components, planar_idx(order_n), K2, K3, (long)L1 * L2, m.comps3, stream));
  // the candidates of every plane at once (the suppression and the count are
  // per image)
  const int P = opt->max_peaks, BP = B * P;
  TTM_PROF(PC_PEAKS, launch_peaks(gp, out_score, opt->threshold, opt->min_dist, P, m.pk, m.cand, m.cand_score,
                                  out_count, stream, B));
  TTM_PROF(PC_POSE, launch_planar_compact(B, P, out_count, m.cand, m.list, m.idx, m.total, stream));
  // the poses of all planes' candidates at once, on the stack; the refinement
  // neighbourhood stays inside each plane
  gs.planar = 1;
  TTM_PROF(PC_STATS, launch_image_stats(images, gs.vol(), nullptr, 0, w.partials, w.stats, stream));
  const int rf = opt->refine == 3 ? 2 : opt->refine;
  TTM_PROF(PC_POSE, launch_pose_tensor(gs, images, m.comps3, mask, order_n, w.stats, opt->eps_v, BP, rf, m.list,
                                       m.total, 0, w.ps, stream));
  TTM_PROF(PC_POSE, launch_pose_solve(gs, out_score, order_n, opt->n_seeds, opt->hopm_max_iter, opt->hopm_tol, BP, rf,
                                      m.list, m.total, 0, images, tmpl, mask, m.pos3, m.quat3, m.lam3, m.score3,
                                      m.flags3, nullptr, w.ps, stream, false, 9, w.moved[0]));
  if (opt->refine == 3) {
    auto tensor = [&](const int* pos, const int* cnt, int cnt_host, const PoseScratch& ps) {
      return launch_pose_tensor(gs, images, m.comps3, mask, order_n, w.stats, opt->eps_v, BP, 2, pos, cnt, cnt_host,
                                ps, stream);
    };
    TTM_CALL(refine_rounds(gs, out_score, order_n, opt, BP, m.total, 0, images, tmpl, mask, m.pos3, m.quat3, m.lam3,
                           m.score3, m.flags3, nullptr, w, tensor, stream));
  }
  TTM_PROF(PC_POSE, launch_planar_scatter(BP, m.total, m.idx, m.pos3, m.quat3, m.lam3, m.score3, m.flags3, out_pos,
                                          out_z, out_lambda, out_peak_score, out_flags, stream));
  return TTM_OK;
}

// --- S'-consistent normalisation ------------------------------------------------
constexpr int kSnormMaxPos = 1 << 16;

static SnormWs snorm_layout(Carve& c, const ttm_dims& L, int n_rot, int max_pos) {
  SnormWs w;
  const int n_pad = snorm_pad(n_rot);
  const size_t nL = (size_t)L.n0 * L.n1 * L.n2;
  const int n_win = max_pos + 1;
  w.quats = c.take<float>(4 * (size_t)n_rot);
  w.weights = c.take<double>((size_t)n_rot);
  w.rtab = c.take<float>(12 * (size_t)n_pad);
  w.kap = c.take<double>((size_t)n_pad);
  w.mlist = c.take<unsigned>(nL);
  w.mval = c.take<float>(nL);
  w.mcount = c.take<int>(2);   // the mask list's count and largest squared radius
  w.slabs = c.take<float>((size_t)n_win * nL);
  w.stat = c.take<double>(4 * (size_t)n_win);
  w.partial = c.take<double>((size_t)n_win * snorm_chunks(n_win, n_pad));
  return w;
}

static bool snorm_box_ok(const ttm_dims& L) {
  return dims_ok(L) && L.n0 <= 1023 && L.n1 <= 1023 && L.n2 <= 1023 && (long)L.n0 * L.n1 * L.n2 <= (1L << 24);
}

size_t ttm_snorm_workspace_bytes(ttm_dims L, int32_t n_rot, int32_t max_pos) {
  if (!snorm_box_ok(L) || n_rot < 1 || max_pos < 1 || max_pos > kSnormMaxPos) return 0;
  Carve c(nullptr);
  snorm_layout(c, L, n_rot, max_pos);
  return c.size();
}

ttm_status ttm_snorm(const float* image, ttm_dims N, const float* tmpl, const float* mask, ttm_dims L,
                     int32_t order_n, const float* quats_host, const double* weights_host, int32_t n_rot,
                     const int32_t* pos, const double* lambda, const int32_t* count, int32_t max_pos,
                     float* out_rho, double* out_D, int32_t* out_flags, void* ws, size_t ws_bytes,
                     hipStream_t stream) {
  if (!image || !tmpl || !mask || !quats_host || !weights_host || !pos || !lambda || !out_rho || !out_D ||
      !out_flags)
    return TTM_E_ARG;
  if (ttm_num_components(order_n) < 0 || n_rot < 1 || max_pos < 1 || max_pos > kSnormMaxPos) return TTM_E_ARG;
  double wsum = 0.0;
  for (int j = 0; j < n_rot; ++j) {
    const float* q = quats_host + 4 * j;
    const double nq = (double)q[0] * q[0] + (double)q[1] * q[1] + (double)q[2] * q[2] + (double)q[3] * q[3];
    if (!std::isfinite(nq) || nq <= 0.0) return TTM_E_ARG;
    if (!std::isfinite(weights_host[j])) return TTM_E_ARG;
    wsum += weights_host[j];
  }
  if (std::fabs(wsum - 1.0) > 1e-6) return TTM_E_ARG;
  if (!snorm_box_ok(L) || !any_dims_ok(N)) return TTM_E_SIZE;
  if (!ws || ws_bytes < ttm_snorm_workspace_bytes(L, n_rot, max_pos)) return TTM_E_WORKSPACE;
  Carve c(ws);
  SnormWs w = snorm_layout(c, L, n_rot, max_pos);
  SnormGeo g;
  g.n0 = N.n0; g.n1 = N.n1; g.n2 = N.n2;
  g.L0 = L.n0; g.L1 = L.n1; g.L2 = L.n2;
  g.max_pos = max_pos;
  g.n_pad = snorm_pad(n_rot);
  TTM_TRY(hipMemcpyAsync(w.quats, quats_host, sizeof(float) * 4 * (size_t)n_rot, hipMemcpyHostToDevice, stream));
  TTM_TRY(hipMemcpyAsync(w.weights, weights_host, sizeof(double) * (size_t)n_rot, hipMemcpyHostToDevice, stream));
  // the host arrays are read before this call returns, so the caller may
  // free or reuse them at once: an asynchronous copy from pageable memory may
  // otherwise be staged after the caller has released it
  TTM_TRY(hipStreamSynchronize(stream));
  TTM_PROF(PC_SNORM, launch_snorm(g, image, tmpl, mask, w.quats, w.weights, n_rot, order_n, pos, count, lambda, w,
                                  out_rho, out_D, out_flags, stream));
  return TTM_OK;
}

// --- low-pass filter -----------------------------------------------------------
size_t ttm_lowpass_workspace_bytes(ttm_dims N) {
  if (!dims_ok(N)) return 0;
  return 2 * sizeof(float) * (size_t)N.n0 * N.n1 * N.n2 + 512;
}

ttm_status ttm_lowpass(const float* in, ttm_dims N, float sigma, int32_t periodic, float* out, void* ws,
                       size_t ws_bytes, hipStream_t stream) {
  if (!in || !out || !std::isfinite(sigma) || sigma < 0.0f || (periodic != 0 && periodic != 1)) return TTM_E_ARG;
  if (!dims_ok(N)) return TTM_E_SIZE;
  const int R = sigma > 0.0f ? (int)std::ceil(3.0 * (double)sigma) : 0;
  if (R > kMaxFilterRadius) return TTM_E_ARG;
  const size_t vol = (size_t)N.n0 * N.n1 * N.n2;
  if (sigma == 0.0f) {
    if (in != out) TTM_TRY(hipMemcpyAsync(out, in, sizeof(float) * vol, hipMemcpyDeviceToDevice, stream));
    return TTM_OK;
  }
  if (!ws || ws_bytes < ttm_lowpass_workspace_bytes(N)) return TTM_E_WORKSPACE;
  // the sampled Gaussian, normalised to unit sum in float64
  FilterTaps taps;
  taps.R = R;
  double h[2 * kMaxFilterRadius + 1], sum = 0.0;
  for (int k = -R; k <= R; ++k) {
    h[k + R] = std::exp(-0.5 * ((double)k / sigma) * ((double)k / sigma));
    sum += h[k + R];
  }
  for (int k = 0; k <= 2 * R; ++k) taps.h[k] = (float)(h[k] / sum);
  Carve c(ws);
  float* a = c.take<float>(vol);
  float* b = c.take<float>(vol);
  TTM_TRY(launch_lowpass(in, out, a, b, N.n0, N.n1, N.n2, periodic, taps, stream));
  return TTM_OK;
}

// --- gradient of the score at fixed positions ----------------------------------
struct GradLayout {
  BuildWs b;
  GradWs g;
  double* stats;
  double* partials;
};
static GradLayout grad_layout(Carve& c, ttm_dims L, int K, int n_rot, int n_pos) {
  GradLayout w;
  w.b = build_layout(c, n_rot, K);
  const long nL = (long)L.n0 * L.n1 * L.n2;
  const long ntiles = (nL + 255) / 256;
  w.g.wv = c.take<double>((size_t)n_pos);
  w.g.mean = c.take<double>((size_t)n_pos);
  w.g.dC = c.take<double>((size_t)n_pos * K);
  w.g.a = c.take<double>((size_t)n_pos);
  w.g.dT = c.take<float>((size_t)K * nL);
  w.g.part = c.take<double>((size_t)ntiles * n_rot * 2);
  w.g.H = c.take<double>((size_t)n_rot * 2);
  w.stats = c.take<double>(4);
  w.partials = c.take<double>(3 * kStatPartials);
  return w;
}

size_t ttm_score_backward_workspace_bytes(ttm_dims L, int32_t order_n, int32_t n_rot, int32_t n_pos) {
  const int K = ttm_num_components(order_n);
  if (K < 0 || n_rot < 1 || n_pos < 1 || !dims_ok(L)) return 0;
  Carve c(nullptr);
  grad_layout(c, L, K, n_rot, n_pos);
  return c.size();
}

ttm_status ttm_score_backward(const float* image, ttm_dims N, const float* tmpl, const float* mask, ttm_dims L,
                              int32_t order_n, const float* quats_host, const double* weights_host, int32_t n_rot,
                              const float* components, const int32_t* positions, int32_t n_pos,
                              const float* grad_score, const ttm_options* opt, float* out_grad_tmpl,
                              float* out_grad_image, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!image || !tmpl || !mask || !quats_host || !weights_host || !components || !positions || !grad_score ||
      !opt)
    return TTM_E_ARG;
  const int K = ttm_num_components(order_n);
  if (K < 0 || n_rot < 1 || n_pos < 1 || !(opt->eps_v >= 0.0f)) return TTM_E_ARG;
  double wsum = 0.0;
  for (int j = 0; j < n_rot; ++j) {
    const float* q = quats_host + 4 * j;
    const double nq = (double)q[0] * q[0] + (double)q[1] * q[1] + (double)q[2] * q[2] + (double)q[3] * q[3];
    if (!std::isfinite(nq) || nq <= 0.0) return TTM_E_ARG;
    if (!std::isfinite(weights_host[j])) return TTM_E_ARG;
    wsum += weights_host[j];
  }
  if (std::fabs(wsum - 1.0) > 1e-6) return TTM_E_ARG;
  // direct window sums: any image extent holds (no FFT)
  if (!dims_ok(L) || !dims_ok(N) || !fits(L, N)) return TTM_E_SIZE;
  if (out_grad_tmpl && (long)L.n0 * L.n1 * L.n2 > kGradMaxTemplate) return TTM_E_SIZE;
  if (!ws || ws_bytes < ttm_score_backward_workspace_bytes(L, order_n, n_rot, n_pos)) return TTM_E_WORKSPACE;
  Carve c(ws);
  GradLayout w = grad_layout(c, L, K, n_rot, n_pos);
  const Geo geo = make_geo(N, L);
  GradGeo g;
  g.n0 = N.n0; g.n1 = N.n1; g.n2 = N.n2; g.L0 = L.n0; g.L1 = L.n1; g.L2 = L.n2;
  g.lo0 = geo.lo0(); g.hi0 = geo.hi0(); g.lo1 = geo.lo1(); g.hi1 = geo.hi1();
  g.lo2 = geo.c2; g.hi2 = N.n2 - L.n2 + geo.c2;
  const long nL = (long)L.n0 * L.n1 * L.n2;
  TTM_PROF(PC_STATS, launch_image_stats(image, geo.vol(), mask, nL, w.partials, w.stats, stream));
  TTM_PROF(PC_POSE, launch_grad_field(g, image, components, mask, order_n, w.stats, opt->eps_v, positions, n_pos,
                                      grad_score, w.g, stream));
  if (out_grad_image) {
    TTM_PROF(PC_POSE, launch_fill_f32(out_grad_image, geo.vol(), 0.0f, stream));
    TTM_PROF(PC_POSE, launch_grad_image(g, image, components, mask, order_n, positions, n_pos, w.g,
                                        out_grad_image, stream));
  }
  if (out_grad_tmpl) {
    TTM_TRY(hipMemcpyAsync(w.b.quats, quats_host, sizeof(float) * 4 * (size_t)n_rot, hipMemcpyHostToDevice,
                           stream));
    TTM_TRY(hipMemcpyAsync(w.b.weights, weights_host, sizeof(double) * (size_t)n_rot, hipMemcpyHostToDevice,
                           stream));
    // the host arrays are read before this call returns, so the caller may
    // free or reuse them at once: an asynchronous copy from pageable memory may
    // otherwise be staged after the caller has released it
    TTM_TRY(hipStreamSynchronize(stream));
    TTM_PROF(PC_BUILD, launch_rot_stats(tmpl, mask, L.n0, L.n1, L.n2, w.b.quats, n_rot, w.b.rstats, stream));
    TTM_PROF(PC_BUILD, launch_build_coef(w.b.quats, w.b.weights, w.b.rstats, n_rot, order_n, w.b.coef, stream));
    TTM_PROF(PC_BUILD, launch_fill_f32(out_grad_tmpl, nL, 0.0f, stream));
    TTM_PROF(PC_BUILD, launch_grad_tmpl(g, image, tmpl, mask, order_n, w.b.quats, n_rot, w.b.coef, w.b.rstats,
                                        w.stats, positions, n_pos, w.g, out_grad_tmpl, stream));
  }
  return TTM_OK;
}

size_t tm_classical_workspace_bytes(ttm_dims N, ttm_dims L, int32_t n_rot) {
  if (!dims_ok(N) || !dims_ok(L) || n_rot < 1) return 0;
  Carve c(nullptr);
  class_layout(c, make_geo(N, L), n_rot);
  return c.size();
}

ttm_status tm_classical(const float* image, ttm_dims N, const float* tmpl, const float* mask, ttm_dims L,
                        const float* quats_host, int32_t n_rot, const ttm_options* opt, float* out_best_ncc,
                        int32_t* out_best_rot, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!image || !tmpl || !mask || !quats_host || !opt || !out_best_ncc || !out_best_rot) return TTM_E_ARG;
  if (n_rot < 1 || !(opt->eps_v >= 0.0f)) return TTM_E_ARG;
  for (int j = 0; j < n_rot; ++j) {
    const float* q = quats_host + 4 * j;
    const double nq = (double)q[0] * q[0] + (double)q[1] * q[1] + (double)q[2] * q[2] + (double)q[3] * q[3];
    if (!std::isfinite(nq) || nq <= 0.0) return TTM_E_ARG;
  }
  if (!dims_ok(L) || !image_dims_ok(N) || !fits(L, N)) return TTM_E_SIZE;
  if (!ws || ws_bytes < tm_classical_workspace_bytes(N, L, n_rot)) return TTM_E_WORKSPACE;
  const Geo g = make_geo(N, L);
  Carve c(ws);
  ClassWs w = class_layout(c, g, n_rot);
  const long half = g.half();
  TTM_TRY(hipMemcpyAsync(w.quats, quats_host, sizeof(float) * 4 * (size_t)n_rot, hipMemcpyHostToDevice, stream));
  // the host arrays are read before this call returns, so the caller may
  // free or reuse them at once: an asynchronous copy from pageable memory may
  // otherwise be staged after the caller has released it
  TTM_TRY(hipStreamSynchronize(stream));
  TTM_CALL(image_forward(g, image, w.Xf, w.Xg, w.stats, w.partials, mask, stream));
  // w(x) from the two masked moments
  TTM_CALL(bank_forward(g, mask, 1, w.bbank, stream));
  const Pass1Args p1{w.Xf, w.bbank, 1, w.Xg, w.bbank, 1, g.bank_slab(), w.H, half};
  TTM_PROF(PC_PASS1, launch_pass1(g, p1, stream));
  TTM_PROF(PC_PEN_INV, pencils_inverse_valid(g, w.H, 2, half, stream));
  Pass3Args a;
  std::memset(&a, 0, sizeof(a));
  a.H = w.H;
  a.pstride = half;
  a.mode = P3_W;
  a.stats = w.stats;
  a.eps_v = opt->eps_v;
  a.out_w = w.w;
  TTM_PROF(PC_PASS3, launch_pass3(g, a, stream));
  // rotation loop in batches
  TTM_PROF(PC_BUILD, launch_rot_stats(tmpl, mask, L.n0, L.n1, L.n2, w.quats, n_rot, w.rstats, stream));
  const int B = n_rot < kClassicalBatch ? n_rot : kClassicalBatch;
  for (int j0 = 0; j0 < n_rot; j0 += B) {
    const int nb = (n_rot - j0) < B ? (n_rot - j0) : B;
    TTM_PROF(PC_BUILD, launch_rot_write(tmpl, mask, L.n0, L.n1, L.n2, w.quats, w.rstats, j0, nb, w.tbatch, stream));
    TTM_CALL(bank_forward(g, w.tbatch, nb, w.bbank, stream));
    const Pass1Args p1{w.Xf, w.bbank, nb, nullptr, nullptr, 0, g.bank_slab(), w.H, half};
    TTM_PROF(PC_PASS1, launch_pass1(g, p1, stream));
    TTM_PROF(PC_PEN_INV, pencils_inverse_valid(g, w.H, nb, half, stream));
    Pass3Args m;
    std::memset(&m, 0, sizeof(m));
    m.H = w.H;
    m.pstride = half;
    m.npairs = nb;
    m.mode = P3_MAX;
    m.best = out_best_ncc;
    m.best_idx = out_best_rot;
    m.first_index = j0;
    m.init = j0 == 0 ? 1 : 0;
    TTM_PROF(PC_PASS3, launch_pass3(g, m, stream));
  }
  TTM_PROF(PC_EPI, launch_classical_final(g, w.w, out_best_ncc, out_best_rot, stream));
  return TTM_OK;
}

void ttm_profile_enable(int32_t on) {
  Prof& p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  p.on = on != 0;
}

int32_t ttm_profile_read(double* ms_out, int64_t* launches_out, int32_t n) {
  Prof& p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  double ms[PC_COUNT] = {0};
  int64_t cnt[PC_COUNT] = {0};
  int32_t status = PC_COUNT;
  for (const auto& u : p.used) {
    const auto& ev = p.pool[u.second];
    if (hipEventSynchronize(ev.second) != hipSuccess) {
      status = TTM_E_HIP;
      continue;
    }
    float t = 0.0f;
    if (hipEventElapsedTime(&t, ev.first, ev.second) != hipSuccess) {
      status = TTM_E_HIP;
      continue;
    }
    ms[u.first] += t;
    cnt[u.first] += 1;
  }
  p.used.clear();
  for (int i = 0; i < n && i < PC_COUNT; ++i) {
    if (ms_out) ms_out[i] = ms[i];
    if (launches_out) launches_out[i] = cnt[i];
  }
  return status;
}

const char* ttm_profile_class_name(int32_t cls) {
  return (cls >= 0 && cls < PC_COUNT) ? kProfNames[cls] : "unknown";
}

}  // extern "C"
