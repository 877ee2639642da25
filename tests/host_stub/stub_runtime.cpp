// The HIP runtime stand-in behind tests/host_stub/hip/*.h and the library's
// launch functions, for running the library's host code on the CPU (under
// AddressSanitizer / UndefinedBehaviorSanitizer in the host-logic test).
//
// Device memory is a registry of address ranges handed out from a reserved
// span that is never dereferenced.  Every launch checks that each buffer it
// is given, with the extent the kernel would touch where that follows from
// the arguments, lies inside one live range.  Streams, events, graphs and
// executable graphs are heap objects freed when destroyed, so a use after
// destruction is a heap-use-after-free.  Capture follows the runtime's
// rules: a side stream joins a capture by waiting on an event recorded in
// it, all of its work must be joined back into the origin stream before the
// capture ends (tracked with vector clocks), nothing synchronises on or
// copies host memory inside a capture, and a capturing stream is not
// destroyed.  Launches made while capturing become graph nodes whose checks
// run again at every replay, against the ranges live at that time.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "../../paper_2311_07561_amd/csrc/ttm_internal.h"

namespace stub {

struct Range {
  uintptr_t base;
  size_t bytes;
  std::string name;
};
struct Check {
  uintptr_t p;
  size_t bytes;
  std::string what;
};
struct Node {
  std::string name;
  std::vector<Check> checks;
};
struct Capture;
constexpr uint32_t kMagicStream = 0x5354524d, kMagicEvent = 0x45564e54, kMagicGraph = 0x47525048,
                   kMagicExec = 0x45584543;

static std::recursive_mutex mu;
static std::map<uintptr_t, Range> ranges;   // live device ranges by base
static uintptr_t next_base = uintptr_t(0x100000000000ull);
static long errors = 0, launches = 0, replays = 0, nodes_replayed = 0;
static long live_streams = 0, live_events = 0, live_graphs = 0, live_execs = 0;

static void fail(const char* fmt, ...) {
  ++errors;
  va_list ap;
  va_start(ap, fmt);
  std::fprintf(stderr, "stub error: ");
  std::vfprintf(stderr, fmt, ap);
  std::fprintf(stderr, "\n");
  va_end(ap);
}

static bool inside(uintptr_t p, size_t bytes) {
  auto it = ranges.upper_bound(p);
  if (it == ranges.begin()) return false;
  --it;
  const Range& r = it->second;
  return p >= r.base && bytes <= r.bytes && p - r.base <= r.bytes - bytes;
}

static void run_checks(const std::string& name, const std::vector<Check>& cs) {
  for (const Check& c : cs) {
    if (c.p == 0) {
      fail("%s: %s is null", name.c_str(), c.what.c_str());
      continue;
    }
    if (!inside(c.p, c.bytes))
      fail("%s: %s [0x%lx, +%zu) is not inside one live device allocation", name.c_str(), c.what.c_str(),
           (unsigned long)c.p, c.bytes);
  }
}

}  // namespace stub

struct StubStream {
  uint32_t magic = stub::kMagicStream;
  int id = 0;
  stub::Capture* cap = nullptr;
  long seq = 0;                        // operations issued on this stream
  std::map<StubStream*, long> clk;     // inside a capture: the operations of each member this stream follows
};
struct StubEvent {
  uint32_t magic = stub::kMagicEvent;
  bool timing = true;
  bool recorded = false;
  stub::Capture* cap = nullptr;        // the capture it was recorded in
  std::map<StubStream*, long> clk;
};
struct StubGraph {
  uint32_t magic = stub::kMagicGraph;
  std::vector<stub::Node> nodes;
};
struct StubExec {
  uint32_t magic = stub::kMagicExec;
  std::vector<stub::Node> nodes;
};

namespace stub {
struct Capture {
  StubStream* origin = nullptr;
  std::set<StubStream*> members;
  std::vector<Node> nodes;
};

static void valid_stream(hipStream_t s, const char* where) {
  if (s && s->magic != kMagicStream) fail("%s: not a live stream", where);
}

// one operation on stream s (a launch or a copy): a node when capturing
static void op(hipStream_t s, const char* name, std::vector<Check> checks) {
  valid_stream(s, name);
  run_checks(name, checks);
  ++launches;
  if (!s) return;
  ++s->seq;
  if (s->cap) {
    s->clk[s] = s->seq;
    s->cap->nodes.push_back(Node{name, std::move(checks)});
  }
}
}  // namespace stub

using namespace stub;

extern "C" {

// --- the harness's side: device ranges --------------------------------------------
void* stub_dev_alloc(size_t bytes, const char* name) {
  std::lock_guard<std::recursive_mutex> lk(mu);
  const uintptr_t b = next_base;
  const size_t span = (bytes + (size_t(1) << 20) - 1) & ~((size_t(1) << 20) - 1);
  next_base += span + (size_t(1) << 20);   // a guard gap between ranges
  ranges[b] = Range{b, bytes, name ? name : "?"};
  return reinterpret_cast<void*>(b);
}
void stub_dev_free(void* p) {
  std::lock_guard<std::recursive_mutex> lk(mu);
  if (ranges.erase(reinterpret_cast<uintptr_t>(p)) != 1) fail("free of an unknown device range");
}
long stub_errors() { return errors; }
long stub_live_handles() { return live_streams + live_events + live_graphs + live_execs; }
void stub_report() {
  std::printf("stub: launches %ld, replays %ld (nodes %ld), errors %ld, live streams %ld events %ld graphs %ld "
              "execs %ld\n",
              launches, replays, nodes_replayed, errors, live_streams, live_events, live_graphs, live_execs);
}
const void* stub_symbol(const void* addr, size_t bytes) {
  std::lock_guard<std::recursive_mutex> lk(mu);
  const uintptr_t b = reinterpret_cast<uintptr_t>(addr);
  if (!ranges.count(b)) ranges[b] = Range{b, bytes, "symbol"};
  return addr;
}

// --- runtime --------------------------------------------------------------------
hipError_t hipGetDevice(int* device) {
  *device = 0;
  return hipSuccess;
}
hipError_t hipStreamGetDevice(hipStream_t stream, hipDevice_t* device) {
  std::lock_guard<std::recursive_mutex> lk(mu);
  valid_stream(stream, "hipStreamGetDevice");
  *device = 0;
  return hipSuccess;
}
hipError_t hipGetLastError(void) { return hipSuccess; }

hipError_t hipStreamCreateWithFlags(hipStream_t* stream, unsigned int) {
  std::lock_guard<std::recursive_mutex> lk(mu);
  static int ids = 0;
  *stream = new StubStream();
  (*stream)->id = ++ids;
  ++live_streams;
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t stream) {
  std::lock_guard<std::recursive_mutex> lk(mu);
  if (!stream) return hipErrorInvalidResourceHandle;
  valid_stream(stream, "hipStreamDestroy");
  if (stream->cap) fail("hipStreamDestroy: the stream is part of an unfinished capture");
  stream->magic = 0;
  delete stream;
  --live_streams;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t stream) {
  std::lock_guard<std::recursive_mutex> lk(mu);
  valid_stream(stream, "hipStreamSynchronize");
  if (stream && stream->cap) {
    fail("hipStreamSynchronize on a capturing stream");
    return hipErrorStreamCaptureUnsupported;
  }
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t stream, hipEvent_t event, unsigned int) {
  std::lock_guard<std::recursive_mutex> lk(mu);
  valid_stream(stream, "hipStreamWaitEvent");
  if (!event || event->magic != kMagicEvent) {
    fail("hipStreamWaitEvent: not a live event");
    return hipErrorInvalidResourceHandle;
  }
  if (!stream) {
    if (event->cap) fail("hipStreamWaitEvent: the null stream waits on an event of a capture");
    return hipSuccess;
  }
  if (event->cap) {
    if (!stream->cap) {
      // the stream joins the capture
      stream->cap = event->cap;
      event->cap->members.insert(stream);
      stream->clk.clear();
      stream->clk[stream] = stream->seq;
    } else if (stream->cap != event->cap) {
      fail("hipStreamWaitEvent: an event of another capture");
      return hipErrorStreamCaptureIsolation;
    }
    for (const auto& kv : event->clk) stream->clk[kv.first] = std::max(stream->clk[kv.first], kv.second);
  } else if (stream->cap) {
    fail("hipStreamWaitEvent: a capturing stream waits on an event recorded outside the capture");
    return hipErrorStreamCaptureIsolation;
  }
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t stream, hipStreamCaptureMode) {
  std::lock_guard<std::recursive_mutex> lk(mu);
  valid_stream(stream, "hipStreamBeginCapture");
  if (!stream) {
    fail("hipStreamBeginCapture on the null stream");
    return hipErrorStreamCaptureUnsupported;
  }
  if (stream->cap) {
    fail("hipStreamBeginCapture: already capturing");
    return hipErrorStreamCaptureUnsupported;
  }
  Capture* c = new Capture();
  c->origin = stream;
  c->members.insert(stream);
  stream->cap = c;
  stream->clk.clear();
  stream->clk[stream] = stream->seq;
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t stream, hipGraph_t* graph) {
  std::lock_guard<std::recursive_mutex> lk(mu);
  valid_stream(stream, "hipStreamEndCapture");
  *graph = nullptr;
  if (!stream || !stream->cap || stream->cap->origin != stream) {
    fail("hipStreamEndCapture: not the origin of a capture");
    return hipErrorStreamCaptureUnsupported;
  }
  Capture* c = stream->cap;
  hipError_t st = hipSuccess;
  for (StubStream* m : c->members) {
    if (m == stream) continue;
    if (m->magic != kMagicStream) {
      fail("hipStreamEndCapture: a member stream was destroyed");
      st = hipErrorStreamCaptureUnjoined;
      continue;
    }
    const long seen = stream->clk.count(m) ? stream->clk[m] : -1;
    if (seen < m->seq) {
      fail("hipStreamEndCapture: stream %d has work not joined into the origin (%ld of %ld)", m->id, seen, m->seq);
      st = hipErrorStreamCaptureUnjoined;
    }
  }
  for (StubStream* m : c->members) {
    if (m->magic != kMagicStream) continue;
    m->cap = nullptr;
    m->clk.clear();
  }
  if (st == hipSuccess) {
    StubGraph* g = new StubGraph();
    g->nodes = std::move(c->nodes);
    *graph = g;
    ++live_graphs;
  }
  delete c;
  return st;
}
hipError_t hipStreamIsCapturing(hipStream_t stream, hipStreamCaptureStatus* status) {
  std::lock_guard<std::recursive_mutex> lk(mu);
  valid_stream(stream, "hipStreamIsCapturing");
  *status = (stream && stream->cap) ? hipStreamCaptureStatusActive : hipStreamCaptureStatusNone;
  return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t* event) { return hipEventCreateWithFlags(event, hipEventDefault); }
hipError_t hipEventCreateWithFlags(hipEvent_t* event, unsigned flags) {
  std::lock_guard<std::recursive_mutex> lk(mu);
  *event = new StubEvent();
  (*event)->timing = !(flags & hipEventDisableTiming);
  ++live_events;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t event, hipStream_t stream) {
  std::lock_guard<std::recursive_mutex> lk(mu);
  valid_stream(stream, "hipEventRecord");
  if (!event || event->magic != kMagicEvent) {
    fail("hipEventRecord: not a live event");
    return hipErrorInvalidResourceHandle;
  }
  event->recorded = true;
  event->cap = stream ? stream->cap : nullptr;
  event->clk = stream && stream->cap ? stream->clk : std::map<StubStream*, long>();
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t event) {
  std::lock_guard<std::recursive_mutex> lk(mu);
  if (!event || event->magic != kMagicEvent) {
    fail("hipEventDestroy: not a live event");
    return hipErrorInvalidResourceHandle;
  }
  event->magic = 0;
  delete event;
  --live_events;
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t event) {
  std::lock_guard<std::recursive_mutex> lk(mu);
  if (!event || event->magic != kMagicEvent) {
    fail("hipEventSynchronize: not a live event");
    return hipErrorInvalidResourceHandle;
  }
  if (event->cap) {
    fail("hipEventSynchronize on an event recorded in a capture");
    return hipErrorStreamCaptureUnsupported;
  }
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t start, hipEvent_t stop) {
  std::lock_guard<std::recursive_mutex> lk(mu);
  for (hipEvent_t e : {start, stop}) {
    if (!e || e->magic != kMagicEvent) {
      fail("hipEventElapsedTime: not a live event");
      return hipErrorInvalidResourceHandle;
    }
    if (!e->timing || !e->recorded || e->cap) {
      fail("hipEventElapsedTime: an event without timing, unrecorded or recorded in a capture");
      return hipErrorInvalidValue;
    }
  }
  *ms = 0.125f;
  return hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t* exec, hipGraph_t graph, hipGraphNode_t*, char*, size_t) {
  std::lock_guard<std::recursive_mutex> lk(mu);
  if (!graph || graph->magic != kMagicGraph) {
    fail("hipGraphInstantiate: not a live graph");
    return hipErrorInvalidValue;
  }
  StubExec* e = new StubExec();
  e->nodes = graph->nodes;
  *exec = e;
  ++live_execs;
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t graph) {
  std::lock_guard<std::recursive_mutex> lk(mu);
  if (!graph || graph->magic != kMagicGraph) {
    fail("hipGraphDestroy: not a live graph");
    return hipErrorInvalidValue;
  }
  graph->magic = 0;
  delete graph;
  --live_graphs;
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t exec) {
  std::lock_guard<std::recursive_mutex> lk(mu);
  if (!exec || exec->magic != kMagicExec) {
    fail("hipGraphExecDestroy: not a live executable graph");
    return hipErrorInvalidValue;
  }
  exec->magic = 0;
  delete exec;
  --live_execs;
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t exec, hipStream_t stream) {
  std::lock_guard<std::recursive_mutex> lk(mu);
  valid_stream(stream, "hipGraphLaunch");
  if (!exec || exec->magic != kMagicExec) {
    fail("hipGraphLaunch: not a live executable graph");
    return hipErrorInvalidValue;
  }
  if (stream && stream->cap) fail("hipGraphLaunch into a capturing stream");
  ++replays;
  for (const Node& n : exec->nodes) {
    run_checks("replay of " + n.name, n.checks);
    ++nodes_replayed;
  }
  if (stream) ++stream->seq;
  return hipSuccess;
}

hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind, hipStream_t stream) {
  std::lock_guard<std::recursive_mutex> lk(mu);
  valid_stream(stream, "hipMemcpyAsync");
  const bool capturing = stream && stream->cap;
  if (kind == hipMemcpyHostToDevice) {
    if (capturing) fail("hipMemcpyAsync from host memory inside a capture");
    // the host side is read here, whole (the sanitizer checks its extent)
    volatile unsigned char acc = 0;
    const unsigned char* h = static_cast<const unsigned char*>(src);
    for (size_t i = 0; i < bytes; ++i) acc = acc ^ h[i];
    op(stream, "hipMemcpyAsync(H2D)", {Check{reinterpret_cast<uintptr_t>(dst), bytes, "dst"}});
  } else if (kind == hipMemcpyDeviceToHost) {
    if (capturing) fail("hipMemcpyAsync to host memory inside a capture");
    std::memset(dst, 0, bytes);
    op(stream, "hipMemcpyAsync(D2H)", {Check{reinterpret_cast<uintptr_t>(src), bytes, "src"}});
  } else if (kind == hipMemcpyDeviceToDevice) {
    op(stream, "hipMemcpyAsync(D2D)", {Check{reinterpret_cast<uintptr_t>(src), bytes, "src"},
                                        Check{reinterpret_cast<uintptr_t>(dst), bytes, "dst"}});
  } else {
    fail("hipMemcpyAsync: a copy kind the library does not use");
    return hipErrorInvalidValue;
  }
  return hipSuccess;
}
hipError_t hipGetSymbolAddress(void** dev_ptr, const void* symbol) {
  *dev_ptr = const_cast<void*>(symbol);
  return hipSuccess;
}

}  // extern "C"

// --- the library's launch functions: argument checks only --------------------------
namespace ttm {

template <class T>
static Check C(const T* p, size_t count, const char* what) {
  return Check{reinterpret_cast<uintptr_t>(p), count * sizeof(T), what};
}
#define LAUNCH(name, s, ...)                                  \
  do {                                                        \
    std::lock_guard<std::recursive_mutex> _lk(stub::mu);      \
    std::vector<Check> _c;                                    \
    __VA_ARGS__                                               \
    stub::op(s, name, std::move(_c));                         \
  } while (0);                                                \
  return hipSuccess

static long L3(int a, int b, int c) { return (long)a * b * c; }

hipError_t launch_image_stats(const float* img, long n, const float* mask, long nm, double* partials,
                              double* stats, hipStream_t s, int mu_order, float* mu) {
  LAUNCH("image_stats", s, _c.push_back(C(img, n, "img")); if (mask) _c.push_back(C(mask, nm, "mask"));
         _c.push_back(C(partials, 3 * kStatPartials, "partials")); _c.push_back(C(stats, 3, "stats"));
         if (mu) _c.push_back(C(mu, num_components(mu_order), "mu")););
}
hipError_t launch_r2c_rows(int n2, const float* src, long src_stride, int len_valid, long nrows, float2* dst0,
                           float2* dst1, long grp, long grp_stride, int mode, const double* stats, hipStream_t s) {
  const long p2 = n2 / 2 + 1;
  const long last = nrows - 1;
  const long rows_out = (last / grp) * grp_stride + last % grp + 1;
  LAUNCH("r2c_rows", s, _c.push_back(C(src, last * src_stride + len_valid, "src"));
         _c.push_back(C(dst0, rows_out * p2, "dst0")); if (mode == 1) {
           _c.push_back(C(dst1, rows_out * p2, "dst1"));
           _c.push_back(C(stats, 2, "stats"));
         });
}
hipError_t launch_pencils(int N, bool, float2* data, long npencils, long Q, long S_outer, long S_axis, int nin,
                          int, int, int shi, int nbatch, long batch_stride, hipStream_t s) {
  const long base_max = ((npencils - 1) / Q) * S_outer + (npencils - 1) % Q;
  const long jmax = std::max<long>(std::min(nin, N) - 1, std::min(shi, N - 1));
  LAUNCH("pencils", s,
         _c.push_back(C(data, base_max + jmax * S_axis + (long)(nbatch - 1) * batch_stride + 1, "data")););
}
static void pass1_checks(const Geo& g, const Pass1Args& a, std::vector<Check>& c) {
  c.push_back(C(a.src0, g.half(), "src0"));
  c.push_back(C(a.tmpl0, (a.nt0 - 1) * a.tmpl_stride + g.bank_slab(), "tmpl0"));
  if (a.nt1 > 0) {
    c.push_back(C(a.src1, g.half(), "src1"));
    c.push_back(C(a.tmpl1, (a.nt1 - 1) * a.tmpl_stride + g.bank_slab(), "tmpl1"));
  }
  c.push_back(C(a.out, (long)(a.nt0 + a.nt1 - 1) * a.out_stride + g.half(), "out"));
}
hipError_t launch_pass1(const Geo& g, const Pass1Args& a, hipStream_t s) {
  LAUNCH("pass1", s, pass1_checks(g, a, _c););
}
bool two_pass_supported(const Geo& g) {
  return g.n1 == 256 && g.n2 == 256 && supported_len(g.n0) && g.n0 <= 256 && g.planar == 0;
}
hipError_t launch_pass1x(const Geo& g, const Pass1Args& a, hipStream_t s) {
  if (!two_pass_supported(g)) return hipErrorInvalidValue;
  LAUNCH("pass1x", s, pass1_checks(g, a, _c););
}
static void pass3_checks(const Geo& g, const Pass3Args& a, std::vector<Check>& c) {
  const long arrays = a.mode == P3_W ? 2 : (a.mode == P3_MAX ? a.npairs : a.npairs + 2);
  c.push_back(C(a.H, (arrays - 1) * a.pstride + g.half(), "H"));
  if (a.mode == P3_SCORE || a.mode == P3_FIELD) {
    c.push_back(C(a.mu, a.npairs, "mu"));
    c.push_back(C(a.stats, 3, "stats"));
  }
  if (a.mode == P3_SCORE) c.push_back(C(a.out_score, g.vol(), "out_score"));
  if (a.out_w) c.push_back(C(a.out_w, g.vol(), "out_w"));
  if (a.mode == P3_MAX) {
    c.push_back(C(a.best, g.vol(), "best"));
    c.push_back(C(a.best_idx, g.vol(), "best_idx"));
  }
  if (a.mode == P3_FIELD) c.push_back(C(a.out_C, a.npairs * a.c_plane, "out_C"));
}
hipError_t launch_pass3(const Geo& g, const Pass3Args& a, hipStream_t s) {
  LAUNCH("pass3", s, pass3_checks(g, a, _c););
}
hipError_t launch_pass3x(const Geo& g, const Pass3Args& a, hipStream_t s) {
  if (!two_pass_supported(g) || a.mode != P3_SCORE || !a.out_w) return hipErrorInvalidValue;
  LAUNCH("pass3x", s, pass3_checks(g, a, _c););
}
hipError_t launch_classical_final(const Geo& g, const float* w, float* best, int* idx, hipStream_t s) {
  LAUNCH("classical_final", s, _c.push_back(C(w, g.vol(), "w")); _c.push_back(C(best, g.vol(), "best"));
         _c.push_back(C(idx, g.vol(), "idx")););
}
hipError_t launch_fill_f32(float* p, long n, float, hipStream_t s) {
  LAUNCH("fill_f32", s, _c.push_back(C(p, n, "p")););
}
hipError_t launch_fill_i32(int* p, long n, int, hipStream_t s) {
  LAUNCH("fill_i32", s, _c.push_back(C(p, n, "p")););
}
hipError_t launch_rot_stats(const float* tmpl, const float* mask, int L0, int L1, int L2, const float* quats, int nrot,
                            double* rstats, hipStream_t s) {
  LAUNCH("rot_stats", s, _c.push_back(C(tmpl, L3(L0, L1, L2), "tmpl")); _c.push_back(C(mask, L3(L0, L1, L2), "mask"));
         _c.push_back(C(quats, 4L * nrot, "quats")); _c.push_back(C(rstats, 2L * nrot, "rstats")););
}
hipError_t launch_build_coef(const float* quats, const double* weights, const double* rstats, int nrot, int order_n,
                             double* coef, hipStream_t s) {
  LAUNCH("build_coef", s, _c.push_back(C(quats, 4L * nrot, "quats")); _c.push_back(C(weights, nrot, "weights"));
         _c.push_back(C(rstats, 2L * nrot, "rstats"));
         _c.push_back(C(coef, (long)nrot * num_components(order_n), "coef")););
}
hipError_t launch_build_accum(const float* tmpl, const float* mask, int L0, int L1, int L2, const float* quats,
                              const double* rstats, const double* coef, int nrot, int K, float* comps, float* rtab,
                              hipStream_t s) {
  LAUNCH("build_accum", s, _c.push_back(C(tmpl, L3(L0, L1, L2), "tmpl"));
         _c.push_back(C(mask, L3(L0, L1, L2), "mask")); _c.push_back(C(quats, 4L * nrot, "quats"));
         _c.push_back(C(rstats, 2L * nrot, "rstats")); _c.push_back(C(coef, (long)nrot * K, "coef"));
         _c.push_back(C(comps, K * L3(L0, L1, L2), "comps")); if (rtab) _c.push_back(C(rtab, 9L * nrot, "rtab")););
}
hipError_t launch_rot_write(const float* tmpl, const float* mask, int L0, int L1, int L2, const float* quats,
                            const double* rstats, int j0, int nb, float* out, hipStream_t s) {
  LAUNCH("rot_write", s, _c.push_back(C(tmpl, L3(L0, L1, L2), "tmpl"));
         _c.push_back(C(mask, L3(L0, L1, L2), "mask")); _c.push_back(C(quats, 4L * (j0 + nb), "quats"));
         _c.push_back(C(rstats, 2L * (j0 + nb), "rstats")); _c.push_back(C(out, nb * L3(L0, L1, L2), "out")););
}
hipError_t launch_multiplicities(int order_n, float* mu, hipStream_t s) {
  LAUNCH("multiplicities", s, _c.push_back(C(mu, num_components(order_n), "mu")););
}

// the scan's 64 sub-lists: runs of 16 planes (1 for a single plane) by
// 8 x 32 columns of the valid region, 16 x 8 x 32 / 8 keys per block (64 for
// one plane), each sub-list long enough for its share of the blocks
long peaks_bigcap(const Geo& g) {
  const long e0 = g.n0 - g.L0 + 1, e1 = g.n1 - g.L1 + 1, e2 = g.n2 - g.L2 + 1;
  const long run = g.n0 == 1 ? 1 : 16, keys = run == 1 ? 64 : run * 32;
  const long nblk = ((e0 + run - 1) / run) * ((e1 + 7) / 8) * ((e2 + 31) / 32);
  return 64 * ((nblk + 63) / 64 * keys);
}
hipError_t launch_peaks(const Geo& g, const float* score, float, float, int max_peaks, const PeakWs& w, int* out_pos,
                        float* out_score, int* out_count, hipStream_t s, int planes) {
  LAUNCH("peaks", s, _c.push_back(C(score, planes * g.vol(), "score"));
         _c.push_back(C(w.hist, (long)planes * kHistBins, "hist"));
         _c.push_back(C(w.ctrl, (long)planes * kPeakCtrlWords, "ctrl"));
         _c.push_back(C(w.allc, planes * peaks_bigcap(g), "allc"));
         _c.push_back(C(w.cand, (long)planes * kCandCap, "cand"));
         _c.push_back(C(out_pos, 3L * planes * max_peaks, "out_pos"));
         _c.push_back(C(out_score, (long)planes * max_peaks, "out_score"));
         _c.push_back(C(out_count, 2L * planes, "out_count")););
}
hipError_t launch_pose_tensor(const Geo& g, const float* image, const float* comps, const float* mask, int order_n,
                              const double* img_stats, float, int max_peaks, int refine, const int* pos_in,
                              const int* count_dev, int, const PoseScratch& ps, hipStream_t s) {
  const long K = num_components(order_n), nb = (long)max_peaks * (refine ? 27 : 1), l3 = L3(g.L0, g.L1, g.L2);
  LAUNCH("pose_tensor", s, _c.push_back(C(image, g.vol(), "image")); _c.push_back(C(comps, K * l3, "comps"));
         _c.push_back(C(mask, l3, "mask")); _c.push_back(C(img_stats, 2, "img_stats"));
         _c.push_back(C(pos_in, 3L * max_peaks, "pos_in")); if (count_dev) _c.push_back(C(count_dev, 1, "count"));
         _c.push_back(C(ps.C, nb * K, "ps.C")); _c.push_back(C(ps.w, nb, "ps.w")); _c.push_back(C(ps.ok, nb, "ps.ok"));
         if (!g.planar) _c.push_back(C(ps.mom, nb * 3, "ps.mom"));
         if (ps.active) _c.push_back(C(ps.active, max_peaks, "ps.active")););
}
hipError_t launch_field_at(const Geo& g, const float2* H, long pstride, int K, const float* wmap, int max_peaks,
                           int refine, const int* pos_in, const int* count_dev, int, const PoseScratch& ps,
                           hipStream_t s) {
  const long nb = (long)max_peaks * (refine ? 27 : 1);
  LAUNCH("field_at", s, _c.push_back(C(H, (long)(K - 1) * pstride + g.half(), "H"));
         _c.push_back(C(wmap, g.vol(), "wmap")); _c.push_back(C(pos_in, 3L * max_peaks, "pos_in"));
         if (count_dev) _c.push_back(C(count_dev, 1, "count")); _c.push_back(C(ps.C, nb * K, "ps.C"));
         _c.push_back(C(ps.w, nb, "ps.w")); _c.push_back(C(ps.ok, nb, "ps.ok"));
         if (ps.active) _c.push_back(C(ps.active, max_peaks, "ps.active")););
}
hipError_t launch_pose_solve(const Geo& g, const float* score, int order_n, int n_seeds, int, double, int max_peaks,
                             int refine, const int* pos_in, const int* count_dev, int, const float* image,
                             const float* tmpl, const float* mask, int* out_pos, float* out_quat, double* out_lambda,
                             float* out_score, int* out_flags, double* out_C, const PoseScratch& ps, hipStream_t s,
                             bool, int, int* moved) {
  const long K = num_components(order_n), nb = (long)max_peaks * (refine ? 27 : 1), l3 = L3(g.L0, g.L1, g.L2);
  const long P = max_peaks;
  LAUNCH("pose_solve", s, if (score) _c.push_back(C(score, g.vol(), "score"));
         _c.push_back(C(ps.seeds, 4L * n_seeds, "ps.seeds")); _c.push_back(C(ps.C, nb * K, "ps.C"));
         _c.push_back(C(ps.ok, nb, "ps.ok")); _c.push_back(C(ps.q, nb * 4, "ps.q"));
         _c.push_back(C(ps.lam, nb, "ps.lam")); _c.push_back(C(ps.flags, nb, "ps.flags"));
         _c.push_back(C(ps.w, nb, "ps.w")); _c.push_back(C(pos_in, 3 * P, "pos_in"));
         if (count_dev) _c.push_back(C(count_dev, 1, "count")); if (refine == 2) {
           _c.push_back(C(image, g.vol(), "image"));
           _c.push_back(C(tmpl, l3, "tmpl"));
           _c.push_back(C(mask, l3, "mask"));
           _c.push_back(C(ps.mlist, l3, "ps.mlist"));
           _c.push_back(C(ps.mval, l3, "ps.mval"));
           _c.push_back(C(ps.mcount, 2, "ps.mcount"));
           _c.push_back(C(ps.ncc, nb, "ps.ncc"));
           _c.push_back(C(ps.mbits, mask_bricks(g.L0, g.L1, g.L2), "ps.mbits"));
         } if (ps.active) _c.push_back(C(ps.active, P, "ps.active"));
         _c.push_back(C(out_pos, 3 * P, "out_pos"));
         _c.push_back(C(out_quat, 4 * P, "out_quat")); _c.push_back(C(out_lambda, P, "out_lambda"));
         _c.push_back(C(out_flags, P, "out_flags")); if (out_score) _c.push_back(C(out_score, P, "out_score"));
         if (out_C) _c.push_back(C(out_C, P * K, "out_C"));
         if (moved) _c.push_back(C(moved, P, "moved")););
}
hipError_t launch_mask_list(const float* mask, int L0, int L1, int L2, unsigned* list, float* mval, int* count,
                            hipStream_t s, unsigned long long* bits) {
  LAUNCH("mask_list", s, _c.push_back(C(mask, L3(L0, L1, L2), "mask"));
         _c.push_back(C(list, L3(L0, L1, L2), "list")); _c.push_back(C(mval, L3(L0, L1, L2), "mval"));
         _c.push_back(C(count, 2, "count")); if (bits) _c.push_back(C(bits, mask_bricks(L0, L1, L2), "bits")););
}

// the rest: each buffer must at least start inside a live range
#define P1(p) _c.push_back(C(p, 1, #p))
hipError_t launch_planar_quats(const float* z, int nrot, float* quats, hipStream_t s) {
  LAUNCH("planar_quats", s, _c.push_back(C(z, 2L * nrot, "z")); _c.push_back(C(quats, 4L * nrot, "quats")););
}
hipError_t launch_planar_mu(int order_n, float* mu, hipStream_t s) {
  LAUNCH("planar_mu", s, _c.push_back(C(mu, num_components(order_n), "mu")););
}
hipError_t launch_planar_gather(const float* comps3, const PlanarIdx&, int, long, float* comps2, hipStream_t s) {
  LAUNCH("planar_gather", s, P1(comps3); P1(comps2););
}
hipError_t launch_planar_embed(const float* comps2, const PlanarIdx&, int, int, long, float* comps3, hipStream_t s) {
  LAUNCH("planar_embed", s, P1(comps2); P1(comps3););
}
hipError_t launch_planar_compact(int, int, const int* counts, const int* cand, int* list, int* idx, int* total,
                                 hipStream_t s) {
  LAUNCH("planar_compact", s, P1(counts); P1(cand); P1(list); P1(idx); P1(total););
}
hipError_t launch_planar_scatter(int, const int* total, const int* idx, const int* pos3, const float* quat3,
                                 const double* lam3, const float* score3, const int* flags3, int* pos2, float* z2,
                                 double* lam, float* score, int* flags, hipStream_t s) {
  LAUNCH("planar_scatter", s, P1(total); P1(idx); P1(pos3); P1(quat3); P1(lam3); P1(flags3); P1(pos2); P1(z2);
         P1(lam); P1(flags); if (score3) P1(score3); if (score) P1(score););
}
int snorm_pad(int n_rot) { return (n_rot + 7) / 8 * 8; }
int snorm_chunks(int n_win, int n_pad) {
  const int groups = n_pad / 8;
  int nchunk = (512 + n_win - 1) / n_win;
  nchunk = std::min(nchunk, std::max(1, (groups + 15) / 16));
  return std::max(1, nchunk);
}
hipError_t launch_snorm(const SnormGeo&, const float* image, const float* tmpl, const float* mask, const float* quats,
                        const double* weights, int, int, const int* pos, const int* count_dev, const double* lambda,
                        const SnormWs& w, float* out_rho, double* out_D, int* out_flags, hipStream_t s) {
  LAUNCH("snorm", s, P1(image); P1(tmpl); P1(mask); P1(quats); P1(weights); P1(pos); P1(count_dev); P1(lambda);
         P1(w.rtab); P1(w.kap); P1(w.mlist); _c.push_back(C(w.mcount, 2, "w.mcount")); P1(w.slabs); P1(w.stat); P1(w.partial); P1(out_rho); P1(out_D);
         P1(out_flags););
}
hipError_t launch_lowpass(const float* in, float* out, float* tmp_a, float* tmp_b, int n0, int n1, int n2, int,
                          const FilterTaps&, hipStream_t s) {
  LAUNCH("lowpass", s, _c.push_back(C(in, L3(n0, n1, n2), "in")); _c.push_back(C(out, L3(n0, n1, n2), "out"));
         _c.push_back(C(tmp_a, L3(n0, n1, n2), "tmp_a")); _c.push_back(C(tmp_b, L3(n0, n1, n2), "tmp_b")););
}
hipError_t launch_grad_field(const GradGeo&, const float* image, const float* comps, const float* mask, int,
                             const double* img_stats, float, const int* pos, int, const float* grad_F,
                             const GradWs& w, hipStream_t s) {
  LAUNCH("grad_field", s, P1(image); P1(comps); P1(mask); P1(img_stats); P1(pos); P1(grad_F); P1(w.wv); P1(w.dC););
}
hipError_t launch_grad_image(const GradGeo&, const float* image, const float* comps, const float* mask, int,
                             const int* pos, int, const GradWs& w, float* grad_image, hipStream_t s) {
  LAUNCH("grad_image", s, P1(image); P1(comps); P1(mask); P1(pos); P1(w.wv); P1(grad_image););
}
hipError_t launch_grad_tmpl(const GradGeo&, const float* image, const float* tmpl, const float* mask, int,
                            const float* quats, int, const double* coef, const double* rstats, const double* stats,
                            const int* pos, int, const GradWs& w, float* grad_tmpl, hipStream_t s) {
  LAUNCH("grad_tmpl", s, P1(image); P1(tmpl); P1(mask); P1(quats); P1(coef); P1(rstats); P1(stats); P1(pos);
         P1(w.dT); P1(grad_tmpl););
}
hipError_t launch_tile_gather(const float* image, const TileGeo& g, float* tile, hipStream_t s) {
  LAUNCH("tile_gather", s, _c.push_back(C(image, L3(g.n0, g.n1, g.n2), "image"));
         _c.push_back(C(tile, L3(g.T, g.T, g.T), "tile")););
}
hipError_t launch_tile_scatter(const float* tscore, const float* tw, const TileGeo& g, float* score, float* w,
                               hipStream_t s) {
  LAUNCH("tile_scatter", s, _c.push_back(C(tscore, L3(g.T, g.T, g.T), "tscore"));
         _c.push_back(C(score, L3(g.n0, g.n1, g.n2), "score")); if (w) {
           _c.push_back(C(tw, L3(g.T, g.T, g.T), "tw"));
           _c.push_back(C(w, L3(g.n0, g.n1, g.n2), "w"));
         });
}
long rmap_table_uint4(int order_n, int n_seeds) {
  return (long)(n_seeds / 32) * 2 * ((num_components(order_n) + 15) / 16) * 32;
}
hipError_t launch_rmap_table(int order_n, const float* seeds, int n_seeds, uint4* table, hipStream_t s) {
  LAUNCH("rmap_table", s, _c.push_back(C(seeds, 4L * n_seeds, "seeds"));
         _c.push_back(C(table, rmap_table_uint4(order_n, n_seeds), "table")););
}
hipError_t launch_rmap_scan(const Geo&, int, const float* planes, const uint4* table, int, int* group, hipStream_t s) {
  LAUNCH("rmap_scan", s, P1(planes); P1(table); P1(group););
}
hipError_t launch_rmap_polish(const Geo&, int, const float* planes, const float* seeds, const int* group, int, double,
                              float* out_score, float* out_quat, float* out_lambda, int* unconv, hipStream_t s) {
  LAUNCH("rmap_polish", s, P1(planes); P1(seeds); P1(group); P1(out_score); P1(out_quat); P1(out_lambda);
         P1(unconv););
}

}  // namespace ttm
