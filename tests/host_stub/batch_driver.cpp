// Drives the library's batching entry points on the CPU, against the HIP
// stand-in of stub_runtime.cpp, with the call sequence of the batching
// benchmark: 64 tomograms (edges read from the job file) against templates of
// 24, 32 and 48 voxels at refine 3, 9 peaks per job; the tile edge of each
// job from ttm_choose_tile over a fixed table; one eager run on one stream,
// one on four branches, one graph of all jobs on four branches replayed
// three times, then one graph per tomogram (its three jobs, three branches)
// created, replayed twice and destroyed, and the outputs released.  A final
// negative control releases one output and replays a graph that uses it:
// the stand-in must report that replay.
//
// usage: batch_driver <job file: one tomogram edge per line>
// exit status 0 when every call returned TTM_OK, the stand-in found no
// misuse, every handle was released and the negative control was caught.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#include "ttm.h"

extern "C" {
void* stub_dev_alloc(size_t bytes, const char* name);
void stub_dev_free(void* p);
long stub_errors();
long stub_live_handles();
void stub_report();
}

namespace {

int failures = 0;
void expect(bool ok, const char* what) {
  if (!ok) {
    ++failures;
    std::fprintf(stderr, "driver: %s\n", what);
  }
}
void expect_ok(ttm_status st, const char* what) {
  if (st != TTM_OK) {
    ++failures;
    std::fprintf(stderr, "driver: %s returned %d (%s)\n", what, (int)st, ttm_status_string(st));
  }
}

struct Template {
  int L;
  const float *tmpl, *mask, *comps;
  const void* bank[3];   // tile edges 64, 128, 256 (null where T < L)
};
struct Outputs {
  float* score;
  int32_t* pos;
  float* quat;
  double* lam;
  float* peak_score;
  int32_t* flags;
  int32_t* count;
  float* image;
};

template <class T>
T* dev(size_t count, const char* name) {
  return static_cast<T*>(stub_dev_alloc(count * sizeof(T), name));
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 2) {
    std::fprintf(stderr, "usage: %s <job file>\n", argv[0]);
    return 2;
  }
  std::vector<int> edges;
  {
    FILE* f = std::fopen(argv[1], "r");
    if (!f) return 2;
    int e;
    while (std::fscanf(f, "%d", &e) == 1) edges.push_back(e);
    std::fclose(f);
  }
  const int order = 4;
  const int K = ttm_num_components(order);
  const int tiles[3] = {64, 128, 256};
  const float tile_ms[3] = {1.1f, 5.3f, 41.0f};   // a fixed stand-in for the autotuner's table

  ttm_options opt;
  ttm_default_options(&opt);
  opt.max_peaks = 9;
  opt.min_dist = 12.0f;
  opt.threshold = 0.0f;
  opt.refine = 3;

  std::vector<Template> temps;
  for (int L : {24, 32, 48}) {
    Template t{};
    t.L = L;
    const size_t l3 = (size_t)L * L * L;
    t.tmpl = dev<float>(l3, "tmpl");
    t.mask = dev<float>(l3, "mask");
    t.comps = dev<float>(l3 * K, "components");
    for (int i = 0; i < 3; ++i)
      if (tiles[i] >= L)
        t.bank[i] = stub_dev_alloc(ttm_bank_bytes(ttm_dims{tiles[i], tiles[i], tiles[i]}, ttm_dims{L, L, L}, K),
                                   "bank");
    temps.push_back(t);
  }

  std::vector<ttm_batch_job> jobs;
  std::vector<Outputs> outs;
  for (int e : edges) {
    const size_t v = (size_t)e * e * e;
    float* image = dev<float>(v, "image");
    for (const Template& t : temps) {
      const ttm_dims N{e, e, e}, L{t.L, t.L, t.L};
      const int T = ttm_choose_tile(N, L, tiles, tile_ms, 3);
      expect(T == 64 || T == 128 || T == 256, "ttm_choose_tile picked no candidate");
      const int ti = T == 64 ? 0 : (T == 128 ? 1 : 2);
      Outputs o{};
      o.image = image;
      o.score = dev<float>(v, "out_score");
      o.pos = dev<int32_t>(3 * (size_t)opt.max_peaks, "out_pos");
      o.quat = dev<float>(4 * (size_t)opt.max_peaks, "out_quat");
      o.lam = dev<double>((size_t)opt.max_peaks, "out_lambda");
      o.peak_score = dev<float>((size_t)opt.max_peaks, "out_peak_score");
      o.flags = dev<int32_t>((size_t)opt.max_peaks, "out_flags");
      o.count = dev<int32_t>(2, "out_count");
      ttm_batch_job j{};
      j.image = image;
      j.N = N;
      j.bank = t.bank[ti];
      j.tile = T;
      j.components = t.comps;
      j.mask = t.mask;
      j.tmpl = t.tmpl;
      j.L = L;
      j.out_score = o.score;
      j.out_w = nullptr;
      j.out_pos = o.pos;
      j.out_quat = o.quat;
      j.out_lambda = o.lam;
      j.out_peak_score = o.peak_score;
      j.out_flags = o.flags;
      j.out_count = o.count;
      jobs.push_back(j);
      outs.push_back(o);
    }
  }
  const int nj = (int)jobs.size();
  const int S = 4;
  const size_t ws_bytes = ttm_batch_workspace_bytes(jobs.data(), nj, order, &opt, S);
  expect(ws_bytes > 0, "ttm_batch_workspace_bytes returned 0");
  void* ws = stub_dev_alloc(ws_bytes, "workspace");
  std::printf("driver: %d jobs, workspace %.1f GiB on %d branches\n", nj, ws_bytes / double(1 << 30), S);

  hipStream_t main_stream = nullptr, side = nullptr;
  expect(hipStreamCreateWithFlags(&main_stream, hipStreamNonBlocking) == hipSuccess, "stream");
  expect(hipStreamCreateWithFlags(&side, hipStreamNonBlocking) == hipSuccess, "stream");

  // eager: one stream, then four branches forked from the main stream
  expect_ok(ttm_batch_match(jobs.data(), nj, order, &opt, 1, ws, ws_bytes, main_stream), "ttm_batch_match (1)");
  expect_ok(ttm_batch_match(jobs.data(), nj, order, &opt, S, ws, ws_bytes, main_stream), "ttm_batch_match (4)");

  // one graph of every job, captured on a side stream, replayed three times
  ttm_graph g = nullptr;
  expect_ok(ttm_batch_graph_create(jobs.data(), nj, order, &opt, S, ws, ws_bytes, side, &g), "graph create (all)");
  for (int r = 0; r < 3; ++r) expect_ok(ttm_graph_launch(g, main_stream), "graph launch (all)");
  ttm_graph_destroy(g);

  // one graph per tomogram: created, replayed twice, destroyed
  const int nk = (int)temps.size();
  for (int i = 0; i + nk <= nj; i += nk) {
    ttm_graph gi = nullptr;
    expect_ok(ttm_batch_graph_create(jobs.data() + i, nk, order, &opt, nk, ws, ws_bytes, side, &gi),
              "graph create (tomogram)");
    expect_ok(ttm_graph_launch(gi, main_stream), "graph launch (tomogram)");
    expect_ok(ttm_graph_launch(gi, main_stream), "graph launch (tomogram)");
    ttm_graph_destroy(gi);
  }

  // calls that must be refused, leaving nothing behind
  {
    ttm_graph gx = nullptr;
    expect(ttm_batch_graph_create(jobs.data(), nj, order, &opt, S, ws, ws_bytes / 2, side, &gx) ==
               TTM_E_WORKSPACE && gx == nullptr,
           "a short workspace is not refused");
    expect(ttm_batch_graph_create(jobs.data(), nj, order, &opt, S, ws, ws_bytes, nullptr, &gx) == TTM_E_ARG,
           "capture on the null stream is not refused");
    ttm_options bad = opt;
    bad.check_finite = 1;
    expect(ttm_batch_match(jobs.data(), nj, order, &bad, 1, ws, ws_bytes, main_stream) == TTM_E_ARG,
           "check_finite in a batch is not refused");
  }
  const long errors_before_control = stub_errors();

  // negative control: a graph whose job output is released before a replay
  {
    ttm_graph gc = nullptr;
    expect_ok(ttm_batch_graph_create(jobs.data(), 1, order, &opt, 1, ws, ws_bytes, side, &gc), "graph create (ctl)");
    stub_dev_free(outs[0].score);
    expect_ok(ttm_graph_launch(gc, main_stream), "graph launch (ctl)");
    ttm_graph_destroy(gc);
    outs[0].score = nullptr;
  }
  const bool control_caught = stub_errors() > errors_before_control;

  // release everything
  for (size_t k = 0; k < outs.size(); ++k) {
    Outputs& o = outs[k];
    if (o.score) stub_dev_free(o.score);
    stub_dev_free(o.pos);
    stub_dev_free(o.quat);
    stub_dev_free(o.lam);
    stub_dev_free(o.peak_score);
    stub_dev_free(o.flags);
    stub_dev_free(o.count);
    if (k % temps.size() == 0) stub_dev_free(o.image);
  }
  for (Template& t : temps) {
    stub_dev_free(const_cast<float*>(t.tmpl));
    stub_dev_free(const_cast<float*>(t.mask));
    stub_dev_free(const_cast<float*>(t.comps));
    for (const void* b : t.bank)
      if (b) stub_dev_free(const_cast<void*>(b));
  }
  stub_dev_free(ws);
  expect(hipStreamDestroy(main_stream) == hipSuccess, "stream destroy");
  expect(hipStreamDestroy(side) == hipSuccess, "stream destroy");

  stub_report();
  expect(stub_live_handles() == 0, "streams, events or graphs left alive");
  std::printf("driver: misuse before the control %ld, control caught %d, call failures %d\n", errors_before_control,
              (int)control_caught, failures);
  return (errors_before_control == 0 && control_caught && failures == 0) ? 0 : 1;
}
