// Autotuner: Delta_d, the round shape and the DCO kernel's launch shape chosen by timing a fixed
// grid of search configurations on a query sample, subject to agreement with a FULL_D search.
#include <algorithm>
#include <string>
#include <unordered_set>
#include <vector>

#include "engine.h"

using namespace dade;

#define FAIL(code, msg)      \
  do {                       \
    dade::set_error(msg);    \
    return (code);           \
  } while (0)

#define HIPC(expr)                                                 \
  do {                                                             \
    hipError_t e_ = (expr);                                        \
    if (e_ != hipSuccess) FAIL(DADE_EDEVICE, hip_msg(e_, #expr));  \
  } while (0)

namespace {

// Device result sets and events of one tuning call (freed on every return).
struct TuneBuffers {
  dade_index* ix = nullptr;
  hipStream_t s = nullptr;
  int64_t* ids[2] = {nullptr, nullptr};
  float* d2[2] = {nullptr, nullptr};
  size_t b_ids = 0, b_d2 = 0;
  hipEvent_t ev[2] = {nullptr, nullptr};
  ~TuneBuffers() {
    (void)hipStreamSynchronize(s);
    for (int i = 0; i < 2; ++i) {
      index_free(ix, ids[i], b_ids);
      index_free(ix, d2[i], b_d2);
      if (ev[i]) (void)hipEventDestroy(ev[i]);
    }
  }
};

}  // namespace

extern "C" int dade_autotune(dade_index* ix, const float* Q, int64_t nq, int32_t k, int32_t nprobe,
                             const int32_t* k_per_query, const int32_t* nprobe_per_query, float min_agreement,
                             int32_t reps, dade_search_opts* opts, dade_tune_result* results, int32_t* n_results,
                             void* stream) {
  if (!ix || !opts) FAIL(DADE_EINVAL, "index and opts are required");
  if (nq < 1) FAIL(DADE_EINVAL, "the sample needs at least one query");
  if (!(min_agreement >= 0.f && min_agreement <= 1.f)) FAIL(DADE_EINVAL, "min_agreement must be in [0, 1]");
  if (reps < 0) FAIL(DADE_EINVAL, "reps must be >= 0");
  if (reps == 0) reps = 5;
  if (opts->mode != DADE_MODE_DADE) FAIL(DADE_EINVAL, "the base options must be in DADE mode");
  if (n_results) *n_results = 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const dade_search_opts base = *opts;
  const int dim = index_dim(ix);
  TuneBuffers B;
  B.ix = ix;
  B.s = s;
  for (int i = 0; i < 2; ++i) {
    void* p = nullptr;
    int rc = index_alloc(ix, &p, sizeof(int64_t) * size_t(nq) * k);
    if (rc) return rc;
    B.ids[i] = static_cast<int64_t*>(p);
    B.b_ids = sizeof(int64_t) * size_t(nq) * k;
    if ((rc = index_alloc(ix, &p, sizeof(float) * size_t(nq) * k))) return rc;
    B.d2[i] = static_cast<float*>(p);
    B.b_d2 = sizeof(float) * size_t(nq) * k;
    HIPC(hipEventCreate(&B.ev[i]));
  }
  // per-query K (host) for the agreement
  std::vector<int32_t> kq(size_t(nq), k);
  if (k_per_query) {
    HIPC(hipMemcpyAsync(kq.data(), k_per_query, sizeof(int32_t) * size_t(nq), hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    for (auto& v : kq) v = std::max(1, std::min(v, k));
  }
  // 1. the FULL_D reference
  dade_search_opts ref = base;
  ref.mode = DADE_MODE_FULL_D;
  ref.stats = nullptr;
  ref.record_times = 0;
  int rc = dade_search(ix, Q, nq, k, nprobe, k_per_query, nprobe_per_query, &ref, B.ids[0], B.d2[0], stream);
  if (rc) return rc;
  std::vector<int64_t> ref_ids(size_t(nq) * k), got(size_t(nq) * k);
  HIPC(hipMemcpyAsync(ref_ids.data(), B.ids[0], sizeof(int64_t) * ref_ids.size(), hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));

  std::vector<dade_tune_result> tried;
  // One candidate: a search for its results, `reps` timed searches, its agreement.
  auto run = [&](const dade_search_opts& o, dade_tune_result& res) -> int {
    int r = dade_search(ix, Q, nq, k, nprobe, k_per_query, nprobe_per_query, &o, B.ids[1], B.d2[1], stream);
    if (r) return r;
    HIPC(hipMemcpyAsync(got.data(), B.ids[1], sizeof(int64_t) * got.size(), hipMemcpyDeviceToHost, s));
    HIPC(hipEventRecord(B.ev[0], s));
    for (int i = 0; i < reps; ++i)
      if ((r = dade_search(ix, Q, nq, k, nprobe, k_per_query, nprobe_per_query, &o, B.ids[1], B.d2[1], stream)))
        return r;
    HIPC(hipEventRecord(B.ev[1], s));
    HIPC(hipEventSynchronize(B.ev[1]));
    float ms = 0.f;
    HIPC(hipEventElapsedTime(&ms, B.ev[0], B.ev[1]));
    double agree = 0.0;
    std::unordered_set<int64_t> want;
    for (int64_t q = 0; q < nq; ++q) {
      want.clear();
      for (int j = 0; j < kq[size_t(q)]; ++j)
        if (ref_ids[size_t(q) * k + j] >= 0) want.insert(ref_ids[size_t(q) * k + j]);
      if (want.empty()) {
        agree += 1.0;
        continue;
      }
      int hit = 0;
      for (int j = 0; j < kq[size_t(q)]; ++j) hit += want.count(got[size_t(q) * k + j]) ? 1 : 0;
      agree += double(hit) / double(want.size());
    }
    res.delta_d = o.delta_d;
    res.schedule = o.schedule;
    res.fill_min = o.fill_min;
    res.growth = o.growth;
    res.scan_blocks_per_cu = o.scan_blocks_per_cu;
    res.ms = ms / float(reps);
    res.agreement = float(agree / double(nq));
    return DADE_OK;
  };

  // 2. Delta_d x round shape
  std::vector<int> dds;
  for (int d : {8, 16, 32, 64, 128})
    if (d <= dim) dds.push_back(d);
  if (dds.empty()) dds.push_back(dim);
  const struct { int schedule, fill_min, growth; } shapes[] = {
      {DADE_SCHED_DOUBLING, 32, 0}, {DADE_SCHED_DOUBLING, 32, 16}, {DADE_SCHED_PER_RANK, 32, 16}};
  int best = -1;
  for (int d : dds)
    for (const auto& sh : shapes) {
      dade_search_opts o = base;
      o.delta_d = d;
      o.schedule = sh.schedule;
      o.fill_min = sh.fill_min;
      o.growth = sh.growth;
      o.scan_blocks_per_cu = 0;
      o.stats = nullptr;
      o.record_times = 0;
      dade_tune_result res{};
      if ((rc = run(o, res))) return rc;
      tried.push_back(res);
    }
  auto better = [&](const dade_tune_result& a, const dade_tune_result& b) {   // is a better than b
    const bool ok_a = a.agreement >= min_agreement, ok_b = b.agreement >= min_agreement;
    if (ok_a != ok_b) return ok_a;
    if (ok_a) return a.ms < b.ms;
    return a.agreement > b.agreement || (a.agreement == b.agreement && a.ms < b.ms);
  };
  for (int i = 0; i < int(tried.size()); ++i)
    if (best < 0 || better(tried[size_t(i)], tried[size_t(best)])) best = i;
  // 3. the launch shape of the winner (results do not change with it)
  const dade_tune_result win = tried[size_t(best)];
  for (int bpc : {1, 2}) {
    dade_search_opts o = base;
    o.delta_d = win.delta_d;
    o.schedule = win.schedule;
    o.fill_min = win.fill_min;
    o.growth = win.growth;
    o.scan_blocks_per_cu = bpc;
    o.stats = nullptr;
    o.record_times = 0;
    dade_tune_result res{};
    if ((rc = run(o, res))) return rc;
    tried.push_back(res);
    if (res.agreement == win.agreement && res.ms < tried[size_t(best)].ms) best = int(tried.size()) - 1;
  }
  const dade_tune_result& w = tried[size_t(best)];
  *opts = base;
  opts->delta_d = w.delta_d;
  opts->schedule = w.schedule;
  opts->fill_min = w.fill_min;
  opts->growth = w.growth;
  opts->scan_blocks_per_cu = w.scan_blocks_per_cu;
  if (results)
    for (size_t i = 0; i < tried.size() && i < size_t(DADE_TUNE_MAX); ++i) results[i] = tried[i];
  if (n_results) *n_results = int32_t(std::min<size_t>(tried.size(), DADE_TUNE_MAX));
  return DADE_OK;
}
