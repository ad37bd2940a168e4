// Serving loop: requests admitted into a device ring by a byte budget, batched as they arrive into
// dade_search launches on the compute stream, with their copies on two copy streams so that the
// next requests' queries go up and finished results come down while a launch runs.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <limits>
#include <string>
#include <thread>
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

struct Request {
  int64_t q0 = 0;          // its first query: row of Q and of the outputs
  int32_t nq = 0, k = 0, np = 0;
  int64_t slot = -1;       // its first ring slot
  int64_t span = 0;        // ring slots it holds: the unused end of the ring it skipped, then nq
  int32_t launched = 0, done = 0;
};

struct Piece {             // queries [off, off + n) of request `req`
  int64_t req;
  int32_t off, n;
};

struct Launch {
  int64_t slot = 0;        // first ring slot
  int32_t n = 0;
  std::vector<Piece> pieces;
  hipEvent_t up = nullptr, scanned = nullptr, down = nullptr;
};

// Everything one dade_serve call holds; the destructor waits for the streams, then frees.
struct Engine {
  dade_index* ix = nullptr;
  hipStream_t comp = nullptr, h2d = nullptr, d2h = nullptr;
  float* d_q = nullptr; int32_t* d_kn = nullptr; int64_t* d_ids = nullptr; float* d_d2 = nullptr;
  size_t b_q = 0, b_kn = 0, b_ids = 0, b_d2 = 0;
  float* h_q = nullptr; int32_t* h_kn = nullptr; int64_t* h_ids = nullptr; float* h_d2 = nullptr;
  std::vector<Launch> launches;

  ~Engine() {
    if (comp) (void)hipStreamSynchronize(comp);
    if (h2d) (void)hipStreamSynchronize(h2d);
    if (d2h) (void)hipStreamSynchronize(d2h);
    index_free(ix, d_q, b_q);
    index_free(ix, d_kn, b_kn);
    index_free(ix, d_ids, b_ids);
    index_free(ix, d_d2, b_d2);
    for (void* p : {static_cast<void*>(h_q), static_cast<void*>(h_kn), static_cast<void*>(h_ids),
                    static_cast<void*>(h_d2)})
      if (p) (void)hipHostFree(p);
    for (auto& L : launches)
      for (hipEvent_t e : {L.up, L.scanned, L.down})
        if (e) (void)hipEventDestroy(e);
    if (h2d) (void)hipStreamDestroy(h2d);
    if (d2h) (void)hipStreamDestroy(d2h);
  }
};

template <typename T>
int dev_array(Engine& E, T** p, size_t count, size_t& bytes) {
  void* v = nullptr;
  const int rc = index_alloc(E.ix, &v, count * sizeof(T));
  if (rc) return rc;
  *p = static_cast<T*>(v);
  bytes = count * sizeof(T);
  return DADE_OK;
}

template <typename T>
int host_array(T** p, size_t count) {
  void* v = nullptr;
  const hipError_t e = hipHostMalloc(&v, count * sizeof(T), hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    FAIL(DADE_ENOMEM, hip_msg(e, "hipHostMalloc"));
  }
  *p = static_cast<T*>(v);
  return DADE_OK;
}

}  // namespace

extern "C" int dade_serve(dade_index* ix, int64_t n_req, const double* arrival_s, const int32_t* req_queries,
                          const int32_t* req_k, const int32_t* req_nprobe, const float* Q,
                          const dade_serve_opts* opts, int64_t* out_ids, float* out_dist2,
                          double* out_latency_s, dade_serve_stats* stats, void* stream) {
  if (!ix) FAIL(DADE_EINVAL, "index is NULL");
  if (!opts) FAIL(DADE_EINVAL, "opts is NULL (k_max and nprobe_max are required)");
  if (n_req < 0) FAIL(DADE_EINVAL, "n_req must be >= 0");
  const int64_t budget = opts->budget_bytes > 0 ? opts->budget_bytes : (int64_t(512) << 20);
  const int32_t max_batch = opts->max_batch > 0 ? opts->max_batch : 1024;
  const int32_t max_inflight = opts->max_inflight > 0 ? opts->max_inflight : 2;
  const int32_t k_max = opts->k_max, np_max = opts->nprobe_max;
  if (opts->budget_bytes < 0 || opts->max_batch < 0 || opts->max_inflight < 0 || max_inflight > 16)
    FAIL(DADE_EINVAL, "budget_bytes, max_batch must be >= 0 and max_inflight in [0, 16]");
  if (k_max < 1 || k_max > kMaxK) FAIL(DADE_EINVAL, "k_max must be in [1, 128]");
  if (np_max < 1) FAIL(DADE_EINVAL, "nprobe_max must be >= 1");
  dade_search_opts so = opts->search;
  so.stats = nullptr;
  so.record_times = 0;
  so.use_graph = 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // options and index state, as dade_search checks them (a search of no queries)
  int rc = dade_search(ix, nullptr, 0, k_max, np_max, nullptr, nullptr, &so, nullptr, nullptr, stream);
  if (rc) return rc;
  if (stats) *stats = dade_serve_stats{};
  if (n_req == 0) return DADE_OK;
  if (!arrival_s || !req_queries || !req_k || !req_nprobe || !Q || !out_ids || !out_dist2)
    FAIL(DADE_EINVAL, "arrival_s, req_queries, req_k, req_nprobe, Q, out_ids and out_dist2 are required");
  std::vector<Request> R(static_cast<size_t>(n_req));
  int64_t total = 0;
  for (int64_t i = 0; i < n_req; ++i) {
    if (!(arrival_s[i] >= 0.0) || !std::isfinite(arrival_s[i]) || (i > 0 && arrival_s[i] < arrival_s[i - 1]))
      FAIL(DADE_EINVAL, "arrival_s must be finite, >= 0 and non-decreasing (request " + std::to_string(i) + ")");
    if (req_queries[i] < 1) FAIL(DADE_EINVAL, "request " + std::to_string(i) + " has no query");
    if (req_k[i] < 1 || req_k[i] > k_max) FAIL(DADE_EINVAL, "request " + std::to_string(i) + ": K not in [1, k_max]");
    if (req_nprobe[i] < 1 || req_nprobe[i] > np_max)
      FAIL(DADE_EINVAL, "request " + std::to_string(i) + ": nprobe not in [1, nprobe_max]");
    R[i].q0 = total;
    R[i].nq = req_queries[i];
    R[i].k = req_k[i];
    R[i].np = req_nprobe[i];
    total += req_queries[i];
  }
  if (total >= (int64_t(1) << 31)) FAIL(DADE_EINVAL, "too many queries (2^31 or more)");
  const int dim = index_dim(ix);
  // queries in pinned host memory are copied to the device from where they are; others are
  // staged in the pinned mirror of the ring first
  bool q_pinned = false;
  {
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, Q) == hipSuccess)
      q_pinned = attr.type == hipMemoryTypeHost;
    else
      (void)hipGetLastError();
  }

  Engine E;
  E.ix = ix;
  E.comp = s;
  // the search workspace for the largest launch, sized now so that no launch synchronises
  int64_t ws = 0;
  if ((rc = index_prepare_search(ix, std::min<int64_t>(max_batch, total), k_max, np_max, so, s, &ws))) return rc;
  // the ring: one slot per query (query row, K and nprobe, k_max results), from what is left
  const int64_t slot_bytes = int64_t(dim) * 4 + 8 + int64_t(k_max) * 12;
  if (budget - ws < slot_bytes)
    FAIL(DADE_ENOMEM, "budget_bytes (" + std::to_string(budget) + ") leaves no ring slot after the search workspace (" +
                          std::to_string(ws) + " bytes)");
  const int64_t C = std::min<int64_t>((budget - ws) / slot_bytes, total);
  if ((rc = dev_array(E, &E.d_q, size_t(C) * dim, E.b_q)) || (rc = dev_array(E, &E.d_kn, size_t(C) * 2, E.b_kn)) ||
      (rc = dev_array(E, &E.d_ids, size_t(C) * k_max, E.b_ids)) ||
      (rc = dev_array(E, &E.d_d2, size_t(C) * k_max, E.b_d2)))
    return rc;
  if ((!q_pinned && (rc = host_array(&E.h_q, size_t(C) * dim))) || (rc = host_array(&E.h_kn, size_t(C) * 2)) ||
      (rc = host_array(&E.h_ids, size_t(C) * k_max)) || (rc = host_array(&E.h_d2, size_t(C) * k_max)))
    return rc;
  HIPC(hipStreamCreateWithFlags(&E.h2d, hipStreamNonBlocking));
  HIPC(hipStreamCreateWithFlags(&E.d2h, hipStreamNonBlocking));
  E.launches.resize(size_t(max_inflight));
  for (auto& L : E.launches) {
    HIPC(hipEventCreateWithFlags(&L.up, hipEventDisableTiming));
    HIPC(hipEventCreateWithFlags(&L.scanned, hipEventDisableTiming));
    HIPC(hipEventCreateWithFlags(&L.down, hipEventDisableTiming));
  }
  // per-slot K in the ring's first C ints, nprobe in the next C
  int32_t* const d_k = E.d_kn;
  int32_t* const d_np = E.d_kn + C;
  dade_serve_stats st{};
  st.ring_slots = C;
  st.workspace_bytes = ws;
  const float inf = std::numeric_limits<float>::infinity();

  const auto t0 = std::chrono::steady_clock::now();
  auto now = [&] { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
  std::deque<int64_t> admitted;     // admitted and not complete, in arrival order
  int64_t first_unlaunched = 0;     // index into `admitted` of the first request with queries to launch
  std::deque<int> inflight;         // launch records on the device, oldest first
  std::vector<int> idle;
  for (int i = max_inflight - 1; i >= 0; --i) idle.push_back(i);
  int64_t next = 0, completed = 0, head = 0, tail = 0, unlaunched = 0;
  std::vector<char> waited(static_cast<size_t>(n_req), 0);

  while (completed < n_req) {
    bool progress = false;
    // 1. launches whose results are on the host: hand them out, complete requests, free slots
    while (!inflight.empty()) {
      Launch& L = E.launches[size_t(inflight.front())];
      const hipError_t e = hipEventQuery(L.down);
      if (e == hipErrorNotReady) break;
      if (e != hipSuccess) FAIL(DADE_EDEVICE, hip_msg(e, "serving launch"));
      const double t = now();
      progress = true;
      for (const Piece& pc : L.pieces) {
        Request& q = R[size_t(pc.req)];
        const int64_t src = q.slot + pc.off, dst = q.q0 + pc.off;
        std::memcpy(out_ids + dst * k_max, E.h_ids + src * k_max, sizeof(int64_t) * size_t(pc.n) * k_max);
        std::memcpy(out_dist2 + dst * k_max, E.h_d2 + src * k_max, sizeof(float) * size_t(pc.n) * k_max);
        q.done += pc.n;
        if (q.done == q.nq) {
          if (out_latency_s) out_latency_s[pc.req] = t - arrival_s[pc.req];
          ++completed;
          ++st.served_requests;
          st.served_queries += q.nq;
        }
      }
      // launches finish in order, so completed requests leave the ring from its oldest end
      while (!admitted.empty() && R[size_t(admitted.front())].done == R[size_t(admitted.front())].nq) {
        tail += R[size_t(admitted.front())].span;
        admitted.pop_front();
        --first_unlaunched;
      }
      idle.push_back(inflight.front());
      inflight.pop_front();
      st.retire_s += now() - t;
    }
    // 2. admit the requests that have arrived, in order, while the ring has room; staging stops
    // once the admitted queries not yet launched fill every launch record (the rest is admitted
    // as launches go out, so a burst of arrivals does not delay the first launch)
    const double tn = now();
    while (next < n_req && arrival_s[next] <= tn && unlaunched < int64_t(max_batch) * max_inflight) {
      Request& q = R[size_t(next)];
      if (q.nq > C) {   // can never fit: rejected
        for (int64_t j = q.q0 * k_max; j < (q.q0 + q.nq) * k_max; ++j) {
          out_ids[j] = -1;
          out_dist2[j] = inf;
        }
        if (out_latency_s) out_latency_s[next] = -1.0;
        ++completed;
        ++st.rejected_requests;
        ++next;
        progress = true;
        continue;
      }
      if (head == tail) head = tail = 0;   // an empty ring starts over at slot 0
      const int64_t pos = head % C;
      const int64_t pad = pos + q.nq > C ? C - pos : 0;   // a request's slots never wrap
      if (head - tail + pad + q.nq > C) {
        if (!waited[size_t(next)]) {
          waited[size_t(next)] = 1;
          ++st.waited_requests;
        }
        break;
      }
      const double t = now();
      q.slot = pad ? 0 : pos;
      q.span = pad + q.nq;
      head += q.span;
      st.peak_slots = std::max(st.peak_slots, head - tail);
      // staged in the pinned mirror of its slots (their last copies and launches have finished);
      // the copy to the device goes with the launch that takes them
      if (!q_pinned) std::memcpy(E.h_q + q.slot * dim, Q + q.q0 * dim, sizeof(float) * size_t(q.nq) * dim);
      std::fill(E.h_kn + q.slot, E.h_kn + q.slot + q.nq, q.k);
      std::fill(E.h_kn + C + q.slot, E.h_kn + C + q.slot + q.nq, q.np);
      st.stage_s += now() - t;
      admitted.push_back(next);
      unlaunched += q.nq;
      ++next;
      progress = true;
    }
    // 3. launch admitted queries while fewer than max_inflight launches are on the device
    while (!idle.empty() && first_unlaunched < int64_t(admitted.size())) {
      const double t = now();
      const int li = idle.back();
      Launch& L = E.launches[size_t(li)];
      L.pieces.clear();
      const Request& f = R[size_t(admitted[size_t(first_unlaunched)])];
      L.slot = f.slot + f.launched;
      L.n = 0;
      int32_t np_batch = 1;
      while (L.n < max_batch && first_unlaunched < int64_t(admitted.size())) {
        const int64_t r = admitted[size_t(first_unlaunched)];
        Request& q = R[size_t(r)];
        if (q.slot + q.launched != L.slot + L.n) break;   // not contiguous (the ring wrapped)
        const int32_t take = std::min(q.nq - q.launched, max_batch - L.n);
        L.pieces.push_back(Piece{r, q.launched, take});
        q.launched += take;
        L.n += take;
        unlaunched -= take;
        np_batch = std::max(np_batch, q.np);
        if (q.launched == q.nq) ++first_unlaunched;
      }
      // the launch's slots go up on the copy stream (while earlier launches run), the scan waits
      // for them, then the results come down on the other copy stream
      if (!q_pinned) {
        HIPC(hipMemcpyAsync(E.d_q + L.slot * dim, E.h_q + L.slot * dim, sizeof(float) * size_t(L.n) * dim,
                            hipMemcpyHostToDevice, E.h2d));
      } else {   // one copy per run of pieces that are consecutive rows of Q
        int64_t row = -1, slot = L.slot, n = 0;
        for (const Piece& pc : L.pieces) {
          const int64_t r0 = R[size_t(pc.req)].q0 + pc.off;
          if (n > 0 && r0 != row + n) {
            HIPC(hipMemcpyAsync(E.d_q + slot * dim, Q + row * dim, sizeof(float) * size_t(n) * dim,
                                hipMemcpyHostToDevice, E.h2d));
            slot += n;
            n = 0;
          }
          if (n == 0) row = r0;
          n += pc.n;
        }
        HIPC(hipMemcpyAsync(E.d_q + slot * dim, Q + row * dim, sizeof(float) * size_t(n) * dim, hipMemcpyHostToDevice,
                            E.h2d));
      }
      HIPC(hipMemcpyAsync(d_k + L.slot, E.h_kn + L.slot, sizeof(int32_t) * size_t(L.n), hipMemcpyHostToDevice, E.h2d));
      HIPC(hipMemcpyAsync(d_np + L.slot, E.h_kn + C + L.slot, sizeof(int32_t) * size_t(L.n), hipMemcpyHostToDevice,
                          E.h2d));
      HIPC(hipEventRecord(L.up, E.h2d));
      HIPC(hipStreamWaitEvent(s, L.up, 0));
      rc = dade_search(ix, E.d_q + L.slot * dim, L.n, k_max, np_batch, d_k + L.slot, d_np + L.slot, &so,
                       E.d_ids + L.slot * k_max, E.d_d2 + L.slot * k_max, stream);
      if (rc) return rc;
      HIPC(hipEventRecord(L.scanned, s));
      HIPC(hipStreamWaitEvent(E.d2h, L.scanned, 0));
      HIPC(hipMemcpyAsync(E.h_ids + L.slot * k_max, E.d_ids + L.slot * k_max, sizeof(int64_t) * size_t(L.n) * k_max,
                          hipMemcpyDeviceToHost, E.d2h));
      HIPC(hipMemcpyAsync(E.h_d2 + L.slot * k_max, E.d_d2 + L.slot * k_max, sizeof(float) * size_t(L.n) * k_max,
                          hipMemcpyDeviceToHost, E.d2h));
      HIPC(hipEventRecord(L.down, E.d2h));
      idle.pop_back();
      inflight.push_back(li);
      ++st.launches;
      st.launch_s += now() - t;
      progress = true;
    }
    if (!progress) std::this_thread::yield();   // waiting for an arrival or a launch
  }
  st.wall_s = now();
  if (stats) *stats = st;
  return DADE_OK;
}
