// C ABI of the DADE-IVF engine: index lifecycle, offline build (k-means lists, FP64 transform,
// eps_d calibration) and the search pipeline (query rotation -> probe selection -> list scan).
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <cstdlib>
#include <limits>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "dade.h"
#include "kernels.h"

using namespace dade;

namespace {
thread_local std::string g_err;

// splitmix64 (Steele, Lea and Flood, OOPSLA 2014), used only when the caller passes no
// seed rows / calibration pairs.
struct SplitMix64 {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  uint64_t below(uint64_t n) { return static_cast<uint64_t>((static_cast<unsigned __int128>(next()) * n) >> 64); }
};

}  // namespace

namespace dade {
void set_error(const std::string& msg) { g_err = msg; }
std::string hip_msg(hipError_t e, const char* what) {
  return std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
}
}  // namespace dade

#define FAIL(code, msg)      \
  do {                       \
    dade::set_error(msg);    \
    return (code);           \
  } while (0)

#define HIPC(expr)                                             \
  do {                                                         \
    hipError_t e_ = (expr);                                    \
    if (e_ != hipSuccess) FAIL(DADE_EDEVICE, hip_msg(e_, #expr)); \
  } while (0)

struct dade_index {
  int device = 0;
  int64_t n = 0;
  int dim = 0, dp = 0, nlist = 0, store = DADE_F32, state = 0;
  int64_t budget = 0, held = 0;
  // device buffers
  float* X = nullptr;          // [n x dp] original vectors (zero padded)
  float* cent = nullptr;       // [nlist x dp] centroids, original basis
  int64_t* d_off = nullptr;    // [nlist + 1]
  int32_t* d_ids = nullptr;    // [n] packed position -> row id
  int64_t* d_pos = nullptr;    // [n] row id -> packed position
  float* d_B = nullptr;        // [dp x ldB] FP32 [W | (C - mu)^T] (zero padded)
  int ldB = 0;                 // dp + nlist rounded up to a multiple of 4 (float4 rows)
  float* d_mu = nullptr;       // [dp]
  float* d_cent_norm = nullptr;// [nlist] ||c - mu||^2
  float* d_cx = nullptr;       // [nlist x dp] c - mu (FP32), the probe refinement's exact rows
  float* d_cnorm = nullptr;    // [nlist] upper bounds of ||c - mu||
  uint16_t* d_cb = nullptr;    // bf16 c - mu in MFMA fragment order (probe_centroid_frags)
  void* d_store = nullptr;     // rotated coordinates in list order, head/tail layout (stored_index)
  float* d_T = nullptr;        // [dim]
  // host artifacts
  std::vector<double> W, mu, lam, T, cent_h;
  double delta = 0.0;
  std::vector<int64_t> off_h, ids_h;
  std::vector<int64_t> sizes_desc;   // list sizes, largest first (round capacities)
  // search workspace (grown on demand, each with its element count)
  float* w_qpad = nullptr; float* w_qrot = nullptr; float* w_pd = nullptr;
  void* w_a1 = nullptr;        // [probe_a_bytes(w_nq, dp)] bf16 queries of the probe selection
  int32_t* w_probes = nullptr;
  int64_t w_nq = 0, w_np = 0;
  unsigned long long* w_topk = nullptr; int64_t w_topk_n = 0;
  unsigned long long* w_keyr = nullptr; int64_t w_keyr_n = 0;
  float* w_r2 = nullptr; int64_t w_r2_n = 0;
  int* w_qint = nullptr; int64_t w_qint_n = 0;      // q_topn, q_kc, q_rounds
  unsigned long long* w_kb = nullptr; int64_t w_kb_n = 0;
  int4* w_items = nullptr; int64_t w_items_n = 0;   // per group and round
  int* w_counter = nullptr; int64_t w_counter_n = 0;  // per group: n_items[rounds]
  int* w_counts = nullptr; int64_t w_counts_n = 0;    // per round and query: item counts / offsets
  int* w_flags = nullptr;                             // sticky: a scan capacity was exceeded
  int scan_occ[3][2][2] = {};                        // resident scan workgroups per CU
  hipEvent_t ev[4] = {};
  bool ev_made = false, ev_used = false;
  // per-kernel events of a timed search, one set per pass: plan (before, after), then per round (before the DCO
  // kernel, between it and the merge, after the merge)
  std::vector<hipEvent_t> kev;
  int kev_rounds = 0, kev_passes = 0;
  int cus = 256;
  hipStream_t cap = nullptr;   // origin stream of graph captures (the caller's may be the null stream)
  hipStream_t side = nullptr;  // the query rotation, concurrent with the probe selection
  hipEvent_t fork = nullptr, join = nullptr;
  // the last captured round-launch sequence and the argument bytes it was captured with
  hipGraphExec_t graph_exec = nullptr;
  hipEvent_t graph_done = nullptr;     // recorded after every launch of the captured sequence
  const float* last_q = nullptr;   // the query buffer of the last search
  std::vector<unsigned char> graph_key;
  // kNN graph (dade_graph_build)
  int32_t* d_nbr = nullptr;    // [n x graph_degree] out-neighbour positions, by position
  int32_t* d_entry = nullptr;  // [nlist x 2] entry positions per list: medoid, farthest from it
  int graph_degree = 0;         // row width of a usable graph (0: none)
  int graph_width = 0;          // row width of d_nbr's allocation
  std::vector<int64_t> pos_h;   // row id -> packed position (host)
  int64_t d_pos_h(int64_t row) const { return pos_h[size_t(row)]; }

  std::vector<void*> owned;
};

namespace {

size_t dtype_size(int dt) { return dt == DADE_F32 ? 4 : 2; }

// Failure injection for tests of error paths: with DADE_FAIL_ALLOC_AFTER=N in the environment,
// every device allocation after the first N made since the variable took its current value fails
// with DADE_ENOMEM before hipMalloc is called.
bool refuse_allocation() {
  static std::mutex mu;
  static std::string last;
  static long count = 0;
  const char* env = std::getenv("DADE_FAIL_ALLOC_AFTER");
  std::lock_guard<std::mutex> lock(mu);
  if (!env) {
    last.clear();
    return false;
  }
  if (last != env) {
    last = env;
    count = 0;
  }
  return count++ >= std::atol(env);
}

int dev_alloc(dade_index* ix, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  if (refuse_allocation()) FAIL(DADE_ENOMEM, "allocation refused (DADE_FAIL_ALLOC_AFTER)");
  if (ix->budget > 0 && ix->held + int64_t(bytes) > ix->budget)
    FAIL(DADE_ENOMEM, "HBM budget exceeded: need " + std::to_string(ix->held + bytes) + " bytes, budget " +
                          std::to_string(ix->budget));
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    FAIL(DADE_ENOMEM, hip_msg(e, "hipMalloc"));
  }
  ix->held += int64_t(bytes);
  ix->owned.push_back(*p);
  return DADE_OK;
}

template <typename T>
int alloc_t(dade_index* ix, T** p, size_t count) {
  void* v = nullptr;
  int rc = dev_alloc(ix, &v, count * sizeof(T));
  *p = static_cast<T*>(v);
  return rc;
}

void dev_free(dade_index* ix, void* p, size_t bytes) {
  if (!p) return;
  auto it = std::find(ix->owned.begin(), ix->owned.end(), p);
  if (it != ix->owned.end()) ix->owned.erase(it);
  (void)hipFree(p);
  ix->held -= int64_t(bytes == 0 ? 16 : bytes);
}

// Make *p hold at least `need` elements (contents are not kept).
template <typename T>
int grow(dade_index* ix, T** p, int64_t& have, int64_t need, hipStream_t s) {
  if (need <= have && *p) return DADE_OK;
  HIPC(hipStreamSynchronize(s));
  dev_free(ix, *p, sizeof(T) * size_t(have));
  *p = nullptr;
  have = 0;
  const int rc = alloc_t(ix, p, size_t(need));
  if (rc) return rc;
  have = need;
  return DADE_OK;
}

int check_device_pointer(const void* p, const char* name) {
  if (!p) FAIL(DADE_EINVAL, std::string(name) + " is NULL");
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    FAIL(DADE_EINVAL, std::string(name) + " is not a device pointer");
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
    FAIL(DADE_EINVAL, std::string(name) + " is not device memory");
  return DADE_OK;
}

// Common index creation: copy X (padded) and record sizes.
int make_index(const float* X, int64_t n, int32_t dim, int32_t nlist, const dade_build_opts* opts,
               hipStream_t s, dade_index** out) {
  if (!out) FAIL(DADE_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 1 || n >= (int64_t(1) << 31)) FAIL(DADE_EINVAL, "n must be in [1, 2^31)");
  if (dim < 1 || dim > 4096) FAIL(DADE_EINVAL, "dim must be in [1, 4096]");
  if (nlist < 1 || nlist > n || nlist > 8192) FAIL(DADE_EINVAL, "nlist must be in [1, min(n, 8192)]");
  int rc = check_device_pointer(X, "X");
  if (rc) return rc;
  int store = opts ? opts->store_dtype : DADE_F32;
  if (store != DADE_F32 && store != DADE_BF16 && store != DADE_F16) FAIL(DADE_EINVAL, "bad store_dtype");
  auto* ix = new dade_index();
  HIPC(hipGetDevice(&ix->device));
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ix->device) == hipSuccess && cus > 0)
    ix->cus = cus;
  ix->n = n; ix->dim = dim; ix->dp = pad_dim(dim); ix->nlist = nlist; ix->store = store;
  ix->budget = opts ? opts->hbm_budget_bytes : 0;
  if ((rc = alloc_t(ix, &ix->X, size_t(n) * ix->dp))) { dade_destroy(ix); return rc; }
  if ((rc = alloc_t(ix, &ix->w_flags, 1))) { dade_destroy(ix); return rc; }
  if (launch_fill_i32(ix->w_flags, 1, 0, s) != hipSuccess) { dade_destroy(ix); FAIL(DADE_EDEVICE, "clear flags"); }
  hipError_t e = launch_pad_rows(X, n, dim, dim, ix->X, ix->dp, s);
  if (e != hipSuccess) { dade_destroy(ix); FAIL(DADE_EDEVICE, hip_msg(e, "pad X")); }
  *out = ix;
  return DADE_OK;
}

// Lists from row labels: stable counting sort (ascending row id inside a list).
int set_lists(dade_index* ix, const std::vector<int32_t>& lab, hipStream_t s) {
  const int64_t n = ix->n;
  ix->off_h.assign(ix->nlist + 1, 0);
  for (int64_t i = 0; i < n; ++i) ix->off_h[lab[i] + 1]++;
  for (int l = 0; l < ix->nlist; ++l) ix->off_h[l + 1] += ix->off_h[l];
  ix->sizes_desc.resize(ix->nlist);
  for (int l = 0; l < ix->nlist; ++l) ix->sizes_desc[l] = ix->off_h[l + 1] - ix->off_h[l];
  std::sort(ix->sizes_desc.begin(), ix->sizes_desc.end(), std::greater<int64_t>());
  ix->ids_h.assign(n, 0);
  std::vector<int64_t> fill(ix->off_h.begin(), ix->off_h.end() - 1);
  for (int64_t i = 0; i < n; ++i) ix->ids_h[fill[lab[i]]++] = i;
  std::vector<int32_t> ids32(n);
  std::vector<int64_t> pos(n);
  for (int64_t p = 0; p < n; ++p) { ids32[p] = int32_t(ix->ids_h[p]); pos[ix->ids_h[p]] = p; }
  ix->pos_h = pos;
  int rc;
  if (!ix->d_off && (rc = alloc_t(ix, &ix->d_off, ix->nlist + 1))) return rc;
  if (!ix->d_ids && (rc = alloc_t(ix, &ix->d_ids, n))) return rc;
  if (!ix->d_pos && (rc = alloc_t(ix, &ix->d_pos, n))) return rc;
  HIPC(hipMemcpyAsync(ix->d_off, ix->off_h.data(), sizeof(int64_t) * (ix->nlist + 1), hipMemcpyHostToDevice, s));
  HIPC(hipMemcpyAsync(ix->d_ids, ids32.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
  HIPC(hipMemcpyAsync(ix->d_pos, pos.data(), sizeof(int64_t) * n, hipMemcpyHostToDevice, s));
  HIPC(hipStreamSynchronize(s));
  return DADE_OK;
}

// Store [W | (C - mu)^T] (host FP64 -> FP32) and ||c - mu||^2 on the device, pack the store.
// The query GEMM multiplies (q - mu) by this matrix: its first dp columns give q' = W^T (q - mu),
// the others (q - mu).(c - mu); W is orthogonal, so ||q' - c'||^2 = ||q - c||^2 (Lemma 1).
int apply_transform(dade_index* ix, hipStream_t s) {
  const int dim = ix->dim, dp = ix->dp, nl = ix->nlist;
  const int64_t ldb = (int64_t(dp) + nl + 3) / 4 * 4;   // the GEMM reads rows as float4
  ix->ldB = int(ldb);
  int rc;
  std::vector<float> Bf(size_t(dp) * ldb, 0.f), muf(dp, 0.f), cn(nl, 0.f);
  for (int i = 0; i < dim; ++i)
    for (int k = 0; k < dim; ++k) Bf[size_t(i) * ldb + k] = float(ix->W[size_t(i) * dim + k]);
  for (int l = 0; l < nl; ++l) {
    double nrm = 0.0;
    for (int i = 0; i < dim; ++i) {
      const double v = ix->cent_h[size_t(l) * dim + i] - ix->mu[i];
      Bf[size_t(i) * ldb + dp + l] = float(v);
      nrm += v * v;
    }
    cn[l] = float(nrm);
  }
  for (int i = 0; i < dim; ++i) muf[i] = float(ix->mu[i]);
  // probe selection: c - mu as FP32 rows (the same values as B's columns), upper bounds of their
  // norms (FP64 over those values, rounded up), and their bf16 fragments
  std::vector<float> cx(size_t(nl) * dp, 0.f), cnorm(nl, 0.f);
  for (int l = 0; l < nl; ++l) {
    double ss = 0.0;
    for (int i = 0; i < dim; ++i) {
      const float v = Bf[size_t(i) * ldb + dp + l];
      cx[size_t(l) * dp + i] = v;
      ss += double(v) * double(v);
    }
    const double up = std::sqrt(ss) * (1.0 + 0x1p-40);
    float f = float(up);
    if (double(f) < up) f = std::nextafter(f, std::numeric_limits<float>::infinity());
    cnorm[l] = f;
  }
  std::vector<uint16_t> cb(probe_centroid_frag_count(nl, dp));
  probe_centroid_frags(cx.data(), nl, dp, cb.data());
  if (!ix->d_B && (rc = alloc_t(ix, &ix->d_B, Bf.size()))) return rc;
  if (!ix->d_mu && (rc = alloc_t(ix, &ix->d_mu, dp))) return rc;
  if (!ix->d_cent_norm && (rc = alloc_t(ix, &ix->d_cent_norm, nl))) return rc;
  if (!ix->d_cx && (rc = alloc_t(ix, &ix->d_cx, cx.size()))) return rc;
  if (!ix->d_cnorm && (rc = alloc_t(ix, &ix->d_cnorm, nl))) return rc;
  if (!ix->d_cb && (rc = alloc_t(ix, &ix->d_cb, cb.size()))) return rc;
  HIPC(hipMemcpyAsync(ix->d_B, Bf.data(), sizeof(float) * Bf.size(), hipMemcpyHostToDevice, s));
  HIPC(hipMemcpyAsync(ix->d_mu, muf.data(), sizeof(float) * dp, hipMemcpyHostToDevice, s));
  HIPC(hipMemcpyAsync(ix->d_cent_norm, cn.data(), sizeof(float) * nl, hipMemcpyHostToDevice, s));
  HIPC(hipMemcpyAsync(ix->d_cx, cx.data(), sizeof(float) * cx.size(), hipMemcpyHostToDevice, s));
  HIPC(hipMemcpyAsync(ix->d_cnorm, cnorm.data(), sizeof(float) * nl, hipMemcpyHostToDevice, s));
  HIPC(hipMemcpyAsync(ix->d_cb, cb.data(), sizeof(uint16_t) * cb.size(), hipMemcpyHostToDevice, s));

  // packed store: row p = W^T (X[ids[p]] - mu), in list order
  if (!ix->d_store && (rc = dev_alloc(ix, &ix->d_store, size_t(ix->n) * dp * dtype_size(ix->store)))) return rc;
  GemmArgs g;
  g.M = int(ix->n); g.N = dp; g.K = dp;
  g.A = ix->X; g.lda = dp; g.a_rows = ix->d_ids; g.a_shift = ix->d_mu;
  g.B = ix->d_B; g.ldb = int(ldb); g.C = ix->d_store; g.ldc = dp; g.split_rows = ix->n;
  const GemmEpilogue epi = ix->store == DADE_F32 ? kEpiPackF32 : (ix->store == DADE_BF16 ? kEpiPackBF16 : kEpiPackF16);
  HIPC(launch_gemm(g, epi, s));
  HIPC(hipStreamSynchronize(s));
  return DADE_OK;
}

int upload_T(dade_index* ix, hipStream_t s) {
  int rc;
  std::vector<float> Tf(ix->dim);
  for (int d = 0; d < ix->dim; ++d) Tf[d] = float(ix->T[d]);
  if (!ix->d_T && (rc = alloc_t(ix, &ix->d_T, ix->dim))) return rc;
  HIPC(hipMemcpyAsync(ix->d_T, Tf.data(), sizeof(float) * ix->dim, hipMemcpyHostToDevice, s));
  HIPC(hipStreamSynchronize(s));
  return DADE_OK;
}

// Query-side workspace: padded and rotated queries, centroid distances and probe lists of nq
// queries with npm probes (grown on demand; growing synchronises `s`).
int grow_query_workspace(dade_index* ix, int64_t nq, int64_t npm, hipStream_t s) {
  int rc;
  const int dp = ix->dp, nl = ix->nlist;
  if (nq > ix->w_nq || npm > ix->w_np) {
    const int64_t new_nq = std::max(nq, ix->w_nq), new_np = std::max<int64_t>(npm, ix->w_np);
    HIPC(hipStreamSynchronize(s));
    dev_free(ix, ix->w_qpad, sizeof(float) * ix->w_nq * dp);
    dev_free(ix, ix->w_qrot, sizeof(float) * ix->w_nq * dp);
    dev_free(ix, ix->w_pd, sizeof(float) * ix->w_nq * nl);
    dev_free(ix, ix->w_probes, sizeof(int32_t) * ix->w_nq * ix->w_np);
    dev_free(ix, ix->w_a1, probe_a_bytes(int(ix->w_nq), dp));
    ix->w_qpad = ix->w_qrot = ix->w_pd = nullptr;
    ix->w_probes = nullptr;
    ix->w_a1 = nullptr;
    ix->w_nq = ix->w_np = 0;
    if ((rc = alloc_t(ix, &ix->w_qpad, size_t(new_nq) * dp)) || (rc = alloc_t(ix, &ix->w_qrot, size_t(new_nq) * dp)) ||
        (rc = alloc_t(ix, &ix->w_pd, size_t(new_nq) * nl)) || (rc = alloc_t(ix, &ix->w_probes, size_t(new_nq) * new_np)) ||
        (rc = dev_alloc(ix, &ix->w_a1, probe_a_bytes(int(new_nq), dp)))) {
      // leave no part of the workspace behind (the next search grows it again)
      dev_free(ix, ix->w_qpad, sizeof(float) * new_nq * dp);
      dev_free(ix, ix->w_qrot, sizeof(float) * new_nq * dp);
      dev_free(ix, ix->w_pd, sizeof(float) * new_nq * nl);
      dev_free(ix, ix->w_probes, sizeof(int32_t) * new_nq * new_np);
      dev_free(ix, ix->w_a1, probe_a_bytes(int(new_nq), dp));
      ix->w_qpad = ix->w_qrot = ix->w_pd = nullptr;
      ix->w_probes = nullptr;
      ix->w_a1 = nullptr;
      return rc;
    }
    ix->w_nq = new_nq; ix->w_np = new_np;
  }
  return DADE_OK;
}

// Device bytes one pass of the list scan may hold in queued keys and work items (a batch that
// needs more runs in passes); a few percent of the device's HBM.
constexpr int64_t kPassWorkspaceBytes = int64_t(8) << 30;

// Sizes of one search's round workspace, from the list sizes, K, nprobe and the schedule.
struct SearchPlan {
  int npm = 0, widest = 1, rounds = 0;
  int64_t kb_cap = 0, first = 0, items_pq = 0;
  int64_t per_q = 0;   // round-workspace bytes per query of a pass
};

// Where one search's buffers live: the index's workspace (grown on demand) or a fixed region.
struct Workspace {
  float* qpad = nullptr;             // [nq x dp] padded queries (when not read in place)
  float* qrot = nullptr;             // [nq x dp] rotated queries
  float* pd = nullptr;               // [nq x nlist] centroid terms, or the probe selection's bounds
  int32_t* probes = nullptr;         // [nq x npm]
  void* a1 = nullptr;                // [probe_a_bytes(nq, dp)] bf16 queries of the probe selection
  unsigned long long* topk = nullptr;   // [chunk x k]
  unsigned long long* keyr = nullptr;   // [chunk]
  float* r2 = nullptr;               // [chunk]
  int* qint = nullptr;               // [chunk x 3]
  unsigned long long* kb = nullptr;  // [chunk x kb_cap]
  int4* items = nullptr;             // [rounds x chunk x items_pq]
  int* counter = nullptr;            // [rounds]
  int* counts = nullptr;             // [rounds x chunk]
  int64_t chunk = 0;                 // queries per pass of the list scan
};

// The plan of a search (k, nprobe: the largest per-query values); no device work.
SearchPlan plan_sizes(const dade_index* ix, int32_t k, int32_t nprobe, const dade_search_opts& o) {
  const int nl = ix->nlist;
  const int npm = std::min<int>(nprobe, nl);
  // the most candidates one round can hold (per-rank: one list; doubling: its widest round;
  // whole: every probed list)
  const std::vector<int64_t>& sizes = ix->sizes_desc;
  int widest = 1, rounds = npm + 1;
  if (o.schedule == DADE_SCHED_DOUBLING) {
    int b = 1, nb = 0;
    while (b < npm) { widest = std::max(widest, std::min(2 * b, npm) - b); b *= 2; ++nb; }
    rounds = nb + 2;
  } else if (o.schedule == DADE_SCHED_WHOLE) {
    widest = npm;
    rounds = 2;
  }
  int64_t kb_cap = 0, most = 0;   // most: the largest candidate count a query can have
  for (int i = 0; i < widest && i < nl; ++i) kb_cap += sizes[i];
  for (int i = 0; i < npm; ++i) most += sizes[i];
  const int64_t first = std::max<int64_t>(k, o.fill_min);
  kb_cap = std::max<int64_t>(kb_cap, std::min(first, most));
  // Rounds cut short by the growth cap: such a round at position p takes growth x p candidates,
  // so it needs more than (1 + growth) p of them and leaves the position at (1 + growth) p.
  // Every query's first round ends at p0 >= min(fill_min, most) or later, so its c-th capped
  // round needs p0 (1 + growth)^c < most.
  if (o.growth > 0)
    for (int64_t p = std::max<int64_t>(1, std::min<int64_t>(o.fill_min, most)) * (1 + o.growth); p < most;
         p *= 1 + o.growth)
      ++rounds;
  // work items of one query in one round: its segments cut at 16 candidates (whole-row rounds;
  // other rounds use 64)
  const int64_t items_pq = std::max<int64_t>((kb_cap + 15) / 16 + widest + 1, (first + 15) / 16 + npm);
  SearchPlan pl;
  pl.npm = npm; pl.widest = widest; pl.rounds = rounds;
  pl.kb_cap = kb_cap; pl.first = first; pl.items_pq = items_pq;
  pl.per_q = kb_cap * 8 + rounds * (items_pq * 16 + 4) + int64_t(k) * 8 + 48;
  return pl;
}

// The index's workspace for a search of nq queries under plan pl, grown on demand (growing
// synchronises `s`; a workspace already large enough is reused as is).
int grow_workspace(dade_index* ix, int64_t nq, int32_t k, const SearchPlan& pl, hipStream_t s, Workspace& ws) {
  int rc;
  // queries per pass: the round workspace stays under kPassWorkspaceBytes
  const int64_t chunk =
      std::max<int64_t>(1, std::min<int64_t>({nq, kPassWorkspaceBytes / pl.per_q, int64_t(kMaxPassQueries)}));
  if ((rc = grow_query_workspace(ix, nq, pl.npm, s))) return rc;
  if ((rc = grow(ix, &ix->w_topk, ix->w_topk_n, chunk * k, s)) || (rc = grow(ix, &ix->w_keyr, ix->w_keyr_n, chunk, s)) ||
      (rc = grow(ix, &ix->w_r2, ix->w_r2_n, chunk, s)) || (rc = grow(ix, &ix->w_qint, ix->w_qint_n, chunk * 3, s)) ||
      (rc = grow(ix, &ix->w_kb, ix->w_kb_n, chunk * pl.kb_cap, s)) ||
      (rc = grow(ix, &ix->w_items, ix->w_items_n, int64_t(pl.rounds) * chunk * pl.items_pq, s)) ||
      (rc = grow(ix, &ix->w_counter, ix->w_counter_n, pl.rounds, s)) ||
      (rc = grow(ix, &ix->w_counts, ix->w_counts_n, int64_t(pl.rounds) * chunk, s)))
    return rc;
  ws.qpad = ix->w_qpad; ws.qrot = ix->w_qrot; ws.pd = ix->w_pd; ws.probes = ix->w_probes; ws.a1 = ix->w_a1;
  ws.topk = ix->w_topk; ws.keyr = ix->w_keyr; ws.r2 = ix->w_r2; ws.qint = ix->w_qint;
  ws.kb = ix->w_kb; ws.items = ix->w_items; ws.counter = ix->w_counter; ws.counts = ix->w_counts;
  ws.chunk = chunk;
  return DADE_OK;
}

}  // namespace

// Hooks for the serving loop (serve.hip): device memory counted against the index's HBM budget,
// and the search workspace sized ahead of time for the largest batch.
namespace dade {
int index_alloc(dade_index* ix, void** p, size_t bytes) { return dev_alloc(ix, p, bytes); }
void index_free(dade_index* ix, void* p, size_t bytes) { dev_free(ix, p, bytes); }
int index_prepare_search(dade_index* ix, int64_t nq, int32_t k, int32_t nprobe, const dade_search_opts& o,
                         hipStream_t s, int64_t* workspace_bytes) {
  const SearchPlan pl = plan_sizes(ix, k, nprobe, o);
  Workspace ws;
  const int rc = grow_workspace(ix, nq, k, pl, s, ws);
  if (rc) return rc;
  const int64_t dp = ix->dp, nl = ix->nlist;
  *workspace_bytes = ix->w_nq * (2 * dp * 4 + nl * 4 + ix->w_np * 4) + int64_t(probe_a_bytes(int(ix->w_nq), int(dp))) +
                     ix->w_topk_n * 8 + ix->w_keyr_n * 8 +
                     ix->w_r2_n * 4 + ix->w_qint_n * 4 + ix->w_kb_n * 8 + ix->w_items_n * 16 + ix->w_counter_n * 4 +
                     ix->w_counts_n * 4;
  return DADE_OK;
}
int index_dim(const dade_index* ix) { return ix->dim; }
}  // namespace dade

// ------------------------------------------------------------------------------------------------
// Scratch of dade_search_noalloc: one array per device (the runtime places it when the library's
// code object is loaded on that device; it is held until the process ends).  Host code never uses
// its name as an address: each device's address is looked up once, with that device current, and
// kept in g_scratch_addr.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// The scratch array's device address on the current device `dev`.
int scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (dev < 0 || dev >= kMaxDevices) FAIL(DADE_EDEVICE, "device id out of range for the scratch table");
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      FAIL(DADE_EDEVICE, hip_msg(e, "hipGetSymbolAddress(scratch)"));
    }
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return DADE_OK;
}

constexpr size_t kScratchAlign = 256;
size_t align_up(size_t x) { return (x + kScratchAlign - 1) / kScratchAlign * kScratchAlign; }

// Bytes of scratch one slice of cn queries takes under plan pl (each region 256-byte aligned).
size_t slice_bytes(const dade_index* ix, const SearchPlan& pl, int32_t k, int64_t cn) {
  const size_t dp = size_t(ix->dp), nl = size_t(ix->nlist), c = size_t(cn);
  return align_up(c * dp * 4) * 2 + align_up(c * nl * 4) + align_up(c * size_t(pl.npm) * 4) +
         align_up(probe_a_bytes(int(cn), ix->dp)) +
         align_up(c * size_t(k) * 8) + align_up(c * 8) + align_up(c * 4) + align_up(c * 12) +
         align_up(c * size_t(pl.kb_cap) * 8) + align_up(size_t(pl.rounds) * c * size_t(pl.items_pq) * 16) +
         align_up(size_t(pl.rounds) * 4) + align_up(size_t(pl.rounds) * c * 4);
}

// A workspace for cn queries carved out of the scratch at `base` (slice_bytes(...) bytes).
Workspace carve(char* base, const dade_index* ix, const SearchPlan& pl, int32_t k, int64_t cn) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base + off;
    off += align_up(bytes);
    return p;
  };
  const size_t dp = size_t(ix->dp), nl = size_t(ix->nlist), c = size_t(cn);
  Workspace ws;
  ws.qpad = reinterpret_cast<float*>(take(c * dp * 4));
  ws.qrot = reinterpret_cast<float*>(take(c * dp * 4));
  ws.pd = reinterpret_cast<float*>(take(c * nl * 4));
  ws.probes = reinterpret_cast<int32_t*>(take(c * size_t(pl.npm) * 4));
  ws.a1 = take(probe_a_bytes(int(cn), ix->dp));
  ws.topk = reinterpret_cast<unsigned long long*>(take(c * size_t(k) * 8));
  ws.keyr = reinterpret_cast<unsigned long long*>(take(c * 8));
  ws.r2 = reinterpret_cast<float*>(take(c * 4));
  ws.qint = reinterpret_cast<int*>(take(c * 12));
  ws.kb = reinterpret_cast<unsigned long long*>(take(c * size_t(pl.kb_cap) * 8));
  ws.items = reinterpret_cast<int4*>(take(size_t(pl.rounds) * c * size_t(pl.items_pq) * 16));
  ws.counter = reinterpret_cast<int*>(take(size_t(pl.rounds) * 4));
  ws.counts = reinterpret_cast<int*>(take(size_t(pl.rounds) * c * 4));
  ws.chunk = cn;
  return ws;
}
}  // namespace

extern "C" {

const char* dade_last_error(void) { return g_err.c_str(); }

void dade_destroy(dade_index* ix) {
  if (!ix) return;
  (void)hipDeviceSynchronize();
  for (void* p : ix->owned) (void)hipFree(p);
  if (ix->graph_exec) (void)hipGraphExecDestroy(ix->graph_exec);
  if (ix->graph_done) (void)hipEventDestroy(ix->graph_done);
  if (ix->cap) (void)hipStreamDestroy(ix->cap);
  if (ix->side) (void)hipStreamDestroy(ix->side);
  if (ix->fork) (void)hipEventDestroy(ix->fork);
  if (ix->join) (void)hipEventDestroy(ix->join);
  for (hipEvent_t e : ix->kev) (void)hipEventDestroy(e);
  if (ix->ev_made)
    for (auto& e : ix->ev) (void)hipEventDestroy(e);
  delete ix;
}

int dade_index_info(const dade_index* ix, int64_t* n, int32_t* dim, int32_t* nlist,
                    int32_t* store_dtype, int32_t* state) {
  if (!ix) FAIL(DADE_EINVAL, "index is NULL");
  if (n) *n = ix->n;
  if (dim) *dim = ix->dim;
  if (nlist) *nlist = ix->nlist;
  if (store_dtype) *store_dtype = ix->store;
  if (state) *state = ix->state;
  return DADE_OK;
}

int dade_build_index(const float* X, int64_t n, int32_t dim, int32_t nlist,
                     const dade_build_opts* opts, void* stream, dade_index** out) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  dade_index* ix = nullptr;
  int rc = make_index(X, n, dim, nlist, opts, s, &ix);
  if (rc) return rc;
  const int dp = ix->dp;
  const int iters = (opts && opts->kmeans_iters > 0) ? opts->kmeans_iters : 10;
  // seed rows
  std::vector<int64_t> init(nlist);
  if (opts && opts->init_rows) {
    std::vector<char> seen(n, 0);
    for (int l = 0; l < nlist; ++l) {
      const int64_t r = opts->init_rows[l];
      if (r < 0 || r >= n || seen[r]) { dade_destroy(ix); FAIL(DADE_EINVAL, "init_rows must be distinct ids in [0, n)"); }
      seen[r] = 1;
      init[l] = r;
    }
  } else {  // Floyd's sampling of nlist distinct rows
    SplitMix64 rng{opts ? opts->seed : 0};
    std::vector<int64_t> chosen;
    std::vector<char> seen(n, 0);
    for (int64_t j = n - nlist; j < n; ++j) {
      int64_t t = int64_t(rng.below(uint64_t(j + 1)));
      if (seen[t]) t = j;
      seen[t] = 1;
      chosen.push_back(t);
    }
    std::sort(chosen.begin(), chosen.end());
    init = chosen;
  }
  int64_t* d_init = nullptr;
  unsigned long long* best = nullptr;
  double* sums = nullptr;
  int* counts = nullptr;
  int32_t* labels = nullptr;
  float* cn = nullptr;
  auto cleanup = [&]() {
    dev_free(ix, cn, sizeof(float) * nlist);
    dev_free(ix, d_init, sizeof(int64_t) * nlist);
    dev_free(ix, best, sizeof(unsigned long long) * n);
    dev_free(ix, sums, sizeof(double) * size_t(nlist) * dp);
    dev_free(ix, counts, sizeof(int) * nlist);
    dev_free(ix, labels, sizeof(int32_t) * n);
  };
#define BUILD_TRY(expr)                          \
  do {                                           \
    int rc_ = (expr);                            \
    if (rc_) { cleanup(); dade_destroy(ix); return rc_; } \
  } while (0)
#define BUILD_HIP(expr)                                                      \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess) { cleanup(); dade_destroy(ix); FAIL(DADE_EDEVICE, hip_msg(e_, #expr)); } \
  } while (0)
  BUILD_TRY(alloc_t(ix, &ix->cent, size_t(nlist) * dp));
  BUILD_TRY(alloc_t(ix, &d_init, nlist));
  BUILD_TRY(alloc_t(ix, &best, n));
  BUILD_TRY(alloc_t(ix, &sums, size_t(nlist) * dp));
  BUILD_TRY(alloc_t(ix, &counts, nlist));
  BUILD_TRY(alloc_t(ix, &labels, n));
  BUILD_TRY(alloc_t(ix, &cn, nlist));
  BUILD_HIP(hipMemcpyAsync(d_init, init.data(), sizeof(int64_t) * nlist, hipMemcpyHostToDevice, s));
  BUILD_HIP(launch_gather_rows(ix->X, dp, d_init, nlist, ix->cent, s));
  GemmArgs g;
  g.M = int(n); g.N = nlist; g.K = dp;
  g.A = ix->X; g.lda = dp; g.B = ix->cent; g.ldb = dp; g.b_trans = true;
  g.col_norm = cn; g.row_best = best;
  for (int it = 0; it <= iters; ++it) {
    BUILD_HIP(launch_row_norms(ix->cent, nlist, dp, cn, s));
    BUILD_HIP(launch_fill_u64(best, n, ~0ull, s));
    BUILD_HIP(launch_gemm(g, kEpiArgmin, s));
    if (it == iters) break;  // final assignment to the last centroids
    BUILD_HIP(launch_fill_f64(sums, int64_t(nlist) * dp, 0.0, s));
    BUILD_HIP(launch_fill_i32(counts, nlist, 0, s));
    BUILD_HIP(launch_kmeans_accumulate(ix->X, n, dp, best, sums, counts, s));
    BUILD_HIP(launch_kmeans_finalize(sums, counts, nlist, dp, ix->cent, s));
  }
  BUILD_HIP(launch_labels_from_best(best, n, labels, s));
  std::vector<int32_t> lab(n);
  std::vector<float> cf(size_t(nlist) * dp);
  BUILD_HIP(hipMemcpyAsync(lab.data(), labels, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
  BUILD_HIP(hipMemcpyAsync(cf.data(), ix->cent, sizeof(float) * cf.size(), hipMemcpyDeviceToHost, s));
  BUILD_HIP(hipStreamSynchronize(s));
  cleanup();
  d_init = nullptr; best = nullptr; sums = nullptr; counts = nullptr; labels = nullptr; cn = nullptr;
#undef BUILD_TRY
#undef BUILD_HIP
  for (int64_t i = 0; i < n; ++i)
    if (lab[i] < 0 || lab[i] >= nlist) { dade_destroy(ix); FAIL(DADE_EDEVICE, "k-means produced an invalid label"); }
  ix->cent_h.assign(size_t(nlist) * dim, 0.0);
  for (int l = 0; l < nlist; ++l)
    for (int i = 0; i < dim; ++i) ix->cent_h[size_t(l) * dim + i] = cf[size_t(l) * dp + i];
  rc = set_lists(ix, lab, s);
  if (rc) { dade_destroy(ix); return rc; }
  ix->state = DADE_STATE_BUILT;
  *out = ix;
  return DADE_OK;
}

int dade_rotate(dade_index* ix, void* stream) {
  if (!ix) FAIL(DADE_EINVAL, "index is NULL");
  if (ix->state < DADE_STATE_BUILT) FAIL(DADE_ESTATE, "rotate needs a built index");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int dim = ix->dim, dp = ix->dp;
  double *mean = nullptr, *C = nullptr, *evals = nullptr, *offd = nullptr;
  rocblas_int* info = nullptr;
  int rc;
  auto cleanup = [&]() {
    dev_free(ix, mean, sizeof(double) * dim);
    dev_free(ix, C, sizeof(double) * size_t(dim) * dim);
    dev_free(ix, evals, sizeof(double) * dim);
    dev_free(ix, offd, sizeof(double) * dim);
    dev_free(ix, info, sizeof(rocblas_int));
  };
  if ((rc = alloc_t(ix, &mean, dim)) || (rc = alloc_t(ix, &C, size_t(dim) * dim)) ||
      (rc = alloc_t(ix, &evals, dim)) || (rc = alloc_t(ix, &offd, dim)) || (rc = alloc_t(ix, &info, 1))) {
    cleanup();
    return rc;
  }
  hipError_t e = launch_column_mean(ix->X, ix->n, dp, dim, mean, s);
  if (e == hipSuccess) e = launch_covariance(ix->X, ix->n, dp, dim, mean, C, dim, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) { cleanup(); FAIL(DADE_EDEVICE, hip_msg(e, "covariance")); }
  rocblas_handle h = nullptr;
  if (rocblas_create_handle(&h) != rocblas_status_success) { cleanup(); FAIL(DADE_EDEVICE, "rocblas_create_handle failed"); }
  rocblas_set_stream(h, s);
  rocblas_status st = rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, dim, C, dim, evals, offd, info);
  std::vector<double> V(size_t(dim) * dim), ev(dim), mu(dim);
  rocblas_int hinfo = 0;
  e = hipSuccess;
  if (st == rocblas_status_success) {
    e = hipMemcpyAsync(V.data(), C, sizeof(double) * V.size(), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(ev.data(), evals, sizeof(double) * dim, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(mu.data(), mean, sizeof(double) * dim, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&hinfo, info, sizeof(rocblas_int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  rocblas_destroy_handle(h);
  cleanup();
  if (st != rocblas_status_success) FAIL(DADE_EDEVICE, std::string("rocsolver_dsyevd: ") + rocblas_status_to_string(st));
  if (e != hipSuccess) FAIL(DADE_EDEVICE, hip_msg(e, "eigen readback"));
  if (hinfo != 0) FAIL(DADE_EDEVICE, "rocsolver_dsyevd did not converge (info " + std::to_string(hinfo) + ")");
  // V is column-major: eigenvector j = V[j*dim + i], eigenvalues ascending.
  std::vector<int> order(dim);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return ev[a] > ev[b]; });
  std::vector<double> W(size_t(dim) * dim), lam(dim);
  for (int k = 0; k < dim; ++k) {
    const int j = order[k];
    lam[k] = ev[j];
    int lead = 0;
    for (int i = 1; i < dim; ++i)
      if (std::fabs(V[size_t(j) * dim + i]) > std::fabs(V[size_t(j) * dim + lead])) lead = i;
    const double sg = V[size_t(j) * dim + lead] < 0 ? -1.0 : 1.0;
    for (int i = 0; i < dim; ++i) W[size_t(i) * dim + k] = sg * V[size_t(j) * dim + i];
  }
  ix->W = W; ix->lam = lam; ix->mu = mu;
  rc = apply_transform(ix, s);
  if (rc) return rc;
  ix->T.clear();
  ix->state = DADE_STATE_ROTATED;
  return DADE_OK;
}

int dade_calibrate(dade_index* ix, double alpha, const int64_t* pairs, int64_t n_pairs,
                   uint64_t seed, void* stream) {
  if (!ix) FAIL(DADE_EINVAL, "index is NULL");
  if (ix->state < DADE_STATE_ROTATED) FAIL(DADE_ESTATE, "calibrate needs a rotated index");
  if (!(alpha > 0.0 && alpha < 1.0)) FAIL(DADE_EINVAL, "alpha must be in (0, 1)");
  if (n_pairs < 1) FAIL(DADE_EINVAL, "n_pairs must be >= 1");
  if (ix->n < 2) FAIL(DADE_EINVAL, "calibration needs at least two rows");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int dim = ix->dim, dp = ix->dp;
  std::vector<int64_t> P(size_t(n_pairs) * 2);
  if (pairs) {
    for (int64_t i = 0; i < 2 * n_pairs; ++i) {
      if (pairs[i] < 0 || pairs[i] >= ix->n) FAIL(DADE_EINVAL, "pair ids must be in [0, n)");
      P[i] = pairs[i];
    }
  } else {
    SplitMix64 rng{seed};
    for (int64_t i = 0; i < n_pairs; ++i) {
      const int64_t a = int64_t(rng.below(uint64_t(ix->n)));
      const int64_t b = (a + 1 + int64_t(rng.below(uint64_t(ix->n - 1)))) % ix->n;
      P[2 * i] = a; P[2 * i + 1] = b;
    }
  }
  int64_t m = n_pairs;
  int64_t* dP = nullptr;
  double *delta = nullptr, *dis2 = nullptr, *Y = nullptr, *f = nullptr, *rel = nullptr, *dW = nullptr;
  auto cleanup = [&]() {
    dev_free(ix, dP, sizeof(int64_t) * 2 * n_pairs);
    dev_free(ix, delta, sizeof(double) * size_t(n_pairs) * dp);
    dev_free(ix, dis2, sizeof(double) * n_pairs);
    dev_free(ix, Y, sizeof(double) * size_t(n_pairs) * dp);
    dev_free(ix, f, sizeof(double) * size_t(std::max(dim - 1, 1)) * n_pairs);
    dev_free(ix, rel, sizeof(double) * n_pairs);
    dev_free(ix, dW, sizeof(double) * size_t(dp) * dp);
    dP = nullptr; delta = dis2 = Y = f = rel = dW = nullptr;
  };
#define CAL_HIP(expr)                                                             \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess) { cleanup(); FAIL(DADE_EDEVICE, hip_msg(e_, #expr)); } \
  } while (0)
  int rc;
  if ((rc = alloc_t(ix, &dP, 2 * n_pairs)) || (rc = alloc_t(ix, &delta, size_t(n_pairs) * dp)) ||
      (rc = alloc_t(ix, &dis2, n_pairs))) {
    cleanup();
    return rc;
  }
  // pass 1: drop pairs whose vectors are equal
  CAL_HIP(hipMemcpyAsync(dP, P.data(), sizeof(int64_t) * 2 * m, hipMemcpyHostToDevice, s));
  CAL_HIP(launch_pair_diff(ix->X, dp, dP, m, delta, dis2, s));
  std::vector<double> d2(m);
  CAL_HIP(hipMemcpyAsync(d2.data(), dis2, sizeof(double) * m, hipMemcpyDeviceToHost, s));
  CAL_HIP(hipStreamSynchronize(s));
  int64_t kept = 0;
  for (int64_t i = 0; i < m; ++i)
    if (d2[i] > 0.0) { P[2 * kept] = P[2 * i]; P[2 * kept + 1] = P[2 * i + 1]; ++kept; }
  if (kept == 0) { cleanup(); FAIL(DADE_EINVAL, "every calibration pair has equal vectors"); }
  if (kept != m) {
    m = kept;
    CAL_HIP(hipMemcpyAsync(dP, P.data(), sizeof(int64_t) * 2 * m, hipMemcpyHostToDevice, s));
    CAL_HIP(launch_pair_diff(ix->X, dp, dP, m, delta, dis2, s));
  }
  // rotated prefix terms: exact FP64 rotation for an FP32 store, stored coordinates otherwise
  if ((rc = alloc_t(ix, &f, size_t(std::max(dim - 1, 1)) * n_pairs)) || (rc = alloc_t(ix, &rel, n_pairs))) {
    cleanup();
    return rc;
  }
  const double* rows = nullptr;
  if (ix->store == DADE_F32) {
    if ((rc = alloc_t(ix, &Y, size_t(n_pairs) * dp)) || (rc = alloc_t(ix, &dW, size_t(dp) * dp))) { cleanup(); return rc; }
    std::vector<double> Wp(size_t(dp) * dp, 0.0);
    for (int i = 0; i < dim; ++i)
      for (int k = 0; k < dim; ++k) Wp[size_t(i) * dp + k] = ix->W[size_t(i) * dim + k];
    CAL_HIP(hipMemcpyAsync(dW, Wp.data(), sizeof(double) * Wp.size(), hipMemcpyHostToDevice, s));
    CAL_HIP(launch_dgemm(delta, dp, dW, dp, Y, dp, int(m), dp, dp, s));
    rows = Y;
  } else {
    if ((rc = alloc_t(ix, &Y, size_t(n_pairs) * dp))) { cleanup(); return rc; }
    CAL_HIP(launch_pair_diff_stored(ix->d_store, ix->store, ix->n, dp, ix->d_pos, dP, m, Y, s));
    rows = Y;
  }
  CAL_HIP(launch_prefix_fraction(rows, dp, m, dim, dis2, f, rel, s));
  std::vector<double> fh(size_t(std::max(dim - 1, 0)) * m), relh(m);
  if (dim > 1) CAL_HIP(hipMemcpyAsync(fh.data(), f, sizeof(double) * fh.size(), hipMemcpyDeviceToHost, s));
  CAL_HIP(hipMemcpyAsync(relh.data(), rel, sizeof(double) * m, hipMemcpyDeviceToHost, s));
  CAL_HIP(hipStreamSynchronize(s));
  cleanup();
#undef CAL_HIP
  // order statistic ceil((1 - alpha) M), 1-based
  auto ostat = [](std::vector<double>::iterator b, int64_t cnt, double p) {
    int64_t k = int64_t(std::ceil(p * double(cnt)));
    k = std::min(std::max<int64_t>(k, 1), cnt);
    std::nth_element(b, b + (k - 1), b + cnt);
    return *(b + (k - 1));
  };
  std::vector<double> T(dim, 1.0);
  for (int d = 0; d + 1 < dim; ++d) T[d] = ostat(fh.begin() + size_t(d) * m, m, 1.0 - alpha);
  ix->T = T;
  ix->delta = (ix->store == DADE_F32) ? 0.0 : ostat(relh.begin(), m, 0.999);
  rc = upload_T(ix, s);
  if (rc) return rc;
  ix->state = DADE_STATE_CALIBRATED;
  return DADE_OK;
}

int dade_export(const dade_index* ix, dade_artifacts* a) {
  if (!ix || !a) FAIL(DADE_EINVAL, "index or artifacts is NULL");
  a->n = ix->n; a->dim = ix->dim; a->nlist = ix->nlist; a->store_dtype = ix->store; a->state = ix->state;
  const size_t D = ix->dim;
  if (a->centroids) std::memcpy(a->centroids, ix->cent_h.data(), sizeof(double) * ix->cent_h.size());
  if (a->list_offsets) std::memcpy(a->list_offsets, ix->off_h.data(), sizeof(int64_t) * ix->off_h.size());
  if (a->list_ids) std::memcpy(a->list_ids, ix->ids_h.data(), sizeof(int64_t) * ix->ids_h.size());
  if (a->W || a->mu || a->lambda) {
    if (ix->state < DADE_STATE_ROTATED) FAIL(DADE_ESTATE, "W, mu and lambda exist after rotate");
    if (a->W) std::memcpy(a->W, ix->W.data(), sizeof(double) * D * D);
    if (a->mu) std::memcpy(a->mu, ix->mu.data(), sizeof(double) * D);
    if (a->lambda) std::memcpy(a->lambda, ix->lam.data(), sizeof(double) * D);
  }
  if (a->T) {
    if (ix->state < DADE_STATE_CALIBRATED) FAIL(DADE_ESTATE, "T exists after calibrate");
    std::memcpy(a->T, ix->T.data(), sizeof(double) * D);
  }
  a->delta = ix->delta;
  return DADE_OK;
}

int dade_import(const dade_artifacts* a, const float* X, const dade_build_opts* opts, void* stream,
                dade_index** out) {
  if (!a) FAIL(DADE_EINVAL, "artifacts is NULL");
  if (!a->W || !a->mu || !a->lambda || !a->centroids || !a->list_offsets || !a->list_ids)
    FAIL(DADE_EINVAL, "import needs W, mu, lambda, centroids and lists");
  hipStream_t s = static_cast<hipStream_t>(stream);
  dade_index* ix = nullptr;
  int rc = make_index(X, a->n, a->dim, a->nlist, opts, s, &ix);
  if (rc) return rc;
  const int dim = ix->dim, nl = ix->nlist;
  const int64_t n = ix->n;
  if (a->list_offsets[0] != 0 || a->list_offsets[nl] != n) { dade_destroy(ix); FAIL(DADE_EINVAL, "list offsets must span [0, n]"); }
  std::vector<int32_t> lab(n, -1);
  for (int l = 0; l < nl; ++l) {
    if (a->list_offsets[l + 1] < a->list_offsets[l]) { dade_destroy(ix); FAIL(DADE_EINVAL, "list offsets must not decrease"); }
    for (int64_t p = a->list_offsets[l]; p < a->list_offsets[l + 1]; ++p) {
      const int64_t id = a->list_ids[p];
      if (id < 0 || id >= n || lab[id] != -1) { dade_destroy(ix); FAIL(DADE_EINVAL, "list ids must be a permutation of [0, n)"); }
      if (p > a->list_offsets[l] && a->list_ids[p - 1] >= id) { dade_destroy(ix); FAIL(DADE_EINVAL, "list ids must ascend inside a list"); }
      lab[id] = l;
    }
  }
  ix->cent_h.assign(a->centroids, a->centroids + size_t(nl) * dim);
  std::vector<float> cf(size_t(nl) * ix->dp, 0.f);
  for (int l = 0; l < nl; ++l)
    for (int i = 0; i < dim; ++i) cf[size_t(l) * ix->dp + i] = float(a->centroids[size_t(l) * dim + i]);
  if ((rc = alloc_t(ix, &ix->cent, cf.size()))) { dade_destroy(ix); return rc; }
  hipError_t e = hipMemcpyAsync(ix->cent, cf.data(), sizeof(float) * cf.size(), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) { dade_destroy(ix); FAIL(DADE_EDEVICE, hip_msg(e, "centroids")); }
  if ((rc = set_lists(ix, lab, s))) { dade_destroy(ix); return rc; }
  ix->W.assign(a->W, a->W + size_t(dim) * dim);
  ix->mu.assign(a->mu, a->mu + dim);
  ix->lam.assign(a->lambda, a->lambda + dim);
  if ((rc = apply_transform(ix, s))) { dade_destroy(ix); return rc; }
  ix->state = DADE_STATE_ROTATED;
  if (a->T) {
    ix->T.assign(a->T, a->T + dim);
    ix->delta = a->delta;
    if ((rc = upload_T(ix, s))) { dade_destroy(ix); return rc; }
    ix->state = DADE_STATE_CALIBRATED;
  }
  *out = ix;
  return DADE_OK;
}

// The launches of one pass of the list scan: planning, then each round's DCO and merge kernels.
// kev (nullable): this pass's events (layout: see dade_index::kev).
static hipError_t enqueue_rounds(dade_index* ix, const RoundArgs& a, int rounds, hipEvent_t* kev, hipStream_t s) {
  hipError_t e;
#define ENQ(x) \
  if ((e = (x)) != hipSuccess) return e
  if (kev) ENQ(hipEventRecord(kev[0], s));
  ENQ(launch_plan(a, const_cast<int*>(a.item_off), s));
  if (kev) ENQ(hipEventRecord(kev[1], s));
  for (int r = 0; r < rounds; ++r) {
    hipEvent_t* ke = kev ? kev + 2 + 3 * r : nullptr;
    if (ke) ENQ(hipEventRecord(ke[0], s));
    ENQ(launch_round(a, r, s));
    if (ke) ENQ(hipEventRecord(ke[1], s));
    ENQ(launch_merge(a, r, s));
    if (ke) ENQ(hipEventRecord(ke[2], s));
  }
#undef ENQ
  return hipSuccess;
}

// dade_search with query rows `ldq` floats apart (the C ABI's queries are dense, ldq = dim; the
// graph build searches the index's own padded rows, ldq = dp).
// fixed (nullable): a workspace laid out by the caller for exactly these nq queries, used instead of the
// index's own (nothing is allocated, the batch is one pass, and nothing is captured into a graph).
static int search_impl(dade_index* ix, const float* Q, int64_t ldq, int64_t nq, int32_t k, int32_t nprobe,
                       const int32_t* k_per_query, const int32_t* nprobe_per_query,
                       const dade_search_opts* opts, int64_t* out_ids, float* out_dist2, void* stream,
                       const Workspace* fixed = nullptr) {
  if (!ix) FAIL(DADE_EINVAL, "index is NULL");
  if (nq < 0 || nq >= (int64_t(1) << 31)) FAIL(DADE_EINVAL, "nq must be in [0, 2^31)");
  if (k < 1 || k > kMaxK) FAIL(DADE_EINVAL, "k must be in [1, 128]");
  if (nprobe < 1) FAIL(DADE_EINVAL, "nprobe must be >= 1");
  dade_search_opts o{};
  o.delta_d = 0; o.mode = DADE_MODE_DADE; o.schedule = DADE_SCHED_PER_RANK; o.rerank_delta = -1.f;
  o.fill_min = 32; o.growth = 16; o.use_graph = 1;
  if (opts) o = *opts;
  if (o.fill_min < 0 || o.growth < 0) FAIL(DADE_EINVAL, "fill_min and growth must be >= 0");
  if (o.rerank_rule != DADE_RERANK_ALL && o.rerank_rule != DADE_RERANK_LAZY) FAIL(DADE_EINVAL, "bad rerank_rule");
  const int dd = o.delta_d > 0 ? o.delta_d : std::min(32, ix->dim);
  if (dd < 1 || dd > ix->dim) FAIL(DADE_EINVAL, "delta_d must be in [1, dim]");
  if (o.mode != DADE_MODE_DADE && o.mode != DADE_MODE_FULL_D) FAIL(DADE_EINVAL, "bad mode");
  if (o.schedule != DADE_SCHED_PER_RANK && o.schedule != DADE_SCHED_DOUBLING && o.schedule != DADE_SCHED_WHOLE)
    FAIL(DADE_EINVAL, "bad schedule");
  if (ix->state < DADE_STATE_ROTATED) FAIL(DADE_ESTATE, "search needs a rotated index");
  if (o.mode == DADE_MODE_DADE && ix->state < DADE_STATE_CALIBRATED) FAIL(DADE_ESTATE, "DADE mode needs a calibrated index");
  if (nq == 0) return DADE_OK;
  int rc;
  if ((rc = check_device_pointer(Q, "Q")) || (rc = check_device_pointer(out_ids, "out_ids")) ||
      (rc = check_device_pointer(out_dist2, "out_dist2")))
    return rc;
  if (k_per_query && (rc = check_device_pointer(k_per_query, "k_per_query"))) return rc;
  if (nprobe_per_query && (rc = check_device_pointer(nprobe_per_query, "nprobe_per_query"))) return rc;
  if (o.stats && (rc = check_device_pointer(o.stats, "stats"))) return rc;
  if (o.query_record && (rc = check_device_pointer(o.query_record, "query_record"))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int dp = ix->dp, nl = ix->nlist;
  const SearchPlan pl = plan_sizes(ix, k, nprobe, o);
  Workspace ws;
  if (fixed) {
    ws = *fixed;
    o.use_graph = 0;
    o.record_times = 0;
  } else if ((rc = grow_workspace(ix, nq, k, pl, s, ws))) {
    return rc;
  }
  const int npm = pl.npm, rounds = pl.rounds;
  const int64_t kb_cap = pl.kb_cap, items_pq = pl.items_pq, chunk = fixed ? nq : ws.chunk;
  if (o.use_graph && !ix->cap) HIPC(hipStreamCreateWithFlags(&ix->cap, hipStreamNonBlocking));
  if (o.scan_blocks_per_cu < 0) FAIL(DADE_EINVAL, "scan_blocks_per_cu must be >= 0");
  int& occ = ix->scan_occ[ix->store][o.mode][dd % 8 != 0];
  if (occ == 0) occ = round_blocks_per_cu(ix->store, o.mode, dd);
  const int blocks_per_cu = o.scan_blocks_per_cu > 0 ? std::min(o.scan_blocks_per_cu, occ) : occ;
  if (o.record_times && !ix->ev_made) {
    for (auto& e : ix->ev) HIPC(hipEventCreate(&e));
    ix->ev_made = true;
  }
  if (o.record_times) HIPC(hipEventRecord(ix->ev[0], s));
  // a1: q' = W^T (q - mu) on the FP32 matrix cores; a2: the probe order by (distance, list
  // id), from bf16 products for every centroid refined in FP32 where a rigorous bound cannot
  // decide.  Queries already of the padded width (and float4-aligned) are read in place, without the
  // padding copy.  The captured launch sequence holds the query pointer, so with graphs on only
  // a buffer passed again (a serving loop's) is read in place; a new buffer is copied, which
  // keeps the captured sequence valid.
  const bool q_in_place = ldq == dp && reinterpret_cast<uintptr_t>(Q) % 16 == 0 &&
                          (!o.use_graph || Q == ix->last_q);
  ix->last_q = Q;
  const float* qpad = q_in_place ? Q : ws.qpad;
  if (!q_in_place) HIPC(launch_pad_rows(Q, nq, ix->dim, ldq, ws.qpad, dp, s));
  GemmArgs g;
  g.M = int(nq); g.N = dp; g.K = dp;
  g.A = qpad; g.lda = dp; g.a_shift = ix->d_mu;
  g.B = ix->d_B; g.ldb = ix->ldB; g.C = ws.qrot; g.ldc = dp;
  g.split_col = dp;   // every column is a rotated coordinate
  // The rotation runs on an internal stream beside the probe selection (both only read the
  // queries), joined before the list scan; timed searches and the fixed-workspace entry point
  // run them in turn.
  const bool overlap = !fixed && !o.record_times;
  if (overlap) {
    if (!ix->side) HIPC(hipStreamCreateWithFlags(&ix->side, hipStreamNonBlocking));
    if (!ix->fork) HIPC(hipEventCreateWithFlags(&ix->fork, hipEventDisableTiming));
    if (!ix->join) HIPC(hipEventCreateWithFlags(&ix->join, hipEventDisableTiming));
    HIPC(hipEventRecord(ix->fork, s));
    HIPC(hipStreamWaitEvent(ix->side, ix->fork, 0));
  }
  HIPC(launch_gemm_rotate(g, overlap ? ix->side : s));
  if (overlap) HIPC(hipEventRecord(ix->join, ix->side));
  if (o.record_times) HIPC(hipEventRecord(ix->ev[1], s));
  ProbeArgs pa;
  pa.M = int(nq); pa.dp = dp; pa.nl = nl; pa.npm = npm;
  pa.q = qpad; pa.ldq = dp; pa.mu = ix->d_mu;
  pa.cb = ix->d_cb; pa.cx = ix->d_cx; pa.cn = ix->d_cent_norm; pa.cnorm = ix->d_cnorm;
  pa.a1 = ws.a1; pa.bnd = reinterpret_cast<uint32_t*>(ws.pd); pa.probes = ws.probes;
  HIPC(launch_probe_select(pa, s));
  if (overlap) HIPC(hipStreamWaitEvent(s, ix->join, 0));
  if (o.record_times) HIPC(hipEventRecord(ix->ev[2], s));
  // a3-a6: the list scan, in rounds, `chunk` queries at a time
  RoundArgs ra;
  std::memset(&ra, 0, sizeof ra);   // zero padding: argument blocks are compared bytewise
  ra.dim = ix->dim; ra.dp = dp; ra.delta_d = dd; ra.schedule = o.schedule;
  ra.fill_min = o.fill_min; ra.growth = o.growth;
  ra.mode = o.mode == DADE_MODE_DADE ? 0 : 1; ra.dtype = ix->store;
  ra.k_max = k; ra.nprobe_max = npm;
  ra.list_off = ix->d_off;
  ra.head = ix->d_store;
  ra.tail = static_cast<const char*>(ix->d_store) + size_t(ix->n) * kHead * dtype_size(ix->store);
  ra.ids = ix->d_ids; ra.X = ix->X; ra.T = ix->d_T;
  ra.rerank_delta = o.rerank_delta >= 0.f ? o.rerank_delta : float(ix->delta);
  ra.kb_cap = kb_cap;
  ra.rounds = rounds;
  ra.grid = ix->cus * blocks_per_cu;
  ra.rerank_rule = o.rerank_rule;
  const int64_t n_pass = (nq + chunk - 1) / chunk;
  std::vector<RoundArgs> passes(static_cast<size_t>(n_pass));
  for (int64_t pi = 0; pi < n_pass; ++pi) {
    const int64_t c0 = pi * chunk, cn = std::min(chunk, nq - c0);
    RoundArgs& a = passes[size_t(pi)];
    std::memcpy(&a, &ra, sizeof ra);
    a.nq = int(cn);
    a.k_pq = k_per_query ? k_per_query + c0 : nullptr;
    a.nprobe_pq = nprobe_per_query ? nprobe_per_query + c0 : nullptr;
    a.qrot = ws.qrot + c0 * dp; a.qorig = qpad + c0 * dp;
    a.probes = ws.probes + c0 * npm;
    a.out_ids = out_ids + c0 * k; a.out_d2 = out_dist2 + c0 * k;
    a.stats = o.stats ? o.stats + c0 * 4 : nullptr;
    a.q_record = o.query_record ? o.query_record + c0 * 3 : nullptr;
    a.q_topk = ws.topk; a.q_keyr = ws.keyr; a.q_r2 = ws.r2;
    a.q_topn = ws.qint; a.q_kc = a.q_topn + cn; a.q_rounds = a.q_topn + 2 * cn;
    a.kb = ws.kb;
    a.items_cap = int(std::min<int64_t>(chunk * items_pq, INT32_MAX));
    a.items = ws.items;
    a.n_items = ws.counter; a.overflow = ix->w_flags;
    a.item_off = ws.counts;
  }
  int graph_state = 0;
  if (o.record_times) {   // one set of events per pass; the reported times sum every pass
    while (ix->kev.size() < size_t(n_pass * (2 + 3 * rounds))) {
      hipEvent_t e;
      HIPC(hipEventCreate(&e));
      ix->kev.push_back(e);
    }
    ix->kev_rounds = rounds;
    ix->kev_passes = int(n_pass);
    for (int64_t pi = 0; pi < n_pass; ++pi) {
      const hipError_t e = enqueue_rounds(ix, passes[size_t(pi)], rounds, ix->kev.data() + size_t(pi) * (2 + 3 * rounds), s);
      if (e != hipSuccess) FAIL(DADE_EDEVICE, hip_msg(e, "list scan launch"));
    }
  } else if (!o.use_graph) {
    for (const RoundArgs& a : passes) {
      const hipError_t e = enqueue_rounds(ix, a, rounds, nullptr, s);
      if (e != hipSuccess) FAIL(DADE_EDEVICE, hip_msg(e, "list scan launch"));
    }
  } else {
    // the launch sequence of every pass, captured into one HIP graph and replayed while it is the
    // same as the last captured one.  Captures start on an internal stream (the caller's may be
    // the null stream, which cannot be captured).
    std::vector<unsigned char> key(sizeof(RoundArgs) * passes.size() + 2 * sizeof(int));
    std::memcpy(key.data(), passes.data(), sizeof(RoundArgs) * passes.size());
    const int tail[2] = {rounds, ix->device};
    std::memcpy(key.data() + sizeof(RoundArgs) * passes.size(), tail, sizeof tail);
    if (!ix->graph_done) HIPC(hipEventCreateWithFlags(&ix->graph_done, hipEventDisableTiming));
    if (ix->graph_exec && key == ix->graph_key) {
      HIPC(hipGraphLaunch(ix->graph_exec, s));
      HIPC(hipEventRecord(ix->graph_done, s));
      graph_state = 2;
    } else {
      HIPC(hipStreamBeginCapture(ix->cap, hipStreamCaptureModeRelaxed));
      hipError_t e = hipSuccess;
      for (const RoundArgs& a : passes)
        if (e == hipSuccess) e = enqueue_rounds(ix, a, rounds, nullptr, ix->cap);
      hipGraph_t g = nullptr;
      const hipError_t e2 = hipStreamEndCapture(ix->cap, &g);
      if (e == hipSuccess) e = e2;
      hipGraphExec_t x = nullptr;
      if (e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
      if (e == hipSuccess) {
        // the replaced sequence may still run from its last launch: wait for it before its
        // executable graph (and the argument blocks it owns) is released
        if (ix->graph_exec) {
          e = hipEventSynchronize(ix->graph_done);
          (void)hipGraphExecDestroy(ix->graph_exec);
          ix->graph_exec = nullptr;
        }
      }
      if (e == hipSuccess) {
        ix->graph_exec = x;
        x = nullptr;
        ix->graph_key.swap(key);
        e = hipGraphLaunch(ix->graph_exec, s);
        if (e == hipSuccess) e = hipEventRecord(ix->graph_done, s);
      }
      if (x) (void)hipGraphExecDestroy(x);
      if (e != hipSuccess) FAIL(DADE_EDEVICE, hip_msg(e, "list scan launch"));
      graph_state = 1;
    }
  }
  if (o.record_times) {
    HIPC(hipEventRecord(ix->ev[3], s));
    ix->ev_used = true;
  }
  if (o.record) {
    dade_search_record& rec = *o.record;
    rec.delta_d = dd; rec.mode = o.mode; rec.schedule = o.schedule;
    rec.fill_min = o.fill_min; rec.growth = o.growth;
    rec.rerank_rule = o.rerank_rule; rec.rerank_delta = ra.rerank_delta;
    rec.k = k; rec.nprobe_requested = nprobe; rec.nprobe = npm; rec.nprobe_clamped = nprobe > nl ? 1 : 0;
    rec.rounds = rounds; rec.passes = int(n_pass); rec.graph = graph_state;
  }
  return DADE_OK;
}

int dade_search(dade_index* ix, const float* Q, int64_t nq, int32_t k, int32_t nprobe,
                const int32_t* k_per_query, const int32_t* nprobe_per_query,
                const dade_search_opts* opts, int64_t* out_ids, float* out_dist2, void* stream) {
  if (!ix) FAIL(DADE_EINVAL, "index is NULL");
  return search_impl(ix, Q, ix->dim, nq, k, nprobe, k_per_query, nprobe_per_query, opts, out_ids, out_dist2, stream);
}

int dade_search_noalloc(dade_index* ix, const float* Q, int64_t nq, int32_t k, int32_t nprobe,
                        const int32_t* k_per_query, const int32_t* nprobe_per_query,
                        const dade_search_opts* opts, int64_t* out_ids, float* out_dist2, void* stream) {
  if (!ix) FAIL(DADE_EINVAL, "index is NULL");
  if (nq < 0 || nq >= (int64_t(1) << 31)) FAIL(DADE_EINVAL, "nq must be in [0, 2^31)");
  if (k < 1 || k > kMaxK) FAIL(DADE_EINVAL, "k must be in [1, 128]");
  if (nprobe < 1) FAIL(DADE_EINVAL, "nprobe must be >= 1");
  dade_search_opts o{};
  o.delta_d = 0; o.mode = DADE_MODE_DADE; o.schedule = DADE_SCHED_PER_RANK; o.rerank_delta = -1.f;
  o.fill_min = 32; o.growth = 16;
  if (opts) o = *opts;
  if (o.record_times) FAIL(DADE_EINVAL, "dade_search_noalloc: record_times needs events, which it does not create");
  o.use_graph = 0;
  if (o.fill_min < 0 || o.growth < 0) FAIL(DADE_EINVAL, "fill_min and growth must be >= 0");
  if (nq == 0) return search_impl(ix, Q, ix->dim, 0, k, nprobe, k_per_query, nprobe_per_query, &o, out_ids, out_dist2, stream);
  int dev = -1;
  HIPC(hipGetDevice(&dev));
  if (dev != ix->device)
    FAIL(DADE_EINVAL, "dade_search_noalloc: the index lives on device " + std::to_string(ix->device) +
                          ", the current device is " + std::to_string(dev));
  void* base = nullptr;
  int rc = scratch_address(dev, &base);
  if (rc) return rc;
  const SearchPlan pl = plan_sizes(ix, k, nprobe, o);
  // the most queries a slice of the scratch holds (slice_bytes is affine in the query count)
  const size_t fixed = slice_bytes(ix, pl, k, 0), per = slice_bytes(ix, pl, k, 1) - fixed;
  int64_t slice = 0;
  if (kScratchBytes > fixed + 13 * kScratchAlign) slice = int64_t((kScratchBytes - fixed - 13 * kScratchAlign) / per);
  while (slice > 0 && slice_bytes(ix, pl, k, slice) > kScratchBytes) --slice;
  if (slice < 1)
    FAIL(DADE_EINVAL, "dade_search_noalloc: one query of this search needs " + std::to_string(fixed + per) +
                          " bytes of scratch (k, nprobe and the round schedule set it), more than the " +
                          std::to_string(kScratchBytes) + " bytes it has");
  dade_search_record rec{};
  int64_t passes = 0;
  for (int64_t s0 = 0; s0 < nq; s0 += slice) {
    const int64_t cn = std::min(slice, nq - s0);
    const Workspace ws = carve(static_cast<char*>(base), ix, pl, k, cn);
    dade_search_opts os = o;
    os.stats = o.stats ? o.stats + s0 * 4 : nullptr;
    os.query_record = o.query_record ? o.query_record + s0 * 3 : nullptr;
    os.record = &rec;
    rc = search_impl(ix, Q + s0 * ix->dim, ix->dim, cn, k, nprobe, k_per_query ? k_per_query + s0 : nullptr,
                     nprobe_per_query ? nprobe_per_query + s0 : nullptr, &os, out_ids + s0 * k, out_dist2 + s0 * k,
                     stream, &ws);
    if (rc) return rc;
    ++passes;
  }
  if (o.record) {
    *o.record = rec;
    o.record->passes = int(passes);
    o.record->graph = 0;
  }
  return DADE_OK;
}

int dade_check(dade_index* ix, void* stream) {
  if (!ix) FAIL(DADE_EINVAL, "index is NULL");
  if (!ix->w_flags) return DADE_OK;
  int f = 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIPC(hipMemcpyAsync(&f, ix->w_flags, sizeof f, hipMemcpyDeviceToHost, s));
  HIPC(hipStreamSynchronize(s));
  if (f) FAIL(DADE_EDEVICE, "a list-scan capacity was exceeded (flags " + std::to_string(f) + ")");
  return DADE_OK;
}

int dade_stage_times(dade_index* ix, dade_times* out) {
  if (!ix || !out) FAIL(DADE_EINVAL, "index or output is NULL");
  if (!ix->ev_used) FAIL(DADE_ESTATE, "no timed search was recorded");
  HIPC(hipEventSynchronize(ix->ev[3]));
  float ms[3];
  for (int i = 0; i < 3; ++i) HIPC(hipEventElapsedTime(&ms[i], ix->ev[i], ix->ev[i + 1]));
  *out = dade_times{};
  out->query_gemm_ms = ms[0];
  out->select_ms = ms[1];
  out->scan_ms = ms[2];
  for (int p = 0; p < ix->kev_passes; ++p) {
    const hipEvent_t* k = ix->kev.data() + size_t(p) * (2 + 3 * ix->kev_rounds);
    float tp;
    HIPC(hipEventElapsedTime(&tp, k[0], k[1]));
    out->plan_ms += tp;
    for (int r = 0; r < ix->kev_rounds; ++r) {
      const hipEvent_t* e = k + 2 + 3 * r;
      float t1, t2;
      HIPC(hipEventElapsedTime(&t1, e[0], e[1]));
      HIPC(hipEventElapsedTime(&t2, e[1], e[2]));
      out->round_kernel_ms += t1;
      out->merge_kernel_ms += t2;
      ++out->round_launches;
    }
  }
  return DADE_OK;
}

namespace {

// Squared distance between rows a and b of the host copy (FP64 over the FP32 coordinates, in
// coordinate order).
double host_d2(const float* xh, int dp, int dim, int64_t a, int64_t b) {
  const float* x = xh + size_t(a) * dp;
  const float* y = xh + size_t(b) * dp;
  double s = 0.0;
  for (int c = 0; c < dim; ++c) {
    const double t = double(x[c]) - double(y[c]);
    s += t * t;
  }
  return s;
}

// True when the squared distance between rows a and b is below `bound`.  The partial sums only
// grow, so the sum can stop once it reaches the bound without changing the answer.
bool host_d2_below(const float* xh, int dp, int dim, int64_t a, int64_t b, double bound) {
  const float* x = xh + size_t(a) * dp;
  const float* y = xh + size_t(b) * dp;
  double s = 0.0;
  for (int c = 0; c < dim; ++c) {
    const double t = double(x[c]) - double(y[c]);
    s += t * t;
    if (s >= bound) return false;
  }
  return s < bound;
}

// HNSW's neighbour selection (Malkov and Yashunin, the simple form of their heuristic: no
// candidate extension, pruned candidates not added back) for row r: its candidates in ascending
// (squared distance, row id) order; a candidate is pruned when a neighbour kept before it is
// strictly closer to it than r is, and kept otherwise, until `degree` are kept.
void select_neighbours(const float* xh, int dp, int dim, int64_t r, const int64_t* cand, int nc, int degree,
                       std::vector<std::pair<double, int64_t>>& order, std::vector<int64_t>& kept) {
  order.clear();
  for (int i = 0; i < nc; ++i)
    if (cand[i] >= 0) order.emplace_back(host_d2(xh, dp, dim, r, cand[i]), cand[i]);
  std::sort(order.begin(), order.end());
  kept.clear();
  for (const auto& c : order) {
    if (int(kept.size()) == degree) break;
    bool keep = true;
    for (int64_t k : kept)
      if (host_d2_below(xh, dp, dim, c.second, k, c.first)) { keep = false; break; }
    if (keep) kept.push_back(c.second);
  }
}

}  // namespace

int dade_graph_build(dade_index* ix, int32_t degree, int32_t reverse, int32_t nprobe, int32_t candidates,
                     void* stream) {
  if (!ix) FAIL(DADE_EINVAL, "index is NULL");
  if (degree < 1 || reverse < 0 || degree + reverse > kGraphMax)
    FAIL(DADE_EINVAL, "degree >= 1, reverse >= 0 and degree + reverse <= 64 are required");
  if (nprobe < 1) FAIL(DADE_EINVAL, "nprobe must be >= 1");
  if (candidates != 0 && (candidates < degree || candidates + 1 > kMaxK))
    FAIL(DADE_EINVAL, "candidates must be 0 or in [degree, 127]");
  if (ix->state < DADE_STATE_ROTATED) FAIL(DADE_ESTATE, "the graph needs a rotated index");
  if (ix->n > kGraphBuildMaxRows)
    FAIL(DADE_EINVAL, "graph build: indexes of more than " + std::to_string(kGraphBuildMaxRows) +
                          " rows are not supported (a build of 1M x 960 rows faulted the GPU; its cause is open)");
  int rc = DADE_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t n = ix->n;
  const int width = degree + reverse;
  const bool select = candidates > 0;
  const int kk = (select ? candidates : degree) + 1;   // FDScanning results per row (the row itself among them)
  ix->graph_degree = 0;   // not usable until complete
  if (ix->d_nbr && ix->graph_width != width) {
    HIPC(hipStreamSynchronize(s));
    dev_free(ix, ix->d_nbr, sizeof(int32_t) * size_t(n) * ix->graph_width);
    ix->d_nbr = nullptr;
    ix->graph_width = 0;
  }
  if (!ix->d_nbr && (rc = alloc_t(ix, &ix->d_nbr, size_t(n) * width))) return rc;
  ix->graph_width = width;
  if (!ix->d_entry && (rc = alloc_t(ix, &ix->d_entry, size_t(ix->nlist) * 2))) return rc;
  // forward lists first, at stride `width`, then the back links merged in on the host
  const int64_t chunk = std::min<int64_t>(n, 65536);
  int64_t* res = nullptr;
  float* rd = nullptr;
  if ((rc = alloc_t(ix, &res, size_t(chunk) * kk))) return rc;
  if ((rc = alloc_t(ix, &rd, size_t(chunk) * kk))) {
    dev_free(ix, res, sizeof(int64_t) * size_t(chunk) * kk);
    return rc;
  }
  dade_search_opts o{};
  o.mode = DADE_MODE_FULL_D;
  o.schedule = DADE_SCHED_DOUBLING;
  o.rerank_delta = -1.f;
  o.fill_min = 32;
  o.growth = 0;
  // with selection: every row's `candidates` nearest other rows (row ids, -1 padded), by row id
  std::vector<int64_t> cand;
  if (select) cand.assign(size_t(n) * candidates, -1);
  std::vector<int64_t> res_h;
  // every row's kk nearest by FDScanning over nprobe lists, then itself dropped
  for (int64_t c0 = 0; c0 < n && rc == DADE_OK; c0 += chunk) {
    const int64_t cn = std::min(chunk, n - c0);
    // the queries are the index's own rows (zero-padded to dp), row id c0 + i at row c0 + i
    rc = search_impl(ix, ix->X + c0 * ix->dp, ix->dp, cn, kk, nprobe, nullptr, nullptr, &o, res, rd, stream);
    if (rc != DADE_OK) break;
    if (!select) {
      const hipError_t e = launch_graph_collect(res, int(cn), c0, degree, width, ix->d_pos, ix->d_nbr, s);
      if (e != hipSuccess) { dade::set_error(hip_msg(e, "graph collect")); rc = DADE_EDEVICE; }
      continue;
    }
    res_h.resize(size_t(cn) * kk);
    hipError_t e = hipMemcpyAsync(res_h.data(), res, sizeof(int64_t) * res_h.size(), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { dade::set_error(hip_msg(e, "graph candidates")); rc = DADE_EDEVICE; break; }
    for (int64_t i = 0; i < cn; ++i) {
      int w = 0;
      for (int j = 0; j < kk && w < candidates; ++j) {
        const int64_t id = res_h[size_t(i) * kk + j];
        if (id >= 0 && id != c0 + i) cand[size_t(c0 + i) * candidates + w++] = id;
      }
    }
  }
  if (rc == DADE_OK) {
    const hipError_t e = launch_graph_entry(ix->X, ix->cent, ix->d_off, ix->d_ids, ix->d_pos, ix->dp, ix->nlist,
                                            ix->d_entry, s);
    if (e != hipSuccess) { dade::set_error(hip_msg(e, "graph entry points")); rc = DADE_EDEVICE; }
  }
  const hipError_t e = hipStreamSynchronize(s);
  dev_free(ix, res, sizeof(int64_t) * size_t(chunk) * kk);
  dev_free(ix, rd, sizeof(float) * size_t(chunk) * kk);
  if (rc) return rc;
  if (e != hipSuccess) FAIL(DADE_EDEVICE, hip_msg(e, "graph build"));
  if (!select && reverse == 0) {
    ix->graph_degree = width;
    return DADE_OK;
  }
  const int dp = ix->dp;
  std::vector<int32_t> nb(size_t(n) * width, -1);   // by position, neighbour positions
  std::vector<float> xh(size_t(n) * dp);             // FP32 rows by row id
  HIPC(hipMemcpy(xh.data(), ix->X, sizeof(float) * xh.size(), hipMemcpyDeviceToHost));
  if (select) {
    // rows are independent: split them over host threads, each writing only its own rows
    const int nt = int(std::max<int64_t>(1, std::min<int64_t>(
        std::min<unsigned>(16u, std::max(1u, std::thread::hardware_concurrency())), n / 256 + 1)));
    auto work = [&](int t) {
      std::vector<std::pair<double, int64_t>> order;
      std::vector<int64_t> kept;
      for (int64_t r = t; r < n; r += nt) {
        select_neighbours(xh.data(), dp, ix->dim, r, cand.data() + size_t(r) * candidates, candidates, degree,
                          order, kept);
        int32_t* row = nb.data() + size_t(ix->d_pos_h(r)) * width;
        for (size_t j = 0; j < kept.size(); ++j) row[j] = int32_t(ix->d_pos_h(kept[j]));
      }
    };
    std::vector<std::thread> pool;
    int started = 0;
    try {
      for (; started < nt; ++started) pool.emplace_back(work, started);
    } catch (...) {
    }
    for (int t = started; t < nt; ++t) work(t);   // shares no thread could take run here
    for (auto& th : pool) th.join();
  } else {
    HIPC(hipMemcpy(nb.data(), ix->d_nbr, sizeof(int32_t) * nb.size(), hipMemcpyDeviceToHost));
  }
  if (reverse > 0) {
    // back links: for each row, the rows listing it that it does not list, nearest first by
    // (squared distance in FP64 over the FP32 vectors, row id), at most `reverse` of them
    std::vector<std::vector<int32_t>> incoming(static_cast<size_t>(n));
    for (int64_t p = 0; p < n; ++p)
      for (int j = 0; j < degree; ++j) {
        const int32_t u = nb[size_t(p) * width + j];
        if (u >= 0) incoming[size_t(u)].push_back(int32_t(p));
      }
    std::vector<std::pair<double, int64_t>> back;   // (distance, row id)
    for (int64_t v = 0; v < n; ++v) {
      int32_t* row = nb.data() + size_t(v) * width;
      const int64_t rv = ix->ids_h[size_t(v)];
      back.clear();
      for (int32_t u : incoming[size_t(v)]) {
        if (std::find(row, row + degree, u) != row + degree) continue;
        const int64_t ru = ix->ids_h[size_t(u)];
        back.emplace_back(host_d2(xh.data(), dp, ix->dim, ru, rv), ru);
      }
      std::sort(back.begin(), back.end());
      back.erase(std::unique(back.begin(), back.end()), back.end());
      int w = 0;
      while (w < degree && row[w] >= 0) ++w;
      for (size_t i = 0; i < back.size() && i < size_t(reverse); ++i) row[w++] = int32_t(ix->d_pos_h(back[i].second));
      for (; w < width; ++w) row[w] = -1;
    }
  }
  HIPC(hipMemcpy(ix->d_nbr, nb.data(), sizeof(int32_t) * nb.size(), hipMemcpyHostToDevice));
  ix->graph_degree = width;
  return DADE_OK;
}

int dade_graph_export(const dade_index* ix, int32_t* degree, int64_t* neighbors, int64_t* entries) {
  if (!ix) FAIL(DADE_EINVAL, "index is NULL");
  if (ix->graph_degree == 0) FAIL(DADE_ESTATE, "no graph has been built");
  if (degree) *degree = ix->graph_degree;
  const int64_t n = ix->n;
  const int deg = ix->graph_degree;
  if (neighbors) {
    std::vector<int32_t> nb(size_t(n) * deg);
    HIPC(hipMemcpy(nb.data(), ix->d_nbr, sizeof(int32_t) * nb.size(), hipMemcpyDeviceToHost));
    for (int64_t p = 0; p < n; ++p) {
      const int64_t row = ix->ids_h[size_t(p)];
      for (int j = 0; j < deg; ++j) {
        const int32_t u = nb[size_t(p) * deg + j];
        neighbors[row * deg + j] = u < 0 ? -1 : ix->ids_h[size_t(u)];
      }
    }
  }
  if (entries) {
    std::vector<int32_t> en(size_t(ix->nlist) * 2);
    HIPC(hipMemcpy(en.data(), ix->d_entry, sizeof(int32_t) * en.size(), hipMemcpyDeviceToHost));
    for (size_t i = 0; i < en.size(); ++i) entries[i] = en[i] < 0 ? -1 : ix->ids_h[size_t(en[i])];
  }
  return DADE_OK;
}

int dade_graph_search(dade_index* ix, const float* Q, int64_t nq, int32_t k, int32_t ef, int32_t n_entry,
                      int32_t max_iters, const dade_search_opts* opts, int64_t* out_ids, float* out_dist2,
                      void* stream) {
  if (!ix) FAIL(DADE_EINVAL, "index is NULL");
  if (ix->graph_degree == 0) FAIL(DADE_ESTATE, "no graph has been built");
  if (nq < 0 || nq >= (int64_t(1) << 31)) FAIL(DADE_EINVAL, "nq must be in [0, 2^31)");
  if (ef < 1 || ef > kGraphMax) FAIL(DADE_EINVAL, "ef must be in [1, 64]");
  if (k < 1 || k > ef) FAIL(DADE_EINVAL, "k must be in [1, ef]");
  if (n_entry < 1 || 2 * n_entry > kGraphMax) FAIL(DADE_EINVAL, "n_entry must be in [1, 32]");
  if (max_iters < 0) FAIL(DADE_EINVAL, "max_iters must be >= 0");
  dade_search_opts o{};
  o.mode = DADE_MODE_DADE;
  if (opts) o = *opts;
  const int dd = o.delta_d > 0 ? o.delta_d : std::min(32, ix->dim);
  if (o.mode != DADE_MODE_DADE && o.mode != DADE_MODE_FULL_D) FAIL(DADE_EINVAL, "bad mode");
  if (o.mode == DADE_MODE_DADE && (dd % 8 != 0 || dd > ix->dim))
    FAIL(DADE_EINVAL, "graph search: delta_d must be a multiple of 8 in [8, dim]");
  if (ix->state < DADE_STATE_ROTATED) FAIL(DADE_ESTATE, "search needs a rotated index");
  if (o.mode == DADE_MODE_DADE && ix->state < DADE_STATE_CALIBRATED) FAIL(DADE_ESTATE, "DADE mode needs a calibrated index");
  const int deg = ix->graph_degree;
  const int npm = std::min<int>(n_entry, ix->nlist);
  const int iters = max_iters > 0 ? max_iters : 2 * ef;
  // the visited table: at least twice the most insertions (seeds + iters x degree), <= 8192 slots
  const int64_t most = 2 * int64_t(npm) + int64_t(iters) * deg;
  int slots_log2 = 6;
  while ((int64_t(1) << slots_log2) < 2 * most) ++slots_log2;
  if (slots_log2 > 13)
    FAIL(DADE_EINVAL, "graph search: 2 n_entry + max_iters x width must be <= 4096 (visited table of 8192 slots)");
  if (nq == 0) return DADE_OK;
  int rc;
  if ((rc = check_device_pointer(Q, "Q")) || (rc = check_device_pointer(out_ids, "out_ids")) ||
      (rc = check_device_pointer(out_dist2, "out_dist2")))
    return rc;
  if (o.stats && (rc = check_device_pointer(o.stats, "stats"))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int dp = ix->dp, nl = ix->nlist;
  if ((rc = grow_query_workspace(ix, nq, npm, s))) return rc;
  // rotation and entry lists: the same GEMM and selection as dade_search
  const bool q_in_place = ix->dim == dp && reinterpret_cast<uintptr_t>(Q) % 16 == 0;
  const float* qpad = q_in_place ? Q : ix->w_qpad;
  if (!q_in_place) HIPC(launch_pad_rows(Q, nq, ix->dim, ix->dim, ix->w_qpad, dp, s));
  GemmArgs g;
  g.M = int(nq); g.N = dp + nl; g.K = dp;
  g.A = qpad; g.lda = dp; g.a_shift = ix->d_mu;
  g.B = ix->d_B; g.ldb = ix->ldB; g.C = ix->w_qrot; g.ldc = dp;
  g.split_col = dp; g.C2 = ix->w_pd; g.ldc2 = nl; g.col_norm = ix->d_cent_norm;
  HIPC(launch_gemm(g, kEpiRotateProbe, s));
  HIPC(launch_select_probes(ix->w_pd, nl, int(nq), nl, npm, ix->w_probes, s));
  GraphArgs a;
  a.nq = int(nq); a.dim = ix->dim; a.dp = dp; a.delta_d = dd;
  a.mode = o.mode == DADE_MODE_DADE ? 0 : 1; a.dtype = ix->store;
  a.K = k; a.ef = ef; a.n_entry = npm; a.npm = npm;
  a.degree = deg; a.max_iters = iters; a.slots_log2 = slots_log2;
  a.head = ix->d_store;
  a.tail = static_cast<const char*>(ix->d_store) + size_t(ix->n) * kHead * dtype_size(ix->store);
  a.qrot = ix->w_qrot; a.qorig = qpad; a.probes = ix->w_probes;
  a.entry = ix->d_entry; a.nbr = ix->d_nbr; a.ids = ix->d_ids; a.X = ix->X; a.T = ix->d_T;
  a.out_ids = out_ids; a.out_d2 = out_dist2; a.stats = o.stats;
  HIPC(launch_graph_search(a, s));
  return DADE_OK;
}

}  // extern "C"
