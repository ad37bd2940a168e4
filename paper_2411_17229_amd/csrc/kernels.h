// Host launchers of the DADE-IVF kernels (each defined next to its kernel).
#pragma once

#include "common.h"

namespace dade {

// ---------------------------------------------------------------- FP32 MFMA GEMM (gemm.hip)
// C[M x N] = op(A)[M x K] * B[K x N] with FP32 inputs and FP32 accumulation on MFMA.
// A row m is A[a_rows ? a_rows[m] : m] minus a_shift (per column k, nullable).
// B is [K x N] (ldb) or, with b_trans, given as [N x K] (ldb).  K % 16 == 0, lda/ldb % 4 == 0.
enum GemmEpilogue {
  kEpiStore = 0,    // C (float) = acc
  kEpiProbe = 1,    // C (float) = col_norm[n] - 2 acc
  kEpiArgmin = 2,   // row_best[m] = min over n of key(col_norm[n] - 2 acc, n)   (atomic)
  kEpiPackF32 = 3,  // C (float)   = acc
  kEpiPackBF16 = 4, // C (bf16)    = RNE(acc)
  kEpiPackF16 = 5,  // C (half)    = RNE(acc)
  kEpiRotateProbe = 6,  // n < split_col: C (float) = acc; else C2[n - split_col] = col_norm - 2 acc
};

struct GemmArgs {
  int M = 0, N = 0, K = 0;
  const float* A = nullptr;
  int lda = 0;
  const int32_t* a_rows = nullptr;
  const float* a_shift = nullptr;
  const float* B = nullptr;
  int ldb = 0;
  bool b_trans = false;
  void* C = nullptr;
  int ldc = 0;
  const float* col_norm = nullptr;
  unsigned long long* row_best = nullptr;
  int64_t split_rows = 0;   // pack epilogues: > 0 writes the head/tail store of that many rows
  int split_col = 0;        // kEpiRotateProbe: first column of the C2 part
  float* C2 = nullptr;
  int ldc2 = 0;
};
hipError_t launch_gemm(const GemmArgs& a, GemmEpilogue epi, hipStream_t s);
// q' = (q - mu) W only (kEpiRotateProbe, N <= split_col), tiled for small M x N.
hipError_t launch_gemm_rotate(const GemmArgs& a, hipStream_t s);

// ---------------------------------------------------------------- probe selection (probe.hip)
// The nprobe nearest lists of each query by t(c) = ||c - mu||^2 - 2 (q - mu).(c - mu), ties by
// list id, ascending: bf16 matrix-core products for every centroid, then the lists a rigorous
// error bound cannot rule out evaluated in FP32.  q: [M x ldq] FP32 queries (16-byte aligned,
// ldq % 4 == 0, zero-padded to dp); cb: the centroid fragments of probe_centroid_frags; cx:
// [nl x dp] FP32 c - mu; cn: [nl] ||c - mu||^2 in FP32; cnorm: [nl] upper bounds of ||c - mu||;
// a1: scratch of probe_a_bytes(M, dp) bytes; bnd: scratch [M x nl] (bounds of every list's
// term).
struct ProbeArgs {
  int M = 0, dp = 0, nl = 0, npm = 0;
  const float* q = nullptr;
  int ldq = 0;
  const float* mu = nullptr;
  const void* cb = nullptr;
  const float* cx = nullptr;
  const float* cn = nullptr;
  const float* cnorm = nullptr;
  void* a1 = nullptr;
  uint32_t* bnd = nullptr;
  int32_t* probes = nullptr;   // [M x npm]
};
hipError_t launch_probe_select(const ProbeArgs& p, hipStream_t s);
size_t probe_a_bytes(int M, int dp);
// bf16 (c - mu) in MFMA fragment order, columns padded with zeros to a multiple of 128:
// probe_centroid_frag_count(nl, dp) values from the [nl x dp] FP32 rows cx.
size_t probe_centroid_frag_count(int nl, int dp);
void probe_centroid_frags(const float* cx, int nl, int dp, uint16_t* out);

// ---------------------------------------------------------------- small kernels (misc.hip)
// dst[r][c] = src[r * lds + c] for c < cols, 0 up to ld.
hipError_t launch_pad_rows(const float* src, int64_t rows, int cols, int64_t lds, float* dst, int ld,
                           hipStream_t s);
hipError_t launch_gather_rows(const float* src, int ld, const int64_t* rows, int64_t count,
                              float* dst, hipStream_t s);
hipError_t launch_row_norms(const float* A, int64_t rows, int ld, float* out, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s);
hipError_t launch_fill_i32(int* p, int64_t n, int v, hipStream_t s);
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s);

// k-means update: FP64 atomic sums of the rows of X per assigned centroid, then the means.
hipError_t launch_kmeans_accumulate(const float* X, int64_t n, int ld,
                                    const unsigned long long* best, double* sums, int* counts,
                                    hipStream_t s);
hipError_t launch_kmeans_finalize(const double* sums, const int* counts, int nlist, int ld,
                                  float* centroids, hipStream_t s);
hipError_t launch_labels_from_best(const unsigned long long* best, int64_t n, int32_t* labels,
                                   hipStream_t s);

// ---------------------------------------------------------------- FP64 kernels (fp64.hip)
hipError_t launch_column_mean(const float* X, int64_t n, int ld, int dim, double* mean,
                              hipStream_t s);
// C[dim x dim] (ld) = (1/n) sum_i (x_i - mean)(x_i - mean)^T, upper and lower triangles.
hipError_t launch_covariance(const float* X, int64_t n, int ld, int dim, const double* mean,
                             double* C, int ldc, hipStream_t s);
// C[M x N] = A[M x K] * B[K x N], FP64, row-major with leading dimensions.
hipError_t launch_dgemm(const double* A, int lda, const double* B, int ldb, double* C, int ldc,
                        int M, int N, int K, hipStream_t s);
// Delta[i] = X[a_i] - X[b_i] in FP64 (ld columns), dis2[i] = ||Delta[i]||^2.
hipError_t launch_pair_diff(const float* X, int ld, const int64_t* pairs, int64_t m,
                            double* delta, double* dis2, hipStream_t s);
// Same from stored coordinates (head/tail store of `rows` rows): rows pos[a], pos[b].
hipError_t launch_pair_diff_stored(const void* store, int dtype, int64_t rows, int ld,
                                   const int64_t* pos, const int64_t* pairs, int64_t m,
                                   double* delta, hipStream_t s);
// f[d][i] = (sum_{k<=d} Y[i][k]^2) / dis2[i] for d < dim; rel[i] = |S_dim - dis2| / dis2.
hipError_t launch_prefix_fraction(const double* Y, int ld, int64_t m, int dim,
                                  const double* dis2, double* f, double* rel, hipStream_t s);

// ---------------------------------------------------------------- probe selection (select.hip)
// probes[q][0..nprobe) = ids of the nprobe smallest (pd[q][c], c), ascending.
hipError_t launch_select_probes(const float* pd, int ld_pd, int nq, int nlist, int nprobe, int32_t* probes,
                                hipStream_t s);

// ---------------------------------------------------------------- the list scan (scan.hip)
// One search runs as rounds (see scan.hip): launch_plan lays out every query's work items for
// all of its rounds; then, for r = 0 .. rounds - 1, launch_round (the DCOs of round r) and
// launch_merge (round r's heap update; a query's result after its last round).
struct RoundArgs {
  int nq = 0;
  int dim = 0;          // real dimensionality D
  int dp = 0;           // padded row length of stored coordinates
  int delta_d = 32;
  int schedule = 0;     // 0 per-rank, 1 doubling, 2 whole
  int fill_min = 32;    // the first round holds at least this many candidates
  int growth = 16;      // a later round holds at most growth x the candidates before it (0: any)
  int mode = 0;         // 0 DADE, 1 FULL_D
  int dtype = 0;        // stored coordinates: 0 f32, 1 bf16, 2 f16
  int k_max = 0;
  int nprobe_max = 0;
  int rounds = 0;       // rounds launched (an upper bound on any query's round count)
  const int32_t* k_pq = nullptr;
  const int32_t* nprobe_pq = nullptr;
  const float* qrot = nullptr;      // [nq x dp] rotated queries
  const float* qorig = nullptr;     // [nq x dp] original queries (rerank)
  const int32_t* probes = nullptr;  // [nq x nprobe_max]
  const int64_t* list_off = nullptr;
  const void* head = nullptr;       // stored coordinates [0, kHead) of each packed row
  const void* tail = nullptr;       // the rest, [n x (dp - kHead)]
  const int32_t* ids = nullptr;     // packed position -> row id
  const float* X = nullptr;         // [n x dp] original vectors by row id (rerank)
  const float* T = nullptr;         // [dim] T_d
  float rerank_delta = 0.f;
  int rerank_rule = 0;              // low-precision rerank: 0 every gated survivor, 1 lazy
  int32_t* q_record = nullptr;      // [nq x 3] per query: K used, nprobe used, rounds (nullable)
  int64_t* out_ids = nullptr;
  float* out_d2 = nullptr;
  int64_t* stats = nullptr;
  // per-query state
  unsigned long long* q_topk = nullptr;  // [nq x k_max] heap keys, ascending
  int* q_topn = nullptr;                 // [nq] heap size
  unsigned long long* q_keyr = nullptr;  // [nq] K-th key at the round's start (~0: not full)
  float* q_r2 = nullptr;                 // [nq] r^2 at the round's start (inf: not full)
  int* q_kc = nullptr;                   // [nq] keys queued in the current round
  int* q_rounds = nullptr;               // [nq] the query's round count
  unsigned long long* kb = nullptr;      // [nq x kb_cap] queued keys
  int64_t kb_cap = 0;
  // work items {query | count << kItemCountShift, first packed position, the query's K-th key at
  // the round's start (high word, low word; ~0: heap not full)}: round r's in
  // items[r * items_cap ...].  The plan writes them with an empty heap's key; the merge that ends
  // round r writes its snapshot into the query's items of round r + 1.
  int4* items = nullptr;
  int items_cap = 0;
  int* n_items = nullptr;          // [rounds]
  const int* item_off = nullptr;   // [rounds x nq] a query's first item in each round
  int* overflow = nullptr;  // [1] nonzero if a capacity was exceeded
  int grid = 0;
};
// Work items pack the query index below bit kItemCountShift and the candidate count (<= 64) above.
constexpr int kItemCountShift = 25;
constexpr int kMaxPassQueries = 1 << kItemCountShift;   // queries one pass of rounds may hold
// counts: device scratch of rounds x nq ints; afterwards it holds item_off.
hipError_t launch_plan(const RoundArgs& a, int* counts, hipStream_t s);
hipError_t launch_round(const RoundArgs& a, int r, hipStream_t s);
hipError_t launch_merge(const RoundArgs& a, int r, hipStream_t s);
// Resident scan_round workgroups per CU for a store type / mode / Delta_d.
int round_blocks_per_cu(int dtype, int mode, int delta_d);

// ---------------------------------------------------------------- graph search (graph.hip)
constexpr int kGraphMax = 64;   // largest degree, ef and n_entry (one wave holds a query's pool)
constexpr int64_t kGraphBuildMaxRows = 20000;   // largest index dade_graph_build accepts
struct GraphArgs {
  int nq = 0, dim = 0, dp = 0, delta_d = 0;   // delta_d % 8 == 0 in DADE mode
  int mode = 0, dtype = 0;                    // mode 0: DADE, 1: FDScanning
  int K = 0, ef = 0, n_entry = 0, npm = 0;    // K <= ef <= 64, n_entry = npm <= 32
  int degree = 0, max_iters = 0, slots_log2 = 0;
  const void* head = nullptr;       // packed store, as RoundArgs
  const void* tail = nullptr;
  const float* qrot = nullptr;      // [nq x dp]
  const float* qorig = nullptr;     // [nq x dp] original queries (final rerank)
  const int32_t* probes = nullptr;  // [nq x npm] list ids in probe order
  const int32_t* entry = nullptr;   // [nlist x 2] entry positions per list (medoid, farthest), -1 if none
  const int32_t* nbr = nullptr;     // [n x degree] out-neighbour positions, -1 padded
  const int32_t* ids = nullptr;     // packed position -> row id
  const float* X = nullptr;         // [n x dp] original vectors by row id
  const float* T = nullptr;         // [dim]
  int64_t* out_ids = nullptr;       // [nq x K]
  float* out_d2 = nullptr;
  int64_t* stats = nullptr;         // [nq x 4]: DCOs, dimensions read, expansions, visited
};
// LDS bytes of one query's workgroup: the visited table (2^slots_log2 ints) and the merge area.
size_t graph_lds_bytes(int slots_log2);
hipError_t launch_graph_search(const GraphArgs& a, hipStream_t s);
hipError_t launch_graph_collect(const int64_t* res, int cn, int64_t c0, int degree, int width, const int64_t* pos,
                                int32_t* nbr, hipStream_t s);
hipError_t launch_graph_entry(const float* X, const float* cent, const int64_t* off, const int32_t* ids,
                              const int64_t* pos, int dp, int nlist, int32_t* entry, hipStream_t s);

}  // namespace dade
