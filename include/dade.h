/*
 * dade.h -- C ABI of an MI355X (gfx950) engine for DADE distance comparisons inside an
 * IVF scan (data-aware distance estimation, arXiv 2411.17229).
 *
 * The operations follow the paper's problem statement:
 *   - Definition 1 (DCO): given q, o and r, decide whether dis(q, o) <= r and return dis.
 *   - Algorithm 1: the DCO runs over growing prefixes of Delta_d transformed dimensions,
 *     estimates the distance with Eq. (13), tests H0: dis < r by rejecting when
 *     dis' > (1 + eps_d) r (eps_d from Eq. (14)), and compares exactly at d = D.
 *   - End of the Methodology section: IVF selects the N_probe clusters nearest to the query
 *     and scans their candidates with one DCO each against the maximum of a size-K heap.
 *   - After Eq. (13): objects are transformed once by the PCA matrix W (Eqs. (10)-(12)) and
 *     stored; eps_d is estimated from sampled data objects.
 *
 * Conventions shared by every call
 *   - Device pointers: X, Q, per-query K / nprobe arrays and outputs are caller-owned device
 *     memory of the current HIP device.  The library copies what it keeps; it keeps no
 *     caller pointer after a call returns.  Host pointers are marked "host".
 *   - Matrices are row-major and dense: X is [n x dim], Q is [nq x dim] (leading dimension
 *     dim), outputs are [nq x k] (leading dimension k).
 *   - stream: a hipStream_t passed as void*.  dade_search only enqueues work on it; its
 *     outputs are valid once the stream has been synchronised.  dade_build_index,
 *     dade_rotate, dade_calibrate and dade_import synchronise the stream before returning.
 *   - Distances are SQUARED Euclidean distances (equal in the original and rotated bases,
 *     Lemma 1).  Ids are 0-based row indices of X.
 *   - Errors: every int-returning call returns DADE_OK or a negative dade_status, and
 *     dade_last_error() returns a message for the calling thread's last failure.  A failed
 *     call leaves the index as it was.  No C++ exception crosses this interface.
 *   - Thread safety: calls on different indexes may run concurrently; calls on one index
 *     must be serialised by the caller.
 */
#ifndef DADE_H
#define DADE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dade_index dade_index; /* opaque; owns every device buffer of one index */

typedef enum {
  DADE_OK = 0,
  DADE_EINVAL = -1,  /* an argument is out of range or a required pointer is NULL */
  DADE_ESTATE = -2,  /* the call is not allowed in the index's current state */
  DADE_ENOMEM = -3,  /* the HBM budget would be exceeded or an allocation failed */
  DADE_EDEVICE = -4  /* a HIP runtime / library error; the message names it */
} dade_status;

typedef enum { DADE_F32 = 0, DADE_BF16 = 1, DADE_F16 = 2 } dade_dtype;

/* FULL_D = FDScanning (Experiments, Algorithms): every DCO reads all D dimensions. */
typedef enum { DADE_MODE_DADE = 0, DADE_MODE_FULL_D = 1 } dade_mode;

/* Which heap state each DCO's threshold r comes from (the paper's IVF updates the heap after
 * every candidate, which makes a parallel scan order-dependent).  A query's candidate
 * sequence (its probed lists in probe order) is split into rounds; every DCO of a round sees
 * the heap as it was when the round started; the round's accepted candidates are merged at its
 * end.  The first round holds the first max(K, fill_min) candidates.  A later round ends at the
 * next probe-rank boundary of the schedule -- PER_RANK: every rank; DOUBLING: ranks 1, 2, 4,
 * 8, ...; WHOLE: none, the probe ranks form one range -- or once it holds growth times the
 * candidates scanned before it, whichever comes first (growth 0: no such cap; WHOLE with
 * growth 0 is two rounds: the first one, then the rest). */
typedef enum { DADE_SCHED_PER_RANK = 0, DADE_SCHED_DOUBLING = 1, DADE_SCHED_WHOLE = 2 } dade_schedule;

/* Index state machine: BUILT -> ROTATED -> CALIBRATED. */
typedef enum { DADE_STATE_BUILT = 1, DADE_STATE_ROTATED = 2, DADE_STATE_CALIBRATED = 3 } dade_state;

typedef struct {
  int32_t kmeans_iters;       /* Lloyd iterations; 0 means 10 */
  int32_t store_dtype;        /* dade_dtype of the stored rotated coordinates */
  const int64_t* init_rows;   /* host, nlist distinct row ids seeding k-means; NULL: drawn
                                 from `seed` */
  uint64_t seed;
  int64_t hbm_budget_bytes;   /* upper bound on device memory this index may hold; 0: none */
} dade_build_opts;

/* Low-precision rerank rules (the paper has no low-precision store).  A DCO that reaches d = D
 * on the stored coordinates passes the gate when the heap is not full or its stored-precision
 * S_D <= (1 + rerank_delta) r^2.  ALL gives every candidate that passed the gate its exact FP32
 * distance from the original vectors.  LAZY gives it to the K smallest of them by stored S_D,
 * then to the others only where S_D <= (1 + rerank_delta) b, b the K-th smallest exact distance
 * of the heap and those K; it keeps what ALL keeps unless a skipped candidate's stored-precision
 * error exceeds rerank_delta.  Either way the keep rule applies to exact distances. */
typedef enum { DADE_RERANK_ALL = 0, DADE_RERANK_LAZY = 1 } dade_rerank_rule;

/* What a dade_search call ran with (host, filled on success when requested): the values that
 * define its results -- Delta_d, the mode, the round schedule and the rerank rule and margin, so
 * that a reference implementation can replay the search -- and how it was launched. */
typedef struct {
  int32_t delta_d;            /* Delta_d used (after the default) */
  int32_t mode;               /* dade_mode */
  int32_t schedule;           /* dade_schedule */
  int32_t fill_min;
  int32_t growth;
  int32_t rerank_rule;        /* dade_rerank_rule (low-precision stores) */
  float rerank_delta;         /* the gate's margin used (low-precision stores) */
  int32_t k;                  /* the k argument: the largest K */
  int32_t nprobe_requested;   /* the nprobe argument */
  int32_t nprobe;             /* after clamping to nlist */
  int32_t nprobe_clamped;     /* 1 when nprobe > nlist was clamped */
  int32_t rounds;             /* round launches per pass (an upper bound on any query's rounds) */
  int32_t passes;             /* the batch ran in this many passes of the list scan */
  int32_t graph;              /* 0: launched one by one; 1: captured into a HIP graph and
                                 launched; 2: an earlier capture replayed */
} dade_search_record;

typedef struct {
  int32_t delta_d;            /* Delta_d of Algorithm 1, in [1, dim]; 0 means 32 (or dim if
                                 smaller) */
  int32_t mode;               /* dade_mode */
  int32_t schedule;           /* dade_schedule */
  float rerank_delta;         /* low-precision stores only: a survivor whose stored-precision
                                 S_D exceeds (1 + rerank_delta) r^2 is dropped before the exact
                                 FP32 rerank; < 0 means the calibrated value */
  int64_t* stats;             /* device, nullable: [nq x 4] int64 per query: DCOs, dimensions
                                 read (sum of the d at which each DCO ended), candidates kept,
                                 candidates reranked */
  int32_t record_times;       /* nonzero: time the stages and kernels with HIP events
                                 (dade_stage_times) */
  int32_t fill_min;           /* >= 0: the first round holds at least this many candidates */
  int32_t growth;             /* >= 0: cap on a later round's size, as a multiple of the
                                 candidates scanned before it; 0 means no cap */
  int32_t use_graph;          /* nonzero: the list scan's kernel sequence is captured once into
                                 a HIP graph and replayed while the arguments (pointers, sizes,
                                 options) stay the same; results are identical either way */
  int32_t scan_blocks_per_cu; /* launch shape of the DCO kernel: workgroups per compute unit of
                                 its persistent grid; 0 (or more than fit) means as many as are
                                 resident at once; results are identical for every value */
  int32_t rerank_rule;        /* dade_rerank_rule for low-precision stores; 0 means ALL */
  dade_search_record* record; /* host, nullable: filled with what the call ran with */
  int32_t* query_record;      /* device, nullable: [nq x 3] int32 per query: K used, nprobe used
                                 (per-query values clamped into [1, k] and [1, nprobe], nprobe
                                 clamped to nlist), and the query's round count */
} dade_search_opts;

/* Host copies of an index's artifacts (for checkpoints and for parity checks).  All arrays
 * are caller-allocated with the sizes dade_index_info reports. */
typedef struct {
  int64_t n;
  int32_t dim;
  int32_t nlist;
  int32_t store_dtype;
  int32_t state;
  double* W;            /* [dim x dim]; W[i*dim + k] = component i of w_k (Eq. (11)) */
  double* mu;           /* [dim] the mean of X (Lemma 1) */
  double* lambda;       /* [dim] eigenvalues, descending (Eq. (12)) */
  double* T;            /* [dim] reduced thresholds T_d, d = 1..dim (T_dim = 1); on import
                           NULL means "not calibrated" */
  double delta;         /* rerank margin (low-precision stores) */
  double* centroids;    /* [nlist x dim] in the original basis */
  int64_t* list_offsets;/* [nlist + 1] */
  int64_t* list_ids;    /* [n] row ids grouped by list, ascending inside a list */
} dade_artifacts;

/*
 * dade_build_index -- IVF lists by k-means (Experiments, Parameter Setting: N_c clusters as in
 * Faiss).  Copies X (device, [n x dim] FP32) into the index, runs `kmeans_iters` Lloyd
 * iterations in FP32 from the seed rows, assigns every row to its nearest final centroid
 * (ties: lower centroid id) and groups rows by list in ascending row id.
 * Requires 1 <= dim <= 4096, 1 <= nlist <= min(n, 8192), n < 2^31.
 * On success *out is a new index in state BUILT.  Synchronises `stream`.
 */
int dade_build_index(const float* X, int64_t n, int32_t dim, int32_t nlist,
                     const dade_build_opts* opts, void* stream, dade_index** out);

/*
 * dade_rotate -- the data-aware transform (Lemma 1; Eqs. (10)-(12)).  Computes mu and the
 * 1/N second moment of the centred data in FP64 on the device, its eigendecomposition in FP64
 * (rocSOLVER syevd), sorts eigenpairs by descending eigenvalue and fixes each eigenvector's
 * sign (largest-magnitude entry positive).  Then stores every object once as W^T (x - mu) in
 * the index's store dtype (round to nearest even), laid out list by list.
 * Requires state >= BUILT; leaves the index ROTATED (a previous calibration is dropped).
 * Synchronises `stream`.
 */
int dade_rotate(dade_index* ix, void* stream);

/*
 * dade_calibrate -- eps_d of Eq. (14) in its reduced form.  For each pair (a, b) of distinct
 * data rows, f_d = S_d / ||x_a - x_b||^2 with S_d the squared norm of the first d rotated
 * coordinates of x_a - x_b (FP64; for BF16/FP16 stores, of the stored coordinates).  Pairs
 * with x_a == x_b are dropped (M pairs remain).  T_d is the ceil((1 - alpha) M)-th smallest
 * f_d (alpha = P_s); rejecting when S_d > T_d r^2 is the same test as dis' > (1 + eps_d) r.
 * For low-precision stores the rerank margin is the ceil(0.999 M)-th smallest relative error
 * |S_D - ||x_a - x_b||^2| / ||x_a - x_b||^2.
 * pairs: host [n_pairs x 2] int64 row ids, or NULL to draw n_pairs uniform ordered pairs with
 * a != b from `seed`.  Requires state >= ROTATED, 0 < alpha < 1, n_pairs >= 1, M >= 1.
 * Leaves the index CALIBRATED.  Synchronises `stream`.
 */
int dade_calibrate(dade_index* ix, double alpha, const int64_t* pairs, int64_t n_pairs,
                   uint64_t seed, void* stream);

/*
 * dade_search -- IVF search with one DCO per candidate (Algorithm 1, or FDScanning in FULL_D
 * mode).  Q: device [nq x dim] FP32.  k, nprobe: the values for every query, or the maxima
 * when k_per_query / nprobe_per_query (device int32 [nq], nullable) are given; per-query
 * values are clamped into [1, k] and [1, nprobe]; nprobe is clamped to nlist.
 * Outputs: out_ids (device int64 [nq x k]) and out_dist2 (device FP32 [nq x k]), each row
 * ascending by (squared distance, id), padded with (-1, +inf) after the query's K results.
 * Requires state CALIBRATED for DADE mode and >= ROTATED for FULL_D; 1 <= k <= 128;
 * nprobe >= 1; nq >= 0 (nq == 0 is a no-op).  opts may be NULL: delta_d 32, DADE mode,
 * PER_RANK, the calibrated rerank_delta and rule ALL, no stats, records or timing, fill_min 32,
 * growth 16, graph, a full grid.
 * Asynchronous on `stream`.
 */
int dade_search(dade_index* ix, const float* Q, int64_t nq, int32_t k, int32_t nprobe,
                const int32_t* k_per_query, const int32_t* nprobe_per_query,
                const dade_search_opts* opts, int64_t* out_ids, float* out_dist2,
                void* stream);

/*
 * dade_search_noalloc -- dade_search for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments,
 * results (bit for bit) and stream semantics as dade_search; it calls no hipMalloc, hipFree or
 * other allocating routine.  Its workspace is a fixed scratch array of 64 MiB per device, held by
 * the library from the first call on that device until the process ends, instead of the index's
 * growable workspace.  The batch runs in slices of as many queries as the scratch holds; a search
 * one query of which needs more than 64 MiB (a huge widest round: large lists, nprobe and K) is
 * rejected with DADE_EINVAL before any device work.  Nothing is captured into a graph: use_graph
 * is ignored and record_times is rejected (DADE_EINVAL).  The index must live on the current
 * device.  Every call on one device shares that device's scratch: calls that overlap on one
 * device (other streams, other threads) race and give undefined results; serialise them.
 */
int dade_search_noalloc(dade_index* ix, const float* Q, int64_t nq, int32_t k, int32_t nprobe,
                        const int32_t* k_per_query, const int32_t* nprobe_per_query,
                        const dade_search_opts* opts, int64_t* out_ids, float* out_dist2, void* stream);

/* dade_check -- synchronises `stream` and reports DADE_EDEVICE if any search on this index
 * since its creation exceeded an internal capacity of the list scan (its results would be
 * incomplete); DADE_OK otherwise.  The capacities are sized so that this does not happen; the
 * call exists so that tests and callers can assert it. */
int dade_check(dade_index* ix, void* stream);

/* dade_index_info -- sizes and state (any pointer may be NULL). */
int dade_index_info(const dade_index* ix, int64_t* n, int32_t* dim, int32_t* nlist,
                    int32_t* store_dtype, int32_t* state);

/* dade_export -- copy the artifacts to caller-allocated host arrays (NULL arrays are skipped).
 * W, mu, lambda need state >= ROTATED; T and delta need CALIBRATED. */
int dade_export(const dade_index* ix, dade_artifacts* out);

/*
 * dade_import -- an index from artifacts (host) and the base vectors X (device [n x dim]).
 * Uses the given lists, centroids, W and mu instead of computing them and packs the store as
 * dade_rotate does; with a non-NULL T it is CALIBRATED, else ROTATED.  opts->store_dtype
 * selects the store.  Synchronises `stream`.
 */
int dade_import(const dade_artifacts* a, const float* X, const dade_build_opts* opts,
                void* stream, dade_index** out);

/* Stage and kernel times of the last dade_search run with record_times set (HIP events on the
 * stream each kernel ran on).  With record_times the scan's kernels are launched one by one (not
 * from a graph), with events around every round's kernels. */
typedef struct {
  float query_gemm_ms;      /* one GEMM: rotated queries and query-centroid distances */
  float select_ms;          /* probe selection */
  float scan_ms;            /* the whole list scan: planning, rounds and merges */
  float round_kernel_ms;    /* sum over rounds (and passes) of the DCO kernel's duration */
  float merge_kernel_ms;    /* sum over rounds (and passes) of the merge kernel's duration */
  float plan_ms;            /* work-item planning (all passes) */
  int32_t round_launches;   /* DCO kernel launches summed in round_kernel_ms; a search whose
                               workspace cannot hold every query at once runs in passes */
} dade_times;

/* dade_stage_times -- wait for the last timed dade_search and report its times. */
int dade_stage_times(dade_index* ix, dade_times* out);

/*
 * Serving loop (continuous batching over an open arrival process).  Every query is the IVF
 * search that dade_search runs (end of the Methodology section); the loop around it -- admission,
 * batching, copies -- is an engineering layer the paper does not describe.
 *
 * dade_serve runs a stream of requests against one index and returns when every request has
 * completed.  Request i arrives arrival_s[i] seconds after the call starts (a non-decreasing
 * schedule, e.g. Poisson arrivals drawn by the caller) and holds req_queries[i] >= 1 queries that
 * share K = req_k[i] and nprobe = req_nprobe[i].  The loop, on the calling thread:
 *   - admits arrived requests in arrival order while the device budget has room: an admitted
 *     request takes one slot per query in a device ring (query row, K, nprobe, k_max results);
 *     its rows are copied to the device from Q itself when Q is pinned host memory
 *     (hipHostMalloc, torch pin_memory), else staged first in a pinned mirror of the ring (a host
 *     copy that costs host bandwidth); a request that
 *     does not fit waits (and those behind it); one larger than the whole ring is rejected.
 *     Admission pauses while the admitted queries not yet launched already fill max_inflight
 *     launches of max_batch;
 *   - whenever fewer than max_inflight searches are on the device, launches the admitted queries
 *     not yet launched (up to max_batch, whole or part requests, contiguous ring slots): their
 *     slots are copied to the device on a copy stream (overlapping the launches before), and one
 *     dade_search with per-query K and nprobe runs on `stream` after the copy; requests that
 *     arrive meanwhile are admitted while it runs and go into the next launch;
 *   - copies each launch's results back on a second copy stream; a request completes when its
 *     last query's results are on the host, and its slots are freed.
 * Each query's result is that of dade_search on the query alone with the same K, nprobe and
 * options (results do not depend on the batch).
 * Q: host [sum(req_queries) x dim] FP32 (pinned or pageable), the requests' queries one after
 * another in request order.  out_ids (host int64) and out_dist2 (host FP32) are [sum(req_queries) x k_max] in the
 * same order, padded as dade_search's; a rejected request's rows are all (-1, +inf).
 * out_latency_s (host, nullable): per request, the time from its arrival to its completion in
 * seconds, -1 for a rejected request.  stats (host, nullable) is filled on success.
 * Device memory: the search workspace for max_batch queries plus the ring, both within
 * opts->budget_bytes and within the index's own HBM budget; the ring is freed on return.
 * Requires the index state search requires; arrival_s non-decreasing and >= 0; 1 <= req_k[i] <=
 * k_max <= 128; 1 <= req_nprobe[i] <= nprobe_max.  Synchronises `stream` before returning.
 */
typedef struct {
  int64_t budget_bytes;     /* device bytes for the search workspace and the request ring;
                               0 means 512 MiB */
  int32_t max_batch;        /* most queries in one launch; 0 means 1024 */
  int32_t max_inflight;     /* most launches on the device at once; 0 means 2 */
  int32_t k_max;            /* result row length (the largest K a request may ask for) */
  int32_t nprobe_max;       /* the largest nprobe a request may ask for */
  dade_search_opts search;  /* as for dade_search; stats, record_times and use_graph are
                               ignored (launches are not captured) */
} dade_serve_opts;

typedef struct {
  double wall_s;             /* from the call's start (arrival time 0) to the last completion */
  int64_t served_requests;
  int64_t rejected_requests;
  int64_t served_queries;
  int64_t launches;          /* dade_search launches */
  int64_t ring_slots;        /* query slots of the ring (what the budget left after the
                                workspace) */
  int64_t peak_slots;        /* most ring slots held at once */
  int64_t waited_requests;   /* requests that found the ring full on arrival and waited */
  int64_t workspace_bytes;   /* device bytes of the search workspace */
  double stage_s;            /* host seconds spent staging admitted queries in pinned memory */
  double launch_s;           /* host seconds spent enqueueing copies and searches */
  double retire_s;           /* host seconds spent handing results out */
} dade_serve_stats;

int dade_serve(dade_index* ix, int64_t n_req, const double* arrival_s, const int32_t* req_queries,
               const int32_t* req_k, const int32_t* req_nprobe, const float* Q,
               const dade_serve_opts* opts, int64_t* out_ids, float* out_dist2,
               double* out_latency_s, dade_serve_stats* stats, void* stream);

/*
 * Autotuner.  The hypothesis tests run at multiples of Delta_d (Algorithm 1); the paper leaves
 * Delta_d as a parameter and reports that its best value depends on the workload (Experiments:
 * the Delta_d study).  dade_autotune picks Delta_d, the round shape and the DCO kernel's launch
 * shape for a given index and query sample by measurement:
 *   1. a FULL_D search of the sample with the same K / nprobe is the reference (its top-K is the
 *      exact top-K of the probed candidates, whatever the round shape);
 *   2. every candidate (Delta_d in {8, 16, 32, 64, 128} within [1, dim], times the round shapes
 *      {doubling, fill_min 32, growth 0}, {doubling, 32, 16}, {per-rank, 32, 16}) is searched
 *      once, its agreement measured (mean over queries of |top-K ids in the reference| / the
 *      reference's valid ids), then timed over `reps` searches with HIP events on `stream`;
 *   3. the fastest candidate with agreement >= min_agreement wins (none: the most agreeing);
 *   4. the winner is timed at scan_blocks_per_cu 1, 2 and 0 (full) and the fastest kept (the
 *      launch shape does not change results).
 * Delta_d and the round shape change which candidates are rejected, so they are part of the
 * result's definition: record them with the results (the oracle takes the same values).
 * Q, k_per_query, nprobe_per_query: as dade_search (device).  opts: in, the base options (mode
 * must be DADE; rerank_delta and use_graph are kept); out, the chosen options.  results (host,
 * nullable): one entry per configuration tried, at most DADE_TUNE_MAX; *n_results (nullable) their
 * count.  Requires a CALIBRATED index, nq >= 1, reps >= 1 (0 means 5), 0 <= min_agreement <= 1.
 * Temporary device buffers (two [nq x k] result sets) count against the index's HBM budget.
 * Synchronises `stream`.
 */
#define DADE_TUNE_MAX 24
typedef struct {
  int32_t delta_d;
  int32_t schedule;
  int32_t fill_min;
  int32_t growth;
  int32_t scan_blocks_per_cu;
  float ms;                 /* mean duration of one search of the sample */
  float agreement;          /* with the FULL_D reference, in [0, 1] */
} dade_tune_result;

int dade_autotune(dade_index* ix, const float* Q, int64_t nq, int32_t k, int32_t nprobe,
                  const int32_t* k_per_query, const int32_t* nprobe_per_query, float min_agreement,
                  int32_t reps, dade_search_opts* opts, dade_tune_result* results, int32_t* n_results,
                  void* stream);

/*
 * Graph search (the paper's graph setting: HNSW with DADE DCOs, Experiments).  The paper's HNSW
 * scans the neighbours of the objects it visits and gives each one DCO against the maximum of
 * its result set (size ef), discarding a neighbour whose DCO answers no.  This engine runs that
 * search on a one-layer graph:
 *
 * dade_graph_build -- the graph of a ROTATED index.  With candidates = 0, each row's `degree`
 * out-neighbours are its degree nearest other rows by this index's FDScanning search (K = degree
 * + 1 over `nprobe` lists, ties by id, the row itself dropped).  With candidates in [degree, 127],
 * the FDScanning search returns each row's `candidates` nearest other rows instead, and its
 * out-neighbours are those that HNSW's neighbour-selection heuristic keeps (Malkov and Yashunin,
 * the simple form): candidates taken in ascending (squared distance in FP64 over the FP32
 * vectors, row id) order, one pruned when a neighbour kept before it is strictly closer to it
 * than the row is, at most `degree` kept (fewer when it prunes; -1 padded).  This selection runs
 * on the host over all rows (threads).  The out-neighbours are followed by up to `reverse` back
 * links: rows that list it and that it does not list, nearest first by (squared distance in FP64
 * over the FP32 vectors, row id); rows are degree + reverse (<= 64) wide, -1 padded.  The entry
 * points of the IVF lists stand in for HNSW's upper layers.  Each list has two entry
 * points: its medoid (the member nearest its centroid in FP32, ties to the lower id) and the
 * member farthest from the medoid (ties to the lower id; -1 for a list of one).  The queries of
 * the FDScanning search are the index's own copy of the vectors it was built from, so row i is
 * searched as row i.  Replaces a previous graph.
 * Requires n <= 20000 (DADE_EINVAL above): larger builds are switched off while a GPU fault seen
 * in a 1M-row build is unexplained.  Synchronises `stream`.
 *
 * dade_graph_search -- per query, a beam of at most ef (1..64) (squared distance, id) entries:
 * seeded with the entry points of the query's n_entry (1..32) nearest lists at their full-D
 * distance; each step expands the nearest unexpanded entry: its unvisited neighbours are
 * marked visited and each gets one DCO (Algorithm 1 at opts->delta_d, a multiple of 8, or
 * FDScanning in FULL_D mode) against the beam's ef-th entry as it was when the step began
 * (no test while the beam holds fewer than ef), kept as dade_search keeps candidates, and
 * merged in (the ef nearest stay).  The search ends when every beam entry is expanded or after
 * max_iters steps (0 means 2 ef; 2 n_entry + max_iters x width must be <= 4096).  The beam
 * uses the stored coordinates; the final beam is reranked with the original FP32 vectors and
 * the k (<= ef) nearest by (squared distance, id) are returned as dade_search returns them.
 * opts: delta_d, mode and stats (device [nq x 4] int64: DCOs, dimensions read, steps, visited)
 * are used; NULL means DADE at Delta_d 32.  Q: device [nq x dim] FP32.  Asynchronous on `stream`.
 *
 * dade_graph_export -- the graph as row ids (host): *degree, the row width (degree + reverse);
 * neighbors [n x width] (row i's neighbours), entries [nlist x 2] (-1 where a list has no
 * such member); NULL arrays are skipped.
 */
int dade_graph_build(dade_index* ix, int32_t degree, int32_t reverse, int32_t nprobe, int32_t candidates,
                     void* stream);
int dade_graph_search(dade_index* ix, const float* Q, int64_t nq, int32_t k, int32_t ef, int32_t n_entry,
                      int32_t max_iters, const dade_search_opts* opts, int64_t* out_ids, float* out_dist2,
                      void* stream);
int dade_graph_export(const dade_index* ix, int32_t* degree, int64_t* neighbors, int64_t* entries);

/* dade_destroy -- free the index and all its device memory (NULL is a no-op). */
void dade_destroy(dade_index* ix);

/* dade_last_error -- message of the calling thread's last failed call ("" if none). */
const char* dade_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DADE_H */
