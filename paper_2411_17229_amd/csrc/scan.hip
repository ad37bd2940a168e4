// The DADE list scan: Algorithm 1 for every candidate of a query's probed lists, the
// size-K heap of the IVF scan (end of the Methodology section) and, for low-precision
// stores, an exact FP32 rerank of the survivors.
//
// Execution model (one persistent launch for the whole batch):
//   * a 256-thread workgroup owns one query at a time, pulled from a global counter, and
//     walks its probe ranks round by round; a round's DCOs all use the heap as it was when
//     the round started (thresholds r^2 and T_d r^2 are fixed for the round), and the round's
//     kept candidates are merged into the top-K in LDS at its end.  Queries never wait for
//     one another, so results do not depend on the batch.
//   * the partial distance of a DCO is always summed in one order: each 8-coordinate unit's
//     squared differences by an FMA chain from zero, then S_d = S_{d-8} + unit sum, unit after
//     unit.  Every code path below keeps that order, so a DCO's S_d (and decision) does not
//     depend on which path ran it, on the tile shape or on the rest of the batch.
//   * dense rounds (heap not yet full, so no test can reject, or FDScanning mode): 16 lanes
//     cooperate on one candidate and fetch up to 512 coordinates of its row per step.
//   * rounds with a full heap: one lane per candidate reads the row up to the first test
//     d = Delta_d (64-byte loads) and tests S_d > T_d r^2 (Eq. (13) + the hypothesis test in
//     reduced form); almost every far candidate stops here.  The survivors go to an LDS queue
//     that 16-lane groups process with wide loads, replaying the remaining tests in order
//     (d = 2 Delta_d, 3 Delta_d, ... below D) and stopping at the first rejection.
//   * at d = D a candidate is kept iff the heap is not full or (S_D, id) < (r^2, id_r).
//   * low-precision stores: a survivor is queued with its stored-precision S_D when the heap
//     is not full or S_D <= (1 + delta) r^2.  After the round the K smallest queued keys are
//     reranked exactly (FP32, from the original vectors); with b the K-th smallest exact
//     distance of the heap and those, the other queued candidates are reranked only where
//     S_D <= (1 + delta) b; the keep rule then applies to the exact values.
#include "kernels.h"

namespace dade {
namespace {

constexpr int kThreads = 256;
constexpr int kGroup = 16;                    // lanes per candidate in the cooperative paths
constexpr int kGroups = kThreads / kGroup;
constexpr int kMaxUnitsPerLane = 8;           // 8-coordinate units a lane fetches per group step
constexpr int kMaxRoundLists = 64;            // lists handled together inside one round
constexpr int kMergeChunk = 512;              // queued keys handled per LDS pass
constexpr int kQueueLds = 512;                // queued keys kept in LDS (more spill to global)
constexpr int kDeepCap = 2 * kThreads;        // first-test survivors of one pass, for the groups
constexpr int kPreloadProbes = 128;           // probed lists whose offsets are kept in LDS
constexpr int kDenseGroupMax = 64;            // dense rounds up to this size use 16-lane groups

// ---- stored-coordinate access ---------------------------------------------------------------
// A unit is 8 consecutive coordinates; a chunk is the 64 bytes one lane loads at a time.
template <typename ST>
struct Store;

template <>
struct Store<float> {
  static constexpr int CH = 16;  // coordinates per chunk
  static constexpr int R = 4;    // units per lane per group step (512 coordinates per step)
  struct Chunk { float4 x[4]; };
  __device__ static inline Chunk load_chunk(const void* base, int64_t pos, int dp, int g) {
    const float4* p = reinterpret_cast<const float4*>(static_cast<const float*>(base) + pos * dp + g * CH);
    return Chunk{{p[0], p[1], p[2], p[3]}};
  }
  __device__ static inline void chunk_unit(const Chunk& c, int i, float* v) {
    const float4 a = c.x[2 * i], b = c.x[2 * i + 1];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  }
  struct Raw { float4 a, b; };
  __device__ static inline Raw unit_raw(const void* base, int64_t pos, int dp, int u) {
    const float4* p = reinterpret_cast<const float4*>(static_cast<const float*>(base) + pos * dp + 8 * u);
    return Raw{p[0], p[1]};
  }
  __device__ static inline void unit_vals(const Raw& r, float* v) {
    v[0] = r.a.x; v[1] = r.a.y; v[2] = r.a.z; v[3] = r.a.w;
    v[4] = r.b.x; v[5] = r.b.y; v[6] = r.b.z; v[7] = r.b.w;
  }
};

template <bool BF16>
struct Store16 {
  static constexpr int CH = 32;
  static constexpr int R = 8;    // units per lane per group step (1024 coordinates per step)
  struct Chunk { uint4 x[4]; };
  __device__ static inline void words(const uint4& r, float* v) {
    const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (BF16) {
        v[2 * j + 0] = __builtin_bit_cast(float, w[j] << 16);
        v[2 * j + 1] = __builtin_bit_cast(float, w[j] & 0xFFFF0000u);
      } else {
        v[2 * j + 0] = float(__builtin_bit_cast(_Float16, uint16_t(w[j] & 0xFFFFu)));
        v[2 * j + 1] = float(__builtin_bit_cast(_Float16, uint16_t(w[j] >> 16)));
      }
    }
  }
  __device__ static inline Chunk load_chunk(const void* base, int64_t pos, int dp, int g) {
    const uint4* p = reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(base) + pos * dp + g * CH);
    return Chunk{{p[0], p[1], p[2], p[3]}};
  }
  __device__ static inline void chunk_unit(const Chunk& c, int i, float* v) { words(c.x[i], v); }
  using Raw = uint4;
  __device__ static inline Raw unit_raw(const void* base, int64_t pos, int dp, int u) {
    return *reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(base) + pos * dp + 8 * u);
  }
  __device__ static inline void unit_vals(const Raw& r, float* v) { words(r, v); }
};

template <>
struct Store<__hip_bfloat16> : Store16<true> {};
template <>
struct Store<__half> : Store16<false> {};

// FMA chain of one unit's squared differences, from zero.
__device__ inline float unit_sum(const float* q, const float* v) {
  float p = 0.f;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const float df = q[i] - v[i];
    p = fmaf(df, df, p);
  }
  return p;
}

__device__ inline void q8(const float* qs, int d, float* q) {
  const float4 a = *reinterpret_cast<const float4*>(qs + d);
  const float4 b = *reinterpret_cast<const float4*>(qs + d + 4);
  q[0] = a.x; q[1] = a.y; q[2] = a.z; q[3] = a.w; q[4] = b.x; q[5] = b.y; q[6] = b.z; q[7] = b.w;
}

// Reads that bypass the CU's L1, for keys other waves of the workgroup wrote to global memory.
__device__ inline unsigned long long load_l2(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One DCO continued by a 16-lane group from unit u_start with running sum S.  Every lane of the
// group fetches Store<ST>::R units per step; the unit sums are staged in the group's LDS slice
// (gs, kGroup * kMaxUnitsPerLane floats) in unit order, and every lane then adds them
// one by one, replaying the tests.  Returns the d at which the DCO ended (rejected, or
// d >= dim) and updates S.  Control flow is uniform within the group.
template <typename ST, bool DADE>
__device__ int group_dco(const void* store, int64_t pos, int dp, int dim, const float* qs,
                         const float* thr, int dd, int u_start, float& S, bool& rejected, int gl,
                         float* gs) {
  using SS = Store<ST>;
  constexpr int R = SS::R;
  constexpr int kStep = kGroup * R;
  const int units = dp >> 3;
  const int u_end = (dim + 7) >> 3;          // units that hold real coordinates
  int u0 = u_start;
  rejected = false;
  int next_test = DADE ? (8 * u_start / dd + 1) * dd : 0;   // first tested d after u_start
  int ti = DADE ? next_test / dd - 1 : 0;
  while (u0 < u_end) {
    typename SS::Raw raw[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {   // clamped, unconditional: all loads in flight
      const int u = u0 + r * kGroup + gl;
      raw[r] = SS::unit_raw(store, pos, dp, u < units ? u : units - 1);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int u = u0 + r * kGroup + gl;
      const int uc = u < units ? u : units - 1;
      float v[8], q[8];
      SS::unit_vals(raw[r], v);
      q8(qs, 8 * uc, q);
      gs[r * kGroup + gl] = unit_sum(q, v);   // units past u_end are never read back
    }
    __builtin_amdgcn_wave_barrier();
    const int n = (u_end - u0 < kStep) ? u_end - u0 : kStep;
    for (int i = 0; i < n; i += 4) {
      const float4 w = *reinterpret_cast<const float4*>(gs + i);
      const float wv[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (i + t < n) {
          S = S + wv[t];
          if (DADE) {
            const int d = 8 * (u0 + i + t + 1);
            if (d == next_test) {
              if (d < dim && S > thr[ti]) {
                rejected = true;
                __builtin_amdgcn_wave_barrier();
                return d;
              }
              next_test += dd;
              ++ti;
            }
          }
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
    u0 += kStep;
  }
  return dim;
}

// heap[0..heap_n) (ascending keys) <- the K smallest of heap and cand[0..n); keys are unique,
// so each key's rank is the count of smaller keys.  cand must have room for n + K entries.
// Ends with a barrier.
__device__ void merge_into(unsigned long long* heap, int& heap_n, unsigned long long* tmp,
                           unsigned long long* cand, int n, int K, int tid) {
  if (n > 0) {
    for (int i = tid; i < heap_n; i += kThreads) cand[n + i] = heap[i];
    __syncthreads();
    const int tot = n + heap_n;
    for (int i = tid; i < tot; i += kThreads) {
      const unsigned long long key = cand[i];
      int rank = 0;
      for (int j = 0; j < tot; ++j) rank += cand[j] < key;
      if (rank < K) tmp[rank] = key;
    }
    __syncthreads();
    heap_n = tot < K ? tot : K;
    for (int i = tid; i < heap_n; i += kThreads) heap[i] = tmp[i];
  }
  __syncthreads();
}

// keys[i] (stored-precision S_D, id) -> (exact FP32 S_D, id), one 16-lane group per key, in the
// canonical unit order over the original vector.  Ends with a barrier.
__device__ void exact_rerank(unsigned long long* keys, int n, const float* __restrict__ X,
                             const float* qo, int dp, int dim, int tid, unsigned& count,
                             float* gsum) {
  const int grp = tid / kGroup, gl = tid % kGroup;
  float* gs = gsum + grp * kGroup * kMaxUnitsPerLane;
  for (int i = grp; i < n; i += kGroups) {
    const uint32_t id = key_id(keys[i]);
    float S = 0.f;
    bool rej;
    group_dco<float, false>(X, int64_t(id), dp, dim, qo, nullptr, 1, 0, S, rej, gl, gs);
    if (gl == 0) {
      keys[i] = make_key(S, id);
      ++count;
    }
  }
  __syncthreads();
}

template <typename ST, bool DADE, bool RERANK, bool PER_DIM_TESTS>
__global__ __launch_bounds__(kThreads, 4) void scan_kernel(ScanArgs a) {
  using SS = Store<ST>;
  constexpr int CH = SS::CH;
  extern __shared__ float dyn[];
  float* qs = dyn;                              // [dp] rotated query
  float* qo = dyn + a.dp;                       // [dp] original query (RERANK only)
  float* thr = dyn + (RERANK ? 2 : 1) * a.dp;   // [ntests] T_d r^2 for the round

  __shared__ unsigned long long topk[kMaxK];
  __shared__ unsigned long long newk[kMaxK];
  __shared__ unsigned long long fk[RERANK ? kMaxK : 1];
  __shared__ unsigned long long cand[kMergeChunk + kMaxK];
  __shared__ int64_t lst_pos[kMaxRoundLists];
  __shared__ int lst_pre[kMaxRoundLists + 1];
  __shared__ int64_t pl_pos[kPreloadProbes];
  __shared__ int pl_len[kPreloadProbes];
  __shared__ int64_t dq_pos[kDeepCap];          // deep queue: survivors of the first test
  __shared__ uint32_t dq_id[kDeepCap];
  __shared__ float dq_S[kDeepCap];
  __shared__ float gsum[kThreads * kMaxUnitsPerLane];   // per-group unit sums (cooperative paths)
  __shared__ unsigned long long qkeys[kQueueLds];      // the round's queued keys
  __shared__ int s_q, s_acc, s_nc, s_ndeep, s_t1, s_off1;
  __shared__ unsigned long long s_b;
  __shared__ unsigned long long s_stat[4];

  const int tid = threadIdx.x;
  const int grp = tid / kGroup, gl = tid % kGroup;
  float* gs = gsum + grp * kGroup * kMaxUnitsPerLane;
  const int dim = a.dim, dp = a.dp, dd = a.delta_d;
  const int ntests = (dim - 1) / dd;
  // lane-serial part of a full-heap round: up to the first test
  const int a_chunks = (dd + CH - 1) / CH;
  unsigned long long* acc = a.acc_buf + int64_t(blockIdx.x) * a.acc_cap;

  for (;;) {
    if (tid == 0) s_q = atomicAdd(a.counter, 1);
    __syncthreads();
    const int qi = s_q;
    if (qi >= a.nq) break;
    int K = a.k_pq ? a.k_pq[qi] : a.k_max;
    K = K < 1 ? 1 : (K > a.k_max ? a.k_max : K);
    int np = a.nprobe_pq ? a.nprobe_pq[qi] : a.nprobe_max;
    np = np < 1 ? 1 : (np > a.nprobe_max ? a.nprobe_max : np);
    for (int c = tid; c < dp; c += kThreads) {
      qs[c] = a.qrot[int64_t(qi) * dp + c];
      if (RERANK) qo[c] = a.qorig[int64_t(qi) * dp + c];
    }
    for (int t = tid; t < np && t < kPreloadProbes; t += kThreads) {
      const int l = a.probes[int64_t(qi) * a.nprobe_max + t];
      const int64_t o0 = a.list_off[l];
      pl_pos[t] = o0;
      pl_len[t] = int(a.list_off[l + 1] - o0);
    }
    if (tid < 4) s_stat[tid] = 0;
    int topk_n = 0;
    unsigned st_dco = 0, st_dims = 0, st_kept = 0, st_rr = 0;   // per thread, per query
    __syncthreads();

    auto list_info = [&](int tt, int64_t& p0, int& len) {
      if (tt < kPreloadProbes) {
        p0 = pl_pos[tt];
        len = pl_len[tt];
      } else {
        const int l = a.probes[int64_t(qi) * a.nprobe_max + tt];
        p0 = a.list_off[l];
        len = int(a.list_off[l + 1] - p0);
      }
    };
    // round cursor: probe rank t and offset inside that list
    int t = 0, off = 0;
    bool fill = true;
    while (t < np) {
      // ---- round extent [(t, off), (t1, off1)): the first round holds the first K candidates
      //      (they fill the heap); later rounds end where the schedule's probe ranks end
      if (tid == 0) {
        int t1 = t + 1, off1 = 0;
        if (fill) {
          int rem = K, tt = t, oo = off;
          while (rem > 0 && tt < np) {
            int64_t p0;
            int len;
            list_info(tt, p0, len);
            if (len - oo > rem) {
              oo += rem;
              rem = 0;
            } else {
              rem -= len - oo;
              ++tt;
              oo = 0;
            }
          }
          t1 = tt;
          off1 = oo;
        } else if (a.schedule != 0) {
          int B = 1;
          while (B <= t) B <<= 1;
          t1 = B < np ? B : np;
        }
        s_t1 = t1;
        s_off1 = off1;
      }
      // ---- round snapshot
      const bool full = topk_n == K;
      const unsigned long long keyr = full ? topk[K - 1] : ~0ull;
      const float r2 = full ? key_dist(keyr) : __builtin_inff();
      const float gate = (1.f + a.rerank_delta) * r2;
      const bool dense = !DADE || !full || ntests == 0;
      if (DADE)
        for (int j = tid; j < ntests; j += kThreads) thr[j] = a.T[(j + 1) * dd - 1] * r2;
      if (tid == 0) s_acc = 0;
      __syncthreads();
      const int t1 = s_t1, off1 = s_off1;
      const int t_last = off1 > 0 ? t1 : t1 - 1;   // last probe rank the round touches

      // queue a finished DCO (FP32 store: the keep rule; low precision: the rerank gate)
      bool wrote_global = false;
      auto finish = [&](float S, uint32_t rid) {
        const bool queue = RERANK ? (!full || S <= gate) : (!full || make_key(S, rid) < keyr);
        if (queue) {
          const int slot = atomicAdd(&s_acc, 1);
          if (slot < kQueueLds) {
            qkeys[slot] = make_key(S, rid);
          } else if (slot - kQueueLds < a.acc_cap) {
            acc[slot - kQueueLds] = make_key(S, rid);
            wrote_global = true;
          } else {
            atomicOr(a.overflow, 1);
          }
        }
      };

      for (int lb = t; lb <= t_last; lb += kMaxRoundLists) {
        const int le = (t_last + 1 - lb < kMaxRoundLists) ? t_last + 1 : lb + kMaxRoundLists;
        const int nl = le - lb;
        if (tid < 64) {   // the round's segment of each list and an exclusive prefix (one wave)
          int len = 0;
          int64_t p0 = 0;
          if (tid < nl) {
            const int tt = lb + tid;
            int L;
            list_info(tt, p0, L);
            const int s0 = (tt == t) ? off : 0;
            const int s1 = (tt == t1) ? off1 : L;
            p0 += s0;
            len = s1 - s0;
          }
          int incl = len;
#pragma unroll
          for (int o = 1; o < 64; o <<= 1) {
            const int v = __shfl_up(incl, o, 64);
            if (tid >= o) incl += v;
          }
          if (tid < nl) {
            lst_pos[tid] = p0;
            lst_pre[tid] = incl - len;
          }
          if (tid == nl - 1) lst_pre[nl] = incl;
        }
        __syncthreads();
        const int total = lst_pre[nl];
        auto locate = [&](int cc, int64_t& pos, uint32_t& rid) {
          int lo = 0, hi = nl - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (lst_pre[mid] <= cc) lo = mid; else hi = mid - 1;
          }
          pos = lst_pos[lo] + (cc - lst_pre[lo]);
          rid = uint32_t(a.ids[pos]);
        };

        if (PER_DIM_TESTS && !dense) {
          // ---- Delta_d not a multiple of 8: one lane per candidate, tests inside units
          for (int c = tid; c < total; c += kThreads) {
            int64_t pos;
            uint32_t rid;
            locate(c, pos, rid);
            float S = 0.f;
            int next_test = dd, ti = 0, dexit = dim;
            bool rej = false;
            for (int u = 0; u < (dim + 7) / 8 && !rej; ++u) {
              const typename SS::Raw raw = SS::unit_raw(a.store, pos, dp, u);
              float v[8], q[8];
              SS::unit_vals(raw, v);
              q8(qs, 8 * u, q);
              float p = 0.f;
              for (int i = 0; i < 8; ++i) {
                const float df = q[i] - v[i];
                p = fmaf(df, df, p);
                const int d = 8 * u + i + 1;
                if (!rej && d == next_test && d < dim) {
                  if (S + p > thr[ti]) { rej = true; dexit = d; }
                  ++ti;
                  next_test += dd;
                }
              }
              S = S + p;
            }
            ++st_dco;
            st_dims += unsigned(dexit);
            if (!rej) finish(S, rid);
          }
        } else if (dense && total > kDenseGroupMax) {
          // ---- dense round, many candidates: one lane per candidate, the next 64-byte chunk
          //      in flight while the current one is summed
          const int nch = (dim + CH - 1) / CH;
          for (int c = tid; c < total; c += kThreads) {
            int64_t pos;
            uint32_t rid;
            locate(c, pos, rid);
            float S = 0.f;
            typename SS::Chunk cur = SS::load_chunk(a.store, pos, dp, 0);
            for (int g = 0; g < nch; ++g) {
              const typename SS::Chunk nxt = SS::load_chunk(a.store, pos, dp, g + 1 < nch ? g + 1 : g);
#pragma unroll
              for (int i = 0; i < CH / 8; ++i) {
                float v[8], q[8];
                SS::chunk_unit(cur, i, v);
                q8(qs, g * CH + 8 * i, q);
                S = S + unit_sum(q, v);
              }
              cur = nxt;
            }
            ++st_dco;
            st_dims += unsigned(dim);
            finish(S, rid);
          }
        } else if (dense) {
          // ---- dense round, few candidates (the fill round): 16 lanes per candidate
          for (int c = grp; c < total; c += kGroups) {
            int64_t pos;
            uint32_t rid;
            locate(c, pos, rid);
            float S = 0.f;
            bool rej;
            const int dexit = group_dco<ST, false>(a.store, pos, dp, dim, qs, thr, dd, 0, S, rej, gl, gs);
            if (gl == 0) {
              ++st_dco;
              st_dims += unsigned(dexit);
              finish(S, rid);
            }
          }
        } else {
          // ---- full heap: passes of 2 x 256 candidates; each lane tests two candidates up to
          //      the first test (both first chunks in flight), survivors go to the deep queue,
          //      which the 16-lane groups drain after the pass
          for (int cb = 0; cb < total; cb += 2 * kThreads) {
            if (tid == 0) s_ndeep = 0;
            __syncthreads();
            const int c0 = cb + tid, c1 = cb + kThreads + tid;
            int64_t pos0, pos1;
            uint32_t rid0, rid1;
            locate(c0 < total ? c0 : total - 1, pos0, rid0);      // clamped: always a valid row
            locate(c1 < total ? c1 : total - 1, pos1, rid1);
            const typename SS::Chunk ch0 = SS::load_chunk(a.store, pos0, dp, 0);
            const typename SS::Chunk ch1 = SS::load_chunk(a.store, pos1, dp, 0);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const int c = h ? c1 : c0;
              if (c >= total) continue;
              const int64_t pos = h ? pos1 : pos0;
              const uint32_t rid = h ? rid1 : rid0;
              float S = 0.f;
              bool rej = false;
              int dexit = dim, next_test = dd, ti = 0;
              int g = 0;
              for (; g < a_chunks && !rej; ++g) {
                const typename SS::Chunk ch = g == 0 ? (h ? ch1 : ch0) : SS::load_chunk(a.store, pos, dp, g);
#pragma unroll
                for (int i = 0; i < CH / 8; ++i) {
                  if (!rej) {
                    float v[8], q[8];
                    SS::chunk_unit(ch, i, v);
                    q8(qs, g * CH + 8 * i, q);
                    S = S + unit_sum(q, v);
                    const int d = g * CH + 8 * i + 8;
                    if (d == next_test && d < dim) {
                      if (S > thr[ti]) { rej = true; dexit = d; }
                      ++ti;
                      next_test += dd;
                    }
                  }
                }
              }
              if (rej || g * CH >= dim) {
                ++st_dco;
                st_dims += unsigned(dexit);
                if (!rej) finish(S, rid);
              } else {
                const int slot = atomicAdd(&s_ndeep, 1);   // < 2 * kThreads <= kDeepCap
                dq_pos[slot] = pos;
                dq_id[slot] = rid;
                dq_S[slot] = S;
              }
            }
            __syncthreads();
            const int nd = s_ndeep;
            for (int j = grp; j < nd; j += kGroups) {
              float S = dq_S[j];
              bool rej;
              const int dexit = group_dco<ST, true>(a.store, dq_pos[j], dp, dim, qs, thr, dd,
                                                    a_chunks * CH / 8, S, rej, gl, gs);
              if (gl == 0) {
                ++st_dco;
                st_dims += unsigned(dexit);
                if (!rej) finish(S, dq_id[j]);
              }
            }
            __syncthreads();
          }
        }
        __syncthreads();
      }
      if (wrote_global) __threadfence();   // spilled queue keys reach L2 before others read them
      __syncthreads();

      const int m = s_acc < kQueueLds + a.acc_cap ? s_acc : int(kQueueLds + a.acc_cap);
      auto queued = [&](int i) -> unsigned long long {
        return i < kQueueLds ? qkeys[i] : load_l2(acc + (i - kQueueLds));
      };
      if (!RERANK) {
        // ---- merge the round's kept keys into the top-K
        for (int base = 0; base < m; base += kMergeChunk) {
          const int cnt = (m - base < kMergeChunk) ? m - base : kMergeChunk;
          const unsigned long long kth = (topk_n == K) ? topk[K - 1] : ~0ull;
          if (tid == 0) s_nc = 0;
          __syncthreads();
          for (int i = tid; i < cnt; i += kThreads) {
            const unsigned long long key = queued(base + i);
            if (key < kth) cand[atomicAdd(&s_nc, 1)] = key;
          }
          __syncthreads();
          st_kept += (tid == 0) ? unsigned(s_nc) : 0u;
          merge_into(topk, topk_n, newk, cand, s_nc, K, tid);
        }
      } else if (m > 0) {
        // ---- F = the K smallest queued keys (stored-precision S_D, id), into cand[0..fn)
        int fn = 0;
        unsigned long long fmax = ~0ull;
        if (m <= K) {
          for (int i = tid; i < m; i += kThreads) cand[i] = queued(i);
          fn = m;
          __syncthreads();
        } else {
          for (int base = 0; base < m; base += kMergeChunk) {
            const int cnt = (m - base < kMergeChunk) ? m - base : kMergeChunk;
            const unsigned long long kth = (fn == K) ? fk[K - 1] : ~0ull;
            if (tid == 0) s_nc = 0;
            __syncthreads();
            for (int i = tid; i < cnt; i += kThreads) {
              const unsigned long long key = queued(base + i);
              if (key < kth) cand[atomicAdd(&s_nc, 1)] = key;
            }
            __syncthreads();
            merge_into(fk, fn, newk, cand, s_nc, K, tid);
          }
          fmax = fk[fn - 1];
          for (int i = tid; i < fn; i += kThreads) cand[i] = fk[i];
          __syncthreads();
        }
        exact_rerank(cand, fn, a.X, qo, dp, dim, tid, st_rr, gsum);
        // b = K-th smallest exact key of the heap snapshot and F
        if (tid == 0) s_b = ~0ull;
        __syncthreads();
        if (topk_n + fn >= K) {
          for (int i = tid; i < topk_n + fn; i += kThreads) {
            const unsigned long long key = i < topk_n ? topk[i] : cand[i - topk_n];
            int rank = 0;
            for (int j = 0; j < topk_n; ++j) rank += topk[j] < key;
            for (int j = 0; j < fn; ++j) rank += cand[j] < key;
            if (rank == K - 1) s_b = key;
          }
        }
        __syncthreads();
        const float bound = (s_b == ~0ull) ? __builtin_inff() : (1.f + a.rerank_delta) * key_dist(s_b);
        if (tid == 0) {
          int w = 0;
          for (int i = 0; i < fn; ++i)
            if (!full || cand[i] < keyr) cand[w++] = cand[i];
          s_nc = w;
          st_kept += unsigned(w);
        }
        __syncthreads();
        merge_into(topk, topk_n, newk, cand, s_nc, K, tid);
        // the rest of the queue, reranked only inside the bound
        for (int base = 0; m > K && base < m; base += kMergeChunk) {
          const int cnt = (m - base < kMergeChunk) ? m - base : kMergeChunk;
          if (tid == 0) s_nc = 0;
          __syncthreads();
          for (int i = tid; i < cnt; i += kThreads) {
            const unsigned long long key = queued(base + i);
            if (key > fmax && key_dist(key) <= bound) cand[atomicAdd(&s_nc, 1)] = key;
          }
          __syncthreads();
          const int nr = s_nc;
          __syncthreads();
          if (nr == 0) continue;
          exact_rerank(cand, nr, a.X, qo, dp, dim, tid, st_rr, gsum);
          if (tid == 0) {
            int w = 0;
            for (int i = 0; i < nr; ++i)
              if (!full || cand[i] < keyr) cand[w++] = cand[i];
            s_nc = w;
            st_kept += unsigned(w);
          }
          __syncthreads();
          merge_into(topk, topk_n, newk, cand, s_nc, K, tid);
        }
      }
      t = t1;
      off = off1;
      fill = false;
    }

    // ---- output row: ascending (dist2, id), padded with (-1, +inf)
    for (int j = tid; j < a.k_max; j += kThreads) {
      const int64_t o = int64_t(qi) * a.k_max + j;
      if (j < topk_n) {
        a.out_ids[o] = int64_t(key_id(topk[j]));
        a.out_d2[o] = key_dist(topk[j]);
      } else {
        a.out_ids[o] = -1;
        a.out_d2[o] = __builtin_inff();
      }
    }
    if (a.stats) {
      atomicAdd(&s_stat[0], (unsigned long long)st_dco);
      atomicAdd(&s_stat[1], (unsigned long long)st_dims);
      atomicAdd(&s_stat[2], (unsigned long long)st_kept);
      atomicAdd(&s_stat[3], (unsigned long long)st_rr);
      __syncthreads();
      if (tid < 4) a.stats[int64_t(qi) * 4 + tid] = int64_t(s_stat[tid]);
    }
    __syncthreads();
  }
}

template <typename ST, bool DADE, bool RERANK>
hipError_t launch_typed(const ScanArgs& a, hipStream_t s) {
  const int ntests = (a.dim - 1) / a.delta_d;
  const size_t lds = sizeof(float) * (size_t(RERANK ? 2 : 1) * a.dp + size_t(ntests > 0 ? ntests : 1));
  const bool per_dim = DADE && (a.delta_d % 8 != 0);
  if (per_dim)
    hipLaunchKernelGGL((scan_kernel<ST, DADE, RERANK, true>), dim3(a.grid), dim3(kThreads), lds, s, a);
  else
    hipLaunchKernelGGL((scan_kernel<ST, DADE, RERANK, false>), dim3(a.grid), dim3(kThreads), lds, s, a);
  return hipGetLastError();
}

template <typename ST>
hipError_t launch_mode(const ScanArgs& a, int mode, bool rerank, hipStream_t s) {
  if (mode == 0)
    return rerank ? launch_typed<ST, true, true>(a, s) : launch_typed<ST, true, false>(a, s);
  return rerank ? launch_typed<ST, false, true>(a, s) : launch_typed<ST, false, false>(a, s);
}

}  // namespace

hipError_t launch_scan(const ScanArgs& a, int dtype, int mode, hipStream_t s) {
  if (a.nq == 0) return hipSuccess;
  if (dtype == 0) return launch_mode<float>(a, mode, false, s);
  if (dtype == 1) return launch_mode<__hip_bfloat16>(a, mode, true, s);
  return launch_mode<__half>(a, mode, true, s);
}

}  // namespace dade
