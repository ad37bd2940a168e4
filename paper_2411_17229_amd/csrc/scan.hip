// The DADE list scan: Algorithm 1 for every candidate of every query's probed lists, the size-K
// heap of the IVF scan (end of the Methodology section) and, for low-precision stores, an exact
// FP32 rerank of the survivors.
//
// Rounds.  A query's candidate sequence (its probed lists in probe order) is cut into rounds:
// the first round is its first max(K, fill_min) candidates (they fill the heap), later rounds
// end where the schedule's probe ranks end (every rank, ranks 1, 2, 4, 8, ..., or only the last) or once they
// hold growth times the candidates scanned before them.  Every DCO of a round sees
// the query's heap as it was when the round started (r^2 and the thresholds T_d r^2 are a
// snapshot), and the round's kept candidates are merged at its end.  Queries never interact, so
// a query's result does not depend on the batch or on how the work is spread over the GPU.
//
// A plan (count pass, per-round prefix sums, write pass) lays out every query's work items for
// every round before the first DCO: round cuts depend only on list sizes, K and the schedule.
// Then the rounds run for all queries at once, two kernels per round:
//   * scan_round: a persistent grid whose waves pull work items (one query, up to 64
//     consecutive candidates of one list, and the query's snapshot).  One lane per candidate
//     reads the head block (coordinates [0, 32), contiguous across a list) and tests
//     S_d > T_d r^2 at d = Delta_d (Eq. (13) with the hypothesis test in reduced form); a far
//     candidate stops there.  A survivor goes on a per-wave LDS stack and is continued later in
//     levels of growing size (all loads of a level in flight at once), each level replaying the
//     tests it covers in order: 64 survivors at a time, one lane each, while items remain; a
//     quad of lanes per survivor once the items are done and at most 16 are left.  Rounds whose
//     heap is not yet full (no test can reject) and FDScanning read whole rows; items of at
//     most 16 candidates take four lanes per row and read the query's chunks from the wave's
//     LDS slice, filled step by step beside the row loads.
//   * merge_round: one workgroup per query merges the round's queued keys into its top-K (for
//     low-precision stores through the rerank rule below), takes the snapshot for the next
//     round and writes it into the query's work items of that round; after the query's last
//     round it writes the output row.
// A DCO's partial distance is summed in one order on every path: each 8-coordinate unit's
// squared differences by an FMA chain from zero, then S_d = S_{d-8} + unit sum, unit after unit.
// Low-precision stores: a survivor is queued with its stored-precision S_D when the heap is not
// full or S_D <= (1 + delta) r^2.  At the merge the plain rule reranks every queued candidate
// exactly (FP32, from the original vectors); the lazy rule reranks the K smallest queued keys
// and, with b the K-th smallest exact distance of the heap and those, the other queued
// candidates only where S_D <= (1 + delta) b.  The keep rule (heap not full, or (S_D, id) <
// (r^2, id_r)) then applies to exact values.
#include "kernels.h"

namespace dade {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kStack = 128;        // deep-stack entries per wave (at most 127 are live)
constexpr int kItem = 64;          // candidates per work item
constexpr int kDenseItem = 16;     // candidates per work item of a whole-row round
constexpr int kMergeChunk = 512;   // queued keys handled per LDS pass of the merge
constexpr int kHeadKeys = 64;      // queued keys a merge fetches with the query's state
constexpr int kBlock = kHead;      // coordinates per block; block 0 is the head
constexpr int kGroup = 16;         // lanes per candidate in the exact rerank
constexpr int kGroups = kThreads / kGroup;

struct Rows {
  const void* head;
  const void* tail;
  int tw;   // tail row length, dp - kBlock
};

// ---- stored-coordinate blocks (32 coordinates) ----------------------------------------------
template <typename ST>
struct Store;

template <>
struct Store<float> {
  static constexpr int kMaxB = 2;   // blocks per level: 256 bytes in flight per lane
  struct Block { float4 x[8]; };
  __device__ static inline Block load(const Rows& r, int64_t p, int bi) {
    const float* base = bi == 0 ? static_cast<const float*>(r.head) + p * kBlock
                                : static_cast<const float*>(r.tail) + p * r.tw + (bi - 1) * kBlock;
    const float4* v = reinterpret_cast<const float4*>(base);
    Block b;
#pragma unroll
    for (int i = 0; i < 8; ++i) b.x[i] = v[i];
    return b;
  }
  __device__ static inline void unit(const Block& b, int j, float* v) {
    const float4 a = b.x[2 * j], c = b.x[2 * j + 1];
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w; v[4] = c.x; v[5] = c.y; v[6] = c.z; v[7] = c.w;
  }
  // one unit (8 coordinates) of a block, for the quad-per-row levels
  static constexpr int kQuadMaxB = 4;   // blocks per quad level: 128 bytes of rows per lane
  struct Unit { float4 a, b; };
  __device__ static inline Unit load_unit(const Rows& r, int64_t p, int bi, int j) {
    const float* base = bi == 0 ? static_cast<const float*>(r.head) + p * kBlock
                                : static_cast<const float*>(r.tail) + p * r.tw + (bi - 1) * kBlock;
    const float4* v = reinterpret_cast<const float4*>(base + 8 * j);
    return Unit{v[0], v[1]};
  }
  __device__ static inline void unit_of(const Unit& u, float* v) {
    v[0] = u.a.x; v[1] = u.a.y; v[2] = u.a.z; v[3] = u.a.w; v[4] = u.b.x; v[5] = u.b.y; v[6] = u.b.z; v[7] = u.b.w;
  }
};

template <bool BF16>
struct Store16 {
  static constexpr int kMaxB = 4;
  struct Block { uint4 x[4]; };
  __device__ static inline Block load(const Rows& r, int64_t p, int bi) {
    const uint16_t* base = bi == 0 ? static_cast<const uint16_t*>(r.head) + p * kBlock
                                   : static_cast<const uint16_t*>(r.tail) + p * r.tw + (bi - 1) * kBlock;
    const uint4* v = reinterpret_cast<const uint4*>(base);
    Block b;
#pragma unroll
    for (int i = 0; i < 4; ++i) b.x[i] = v[i];
    return b;
  }
  __device__ static inline void unit(const Block& b, int j, float* v) { unit_of(Unit{b.x[j]}, v); }
  // one unit (8 coordinates) of a block, for the quad-per-row levels
  static constexpr int kQuadMaxB = 8;   // blocks per quad level: 128 bytes of rows per lane
  struct Unit { uint4 x; };
  __device__ static inline Unit load_unit(const Rows& r, int64_t p, int bi, int j) {
    const uint16_t* base = bi == 0 ? static_cast<const uint16_t*>(r.head) + p * kBlock
                                   : static_cast<const uint16_t*>(r.tail) + p * r.tw + (bi - 1) * kBlock;
    return Unit{*reinterpret_cast<const uint4*>(base + 8 * j)};
  }
  __device__ static inline void unit_of(const Unit& u, float* v) {
    const uint32_t w[4] = {u.x.x, u.x.y, u.x.z, u.x.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (BF16) {
        v[2 * k + 0] = __builtin_bit_cast(float, w[k] << 16);
        v[2 * k + 1] = __builtin_bit_cast(float, w[k] & 0xFFFF0000u);
      } else {
        v[2 * k + 0] = float(__builtin_bit_cast(_Float16, uint16_t(w[k] & 0xFFFFu)));
        v[2 * k + 1] = float(__builtin_bit_cast(_Float16, uint16_t(w[k] >> 16)));
      }
    }
  }
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

// Lane J's value of this lane's quad (a DPP quad broadcast).
template <int J>
__device__ inline float quad_get(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), J * 0x55, 0xF, 0xF, false));
}

// Bits of m set below this lane.
__device__ inline int lanes_below(unsigned long long m) {
  return int(__builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u)));
}

// One level of a DCO: blocks [b, b + nb) of row p (nb <= NB), with all of their loads issued
// first.  Adds the units below dim to S in the canonical order and, with tests on, rejects at
// the first tested d (a multiple of dd, below dim) where S_d > T_d r^2.
template <typename ST, bool PER_DIM, int NB>
__device__ inline void advance(const Rows& rows, int64_t p, const float* qv, float r2,
                               const float* __restrict__ T, int dim, int dd, bool tests, int b,
                               int nb, float& S, bool& rej, int& dexit) {
  using SS = Store<ST>;
  typename SS::Block blk[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) blk[i] = SS::load(rows, p, b + (i < nb ? i : nb - 1));
  int nt = tests ? (b * kBlock / dd + 1) * dd : 0x7fffffff;   // next tested d
  if (!PER_DIM) {
    // Branch-free: every unit of the loaded blocks is summed (its query and threshold loads
    // can then all be issued ahead), and only the units the DCO reaches are accumulated and
    // tested.  Padding units and clamped repeat blocks are loaded in bounds and not counted.
#pragma unroll
    for (int i = 0; i < NB; ++i) {
#pragma unroll
      for (int j = 0; j < kBlock / 8; ++j) {
        const int d0 = (b + i) * kBlock + 8 * j;
        float v[8], qq[8];
        SS::unit(blk[i], j, v);
        q8(qv, d0, qq);
        const float Sn = S + unit_sum(qq, v);
        const bool act = i < nb && !rej && d0 < dim;
        const int d = d0 + 8;
        // with dd a multiple of kBlock only a block's last unit can end at a tested d
        const float thr = T[(d < dim ? d : dim) - 1] * r2;
        const bool at = act && d == nt;
        const bool rj = at && d < dim && Sn > thr;
        S = act ? Sn : S;
        dexit = rj ? d : dexit;
        rej = rej || rj;
        nt = at ? nt + dd : nt;
      }
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < NB; ++i) {
#pragma unroll
    for (int j = 0; j < kBlock / 8; ++j) {
      const int d0 = (b + i) * kBlock + 8 * j;
      if (i < nb && !rej && d0 < dim) {
        float v[8], qq[8];
        SS::unit(blk[i], j, v);
        q8(qv, d0, qq);
        if (PER_DIM) {
          float pp = 0.f;
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            const float df = qq[c] - v[c];
            pp = fmaf(df, df, pp);
            const int d = d0 + c + 1;
            if (d == nt) {
              if (!rej && d < dim && S + pp > T[d - 1] * r2) {
                rej = true;
                dexit = d;
              }
              nt += dd;
            }
          }
          S = S + pp;
        } else {
          S = S + unit_sum(qq, v);
          const int d = d0 + 8;
          if (d == nt) {
            if (d < dim && S > T[d - 1] * r2) {
              rej = true;
              dexit = d;
            }
            nt += dd;
          }
        }
      }
    }
  }
}

// Lane k's value of this lane's group of G lanes (G = 4: a DPP quad broadcast).
template <int G>
__device__ inline float group_get(float x, int k) {
  return __shfl(x, (static_cast<int>(threadIdx.x) & 63 & ~(G - 1)) | k, 64);
}

// One level of a DCO worked by a group of G lanes (G = 4 or 16; tests at multiples of dd, itself a
// multiple of 8).  Lane l of the group takes unit l % 4 of block offset l / 4 within each step of
// G / 4 consecutive blocks: it reads that unit of the blocks b + i G/4 + l/4 (steps i < NB; blocks
// below b + nb) and the query coordinates it meets, all loads first.  The group exchanges its unit
// sums and every lane adds them to S unit by unit in coordinate order, so S and the test decisions
// are those of advance() over the same blocks.  All lanes of a group must be active.
template <typename ST, int NB, int G>
__device__ inline void advance_group(const Rows& rows, int64_t p, const float* qv, float r2,
                                     const float* __restrict__ T, int dim, int dd, int b, int nb, float& S,
                                     bool& rej, int& dexit, int gl) {
  using SS = Store<ST>;
  constexpr int BPS = G / 4;   // blocks per step
  const int j = gl & 3, bo = gl >> 2;
  typename SS::Unit u[NB];
  float qq[NB][8];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    int bi = b + i * BPS + bo;
    bi = bi < b + nb ? bi : b + nb - 1;   // clamped repeats are loaded in bounds, not counted
    u[i] = SS::load_unit(rows, p, bi, j);
    q8(qv, bi * kBlock + 8 * j, qq[i]);
  }
  int nt = (b * kBlock / dd + 1) * dd;   // next tested d
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    if (i * BPS >= nb) break;   // the same in every lane of the group
    float v[8];
    SS::unit_of(u[i], v);
    const float us = unit_sum(qq[i], v);
    float su[G];
    if (G == 4) {
      su[0] = quad_get<0>(us); su[1] = quad_get<1>(us); su[2] = quad_get<2>(us); su[3] = quad_get<3>(us);
    } else {
#pragma unroll
      for (int k = 0; k < G; ++k) su[k] = group_get<G>(us, k);
    }
#pragma unroll
    for (int k = 0; k < G; ++k) {   // block i BPS + k / 4, unit k % 4
      const int d0 = (b + i * BPS + (k >> 2)) * kBlock + 8 * (k & 3);
      const float Sn = S + su[k];
      const bool act = i * BPS + (k >> 2) < nb && !rej && d0 < dim;
      const int d = d0 + 8;
      const bool at = act && d == nt;
      const float thr = (dd % kBlock != 0 || (k & 3) == 3) ? T[(d < dim ? d : dim) - 1] * r2 : 0.f;
      const bool rj = at && d < dim && Sn > thr;
      S = act ? Sn : S;
      dexit = rj ? d : dexit;
      rej = rej || rj;
      nt = at ? nt + dd : nt;
    }
  }
}

// The round's filter on a finished DCO (d reached D): queue it for the merge or drop it.
template <bool RERANK>
__device__ inline bool passes(float S, uint32_t rid, bool full, unsigned long long keyr, float gate) {
  return RERANK ? (!full || S <= gate) : (!full || make_key(S, rid) < keyr);
}

__device__ inline void put_key(const RoundArgs& a, int q, int slot, unsigned long long key) {
  if (slot < a.kb_cap) a.kb[int64_t(q) * a.kb_cap + slot] = key;
  else atomicOr(a.overflow, 1);
}

// Wave-wide: queue key (S, rid) of query q on lanes with `queue` set (one atomic per wave).
__device__ inline void append_keys(const RoundArgs& a, int q, bool queue, unsigned long long key, int lane) {
  const unsigned long long m = __ballot(queue);
  if (!m) return;
  int slot = 0;
  if (lane == 0) slot = atomicAdd(a.q_kc + q, __popcll(m));
  slot = __shfl(slot, 0);
  if (queue) put_key(a, q, slot + lanes_below(m), key);
}

// Wave-wide: DCO counts and dimensions read by the lanes with `fin` set, added to query q's stats.
__device__ inline void add_stats(const RoundArgs& a, int q, bool fin, int dexit, int lane) {
  unsigned nd = fin ? 1u : 0u, ds = fin ? unsigned(dexit) : 0u;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    nd += __shfl_xor(nd, o, 64);
    ds += __shfl_xor(ds, o, 64);
  }
  if (lane == 0 && nd) {
    atomicAdd(reinterpret_cast<unsigned long long*>(a.stats + int64_t(q) * 4 + 0), (unsigned long long)nd);
    atomicAdd(reinterpret_cast<unsigned long long*>(a.stats + int64_t(q) * 4 + 1), (unsigned long long)ds);
  }
}

// Whole-row items read a query chunk for every unit of every block.  Read from the query rows
// in memory, one per unit, those reads cost about as much as the rows themselves (the rows of a
// fresh batch of queries are not yet in this CU's caches).  So each step of a whole-row item
// copies the query coordinates of its blocks into the wave's LDS slice, with the loads issued
// beside the step's row loads, and its units read their chunks from there.  The per-dimension
// kernels (Delta_d not a multiple of 8) read in place and are launched without the slices.
template <typename ST>
__host__ __device__ constexpr int stage_span() { return 4 * Store<ST>::kMaxB * kBlock; }   // coordinates per step

__host__ __device__ inline size_t round_lds_bytes(int dtype) {
  const int span = dtype == 0 ? stage_span<float>() : stage_span<__hip_bfloat16>();
  return size_t(kWaves) * size_t(span) * sizeof(float);
}

// Wave-wide: whole-row distances of a small item's candidates (no test can reject them).  Four
// lanes per candidate, 16 candidates per pass; lane j of a quad sums blocks j, j + 4, j + 8, ...
// in order, and the quad's partials combine as (P0 + P1) + (P2 + P3).
template <typename ST, bool RERANK, bool STAGE>
__device__ void dense_item(const RoundArgs& a, const Rows& rows, int q, int cnt, int p0, const float* qv,
                           float* qs, bool full, unsigned long long keyr, float gate, int nblk, int lane) {
  using SS = Store<ST>;
  constexpr int MB = SS::kMaxB;
  constexpr int kSpan = stage_span<ST>();
  const int dim = a.dim;
  const int quad = lane >> 2, ql = lane & 3;
  for (int c0 = 0; c0 < cnt; c0 += 16) {
    const int ci = c0 + quad;
    const bool hv = ci < cnt;
    const int64_t p = p0 + (hv ? ci : 0);
    const bool lead = hv && ql == 0;
    const uint32_t rid = lead ? uint32_t(a.ids[p]) : 0u;
    float part = 0.f;
    for (int b0 = 0; b0 < nblk; b0 += 4 * MB) {
      // STAGE: this step's query coordinates [b0 kBlock, b0 kBlock + kSpan) go into the wave's
      // slice, loaded before the rows (loads past the padded row are clamped to its last float4,
      // and their copies are never read)
      float4 qt[kSpan / 256];
      if constexpr (STAGE) {
#pragma unroll
        for (int i = 0; i < kSpan / 256; ++i) {
          const int c = b0 * kBlock + 4 * lane + 256 * i;
          qt[i] = *reinterpret_cast<const float4*>(qv + (c < a.dp ? c : a.dp - 4));
        }
      }
      typename SS::Block blk[MB];
#pragma unroll
      for (int i = 0; i < MB; ++i) {
        const int bi = b0 + ql + 4 * i;
        blk[i] = SS::load(rows, p, bi < nblk ? bi : nblk - 1);
      }
      if constexpr (STAGE) {
#pragma unroll
        for (int i = 0; i < kSpan / 256; ++i) *reinterpret_cast<float4*>(qs + 4 * lane + 256 * i) = qt[i];
        __builtin_amdgcn_wave_barrier();
        // Branch-free: every unit is summed with its query chunk from the slice, at the clamped
        // block (bc >= b0: a clamped block is the last one, and b0 is at most that); the addend
        // of a unit at or past dim, or of a clamped repeat block, is +0, which leaves the
        // non-negative sum unchanged, so the units below dim are added in the same order.
#pragma unroll
        for (int i = 0; i < MB; ++i) {
          const int bi = b0 + ql + 4 * i;
          const int bc = bi < nblk ? bi : nblk - 1;
#pragma unroll
          for (int j = 0; j < kBlock / 8; ++j) {
            float v[8], qq[8];
            SS::unit(blk[i], j, v);
            q8(qs, (bc - b0) * kBlock + 8 * j, qq);
            const float us = unit_sum(qq, v);
            part = part + ((bi < nblk && bi * kBlock + 8 * j < dim) ? us : 0.f);
          }
        }
      } else {
        // unit by unit, the query chunk read from memory (the per-dimension kernels: the staged
        // loop's registers would cost them an occupancy level)
#pragma unroll
        for (int i = 0; i < MB; ++i) {
          const int bi = b0 + ql + 4 * i;
#pragma unroll
          for (int j = 0; j < kBlock / 8; ++j) {
            const int d0 = bi * kBlock + 8 * j;
            if (bi < nblk && d0 < dim) {
              float v[8], qq[8];
              SS::unit(blk[i], j, v);
              q8(qv, d0, qq);
              part = part + unit_sum(qq, v);
            }
          }
        }
      }
    }
    const float pair = part + __shfl_xor(part, 1, 64);
    const float S = pair + __shfl_xor(pair, 2, 64);
    append_keys(a, q, lead && passes<RERANK>(S, rid, full, keyr, gate), make_key(S, rid), lane);
    if (a.stats) add_stats(a, q, lead, dim, lane);
  }
}

// ------------------------------------------------------------------------------------------------
// scan_round: the DCOs of one round for every query.
template <typename ST, bool DADE, bool RERANK, bool PER_DIM>
// qrot and T are passed on their own, restrict-qualified: nothing the kernel stores aliases them,
// so the reads of a work item's query (one query per item) and of the thresholds of its first
// test can go through the scalar cache.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3))) void scan_round_kernel(RoundArgs a, int r, const float* __restrict__ qrot,
                                                              const float* __restrict__ T) {
  using SS = Store<ST>;
  constexpr int MB = SS::kMaxB;
  __shared__ int4 stack_lds[kWaves][kStack];
  __shared__ int s_claim;
  extern __shared__ float4 q_stage[];   // [kWaves][stage span] floats: whole-row items' query chunks
  const int lane = threadIdx.x & 63;
  int4* stk = stack_lds[threadIdx.x >> 6];
  const int dim = a.dim, dp = a.dp, dd = a.delta_d;
  const int nblk = (dim + kBlock - 1) / kBlock;
  int nb0 = ((dd < dim ? dd : dim) + kBlock - 1) / kBlock;   // level 0 reaches the first test
  nb0 = nb0 > MB ? MB : nb0;
  nb0 = nb0 > nblk ? nblk : nb0;
  const bool any_tests = DADE && dd < dim;
  const Rows rows{a.head, a.tail, dp - kBlock};
  const int n_queued = a.n_items[r];
  const int n_items = n_queued < a.items_cap ? n_queued : a.items_cap;
  const int4* items = a.items + int64_t(r) * a.items_cap;
  const float gate_f = 1.f + a.rerank_delta;
  // Workgroup g owns items g, g + grid, g + 2 grid, ... (a query's items are spread over the
  // grid); its waves take them in turn from an LDS counter, so claims need no global atomics.
  if (threadIdx.x == 0) s_claim = 0;
  __syncthreads();

  int sn = 0;             // live stack entries (wave-uniform)
  // The next work item and its query's round snapshot are fetched one item ahead, so that their
  // dependent loads overlap the current item's work.
  // (an item carries its query's snapshot, so it is all a DCO needs besides the rows; it is
  // fetched together with the round's item count, inside the region's capacity)
  auto claim = [&](int4& it) {
    int k = 0;
    if (lane == 0) k = atomicAdd(&s_claim, 1);
    k = __builtin_amdgcn_readfirstlane(k);   // every lane is active here
    const int64_t idx = int64_t(blockIdx.x) + int64_t(k) * gridDim.x;
    if (idx >= a.items_cap) return false;
    it = items[idx];
    return idx < n_items;
  };
  int4 nit = make_int4(0, 0, 0, 0);
  bool nvalid = claim(nit);
  for (;;) {
    const bool drained = !nvalid;   // no work item left in this round
    if ((sn >= 64 || (drained && sn > 0)) && !PER_DIM && sn <= 16) {
      // ---- the wave's items are done and at most 16 survivors are left: continue each by a
      //      group of lanes (a quad, or 16 lanes when at most 4 are left), in levels of the
      //      largest size the group's registers hold (QB blocks for a quad, 2 QB for 16 lanes)
      constexpr int QB = SS::kQuadMaxB;
      const bool wide = sn <= 4;
      const int G = wide ? 16 : 4;
      const int take = sn;
      const int slot = wide ? lane >> 4 : lane >> 2, gl = wide ? lane & 15 : lane & 3;
      const bool act = slot < take;
      int4 e = make_int4(0, 0, 0, 0);
      if (act) e = stk[slot];
      sn = 0;
      const int q = e.x, p = e.y, lev = e.w & 255;
      int b = e.w >> 8;
      float S = __int_as_float(e.z);
      bool cont = false;
      if (act) {
        const float r2 = a.q_r2[q];
        int nb = wide ? (QB / 2) * 4 : QB;
        nb = nb > nblk - b ? nblk - b : nb;
        bool rej = false;
        int dexit = dim;
        const float* qq = qrot + int64_t(q) * dp;
        if (wide)
          advance_group<ST, QB / 2, 16>(rows, p, qq, r2, T, dim, dd, b, nb, S, rej, dexit, gl);
        else
          advance_group<ST, QB, 4>(rows, p, qq, r2, T, dim, dd, b, nb, S, rej, dexit, gl);
        b += nb;
        if (rej || b >= nblk) {
          if (gl == 0) {
            if (a.stats) {
              atomicAdd(reinterpret_cast<unsigned long long*>(a.stats + int64_t(q) * 4 + 0), 1ull);
              atomicAdd(reinterpret_cast<unsigned long long*>(a.stats + int64_t(q) * 4 + 1),
                        (unsigned long long)dexit);
            }
            const uint32_t rid = uint32_t(a.ids[p]);
            if (!rej && passes<RERANK>(S, rid, true, a.q_keyr[q], gate_f * r2))
              put_key(a, q, atomicAdd(a.q_kc + q, 1), make_key(S, rid));
          }
        } else {
          cont = gl == 0;
        }
      }
      const unsigned long long m = __ballot(cont);
      if (cont) stk[sn + lanes_below(m)] = make_int4(q, p, __float_as_int(S), (b << 8) | (lev < 255 ? lev + 1 : 255));
      sn += __popcll(m);
      continue;
    }
    if (sn >= 64 || (drained && sn > 0)) {
      // ---- continue up to 64 stacked survivors by one level each
      const int take = sn < 64 ? sn : 64;
      const int base = sn - take;
      const bool act = lane < take;
      int4 e = make_int4(0, 0, 0, 0);
      if (act) e = stk[base + lane];
      sn = base;
      const int q = e.x, p = e.y, lev = e.w & 255;
      int b = e.w >> 8;
      float S = __int_as_float(e.z);
      bool cont = false;
      if (act) {
        const float r2 = a.q_r2[q];
        int nb = 1 << (lev - 1 < 4 ? lev - 1 : 4);
        nb = nb < nb0 ? nb0 : nb;
        nb = nb > MB ? MB : nb;
        nb = nb > nblk - b ? nblk - b : nb;
        bool rej = false;
        int dexit = dim;
        advance<ST, PER_DIM, MB>(rows, p, qrot + int64_t(q) * dp, r2, T, dim, dd, true, b, nb, S,
                                 rej, dexit);
        b += nb;
        if (rej || b >= nblk) {
          if (a.stats) {
            atomicAdd(reinterpret_cast<unsigned long long*>(a.stats + int64_t(q) * 4 + 0), 1ull);
            atomicAdd(reinterpret_cast<unsigned long long*>(a.stats + int64_t(q) * 4 + 1),
                      (unsigned long long)dexit);
          }
          const uint32_t rid = uint32_t(a.ids[p]);
          if (!rej && passes<RERANK>(S, rid, true, a.q_keyr[q], gate_f * r2))
            put_key(a, q, atomicAdd(a.q_kc + q, 1), make_key(S, rid));
        } else {
          cont = true;
        }
      }
      const unsigned long long m = __ballot(cont);
      if (cont) stk[sn + lanes_below(m)] = make_int4(q, p, __float_as_int(S), (b << 8) | (lev < 255 ? lev + 1 : 255));
      sn += __popcll(m);
      continue;
    }
    if (drained) break;

    // ---- the prefetched work item; claim the next one
    const int4 it = nit;
    nvalid = claim(nit);
    // an item's fields are the same in every lane
    const uint32_t qc = uint32_t(__builtin_amdgcn_readfirstlane(it.x));
    const int q = int(qc & ((1u << kItemCountShift) - 1)), cnt = int(qc >> kItemCountShift);
    const int p_item = __builtin_amdgcn_readfirstlane(it.y);
    const unsigned long long keyr = (static_cast<unsigned long long>(uint32_t(__builtin_amdgcn_readfirstlane(it.z))) << 32) |
                                    uint32_t(__builtin_amdgcn_readfirstlane(it.w));
    const bool full = keyr != ~0ull;
    const float r2 = full ? key_dist(keyr) : __builtin_inff();
    const float* qv = qrot + int64_t(q) * dp;
    const bool dense = !any_tests || !full;   // no test can reject: whole rows
    if (dense && cnt <= 16) {
      // few candidates (the rounds that fill the heap): four lanes per row
      float* qs = reinterpret_cast<float*>(q_stage) + (threadIdx.x >> 6) * stage_span<ST>();
      dense_item<ST, RERANK, !PER_DIM>(a, rows, q, cnt, p_item, qv, qs, full, keyr, gate_f * r2, nblk, lane);
      continue;
    }
    const bool has = lane < cnt;
    const int p = p_item + (has ? lane : 0);
    float S = 0.f;
    bool rej = false, done = true;
    int dexit = dim;
    if (!dense && !PER_DIM && nb0 == 1) {
      // level 0 (the first test inside the head block)
      if (has) {
        const typename SS::Block blk = SS::load(rows, p, 0);
        int nt = dd;
#pragma unroll
        for (int j = 0; j < kBlock / 8; ++j) {   // branch-free, as in advance()
          const int d = 8 * j + 8;
          float v[8], qq[8];
          SS::unit(blk, j, v);
          q8(qv, 8 * j, qq);
          const float Sn = S + unit_sum(qq, v);
          const bool act = !rej && d - 8 < dim;
          const float thr = T[(d < dim ? d : dim) - 1] * r2;
          const bool at = act && d == nt;
          const bool rj = at && d < dim && Sn > thr;
          S = act ? Sn : S;
          dexit = rj ? d : dexit;
          rej = rej || rj;
          nt = at ? nt + dd : nt;
        }
        done = rej || 1 >= nblk;
      }
    }
    if (!dense && !PER_DIM && nb0 == 1) {
      // done above
    } else if (dense) {
      // one lane per row (FDScanning, or no d below D to test)
      if (has)
        for (int b = 0; b < nblk; b += MB)
          advance<ST, false, MB>(rows, p, qv, r2, T, dim, dd, false, b, nblk - b < MB ? nblk - b : MB, S,
                                 rej, dexit);
    } else if (has) {
      // level 0: up to the first test
      if (nb0 == 1)
        advance<ST, PER_DIM, 1>(rows, p, qv, r2, T, dim, dd, true, 0, 1, S, rej, dexit);
      else
        advance<ST, PER_DIM, MB>(rows, p, qv, r2, T, dim, dd, true, 0, nb0, S, rej, dexit);
      done = rej || nb0 >= nblk;
    }
    const bool fin = has && done;
    const uint32_t rid = fin && !rej ? uint32_t(a.ids[p]) : 0u;   // ids only of finished DCOs
    append_keys(a, q, fin && !rej && passes<RERANK>(S, rid, full, keyr, gate_f * r2), make_key(S, rid), lane);
    if (a.stats) add_stats(a, q, fin, dexit, lane);
    const bool deep = has && !done;
    const unsigned long long md = __ballot(deep);
    if (deep) stk[sn + lanes_below(md)] = make_int4(q, p, __float_as_int(S), (nb0 << 8) | 1);
    sn += __popcll(md);
  }
}

// ------------------------------------------------------------------------------------------------
// merge_round helpers (one workgroup per query, keys in LDS).

__device__ inline int pad8(int n) { return (n + 7) & ~7; }

// Number of keys of c[0..n8) below key, n8 a multiple of 8, c 16-byte aligned; entries past the
// live ones hold ~0, which no key reaches.  Reads 8 keys per step as 16-byte LDS loads, so the
// loads of a step are in flight together.
__device__ inline int count_below(const unsigned long long* c, int n8, unsigned long long key) {
  const ulonglong2* c2 = reinterpret_cast<const ulonglong2*>(c);
  int r0 = 0, r1 = 0;
  for (int j = 0; j < n8 / 2; j += 4) {
    const ulonglong2 v0 = c2[j], v1 = c2[j + 1], v2 = c2[j + 2], v3 = c2[j + 3];
    r0 += int(v0.x < key) + int(v0.y < key) + int(v1.x < key) + int(v1.y < key);
    r1 += int(v2.x < key) + int(v2.y < key) + int(v3.x < key) + int(v3.y < key);
  }
  return r0 + r1;
}

// Appends key to c at a slot taken from *n (one LDS atomic per wave), for the lanes with take.
__device__ inline void append_lds(unsigned long long* c, int* n, bool take, unsigned long long key, int lane) {
  const unsigned long long m = __ballot(take);
  if (m == 0) return;
  int base = 0;
  if (lane == 0) base = atomicAdd(n, __popcll(m));
  base = __shfl(base, 0);
  if (take) c[base + lanes_below(m)] = key;
}

// c[0..n) <- its keys below lim, in order (wave 0; the count goes to *cnt).  Ends with a barrier.
__device__ inline void keep_below(unsigned long long* c, int n, unsigned long long lim, int* cnt, int tid) {
  if (tid < 64) {
    int w = 0;
    for (int base = 0; base < n; base += 64) {
      const int i = base + tid;
      const unsigned long long key = i < n ? c[i] : ~0ull;
      const bool keep = i < n && key < lim;
      const unsigned long long m = __ballot(keep);
      if (keep) c[w + lanes_below(m)] = key;
      w += __popcll(m);
    }
    if (tid == 0) *cnt = w;
  }
  __syncthreads();
}

// An upper bound on the K-th smallest of c(0..n): the K-th smallest of its first 64 entries
// (wave 0 ranks them by shuffles), or ~0 when that cannot help (n <= 96, K > 64).  Keys are
// unique.  To *t; ends with a barrier.
template <typename GetFn>
__device__ inline void sample_bound(GetFn c, int n, int K, unsigned long long* t, int tid) {
  if (tid == 0) *t = ~0ull;
  if (n > 96 && K <= 64 && tid < 64) {
    const unsigned long long key = c(tid);
    int rank = 0;
    for (int j = 0; j < 64; ++j) rank += int(__shfl(key, j) < key);
    if (rank == K - 1) *t = key;
  }
  __syncthreads();
}

// heap[0..heap_n) (ascending keys) <- the K smallest of heap and cand[0..n); keys are unique,
// so each key's rank is the count of smaller keys.  cand must have room for pad8(n + K)
// entries.  Ends with a barrier.
__device__ void merge_into(unsigned long long* heap, int& heap_n, unsigned long long* tmp,
                           unsigned long long* cand, int n, int K, int tid) {
  if (n > 0) {
    const int tot = n + heap_n, tot8 = pad8(tot);
    for (int i = tid; i < tot8 - n; i += kThreads) cand[n + i] = i < heap_n ? heap[i] : ~0ull;
    __syncthreads();
    for (int i = tid; i < tot; i += kThreads) {
      const unsigned long long key = cand[i];
      const int rank = count_below(cand, tot8, key);
      if (rank < K) tmp[rank] = key;
    }
    __syncthreads();
    heap_n = tot < K ? tot : K;
    for (int i = tid; i < heap_n; i += kThreads) heap[i] = tmp[i];
  }
  __syncthreads();
}

// keys[i] (stored-precision S_D, id) -> (exact FP32 S_D, id) over the original vectors: 16 lanes
// per key, each summing its units (u = lane, lane + 16, ...) in order, then a fixed butterfly
// over the 16 lanes.  Ends with a barrier.
__device__ void exact_rerank(unsigned long long* keys, int n, const float* __restrict__ X,
                             const float* qo, int dp, int dim, int tid, unsigned& count) {
  const int g = tid / kGroup, gl = tid % kGroup;
  const int u_end = (dim + 7) / 8;
  for (int i = g; i < n; i += kGroups) {
    const uint32_t id = key_id(keys[i]);
    const float* x = X + int64_t(id) * dp;
    float acc = 0.f;
    for (int u0 = gl; u0 < u_end; u0 += 8 * kGroup) {
      float4 ra[8], rb[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        int u = u0 + k * kGroup;
        u = u < u_end ? u : u_end - 1;
        ra[k] = *reinterpret_cast<const float4*>(x + 8 * u);
        rb[k] = *reinterpret_cast<const float4*>(x + 8 * u + 4);
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int u = u0 + k * kGroup;
        if (u < u_end) {
          const float v[8] = {ra[k].x, ra[k].y, ra[k].z, ra[k].w, rb[k].x, rb[k].y, rb[k].z, rb[k].w};
          float qq[8];
          q8(qo, 8 * u, qq);
          acc = acc + unit_sum(qq, v);
        }
      }
    }
#pragma unroll
    for (int o = kGroup / 2; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, kGroup);
    if (gl == 0) {
      keys[i] = make_key(acc, id);
      ++count;
    }
  }
  __syncthreads();
}

// A work item of cnt candidates from packed position p, with an empty heap's snapshot.
__device__ inline int4 make_item(int q, int cnt, int p) {
  return make_int4(int(uint32_t(q) | (uint32_t(cnt) << kItemCountShift)), p, -1, -1);
}

// End (t1, off1) of the round that starts at (t, off) after pos candidates; returns its
// candidate count.  The first round holds the first max(K, fill_min) candidates; a later round
// ends at the schedule's next probe-rank boundary (every rank, ranks 1, 2, 4, ..., or none before
// the last) or after growth * pos candidates if that comes first (growth 0: no cap).
template <typename LenFn>
__device__ int64_t round_end(const RoundArgs& a, int t, int off, int64_t pos, bool first, int K, int np,
                             LenFn len_of, int& t1, int& off1) {
  int tb = np;
  int64_t rem;
  if (first) {
    rem = K > a.fill_min ? K : a.fill_min;
  } else {
    if (a.schedule == 0) {
      tb = t + 1;
    } else if (a.schedule == 1) {
      int B = 1;
      while (B <= t) B <<= 1;
      tb = B < np ? B : np;
    }   // schedule 2 (whole): no boundary before np
    rem = a.growth > 0 ? int64_t(a.growth) * pos : INT64_MAX;
  }
  int tt = t, oo = off;
  int64_t took = 0;
  while (tt < tb && rem > 0) {
    const int avail = len_of(tt) - oo;
    if (avail > rem) {
      oo += int(rem);
      took += rem;
      rem = 0;
    } else {
      rem -= avail;
      took += avail;
      ++tt;
      oo = 0;
    }
  }
  t1 = tt;
  off1 = oo;
  return took;
}

// Work items of query q's round [(t, off), (t1, off1)): every list segment of the round cut
// into items of at most kItem candidates.  With items == nullptr only counts them.
template <typename LenFn, typename PosFn>
__device__ int round_items(const RoundArgs& a, int4* items, int cap, int slot, int q, int t, int off, int t1,
                           int off1, int per, LenFn len_of, PosFn pos_of) {
  const int t_last = off1 > 0 ? t1 : t1 - 1;
  int n = 0;
  for (int tt = t; tt <= t_last; ++tt) {
    const int s0 = tt == t ? off : 0;
    const int s1 = tt == t1 ? off1 : len_of(tt);
    if (s1 <= s0) continue;
    if (!items) {
      n += (s1 - s0 + per - 1) / per;
      continue;
    }
    const int p0 = int(pos_of(tt));
    for (int ss = s0; ss < s1; ss += per, ++n) {
      if (slot + n < cap) items[slot + n] = make_item(q, s1 - ss < per ? s1 - ss : per, p0 + ss);
      else atomicOr(a.overflow, 2);
    }
  }
  return n;
}

// ------------------------------------------------------------------------------------------------
// plan: the round cuts of every query's whole candidate sequence (they depend only on the list
// sizes, K and the schedule), and each round's work items in that round's region.  Three
// passes without atomics: per query, its item count in every round; per round, an exclusive
// prefix sum over the queries; per query, its items written at its offsets.  The first pass
// also sets the query's heap state to empty.
constexpr int kPlanLists = 2048;   // probed lists whose (position, length) are staged in LDS

constexpr int kPlanRounds = 1024;  // rounds whose cuts are staged in LDS for the writing pass

template <bool WRITE>
__global__ __launch_bounds__(64) void plan_kernel(RoundArgs a, int* counts) {
  __shared__ int2 lst[kPlanLists];
  __shared__ int4 cuts[WRITE ? kPlanRounds : 1];
  __shared__ int s_nr;
  const int q = blockIdx.x;
  const int lane = threadIdx.x;
  int K = a.k_pq ? a.k_pq[q] : a.k_max;
  K = K < 1 ? 1 : (K > a.k_max ? a.k_max : K);
  int np = a.nprobe_pq ? a.nprobe_pq[q] : a.nprobe_max;
  np = np < 1 ? 1 : (np > a.nprobe_max ? a.nprobe_max : np);
  const int32_t* pr = a.probes + int64_t(q) * a.nprobe_max;
  for (int t = lane; t < np && t < kPlanLists; t += 64) {
    const int l = pr[t];
    const int64_t o = a.list_off[l];
    lst[t] = make_int2(int(o), int(a.list_off[l + 1] - o));
  }
  __syncthreads();
  auto len_of = [&](int tt) {
    return tt < kPlanLists ? lst[tt].y : int(a.list_off[pr[tt] + 1] - a.list_off[pr[tt]]);
  };
  auto pos_of = [&](int tt) { return tt < kPlanLists ? int64_t(lst[tt].x) : a.list_off[pr[tt]]; };
  if (lane == 0) {
    int t = 0, off = 0, r = 0;
    int64_t pos = 0;
    while (t < np && r < a.rounds) {
      int t1, off1;
      // rounds that start before K candidates have been merged hold few candidates and read
      // whole rows: smaller items spread them over more waves
      const int per = pos < K ? kDenseItem : kItem;
      pos += round_end(a, t, off, pos, r == 0, K, np, len_of, t1, off1);
      if (!WRITE) {
        counts[int64_t(r) * a.nq + q] = round_items(a, nullptr, 0, 0, q, t, off, t1, off1, per, len_of, pos_of);
      } else if (r < kPlanRounds) {
        cuts[r] = make_int4(t, off, t1, off1 | (per == kDenseItem ? int(0x80000000u) : 0));
      } else {
        round_items(a, a.items + int64_t(r) * a.items_cap, a.items_cap, counts[int64_t(r) * a.nq + q], q, t, off,
                    t1, off1, per, len_of, pos_of);
      }
      t = t1;
      off = off1;
      ++r;
    }
    if (WRITE) {
      s_nr = r < kPlanRounds ? r : kPlanRounds;
    } else {
      for (int rr = r; rr < a.rounds; ++rr) counts[int64_t(rr) * a.nq + q] = 0;
      if (t < np) atomicOr(a.overflow, 4);   // more rounds than the launch sequence holds
      a.q_rounds[q] = r;
      if (a.q_record) {
        a.q_record[int64_t(q) * 3 + 0] = K;
        a.q_record[int64_t(q) * 3 + 1] = np;
        a.q_record[int64_t(q) * 3 + 2] = r;
      }
      a.q_topn[q] = 0;
      a.q_kc[q] = 0;
      a.q_keyr[q] = ~0ull;
      a.q_r2[q] = __builtin_inff();
      if (a.stats)
        for (int i = 0; i < 4; ++i) a.stats[int64_t(q) * 4 + i] = 0;
    }
  }
  if (!WRITE) return;
  __syncthreads();
  // the staged rounds' items: for each round and each list segment of it, the wave writes the
  // segment's items in parallel (item j of a segment by lane j % 64)
  for (int r = 0; r < s_nr; ++r) {
    const int4 c = cuts[r];
    const int t = c.x, off = c.y, t1 = c.z, off1 = c.w & 0x7FFFFFFF;
    const int per = c.w < 0 ? kDenseItem : kItem;
    int4* items = a.items + int64_t(r) * a.items_cap;
    int slot = counts[int64_t(r) * a.nq + q];
    const int t_last = off1 > 0 ? t1 : t1 - 1;
    for (int tt = t; tt <= t_last; ++tt) {
      const int s0 = tt == t ? off : 0;
      const int s1 = tt == t1 ? off1 : len_of(tt);
      if (s1 <= s0) continue;
      const int n = (s1 - s0 + per - 1) / per;
      const int p0 = int(pos_of(tt));
      for (int j = lane; j < n; j += 64) {
        const int ss = s0 + j * per;
        if (slot + j < a.items_cap) items[slot + j] = make_item(q, s1 - ss < per ? s1 - ss : per, p0 + ss);
        else atomicOr(a.overflow, 2);
      }
      slot += n;
    }
  }
}

// counts[r][0..nq) -> exclusive prefix sums in place, n_items[r] = the total.  One workgroup per
// round.
constexpr int kScanThreads = 1024;
__global__ __launch_bounds__(kScanThreads) void plan_offsets_kernel(RoundArgs a, int* counts) {
  __shared__ int part[kScanThreads / 64];
  __shared__ int s_carry;
  int* c = counts + int64_t(blockIdx.x) * a.nq;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) s_carry = 0;
  __syncthreads();
  for (int base = 0; base < a.nq; base += kScanThreads) {
    const int i = base + tid;
    const int v = i < a.nq ? c[i] : 0;
    int x = v;   // inclusive scan within the wave
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) part[wave] = x;
    __syncthreads();
    int before = s_carry;
    for (int w = 0; w < wave; ++w) before += part[w];
    if (i < a.nq) c[i] = before + x - v;
    __syncthreads();
    if (tid == kScanThreads - 1) s_carry = before + x;
    __syncthreads();
  }
  if (tid == 0) a.n_items[blockIdx.x] = s_carry;
}

// ------------------------------------------------------------------------------------------------
// merge_round: per query, merge round r's queued keys into the top-K and take the snapshot for
// the next round; after the query's last round, write its result.
template <bool RERANK>
__global__ __launch_bounds__(kThreads) void merge_round_kernel(RoundArgs a, int r) {
  extern __shared__ float4 qo4[];   // [dp] original query (RERANK)
  float* qo = reinterpret_cast<float*>(qo4);
  __shared__ __align__(16) unsigned long long topk[kMaxK];
  __shared__ __align__(16) unsigned long long newk[kMaxK];
  __shared__ __align__(16) unsigned long long fk[RERANK ? kMaxK : 8];
  __shared__ __align__(16) unsigned long long cand[kMergeChunk + kMaxK];
  __shared__ __align__(16) unsigned long long qk[kMergeChunk];   // the queued keys, when they fit
  __shared__ int s_nc, s_below;
  __shared__ unsigned long long s_b, s_t;

  const int q = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63;
  const int dp = a.dp, dim = a.dim;
  unsigned long long* gtop = a.q_topk + int64_t(q) * a.k_max;
  const unsigned long long* kb = a.kb + int64_t(q) * a.kb_cap;
  // the query's state, its heap (all k_max slots; those past its size are not used) and the
  // head of its queue are fetched together, before it is known whether the round queued any key
  const int rq = a.q_rounds[q];
  const int kc = a.q_kc[q];
  int topk_n = a.q_topn[q];
  const unsigned long long keyr = a.q_keyr[q];
  const int n_head = a.kb_cap < kHeadKeys ? int(a.kb_cap) : kHeadKeys;
  for (int i = tid; i < a.k_max; i += kThreads) topk[i] = gtop[i];
  if (tid < n_head) qk[tid] = kb[tid];
  // and the original query for the rerank, 16 bytes per thread (one step for dp <= 1024)
  if (RERANK)
    for (int c = 4 * tid; c < dp; c += 4 * kThreads)
      *reinterpret_cast<float4*>(qo + c) = *reinterpret_cast<const float4*>(a.qorig + int64_t(q) * dp + c);
  // the query's items of round r + 1 (they get the snapshot its scan tests against)
  const bool has_next = r + 1 < a.rounds;
  const int64_t ro = int64_t(r + 1) * a.nq;
  const int it_b = has_next ? a.item_off[ro + q] : 0;
  const int it_e = !has_next ? 0 : (q + 1 < a.nq ? a.item_off[ro + q + 1] : a.n_items[r + 1]);
  auto put_snapshot = [&](unsigned long long key) {
    int2* nx = reinterpret_cast<int2*>(a.items + int64_t(r + 1) * a.items_cap);
    const int e = it_e < a.items_cap ? it_e : a.items_cap;
    for (int i = it_b + tid; i < e; i += kThreads) nx[2 * i + 1] = make_int2(int(key >> 32), int(uint32_t(key)));
  };
  if (r >= rq) return;                    // finished in an earlier round
  const bool last = r == rq - 1;
  if (kc == 0 && !last) {                 // nothing queued: heap and snapshot stay as they are
    put_snapshot(keyr);
    return;
  }
  int K = a.k_pq ? a.k_pq[q] : a.k_max;
  K = K < 1 ? 1 : (K > a.k_max ? a.k_max : K);
  const int m = kc < a.kb_cap ? kc : int(a.kb_cap);
  const bool in_lds = m <= kMergeChunk;
  if (in_lds)
    for (int i = n_head + tid; i < m; i += kThreads) qk[i] = kb[i];
  const bool full = keyr != ~0ull;
  auto queued = [&](int i) { return in_lds ? qk[i] : kb[i]; };
  unsigned st_kept = 0, st_rr = 0;
  __syncthreads();

  if (!RERANK) {
    for (int base = 0; base < m; base += kMergeChunk) {
      const int cnt = m - base < kMergeChunk ? m - base : kMergeChunk;
      // only keys below the heap's K-th, and (a bound from a sample) among the chunk's K smallest
      sample_bound([&](int i) { return queued(base + i); }, cnt, K, &s_t, tid);
      const unsigned long long kth = topk_n == K ? topk[K - 1] : ~0ull;
      const unsigned long long lim = s_t < kth ? s_t : kth;
      if (tid == 0) {
        s_nc = 0;
        s_below = 0;
      }
      __syncthreads();
      for (int i0 = 0; i0 < cnt; i0 += kThreads) {
        const int i = i0 + tid;
        const unsigned long long key = i < cnt ? queued(base + i) : ~0ull;
        const bool below = i < cnt && key < kth;   // kept: below the heap's K-th
        const unsigned long long mb = __ballot(below);
        if (lane == 0 && mb) atomicAdd(&s_below, __popcll(mb));
        append_lds(cand, &s_nc, below && key <= lim, key, lane);
      }
      __syncthreads();
      if (tid == 0) st_kept += unsigned(s_below);
      merge_into(topk, topk_n, newk, cand, s_nc, K, tid);
    }
  } else if (m > 0 && a.rerank_rule == 0) {
    // plain rule: every queued key (a survivor that passed the gate) gets its exact distance
    for (int base = 0; base < m; base += kMergeChunk) {
      const int cnt = m - base < kMergeChunk ? m - base : kMergeChunk;
      for (int i = tid; i < cnt; i += kThreads) cand[i] = queued(base + i);
      __syncthreads();
      exact_rerank(cand, cnt, a.X, qo, dp, dim, tid, st_rr);
      keep_below(cand, cnt, keyr, &s_nc, tid);   // keyr is ~0 while the heap is not full
      if (tid == 0) st_kept += unsigned(s_nc);
      merge_into(topk, topk_n, newk, cand, s_nc, K, tid);
    }
  } else if (m > 0) {
    // lazy rule.  F = the K smallest queued keys (stored-precision S_D, id), into cand[0..fn)
    int fn = 0;
    unsigned long long fmax = ~0ull;
    if (m <= K) {
      for (int i = tid; i < m; i += kThreads) cand[i] = queued(i);
      fn = m;
      __syncthreads();
    } else {
      for (int base = 0; base < m; base += kMergeChunk) {
        const int cnt = m - base < kMergeChunk ? m - base : kMergeChunk;
        sample_bound([&](int i) { return queued(base + i); }, cnt, K, &s_t, tid);
        const unsigned long long kth = fn == K ? fk[K - 1] : ~0ull;
        const unsigned long long lim = s_t < kth ? s_t : kth;
        if (tid == 0) s_nc = 0;
        __syncthreads();
        for (int i0 = 0; i0 < cnt; i0 += kThreads) {
          const int i = i0 + tid;
          const unsigned long long key = i < cnt ? queued(base + i) : ~0ull;
          append_lds(cand, &s_nc, i < cnt && key < kth && key <= lim, key, lane);
        }
        __syncthreads();
        merge_into(fk, fn, newk, cand, s_nc, K, tid);
      }
      fmax = fk[fn - 1];
      for (int i = tid; i < fn; i += kThreads) cand[i] = fk[i];
      __syncthreads();
    }
    exact_rerank(cand, fn, a.X, qo, dp, dim, tid, st_rr);
    // b = K-th smallest exact key of the heap snapshot and F
    if (tid == 0) s_b = ~0ull;
    for (int i = topk_n + tid; i < pad8(topk_n); i += kThreads) topk[i] = ~0ull;
    for (int i = fn + tid; i < pad8(fn); i += kThreads) cand[i] = ~0ull;
    __syncthreads();
    if (topk_n + fn >= K) {
      for (int i = tid; i < topk_n + fn; i += kThreads) {
        const unsigned long long key = i < topk_n ? topk[i] : cand[i - topk_n];
        const int rank = count_below(topk, pad8(topk_n), key) + count_below(cand, pad8(fn), key);
        if (rank == K - 1) s_b = key;
      }
    }
    __syncthreads();
    const float bound = s_b == ~0ull ? __builtin_inff() : (1.f + a.rerank_delta) * key_dist(s_b);
    keep_below(cand, fn, keyr, &s_nc, tid);   // keyr is ~0 while the heap is not full
    if (tid == 0) st_kept += unsigned(s_nc);
    merge_into(topk, topk_n, newk, cand, s_nc, K, tid);
    // the rest of the queue, reranked only inside the bound
    for (int base = 0; m > K && base < m; base += kMergeChunk) {
      const int cnt = m - base < kMergeChunk ? m - base : kMergeChunk;
      if (tid == 0) s_nc = 0;
      __syncthreads();
      for (int i0 = 0; i0 < cnt; i0 += kThreads) {
        const int i = i0 + tid;
        const unsigned long long key = i < cnt ? queued(base + i) : ~0ull;
        append_lds(cand, &s_nc, i < cnt && key > fmax && key_dist(key) <= bound, key, lane);
      }
      __syncthreads();
      const int nr = s_nc;
      __syncthreads();
      if (nr == 0) continue;
      exact_rerank(cand, nr, a.X, qo, dp, dim, tid, st_rr);
      keep_below(cand, nr, keyr, &s_nc, tid);
      if (tid == 0) st_kept += unsigned(s_nc);
      merge_into(topk, topk_n, newk, cand, s_nc, K, tid);
    }
  }

  // ---- store the heap and the next round's snapshot, or write the result
  for (int i = tid; i < topk_n; i += kThreads) gtop[i] = topk[i];
  if (a.stats) {
    if (st_kept)
      atomicAdd(reinterpret_cast<unsigned long long*>(a.stats + int64_t(q) * 4 + 2), (unsigned long long)st_kept);
    if (st_rr)
      atomicAdd(reinterpret_cast<unsigned long long*>(a.stats + int64_t(q) * 4 + 3), (unsigned long long)st_rr);
  }
  const bool nfull = topk_n == K;
  const unsigned long long nkey = nfull ? topk[K - 1] : ~0ull;
  if (tid == 0) {
    a.q_topn[q] = topk_n;
    a.q_kc[q] = 0;
    a.q_keyr[q] = nkey;
    a.q_r2[q] = nfull ? key_dist(nkey) : __builtin_inff();
  }
  if (!last) put_snapshot(nkey);
  if (last) {
    for (int j = tid; j < a.k_max; j += kThreads) {
      const int64_t o = int64_t(q) * a.k_max + j;
      if (j < topk_n) {
        a.out_ids[o] = int64_t(key_id(topk[j]));
        a.out_d2[o] = key_dist(topk[j]);
      } else {
        a.out_ids[o] = -1;
        a.out_d2[o] = __builtin_inff();
      }
    }
  }
}

template <typename ST, bool DADE, bool RERANK>
hipError_t launch_round_typed(const RoundArgs& a, int r, hipStream_t s) {
  const size_t lds = round_lds_bytes(a.dtype);   // the staging slices (not used per dimension)
  if (DADE && a.delta_d % 8 != 0)
    hipLaunchKernelGGL((scan_round_kernel<ST, DADE, RERANK, true>), dim3(a.grid), dim3(kThreads), 0, s, a, r, a.qrot,
                       a.T);
  else
    hipLaunchKernelGGL((scan_round_kernel<ST, DADE, RERANK, false>), dim3(a.grid), dim3(kThreads), lds, s, a, r,
                       a.qrot, a.T);
  return hipGetLastError();
}

template <typename ST, bool RERANK>
hipError_t launch_round_mode(const RoundArgs& a, int r, hipStream_t s) {
  return a.mode == 0 ? launch_round_typed<ST, true, RERANK>(a, r, s)
                     : launch_round_typed<ST, false, RERANK>(a, r, s);
}

}  // namespace

hipError_t launch_round(const RoundArgs& a, int r, hipStream_t s) {
  if (a.nq == 0) return hipSuccess;
  if (a.dtype == 0) return launch_round_mode<float, false>(a, r, s);
  if (a.dtype == 1) return launch_round_mode<__hip_bfloat16, true>(a, r, s);
  return launch_round_mode<__half, true>(a, r, s);
}

hipError_t launch_plan(const RoundArgs& a, int* counts, hipStream_t s) {
  if (a.nq == 0) return hipSuccess;
  hipLaunchKernelGGL((plan_kernel<false>), dim3(a.nq), dim3(64), 0, s, a, counts);
  hipLaunchKernelGGL(plan_offsets_kernel, dim3(a.rounds), dim3(kScanThreads), 0, s, a, counts);
  hipLaunchKernelGGL((plan_kernel<true>), dim3(a.nq), dim3(64), 0, s, a, counts);
  return hipGetLastError();
}

int round_blocks_per_cu(int dtype, int mode, int delta_d) {
  int n = 0;
  hipError_t e = hipSuccess;
  const bool pd = mode == 0 && delta_d % 8 != 0;
  const size_t lds = round_lds_bytes(dtype);
#define DADE_OCC(ST, D, R, P) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, scan_round_kernel<ST, D, R, P>, kThreads, P ? 0 : lds)
  if (dtype == 0) {
    if (mode != 0) DADE_OCC(float, false, false, false);
    else if (pd) DADE_OCC(float, true, false, true);
    else DADE_OCC(float, true, false, false);
  } else if (dtype == 1) {
    if (mode != 0) DADE_OCC(__hip_bfloat16, false, true, false);
    else if (pd) DADE_OCC(__hip_bfloat16, true, true, true);
    else DADE_OCC(__hip_bfloat16, true, true, false);
  } else {
    if (mode != 0) DADE_OCC(__half, false, true, false);
    else if (pd) DADE_OCC(__half, true, true, true);
    else DADE_OCC(__half, true, true, false);
  }
#undef DADE_OCC
  return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_merge(const RoundArgs& a, int r, hipStream_t s) {
  if (a.nq == 0) return hipSuccess;
  const size_t lds = a.dtype == 0 ? 0 : sizeof(float) * size_t(a.dp);
  if (a.dtype == 0)
    hipLaunchKernelGGL((merge_round_kernel<false>), dim3(a.nq), dim3(kThreads), lds, s, a, r);
  else
    hipLaunchKernelGGL((merge_round_kernel<true>), dim3(a.nq), dim3(kThreads), lds, s, a, r);
  return hipGetLastError();
}

}  // namespace dade
