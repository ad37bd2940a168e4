// The DADE list scan: Algorithm 1 for every candidate of a query's probed lists, the
// size-K heap of the IVF scan (end of the Methodology section) and, for low-precision
// stores, an exact FP32 rerank of the survivors.
//
// Execution model (one persistent launch for the whole batch):
//   * a 256-thread workgroup owns one query at a time, pulled from a global counter, and
//     walks its probe ranks round by round; a round's DCOs all use the heap as it was when
//     the round started (thresholds r^2 and T_d r^2 are fixed for the round), and the
//     round's kept candidates are merged into the top-K in LDS at its end.  Queries never
//     wait for one another, so results do not depend on the batch.
//   * inside a round every lane runs its own candidate's DCO: it reads the candidate's
//     rotated row 64 bytes at a time (16 FP32 or 32 BF16/FP16 coordinates), accumulates
//     S_d = sum (q'_k - o'_k)^2 in FP32 in dimension order, and at every d = Delta_d,
//     2 Delta_d, ... below D tests S_d > T_d r^2 (Eq. (13) + the hypothesis test in reduced
//     form).  A lane whose candidate is rejected or finished immediately starts the next
//     candidate of the round (lane refill), so early exits free lanes instead of idling them.
//   * at d = D a candidate is kept iff the heap is not full or (S_D, id) < (r^2, id_r).
//     Low-precision stores: a survivor is kept for rerank iff S_D <= (1 + delta) r^2 (or the
//     heap is not full); its exact FP32 distance is then read from the original vector.
#include "kernels.h"

namespace dade {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxRoundLists = 64;   // lists handled together inside one round
constexpr int kMergeChunk = 1024;    // accepted keys merged per LDS pass

// 64 bytes of a stored row as floats.
template <typename ST>
struct Row;

template <>
struct Row<float> {
  static constexpr int CH = 16;
  __device__ static inline void load(const void* base, int64_t pos, int dp, int g, float* v) {
    const float4* p = reinterpret_cast<const float4*>(static_cast<const float*>(base) + pos * dp + g * CH);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float4 x = p[i];
      v[4 * i + 0] = x.x; v[4 * i + 1] = x.y; v[4 * i + 2] = x.z; v[4 * i + 3] = x.w;
    }
  }
};

template <>
struct Row<__hip_bfloat16> {
  static constexpr int CH = 32;
  __device__ static inline void load(const void* base, int64_t pos, int dp, int g, float* v) {
    const uint4* p = reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(base) + pos * dp + g * CH);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint4 x = p[i];
      const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        v[8 * i + 2 * j + 0] = __builtin_bit_cast(float, w[j] << 16);
        v[8 * i + 2 * j + 1] = __builtin_bit_cast(float, w[j] & 0xFFFF0000u);
      }
    }
  }
};

template <>
struct Row<__half> {
  static constexpr int CH = 32;
  __device__ static inline void load(const void* base, int64_t pos, int dp, int g, float* v) {
    const uint4* p = reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(base) + pos * dp + g * CH);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint4 x = p[i];
      const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        v[8 * i + 2 * j + 0] = float(__builtin_bit_cast(_Float16, uint16_t(w[j] & 0xFFFFu)));
        v[8 * i + 2 * j + 1] = float(__builtin_bit_cast(_Float16, uint16_t(w[j] >> 16)));
      }
    }
  }
};

__device__ inline unsigned long long load_l2(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename ST, bool DADE, bool RERANK, bool PER_DIM_TESTS>
__global__ __launch_bounds__(kThreads) void scan_kernel(ScanArgs a) {
  using R = Row<ST>;
  constexpr int CH = R::CH;
  extern __shared__ float dyn[];
  float* qs = dyn;                       // [dp] rotated query
  float* qo = dyn + a.dp;                // [dp] original query (RERANK only)
  float* thr = dyn + (RERANK ? 2 : 1) * a.dp;  // [ntests] T_d r^2 for the round

  __shared__ unsigned long long topk[kMaxK];
  __shared__ unsigned long long newk[kMaxK];
  __shared__ unsigned long long cand[kMergeChunk + kMaxK];
  __shared__ int64_t lst_pos[kMaxRoundLists];
  __shared__ int lst_pre[kMaxRoundLists + 1];
  __shared__ int s_q, s_acc, s_nc;
  __shared__ unsigned long long s_stat[4];

  const int tid = threadIdx.x;
  const int dim = a.dim, dp = a.dp, dd = a.delta_d;
  const int ntests = (dim - 1) / dd;
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
    if (tid < 4) s_stat[tid] = 0;
    int topk_n = 0;
    unsigned long long st_dco = 0, st_dims = 0, st_kept = 0, st_rr = 0;
    __syncthreads();

    int b = 0;
    while (b < np) {
      const int e = (a.schedule == 0) ? b + 1 : (b == 0 ? 1 : (2 * b < np ? 2 * b : np));
      // ---- round snapshot
      const bool full = topk_n == K;
      const unsigned long long keyr = full ? topk[K - 1] : ~0ull;
      const float r2 = full ? key_dist(keyr) : __builtin_inff();
      const float gate = (1.f + a.rerank_delta) * r2;
      if (DADE)
        for (int j = tid; j < ntests; j += kThreads) thr[j] = a.T[(j + 1) * dd - 1] * r2;
      if (tid == 0) s_acc = 0;
      __syncthreads();

      for (int lb = b; lb < e; lb += kMaxRoundLists) {
        const int le = (e - lb < kMaxRoundLists) ? e : lb + kMaxRoundLists;
        if (tid == 0) {
          int tot = 0;
          for (int j = 0; j < le - lb; ++j) {
            const int l = a.probes[int64_t(qi) * a.nprobe_max + lb + j];
            lst_pre[j] = tot;
            lst_pos[j] = a.list_off[l];
            tot += int(a.list_off[l + 1] - a.list_off[l]);
          }
          lst_pre[le - lb] = tot;
        }
        __syncthreads();
        const int nl = le - lb;
        const int total = lst_pre[nl];

        // ---- per-lane DCOs with refill
        int c = tid;
        int64_t pos = 0;
        uint32_t rid = 0;
        auto locate = [&](int cc) {
          int lo = 0, hi = nl - 1;
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (lst_pre[mid] <= cc) lo = mid; else hi = mid - 1;
          }
          pos = lst_pos[lo] + (cc - lst_pre[lo]);
          rid = uint32_t(a.ids[pos]);
        };
        if (c < total) locate(c);
        int g = 0, next_test = dd, ti = 0;
        float S = 0.f;
        while (c < total) {
          float v[CH];
          R::load(a.store, pos, dp, g, v);
          const int base = g * CH;
          bool rej = false;
          int dexit = dim;
#pragma unroll
          for (int sub = 0; sub < CH / 8; ++sub) {
            if (!rej) {
              const float4 q0 = *reinterpret_cast<const float4*>(qs + base + 8 * sub);
              const float4 q1 = *reinterpret_cast<const float4*>(qs + base + 8 * sub + 4);
              const float qv[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
              for (int i = 0; i < 8; ++i) {
                const float df = qv[i] - v[8 * sub + i];
                S = fmaf(df, df, S);
                if (DADE && PER_DIM_TESTS) {
                  const int d = base + 8 * sub + i + 1;
                  if (d == next_test && d < dim) {
                    if (S > thr[ti]) { rej = true; dexit = d; }
                    ++ti;
                    next_test += dd;
                  }
                }
              }
              if (DADE && !PER_DIM_TESTS) {
                const int d = base + 8 * sub + 8;
                if (d == next_test && d < dim) {
                  if (S > thr[ti]) { rej = true; dexit = d; }
                  ++ti;
                  next_test += dd;
                }
              }
            }
          }
          const bool last = (g + 1) * CH >= dim;
          if (!rej && !last) {
            ++g;
            continue;
          }
          ++st_dco;
          st_dims += unsigned(dexit);
          if (!rej) {
            float Sf = S;
            bool keep;
            if (RERANK) {
              keep = false;
              if (!full || S <= gate) {
                const float4* xr = reinterpret_cast<const float4*>(a.X + int64_t(rid) * dp);
                float Sx = 0.f;
                for (int k4 = 0; k4 < dp / 4; ++k4) {
                  const float4 x = xr[k4];
                  const float4 qq = *reinterpret_cast<const float4*>(qo + 4 * k4);
                  float df = qq.x - x.x; Sx = fmaf(df, df, Sx);
                  df = qq.y - x.y; Sx = fmaf(df, df, Sx);
                  df = qq.z - x.z; Sx = fmaf(df, df, Sx);
                  df = qq.w - x.w; Sx = fmaf(df, df, Sx);
                }
                ++st_rr;
                Sf = Sx;
                keep = !full || make_key(Sx, rid) < keyr;
              }
            } else {
              keep = !full || make_key(S, rid) < keyr;
            }
            if (keep) {
              ++st_kept;
              const int slot = atomicAdd(&s_acc, 1);
              if (slot < a.acc_cap) acc[slot] = make_key(Sf, rid);
              else atomicOr(a.overflow, 1);
            }
          }
          c += kThreads;
          if (c < total) locate(c);
          g = 0; next_test = dd; ti = 0; S = 0.f;
        }
        __syncthreads();
      }
      __threadfence();   // kept keys reach L2 before the merge reads them back
      __syncthreads();

      // ---- merge the round's kept keys into the top-K (ranks by counting; keys are unique)
      const int m = s_acc < a.acc_cap ? s_acc : int(a.acc_cap);
      for (int base = 0; base < m; base += kMergeChunk) {
        const int cnt = (m - base < kMergeChunk) ? m - base : kMergeChunk;
        const unsigned long long kth = (topk_n == K) ? topk[K - 1] : ~0ull;
        if (tid == 0) s_nc = 0;
        __syncthreads();
        for (int i = tid; i < cnt; i += kThreads) {
          const unsigned long long key = load_l2(acc + base + i);
          if (key < kth) cand[atomicAdd(&s_nc, 1)] = key;
        }
        __syncthreads();
        const int n = s_nc;
        if (n > 0) {
          for (int i = tid; i < topk_n; i += kThreads) cand[n + i] = topk[i];
          __syncthreads();
          const int tot = n + topk_n;
          for (int i = tid; i < tot; i += kThreads) {
            const unsigned long long key = cand[i];
            int rank = 0;
            for (int j = 0; j < tot; ++j) rank += cand[j] < key;
            if (rank < K) newk[rank] = key;
          }
          __syncthreads();
          topk_n = tot < K ? tot : K;
          for (int i = tid; i < topk_n; i += kThreads) topk[i] = newk[i];
        }
        __syncthreads();
      }
      b = e;
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
      atomicAdd(&s_stat[0], st_dco);
      atomicAdd(&s_stat[1], st_dims);
      atomicAdd(&s_stat[2], st_kept);
      atomicAdd(&s_stat[3], st_rr);
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
