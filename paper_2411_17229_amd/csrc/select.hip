// Probe selection: for each query, the nprobe lists whose centroids are nearest (end of the
// Methodology section: IVF scans the N_probe clusters nearest to the query), ordered by
// (squared distance, list id).
//
// One wave per query.  The nlist distances sit in registers (KPL per lane); a binary search on
// their bit patterns (non-negative floats order like their bits) finds the nprobe-th smallest
// value T with a wave-wide count per step; the keys at or below T are then gathered into LDS and
// sorted by (distance bits << 32 | list id) with a bitonic network.
#include "kernels.h"

namespace dade {
namespace {

__device__ inline unsigned wave_sum(unsigned v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int KPL>
__global__ __launch_bounds__(64) void select_kernel(const float* __restrict__ pd, int ld_pd,
                                                    const float* __restrict__ qrot, int ld_q,
                                                    int dim_p, int nlist, int P, int nprobe,
                                                    int32_t* __restrict__ probes) {
  extern __shared__ unsigned long long sel[];   // P entries
  const int q = blockIdx.x;
  const int lane = threadIdx.x;
  // ||q'||^2: lane-strided FMA partials, then a fixed butterfly
  float s = 0.f;
  for (int c = lane; c < dim_p; c += 64) {
    const float v = qrot[int64_t(q) * ld_q + c];
    s = fmaf(v, v, s);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  // lane holds columns c = 64 j + lane, j < KPL
  uint32_t bits[KPL];
  uint32_t lo = 0xFFFFFFFFu, hi = 0u;
#pragma unroll
  for (int j = 0; j < KPL; ++j) {
    const int c = 64 * j + lane;
    uint32_t b = 0xFFFFFFFFu;   // absent columns sort last and are never selected
    if (c < nlist) {
      float d = s + pd[int64_t(q) * ld_pd + c];
      d = d > 0.f ? d : 0.f;
      b = __builtin_bit_cast(uint32_t, d);
      lo = b < lo ? b : lo;
      hi = b > hi ? b : hi;
    }
    bits[j] = b;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const uint32_t l2 = __shfl_xor(lo, o, 64), h2 = __shfl_xor(hi, o, 64);
    lo = l2 < lo ? l2 : lo;
    hi = h2 > hi ? h2 : hi;
  }
  // smallest T with #{bits <= T} >= nprobe (nprobe <= nlist)
  while (lo < hi) {
    const uint32_t mid = lo + (hi - lo) / 2;
    unsigned cnt = 0;
#pragma unroll
    for (int j = 0; j < KPL; ++j) cnt += bits[j] <= mid ? 1u : 0u;
    if (wave_sum(cnt) >= unsigned(nprobe)) hi = mid;
    else lo = mid + 1;
  }
  const uint32_t T = lo;
  // gather the keys at or below T
  int total = 0;
#pragma unroll
  for (int j = 0; j < KPL; ++j) {
    const bool take = bits[j] <= T && bits[j] != 0xFFFFFFFFu;
    const unsigned long long m = __ballot(take);
    if (take) {
      const int below = int(__builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u)));
      sel[total + below] = (static_cast<unsigned long long>(bits[j]) << 32) | uint32_t(64 * j + lane);
    }
    total += __popcll(m);
  }
  int P2 = 1;
  while (P2 < total) P2 <<= 1;
  for (int i = total + lane; i < P2; i += 64) sel[i] = ~0ull;
  __syncthreads();
  for (int k = 2; k <= P2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = lane; i < P2; i += 64) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const unsigned long long a = sel[i], b = sel[ixj];
          if ((a > b) == ((i & k) == 0)) {
            sel[i] = b;
            sel[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = lane; i < nprobe; i += 64) probes[int64_t(q) * nprobe + i] = int32_t(key_id(sel[i]));
}

template <int KPL>
void launch_kpl(dim3 g, size_t lds, hipStream_t s, const float* pd, int ld_pd, const float* qrot, int ld_q,
                int dim_p, int nlist, int P, int nprobe, int32_t* probes) {
  hipLaunchKernelGGL((select_kernel<KPL>), g, dim3(64), lds, s, pd, ld_pd, qrot, ld_q, dim_p, nlist, P,
                     nprobe, probes);
}

}  // namespace

hipError_t launch_select_probes(const float* pd, int ld_pd, const float* qrot, int ld_q, int nq,
                                int dim_p, int nlist, int nprobe, int32_t* probes,
                                hipStream_t s) {
  if (nq == 0) return hipSuccess;
  if (nprobe < 1 || nprobe > nlist || nlist > kMaxNlist) return hipErrorInvalidValue;
  int P = 1;
  while (P < nlist) P <<= 1;
  const size_t lds = size_t(P) * sizeof(unsigned long long);
  const dim3 g(nq);
  if (nlist <= 64 * 16)
    launch_kpl<16>(g, lds, s, pd, ld_pd, qrot, ld_q, dim_p, nlist, P, nprobe, probes);
  else if (nlist <= 64 * 32)
    launch_kpl<32>(g, lds, s, pd, ld_pd, qrot, ld_q, dim_p, nlist, P, nprobe, probes);
  else if (nlist <= 64 * 64)
    launch_kpl<64>(g, lds, s, pd, ld_pd, qrot, ld_q, dim_p, nlist, P, nprobe, probes);
  else
    launch_kpl<128>(g, lds, s, pd, ld_pd, qrot, ld_q, dim_p, nlist, P, nprobe, probes);
  return hipGetLastError();
}

}  // namespace dade
