// Probe selection: for each query, the nprobe lists whose centroids are nearest (end of the
// Methodology section: IVF scans the N_probe clusters nearest to the query), ordered by
// (squared distance, list id).
//
// The input row holds ||c - mu||^2 - 2 (q - mu).(c - mu) per list: the squared distance minus
// ||q - mu||^2, a constant of the row, so it orders the lists like their distances.
// One wave per query.  The nlist values sit in registers (KPL per lane) as order-preserving
// 32-bit patterns.  A bound T with at least nprobe keys at or below it is found, the keys at or
// below T are gathered into LDS and sorted by (value bits << 32 | list id) with a bitonic
// network, and the first nprobe are the probes.
#include "kernels.h"

namespace dade {
namespace {

__device__ inline unsigned wave_sum(unsigned v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int KPL>
__global__ __launch_bounds__(64) void select_kernel(const float* __restrict__ pd, int ld_pd, int nlist, int P,
                                                    int nprobe, int32_t* __restrict__ probes) {
  extern __shared__ unsigned long long sel[];   // P entries
  const int q = blockIdx.x;
  const int lane = threadIdx.x;
  // lane holds columns c = 64 j + lane, j < KPL
  uint32_t bits[KPL];
  uint32_t lo = 0xFFFFFFFFu, hi = 0u;
#pragma unroll
  for (int j = 0; j < KPL; ++j) {
    const int c = 64 * j + lane;
    const float v = pd[int64_t(q) * ld_pd + (c < nlist ? c : nlist - 1)];   // in-bounds load
    const uint32_t b = ordered_bits(v);
    bits[j] = c < nlist ? b : 0xFFFFFFFFu;   // absent columns sort last and are never selected
    if (c < nlist) {
      lo = b < lo ? b : lo;
      hi = b > hi ? b : hi;
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const uint32_t l2 = __shfl_xor(lo, o, 64), h2 = __shfl_xor(hi, o, 64);
    lo = l2 < lo ? l2 : lo;
    hi = h2 > hi ? h2 : hi;
  }
  // T: a value with at least nprobe keys at or below it (nprobe <= nlist).  For nprobe <= 64
  // the nprobe-th smallest lane minimum is one (the nprobe smallest minima come from distinct
  // lanes), and typically only a few more keys lie below it; otherwise T is the nprobe-th
  // smallest key itself, from a binary search on the bit patterns.
  uint32_t T;
  if (nprobe <= 64) {
    uint32_t mn = 0xFFFFFFFFu;
#pragma unroll
    for (int j = 0; j < KPL; ++j) mn = bits[j] < mn ? bits[j] : mn;
    uint32_t a = lo, b = hi;
    while (a < b) {   // the nprobe-th smallest lane minimum
      const uint32_t mid = a + (b - a) / 2;
      if (__popcll(__ballot(mn <= mid)) >= nprobe) b = mid;
      else a = mid + 1;
    }
    T = a;
  } else {
    while (lo < hi) {
      const uint32_t mid = lo + (hi - lo) / 2;
      unsigned cnt = 0;
#pragma unroll
      for (int j = 0; j < KPL; ++j) cnt += bits[j] <= mid ? 1u : 0u;
      if (wave_sum(cnt) >= unsigned(nprobe)) hi = mid;
      else lo = mid + 1;
    }
    T = lo;
  }
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
void launch_kpl(dim3 g, size_t lds, hipStream_t s, const float* pd, int ld_pd, int nlist, int P, int nprobe,
                int32_t* probes) {
  hipLaunchKernelGGL((select_kernel<KPL>), g, dim3(64), lds, s, pd, ld_pd, nlist, P, nprobe, probes);
}

}  // namespace

hipError_t launch_select_probes(const float* pd, int ld_pd, int nq, int nlist, int nprobe, int32_t* probes,
                                hipStream_t s) {
  if (nq == 0) return hipSuccess;
  if (nprobe < 1 || nprobe > nlist || nlist > kMaxNlist) return hipErrorInvalidValue;
  int P = 1;
  while (P < nlist) P <<= 1;
  const size_t lds = size_t(P) * sizeof(unsigned long long);
  const dim3 g(nq);
  if (nlist <= 64 * 16)
    launch_kpl<16>(g, lds, s, pd, ld_pd, nlist, P, nprobe, probes);
  else if (nlist <= 64 * 32)
    launch_kpl<32>(g, lds, s, pd, ld_pd, nlist, P, nprobe, probes);
  else if (nlist <= 64 * 64)
    launch_kpl<64>(g, lds, s, pd, ld_pd, nlist, P, nprobe, probes);
  else
    launch_kpl<128>(g, lds, s, pd, ld_pd, nlist, P, nprobe, probes);
  return hipGetLastError();
}

}  // namespace dade
