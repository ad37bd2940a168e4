// Probe selection: for each query, the nprobe lists whose centroids are nearest (end of the
// Methodology section: IVF scans the N_probe clusters nearest to the query), ordered by
// (squared distance, list id).  One workgroup per query sorts nlist 64-bit keys
// (distance bits << 32 | list id) with a bitonic network in LDS.
#include "kernels.h"

namespace dade {
namespace {

constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void select_kernel(const float* __restrict__ pd, int ld_pd,
                                                        const float* __restrict__ qrot, int ld_q,
                                                        int dim_p, int nlist, int P, int nprobe,
                                                        int32_t* __restrict__ probes) {
  extern __shared__ unsigned long long keys[];   // P >= 4 entries
  const int q = blockIdx.x;
  const int tid = threadIdx.x;
  // ||q'||^2 (fixed order: thread-strided partials, wave butterfly, then 4 partials in order);
  // the first 4 key slots hold the wave partials before the keys are written.
  float s = 0.f;
  for (int c = tid; c < dim_p; c += kBlock) {
    const float v = qrot[int64_t(q) * ld_q + c];
    s = fmaf(v, v, s);
  }
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  float* red = reinterpret_cast<float*>(keys);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  const float qn = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  for (int c = tid; c < P; c += kBlock) {
    unsigned long long k = ~0ull;
    if (c < nlist) {
      float d = qn + pd[int64_t(q) * ld_pd + c];
      d = d > 0.f ? d : 0.f;
      k = make_key(d, uint32_t(c));
    }
    keys[c] = k;
  }
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < P; i += kBlock) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const unsigned long long a = keys[i], b = keys[ixj];
          const bool up = (i & k) == 0;
          if ((a > b) == up) {
            keys[i] = b;
            keys[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < nprobe; i += kBlock)
    probes[int64_t(q) * nprobe + i] = i < nlist ? int32_t(key_id(keys[i])) : -1;
}

}  // namespace

hipError_t launch_select_probes(const float* pd, int ld_pd, const float* qrot, int ld_q, int nq,
                                int dim_p, int nlist, int nprobe, int32_t* probes,
                                hipStream_t s) {
  if (nq == 0) return hipSuccess;
  int P = 4;
  while (P < nlist) P <<= 1;
  const size_t lds = size_t(P) * sizeof(unsigned long long);
  hipLaunchKernelGGL(select_kernel, dim3(nq), dim3(kBlock), lds, s, pd, ld_pd, qrot, ld_q, dim_p,
                     nlist, P, nprobe, probes);
  return hipGetLastError();
}

}  // namespace dade
