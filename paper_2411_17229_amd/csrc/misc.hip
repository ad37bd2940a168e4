// Small element-wise kernels: padding, gathers, norms, fills and the k-means update.
// Fills are kernels (not hipMemsetAsync) so that every step can live in a captured graph.
#include "kernels.h"

namespace dade {
namespace {

constexpr int kBlock = 256;

inline int blocks_for(int64_t n, int per = kBlock) {
  int64_t b = (n + per - 1) / per;
  return int(b < 65535 * 16 ? b : 65535 * 16);
}

__global__ void pad_rows_kernel(const float* __restrict__ src, int64_t rows, int cols, int64_t lds,
                                float* __restrict__ dst, int ld) {
  const int64_t total = rows * ld;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t r = e / ld;
    const int c = int(e % ld);
    dst[e] = c < cols ? src[r * lds + c] : 0.f;
  }
}

__global__ void gather_rows_kernel(const float* __restrict__ src, int ld,
                                   const int64_t* __restrict__ rows, int64_t count,
                                   float* __restrict__ dst) {
  const int64_t total = count * ld;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t r = e / ld;
    dst[e] = src[rows[r] * ld + e % ld];
  }
}

// One wave per row: ||A_r||^2 in FP32 (fixed order: lane-strided partial sums, then a
// fixed butterfly).
__global__ void row_norms_kernel(const float* __restrict__ A, int64_t rows, int ld,
                                 float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t r = blockIdx.x * int64_t(blockDim.x / 64) + (threadIdx.x >> 6);
  if (r >= rows) return;
  float s = 0.f;
  for (int c = lane; c < ld; c += 64) {
    const float v = A[r * ld + c];
    s = fmaf(v, v, s);
  }
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) out[r] = s;
}

template <typename T>
__global__ void fill_kernel(T* p, int64_t n, T v) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < n;
       e += int64_t(gridDim.x) * blockDim.x)
    p[e] = v;
}

// One wave per row: add the row into its centroid's FP64 sums.
__global__ void kmeans_accumulate_kernel(const float* __restrict__ X, int64_t n, int ld,
                                         const unsigned long long* __restrict__ best,
                                         double* __restrict__ sums, int* __restrict__ counts) {
  const int lane = threadIdx.x & 63;
  const int64_t r = blockIdx.x * int64_t(blockDim.x / 64) + (threadIdx.x >> 6);
  if (r >= n) return;
  const int c = int(static_cast<uint32_t>(best[r]));
  for (int k = lane; k < ld; k += 64) atomicAdd(sums + int64_t(c) * ld + k, double(X[r * ld + k]));
  if (lane == 0) atomicAdd(counts + c, 1);
}

// Empty clusters keep their centroid.
__global__ void kmeans_finalize_kernel(const double* __restrict__ sums,
                                       const int* __restrict__ counts, int nlist, int ld,
                                       float* __restrict__ C) {
  const int64_t total = int64_t(nlist) * ld;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int c = int(e / ld);
    const int cnt = counts[c];
    if (cnt > 0) C[e] = float(sums[e] / double(cnt));
  }
}

__global__ void labels_kernel(const unsigned long long* __restrict__ best, int64_t n,
                              int32_t* __restrict__ labels) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < n;
       e += int64_t(gridDim.x) * blockDim.x)
    labels[e] = int32_t(static_cast<uint32_t>(best[e]));
}

}  // namespace

hipError_t launch_pad_rows(const float* src, int64_t rows, int cols, int64_t lds, float* dst, int ld,
                           hipStream_t s) {
  if (rows == 0) return hipSuccess;
  hipLaunchKernelGGL(pad_rows_kernel, dim3(blocks_for(rows * ld)), dim3(kBlock), 0, s, src, rows,
                     cols, lds, dst, ld);
  return hipGetLastError();
}

hipError_t launch_gather_rows(const float* src, int ld, const int64_t* rows, int64_t count,
                              float* dst, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_rows_kernel, dim3(blocks_for(count * ld)), dim3(kBlock), 0, s, src,
                     ld, rows, count, dst);
  return hipGetLastError();
}

hipError_t launch_row_norms(const float* A, int64_t rows, int ld, float* out, hipStream_t s) {
  if (rows == 0) return hipSuccess;
  hipLaunchKernelGGL(row_norms_kernel, dim3(int((rows + 3) / 4)), dim3(kBlock), 0, s, A, rows,
                     ld, out);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel<unsigned long long>, dim3(blocks_for(n)), dim3(kBlock), 0, s, p,
                     n, v);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int* p, int64_t n, int v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel<int>, dim3(blocks_for(n)), dim3(kBlock), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel<double>, dim3(blocks_for(n)), dim3(kBlock), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_kmeans_accumulate(const float* X, int64_t n, int ld,
                                    const unsigned long long* best, double* sums, int* counts,
                                    hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(kmeans_accumulate_kernel, dim3(int((n + 3) / 4)), dim3(kBlock), 0, s, X, n,
                     ld, best, sums, counts);
  return hipGetLastError();
}

hipError_t launch_kmeans_finalize(const double* sums, const int* counts, int nlist, int ld,
                                  float* centroids, hipStream_t s) {
  hipLaunchKernelGGL(kmeans_finalize_kernel, dim3(blocks_for(int64_t(nlist) * ld)), dim3(kBlock),
                     0, s, sums, counts, nlist, ld, centroids);
  return hipGetLastError();
}

hipError_t launch_labels_from_best(const unsigned long long* best, int64_t n, int32_t* labels,
                                   hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(labels_kernel, dim3(blocks_for(n)), dim3(kBlock), 0, s, best, n, labels);
  return hipGetLastError();
}

}  // namespace dade
