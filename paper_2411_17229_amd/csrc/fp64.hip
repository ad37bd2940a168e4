// FP64 kernels of the offline path: the mean and second moment of the data (Lemma 1,
// Eq. (10)), FP64 products for the rotation of calibration pairs and centroids, and the
// per-pair prefix fractions f_d behind the eps_d estimate of Eq. (14).
#include "kernels.h"

namespace dade {
namespace {

constexpr int kBlock = 256;

// Column sums of X (FP64), block = a chunk of rows, thread = a set of columns.
__global__ void column_sum_kernel(const float* __restrict__ X, int64_t n, int ld, int dim,
                                  int64_t rows_per_block, double* __restrict__ sum) {
  const int64_t r0 = blockIdx.x * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < n ? r0 + rows_per_block : n;
  for (int c = threadIdx.x; c < dim; c += blockDim.x) {
    double s = 0.0;
    for (int64_t r = r0; r < r1; ++r) s += double(X[r * ld + c]);
    atomicAdd(sum + c, s);
  }
}

__global__ void scale_kernel(double* p, int n, double f) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] *= f;
}

// One 64 x 64 tile (ti <= tj) of sum_r (x_r - mu)(x_r - mu)^T over a chunk of rows, added
// atomically (scaled by 1/n) into C and mirrored into the lower triangle.
__global__ __launch_bounds__(kBlock) void covariance_kernel(
    const float* __restrict__ X, int64_t n, int ld, int dim, const double* __restrict__ mu,
    double inv_n, int ntiles, int64_t rows_per_chunk, double* __restrict__ C, int ldc) {
  __shared__ double Ai[16][64];
  __shared__ double Bj[16][64];
  // decode the upper-triangular tile pair
  int p = blockIdx.x, ti = 0;
  while (p >= ntiles - ti) { p -= ntiles - ti; ++ti; }
  const int tj = ti + p;
  const int64_t r0 = blockIdx.y * rows_per_chunk;
  const int64_t r1 = r0 + rows_per_chunk < n ? r0 + rows_per_chunk : n;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc[4][4] = {};
  for (int64_t rb = r0; rb < r1; rb += 16) {
    for (int e = threadIdx.x; e < 16 * 64; e += kBlock) {
      const int rr = e / 64, cc = e % 64;
      const int64_t r = rb + rr;
      const int ci = ti * 64 + cc, cj = tj * 64 + cc;
      Ai[rr][cc] = (r < r1 && ci < dim) ? double(X[r * ld + ci]) - mu[ci] : 0.0;
      Bj[rr][cc] = (r < r1 && cj < dim) ? double(X[r * ld + cj]) - mu[cj] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < 16; ++rr) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = Ai[rr][ty * 4 + u];
#pragma unroll
      for (int u = 0; u < 4; ++u) b[u] = Bj[rr][tx * 4 + u];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = ti * 64 + ty * 4 + u, j = tj * 64 + tx * 4 + v;
      if (i < dim && j < dim) {
        atomicAdd(C + int64_t(i) * ldc + j, acc[u][v] * inv_n);
        if (ti != tj) atomicAdd(C + int64_t(j) * ldc + i, acc[u][v] * inv_n);
      }
    }
}

// C = A B (FP64), 64 x 64 tiles, 4 x 4 outputs per thread.
__global__ __launch_bounds__(kBlock) void dgemm_kernel(const double* __restrict__ A, int lda,
                                                       const double* __restrict__ B, int ldb,
                                                       double* __restrict__ C, int ldc, int M,
                                                       int N, int K) {
  __shared__ double As[16][64];
  __shared__ double Bs[16][64];
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int e = threadIdx.x; e < 16 * 64; e += kBlock) {
      const int kk = e % 16, mm = e / 16;
      const int gm = m0 + mm, gk = k0 + kk;
      As[kk][mm] = (gm < M && gk < K) ? A[int64_t(gm) * lda + gk] : 0.0;
      const int kb = e / 64, nn = e % 64;
      const int gn = n0 + nn, gkb = k0 + kb;
      Bs[kb][nn] = (gn < N && gkb < K) ? B[int64_t(gkb) * ldb + gn] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 16; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = As[kk][ty * 4 + u];
#pragma unroll
      for (int u = 0; u < 4; ++u) b[u] = Bs[kk][tx * 4 + u];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = m0 + ty * 4 + u, j = n0 + tx * 4 + v;
      if (i < M && j < N) C[int64_t(i) * ldc + j] = acc[u][v];
    }
}

// One wave per pair: the FP64 difference row and its squared norm (fixed reduction order).
__global__ void pair_diff_kernel(const float* __restrict__ X, int ld,
                                 const int64_t* __restrict__ pairs, int64_t m,
                                 double* __restrict__ delta, double* __restrict__ dis2) {
  const int lane = threadIdx.x & 63;
  const int64_t i = blockIdx.x * int64_t(blockDim.x / 64) + (threadIdx.x >> 6);
  if (i >= m) return;
  const int64_t a = pairs[2 * i], b = pairs[2 * i + 1];
  double s = 0.0;
  for (int k = lane; k < ld; k += 64) {
    const double d = double(X[a * ld + k]) - double(X[b * ld + k]);
    delta[i * ld + k] = d;
    s = fma(d, d, s);
  }
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) dis2[i] = s;
}

template <typename T>
__device__ inline double load_stored(const void* p, int64_t e);
template <>
__device__ inline double load_stored<float>(const void* p, int64_t e) {
  return double(static_cast<const float*>(p)[e]);
}
template <>
__device__ inline double load_stored<__hip_bfloat16>(const void* p, int64_t e) {
  const uint32_t u = uint32_t(static_cast<const uint16_t*>(p)[e]) << 16;
  return double(__builtin_bit_cast(float, u));
}
template <>
__device__ inline double load_stored<__half>(const void* p, int64_t e) {
  return double(__half2float(static_cast<const __half*>(p)[e]));
}

template <typename T>
__global__ void pair_diff_stored_kernel(const void* __restrict__ store, int64_t rows, int ld,
                                        const int64_t* __restrict__ pos,
                                        const int64_t* __restrict__ pairs, int64_t m,
                                        double* __restrict__ delta) {
  const int lane = threadIdx.x & 63;
  const int64_t i = blockIdx.x * int64_t(blockDim.x / 64) + (threadIdx.x >> 6);
  if (i >= m) return;
  const int64_t pa = pos[pairs[2 * i]], pb = pos[pairs[2 * i + 1]];
  for (int k = lane; k < ld; k += 64)
    delta[i * ld + k] = load_stored<T>(store, stored_index(pa, k, rows, ld)) -
                        load_stored<T>(store, stored_index(pb, k, rows, ld));
}

// One thread per pair: running prefix of squared rotated coordinates.
__global__ void prefix_fraction_kernel(const double* __restrict__ Y, int ld, int64_t m, int dim,
                                       const double* __restrict__ dis2, double* __restrict__ f,
                                       double* __restrict__ rel) {
  const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
  if (i >= m) return;
  const double inv = 1.0 / dis2[i];
  double s = 0.0;
  for (int d = 0; d < dim; ++d) {
    const double y = Y[i * ld + d];
    s = fma(y, y, s);
    if (d + 1 < dim) f[int64_t(d) * m + i] = s * inv;
  }
  rel[i] = fabs(s - dis2[i]) * inv;
}

}  // namespace

hipError_t launch_column_mean(const float* X, int64_t n, int ld, int dim, double* mean,
                              hipStream_t s) {
  hipError_t e = launch_fill_f64(mean, dim, 0.0, s);
  if (e != hipSuccess) return e;
  const int64_t per = 1024;
  const int64_t blocks = (n + per - 1) / per;
  hipLaunchKernelGGL(column_sum_kernel, dim3(int(blocks)), dim3(kBlock), 0, s, X, n, ld, dim, per,
                     mean);
  hipLaunchKernelGGL(scale_kernel, dim3((dim + 255) / 256), dim3(256), 0, s, mean, dim,
                     1.0 / double(n));
  return hipGetLastError();
}

hipError_t launch_covariance(const float* X, int64_t n, int ld, int dim, const double* mean,
                             double* C, int ldc, hipStream_t s) {
  hipError_t e = launch_fill_f64(C, int64_t(dim) * ldc, 0.0, s);
  if (e != hipSuccess) return e;
  const int ntiles = (dim + 63) / 64;
  const int npairs = ntiles * (ntiles + 1) / 2;
  int64_t nchunks = 4096 / npairs;
  if (nchunks < 1) nchunks = 1;
  if (nchunks > (n + 15) / 16) nchunks = (n + 15) / 16;
  int64_t per = (n + nchunks - 1) / nchunks;
  per = (per + 15) / 16 * 16;
  nchunks = (n + per - 1) / per;
  hipLaunchKernelGGL(covariance_kernel, dim3(npairs, int(nchunks)), dim3(kBlock), 0, s, X, n, ld,
                     dim, mean, 1.0 / double(n), ntiles, per, C, ldc);
  return hipGetLastError();
}

hipError_t launch_dgemm(const double* A, int lda, const double* B, int ldb, double* C, int ldc,
                        int M, int N, int K, hipStream_t s) {
  if (M == 0 || N == 0) return hipSuccess;
  hipLaunchKernelGGL(dgemm_kernel, dim3((N + 63) / 64, (M + 63) / 64), dim3(kBlock), 0, s, A, lda,
                     B, ldb, C, ldc, M, N, K);
  return hipGetLastError();
}

hipError_t launch_pair_diff(const float* X, int ld, const int64_t* pairs, int64_t m,
                            double* delta, double* dis2, hipStream_t s) {
  if (m == 0) return hipSuccess;
  hipLaunchKernelGGL(pair_diff_kernel, dim3(int((m + 3) / 4)), dim3(kBlock), 0, s, X, ld, pairs,
                     m, delta, dis2);
  return hipGetLastError();
}

hipError_t launch_pair_diff_stored(const void* store, int dtype, int64_t rows, int ld,
                                   const int64_t* pos, const int64_t* pairs, int64_t m,
                                   double* delta, hipStream_t s) {
  if (m == 0) return hipSuccess;
  const dim3 g(int((m + 3) / 4)), b(kBlock);
  if (dtype == 0)
    hipLaunchKernelGGL(pair_diff_stored_kernel<float>, g, b, 0, s, store, rows, ld, pos, pairs, m,
                       delta);
  else if (dtype == 1)
    hipLaunchKernelGGL(pair_diff_stored_kernel<__hip_bfloat16>, g, b, 0, s, store, rows, ld, pos,
                       pairs, m, delta);
  else
    hipLaunchKernelGGL(pair_diff_stored_kernel<__half>, g, b, 0, s, store, rows, ld, pos, pairs, m,
                       delta);
  return hipGetLastError();
}

hipError_t launch_prefix_fraction(const double* Y, int ld, int64_t m, int dim,
                                  const double* dis2, double* f, double* rel, hipStream_t s) {
  if (m == 0) return hipSuccess;
  hipLaunchKernelGGL(prefix_fraction_kernel, dim3(int((m + 255) / 256)), dim3(256), 0, s, Y, ld, m,
                     dim, dis2, f, rel);
  return hipGetLastError();
}

}  // namespace dade
