// FP32 GEMM on gfx950 matrix cores (v_mfma_f32_32x32x2_f32) with fused epilogues.
//
// Used for the dense contractions of the path: the query rotation Q' = (Q - mu) W fused with
// the query-centroid distances of probe selection (one GEMM against [W | (C - mu)^T]; W is
// orthogonal, so (q - mu).(c - mu) needs no rotation), the k-means assignment (argmin fused, no
// distance matrix is written) and the packing of the rotated base (X[ids] - mu) W into the
// list-ordered store.
//
// Tiling: a 256-thread workgroup (4 wave64s, 2 x 2) owns a BM x BN tile of C; each wave owns
// (BM/2) x (BN/2) as a grid of 32 x 32 MFMA accumulators.  Each K-step stages a BK x BM slice
// of A and a BK x BN slice of B in LDS, k-major, so that the MFMA operand reads of a half-wave
// hit 32 consecutive floats; the next slice is fetched into registers during the MFMAs.  The blockIdx -> tile mapping keeps consecutive N-tiles of one
// M-tile on one XCD (blocks are dealt round-robin to the 8 XCDs).
#include "kernels.h"

namespace dade {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kThreads = 256;

template <int BM, int BN, int BK, int EPI, bool BT>
__global__ __launch_bounds__(kThreads) void gemm_kernel(GemmArgs g) {
  constexpr int WM = BM / 2, WN = BN / 2;      // per-wave tile
  constexpr int TM = WM / 32, TN = WN / 32;    // MFMA tiles per wave
  constexpr int PA = BM + 4, PB = BN + 4;      // padded LDS rows
  constexpr int LA = BM * (BK / 4) / kThreads; // float4 loads per thread per K-slice of A
  constexpr int LB = BN * (BK / 4) / kThreads; // ... and of B
  static_assert(LA >= 1 && LB >= 1, "tile too small for the thread count");
  __shared__ float As[BK * PA];
  __shared__ float Bs[BK * PB];

  const int tiles_n = (g.N + BN - 1) / BN;
  const int tiles_m = (g.M + BM - 1) / BM;
  const int nblk = tiles_n * tiles_m;
  // XCD-aware remap: hardware sends block b to XCD b % 8; give each XCD a contiguous range
  // of logical tiles so neighbouring tiles (sharing an A panel) share that XCD's L2.
  int b = blockIdx.x;
  int logical = b;
  if (nblk >= 64 && nblk % 8 == 0) logical = (b % 8) * (nblk / 8) + b / 8;
  const int tm = logical / tiles_n, tn = logical % tiles_n;
  const int m0 = tm * BM, n0 = tn * BN;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;

  floatx16 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

  // The K-slice [k0, k0 + BK) of A and B is fetched into registers one slice ahead of the
  // MFMAs that use it, so global loads overlap the matrix work.
  const float* arow[LA];
#pragma unroll
  for (int l = 0; l < LA; ++l) {
    const int r = (tid + l * kThreads) / (BK / 4);
    const int gm = m0 + r;
    arow[l] = nullptr;
    if (gm < g.M) arow[l] = g.A + (g.a_rows ? int64_t(g.a_rows[gm]) : int64_t(gm)) * g.lda;
  }
  float4 ra[LA], rb[LB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int l = 0; l < LA; ++l) {
      const int q = (tid + l * kThreads) % (BK / 4);
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (arow[l]) {
        v = *reinterpret_cast<const float4*>(arow[l] + k0 + 4 * q);
        if (g.a_shift) {
          const float4 sh = *reinterpret_cast<const float4*>(g.a_shift + k0 + 4 * q);
          v.x -= sh.x; v.y -= sh.y; v.z -= sh.z; v.w -= sh.w;
        }
      }
      ra[l] = v;
    }
#pragma unroll
    for (int l = 0; l < LB; ++l) {
      const int e = tid + l * kThreads;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (!BT) {
        const int kk = e / (BN / 4), q = e % (BN / 4);
        const int gn = n0 + 4 * q;
        const float* src = g.B + int64_t(k0 + kk) * g.ldb + gn;
        if (gn + 3 < g.N) {
          v = *reinterpret_cast<const float4*>(src);
        } else {
          if (gn + 0 < g.N) v.x = src[0];
          if (gn + 1 < g.N) v.y = src[1];
          if (gn + 2 < g.N) v.z = src[2];
        }
      } else {
        const int c = e / (BK / 4), q = e % (BK / 4);
        const int gn = n0 + c;
        if (gn < g.N) v = *reinterpret_cast<const float4*>(g.B + int64_t(gn) * g.ldb + k0 + 4 * q);
      }
      rb[l] = v;
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int l = 0; l < LA; ++l) {
      const int e = tid + l * kThreads;
      const int r = e / (BK / 4), q = e % (BK / 4);
      As[(4 * q + 0) * PA + r] = ra[l].x;
      As[(4 * q + 1) * PA + r] = ra[l].y;
      As[(4 * q + 2) * PA + r] = ra[l].z;
      As[(4 * q + 3) * PA + r] = ra[l].w;
    }
#pragma unroll
    for (int l = 0; l < LB; ++l) {
      const int e = tid + l * kThreads;
      if (!BT) {
        const int kk = e / (BN / 4), q = e % (BN / 4);
        *reinterpret_cast<float4*>(&Bs[kk * PB + 4 * q]) = rb[l];
      } else {
        const int c = e / (BK / 4), q = e % (BK / 4);
        Bs[(4 * q + 0) * PB + c] = rb[l].x;
        Bs[(4 * q + 1) * PB + c] = rb[l].y;
        Bs[(4 * q + 2) * PB + c] = rb[l].z;
        Bs[(4 * q + 3) * PB + c] = rb[l].w;
      }
    }
  };

  fetch(0);
  for (int k0 = 0; k0 < g.K; k0 += BK) {
    __syncthreads();   // the previous slice's MFMAs are done with the LDS tiles
    stage();
    __syncthreads();
    if (k0 + BK < g.K) fetch(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 2) {
      const int kr = kk + (lane >> 5);
      float av[TM], bv[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) av[i] = As[kr * PA + wm + 32 * i + (lane & 31)];
#pragma unroll
      for (int j = 0; j < TN; ++j) bv[j] = Bs[kr * PB + wn + 32 * j + (lane & 31)];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
  }

  // ---- epilogue.  Accumulator v of a lane holds C[row][col] with
  //      col = lane % 32, row = 8 (v / 4) + 4 (lane / 32) + v % 4   (32x32 tile).
#pragma unroll
  for (int i = 0; i < TM; ++i) {
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int col = n0 + wn + 32 * j + (lane & 31);
      if (EPI == kEpiArgmin) {
        const bool cok = col < g.N;
        const float cn = cok ? g.col_norm[col] : 0.f;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int row = m0 + wm + 32 * i + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
          unsigned long long key = ~0ull;
          if (cok) key = (static_cast<unsigned long long>(ordered_bits(cn - 2.f * acc[i][j][v])) << 32) |
                         static_cast<unsigned>(col);
#pragma unroll
          for (int off = 16; off >= 1; off >>= 1) {
            const unsigned long long o = __shfl_xor(key, off, 32);
            key = o < key ? o : key;
          }
          if ((lane & 31) == 0 && row < g.M) atomicMin(g.row_best + row, key);
        }
      } else if (EPI == kEpiRotateProbe) {
        // columns [0, split_col): the rotated query; the rest: ||c - mu||^2 - 2 (q - mu).(c - mu)
        if (col >= g.N) continue;
        const bool rot = col < g.split_col;
        const float cn = rot ? 0.f : g.col_norm[col - g.split_col];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int row = m0 + wm + 32 * i + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
          if (row >= g.M) continue;
          const float x = acc[i][j][v];
          if (rot) static_cast<float*>(g.C)[int64_t(row) * g.ldc + col] = x;
          else g.C2[int64_t(row) * g.ldc2 + (col - g.split_col)] = cn - 2.f * x;
        }
      } else {
        if (col >= g.N) continue;
        const float cn = (EPI == kEpiProbe) ? g.col_norm[col] : 0.f;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int row = m0 + wm + 32 * i + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
          if (row >= g.M) continue;
          const float x = acc[i][j][v];
          const int64_t o = (EPI >= kEpiPackF32 && g.split_rows > 0)
                                ? stored_index(row, col, g.split_rows, g.ldc)
                                : int64_t(row) * g.ldc + col;
          if (EPI == kEpiStore || EPI == kEpiPackF32) {
            static_cast<float*>(g.C)[o] = x;
          } else if (EPI == kEpiProbe) {
            static_cast<float*>(g.C)[o] = cn - 2.f * x;
          } else if (EPI == kEpiPackBF16) {
            static_cast<uint16_t*>(g.C)[o] = f32_to_bf16_rne(x);
          } else if (EPI == kEpiPackF16) {
            static_cast<__half*>(g.C)[o] = __float2half_rn(x);
          }
        }
      }
    }
  }
}

template <int BM, int BN, int BK, int EPI>
hipError_t launch_tile(const GemmArgs& a, hipStream_t s) {
  const int tiles = ((a.M + BM - 1) / BM) * ((a.N + BN - 1) / BN);
  if (tiles == 0) return hipSuccess;
  if (a.b_trans)
    hipLaunchKernelGGL((gemm_kernel<BM, BN, BK, EPI, true>), dim3(tiles), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL((gemm_kernel<BM, BN, BK, EPI, false>), dim3(tiles), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

template <int EPI>
hipError_t launch_epi(const GemmArgs& a, hipStream_t s) {
  // Large problems use 128 x 128 tiles (2 x 2 MFMA tiles per wave), small ones 64 x 64 so
  // that the grid still covers the 256 CUs.
  const int64_t big_tiles = int64_t((a.M + 127) / 128) * ((a.N + 127) / 128);
  if (big_tiles >= 1024) return launch_tile<128, 128, 16, EPI>(a, s);
  return launch_tile<64, 64, 16, EPI>(a, s);
}

}  // namespace

hipError_t launch_gemm(const GemmArgs& a, GemmEpilogue epi, hipStream_t s) {
  if (a.K % 16 != 0 || a.lda % 4 != 0 || a.ldb % 4 != 0) return hipErrorInvalidValue;
  switch (epi) {
    case kEpiStore: return launch_epi<kEpiStore>(a, s);
    case kEpiProbe: return launch_epi<kEpiProbe>(a, s);
    case kEpiArgmin: return launch_epi<kEpiArgmin>(a, s);
    case kEpiPackF32: return launch_epi<kEpiPackF32>(a, s);
    case kEpiPackBF16: return launch_epi<kEpiPackBF16>(a, s);
    case kEpiPackF16: return launch_epi<kEpiPackF16>(a, s);
    case kEpiRotateProbe: return launch_epi<kEpiRotateProbe>(a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace dade

// ------------------------------------------------------------------------------------------------
// The query GEMM on bf16 matrix cores (see kernels.h): six v_mfma_f32_32x32x16_bf16 products per
// 16-deep K step.  split_a_kernel first writes A - shift as three bf16 parts in MFMA fragment order
// (the layout split_b3 gives B).  A workgroup of four waves (2 x 2) then owns a 64 x 64 tile of C,
// each wave one 32 x 32 MFMA block with a leading-product and a correction accumulator.  Each K
// step's twelve fragments (two A blocks, two B blocks, three parts each; one contiguous 1 KB load
// apiece) are staged in LDS, double-buffered with one barrier per step.  Small tiles keep five
// workgroups per CU resident, so one workgroup's MFMAs overlap the others' operand loads; the
// time is still set by the operands' latency (about 1.3 us per step), not by the matrix cores.
// Workgroups are dealt to the XCDs in contiguous ranges of column tiles, so an XCD's L2 holds its
// share of B while A streams.
namespace dade {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// x -> three bf16 parts (bit patterns), round to nearest even at each step.
__host__ __device__ inline void split3(float x, uint16_t& h0, uint16_t& h1, uint16_t& h2) {
  h0 = f32_to_bf16_rne(x);
  const float r1 = x - __builtin_bit_cast(float, uint32_t(h0) << 16);
  h1 = f32_to_bf16_rne(r1);
  const float r2 = r1 - __builtin_bit_cast(float, uint32_t(h1) << 16);
  h2 = f32_to_bf16_rne(r2);
}

// A3[s][mb][ks][lane] (uint4 = 8 bf16): part s of (A - shift) at rows 32 mb + lane % 32 (zero past M)
// and columns 16 ks + 8 (lane / 32) + 0..7.  One thread per (mb, ks, lane).
__global__ __launch_bounds__(256) void split_a_kernel(const float* __restrict__ A, int lda, const float* __restrict__ shift,
                                                      int M, int KS, int MB32, uint4* __restrict__ a3) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= int64_t(MB32) * KS * 64) return;
  const int lane = int(e % 64), ks = int((e / 64) % KS), mb = int(e / (64 * int64_t(KS)));
  const int row = 32 * mb + (lane & 31), c0 = 16 * ks + 8 * (lane >> 5);
  float x[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (row < M) {
    const float4 u = *reinterpret_cast<const float4*>(A + int64_t(row) * lda + c0);
    const float4 v = *reinterpret_cast<const float4*>(A + int64_t(row) * lda + c0 + 4);
    x[0] = u.x; x[1] = u.y; x[2] = u.z; x[3] = u.w; x[4] = v.x; x[5] = v.y; x[6] = v.z; x[7] = v.w;
    if (shift)
      for (int j = 0; j < 8; ++j) x[j] -= shift[c0 + j];
  }
  uint32_t p[3][4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    uint16_t a[3], b[3];
    split3(x[2 * j], a[0], a[1], a[2]);
    split3(x[2 * j + 1], b[0], b[1], b[2]);
#pragma unroll
    for (int s = 0; s < 3; ++s) p[s][j] = uint32_t(a[s]) | (uint32_t(b[s]) << 16);
  }
  const int64_t per_split = int64_t(MB32) * KS * 64;
#pragma unroll
  for (int s = 0; s < 3; ++s) a3[s * per_split + e] = make_uint4(p[s][0], p[s][1], p[s][2], p[s][3]);
}

constexpr int kSplitTile = 64;                 // rows and columns of C per workgroup
constexpr int kSplitFrags = 12;                // fragments per K step: 2 A blocks + 2 B blocks, 3 parts each

__device__ inline floatx16 mfma_bf16(const uint4& a, const uint4& b, const floatx16& c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5)))
void gemm_split3_kernel(GemmArgs g, const uint4* __restrict__ a3, const uint4* __restrict__ b3) {
  __shared__ uint4 fr[2][kSplitFrags * 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tiles_m = (g.M + kSplitTile - 1) / kSplitTile;
  const int npad = (g.N + kSplitNPad - 1) / kSplitNPad * kSplitNPad;
  const int tiles_n = npad / kSplitTile;
  const int nblk = tiles_m * tiles_n;
  int logical = blockIdx.x;
  if (nblk >= 64 && nblk % 8 == 0) logical = (blockIdx.x % 8) * (nblk / 8) + blockIdx.x / 8;
  const int tm = logical % tiles_m, tn = logical / tiles_m;
  const int KS = g.K / 16, MB32 = (g.M + 31) / 32, NB32 = npad / 32;
  // this thread's three fragment entries of every K step: fragment f = e / 64 (A blocks then B
  // blocks, part-major inside each), lane l = e % 64
  const uint4* src[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int e = tid + 256 * i, f = e / 64, l = e % 64;
    if (f < 6) {
      const int mb = 2 * tm + f / 3, sp = f % 3;
      src[i] = (mb < MB32) ? a3 + ((int64_t(sp) * MB32 + mb) * KS) * 64 + l : nullptr;
    } else {
      const int nb = 2 * tn + (f - 6) / 3, sp = (f - 6) % 3;
      src[i] = b3 + ((int64_t(sp) * NB32 + nb) * KS) * 64 + l;
    }
  }
  uint4 nx[3];
  auto fetch = [&](int ks) {
#pragma unroll
    for (int i = 0; i < 3; ++i) nx[i] = src[i] ? src[i][int64_t(ks) * 64] : make_uint4(0u, 0u, 0u, 0u);
  };
  fetch(0);
#pragma unroll
  for (int i = 0; i < 3; ++i) fr[0][tid + 256 * i] = nx[i];
  __syncthreads();
  const int wm = wave >> 1, wn = wave & 1;
  floatx16 acc = {}, cor = {};
  for (int ks = 0; ks < KS; ++ks) {
    const int buf = ks & 1;
    if (ks + 1 < KS) fetch(ks + 1);
    const uint4* fa = fr[buf] + (3 * wm) * 64 + lane;
    const uint4* fb = fr[buf] + (6 + 3 * wn) * 64 + lane;
    const uint4 a0 = fa[0], a1 = fa[64], a2 = fa[128];
    const uint4 b0 = fb[0], b1 = fb[64], b2 = fb[128];
    // the leading product, then the corrections smallest first
    acc = mfma_bf16(a0, b0, acc);
    cor = mfma_bf16(a2, b0, cor);
    cor = mfma_bf16(a1, b1, cor);
    cor = mfma_bf16(a0, b2, cor);
    cor = mfma_bf16(a1, b0, cor);
    cor = mfma_bf16(a0, b1, cor);
    if (ks + 1 < KS) {
#pragma unroll
      for (int i = 0; i < 3; ++i) fr[buf ^ 1][tid + 256 * i] = nx[i];
    }
    __syncthreads();
  }
  // epilogue (kEpiRotateProbe): accumulator v of a lane holds C[row][col], col = lane % 32 of its
  // block, row = 8 (v / 4) + 4 (lane / 32) + v % 4
  const int col = tn * kSplitTile + 32 * wn + (lane & 31);
  if (col >= g.N) return;
  const bool rot = col < g.split_col;
  const float cn = rot ? 0.f : g.col_norm[col - g.split_col];
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int r = tm * kSplitTile + 32 * wm + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    if (r >= g.M) continue;
    const float x = acc[v] + cor[v];
    if (rot) static_cast<float*>(g.C)[int64_t(r) * g.ldc + col] = x;
    else g.C2[int64_t(r) * g.ldc2 + (col - g.split_col)] = cn - 2.f * x;
  }
}

}  // namespace

void split_b3(const float* B, int ldb, int K, int N, uint16_t* out) {
  const int npad = (N + kSplitNPad - 1) / kSplitNPad * kSplitNPad;
  const int KS = K / 16, NB32 = npad / 32;
  const size_t per_split = size_t(NB32) * KS * 512;
  for (int n = 0; n < npad; ++n)
    for (int k = 0; k < K; ++k) {
      const float x = n < N ? B[size_t(k) * ldb + n] : 0.f;
      uint16_t h[3];
      split3(x, h[0], h[1], h[2]);
      const int lane = 32 * ((k % 16) / 8) + n % 32;
      const size_t off = (size_t(n / 32) * KS + k / 16) * 512 + size_t(lane) * 8 + k % 8;
      for (int s = 0; s < 3; ++s) out[s * per_split + off] = h[s];
    }
}

size_t split_a_bytes(int M, int K) { return size_t(3) * ((M + 31) / 32) * 32 * size_t(K) * 2; }

hipError_t launch_gemm_split3(const GemmArgs& a, const uint16_t* b3, void* a3, hipStream_t s) {
  if (a.M == 0) return hipSuccess;
  if (a.K % 32 != 0 || a.lda % 4 != 0 || !b3 || !a3) return hipErrorInvalidValue;
  const int KS = a.K / 16, MB32 = (a.M + 31) / 32;
  const int64_t n_a = int64_t(MB32) * KS * 64;
  hipLaunchKernelGGL(split_a_kernel, dim3(unsigned((n_a + 255) / 256)), dim3(256), 0, s, a.A, a.lda, a.a_shift, a.M,
                     KS, MB32, static_cast<uint4*>(a3));
  const int tiles_m = (a.M + kSplitTile - 1) / kSplitTile;
  const int npad = (a.N + kSplitNPad - 1) / kSplitNPad * kSplitNPad;
  hipLaunchKernelGGL(gemm_split3_kernel, dim3(tiles_m * (npad / kSplitTile)), dim3(256), 0, s, a,
                     static_cast<const uint4*>(a3), reinterpret_cast<const uint4*>(b3));
  return hipGetLastError();
}

}  // namespace dade
