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
  // A and its shift are kept apart until stage(): nothing in fetch() uses a loaded value, so all
  // of a slice's loads are issued before any of them is waited for.  (x - +0 is x, so rows with
  // no shift, and rows past M, which load nothing, stage the same values.)
  float4 ra[LA], rs[LA], rb[LB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int l = 0; l < LA; ++l) {
      const int q = (tid + l * kThreads) % (BK / 4);
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f), sh = make_float4(0.f, 0.f, 0.f, 0.f);
      if (arow[l]) {
        v = *reinterpret_cast<const float4*>(arow[l] + k0 + 4 * q);
        if (g.a_shift) sh = *reinterpret_cast<const float4*>(g.a_shift + k0 + 4 * q);
      }
      ra[l] = v;
      rs[l] = sh;
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
      As[(4 * q + 0) * PA + r] = ra[l].x - rs[l].x;
      As[(4 * q + 1) * PA + r] = ra[l].y - rs[l].y;
      As[(4 * q + 2) * PA + r] = ra[l].z - rs[l].z;
      As[(4 * q + 3) * PA + r] = ra[l].w - rs[l].w;
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

// The query rotation (kEpiRotateProbe with N = split_col): 64 x 64 tiles with 16-deep K slices
// (at 1000 x 960 x 960, 45 us against 51 us with 64-deep slices).
hipError_t launch_gemm_rotate(const GemmArgs& a, hipStream_t s) {
  if (a.K % 16 != 0 || a.lda % 4 != 0 || a.ldb % 4 != 0 || a.N > a.split_col) return hipErrorInvalidValue;
  return launch_tile<64, 64, 16, kEpiRotateProbe>(a, s);
}

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
