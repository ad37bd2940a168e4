// Probe selection through bf16 matrix-core products refined exactly (end of the Methodology
// section: IVF scans the nprobe lists whose centroids are nearest to the query).
//
// The lists are ordered by t(c) = ||c - mu||^2 - 2 (q - mu).(c - mu), the squared distance minus
// ||q - mu||^2 (a constant of the query), ties by list id.  Computing t for every centroid in
// FP32 is most of the query-side work (nlist columns against dp for the rotation).  Here:
//
//  1. probe_prep_kernel: q - mu (FP32, as the exact path forms it) rounded to bf16 in MFMA
//     fragment order;
//  2. cgemm_kernel: t~(c) = ||c - mu||^2 - 2 bf16(q - mu).bf16(c - mu) for every centroid, one
//     v_mfma_f32_32x32x16_bf16 product per 16-deep step, FP32 accumulation, and a bound
//     E(c) >= |t~(c) - t*(c)| + |t(c) - t*(c)|, where t* is the real-number value of the FP32
//     inputs and t the FP32 value of the exact path.  E follows from the bf16 rounding (relative
//     2^-8 per factor), FP32 accumulation over dp terms (relative 2^-23 per addition, which also
//     covers a truncating adder) and Cauchy-Schwarz (sum |q_i c_i| <= ||q - mu|| ||c - mu||).
//     The kernel writes the bits of floats just above t~ + E and just below t~ - E;
//  3. refine_kernel, one workgroup per query: with U such that at least nprobe upper bounds are at or
//     below it, every list whose lower bound exceeds U has t above the t of nprobe other lists,
//     so it cannot be a probe.  The remaining lists (typically a few more than nprobe) get t in
//     FP32 from the FP32 vectors, and the nprobe smallest by (t, list id) are the probes,
//     ascending.
//
// The probes equal those of a plain FP32 evaluation of every t (up to the FP32 summation order
// of the exact dot products, which only matters at ties within rounding).
#include "kernels.h"

namespace dade {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kPT = 128;   // rows (queries) and columns (centroids) of a cgemm tile

__device__ inline uint32_t pack_bf16(float lo, float hi) {
  return uint32_t(f32_to_bf16_rne(lo)) | (uint32_t(f32_to_bf16_rne(hi)) << 16);
}

// a1[mb][ks][lane] (uint4 = 8 bf16): bf16(q - mu) at query 32 mb + lane % 32 and coordinates
// 16 ks + 8 (lane / 32) + 0..7, zero past M rows and past dp coordinates, for mb < MBp and
// ks < KSp (dp / 16 rounded up to the prefetch depth).  One thread per entry.
__global__ __launch_bounds__(256) void probe_prep_kernel(const float* __restrict__ q, int ldq,
                                                         const float* __restrict__ mu, int M, int dp, int KSp,
                                                         int MBp, uint4* __restrict__ a1) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= int64_t(MBp) * KSp * 64) return;
  const int lane = int(e % 64), ks = int((e / 64) % KSp), mb = int(e / (64 * int64_t(KSp)));
  const int row = 32 * mb + (lane & 31), c0 = 16 * ks + 8 * (lane >> 5);
  float x[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (row < M && c0 < dp) {   // dp % 16 == 0: the 8 coordinates are all inside or all outside
    const float4 u = *reinterpret_cast<const float4*>(q + int64_t(row) * ldq + c0);
    const float4 v = *reinterpret_cast<const float4*>(q + int64_t(row) * ldq + c0 + 4);
    const float4 m0 = *reinterpret_cast<const float4*>(mu + c0);
    const float4 m1 = *reinterpret_cast<const float4*>(mu + c0 + 4);
    x[0] = u.x - m0.x; x[1] = u.y - m0.y; x[2] = u.z - m0.z; x[3] = u.w - m0.w;
    x[4] = v.x - m1.x; x[5] = v.y - m1.y; x[6] = v.z - m1.z; x[7] = v.w - m1.w;
  }
  a1[e] = make_uint4(pack_bf16(x[0], x[1]), pack_bf16(x[2], x[3]), pack_bf16(x[4], x[5]), pack_bf16(x[6], x[7]));
}

__device__ inline floatx16 mfma_bf16(const uint4& a, const uint4& b, const floatx16& c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

constexpr int kPrefetch = 4;   // K steps of operands in flight per thread (KSp is a multiple)

// Bounds of t(row, col) for row < M, col < N: t~ = cn[col] - 2 a1(row) . cb(col) on the matrix
// cores, E = cqc ||q - mu|| cnorm[col] + ccn cn[col] (+ a denormal slack), and the
// order-preserving bits of the next floats above t~ + E and below t~ - E, cut to their top 16
// bits (the upper rounded up, the lower down) and packed as (upper << 16 | lower) into
// bnd[row][col].  ||q - mu|| <= ||bf16(q - mu)|| / (1 - u)
// is taken from the A fragments as they pass (FP32 sums of squares, bounded through qn_scale).
// A workgroup of four waves (2 x 2) owns a 128 x 128 tile, each wave 64 x 64 as 2 x 2 MFMA
// blocks.  Per 16-deep step the tile's four A and four B fragments (1 KB each, one 16-byte load
// per thread apiece) pass through LDS, double-buffered with one barrier per step; each thread
// keeps kPrefetch steps of its two entries in flight in registers.  The loop has no branches
// (the operands' K steps are zero-padded to a multiple of kPrefetch and loads past the end
// re-read the last step), so the compiler's waits count only the oldest loads.  Tiles are dealt
// to the XCDs in contiguous runs of the column-major tile order, so an XCD's L2 holds its share
// of the centroid fragments.
struct CgemmArgs {
  const uint4* a1;
  const uint4* cb;
  const float* cn;
  const float* cnorm;
  int M, N, KSp;
  float cqc, ccn, qn_scale;
  uint32_t* bnd;
};

__device__ inline float sumsq_bf16x8(const uint4& v, float s) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float lo = __uint_as_float(w[i] << 16), hi = __uint_as_float(w[i] & 0xFFFF0000u);
    s = fmaf(lo, lo, s);
    s = fmaf(hi, hi, s);
  }
  return s;
}

__global__ __launch_bounds__(256) void cgemm_kernel(CgemmArgs g) {
  __shared__ uint4 fa[2][4 * 64];
  __shared__ uint4 fb[2][4 * 64];
  const int M = g.M, N = g.N, KSp = g.KSp;
  const uint4* __restrict__ a1 = g.a1;
  const uint4* __restrict__ cb = g.cb;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tiles_m = (M + kPT - 1) / kPT, tiles_n = (N + kPT - 1) / kPT;
  const int nblk = tiles_m * tiles_n;
  int logical = blockIdx.x;
  if (nblk >= 64 && nblk % 8 == 0) logical = (blockIdx.x % 8) * (nblk / 8) + blockIdx.x / 8;
  const int tm = logical % tiles_m, tn = logical / tiles_m;
  // this thread's entry of every step: fragment tid / 64 of the tile's A blocks and of its B
  // blocks, lane tid % 64
  const uint4* pa = a1 + (int64_t(4 * tm + (tid >> 6)) * KSp) * 64 + (tid & 63);
  const uint4* pb = cb + (int64_t(4 * tn + (tid >> 6)) * KSp) * 64 + (tid & 63);
  auto at = [&](int t) { return int64_t(t < KSp ? t : KSp - 1) * 64; };
  // four register pairs: step t's entries live in pair t % 4 until they are written to LDS
  uint4 ra0 = pa[0], rb0 = pb[0];
  uint4 ra1 = pa[at(1)], rb1 = pb[at(1)];
  uint4 ra2 = pa[at(2)], rb2 = pb[at(2)];
  uint4 ra3 = pa[at(3)], rb3 = pb[at(3)];
  fa[0][tid] = ra0;
  fb[0][tid] = rb0;
  ra0 = pa[at(kPrefetch)];
  rb0 = pb[at(kPrefetch)];
  __syncthreads();
  const int wm = wave >> 1, wn = wave & 1;
  floatx16 acc00 = {}, acc01 = {}, acc10 = {}, acc11 = {};
  float sq0 = 0.f, sq1 = 0.f;   // this lane's share of its rows' sums of squares (blocks 2 wm, 2 wm + 1)
  // step ks from LDS buffer ks % 2; step ks + 1 (held in pair rA, rB) into the other buffer, and
  // that pair refilled with step ks + 1 + kPrefetch
  auto step = [&](int ks, int buf, uint4& rA, uint4& rB) {
    const uint4 a0 = fa[buf][(2 * wm) * 64 + lane], a1v = fa[buf][(2 * wm + 1) * 64 + lane];
    const uint4 b0 = fb[buf][(2 * wn) * 64 + lane], b1v = fb[buf][(2 * wn + 1) * 64 + lane];
    sq0 = sumsq_bf16x8(a0, sq0);
    sq1 = sumsq_bf16x8(a1v, sq1);
    acc00 = mfma_bf16(a0, b0, acc00);
    acc01 = mfma_bf16(a0, b1v, acc01);
    acc10 = mfma_bf16(a1v, b0, acc10);
    acc11 = mfma_bf16(a1v, b1v, acc11);
    fa[buf ^ 1][tid] = rA;
    fb[buf ^ 1][tid] = rB;
    rA = pa[at(ks + 1 + kPrefetch)];
    rB = pb[at(ks + 1 + kPrefetch)];
    __syncthreads();
  };
  for (int k0 = 0; k0 < KSp; k0 += kPrefetch) {
    step(k0, 0, ra1, rb1);
    step(k0 + 1, 1, ra2, rb2);
    step(k0 + 2, 0, ra3, rb3);
    step(k0 + 3, 1, ra0, rb0);
  }
  const floatx16 acc[2][2] = {{acc00, acc01}, {acc10, acc11}};
  // a row's sum of squares: lanes r and r + 32 hold the two halves of every step of row r
  const float qn0 = sqrtf(sq0 + __shfl_xor(sq0, 32, 64)) * g.qn_scale;
  const float qn1 = sqrtf(sq1 + __shfl_xor(sq1, 32, 64)) * g.qn_scale;
  // epilogue: accumulator v of a lane holds block element row 8 (v / 4) + 4 (lane / 32) + v % 4,
  // column lane % 32
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int col = tn * kPT + 32 * (2 * wn + j) + (lane & 31);
    const bool cok = col < N;
    const float c2 = cok ? g.cn[col] : 0.f, cnrm = cok ? g.cnorm[col] : 0.f;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int rl = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const float qn = __shfl(i == 0 ? qn0 : qn1, rl, 64);
        const int row = tm * kPT + 32 * (2 * wm + i) + rl;
        if (cok && row < M) {
          const float t = c2 - 2.f * acc[i][j][v];
          const float qc = qn * cnrm;
          const float e = g.cqc * qc + g.ccn * c2 + 0x1p-100f * (1.f + c2 + qc);
          const uint32_t ub = ordered_bits(t + e) + 1u, lb = ordered_bits(t - e) - 1u;
          const uint32_t ub16 = (ub >> 16) + ((ub & 0xFFFFu) != 0u ? 1u : 0u);   // rounded up
          g.bnd[int64_t(row) * N + col] = ((ub16 < 0xFFFFu ? ub16 : 0xFFFFu) << 16) | (lb >> 16);
        }
      }
    }
  }
}

struct RefineArgs {
  const uint32_t* bnd;  // [M x nl] packed bounds of every t (cgemm_kernel)
  int nl, npm, dp;
  const float* q;       // [M x ldq] queries (FP32)
  int ldq;
  const float* mu;      // [dp]
  const float* cx;      // [nl x dp] c - mu (FP32)
  const float* cn;      // [nl] ||c - mu||^2 (FP32)
  int32_t* probes;      // [M x npm]
};

constexpr int kRefineMaxChunks = 16;   // dp <= 16 x 64
constexpr int kRefineThreads = 256;    // one workgroup (four waves) per query
constexpr int kBatch = 16;             // columns a thread loads per batch

// One workgroup per query; the row of packed bounds is streamed in batches of kBatch columns per
// thread (loads clamped in range, so none waits on a branch).
__global__ __launch_bounds__(kRefineThreads) void refine_kernel(RefineArgs a) {
  extern __shared__ unsigned long long sel[];   // P entries: candidate columns, then their keys
  __shared__ uint32_t hist[256];
  __shared__ uint32_t s_cnt[kRefineThreads / 64];
  __shared__ int s_total;
  const int q = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = tid >> 4, gl = tid & 15;
  const float* qrow = a.q + int64_t(q) * a.ldq;
  const uint32_t* brow = a.bnd + int64_t(q) * a.nl;
  constexpr int kStride = kRefineThreads * kBatch;
  const int nbatch = (a.nl + kStride - 1) / kStride;
  auto col = [&](int b, int j) { return kStride * b + kRefineThreads * j + tid; };
  // upper bound of column c (16 bits), above every present one for absent columns
  auto upper = [&](uint32_t v, int c) { return c < a.nl ? v >> 16 : 0x10000u; };
  // workgroup-wide count of a predicate
  auto count = [&](bool pred) -> uint32_t {
    const unsigned long long m = __ballot(pred);
    if (lane == 0) s_cnt[wave] = uint32_t(__popcll(m));
    __syncthreads();
    uint32_t t = 0;
#pragma unroll
    for (int w = 0; w < kRefineThreads / 64; ++w) t += s_cnt[w];
    __syncthreads();
    return t;
  };
  // U: a value with at least npm upper bounds at or below it.  Any such U is sound: those npm
  // lists have t <= U, and a list whose lower bound exceeds U has t > U.
  uint32_t U;
  if (a.npm <= kRefineThreads) {
    // the npm-th smallest thread minimum (the npm smallest minima come from distinct threads;
    // at least min(nl, 256) >= npm threads hold a column)
    uint32_t mn = 0x10000u;
    for (int b = 0; b < nbatch; ++b) {
      uint32_t v[kBatch];
#pragma unroll
      for (int j = 0; j < kBatch; ++j) {
        const int c = col(b, j);
        v[j] = brow[c < a.nl ? c : a.nl - 1];
      }
#pragma unroll
      for (int j = 0; j < kBatch; ++j) {
        const uint32_t ub = upper(v[j], col(b, j));
        mn = ub < mn ? ub : mn;
      }
    }
    uint32_t x = 0u, y = 0x10000u;
    while (x < y) {
      const uint32_t mid = x + (y - x) / 2;
      if (count(mn <= mid) >= uint32_t(a.npm)) y = mid;
      else x = mid + 1;
    }
    U = x;
  } else {
    // the npm-th smallest upper bound: radix selection on its two bytes, LDS histograms
    uint32_t prefix = 0, need = uint32_t(a.npm);
    for (int digit = 1; digit >= 0; --digit) {
      for (int i = tid; i < 256; i += kRefineThreads) hist[i] = 0;
      __syncthreads();
      for (int b = 0; b < nbatch; ++b) {
        uint32_t v[kBatch];
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
          const int c = col(b, j);
          v[j] = brow[c < a.nl ? c : a.nl - 1];
        }
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
          const int c = col(b, j);
          const uint32_t ub = upper(v[j], c);
          if (c < a.nl && (digit == 1 || (ub >> 8) == prefix)) atomicAdd(&hist[(ub >> (8 * digit)) & 0xFFu], 1u);
        }
      }
      __syncthreads();
      // the first bin whose inclusive prefix count reaches `need`, found by wave 0 (lane l holds
      // bins 4 l .. 4 l + 3); every thread reads the result from LDS
      if (wave == 0) {
        uint32_t h[4], sum = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          h[k] = hist[4 * lane + k];
          sum += h[k];
        }
        uint32_t incl = sum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const uint32_t y = __shfl_up(incl, o, 64);
          if (lane >= o) incl += y;
        }
        uint32_t before = incl - sum;
        int bin = -1;
        uint32_t below = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if (bin < 0 && before + h[k] >= need) {
            bin = 4 * lane + k;
            below = before;
          }
          before += h[k];
        }
        const unsigned long long m = __ballot(bin >= 0);
        const int src = __builtin_ctzll(m);
        if (lane == src) {
          s_cnt[0] = uint32_t(bin);
          s_cnt[1] = below;
        }
      }
      __syncthreads();
      prefix = (prefix << 8) | s_cnt[0];
      need -= s_cnt[1];
      __syncthreads();
    }
    U = prefix;
  }
  // candidates, the lists whose lower bound is at most U (their order in sel does not matter:
  // they are sorted by key below)
  if (tid == 0) s_total = 0;
  __syncthreads();
  for (int b = 0; b < nbatch; ++b) {
    uint32_t v[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int c = col(b, j);
      v[j] = brow[c < a.nl ? c : a.nl - 1];
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int c = col(b, j);
      const bool take = c < a.nl && (v[j] & 0xFFFFu) <= U;
      const unsigned long long m = __ballot(take);
      int base = 0;
      if (lane == 0 && m) base = atomicAdd(&s_total, __popcll(m));
      base = __shfl(base, 0, 64);
      if (take) {
        const int below = int(__builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u)));
        sel[base + below] = uint64_t(uint32_t(c));
      }
    }
  }
  __syncthreads();
  const int total = s_total;
  const int nch = a.dp / 4;   // float4 chunks of a row
  // t in FP32 for the candidates, sixteen at a time: group g (16 threads) takes candidate i0 + g,
  // its threads the float4 chunks 16 ch + tid % 16 (chunks past the row are loaded clamped and
  // weighted zero, so no load sits behind a branch)
  constexpr int kGroups = kRefineThreads / 16;
  for (int i0 = 0; i0 < total; i0 += kGroups) {
    const int i = i0 + g;
    const int c = i < total ? int(uint32_t(sel[i])) : 0;
    const float* crow = a.cx + int64_t(c) * a.dp;
    float s = 0.f;
#pragma unroll 4
    for (int ch = 0; ch < kRefineMaxChunks; ++ch) {
      const int k = 16 * ch + gl, kc = k < nch ? k : nch - 1;
      const float w = k < nch ? 1.f : 0.f;
      const float4 qv = *reinterpret_cast<const float4*>(qrow + 4 * kc);
      const float4 mv = *reinterpret_cast<const float4*>(a.mu + 4 * kc);
      const float4 cv = *reinterpret_cast<const float4*>(crow + 4 * kc);
      s = fmaf((qv.x - mv.x) * w, cv.x, s);
      s = fmaf((qv.y - mv.y) * w, cv.y, s);
      s = fmaf((qv.z - mv.z) * w, cv.z, s);
      s = fmaf((qv.w - mv.w) * w, cv.w, s);
    }
#pragma unroll
    for (int o = 8; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
    const float t = a.cn[c] - 2.f * s;
    __syncthreads();   // every group has read its sel entry
    if (gl == 0 && i < total) sel[i] = (static_cast<unsigned long long>(ordered_bits(t)) << 32) | uint32_t(c);
    __syncthreads();
  }
  int P2 = 1;
  while (P2 < total) P2 <<= 1;
  for (int i = total + tid; i < P2; i += kRefineThreads) sel[i] = ~0ull;
  __syncthreads();
  for (int k = 2; k <= P2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = tid; i < P2; i += kRefineThreads) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const unsigned long long x = sel[i], y = sel[ixj];
          if ((x > y) == ((i & k) == 0)) {
            sel[i] = y;
            sel[ixj] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < a.npm; i += kRefineThreads) a.probes[int64_t(q) * a.npm + i] = int32_t(key_id(sel[i]));
}

int ks_padded(int dp) { return (dp / 16 + kPrefetch - 1) / kPrefetch * kPrefetch; }

}  // namespace

size_t probe_a_bytes(int M, int dp) {
  return size_t((M + kPT - 1) / kPT) * kPT * size_t(ks_padded(dp)) * 16 * 2;
}

size_t probe_centroid_frag_count(int nl, int dp) {
  return size_t((nl + kPT - 1) / kPT) * kPT * size_t(ks_padded(dp)) * 16;
}

void probe_centroid_frags(const float* cx, int nl, int dp, uint16_t* out) {
  const int KSp = ks_padded(dp), NB = (nl + kPT - 1) / kPT * (kPT / 32);
  for (int nb = 0; nb < NB; ++nb)
    for (int ks = 0; ks < KSp; ++ks)
      for (int lane = 0; lane < 64; ++lane) {
        const int col = 32 * nb + (lane & 31), k0 = 16 * ks + 8 * (lane >> 5);
        uint16_t* o = out + ((size_t(nb) * KSp + ks) * 64 + lane) * 8;
        for (int j = 0; j < 8; ++j)
          o[j] = col < nl && k0 < dp ? f32_to_bf16_rne(cx[size_t(col) * dp + k0 + j]) : uint16_t(0);
      }
}

hipError_t launch_probe_select(const ProbeArgs& p, hipStream_t s) {
  if (p.M == 0) return hipSuccess;
  if (p.npm < 1 || p.npm > p.nl || p.nl > kMaxNlist || p.dp % 16 != 0 || p.dp > 64 * kRefineMaxChunks ||
      p.ldq % 4 != 0 || !p.a1 || !p.cb || !p.bnd)
    return hipErrorInvalidValue;
  const int KSp = ks_padded(p.dp);
  const int tiles_m = (p.M + kPT - 1) / kPT, tiles_n = (p.nl + kPT - 1) / kPT;
  const int MBp = tiles_m * (kPT / 32);
  const int64_t n_a = int64_t(MBp) * KSp * 64;
  hipLaunchKernelGGL(probe_prep_kernel, dim3(unsigned((n_a + 255) / 256)), dim3(256), 0, s, p.q, p.ldq, p.mu, p.M,
                     p.dp, KSp, MBp, static_cast<uint4*>(p.a1));
  // The bound (see the file comment): bf16 rounding u per factor, FP32 sums of dp terms with
  // relative error 2^-23 per addition, the final t = cn - 2 x of both paths; then inflated by
  // 2^-16 for E's own FP32 evaluation (three roundings of 2^-24 at most).
  const double u = 0x1p-8;
  const double gm = double(16 * KSp) * 0x1p-23 / (1.0 - double(16 * KSp) * 0x1p-23);
  const double ax = (1.0 + u) * (1.0 + u) * (1.0 + gm);   // |x~| <= ax sum |q_i c_i|
  const double cqc =
      2.0 * (2.0 * u + u * u) + 2.0 * gm * (1.0 + u) * (1.0 + u) + 2.0 * gm + 0x1p-23 * (ax + 1.0 + gm);
  CgemmArgs cg;
  cg.a1 = static_cast<const uint4*>(p.a1);
  cg.cb = static_cast<const uint4*>(p.cb);
  cg.cn = p.cn;
  cg.cnorm = p.cnorm;
  cg.M = p.M; cg.N = p.nl; cg.KSp = KSp;
  cg.cqc = float(cqc * (1.0 + 0x1p-16));
  cg.ccn = float(0x1p-23 * (1.0 + 0x1p-16));
  // ||q - mu|| <= ||b|| / (1 - u) for b = bf16(q - mu); the FP32 sum of squares is within a factor
  // (1 - gm) of the exact one, its square root and the product add a few roundings
  cg.qn_scale = float((1.0 + gm) / (1.0 - u) * (1.0 + 0x1p-20));
  cg.bnd = p.bnd;
  hipLaunchKernelGGL(cgemm_kernel, dim3(tiles_m * tiles_n), dim3(256), 0, s, cg);
  RefineArgs r;
  r.bnd = p.bnd;
  r.nl = p.nl; r.npm = p.npm; r.dp = p.dp;
  r.q = p.q; r.ldq = p.ldq; r.mu = p.mu;
  r.cx = p.cx; r.cn = p.cn;
  r.probes = p.probes;
  int P = 1;
  while (P < p.nl) P <<= 1;
  hipLaunchKernelGGL(refine_kernel, dim3(p.M), dim3(kRefineThreads), size_t(P) * sizeof(unsigned long long), s, r);
  return hipGetLastError();
}

}  // namespace dade
