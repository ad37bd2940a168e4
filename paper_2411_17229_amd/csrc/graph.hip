// Graph search with DADE distance comparisons: the paper's graph setting (HNSW with DADE DCOs,
// Experiments) on a one-layer kNN graph.  One wavefront runs one query's beam: the pool of ef
// (dist^2, id) keys lives one per lane, the visited set in an LDS hash table, and every expansion
// gives each unvisited neighbour one DCO (Algorithm 1 with the reduced test S_d > T_d r^2, or
// FDScanning) against the pool's snapshot at the expansion's start.
#include "kernels.h"

namespace dade {
namespace {

constexpr unsigned long long kEmpty = ~0ull;

__device__ inline float bf16_to_f(uint32_t h) { return __uint_as_float(h << 16); }
__device__ inline float f16_to_f(uint32_t h) {
  return __half2float(__ushort_as_half(static_cast<unsigned short>(h)));
}

// Address of coordinates [c, c + 8) of stored row p (c a multiple of 8; the head block holds
// [0, 32)): 16 bytes for a 16-bit store, 32 for FP32.
template <int DT>
__device__ inline const uint4* chunk_ptr(const GraphArgs& a, int64_t p, int c) {
  const int64_t off = c < kHead ? p * kHead + c : p * (a.dp - kHead) + (c - kHead);
  return reinterpret_cast<const uint4*>(static_cast<const char*>(c < kHead ? a.head : a.tail) +
                                        off * (DT == 0 ? 4 : 2));
}

// The 8 coordinates of a chunk loaded as raw words (lo; hi holds coordinates 4..7 for FP32).
template <int DT>
__device__ inline void unpack8(const uint4& lo, const uint4& hi, float v[8]) {
  if (DT == 0) {
    v[0] = __uint_as_float(lo.x); v[1] = __uint_as_float(lo.y); v[2] = __uint_as_float(lo.z);
    v[3] = __uint_as_float(lo.w); v[4] = __uint_as_float(hi.x); v[5] = __uint_as_float(hi.y);
    v[6] = __uint_as_float(hi.z); v[7] = __uint_as_float(hi.w);
  } else {
    const uint32_t w[4] = {lo.x, lo.y, lo.z, lo.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      v[2 * i] = DT == 1 ? bf16_to_f(w[i] & 0xffffu) : f16_to_f(w[i] & 0xffffu);
      v[2 * i + 1] = DT == 1 ? bf16_to_f(w[i] >> 16) : f16_to_f(w[i] >> 16);
    }
  }
}

// One DCO of stored row p against r2: S over growing prefixes, rejected at the first tested d
// (a multiple of delta_d below dim) where S_d > T_d r2.  TEST false: FDScanning.  The row is
// read kBatch chunks of 8 coordinates at a time, all row loads of a batch issued before the
// first chunk is used (a chunk past dim loads the last chunk again and is not used), so a batch
// costs one memory trip.  With tests, the chunks are then taken in order, each test as soon as
// its prefix is summed, so a rejected DCO stops reading query chunks and thresholds at its exit.
// Without tests, the batch's query chunks are read and summed with no branch between them.  The
// sum takes the coordinates in order, so S, the exit and the dimensions counted are those of a
// chunk-by-chunk loop.
template <int DT, bool TEST>
__device__ inline void dco(const GraphArgs& a, int64_t p, const float* qr, float r2, float& S, bool& rej,
                           int& dexit) {
  constexpr int kBatch = DT == 0 ? 8 : 16;
  float s = 0.f;
  rej = false;
  dexit = a.dim;
  const int last = (a.dim - 1) / 8 * 8;   // first coordinate of the last chunk
  for (int c0 = 0; c0 < a.dim; c0 += 8 * kBatch) {
    uint4 lo[kBatch], hi[kBatch];
#pragma unroll
    for (int b = 0; b < kBatch; ++b) {
      const uint4* src = chunk_ptr<DT>(a, p, min(c0 + 8 * b, last));
      lo[b] = src[0];
      if (DT == 0) hi[b] = src[1];
    }
    if constexpr (TEST) {
#pragma unroll
      for (int b = 0; b < kBatch; ++b) {
        const int c = c0 + 8 * b;
        if (c >= a.dim) break;
        float v[8];
        unpack8<DT>(lo[b], hi[b], v);
        const float4 q0 = *reinterpret_cast<const float4*>(qr + c), q1 = *reinterpret_cast<const float4*>(qr + c + 4);
        const float qv[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const float t = qv[i] - v[i];
          s = fmaf(t, t, s);
        }
        const int e = c + 8;
        if (e < a.dim && e % a.delta_d == 0 && s > a.T[e - 1] * r2) {
          S = s;
          rej = true;
          dexit = e;
          return;
        }
      }
    } else {
      float pre[kBatch];
#pragma unroll
      for (int b = 0; b < kBatch; ++b) {
        const int c = min(c0 + 8 * b, last);
        float v[8];
        unpack8<DT>(lo[b], hi[b], v);
        const float4 q0 = *reinterpret_cast<const float4*>(qr + c), q1 = *reinterpret_cast<const float4*>(qr + c + 4);
        const float qv[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const float t = qv[i] - v[i];
          s = fmaf(t, t, s);
        }
        pre[b] = s;
      }
      // the sum through the batch's last chunk below dim
      const int n_in = min(kBatch, (a.dim - c0 + 7) / 8);
#pragma unroll
      for (int b = 0; b < kBatch; ++b)
        if (b == n_in - 1) s = pre[b];
    }
  }
  S = s;
}

// Inserts position u into the visited table; true if it was not there.  The table always has a
// free slot (the host sizes it to at least twice the most insertions a search can make), so the
// probe sequence ends.
__device__ inline bool visit(int* tab, uint32_t mask, int u) {
  uint32_t h = (uint32_t(u) * 2654435761u) & mask;
  for (;;) {
    const int old = atomicCAS(&tab[h], -1, u);
    if (old == -1) return true;
    if (old == u) return false;
    h = (h + 1) & mask;
  }
}

__device__ inline unsigned long long make_key(float d2, uint32_t id) {
  return (static_cast<unsigned long long>(__float_as_uint(d2)) << 32) | id;
}

// The pool (lane i: key, position, expanded flag; sorted ascending in lanes 0..n_pool-1, kEmpty
// beyond) merged with one new key per lane (kEmpty: none): the ef smallest, in order, in lanes
// 0..ef-1 (kEmpty beyond).  Keys are unique (distinct row ids: a new key's row was unvisited), so
// a pool entry's rank is its lane plus the new keys below it, and a new key's rank counts the
// pool entries and new keys below it; every slot below min(ef, total) is written exactly once
// and the slots from there to ef are cleared.
__device__ inline void merge_pool(unsigned long long& pk, int& pp, int& pe, unsigned long long nk, int np, int ef,
                                  unsigned long long* mk, int* mp, int* me, int lane) {
  const unsigned long long mnew = __ballot(nk != kEmpty);
  const int n_new = __popcll(mnew);
  const int n_pool = __popcll(__ballot(pk != kEmpty));
  const int slot = int(__builtin_amdgcn_mbcnt_hi(uint32_t(mnew >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(mnew), 0u)));
  mk[lane] = pk; mp[lane] = pp; me[lane] = pe;
  if (nk != kEmpty) { mk[64 + slot] = nk; mp[64 + slot] = np; }
  __syncthreads();
  int r0 = lane, r1 = 0;
  for (int j = 0; j < n_new; ++j) {
    const unsigned long long kj = mk[64 + j];
    r0 += kj < pk ? 1 : 0;
    r1 += kj < nk ? 1 : 0;
  }
  for (int f = 0; f < n_pool; ++f) r1 += mk[f] < nk ? 1 : 0;
  __syncthreads();
  const int total = n_pool + n_new;
  if (pk != kEmpty && r0 < ef) { mk[r0] = pk; mp[r0] = pp; me[r0] = pe; }
  if (nk != kEmpty && r1 < ef) { mk[r1] = nk; mp[r1] = np; me[r1] = 0; }
  if (lane >= total && lane < ef) { mk[lane] = kEmpty; mp[lane] = -1; me[lane] = 1; }
  __syncthreads();
  pk = lane < ef ? mk[lane] : kEmpty;
  pp = lane < ef ? mp[lane] : -1;
  pe = lane < ef ? me[lane] : 1;
  __syncthreads();
}

template <int DT, bool DADE>
__global__ __launch_bounds__(64) void graph_search_kernel(GraphArgs a) {
  extern __shared__ int smem[];
  const int lane = threadIdx.x;
  const int q = blockIdx.x;
  const uint32_t slots = 1u << a.slots_log2, mask = slots - 1;
  int* tab = smem;
  unsigned long long* mk = reinterpret_cast<unsigned long long*>(smem + slots);
  int* mp = reinterpret_cast<int*>(mk + 128);
  int* me = mp + 128;
  for (uint32_t i = lane; i < slots; i += 64) tab[i] = -1;
  __syncthreads();
  const float* qr = a.qrot + int64_t(q) * a.dp;
  const int ef = a.ef, deg = a.degree;
  long long n_dco = 0, n_dims = 0, n_vis = 0;

  // seeds: the entry points of the query's n_entry nearest lists, full-D distances
  unsigned long long pk = kEmpty;
  int pp = -1, pe = 1;
  unsigned long long nk = kEmpty;
  int np = -1;
  if (lane < 2 * a.n_entry) {   // two entry points per list: lanes 2j and 2j + 1 take list j's
    const int l = a.probes[int64_t(q) * a.npm + (lane >> 1)];
    const int p = a.entry[2 * l + (lane & 1)];
    if (p >= 0 && visit(tab, mask, p)) {
      ++n_vis;
      float S;
      bool rej;
      int dx;
      dco<DT, false>(a, p, qr, 0.f, S, rej, dx);
      nk = make_key(S, uint32_t(a.ids[p]));
      np = p;
    }
  }
  merge_pool(pk, pp, pe, nk, np, ef, mk, mp, me, lane);

  int it = 0;
  for (; it < a.max_iters; ++it) {
    const unsigned long long open = __ballot(lane < ef && pk != kEmpty && !pe);
    if (open == 0) break;
    const int c = __builtin_ctzll(open);
    const int cp = __shfl(pp, c);
    if (lane == c) pe = 1;
    const unsigned long long worst = __shfl(pk, ef - 1);   // the snapshot of this expansion
    const bool full = worst != kEmpty;
    const float r2 = full ? __uint_as_float(uint32_t(worst >> 32)) : __builtin_inff();
    nk = kEmpty;
    np = -1;
    if (lane < deg) {
      const int u = a.nbr[int64_t(cp) * deg + lane];
      if (u >= 0 && visit(tab, mask, u)) {
        ++n_vis;
        const uint32_t rid = uint32_t(a.ids[u]);   // read beside the DCO's loads, not after them
        float S;
        bool rej;
        int dx;
        if (DADE && full)
          dco<DT, true>(a, u, qr, r2, S, rej, dx);
        else
          dco<DT, false>(a, u, qr, r2, S, rej, dx);
        ++n_dco;
        n_dims += dx;
        if (!rej) {
          const unsigned long long k = make_key(S, rid);
          if (!full || k < worst) {
            nk = k;
            np = u;
          }
        }
      }
    }
    // nothing kept: the pool stays as it is (the expanded flag is already in its lane)
    if (__ballot(nk != kEmpty) != 0) merge_pool(pk, pp, pe, nk, np, ef, mk, mp, me, lane);
  }

  // the final pool, reranked with the exact vectors; the K smallest by (exact dist^2, id)
  unsigned long long ek = kEmpty;
  if (pk != kEmpty) {
    const uint32_t rid = uint32_t(pk);
    const float* x = a.X + int64_t(rid) * a.dp;
    const float* qo = a.qorig + int64_t(q) * a.dp;
    float s = 0.f;
    for (int c = 0; c < a.dp; c += 4) {
      const float4 xv = *reinterpret_cast<const float4*>(x + c), qv = *reinterpret_cast<const float4*>(qo + c);
      float t = qv.x - xv.x; s = fmaf(t, t, s);
      t = qv.y - xv.y; s = fmaf(t, t, s);
      t = qv.z - xv.z; s = fmaf(t, t, s);
      t = qv.w - xv.w; s = fmaf(t, t, s);
    }
    ek = make_key(s, rid);
  }
  mk[lane] = ek;
  __syncthreads();
  int rank = 0;
  for (int f = 0; f < 64; ++f) {
    const unsigned long long kf = mk[f];
    rank += (kf < ek || (kf == ek && f < lane)) ? 1 : 0;
  }
  const int n_valid = __popcll(__ballot(ek != kEmpty));
  int64_t* oi = a.out_ids + int64_t(q) * a.K;
  float* od = a.out_d2 + int64_t(q) * a.K;
  if (ek != kEmpty && rank < a.K) {
    oi[rank] = int64_t(uint32_t(ek));
    od[rank] = __uint_as_float(uint32_t(ek >> 32));
  }
  if (lane >= n_valid && lane < a.K) {
    oi[lane] = -1;
    od[lane] = __builtin_inff();
  }
  if (a.stats) {
    for (int o = 32; o > 0; o >>= 1) {
      n_dco += __shfl_down(n_dco, o);
      n_dims += __shfl_down(n_dims, o);
      n_vis += __shfl_down(n_vis, o);
    }
    if (lane == 0) {
      int64_t* st = a.stats + int64_t(q) * 4;
      st[0] = n_dco;
      st[1] = n_dims;
      st[2] = it;
      st[3] = n_vis;
    }
  }
}

// Out-neighbours of query rows [c0, c0 + cn) from their FDScanning results (K = degree + 1):
// the row itself dropped, positions written at the row's own position (rows of `width`),
// -1 padded up to degree.
__global__ void graph_collect_kernel(const int64_t* res, int cn, int64_t c0, int degree, int width,
                                     const int64_t* pos, int32_t* nbr) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cn) return;
  const int64_t i = c0 + t;
  int32_t* out = nbr + pos[i] * width;
  int w = 0;
  for (int j = 0; j <= degree; ++j) {
    const int64_t id = res[int64_t(t) * (degree + 1) + j];
    if (id < 0 || id == i || w == degree) continue;
    out[w++] = int32_t(pos[id]);
  }
  for (; w < degree; ++w) out[w] = -1;
}

// Squared FP32 distance between two padded rows.
__device__ inline float row_d2(const float* x, const float* y, int dp) {
  float s = 0.f;
  for (int k = 0; k < dp; k += 4) {
    const float4 xv = *reinterpret_cast<const float4*>(x + k), yv = *reinterpret_cast<const float4*>(y + k);
    float t = xv.x - yv.x; s = fmaf(t, t, s);
    t = xv.y - yv.y; s = fmaf(t, t, s);
    t = xv.z - yv.z; s = fmaf(t, t, s);
    t = xv.w - yv.w; s = fmaf(t, t, s);
  }
  return s;
}

// The smallest key of the workgroup (256 threads), to every thread.
__device__ inline unsigned long long block_min(unsigned long long v, unsigned long long* red) {
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long u = __shfl_down(v, o);
    v = u < v ? u : v;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  v = red[0];
  for (int w = 1; w < 4; ++w) v = red[w] < v ? red[w] : v;
  __syncthreads();
  return v;
}

// Each list's two entry points, as positions: its medoid (the member with the smallest (FP32
// squared distance to the centroid, row id)), then the member farthest from the medoid (largest
// distance, then smallest row id); -1 where the list has no such member.  One workgroup per list.
__global__ __launch_bounds__(256) void graph_entry_kernel(const float* X, const float* cent, const int64_t* off,
                                                          const int32_t* ids, const int64_t* pos, int dp,
                                                          int32_t* entry) {
  __shared__ unsigned long long red[4];
  const int l = blockIdx.x;
  unsigned long long best = kEmpty;
  for (int64_t p = off[l] + threadIdx.x; p < off[l + 1]; p += blockDim.x) {
    const uint32_t rid = uint32_t(ids[p]);
    const unsigned long long k = make_key(row_d2(X + int64_t(rid) * dp, cent + int64_t(l) * dp, dp), rid);
    best = k < best ? k : best;
  }
  best = block_min(best, red);
  unsigned long long far = kEmpty;
  if (best != kEmpty) {
    const uint32_t mid = uint32_t(best);
    const float* xm = X + int64_t(mid) * dp;
    for (int64_t p = off[l] + threadIdx.x; p < off[l + 1]; p += blockDim.x) {
      const uint32_t rid = uint32_t(ids[p]);
      if (rid == mid) continue;
      // largest distance first: the complement of the distance bits orders descending
      const unsigned long long k =
          (static_cast<unsigned long long>(~__float_as_uint(row_d2(X + int64_t(rid) * dp, xm, dp))) << 32) | rid;
      far = k < far ? k : far;
    }
  }
  far = block_min(far, red);
  if (threadIdx.x == 0) {
    entry[2 * l] = best == kEmpty ? -1 : int32_t(pos[uint32_t(best)]);
    entry[2 * l + 1] = far == kEmpty ? -1 : int32_t(pos[uint32_t(far)]);
  }
}

}  // namespace

size_t graph_lds_bytes(int slots_log2) { return (size_t(1) << slots_log2) * 4 + 128 * 8 + 128 * 4 * 2; }

hipError_t launch_graph_search(const GraphArgs& a, hipStream_t s) {
  if (a.nq == 0) return hipSuccess;
  const size_t lds = graph_lds_bytes(a.slots_log2);
#define DADE_GRAPH(DT, M) hipLaunchKernelGGL((graph_search_kernel<DT, M>), dim3(a.nq), dim3(64), lds, s, a)
  if (a.dtype == 0) {
    if (a.mode == 0) DADE_GRAPH(0, true); else DADE_GRAPH(0, false);
  } else if (a.dtype == 1) {
    if (a.mode == 0) DADE_GRAPH(1, true); else DADE_GRAPH(1, false);
  } else {
    if (a.mode == 0) DADE_GRAPH(2, true); else DADE_GRAPH(2, false);
  }
#undef DADE_GRAPH
  return hipGetLastError();
}

hipError_t launch_graph_collect(const int64_t* res, int cn, int64_t c0, int degree, int width, const int64_t* pos,
                                int32_t* nbr, hipStream_t s) {
  if (cn == 0) return hipSuccess;
  hipLaunchKernelGGL(graph_collect_kernel, dim3((cn + 255) / 256), dim3(256), 0, s, res, cn, c0, degree, width,
                     pos, nbr);
  return hipGetLastError();
}

hipError_t launch_graph_entry(const float* X, const float* cent, const int64_t* off, const int32_t* ids,
                              const int64_t* pos, int dp, int nlist, int32_t* entry, hipStream_t s) {
  hipLaunchKernelGGL(graph_entry_kernel, dim3(nlist), dim3(256), 0, s, X, cent, off, ids, pos, dp, entry);
  return hipGetLastError();
}

}  // namespace dade
