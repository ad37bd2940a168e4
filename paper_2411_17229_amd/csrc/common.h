// Shared definitions of the DADE-IVF HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace dade {

constexpr int kWave = 64;
constexpr int kMaxK = 128;          // largest K a search supports
constexpr int kDimAlign = 32;       // stored rows are padded to a multiple of 32 coordinates
constexpr int kMaxNlist = 8192;     // probe selection sorts nlist keys in LDS (64 KB)

inline int pad_dim(int dim) { return (dim + kDimAlign - 1) / kDimAlign * kDimAlign; }

// Packed store of the rotated coordinates: a head block holding coordinates [0, kHead) of every
// row ([n x kHead]), then a tail block holding the rest ([n x (dp - kHead)]).  The first
// hypothesis test of a scan reads only the head, so a list's first-test reads are contiguous.
constexpr int kHead = 32;
__host__ __device__ inline int64_t stored_index(int64_t p, int c, int64_t n, int dp) {
  return c < kHead ? p * kHead + c : n * kHead + p * (dp - kHead) + (c - kHead);
}

// Error state for the C ABI (thread-local message).
void set_error(const std::string& msg);
std::string hip_msg(hipError_t e, const char* what);

// Storage types of the rotated coordinates.
using bf16_raw = uint16_t;
using f16_raw = uint16_t;

// float -> bfloat16, round to nearest even (inputs are finite).
__host__ __device__ inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}

// A float that orders like an unsigned integer (negative values below positive ones).
__host__ __device__ inline uint32_t ordered_bits(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Heap key: non-negative squared distance bits in the high word, id in the low word, so
// that comparing keys as integers is the total order on (dist2, id).
__host__ __device__ inline uint64_t make_key(float d2, uint32_t id) {
  return (static_cast<uint64_t>(__builtin_bit_cast(uint32_t, d2)) << 32) | id;
}
__host__ __device__ inline float key_dist(uint64_t k) {
  return __builtin_bit_cast(float, static_cast<uint32_t>(k >> 32));
}
__host__ __device__ inline uint32_t key_id(uint64_t k) { return static_cast<uint32_t>(k); }

}  // namespace dade
