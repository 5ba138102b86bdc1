// Device helpers shared by the solver's kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rqp {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------------------------
// Flag-in-data exchange words. A producer publishes a value together with a 32-bit tag in one
// 8-byte store; a consumer polls the 8-byte word until the tag matches. An aligned 8-byte
// access is single-copy atomic, so a matching tag guarantees a matching value without any
// fence. Agent-scope (device-wide) relaxed atomics make the stores and loads coherent across
// the XCDs' separate L2 caches. FP64 values take two words (low and high halves, same tag).

__device__ __forceinline__ void ll_store_word(uint64_t* p, uint32_t bits, uint32_t tag) {
  __hip_atomic_store(p, ((uint64_t)tag << 32) | (uint64_t)bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ll_load_word(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ll_tag(uint64_t w) { return (uint32_t)(w >> 32); }

template <typename T>
struct LLWords;
template <>
struct LLWords<float> {
  static constexpr int kWords = 1;
};
template <>
struct LLWords<double> {
  static constexpr int kWords = 2;
};

__device__ __forceinline__ void ll_store(uint64_t* p, float v, uint32_t tag) { ll_store_word(p, __float_as_uint(v), tag); }
__device__ __forceinline__ void ll_store(uint64_t* p, double v, uint32_t tag) {
  uint64_t b = (uint64_t)__double_as_longlong(v);
  ll_store_word(p, (uint32_t)b, tag);
  ll_store_word(p + 1, (uint32_t)(b >> 32), tag);
}
__device__ __forceinline__ void ll_store_bits64(uint64_t* p, uint64_t b, uint32_t tag) {
  ll_store_word(p, (uint32_t)b, tag);
  ll_store_word(p + 1, (uint32_t)(b >> 32), tag);
}
__device__ __forceinline__ float ll_value_f(uint64_t w) { return __uint_as_float((uint32_t)w); }
__device__ __forceinline__ uint64_t ll_bits64(uint64_t lo, uint64_t hi) {
  return (uint64_t)(uint32_t)lo | ((uint64_t)(uint32_t)hi << 32);
}

// ---------------------------------------------------------------------------------------------
// Infinity norms as ordered bit patterns: for x >= 0 (sign cleared) the IEEE bit pattern is
// monotone in the value, and NaN patterns order above +inf, so an integer max over
// (bits & ~sign) is an exact, order-independent inf-norm that also flags NaN.

__device__ __forceinline__ uint64_t abs_bits(double v) {
  return (uint64_t)__double_as_longlong(v) & 0x7fffffffffffffffull;
}
__device__ __forceinline__ double bits_to_double(uint64_t b) { return __longlong_as_double((long long)b); }
constexpr uint64_t kInfBits = 0x7ff0000000000000ull;

// Wave-wide sum with DPP lane permutations (VALU, no LDS round trip): quad swaps, half-row
// and row mirrors give 16-lane sums in every lane, then the two row broadcasts fold the four
// rows so that lane 63 holds the total. Only lane 63's result is meaningful.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float v) {
  const int t = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xf, false);
  return v + __builtin_bit_cast(float, t);
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, ROW_MASK, 0xf, false);
  const uint64_t r = (uint64_t)(uint32_t)lo | ((uint64_t)(uint32_t)hi << 32);
  return v + __builtin_bit_cast(double, r);
}
template <typename T>
__device__ __forceinline__ T wave_sum_to_last(T v) {
  v = dpp_add<0xb1, 0xf>(v);   // quad_perm [1,0,3,2]
  v = dpp_add<0x4e, 0xf>(v);   // quad_perm [2,3,0,1]
  v = dpp_add<0x141, 0xf>(v);  // row_half_mirror
  v = dpp_add<0x140, 0xf>(v);  // row_mirror
  v = dpp_add<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_add<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}
constexpr int kLastLane = kWave - 1;

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    uint64_t o = __shfl_xor(v, off, kWave);
    v = o > v ? o : v;
  }
  return v;
}

// Projection onto [l, u] (eq. clamp). Equal to t - ReLU(t - u) + ReLU(l - t) for l <= u, but
// evaluated by selection so the bound is hit exactly (no cancellation of t - (t - u)) and NaN
// propagates (both comparisons are false for NaN).
template <typename T>
__device__ __forceinline__ T box_clamp(T t, T l, T u) {
  return t < l ? l : (t > u ? u : t);
}

}  // namespace rqp
