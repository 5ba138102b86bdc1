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

// Lower bound of a norm term from its computed value v >= 0 and rounding bound d (NaN stays).
__device__ __forceinline__ double lower_bound(double v, double d) {
  const double w = v - d;
  return w > 0.0 ? w : (w != w ? w : 0.0);
}
// the host's abort flag is polled at every kAbortEvery-th check of a launch
constexpr int kAbortEvery = 16;

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

// ---------------------------------------------------------------------------------------------
// Sum of R values per lane over the wave, R a power of two <= 64, in ~R + log2(64/R) steps
// instead of 6 R: at each of the first log2(R) pair steps a lane keeps half of its rows and adds
// its partner's copy of them (cross-half swaps v_permlane32/16_swap for distances 32 and 16,
// DPP for 8 and 4 (and 2, 1)); the remaining steps are plain pairwise sums. Every lane ends with
// the complete sum of one row; which row is fixed by the network and found once with
// rows_held() below. Lanes whose low log2(64/R) bits are zero hold distinct rows.

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xf, 0xf, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, (uint64_t)lo | ((uint64_t)hi << 32));
}
// x' + y' after swapping the upper half-group of x with the lower half-group of y
template <int D>
__device__ __forceinline__ float swap_add(float x, float y) {
  const uint32_t a = __builtin_bit_cast(uint32_t, x), b = __builtin_bit_cast(uint32_t, y);
  if constexpr (D == 32) {
    auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    return __builtin_bit_cast(float, (uint32_t)r[0]) + __builtin_bit_cast(float, (uint32_t)r[1]);
  } else {
    auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
    return __builtin_bit_cast(float, (uint32_t)r[0]) + __builtin_bit_cast(float, (uint32_t)r[1]);
  }
}
template <int D>
__device__ __forceinline__ double swap_add(double x, double y) {
  const uint64_t a = __builtin_bit_cast(uint64_t, x), b = __builtin_bit_cast(uint64_t, y);
  uint32_t xl, xh, yl, yh;
  if constexpr (D == 32) {
    auto rl = __builtin_amdgcn_permlane32_swap((uint32_t)a, (uint32_t)b, false, false);
    auto rh = __builtin_amdgcn_permlane32_swap((uint32_t)(a >> 32), (uint32_t)(b >> 32), false, false);
    xl = rl[0]; yl = rl[1]; xh = rh[0]; yh = rh[1];
  } else {
    auto rl = __builtin_amdgcn_permlane16_swap((uint32_t)a, (uint32_t)b, false, false);
    auto rh = __builtin_amdgcn_permlane16_swap((uint32_t)(a >> 32), (uint32_t)(b >> 32), false, false);
    xl = rl[0]; yl = rl[1]; xh = rh[0]; yh = rh[1];
  }
  return __builtin_bit_cast(double, (uint64_t)xl | ((uint64_t)xh << 32)) +
         __builtin_bit_cast(double, (uint64_t)yl | ((uint64_t)yh << 32));
}

// one step at distance D on C values (C even: pair step; C == 1: plain step)
template <int D, int C, typename T, int N>
__device__ __forceinline__ void rr_step(T (&v)[N], int lane) {
  if constexpr (C >= 2) {
    constexpr int H = C / 2;
    if constexpr (D >= 16) {
#pragma unroll
      for (int i = 0; i < H; ++i) v[i] = swap_add<D>(v[i], v[i + H]);
    } else {
      const bool hi = (lane & D) != 0;
#pragma unroll
      for (int i = 0; i < H; ++i) {
        const T send = hi ? v[i] : v[i + H];
        const T keep = hi ? v[i + H] : v[i];
        T recv;
        if constexpr (D == 8) recv = dpp_mov<0x128>(send);       // row_ror:8 = lane ^ 8 in a row
        else if constexpr (D == 4) recv = dpp_mov<0x141>(send);  // row_half_mirror: i <-> 7 - i
        else if constexpr (D == 2) recv = dpp_mov<0x4e>(send);   // quad_perm [2,3,0,1]
        else recv = dpp_mov<0xb1>(send);                         // quad_perm [1,0,3,2]
        v[i] = keep + recv;
      }
    }
  } else {
    if constexpr (D >= 16) v[0] = swap_add<D>(v[0], v[0]);
    else if constexpr (D == 8) v[0] += dpp_mov<0x128>(v[0]);
    else if constexpr (D == 4) v[0] += dpp_mov<0x141>(v[0]);
    else if constexpr (D == 2) v[0] += dpp_mov<0x4e>(v[0]);
    else v[0] += dpp_mov<0xb1>(v[0]);
  }
}

template <int R, typename T, int N>
__device__ __forceinline__ T reduce_rows(T (&v)[N]) {
  static_assert(N >= R, "need R values");
  static_assert(R == 1 || R == 2 || R == 4 || R == 8 || R == 16 || R == 32 || R == 64, "R must be a power of two");
  const int lane = threadIdx.x % kWave;
  constexpr int C1 = R, C2 = R > 1 ? R / 2 : 1, C3 = R > 2 ? R / 4 : 1, C4 = R > 4 ? R / 8 : 1,
                C5 = R > 8 ? R / 16 : 1, C6 = R > 16 ? R / 32 : 1;
  rr_step<32, C1>(v, lane);
  rr_step<16, C2>(v, lane);
  rr_step<8, C3>(v, lane);
  rr_step<4, C4>(v, lane);
  rr_step<2, C5>(v, lane);
  rr_step<1, C6>(v, lane);
  return v[0];
}

// Row whose total this lane holds after reduce_rows<R> (found by reducing row numbers).
template <int R>
__device__ __forceinline__ int rows_held() {
  float v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = (float)(r + 1);
  const float s = reduce_rows<R>(v);
  return (int)(s / (float)kWave + 0.5f) - 1;
}
template <int R>
__device__ __forceinline__ bool row_writer() {
  return ((threadIdx.x % kWave) & (kWave / R - 1)) == 0;
}

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
