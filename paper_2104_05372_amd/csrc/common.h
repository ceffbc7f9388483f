// Device-side helpers shared by the libdexmi kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>
#include <utility>

#define DEX_DEV __device__ __forceinline__

namespace dexk {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef __attribute__((__vector_size__(8 * sizeof(float)))) float f32x8;

constexpr int kWave = 64;

// f(integral_constant<int, 0>), ..., f(integral_constant<int, N - 1>), in order:
// a loop whose index is a compile-time constant in the body.
template <typename F, int... I>
DEX_DEV void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
DEX_DEV void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// ---- wave-level exchange -------------------------------------------------
// gfx950 lane swaps (VALU, no LDS traffic, no lgkm wait). As measured on the
// hardware, swap32(a, b) returns {[a_lo, b_lo], [a_hi, b_hi]} where lo / hi
// are lanes 0-31 / 32-63, and swap16(a, b) returns
// {[a_r0, b_r0, a_r2, b_r2], [a_r1, b_r1, a_r3, b_r3]} where r is a row of 16
// lanes. So, per lane, the two results of swap32(a, b) are a's (or b's, in the
// upper half) values at lanes l and l ^ 32 in lane order, and likewise for
// swap16 with rows.
struct LanePair {
  float first, second;  // value at the lower / upper lane of the pair
};
DEX_DEV LanePair swap32(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  return {__uint_as_float(r[0]), __uint_as_float(r[1])};
}
DEX_DEV LanePair swap16(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  return {__uint_as_float(r[0]), __uint_as_float(r[1])};
}
// Sum / max over the lane pair (l, l ^ 32) or (l, l ^ 16); both lanes get the
// same bits (the lower lane's value is always the first operand).
DEX_DEV float pair_sum32(float v) {
  const LanePair p = swap32(v, v);
  return p.first + p.second;
}
DEX_DEV float pair_sum16(float v) {
  const LanePair p = swap16(v, v);
  return p.first + p.second;
}
DEX_DEV float pair_max32(float v) {
  const LanePair p = swap32(v, v);
  return fmaxf(p.first, p.second);
}
DEX_DEV float pair_max16(float v) {
  const LanePair p = swap16(v, v);
  return fmaxf(p.first, p.second);
}

// Value of `v` held by lane (lane ^ mask).
template <typename T>
DEX_DEV T xor_lane(T v, int mask) {
  if constexpr (sizeof(T) == 4) {
    const bool upper = (threadIdx.x & mask) != 0;
    if (mask == 32) {
      const LanePair p = swap32(__builtin_bit_cast(float, v), __builtin_bit_cast(float, v));
      return __builtin_bit_cast(T, upper ? p.first : p.second);
    }
    if (mask == 16) {
      const LanePair p = swap16(__builtin_bit_cast(float, v), __builtin_bit_cast(float, v));
      return __builtin_bit_cast(T, upper ? p.first : p.second);
    }
  }
  return __shfl_xor(v, mask, kWave);
}

template <typename T>
DEX_DEV T wave_sum(T v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += xor_lane(v, m);
  return v;
}

DEX_DEV float wave_max(float v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = fmaxf(v, xor_lane(v, m));
  return v;
}

// ---- compensated (Neumaier) accumulation ------------------------------------
// A running sum s with a correction term c; the represented value is s + c.
template <typename T>
struct Comp {
  T s, c;
  DEX_DEV Comp() : s(0), c(0) {}
  DEX_DEV void add(T x) {
    T t = s + x;
    if (fabs(s) >= fabs(x))
      c += (s - t) + x;
    else
      c += (x - t) + s;
    s = t;
  }
  DEX_DEV T value() const { return s + c; }
};

// ---- block reduction (fixed order, deterministic) --------------------------
// Sums `v` over the block; every thread gets the result. `sh` holds >= 32 T.
template <typename T>
DEX_DEV T block_sum(T v, T* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  T r = 0;
  for (int i = 0; i < nw; ++i) r += sh[i];
  return r;
}

}  // namespace dexk
