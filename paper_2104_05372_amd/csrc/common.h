// Device-side helpers shared by the libdexmi kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define DEX_DEV __device__ __forceinline__

namespace dexk {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef __attribute__((__vector_size__(8 * sizeof(float)))) float f32x8;

constexpr int kWave = 64;

// ---- wave-level exchange -------------------------------------------------
// Value of `v` held by lane (lane ^ 32) / (lane ^ 16), through the gfx950 lane
// swaps (VALU, no LDS traffic, no lgkm wait). The swap leaves the lane's own
// value in one of the two results and its partner's in the other; the own
// value is recognised by its bits, so the choice does not depend on which
// half the instruction moves.
DEX_DEV uint32_t swap_partner32(uint32_t v) {
  const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  return r[0] == v ? r[1] : r[0];
}
DEX_DEV uint32_t swap_partner16(uint32_t v) {
  const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  return r[0] == v ? r[1] : r[0];
}

// Value of `v` held by lane (lane ^ mask).
template <typename T>
DEX_DEV T xor_lane(T v, int mask) {
  if constexpr (sizeof(T) == 4) {
    if (mask == 32) return __builtin_bit_cast(T, swap_partner32(__builtin_bit_cast(uint32_t, v)));
    if (mask == 16) return __builtin_bit_cast(T, swap_partner16(__builtin_bit_cast(uint32_t, v)));
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
