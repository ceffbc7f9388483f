// Indexed read (gather) and its transpose, the scatter-accumulate
// `runAccum \acc. for j. acc!(idx.j) += scale.j * vals.j` (Sec. 2.3.2-2.3.3,
// Sec. 5.3.3), and the integer histogram `for i. hist!(keys.i) += 1`
// (Sec. 6.1.2), for gfx950.
//
// Float rows: each block sorts a chunk of (index, position) pairs in LDS, so
// that equal indices become runs; each wave walks a slice of the sorted chunk,
// summing the rows of a run in registers, and adds a run's sum to the table
// with one atomic per column (the segmented reduction before global atomics).
// Work stays O(n * row_len) and every update is applied once; rows that never
// appear are not touched.
//
// Histogram: one block per compute unit keeps a private histogram of 16-bit
// counters packed two per LDS word. A counter that reaches 2^14 is drained by
// the thread that saw it reach that value (one global atomic of 2^14 and an LDS
// subtraction), so a counter never overflows however skewed the keys are. At
// the end each block writes its counters to the workspace and a second kernel
// adds them per bin. Integer addition is exact, so the result is identical
// under any schedule.
#include <algorithm>
#include <type_traits>
#include <utility>

#include "common.h"
#include "internal.h"

namespace dexk {

constexpr int kChunk = 2048;          // indices per block for the row scatter
constexpr uint32_t kDrain = 1u << 14;  // histogram drain threshold

__global__ void fill_zero_kernel(uint32_t* p, size_t nwords) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < nwords; i += stride) p[i] = 0u;
}

__global__ void fill_zero_bytes(uint8_t* p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

DEX_DEV void count_oob(int bad, int64_t* oob) {
  // block-level sum of per-thread counts, one atomic per block
  __shared__ int sh[16];
  int v = wave_sum(bad);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long t = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
    if (t) atomicAdd((unsigned long long*)oob, (unsigned long long)t);
  }
}

template <typename IdxT>
DEX_DEV int64_t load_index(const IdxT* idx, int64_t j) {
  return (int64_t)idx[j];
}

// Bitonic sort of kChunk 64-bit keys in LDS (ascending).
DEX_DEV void lds_bitonic_sort(uint64_t* key) {
  for (int size = 2; size <= kChunk; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (int t = threadIdx.x; t < kChunk / 2; t += blockDim.x) {
        const int i = 2 * t - (t & (stride - 1));
        const int j = i + stride;
        const bool up = (i & size) == 0;
        uint64_t a = key[i], b = key[j];
        if ((a > b) == up) {
          key[i] = b;
          key[j] = a;
        }
      }
    }
  }
  __syncthreads();
}

// acc[idx[j], :] += scale[j] * vals[j, :] for float or int rows.
// Sorted keys hold (row << 12) | local position; invalid rows sort last.
// HV: vals given (else ones); HS: scale given. Both are template parameters so
// the hot loop has no branches between its loads and their use.
template <typename T, typename IdxT, int U, bool HV, bool HS>
__global__ void __launch_bounds__(256) scatter_rows_kernel(T* __restrict__ acc, int64_t n_rows,
                                                           int R, const IdxT* __restrict__ idx,
                                                           const T* __restrict__ vals,
                                                           const float* __restrict__ scale,
                                                           int64_t n, int64_t* oob) {
  __shared__ uint64_t key[kChunk];
  const int64_t j0 = (int64_t)blockIdx.x * kChunk;
  const int cnt = (int)min<int64_t>(kChunk, n - j0);
  int bad = 0;
  for (int t = threadIdx.x; t < kChunk; t += blockDim.x) {
    uint64_t kv = ~uint64_t(0);
    if (t < cnt) {
      const int64_t v = load_index(idx, j0 + t);
      if (v >= 0 && v < n_rows)
        kv = ((uint64_t)v << 12) | (uint64_t)t;
      else
        ++bad;
    }
    key[t] = kv;
  }
  if (oob) count_oob(bad, oob);
  lds_bitonic_sort(key);

  // each wave takes a contiguous slice of the sorted chunk. The values of the
  // next U sorted entries are loaded before the run sums (and atomics) of the
  // current U are issued: vector memory operations retire in issue order, so
  // waiting for a batch of loads never waits for atomics issued after it.
  // Loads are unconditional (clamped to a valid element, then masked), which
  // keeps branches out from between loads and their use.
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int per = (kChunk + nw - 1) / nw;
  const int e0 = wv * per, e1 = min(kChunk, e0 + per);
  constexpr uint64_t kNone = ~uint64_t(0);
  for (int c0 = 0; c0 < R; c0 += 64) {
    const int col = c0 + lane;
    const bool cv = col < R;
    const int colc = cv ? col : R - 1;
    auto fetch = [&](int e, uint64_t(&kk)[U], T(&r)[U]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        kk[u] = (e + u < e1) ? key[e + u] : kNone;
        const bool ok = kk[u] != kNone;
        const int64_t j = j0 + (ok ? (int64_t)(kk[u] & 4095u) : 0);
        T v = T(1);
        if constexpr (HV) v = vals[j * R + colc];
        if constexpr (HS) v = v * scale[j];
        r[u] = ok ? v : T(0);
      }
    };
    uint64_t cur = kNone;
    T sum = 0;
    auto consume = [&](const uint64_t(&kk)[U], const T(&r)[U]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (kk[u] == kNone) continue;
        if ((kk[u] >> 12) != (cur >> 12)) {
          if (cur != kNone && cv) atomicAdd(&acc[(int64_t)(cur >> 12) * R + col], sum);
          cur = kk[u];
          sum = 0;
        }
        sum += r[u];
      }
    };
    uint64_t ka[U], kb[U];
    T ra[U], rb[U];
    fetch(e0, ka, ra);
    for (int e = e0; e < e1; e += 2 * U) {
      fetch(e + U, kb, rb);
      __builtin_amdgcn_sched_barrier(0);
      consume(ka, ra);
      __builtin_amdgcn_sched_barrier(0);
      fetch(e + 2 * U, ka, ra);
      __builtin_amdgcn_sched_barrier(0);
      consume(kb, rb);
      __builtin_amdgcn_sched_barrier(0);
    }
    if (cur != kNone && cv) atomicAdd(&acc[(int64_t)(cur >> 12) * R + col], sum);
  }
}

// Private packed-16-bit histogram per block; see the file comment.
template <typename IdxT>
__global__ void __launch_bounds__(1024) hist_private_kernel(int32_t* __restrict__ acc,
                                                            int n_bins,
                                                            const IdxT* __restrict__ keys,
                                                            int64_t n, int64_t per_block,
                                                            uint32_t* __restrict__ partial,
                                                            int64_t* oob) {
  extern __shared__ uint32_t cnt[];
  const int nwords = (n_bins + 1) >> 1;
  for (int i = threadIdx.x; i < nwords; i += blockDim.x) cnt[i] = 0u;
  __syncthreads();
  const int64_t b0 = (int64_t)blockIdx.x * per_block;
  const int64_t b1 = min<int64_t>(n, b0 + per_block);
  int bad = 0;
  auto bump = [&](int64_t kv) {
    if (kv < 0 || kv >= n_bins) {
      ++bad;
      return;
    }
    const uint32_t k = (uint32_t)kv;
    const uint32_t sh = (k & 1u) << 4;
    const uint32_t old = atomicAdd(&cnt[k >> 1], 1u << sh);
    if (((old >> sh) & 0xFFFFu) == kDrain - 1u) {
      atomicSub(&cnt[k >> 1], kDrain << sh);
      atomicAdd(&acc[k], (int32_t)kDrain);
    }
  };
  // vectorised body (4 keys per thread per step) on the aligned middle part
  if constexpr (sizeof(IdxT) == 4) {
    int64_t a0 = (b0 + 3) & ~int64_t(3);
    int64_t a1 = b1 & ~int64_t(3);
    if (a1 < a0) a1 = a0;
    for (int64_t j = b0 + threadIdx.x; j < min(a0, b1); j += blockDim.x) bump(load_index(keys, j));
    typedef __attribute__((__vector_size__(4 * sizeof(uint32_t)))) uint32_t u32x4;
    const u32x4* k4 = reinterpret_cast<const u32x4*>(keys);
    // four 16-byte loads per thread per round; the next round's loads are
    // issued before this round's LDS updates
    const int64_t q1 = a1 / 4;
    const int64_t step = (int64_t)blockDim.x;
    auto load4 = [&](int64_t q, u32x4(&v)[4]) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
        v[i] = (q + i * step < q1) ? __builtin_nontemporal_load(k4 + q + i * step)
                                   : u32x4{0u, 0u, 0u, 0u};
    };
    u32x4 vn[4];
    load4(a0 / 4 + threadIdx.x, vn);
    for (int64_t q = a0 / 4 + threadIdx.x; q < q1; q += 4 * step) {
      u32x4 v[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] = vn[i];
      load4(q + 4 * step, vn);
      // the 16 LDS additions are issued back to back and their results
      // checked afterwards (a drain then waits at most 16 increments per
      // thread, far inside the 2^16 - 2^14 headroom of a counter)
      uint32_t old[4][4], kk[4][4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const bool live = q + i * step < q1;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          int64_t kv;
          if constexpr (IdxT(-1) < IdxT(0))
            kv = (int64_t)(int32_t)v[i][e];
          else
            kv = (int64_t)v[i][e];
          const bool ok = live && kv >= 0 && kv < n_bins;
          bad += live && !ok;
          kk[i][e] = ok ? (uint32_t)kv : 0xFFFFFFFFu;
          old[i][e] = ok ? atomicAdd(&cnt[(uint32_t)kv >> 1], 1u << (((uint32_t)kv & 1u) << 4)) : 0u;
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const uint32_t k = kk[i][e], sh = (k & 1u) << 4;
          if (k != 0xFFFFFFFFu && ((old[i][e] >> sh) & 0xFFFFu) == kDrain - 1u) {
            atomicSub(&cnt[k >> 1], kDrain << sh);
            atomicAdd(&acc[k], (int32_t)kDrain);
          }
        }
    }
    for (int64_t j = max(a1, a0) + threadIdx.x; j < b1; j += blockDim.x) bump(load_index(keys, j));
  } else {
    for (int64_t j = b0 + threadIdx.x; j < b1; j += blockDim.x) bump(load_index(keys, j));
  }
  if (oob) count_oob(bad, oob);
  __syncthreads();
  uint32_t* mine = partial + (size_t)blockIdx.x * nwords;
  for (int i = threadIdx.x; i < nwords; i += blockDim.x) mine[i] = cnt[i];
}

// acc[b] += sum over blocks of the packed partial counters. Thread (w, y) adds
// the counters of word w over blocks y * kHistGroup .. + kHistGroup - 1 (their
// loads issued together) and adds the two bins' totals with integer atomics:
// integer addition is exact, so the result does not depend on their order.
constexpr int kHistGroup = 16;
__global__ void __launch_bounds__(256) hist_reduce_kernel(int32_t* __restrict__ acc, int n_bins,
                                                          const uint32_t* __restrict__ partial,
                                                          int nblocks) {
  const int w = blockIdx.x * 256 + threadIdx.x;
  const int nwords = (n_bins + 1) >> 1;
  if (w >= nwords) return;
  const int b0 = blockIdx.y * kHistGroup;
  uint32_t v[kHistGroup];
#pragma unroll
  for (int i = 0; i < kHistGroup; ++i)
    v[i] = b0 + i < nblocks ? partial[(size_t)(b0 + i) * nwords + w] : 0u;
  uint32_t lo = 0, hi = 0;
#pragma unroll
  for (int i = 0; i < kHistGroup; ++i) {
    lo += v[i] & 0xFFFFu;
    hi += v[i] >> 16;
  }
  if (lo) atomicAdd(&acc[2 * w], (int32_t)lo);
  if (hi && 2 * w + 1 < n_bins) atomicAdd(&acc[2 * w + 1], (int32_t)hi);
}

// Generic integer accumulation (exact): one thread per (index, column).
template <typename IdxT>
__global__ void __launch_bounds__(256) scatter_int_generic(int32_t* __restrict__ acc,
                                                           int64_t n_rows, int64_t R,
                                                           const IdxT* __restrict__ idx,
                                                           const int32_t* __restrict__ vals,
                                                           int64_t n, int64_t* oob) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int bad = 0;
  if (t < n * R) {
    const int64_t j = t / R, col = t % R;
    const int64_t v = load_index(idx, j);
    if (v >= 0 && v < n_rows)
      atomicAdd(&acc[v * R + col], vals ? vals[t] : 1);
    else if (col == 0)
      bad = 1;
  }
  if (oob) count_oob(bad, oob);
}

// Rows a half-wave has in flight in the gathers: the index and weight loads of
// kGU rows are issued together, then their kGU row loads, so the two dependent
// global reads (index, then row) are paid once per kGU rows.
constexpr int kGU = 4;

// out[j, :] = w[j] * T[idx[j], :]; half a wave per row, 4 floats per lane.
__global__ void __launch_bounds__(256) gather_scale_kernel(const float* __restrict__ T,
                                                           const int32_t* __restrict__ idx,
                                                           const float* __restrict__ w,
                                                           int64_t V, int R, int64_t n,
                                                           float* __restrict__ out,
                                                           int64_t* oob) {
  const int half = threadIdx.x >> 5, hl = threadIdx.x & 31;
  const int64_t stride = (int64_t)gridDim.x * 8;  // rows per round of the grid
  int bad = 0;
  for (int64_t j0 = (int64_t)blockIdx.x * 8 + half; j0 < n; j0 += stride * kGU) {
    int64_t v[kGU];
    float s[kGU];
    bool live[kGU], ok[kGU];
#pragma unroll
    for (int u = 0; u < kGU; ++u) {
      const int64_t j = j0 + u * stride;
      live[u] = j < n;
      v[u] = live[u] ? (int64_t)idx[j] : 0;
      s[u] = live[u] ? w[j] : 0.f;
      ok[u] = live[u] && v[u] >= 0 && v[u] < V;
      if (live[u] && !ok[u] && hl == 0) ++bad;
    }
    for (int c = 4 * hl; c < R; c += 128) {
      f32x4 t[kGU];
#pragma unroll
      for (int u = 0; u < kGU; ++u)
        t[u] = ok[u] ? *reinterpret_cast<const f32x4*>(T + v[u] * R + c) : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int u = 0; u < kGU; ++u)
        if (live[u])
          __builtin_nontemporal_store(t[u] * s[u],
                                      reinterpret_cast<f32x4*>(out + (j0 + u * stride) * R + c));
    }
  }
  if (oob) count_oob(bad, oob);
}

// Forward mode of the gather (the linear map of its linearization, Sec. 5.1;
// idx is an integer, so it carries no tangent):
//   tout[j, :] = tw[j] * T[idx[j], :] + w[j] * tT[idx[j], :]
// Same layout as the gather: half a wave per row, 4 floats per lane, kGU rows
// in flight; rows with an index outside [0, V) give zeros.
__global__ void __launch_bounds__(256) gather_jvp_kernel(const float* __restrict__ T,
                                                         const float* __restrict__ tT,
                                                         const int32_t* __restrict__ idx,
                                                         const float* __restrict__ w,
                                                         const float* __restrict__ tw, int64_t V,
                                                         int R, int64_t n,
                                                         float* __restrict__ tout) {
  const int half = threadIdx.x >> 5, hl = threadIdx.x & 31;
  const int64_t stride = (int64_t)gridDim.x * 8;
  for (int64_t j0 = (int64_t)blockIdx.x * 8 + half; j0 < n; j0 += stride * kGU) {
    int64_t v[kGU];
    float a[kGU], b[kGU];
    bool live[kGU], ok[kGU];
#pragma unroll
    for (int u = 0; u < kGU; ++u) {
      const int64_t j = j0 + u * stride;
      live[u] = j < n;
      v[u] = live[u] ? (int64_t)idx[j] : 0;
      a[u] = live[u] ? tw[j] : 0.f;
      b[u] = live[u] ? w[j] : 0.f;
      ok[u] = live[u] && v[u] >= 0 && v[u] < V;
    }
    for (int c = 4 * hl; c < R; c += 128) {
      f32x4 x[kGU], y[kGU];
#pragma unroll
      for (int u = 0; u < kGU; ++u) {
        x[u] = ok[u] ? *reinterpret_cast<const f32x4*>(T + v[u] * R + c) : f32x4{0.f, 0.f, 0.f, 0.f};
        y[u] = ok[u] ? *reinterpret_cast<const f32x4*>(tT + v[u] * R + c) : f32x4{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int u = 0; u < kGU; ++u) {
        if (!live[u]) continue;
        f32x4 o = f32x4{0.f, 0.f, 0.f, 0.f};
        if (ok[u]) {
#pragma unroll
          for (int e = 0; e < 4; ++e) o[e] = fmaf(b[u], y[u][e], a[u] * x[u][e]);
        }
        __builtin_nontemporal_store(o, reinterpret_cast<f32x4*>(tout + (j0 + u * stride) * R + c));
      }
    }
  }
}

// Scalar form for row lengths that are not a multiple of 4.
__global__ void __launch_bounds__(256) gather_jvp_scalar(const float* __restrict__ T,
                                                         const float* __restrict__ tT,
                                                         const int32_t* __restrict__ idx,
                                                         const float* __restrict__ w,
                                                         const float* __restrict__ tw, int64_t V,
                                                         int R, int64_t n,
                                                         float* __restrict__ tout) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t < n * R) {
    const int64_t j = t / R, c = t % R;
    const int64_t v = idx[j];
    const bool ok = v >= 0 && v < V;
    tout[t] = ok ? fmaf(w[j], tT[v * R + c], tw[j] * T[v * R + c]) : 0.f;
  }
}

// Scalar-path gather for row lengths that are not a multiple of 4.
__global__ void __launch_bounds__(256) gather_scale_scalar(const float* __restrict__ T,
                                                           const int32_t* __restrict__ idx,
                                                           const float* __restrict__ w,
                                                           int64_t V, int R, int64_t n,
                                                           float* __restrict__ out,
                                                           int64_t* oob) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int bad = 0;
  if (t < n * R) {
    const int64_t j = t / R, c = t % R;
    const int64_t v = idx[j];
    const bool ok = v >= 0 && v < V;
    if (!ok && c == 0) bad = 1;
    out[t] = ok ? w[j] * T[v * R + c] : 0.f;
  }
  if (oob) count_oob(bad, oob);
}

// dw[j] (=|+=) <T[idx[j], :], g[j, :]>; half a wave per row.
__global__ void __launch_bounds__(256) gather_dw_kernel(const float* __restrict__ T,
                                                        const int32_t* __restrict__ idx,
                                                        const float* __restrict__ g, int64_t V,
                                                        int R, int64_t n, float* __restrict__ dw,
                                                        int accumulate) {
  const int half = threadIdx.x >> 5, hl = threadIdx.x & 31;
  const int64_t rows_per_iter = (int64_t)gridDim.x * 8;
  for (int64_t j = (int64_t)blockIdx.x * 8 + half; j < n; j += rows_per_iter) {
    const int64_t v = idx[j];
    const bool ok = v >= 0 && v < V;
    float s = 0.f;
    if (ok) {
      if ((R & 3) == 0) {
        for (int c = 4 * hl; c < R; c += 128) {
          const f32x4 t = *reinterpret_cast<const f32x4*>(T + v * R + c);
          const f32x4 q = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(g + j * R + c));
#pragma unroll
          for (int e = 0; e < 4; ++e) s = fmaf(t[e], q[e], s);
        }
      } else {
        for (int c = hl; c < R; c += 32) s = fmaf(T[v * R + c], g[j * R + c], s);
      }
    }
#pragma unroll
    for (int m = 16; m >= 1; m >>= 1) s += xor_lane(s, m);
    if (hl == 0) dw[j] = accumulate ? dw[j] + s : s;
  }
}


// ---------------------------------------------------------------------------
// Deterministic float scatter: a stable LSD radix sort of (row, position) pairs
// followed by run sums with a fixed owner per run, so the rounding order of
// every row's sum is fixed (bit-reproducible), and no atomics are used.
constexpr int kRsTile = 8192;   // keys per sort block (1024 threads x 8 rounds)

// keys[j] = idx[j] if it is inside [0, n_rows), else n_rows (sorts last and is
// skipped); vals[j] = j.
// Radix digits of kRsBits bits (a million rows: 20-bit keys, three passes). With
// 8192-key tiles a digit gets about 32 keys per tile, so the scatter writes runs
// of 128 bytes of keys (wider digits leave runs too short to write efficiently).
constexpr int kRsBits = 8;
constexpr int kRsDigits = 1 << kRsBits;

// Lanes of this wave holding the same kRsBits-bit digit as this lane (among `live`).
DEX_DEV uint64_t digit_peers(uint32_t d, uint64_t live) {
  uint64_t m = live;
#pragma unroll
  for (int b = 0; b < kRsBits; ++b) {
    const uint64_t bal = __ballot((d >> b) & 1u);
    m &= ((d >> b) & 1u) ? bal : ~bal;
  }
  return m;
}

// The sort key of entry j: its row, or n_rows (sorts last, skipped) when the
// index is outside [0, n_rows).
template <typename IdxT>
DEX_DEV uint32_t row_key(const IdxT* __restrict__ idx, int64_t j, int64_t n_rows, int& bad) {
  const int64_t v = load_index(idx, j);
  const bool ok = v >= 0 && v < n_rows;
  bad += !ok;
  return ok ? (uint32_t)v : (uint32_t)n_rows;
}

// Digit counts of one tile: cnt[digit * ntiles + tile]. Exact, order-free. The
// lanes of a wave that share a digit add their count with one LDS atomic (skewed
// keys would otherwise queue on one counter). The first pass reads the indices
// themselves (and counts those outside the table, and clears the combine
// lists' counters); later passes read the keys the previous pass wrote.
template <bool FIRST, typename IdxT>
__global__ void __launch_bounds__(1024) rs_hist(const IdxT* __restrict__ idx,
                                                const uint32_t* __restrict__ keys, int64_t n,
                                                int64_t n_rows, int shift,
                                                uint32_t* __restrict__ cnt, int ntiles,
                                                uint32_t* __restrict__ nlist, int64_t* oob) {
  __shared__ uint32_t h[kRsDigits];
  for (int i = threadIdx.x; i < kRsDigits; i += 1024) h[i] = 0u;
  if (FIRST && blockIdx.x == 0 && threadIdx.x < 2) nlist[threadIdx.x] = 0u;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t t0 = (int64_t)blockIdx.x * kRsTile;
  uint32_t kv[kRsTile / 1024];
  int bad = 0;
#pragma unroll
  for (int r = 0; r < kRsTile / 1024; ++r) {  // all of a thread's loads in flight together
    const int64_t j = t0 + r * 1024 + threadIdx.x;
    if constexpr (FIRST)
      kv[r] = j < n ? row_key(idx, j, n_rows, bad) : 0u;
    else
      kv[r] = j < n ? keys[j] : 0u;
  }
#pragma unroll
  for (int r = 0; r < kRsTile / 1024; ++r) {
    const bool valid = t0 + r * 1024 + threadIdx.x < n;
    const uint32_t d = (kv[r] >> shift) & (kRsDigits - 1);
    const uint64_t peers = digit_peers(d, __ballot(valid));
    if (valid && (peers & lt) == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
  }
  if (FIRST && oob) count_oob(bad, oob);
  __syncthreads();
  for (int i = threadIdx.x; i < kRsDigits; i += 1024) cnt[(size_t)i * ntiles + blockIdx.x] = h[i];
}

// Per digit (one block each): exclusive prefix of the tile counts, and the total.
__global__ void __launch_bounds__(256) rs_digit_scan(uint32_t* __restrict__ cnt, int ntiles,
                                                     uint32_t* __restrict__ tot) {
  __shared__ uint32_t wsh[4];
  uint32_t carry = 0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t* row = cnt + (size_t)blockIdx.x * ntiles;
  for (int b = 0; b < ntiles; b += 256) {
    const int i = b + threadIdx.x;
    const uint32_t v = i < ntiles ? row[i] : 0u;
    uint32_t x = v;  // inclusive scan: within the wave by shuffles, across waves by LDS
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsh[wv] = x;
    __syncthreads();
    uint32_t pre = 0, all = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      pre += w < wv ? wsh[w] : 0u;
      all += wsh[w];
    }
    if (i < ntiles) row[i] = carry + pre + x - v;
    carry += all;
    __syncthreads();
  }
  if (threadIdx.x == 0) tot[blockIdx.x] = carry;
}

// Stable scatter of one tile by digit. Wave w ranks the tile's keys
// [512 w, 512 w + 512) in index order, 64 at a time: ballots rank a key among
// the equal digits of its 64, and a per-wave running count per digit in LDS
// (read, then bumped by the first of the peers) ranks it among the wave's
// earlier keys; no barrier is needed until the wave is done. The per-digit
// counts of the 16 waves then give every key its place in the tile ordered by
// digit (wave order within a digit, so index order is kept); the tile is
// reordered in LDS and written out by consecutive threads, so each digit's keys
// leave as one contiguous run. No atomics: the output order is fixed.
// The first pass reads the indices and scales themselves: an entry's value is
// its position j with its scale's bits above (the run sums then read the scales
// in sorted order, not scattered).
template <bool FIRST, typename IdxT>
__global__ void __launch_bounds__(1024) rs_scatter(const IdxT* __restrict__ idx,
                                                   const float* __restrict__ scale,
                                                   int64_t n_rows,
                                                   const uint32_t* __restrict__ kin,
                                                   const uint64_t* __restrict__ vin,
                                                   uint32_t* __restrict__ kout,
                                                   uint64_t* __restrict__ vout, int64_t n,
                                                   int shift, const uint32_t* __restrict__ cnt,
                                                   const uint32_t* __restrict__ tot, int ntiles) {
  static_assert(kRsDigits <= 256 && kRsTile == 16 * 512, "digits in the first four waves");
  __shared__ uint32_t gbase[kRsDigits];   // where digit d of this tile starts in the output
  __shared__ uint32_t lbase[kRsDigits];   // where digit d starts inside the reordered tile
  __shared__ uint32_t hw[16][kRsDigits];  // per-wave digit counts, then per-wave offsets
  __shared__ uint32_t wsum[2][4];
  __shared__ uint32_t sk[kRsTile];
  __shared__ uint64_t sv[kRsTile];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t tile0 = (int64_t)blockIdx.x * kRsTile;
  const int64_t t0 = tile0 + (int64_t)wv * 512;
  const int tlen = (int)min<int64_t>(kRsTile, n - tile0);
  constexpr int R = 512 / 64;
  uint32_t kk[R], rk[R];
  uint64_t vv[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {  // the wave's loads issued together
    const int64_t j = t0 + r * 64 + lane;
    if constexpr (FIRST) {
      int bad = 0;
      kk[r] = j < n ? row_key(idx, j, n_rows, bad) : 0u;
      const float w = (j < n && scale) ? scale[j] : 1.f;
      vv[r] = ((uint64_t)__float_as_uint(w) << 32) | (uint64_t)(uint32_t)j;
    } else {
      kk[r] = j < n ? kin[j] : 0u;
      vv[r] = j < n ? vin[j] : 0ull;
    }
  }
  const bool dig = tid < kRsDigits;  // thread tid owns digit tid in the prefix steps
  if (dig) {
#pragma unroll
    for (int w = 0; w < 16; ++w) hw[w][tid] = 0u;
  }
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const bool valid = t0 + r * 64 + lane < n;
    const uint32_t d = (kk[r] >> shift) & (kRsDigits - 1);
    const uint64_t peers = digit_peers(d, __ballot(valid));
    const uint32_t before = (uint32_t)__popcll(peers & lt);
    const uint32_t prev = hw[wv][d];
    rk[r] = prev + before;
    if (valid && before == 0) hw[wv][d] = prev + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  // digit threads: this tile's count of digit d, its exclusive scans over the
  // digits (inside the tile) and over the digit totals (the whole array)
  uint32_t c = 0, g = 0;
  if (dig) {
#pragma unroll
    for (int w = 0; w < 16; ++w) c += hw[w][tid];
    g = tot[tid];
  }
  uint32_t xc = c, xg = g;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t yc = __shfl_up(xc, o, 64), yg = __shfl_up(xg, o, 64);
    if (lane >= o) {
      xc += yc;
      xg += yg;
    }
  }
  if (lane == 63 && wv < 4) {
    wsum[0][wv] = xc;
    wsum[1][wv] = xg;
  }
  __syncthreads();
  if (dig) {
    uint32_t pc = 0, pg = 0;
    for (int w = 0; w < wv; ++w) {
      pc += wsum[0][w];
      pg += wsum[1][w];
    }
    const uint32_t lb = pc + xc - c;
    lbase[tid] = lb;
    gbase[tid] = pg + xg - g + cnt[(size_t)tid * ntiles + blockIdx.x];
    uint32_t run = lb;
#pragma unroll
    for (int w = 0; w < 16; ++w) {
      const uint32_t cw = hw[w][tid];
      hw[w][tid] = run;
      run += cw;
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (t0 + r * 64 + lane < n) {
      const uint32_t lp = hw[wv][(kk[r] >> shift) & (kRsDigits - 1)] + rk[r];
      sk[lp] = kk[r];
      sv[lp] = vv[r];
    }
  }
  __syncthreads();
  for (int i = tid; i < tlen; i += 1024) {
    const uint32_t key = sk[i];
    const uint32_t d = (key >> shift) & (kRsDigits - 1);
    const uint32_t pos = gbase[d] + (uint32_t)i - lbase[d];
    kout[pos] = key;
    vout[pos] = sv[i];
  }
}

// ---------------------------------------------------------------------------
// Owner-per-run sum over the sorted (row, position, scale) entries, the default
// form of the transposed gather. Each wave takes kOwnSeg consecutive sorted
// entries; a lane holds VW consecutive columns of a row (a 128-column row is
// one wave load of 512 bytes). A run of equal rows wholly inside the segment
// has exactly one owner, this wave, which writes the row once: a plain store
// (OVR: the table was cleared first) or a read-modify-write of the row (the
// row's value is loaded with the run's first entry) -- no atomics, and the
// rounding order of every row is fixed. The first run of a segment, when it
// began in an earlier segment, leaves its partial in head[seg]; the last run,
// when it began here and continues into the next segment, leaves its partial in
// tail[seg], and the segment is put on the list for own_fix (the list's order
// does not matter: each entry is combined on its own, in a fixed order). The
// values of the next U entries are loaded before the current U are summed.
constexpr int kOwnSeg = 512;

template <int VW, int U, bool HV, bool OVR>
__global__ void __launch_bounds__(256) own_sum(const uint32_t* __restrict__ skey,
                                               const uint64_t* __restrict__ sval, int64_t n,
                                               uint32_t sentinel, const float* __restrict__ vals,
                                               int R, float* __restrict__ acc,
                                               float* __restrict__ head, float* __restrict__ tail,
                                               uint32_t* __restrict__ list,
                                               uint32_t* __restrict__ nlist) {
  typedef float VT __attribute__((ext_vector_type(VW)));
  constexpr int G = kOwnSeg / 64;  // groups of 64 entries
  constexpr int NB = 64 / U;       // batches of U entries per group
  static_assert(64 % U == 0 && NB % 2 == 0, "whole batch pairs per group");
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t seg = (int64_t)blockIdx.x * 4 + wv;
  const int64_t e0 = seg * kOwnSeg;
  if (e0 >= n) return;
  const int len = (int)min<int64_t>(kOwnSeg, n - e0);
  const uint32_t first = __builtin_amdgcn_readfirstlane(skey[e0]);
  const uint32_t lastk = __builtin_amdgcn_readfirstlane(skey[e0 + len - 1]);
  if (first == sentinel) return;
  const bool cont_in = e0 > 0 && skey[e0 - 1] == first;
  const bool cont_out = e0 + len < n && skey[e0 + len] == lastk && lastk != sentinel;
  if (cont_out && !(cont_in && first == lastk) && lane == 0)
    list[atomicAdd(nlist, 1u)] = (uint32_t)seg;  // a run starts here and spans segments
  // lane t holds entry 64 g + t of the current group (key, position, scale);
  // each entry is read back with readlane, so keys, positions and the run logic
  // are wave-uniform (scalar) and a batch's row loads are issued back to back
  struct Ent {
    uint32_t k, j, s;
  };
  auto load_group = [&](int gq) {
    const int e = gq * 64 + lane;
    const bool in = gq < G && e < len;
    const uint64_t pv = in ? sval[e0 + e] : 0ull;
    return Ent{in ? skey[e0 + e] : sentinel, (uint32_t)pv, (uint32_t)(pv >> 32)};
  };
  for (int c0 = 0; c0 < R; c0 += 64 * VW) {
    const int col = c0 + VW * lane;
    const bool cv = col < R;  // R is a multiple of VW
    const int colc = cv ? col : 0;
    uint32_t cur = first;
    bool started_before = cont_in;
    VT sum = VT(0.f), base = VT(0.f);
    auto flush = [&](bool continues) {
      if (!cv || cur == sentinel) return;
      if (started_before)
        *reinterpret_cast<VT*>(&head[seg * R + col]) = sum;
      else if (continues)
        *reinterpret_cast<VT*>(&tail[seg * R + col]) = sum;
      else
        *reinterpret_cast<VT*>(&acc[(int64_t)cur * R + col]) = OVR ? sum : base + sum;
    };
    auto fetch = [&](auto l0c, const Ent& g, uint32_t(&kk)[U], VT(&rv)[U], VT(&av)[U]) {
      constexpr int l0 = decltype(l0c)::value;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        kk[u] = __builtin_amdgcn_readlane(g.k, l0 + u);
        const uint32_t j = __builtin_amdgcn_readlane(g.j, l0 + u);
        const float sc = __uint_as_float(__builtin_amdgcn_readlane(g.s, l0 + u));
        const bool ok = kk[u] != sentinel;
        VT v = VT(1.f);
        if constexpr (HV) v = *reinterpret_cast<const VT*>(&vals[(int64_t)j * R + colc]);
        rv[u] = ok ? v * sc : VT(0.f);
        if constexpr (!OVR) {
          const int64_t row = ok ? (int64_t)kk[u] : 0;
          av[u] = *reinterpret_cast<const VT*>(&acc[row * R + colc]);
        }
      }
    };
    auto consume = [&](const uint32_t(&kk)[U], const VT(&rv)[U], const VT(&av)[U]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (kk[u] == sentinel) continue;
        if (kk[u] != cur) {
          flush(false);
          cur = kk[u];
          started_before = false;
          sum = VT(0.f);
          base = av[u];
        }
        sum += rv[u];
      }
    };
    uint32_t ka[U], kb[U];
    VT ra[U], rb[U], aa[U], ab[U];
    Ent gc = load_group(0);
    fetch(std::integral_constant<int, 0>{}, gc, ka, ra, aa);
    base = aa[0];  // the first run's row (unused when it began earlier)
    // per group: batches 2p (set A) and 2p + 1 (set B); the next batch's loads
    // (the next group's first batch after the last) are issued before the
    // current batch is summed
    for (int gq = 0; gq < G && gq * 64 < len; ++gq) {
      const Ent gn = load_group(gq + 1);
      static_for<NB / 2>([&](auto pc) {
        constexpr int P = decltype(pc)::value;
        fetch(std::integral_constant<int, (2 * P + 1) * U>{}, gc, kb, rb, ab);
        __builtin_amdgcn_sched_barrier(0);
        consume(ka, ra, aa);
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (2 * P + 2 < NB)
          fetch(std::integral_constant<int, (2 * P + 2) * U>{}, gc, ka, ra, aa);
        else
          fetch(std::integral_constant<int, 0>{}, gn, ka, ra, aa);
        __builtin_amdgcn_sched_barrier(0);
        consume(kb, rb, ab);
        __builtin_amdgcn_sched_barrier(0);
      });
      gc = gn;
    }
    flush(cont_out);
  }
}

// Runs that span segments: each list entry is a run's first segment s0. One
// wave per entry: lane t tests whether segment s0 + 1 + t begins with the run's
// row; the first failing test ends the run. Runs over at most 64 later
// segments are combined by the wave itself -- tail[s0] and head[] of those
// segments in a fixed order (eight interleaved sums, then in order) -- and the
// total is the row's only write (store, or added to the row's value). Longer
// runs (the hottest rows) go to a second list for own_fix_long.
template <int VW, bool OVR>
__global__ void __launch_bounds__(256) own_fix(const uint32_t* __restrict__ skey, int64_t n,
                                               int R, float* __restrict__ acc,
                                               const float* __restrict__ head,
                                               const float* __restrict__ tail,
                                               const uint32_t* __restrict__ list,
                                               const uint32_t* __restrict__ nlist,
                                               uint32_t* __restrict__ llist,
                                               uint32_t* __restrict__ nllist) {
  typedef float VT __attribute__((ext_vector_type(VW)));
  const int lane = threadIdx.x & 63;
  const int64_t nseg = (n + kOwnSeg - 1) / kOwnSeg;
  const uint32_t items = *nlist;
  const uint32_t gw = blockIdx.x * 4 + (threadIdx.x >> 6), nw = gridDim.x * 4;
  for (uint32_t it = gw; it < items; it += nw) {
    const int64_t s0 = __builtin_amdgcn_readfirstlane(list[it]);
    const int64_t e1 = min<int64_t>(n, (s0 + 1) * kOwnSeg);
    const uint32_t row = __builtin_amdgcn_readfirstlane(skey[e1 - 1]);
    const int64_t st = s0 + 1 + lane;
    const bool in = st < nseg && skey[st * kOwnSeg] == row;
    const uint64_t miss = __ballot(!in);
    if (miss == 0) {  // continues past 64 more segments
      if (lane == 0) llist[atomicAdd(nllist, 1u)] = (uint32_t)s0;
      continue;
    }
    const int64_t send = s0 + __ffsll((long long)miss) - 1;  // last segment of the run
    for (int c0 = 0; c0 < R; c0 += 64 * VW) {
      const int col = c0 + VW * lane;
      const bool cv = col < R;
      const int colc = cv ? col : 0;
      VT a8[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) a8[q] = VT(0.f);
      int64_t s = s0 + 1;
      for (; s + 7 <= send; s += 8) {
#pragma unroll
        for (int q = 0; q < 8; ++q) a8[q] += *reinterpret_cast<const VT*>(&head[(s + q) * R + colc]);
      }
#pragma unroll
      for (int q = 0; q < 7; ++q)
        if (s + q <= send) a8[q] += *reinterpret_cast<const VT*>(&head[(s + q) * R + colc]);
      if (cv) {
        const VT t = *reinterpret_cast<const VT*>(&tail[s0 * R + col]) +
                     (((a8[0] + a8[1]) + (a8[2] + a8[3])) + ((a8[4] + a8[5]) + (a8[6] + a8[7])));
        VT* p = reinterpret_cast<VT*>(&acc[(int64_t)row * R + col]);
        *p = OVR ? t : *p + t;
      }
    }
  }
}

// The runs own_fix left: one block of 16 waves per entry. Thread t tests segment
// s0 + 1 + t (in rounds of 1024) and the first failing test ends the run; the
// waves add head[] over the run's later segments in a fixed order (wave w takes
// every 16th, eight interleaved sums each), the wave sums are combined in wave
// order with tail[s0], and the total is the row's only write.
template <int VW, bool OVR>
__global__ void __launch_bounds__(1024) own_fix_long(const uint32_t* __restrict__ skey, int64_t n,
                                                     int R, float* __restrict__ acc,
                                                     const float* __restrict__ head,
                                                     const float* __restrict__ tail,
                                                     const uint32_t* __restrict__ llist,
                                                     const uint32_t* __restrict__ nllist) {
  typedef float VT __attribute__((ext_vector_type(VW)));
  __shared__ VT wsum[16][64];
  __shared__ int64_t first_miss[16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t nseg = (n + kOwnSeg - 1) / kOwnSeg;
  const uint32_t items = *nllist;
  for (uint32_t it = blockIdx.x; it < items; it += gridDim.x) {
    const int64_t s0 = llist[it];
    const int64_t e1 = min<int64_t>(n, (s0 + 1) * kOwnSeg);
    const uint32_t row = skey[e1 - 1];
    int64_t send = s0;
    for (int64_t b = s0 + 1;; b += 1024) {
      const int64_t st = b + threadIdx.x;
      const bool in = st < nseg && skey[st * kOwnSeg] == row;
      const uint64_t miss = __ballot(!in);
      __syncthreads();
      first_miss[wv] = miss ? (int64_t)(64 * wv + __ffsll((long long)miss) - 1) : 1024;
      __syncthreads();
      int64_t m = 1024;
#pragma unroll
      for (int w = 0; w < 16; ++w) m = min(m, first_miss[w]);
      send = b + m - 1;
      if (m < 1024) break;
    }
    for (int c0 = 0; c0 < R; c0 += 64 * VW) {
      const int col = c0 + VW * lane;
      const bool cv = col < R;
      const int colc = cv ? col : 0;
      VT a8[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) a8[q] = VT(0.f);
      int64_t s = s0 + 1 + wv;
      for (; s + 7 * 16 <= send; s += 8 * 16) {
#pragma unroll
        for (int q = 0; q < 8; ++q)
          a8[q] += *reinterpret_cast<const VT*>(&head[(s + 16 * q) * R + colc]);
      }
#pragma unroll
      for (int q = 0; q < 7; ++q)
        if (s + 16 * q <= send) a8[q] += *reinterpret_cast<const VT*>(&head[(s + 16 * q) * R + colc]);
      __syncthreads();
      wsum[wv][lane] = ((a8[0] + a8[1]) + (a8[2] + a8[3])) + ((a8[4] + a8[5]) + (a8[6] + a8[7]));
      __syncthreads();
      if (wv == 0 && cv) {
        VT t = *reinterpret_cast<const VT*>(&tail[s0 * R + col]);
#pragma unroll
        for (int w = 0; w < 16; ++w) t += wsum[w][lane];
        VT* p = reinterpret_cast<VT*>(&acc[(int64_t)row * R + col]);
        *p = OVR ? t : *p + t;
      }
    }
  }
}

}  // namespace dexk

// ===========================================================================
namespace dexi {
using namespace dexk;

static int hist_blocks() { return num_cus(); }

size_t sorted_scatter_ws_bytes(int64_t n, int64_t R);

size_t scatter_ws_bytes(int32_t acc_dtype, int64_t n_rows, int64_t row_len, int64_t n,
                        bool has_vals, bool deterministic) {
  if (acc_dtype == DEX_I32 && row_len == 1 && !has_vals && n_rows <= 65536)
    return align256((size_t)hist_blocks() * ((n_rows + 1) / 2) * 4);
  if (acc_dtype == DEX_F32 && deterministic) return sorted_scatter_ws_bytes(n, row_len);
  return 0;
}

dex_status fill_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return DEX_OK;
  if ((bytes & 3) == 0 && (((uintptr_t)p) & 3) == 0) {
    const size_t nw = bytes / 4;
    unsigned blocks = (unsigned)std::min<size_t>((nw + 255) / 256, 65536);
    hipLaunchKernelGGL(fill_zero_kernel, dim3(blocks), dim3(256), 0, s, (uint32_t*)p, nw);
  } else {
    hipLaunchKernelGGL(fill_zero_bytes, dim3((unsigned)((bytes + 255) / 256)), dim3(256), 0, s,
                       (uint8_t*)p, bytes);
  }
  return check_hip(hipGetLastError(), "fill_zero");
}

template <typename IdxT>
static dex_status scatter_typed(void* acc, int32_t acc_dtype, int64_t n_rows, int64_t R,
                                const IdxT* idx, const void* vals, const float* scale, int64_t n,
                                int64_t* oob, void* ws, size_t ws_bytes, hipStream_t s) {
  if (acc_dtype == DEX_I32 && R == 1 && !vals && n_rows <= 65536) {
    const int nb = hist_blocks();
    const size_t need = scatter_ws_bytes(acc_dtype, n_rows, R, n, false, false);
    if (!ws || ws_bytes < need)
      return fail(DEX_ERR_WORKSPACE, "histogram needs %zu workspace bytes, got %zu", need, ws_bytes);
    const int64_t per = ((n + nb - 1) / nb + 3) & ~int64_t(3);
    const int nwords = (int)((n_rows + 1) / 2);
    // up to 128 KiB of dynamic LDS (gfx950 has 160 KiB per compute unit)
    hipError_t ae = hipFuncSetAttribute((const void*)hist_private_kernel<IdxT>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, nwords * 4);
    if (ae != hipSuccess) return check_hip(ae, "histogram LDS size");
    ProfRange pr(DEX_PROF_HIST, s);
    hipLaunchKernelGGL((hist_private_kernel<IdxT>), dim3(nb), dim3(1024), nwords * 4, s,
                       (int32_t*)acc, (int)n_rows, idx, n, per, (uint32_t*)ws, oob);
    pr.end(1);
    hipLaunchKernelGGL(hist_reduce_kernel,
                       dim3((unsigned)((nwords + 255) / 256), (unsigned)((nb + kHistGroup - 1) / kHistGroup)),
                       dim3(256), 0, s, (int32_t*)acc, (int)n_rows, (const uint32_t*)ws, nb);
    return check_hip(hipGetLastError(), "histogram");
  }
  if (acc_dtype == DEX_I32 && scale)
    return fail(DEX_ERR_INVALID_ARG, "integer accumulation takes no float scale");
  if (acc_dtype == DEX_I32 && R > 1 && !vals) {
    // ones into every column of a row: generic exact path
  }
  const unsigned nchunks = (unsigned)((n + kChunk - 1) / kChunk);
  if (n_rows >= (int64_t(1) << 51)) return fail(DEX_ERR_UNSUPPORTED, "n_rows too large");
  if (acc_dtype == DEX_F32) {
    ProfRange pr(DEX_PROF_SCATTER, s);
    float* a = (float*)acc;
    const float* v = (const float*)vals;
    if (vals && scale)
      hipLaunchKernelGGL((scatter_rows_kernel<float, IdxT, 8, true, true>), dim3(nchunks),
                         dim3(256), 0, s, a, n_rows, (int)R, idx, v, scale, n, oob);
    else if (vals)
      hipLaunchKernelGGL((scatter_rows_kernel<float, IdxT, 8, true, false>), dim3(nchunks),
                         dim3(256), 0, s, a, n_rows, (int)R, idx, v, scale, n, oob);
    else if (scale)
      hipLaunchKernelGGL((scatter_rows_kernel<float, IdxT, 8, false, true>), dim3(nchunks),
                         dim3(256), 0, s, a, n_rows, (int)R, idx, v, scale, n, oob);
    else
      hipLaunchKernelGGL((scatter_rows_kernel<float, IdxT, 8, false, false>), dim3(nchunks),
                         dim3(256), 0, s, a, n_rows, (int)R, idx, v, scale, n, oob);
    pr.end(1);
  } else {
    if (R <= 4) {
      const int64_t tot = n * R;
      hipLaunchKernelGGL((scatter_int_generic<IdxT>), dim3((unsigned)((tot + 255) / 256)), dim3(256),
                         0, s, (int32_t*)acc, n_rows, R, idx, (const int32_t*)vals, n, oob);
    } else {
      if (vals)
        hipLaunchKernelGGL((scatter_rows_kernel<int32_t, IdxT, 8, true, false>), dim3(nchunks),
                           dim3(256), 0, s, (int32_t*)acc, n_rows, (int)R, idx,
                           (const int32_t*)vals, nullptr, n, oob);
      else
        hipLaunchKernelGGL((scatter_rows_kernel<int32_t, IdxT, 8, false, false>), dim3(nchunks),
                           dim3(256), 0, s, (int32_t*)acc, n_rows, (int)R, idx,
                           (const int32_t*)vals, nullptr, n, oob);
    }
  }
  return check_hip(hipGetLastError(), "accum_scatter");
}

// Workspace of the sorted (deterministic) float scatter.
struct SortWs {
  uint32_t *ka, *kb, *cnt, *tot, *list, *nlist, *llist;
  uint64_t *va, *vb;
  float *pf, *pl;
  size_t bytes;
};

static SortWs sort_ws(int64_t n, int64_t R, char* base) {
  SortWs w{};
  size_t o = 0;
  auto take = [&](size_t b) {
    size_t at = o;
    o += align256(b);
    return base ? (void*)(base + at) : nullptr;
  };
  const int64_t ntiles = (n + kRsTile - 1) / kRsTile;
  const int64_t nseg = (n + kOwnSeg - 1) / kOwnSeg;
  w.ka = (uint32_t*)take((size_t)n * 4);
  w.kb = (uint32_t*)take((size_t)n * 4);
  w.va = (uint64_t*)take((size_t)n * 8);
  w.vb = (uint64_t*)take((size_t)n * 8);
  w.cnt = (uint32_t*)take((size_t)kRsDigits * ntiles * 4);
  w.tot = (uint32_t*)take(kRsDigits * 4);
  w.pf = (float*)take((size_t)nseg * R * 4);
  w.pl = (float*)take((size_t)nseg * R * 4);
  w.list = (uint32_t*)take((size_t)nseg * 4);
  w.llist = (uint32_t*)take((size_t)nseg * 4);
  w.nlist = (uint32_t*)take(8);  // [0]: spanning runs, [1]: the long ones among them
  w.bytes = o;
  return w;
}

size_t sorted_scatter_ws_bytes(int64_t n, int64_t R) { return sort_ws(n, R, nullptr).bytes; }

template <int VW, bool OVR>
static void launch_own(const SortWs& w, const uint32_t* skey, const uint64_t* sval, int64_t n,
                       uint32_t sentinel, const float* vals, int R, float* acc, hipStream_t s) {
  const int64_t nseg = (n + kOwnSeg - 1) / kOwnSeg;
  const unsigned sb = (unsigned)((nseg + 3) / 4);
  if (vals)
    hipLaunchKernelGGL((own_sum<VW, 16, true, OVR>), dim3(sb), dim3(256), 0, s, skey, sval, n,
                       sentinel, vals, R, acc, w.pf, w.pl, w.list, w.nlist);
  else
    hipLaunchKernelGGL((own_sum<VW, 16, false, OVR>), dim3(sb), dim3(256), 0, s, skey, sval, n,
                       sentinel, vals, R, acc, w.pf, w.pl, w.list, w.nlist);
  // fixed grids that walk the lists of spanning runs (their lengths stay on the device)
  const unsigned fb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((nseg + 3) / 4, 4 * num_cus()));
  hipLaunchKernelGGL((own_fix<VW, OVR>), dim3(fb), dim3(256), 0, s, skey, n, R, acc, w.pf, w.pl,
                     w.list, w.nlist, w.llist, w.nlist + 1);
  hipLaunchKernelGGL((own_fix_long<VW, OVR>), dim3((unsigned)num_cus()), dim3(1024), 0, s, skey, n,
                     R, acc, w.pf, w.pl, w.llist, w.nlist + 1);
}

template <typename IdxT>
static dex_status scatter_sorted(float* acc, int64_t n_rows, int64_t R, const IdxT* idx,
                                 const float* vals, const float* scale, int64_t n, int64_t* oob,
                                 bool overwrite, void* ws, size_t ws_bytes, hipStream_t s) {
  if (n_rows > 0xFFFFFFFEll || n > 0xFFFFFFFFll)
    return fail(DEX_ERR_UNSUPPORTED, "sorted scatter: at most 2^32-2 rows and 2^32 indices");
  const SortWs w = sort_ws(n, R, (char*)ws);
  if (!ws || ws_bytes < w.bytes)
    return fail(DEX_ERR_WORKSPACE, "sorted scatter needs %zu workspace bytes, got %zu", w.bytes, ws_bytes);
  const int ntiles = (int)((n + kRsTile - 1) / kRsTile);
  const int nbits = 64 - __builtin_clzll((unsigned long long)n_rows);  // n_rows itself is the sentinel
  const int passes = (nbits + kRsBits - 1) / kRsBits;
  ProfRange pr(DEX_PROF_SCATTER, s);
  // pass 0 reads the indices and scales directly; the sorted pairs then
  // alternate between the two buffers
  uint32_t *kin = w.ka, *kout = w.kb;
  uint64_t *vin = w.va, *vout = w.vb;
  for (int p = 0; p < passes; ++p) {
    const int shift = kRsBits * p;
    if (p == 0)
      hipLaunchKernelGGL((rs_hist<true, IdxT>), dim3(ntiles), dim3(1024), 0, s, idx, kin, n, n_rows,
                         shift, w.cnt, ntiles, w.nlist, oob);
    else
      hipLaunchKernelGGL((rs_hist<false, IdxT>), dim3(ntiles), dim3(1024), 0, s, idx, kin, n,
                         n_rows, shift, w.cnt, ntiles, w.nlist, oob);
    hipLaunchKernelGGL(rs_digit_scan, dim3(kRsDigits), dim3(256), 0, s, w.cnt, ntiles, w.tot);
    if (p == 0)
      hipLaunchKernelGGL((rs_scatter<true, IdxT>), dim3(ntiles), dim3(1024), 0, s, idx, scale, n_rows,
                         kin, vin, kout, vout, n, shift, w.cnt, w.tot, ntiles);
    else
      hipLaunchKernelGGL((rs_scatter<false, IdxT>), dim3(ntiles), dim3(1024), 0, s, idx, scale,
                         n_rows, kin, vin, kout, vout, n, shift, w.cnt, w.tot, ntiles);
    std::swap(kin, kout);
    std::swap(vin, vout);
  }
  // widest column vector the row length and the pointers' alignment allow
  const uintptr_t al = (uintptr_t)acc | (uintptr_t)(vals ? vals : acc);
  const int vw = (R % 4 == 0 && R >= 256 && (al & 15) == 0) ? 4 : (R % 2 == 0 && (al & 7) == 0) ? 2 : 1;
  const uint32_t sent = (uint32_t)n_rows;
#define DEX_OWNL(V)                                                                   \
  (overwrite ? launch_own<V, true>(w, kin, vin, n, sent, vals, (int)R, acc, s)        \
             : launch_own<V, false>(w, kin, vin, n, sent, vals, (int)R, acc, s))
  if (vw == 4)
    DEX_OWNL(4);
  else if (vw == 2)
    DEX_OWNL(2);
  else
    DEX_OWNL(1);
#undef DEX_OWNL
  pr.end(1);
  return check_hip(hipGetLastError(), "sorted scatter");
}

dex_status accum_scatter(void* acc, int32_t acc_dtype, int64_t n_rows, int64_t row_len,
                         const void* idx, int32_t idx_dtype, const void* vals,
                         const float* scale, int64_t n, bool count_oob, int64_t* oob, void* ws,
                         size_t ws_bytes, int path, hipStream_t s, bool overwrite) {
  if (n == 0) return DEX_OK;
  int64_t* o = count_oob ? oob : nullptr;
  if (path == kScatterSorted && acc_dtype == DEX_F32) {
    if (idx_dtype == DEX_I32)
      return scatter_sorted<int32_t>((float*)acc, n_rows, row_len, (const int32_t*)idx,
                                     (const float*)vals, scale, n, o, overwrite, ws, ws_bytes, s);
    return scatter_sorted<uint32_t>((float*)acc, n_rows, row_len, (const uint32_t*)idx,
                                    (const float*)vals, scale, n, o, overwrite, ws, ws_bytes, s);
  }
  if (idx_dtype == DEX_I32)
    return scatter_typed<int32_t>(acc, acc_dtype, n_rows, row_len, (const int32_t*)idx, vals,
                                  scale, n, o, ws, ws_bytes, s);
  return scatter_typed<uint32_t>(acc, acc_dtype, n_rows, row_len, (const uint32_t*)idx, vals,
                                 scale, n, o, ws, ws_bytes, s);
}

dex_status gather_fwd(const float* T, const int32_t* idx, const float* w, int64_t V, int64_t R,
                      int64_t n, float* out, bool count, int64_t* oob, hipStream_t s) {
  if (n == 0) return DEX_OK;
  int64_t* o = count ? oob : nullptr;
  const bool vec = (R % 4) == 0 && ((uintptr_t)T & 15) == 0 && ((uintptr_t)out & 15) == 0;
  ProfRange pr(DEX_PROF_GATHER, s);
  if (vec) {
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 7) / 8, (int64_t)num_cus() * 32);
    hipLaunchKernelGGL(gather_scale_kernel, dim3(blocks), dim3(256), 0, s, T, idx, w, V, (int)R, n,
                       out, o);
  } else {
    hipLaunchKernelGGL(gather_scale_scalar, dim3((unsigned)((n * R + 255) / 256)), dim3(256), 0, s,
                       T, idx, w, V, (int)R, n, out, o);
  }
  pr.end(1);
  return check_hip(hipGetLastError(), "gather_fwd");
}

dex_status gather_jvp(const float* T, const float* tT, const int32_t* idx, const float* w,
                      const float* tw, int64_t V, int64_t R, int64_t n, float* tout,
                      hipStream_t s) {
  if (n == 0) return DEX_OK;
  const bool vec = (R % 4) == 0 && ((uintptr_t)T & 15) == 0 && ((uintptr_t)tT & 15) == 0 &&
                   ((uintptr_t)tout & 15) == 0;
  ProfRange pr(DEX_PROF_GATHER_JVP, s);
  if (vec) {
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 7) / 8, (int64_t)num_cus() * 32);
    hipLaunchKernelGGL(gather_jvp_kernel, dim3(blocks), dim3(256), 0, s, T, tT, idx, w, tw, V,
                       (int)R, n, tout);
  } else {
    hipLaunchKernelGGL(gather_jvp_scalar, dim3((unsigned)((n * R + 255) / 256)), dim3(256), 0, s,
                       T, tT, idx, w, tw, V, (int)R, n, tout);
  }
  pr.end(1);
  return check_hip(hipGetLastError(), "gather_jvp");
}

dex_status gather_dw(const float* T, const int32_t* idx, const float* g, int64_t V, int64_t R,
                     int64_t n, float* dw, bool accumulate, hipStream_t s) {
  if (n == 0) return DEX_OK;
  const bool vec = (R % 4) == 0 && ((uintptr_t)T & 15) == 0 && ((uintptr_t)g & 15) == 0;
  const unsigned blocks = (unsigned)std::min<int64_t>((n + 7) / 8, (int64_t)num_cus() * 32);
  (void)vec;
  ProfRange pr(DEX_PROF_GATHER_DW, s);
  hipLaunchKernelGGL(gather_dw_kernel, dim3(blocks), dim3(256), 0, s, T, idx, g, V, (int)R, n, dw,
                     accumulate ? 1 : 0);
  pr.end(1);
  return check_hip(hipGetLastError(), "gather_dw");
}

}  // namespace dexi
