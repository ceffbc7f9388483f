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
    // four 16-byte loads in flight per thread before the LDS updates
    const int64_t q1 = a1 / 4;
    const int64_t step = (int64_t)blockDim.x;
    for (int64_t q = a0 / 4 + threadIdx.x; q < q1; q += 4 * step) {
      u32x4 v[4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        v[i] = (q + i * step < q1) ? __builtin_nontemporal_load(k4 + q + i * step)
                                   : u32x4{0u, 0u, 0u, 0u};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (q + i * step >= q1) break;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if constexpr (IdxT(-1) < IdxT(0))
            bump((int64_t)(int32_t)v[i][e]);
          else
            bump((int64_t)v[i][e]);
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

// acc[b] += sum over blocks of the packed partial counters (fixed order).
__global__ void __launch_bounds__(256) hist_reduce_kernel(int32_t* __restrict__ acc, int n_bins,
                                                          const uint32_t* __restrict__ partial,
                                                          int nblocks) {
  const int w = blockIdx.x * 256 + threadIdx.x;
  const int nwords = (n_bins + 1) >> 1;
  if (w >= nwords) return;
  uint32_t lo = 0, hi = 0;
  for (int b = 0; b < nblocks; ++b) {
    const uint32_t v = partial[(size_t)b * nwords + w];
    lo += v & 0xFFFFu;
    hi += v >> 16;
  }
  acc[2 * w] += (int32_t)lo;
  if (2 * w + 1 < n_bins) acc[2 * w + 1] += (int32_t)hi;
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

// out[j, :] = w[j] * T[idx[j], :]; half a wave per row, 4 floats per lane.
__global__ void __launch_bounds__(256) gather_scale_kernel(const float* __restrict__ T,
                                                           const int32_t* __restrict__ idx,
                                                           const float* __restrict__ w,
                                                           int64_t V, int R, int64_t n,
                                                           float* __restrict__ out,
                                                           int64_t* oob) {
  const int half = threadIdx.x >> 5, hl = threadIdx.x & 31;
  const int64_t rows_per_iter = (int64_t)gridDim.x * 8;
  int bad = 0;
  for (int64_t j = (int64_t)blockIdx.x * 8 + half; j < n; j += rows_per_iter) {
    const int64_t v = idx[j];
    const bool ok = v >= 0 && v < V;
    if (!ok && hl == 0) ++bad;
    const float s = w[j];
    for (int c = 4 * hl; c < R; c += 128) {
      f32x4 t = ok ? *reinterpret_cast<const f32x4*>(T + v * R + c) : f32x4{0.f, 0.f, 0.f, 0.f};
      const f32x4 o = t * s;
      __builtin_nontemporal_store(o, reinterpret_cast<f32x4*>(out + j * R + c));
    }
  }
  if (oob) count_oob(bad, oob);
}

// Forward mode of the gather (the linear map of its linearization, Sec. 5.1;
// idx is an integer, so it carries no tangent):
//   tout[j, :] = tw[j] * T[idx[j], :] + w[j] * tT[idx[j], :]
// Same layout as the gather: half a wave per row, 4 floats per lane; rows with
// an index outside [0, V) give zeros.
__global__ void __launch_bounds__(256) gather_jvp_kernel(const float* __restrict__ T,
                                                         const float* __restrict__ tT,
                                                         const int32_t* __restrict__ idx,
                                                         const float* __restrict__ w,
                                                         const float* __restrict__ tw, int64_t V,
                                                         int R, int64_t n,
                                                         float* __restrict__ tout) {
  const int half = threadIdx.x >> 5, hl = threadIdx.x & 31;
  const int64_t rows_per_iter = (int64_t)gridDim.x * 8;
  for (int64_t j = (int64_t)blockIdx.x * 8 + half; j < n; j += rows_per_iter) {
    const int64_t v = idx[j];
    const bool ok = v >= 0 && v < V;
    const float a = tw[j], b = w[j];
    for (int c = 4 * hl; c < R; c += 128) {
      f32x4 o = f32x4{0.f, 0.f, 0.f, 0.f};
      if (ok) {
        const f32x4 x = *reinterpret_cast<const f32x4*>(T + v * R + c);
        const f32x4 y = *reinterpret_cast<const f32x4*>(tT + v * R + c);
#pragma unroll
        for (int e = 0; e < 4; ++e) o[e] = fmaf(b, y[e], a * x[e]);
      }
      __builtin_nontemporal_store(o, reinterpret_cast<f32x4*>(tout + j * R + c));
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
constexpr int kSeg = 256;       // sorted entries per wave in the run-sum pass

// keys[j] = idx[j] if it is inside [0, n_rows), else n_rows (sorts last and is
// skipped); vals[j] = j.
template <typename IdxT>
__global__ void __launch_bounds__(256) rs_init(const IdxT* __restrict__ idx, int64_t n,
                                               int64_t n_rows, uint32_t* __restrict__ keys,
                                               uint32_t* __restrict__ vals, int64_t* oob) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int bad = 0;
  if (j < n) {
    const int64_t v = load_index(idx, j);
    const bool ok = v >= 0 && v < n_rows;
    bad = !ok;
    keys[j] = ok ? (uint32_t)v : (uint32_t)n_rows;
    vals[j] = (uint32_t)j;
  }
  if (oob) count_oob(bad, oob);
}

// Digit counts of one tile: cnt[digit * ntiles + tile]. Exact, order-free.
__global__ void __launch_bounds__(1024) rs_hist(const uint32_t* __restrict__ keys, int64_t n,
                                                int shift, uint32_t* __restrict__ cnt, int ntiles) {
  __shared__ uint32_t h[256];
  if (threadIdx.x < 256) h[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t t0 = (int64_t)blockIdx.x * kRsTile;
#pragma unroll
  for (int r = 0; r < kRsTile / 1024; ++r) {
    const int64_t j = t0 + r * 1024 + threadIdx.x;
    if (j < n) atomicAdd(&h[(keys[j] >> shift) & 255u], 1u);
  }
  __syncthreads();
  if (threadIdx.x < 256) cnt[(size_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Per digit (one block each): exclusive prefix of the tile counts, and the total.
__global__ void __launch_bounds__(256) rs_digit_scan(uint32_t* __restrict__ cnt, int ntiles,
                                                     uint32_t* __restrict__ tot) {
  __shared__ uint32_t sh[256];
  uint32_t carry = 0;
  uint32_t* row = cnt + (size_t)blockIdx.x * ntiles;
  for (int b = 0; b < ntiles; b += 256) {
    const int i = b + threadIdx.x;
    const uint32_t v = i < ntiles ? row[i] : 0u;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {  // inclusive Hillis-Steele scan
      const uint32_t t = threadIdx.x >= o ? sh[threadIdx.x - o] : 0u;
      __syncthreads();
      sh[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < ntiles) row[i] = carry + sh[threadIdx.x] - v;
    carry += sh[255];
    __syncthreads();
  }
  if (threadIdx.x == 0) tot[blockIdx.x] = carry;
}

// Lanes of this wave holding the same 8-bit digit as this lane (among `live`).
DEX_DEV uint64_t digit_peers(uint32_t d, uint64_t live) {
  uint64_t m = live;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const uint64_t bal = __ballot((d >> b) & 1u);
    m &= ((d >> b) & 1u) ? bal : ~bal;
  }
  return m;
}

// Stable scatter of one tile by digit: keys are taken in index order (round r,
// then thread), ranked within the wave by ballots and across waves by
// per-wave digit counts in LDS; no atomics, so the output order is fixed.
__global__ void __launch_bounds__(1024) rs_scatter(const uint32_t* __restrict__ kin,
                                                   const uint32_t* __restrict__ vin,
                                                   uint32_t* __restrict__ kout,
                                                   uint32_t* __restrict__ vout, int64_t n,
                                                   int shift, const uint32_t* __restrict__ cnt,
                                                   const uint32_t* __restrict__ tot, int ntiles) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t whist[16][256];
  __shared__ uint32_t wsum[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // exclusive scan of the digit totals by the first 4 waves (whole waves)
  uint32_t v = 0, x = 0;
  if (tid < 256) {
    v = tot[tid];
    x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wv] = x;
  }
  __syncthreads();
  if (tid < 256) {
    uint32_t pre = 0;
    for (int w = 0; w < wv; ++w) pre += wsum[w];
    base[tid] = pre + x - v + cnt[(size_t)tid * ntiles + blockIdx.x];
  }
  const int64_t t0 = (int64_t)blockIdx.x * kRsTile;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int r = 0; r < kRsTile / 1024; ++r) {
    for (int e = tid; e < 16 * 256; e += 1024) (&whist[0][0])[e] = 0u;
    const int64_t j = t0 + r * 1024 + tid;
    const bool valid = j < n;
    const uint32_t key = valid ? kin[j] : 0u;
    const uint32_t val = valid ? vin[j] : 0u;
    const uint32_t d = (key >> shift) & 255u;
    const uint64_t live = __ballot(valid);
    const uint64_t peers = digit_peers(d, live);
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    __syncthreads();
    if (valid && rank == 0) whist[wv][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (tid < 256) {
      uint32_t run = base[tid];
#pragma unroll
      for (int w = 0; w < 16; ++w) {
        const uint32_t c = whist[w][tid];
        whist[w][tid] = run;
        run += c;
      }
      base[tid] = run;
    }
    __syncthreads();
    if (valid) {
      const uint32_t pos = whist[wv][d] + rank;
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
  }
}

// One wave per segment of kSeg sorted entries. Runs of equal rows are summed in
// registers (row_len columns over the lanes); a run wholly inside the segment
// is added to acc by this wave alone; a run that starts earlier leaves its
// partial in part_first[seg], one that continues past the segment in
// part_last[seg], for seg_fix. Every row thus receives exactly one addition
// (here or in seg_fix), so a non-returning atomic add gives a fixed result and
// never stalls the loop; the segment's keys and positions are staged in LDS
// and the values of the next U entries are loaded before the current U are
// summed (loads retire in issue order, so they never wait for the adds).
template <int U, bool HV, bool HS>
__global__ void __launch_bounds__(256) seg_sum(const uint32_t* __restrict__ skey,
                                               const uint32_t* __restrict__ spos, int64_t n,
                                               uint32_t sentinel, const float* __restrict__ vals,
                                               const float* __restrict__ scale, int R,
                                               float* __restrict__ acc,
                                               float* __restrict__ part_first,
                                               float* __restrict__ part_last) {
  __shared__ uint32_t sk[4][kSeg], sp[4][kSeg];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t seg = (int64_t)blockIdx.x * 4 + wv;
  const int64_t e0 = seg * kSeg;
  if (e0 >= n) return;
  const int len = (int)min<int64_t>(kSeg, n - e0);
#pragma unroll
  for (int q = 0; q < kSeg / 64; ++q) {
    const int e = q * 64 + lane;
    sk[wv][e] = e < len ? skey[e0 + e] : sentinel;
    sp[wv][e] = e < len ? spos[e0 + e] : 0u;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const uint32_t first = sk[wv][0];
  if (first == sentinel) return;
  const bool cont_in = e0 > 0 && skey[e0 - 1] == first;
  const uint32_t lastk = sk[wv][len - 1];
  const bool cont_out = e0 + len < n && skey[e0 + len] == lastk && lastk != sentinel;
  for (int c0 = 0; c0 < R; c0 += 64) {
    const int col = c0 + lane;
    const bool cv = col < R;
    const int colc = cv ? col : R - 1;
    uint32_t cur = first;
    bool started_before = cont_in;
    float sum = 0.f;
    auto flush = [&](bool continues) {
      if (!cv || cur == sentinel) return;
      if (started_before)
        part_first[seg * R + col] = sum;
      else if (continues)
        part_last[seg * R + col] = sum;
      else
        atomicAdd(&acc[(int64_t)cur * R + col], sum);
    };
    auto fetch = [&](int e, uint32_t(&kk)[U], float(&rv)[U]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int ec = min(e + u, kSeg - 1);
        kk[u] = e + u < len ? sk[wv][ec] : sentinel;
        const bool ok = kk[u] != sentinel;
        const int64_t j = ok ? (int64_t)sp[wv][ec] : 0;
        float v = 1.f;
        if constexpr (HV) v = vals[j * R + colc];
        if constexpr (HS) v *= scale[j];
        rv[u] = ok ? v : 0.f;
      }
    };
    auto consume = [&](const uint32_t(&kk)[U], const float(&rv)[U]) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (kk[u] == sentinel) continue;
        if (kk[u] != cur) {
          flush(false);
          cur = kk[u];
          started_before = false;
          sum = 0.f;
        }
        sum += rv[u];
      }
    };
    uint32_t ka[U], kb[U];
    float ra[U], rb[U];
    fetch(0, ka, ra);
    for (int e = 0; e < len; e += 2 * U) {
      fetch(e + U, kb, rb);
      __builtin_amdgcn_sched_barrier(0);
      consume(ka, ra);
      __builtin_amdgcn_sched_barrier(0);
      fetch(e + 2 * U, ka, ra);
      __builtin_amdgcn_sched_barrier(0);
      consume(kb, rb);
      __builtin_amdgcn_sched_barrier(0);
    }
    flush(cont_out);
  }
}

// For each segment whose last run starts in it and continues into the next
// segments: the run's end is found by binary search in the sorted keys; the
// block then adds the segment's partial and the following segments' first-run
// partials in a fixed order (wave w takes every fourth segment, the four wave
// sums are combined in wave order) and adds the total to acc, the row's only
// addition. One block per segment; most exit after two key reads.
__global__ void __launch_bounds__(256) seg_fix(const uint32_t* __restrict__ skey, int64_t n,
                                               uint32_t sentinel, int R, float* __restrict__ acc,
                                               const float* __restrict__ part_first,
                                               const float* __restrict__ part_last) {
  __shared__ float wsum[4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t seg = blockIdx.x;
  const int64_t e0 = seg * kSeg, e1 = min<int64_t>(n, e0 + kSeg);
  if (e0 >= n) return;
  const uint32_t row = skey[e1 - 1];
  if (row == sentinel) return;
  const bool cont_out = e1 < n && skey[e1] == row;
  if (!cont_out) return;
  const bool whole_from_before = e0 > 0 && skey[e0 - 1] == row && skey[e0] == row;
  if (whole_from_before) return;  // the run started in an earlier segment
  // last position of the run: largest q with skey[q] == row (keys ascending)
  int64_t lo = e1, hi = n - 1;
  while (lo < hi) {
    const int64_t mid = hi - (hi - lo) / 2;
    if (skey[mid] == row)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int64_t send = lo / kSeg;  // segments seg+1 .. send hold the rest of the run
  for (int c0 = 0; c0 < R; c0 += 64) {
    const int col = c0 + lane;
    const bool cv = col < R;
    float s = 0.f;
    if (cv)
      for (int64_t s2 = seg + 1 + wv; s2 <= send; s2 += 4) s += part_first[s2 * R + col];
    __syncthreads();
    wsum[wv][lane] = s;
    __syncthreads();
    if (wv == 0 && cv) {
      const float total =
          part_last[seg * R + col] + (((wsum[0][lane] + wsum[1][lane]) + wsum[2][lane]) + wsum[3][lane]);
      atomicAdd(&acc[(int64_t)row * R + col], total);  // the row's only addition
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
    hipLaunchKernelGGL(hist_reduce_kernel, dim3((unsigned)((nwords + 255) / 256)), dim3(256), 0, s,
                       (int32_t*)acc, (int)n_rows, (const uint32_t*)ws, nb);
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
  uint32_t *ka, *va, *kb, *vb, *cnt, *tot;
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
  const int64_t nseg = (n + kSeg - 1) / kSeg;
  w.ka = (uint32_t*)take((size_t)n * 4);
  w.va = (uint32_t*)take((size_t)n * 4);
  w.kb = (uint32_t*)take((size_t)n * 4);
  w.vb = (uint32_t*)take((size_t)n * 4);
  w.cnt = (uint32_t*)take((size_t)256 * ntiles * 4);
  w.tot = (uint32_t*)take(256 * 4);
  w.pf = (float*)take((size_t)nseg * R * 4);
  w.pl = (float*)take((size_t)nseg * R * 4);
  w.bytes = o;
  return w;
}

size_t sorted_scatter_ws_bytes(int64_t n, int64_t R) { return sort_ws(n, R, nullptr).bytes; }

template <typename IdxT>
static dex_status scatter_sorted(float* acc, int64_t n_rows, int64_t R, const IdxT* idx,
                                 const float* vals, const float* scale, int64_t n, int64_t* oob,
                                 void* ws, size_t ws_bytes, hipStream_t s) {
  if (n_rows > 0xFFFFFFFEll || n > 0xFFFFFFFFll)
    return fail(DEX_ERR_UNSUPPORTED, "sorted scatter: at most 2^32-2 rows and 2^32 indices");
  const SortWs w = sort_ws(n, R, (char*)ws);
  if (!ws || ws_bytes < w.bytes)
    return fail(DEX_ERR_WORKSPACE, "sorted scatter needs %zu workspace bytes, got %zu", w.bytes, ws_bytes);
  const int ntiles = (int)((n + kRsTile - 1) / kRsTile);
  const int64_t nseg = (n + kSeg - 1) / kSeg;
  const int nbits = 64 - __builtin_clzll((unsigned long long)n_rows);  // n_rows itself is the sentinel
  const int passes = (nbits + 7) / 8;
  ProfRange pr(DEX_PROF_SCATTER, s);
  hipLaunchKernelGGL((rs_init<IdxT>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, idx, n,
                     n_rows, w.ka, w.va, oob);
  uint32_t *kin = w.ka, *vin = w.va, *kout = w.kb, *vout = w.vb;
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    hipLaunchKernelGGL(rs_hist, dim3(ntiles), dim3(1024), 0, s, kin, n, shift, w.cnt, ntiles);
    hipLaunchKernelGGL(rs_digit_scan, dim3(256), dim3(256), 0, s, w.cnt, ntiles, w.tot);
    hipLaunchKernelGGL(rs_scatter, dim3(ntiles), dim3(1024), 0, s, kin, vin, kout, vout, n, shift,
                       w.cnt, w.tot, ntiles);
    std::swap(kin, kout);
    std::swap(vin, vout);
  }
  const unsigned sb = (unsigned)((nseg + 3) / 4);
  if (vals && scale)
    hipLaunchKernelGGL((seg_sum<8, true, true>), dim3(sb), dim3(256), 0, s, kin, vin, n,
                       (uint32_t)n_rows, vals, scale, (int)R, acc, w.pf, w.pl);
  else if (vals)
    hipLaunchKernelGGL((seg_sum<8, true, false>), dim3(sb), dim3(256), 0, s, kin, vin, n,
                       (uint32_t)n_rows, vals, scale, (int)R, acc, w.pf, w.pl);
  else if (scale)
    hipLaunchKernelGGL((seg_sum<8, false, true>), dim3(sb), dim3(256), 0, s, kin, vin, n,
                       (uint32_t)n_rows, vals, scale, (int)R, acc, w.pf, w.pl);
  else
    hipLaunchKernelGGL((seg_sum<8, false, false>), dim3(sb), dim3(256), 0, s, kin, vin, n,
                       (uint32_t)n_rows, vals, scale, (int)R, acc, w.pf, w.pl);
  hipLaunchKernelGGL(seg_fix, dim3((unsigned)nseg), dim3(256), 0, s, kin, n, (uint32_t)n_rows,
                     (int)R, acc, w.pf, w.pl);
  pr.end(1);
  return check_hip(hipGetLastError(), "sorted scatter");
}

dex_status accum_scatter(void* acc, int32_t acc_dtype, int64_t n_rows, int64_t row_len,
                         const void* idx, int32_t idx_dtype, const void* vals,
                         const float* scale, int64_t n, bool count_oob, int64_t* oob, void* ws,
                         size_t ws_bytes, int cfg, hipStream_t s) {
  if (n == 0) return DEX_OK;
  int64_t* o = count_oob ? oob : nullptr;
  if (cfg == 1 && acc_dtype == DEX_F32) {
    if (idx_dtype == DEX_I32)
      return scatter_sorted<int32_t>((float*)acc, n_rows, row_len, (const int32_t*)idx,
                                     (const float*)vals, scale, n, o, ws, ws_bytes, s);
    return scatter_sorted<uint32_t>((float*)acc, n_rows, row_len, (const uint32_t*)idx,
                                    (const float*)vals, scale, n, o, ws, ws_bytes, s);
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
