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
template <typename T, typename IdxT, int U>
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

  // each wave takes a contiguous slice of the sorted chunk
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int per = (kChunk + nw - 1) / nw;
  const int e0 = wv * per, e1 = min(kChunk, e0 + per);
  for (int c0 = 0; c0 < R; c0 += 64) {
    const int col = c0 + lane;
    const bool cv = col < R;
    uint64_t cur = ~uint64_t(0);
    T sum = 0;
    for (int e = e0; e < e1; e += U) {
      T r[U];
      uint64_t kk[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        kk[u] = (e + u < e1) ? key[e + u] : ~uint64_t(0);
        r[u] = 0;
        if (kk[u] != ~uint64_t(0) && cv) {
          const int64_t j = j0 + (int64_t)(kk[u] & 4095u);
          T v = vals ? vals[j * R + col] : T(1);
          if constexpr (std::is_floating_point<T>::value) {
            if (scale) v = v * scale[j];
          }
          r[u] = v;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (kk[u] == ~uint64_t(0)) continue;
        const uint64_t row = kk[u] >> 12;
        if (row != (cur >> 12)) {
          if (cur != ~uint64_t(0) && cv) atomicAdd(&acc[(int64_t)(cur >> 12) * R + col], sum);
          cur = kk[u];
          sum = 0;
        }
        sum += r[u];
      }
    }
    if (cur != ~uint64_t(0) && cv) atomicAdd(&acc[(int64_t)(cur >> 12) * R + col], sum);
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
    for (int64_t q = a0 / 4 + threadIdx.x; q < a1 / 4; q += blockDim.x) {
      const u32x4 v = __builtin_nontemporal_load(k4 + q);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if constexpr (IdxT(-1) < IdxT(0))
          bump((int64_t)(int32_t)v[e]);
        else
          bump((int64_t)v[e]);
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

}  // namespace dexk

// ===========================================================================
namespace dexi {
using namespace dexk;

static int hist_blocks() { return num_cus(); }

size_t scatter_ws_bytes(int32_t acc_dtype, int64_t n_rows, int64_t row_len, int64_t n,
                        bool has_vals) {
  (void)n;
  if (acc_dtype == DEX_I32 && row_len == 1 && !has_vals && n_rows <= 65536)
    return align256((size_t)hist_blocks() * ((n_rows + 1) / 2) * 4);
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
    const size_t need = scatter_ws_bytes(acc_dtype, n_rows, R, n, false);
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
    hipLaunchKernelGGL((scatter_rows_kernel<float, IdxT, 8>), dim3(nchunks), dim3(256), 0, s,
                       (float*)acc, n_rows, (int)R, idx, (const float*)vals, scale, n, oob);
    pr.end(1);
  } else {
    if (R <= 4) {
      const int64_t tot = n * R;
      hipLaunchKernelGGL((scatter_int_generic<IdxT>), dim3((unsigned)((tot + 255) / 256)), dim3(256),
                         0, s, (int32_t*)acc, n_rows, R, idx, (const int32_t*)vals, n, oob);
    } else {
      hipLaunchKernelGGL((scatter_rows_kernel<int32_t, IdxT, 8>), dim3(nchunks), dim3(256), 0, s,
                         (int32_t*)acc, n_rows, (int)R, idx, (const int32_t*)vals, nullptr, n, oob);
    }
  }
  return check_hip(hipGetLastError(), "accum_scatter");
}

dex_status accum_scatter(void* acc, int32_t acc_dtype, int64_t n_rows, int64_t row_len,
                         const void* idx, int32_t idx_dtype, const void* vals,
                         const float* scale, int64_t n, bool count_oob, int64_t* oob, void* ws,
                         size_t ws_bytes, int cfg, hipStream_t s) {
  (void)cfg;
  if (n == 0) return DEX_OK;
  int64_t* o = count_oob ? oob : nullptr;
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
