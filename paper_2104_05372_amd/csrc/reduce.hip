// Regular segmented reduction and complete reduction (Sec. 6.1.3: the two
// accumulator indexing patterns besides the irregular one of the scatter):
//   segmented  for i j. acc!i += values.i.j   -> out[i] = sum_j values[i, j]
//   complete   for i.   acc   += values.i     -> out    = sum_i values[i]
// Both are HBM bound (4 bytes per value) and sum in FP64 in a fixed order, so
// the results do not depend on scheduling.
#include <mutex>
#include <unordered_map>

#include "common.h"
#include "internal.h"

namespace dexk {

// G lanes per row (G a power of two, 4 <= G <= 64, chosen so a row is about 8
// values per lane): lane l of a group sums the row's elements 4l, 4l + 4G, ...
// (16-byte loads when rows are aligned, else scalar ones at l, l + G, ...), then
// a fixed butterfly over the group.
template <int G>
__global__ void __launch_bounds__(256) reduce_rows_kernel(const float* __restrict__ v,
                                                          int64_t rows, int64_t cols, bool vec,
                                                          bool accumulate, float* __restrict__ out) {
  const int l = threadIdx.x & (G - 1);
  const int64_t r = ((int64_t)blockIdx.x * 256 + threadIdx.x) / G;
  const bool live = r < rows;
  const float* row = v + (live ? r : 0) * cols;
  double s0 = 0.0, s1 = 0.0;
  if (live) {
    if (vec) {
      int64_t c = 4 * l;
      for (; c + 4 * G < cols; c += 8 * G) {
        const f32x4 a = *reinterpret_cast<const f32x4*>(row + c);
        const f32x4 b = *reinterpret_cast<const f32x4*>(row + c + 4 * G);
        s0 += ((double)a[0] + (double)a[1]) + ((double)a[2] + (double)a[3]);
        s1 += ((double)b[0] + (double)b[1]) + ((double)b[2] + (double)b[3]);
      }
      if (c < cols) {
        const f32x4 a = *reinterpret_cast<const f32x4*>(row + c);
        s0 += ((double)a[0] + (double)a[1]) + ((double)a[2] + (double)a[3]);
      }
    } else {
      for (int64_t c = l; c < cols; c += G) s0 += (double)row[c];
    }
  }
  double s = s0 + s1;
#pragma unroll
  for (int m = 1; m < G; m <<= 1) s += __shfl_xor(s, m, 64);
  if (live && l == 0) out[r] = accumulate ? (float)((double)out[r] + s) : (float)s;
}

// Complete reduction, first pass: block b sums the grid-strided 4-value pieces
// it owns (a fixed set for the fixed grid; the n mod 4 tail goes to block 0),
// two FP64 accumulators per thread.
__global__ void __launch_bounds__(256) reduce_all_partial(const float* __restrict__ v, int64_t n,
                                                          bool vec, double* __restrict__ part) {
  __shared__ double sh[32];
  double s0 = 0.0, s1 = 0.0;
  const int64_t stride = (int64_t)gridDim.x * 256;
  if (vec) {
    const int64_t n4 = n / 4;
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    for (; i + stride < n4; i += 2 * stride) {
      const f32x4 a = reinterpret_cast<const f32x4*>(v)[i];
      const f32x4 b = reinterpret_cast<const f32x4*>(v)[i + stride];
      s0 += ((double)a[0] + (double)a[1]) + ((double)a[2] + (double)a[3]);
      s1 += ((double)b[0] + (double)b[1]) + ((double)b[2] + (double)b[3]);
    }
    if (i < n4) {
      const f32x4 a = reinterpret_cast<const f32x4*>(v)[i];
      s0 += ((double)a[0] + (double)a[1]) + ((double)a[2] + (double)a[3]);
    }
    if (blockIdx.x == 0 && threadIdx.x < (n & 3)) s1 += (double)v[4 * n4 + threadIdx.x];
  } else {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride)
      s0 += (double)v[i];
  }
  double s = block_sum(s0 + s1, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void reduce_all_final(const double* __restrict__ part, int nb, bool accumulate,
                                 float* __restrict__ out) {
  __shared__ double sh[32];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) s += part[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[0] = accumulate ? (float)((double)out[0] + s) : (float)s;
}

}  // namespace dexk

// Scratch of the allocation-free complete reduction: the FP64 block partials,
// in device memory the library itself holds (one copy per GPU, until the
// process ends). On the host `scratch` is only a stand-in symbol, never a
// device address: host code uses the address hipGetSymbolAddress returns for
// the current device, kept per device by reduce_scratch_init.
static __device__ __align__(256) double scratch[dexi::kReduceBlocks];

namespace dexi {
using namespace dexk;

namespace {
std::mutex g_scratch_mu;
std::unordered_map<int, void*> g_scratch;  // device -> address of its `scratch`
}  // namespace

dex_status reduce_scratch_init() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return check_hip(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch.count(dev)) return DEX_OK;
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) return check_hip(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                              "hipGetSymbolAddress(scratch)");
  g_scratch[dev] = p;
  return DEX_OK;
}

dex_status reduce_rows(float* out, const float* values, int64_t rows, int64_t cols,
                       bool accumulate, hipStream_t s) {
  if (rows == 0) return DEX_OK;
  const bool vec = (cols % 4) == 0 && ((uintptr_t)values & 15) == 0;
  int G = 4;  // lanes per row: about 8 values each
  while (G < 64 && 8 * G < cols) G *= 2;
  const unsigned blocks = (unsigned)((rows * G + 255) / 256);
  ProfRange pr(DEX_PROF_REDUCE_ROWS, s);
#define DEX_RR(g)                                                                             \
  case g:                                                                                     \
    hipLaunchKernelGGL((reduce_rows_kernel<g>), dim3(blocks), dim3(256), 0, s, values, rows, \
                       cols, vec, accumulate, out);                                           \
    break;
  switch (G) {
    DEX_RR(4)
    DEX_RR(8)
    DEX_RR(16)
    DEX_RR(32)
    DEX_RR(64)
  }
#undef DEX_RR
  pr.end(1);
  return check_hip(hipGetLastError(), "reduce_rows");
}

dex_status reduce_all(float* out, const float* values, int64_t n, bool accumulate, void* ws,
                      hipStream_t s) {
  double* part = (double*)ws;
  const int nb = kReduceBlocks;
  const bool vec = ((uintptr_t)values & 15) == 0;
  ProfRange pr(DEX_PROF_REDUCE_ALL, s);
  hipLaunchKernelGGL(reduce_all_partial, dim3(nb), dim3(256), 0, s, values, n, vec, part);
  hipLaunchKernelGGL(reduce_all_final, dim3(1), dim3(256), 0, s, (const double*)part, nb,
                     accumulate, out);
  pr.end(1);
  return check_hip(hipGetLastError(), "reduce_all");
}

dex_status reduce_all_noalloc(float* out, const float* values, int64_t n, bool accumulate,
                              hipStream_t s) {
  const dex_status st = reduce_scratch_init();
  if (st != DEX_OK) return st;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return check_hip(e, "hipGetDevice");
  void* p = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    p = g_scratch[dev];
  }
  // every partial is written by the first kernel before the second reads it,
  // so nothing has to be cleared between calls
  return reduce_all(out, values, n, accumulate, p, s);
}

}  // namespace dexi
