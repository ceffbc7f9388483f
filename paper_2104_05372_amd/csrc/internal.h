// Host-side interfaces between the C ABI layer (abi.cpp) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "../../include/dex.h"

namespace dexi {

// Record a failure for dex_last_error() and return its status.
dex_status fail(dex_status st, const char* fmt, ...);
// Map a HIP error (after a launch or runtime call) to DEX_ERR_HIP.
dex_status check_hip(hipError_t e, const char* what);
// Round up to a multiple of 256 bytes.
inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
// Number of compute units on the current device (cached).
int num_cus();

// Live timing of the main kernels (dex_profile_*): a range covers `launches`
// kernel launches enqueued between prof_begin and prof_end on stream s.
struct ProfRange {
  int id;
  hipEvent_t e0 = nullptr;
  hipStream_t s;
  ProfRange(int id_, hipStream_t s_);
  void end(int64_t launches);
};

// ---------------------------------------------------------------- GMM -----
struct GmmPtrs {
  const void *alphas, *means, *qd, *l, *x;
};
struct GmmGrads {
  void *d_alphas, *d_means, *d_qd, *d_l;
};

size_t gmm_cache_bytes(const dex_desc& d);
size_t gmm_ws_bytes(const dex_desc& d, int role);
int gmm_num_configs(const dex_desc& d, int role);
dex_status gmm_fwd(const dex_desc& d, int cfg, const GmmPtrs& in, void* F, void* f,
                   void* cache, void* ws, hipStream_t s);
// Forward mode of the scalar objective: the linearized loop run forward over
// the tangents (matrix-core tangent products for the 16-bit variant at D = 64,
// a vector-ALU pass otherwise), FP64 fixed-order sums.
dex_status gmm_jvp(const dex_desc& d, int cfg, const GmmPtrs& in, const void* f,
                   const void* cache, const GmmGrads& t, void* dF, void* ws, hipStream_t st);
dex_status gmm_vjp(const dex_desc& d, int cfg, const GmmPtrs& in, const void* f,
                   const void* cache, const void* ct, const GmmGrads& out, bool accumulate,
                   void* ws, hipStream_t s);

// ------------------------------------------------------- batched GMM -----
size_t gmm_batched_plan_bytes(int64_t B, const int64_t* shapes, int32_t variant);
dex_status gmm_batched_plan(const int64_t* shapes, int64_t B, int32_t variant, dex_desc* d,
                            void* plan, size_t plan_bytes);
size_t gmm_batched_ws_bytes(const dex_desc& d, int role);
int gmm_batched_num_configs(const dex_desc& d, int role);
dex_status gmm_batched_fwd(const dex_desc& d, int cfg, const void* plan, const GmmPtrs& in,
                           void* F, void* f, void* cache, void* ws, hipStream_t s);
dex_status gmm_batched_vjp(const dex_desc& d, int cfg, const void* plan, const GmmPtrs& in,
                           const void* f, const void* cache, const void* ct, const GmmGrads& out,
                           bool accumulate, void* ws, hipStream_t s);

// ------------------------------------------------ scatter / gather -----
size_t scatter_ws_bytes(int32_t acc_dtype, int64_t n_rows, int64_t row_len, int64_t n,
                        bool has_vals, bool deterministic);
// path: kScatterAtomic (block sort + run sums + atomics, no workspace) or
// kScatterSorted (radix sort + one owner per row, deterministic, workspace).
// overwrite (sorted path): acc was cleared by the caller and untouched rows stay
// zero, so a row's owner stores its sum without reading the row.
constexpr int kScatterAtomic = 0, kScatterSorted = 1;
dex_status accum_scatter(void* acc, int32_t acc_dtype, int64_t n_rows, int64_t row_len,
                         const void* idx, int32_t idx_dtype, const void* vals,
                         const float* scale, int64_t n, bool count_oob, int64_t* oob,
                         void* ws, size_t ws_bytes, int path, hipStream_t s,
                         bool overwrite = false);
dex_status gather_fwd(const float* T, const int32_t* idx, const float* w, int64_t V, int64_t R,
                      int64_t n, float* out, bool count_oob, int64_t* oob, hipStream_t s);
dex_status gather_jvp(const float* T, const float* tT, const int32_t* idx, const float* w,
                      const float* tw, int64_t V, int64_t R, int64_t n, float* tout,
                      hipStream_t s);
dex_status gather_dw(const float* T, const int32_t* idx, const float* g, int64_t V, int64_t R,
                     int64_t n, float* dw, bool accumulate, hipStream_t s);
dex_status fill_zero(void* p, size_t bytes, hipStream_t s);

// ------------------------------------------------------- reductions -----
constexpr int kReduceBlocks = 1024;  // complete reduction: partials (FP64) per call
dex_status reduce_rows(float* out, const float* values, int64_t rows, int64_t cols,
                       bool accumulate, hipStream_t s);
dex_status reduce_all(float* out, const float* values, int64_t n, bool accumulate, void* ws,
                      hipStream_t s);
// The allocation-free complete reduction: partials in the library's own
// per-GPU device array, whose address reduce_scratch_init looks up once per
// device (called from device set-up).
dex_status reduce_scratch_init();
dex_status reduce_all_noalloc(float* out, const float* values, int64_t n, bool accumulate,
                              hipStream_t s);

// ----------------------------------------------------------- stencil -----
dex_status stencil_jvp(const dex_desc& d, const float* u0, const float* target, const float* du0,
                       const float* dtarget, float* tL, void* ws, hipStream_t st);
size_t stencil_ws_bytes(const dex_desc& d, int role);
int stencil_num_configs(const dex_desc& d, int role);
dex_status stencil_fwd(const dex_desc& d, int cfg, const float* u0, const float* target,
                       float* L, float* uT, float* ckpt, void* ws, hipStream_t s);
dex_status stencil_vjp(const dex_desc& d, int cfg, const float* u0, const float* target,
                       const float* ckpt, const float* uT_in, const float* dL, float* du0,
                       bool accumulate, void* ws, hipStream_t s);

}  // namespace dexi
