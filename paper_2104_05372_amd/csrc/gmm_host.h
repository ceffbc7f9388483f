// Host-side launch interface of the GMM matrix-core kernels; one explicit
// specialisation per operand precision (gmm_mfma_inst.hip is compiled once per
// precision).
#pragma once

#include <hip/hip_runtime.h>

#include "gmm_dev.h"

namespace dexi {

struct GmmGeom {
  int64_t N, D, K, Npad;
  int DP;
};

struct FwdCfg {
  int cb, sk, ck;  // points per wave / 16, k-splits, contraction chunk depth
};
struct BwdCfg {
  int gw, s;  // components per wave, point chunks
};

// Point-chunk length (a multiple of 64) and count for `s` requested chunks.
inline void bwd_chunks(int64_t Npad, int s, int64_t* chunk, int* n) {
  int64_t c = (Npad + s - 1) / s;
  c = (c + 63) / 64 * 64;
  *chunk = c;
  *n = (int)((Npad + c - 1) / c);
}

template <int PREC>
void mfma_prep(const GmmGeom& g, const float* x, const float* alphas, const float* means,
               const float* qd, const float* l, void* xh, void* xl, void* xhT, void* xlT, void* Qh,
               void* Ql, float* negc, float* kappa, hipStream_t st);
template <int PREC>
void mfma_fwd(const GmmGeom& g, const FwdCfg& c, const dexk::MfmaOps& o, float* beta, float2* ml,
              hipStream_t st);
template <int PREC>
void mfma_bwd(const GmmGeom& g, const BwdCfg& c, const dexk::MfmaOps& o, const float* beta,
              const float* f, const float* ct, float* part, hipStream_t st);

template <>
void mfma_prep<dexk::PREC_F32>(const GmmGeom&, const float*, const float*, const float*,
                               const float*, const float*, void*, void*, void*, void*, void*,
                               void*, float*, float*, hipStream_t);
template <>
void mfma_prep<dexk::PREC_BF16>(const GmmGeom&, const float*, const float*, const float*,
                                const float*, const float*, void*, void*, void*, void*, void*,
                                void*, float*, float*, hipStream_t);
template <>
void mfma_prep<dexk::PREC_BF16X3>(const GmmGeom&, const float*, const float*, const float*,
                                  const float*, const float*, void*, void*, void*, void*, void*,
                                  void*, float*, float*, hipStream_t);
template <>
void mfma_fwd<dexk::PREC_F32>(const GmmGeom&, const FwdCfg&, const dexk::MfmaOps&, float*,
                              float2*, hipStream_t);
template <>
void mfma_fwd<dexk::PREC_BF16>(const GmmGeom&, const FwdCfg&, const dexk::MfmaOps&, float*,
                               float2*, hipStream_t);
template <>
void mfma_fwd<dexk::PREC_BF16X3>(const GmmGeom&, const FwdCfg&, const dexk::MfmaOps&, float*,
                                 float2*, hipStream_t);
template <>
void mfma_bwd<dexk::PREC_F32>(const GmmGeom&, const BwdCfg&, const dexk::MfmaOps&, const float*,
                              const float*, const float*, float*, hipStream_t);
template <>
void mfma_bwd<dexk::PREC_BF16>(const GmmGeom&, const BwdCfg&, const dexk::MfmaOps&, const float*,
                               const float*, const float*, float*, hipStream_t);
template <>
void mfma_bwd<dexk::PREC_BF16X3>(const GmmGeom&, const BwdCfg&, const dexk::MfmaOps&,
                                 const float*, const float*, const float*, float*, hipStream_t);

}  // namespace dexi
