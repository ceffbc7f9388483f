// Host-side launch interface of the GMM matrix-core kernels; one explicit
// specialisation per operand precision (gmm_mfma_inst.hip is compiled once per
// precision).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "gmm_dev.h"

namespace dexi {

struct GmmGeom {
  int64_t N, D, K, Npad;
  int DP;
};

// wps: waves per SIMD to launch (0: as many as can be resident).
struct FwdCfg {
  int nkq, wps, pd;  // components resident per wave (2 or 4; 4 for BF16 only; 0: the
                     // feature-product form), waves (blocks for nkq = 0) per SIMD (CU),
                     // x~ tiles loaded ahead (1 or 2)
};
struct BwdCfg {
  int gw, wps;  // components per wave, waves per SIMD
  int db = 1;   // FP16 form: scaled rows double-buffered (more registers)
};

// The single-instance forward and reverse kernels split their work evenly
// over the waves of each XCD (split_lo). Forward units are (group of nkq
// components, 16-point tile); each group leaves one log-sum-exp partial per
// point (sk = number of groups). Reverse units are (group of gw components,
// 32-point step); XCD x owns the x-th eighth of the steps, W waves each, and
// a wave writes one moment partial per group it touches, in the slots
// x * T + rank (T = slots per XCD).
struct FlatSplit {
  int64_t T;
  int W;
  int sk;  // forward
  int gw;  // reverse
  int64_t nsteps;
};

// Waves a launch may use at most (256 CUs x 4 SIMDs x 8 waves).
constexpr int kMaxWaves = 8192;

// Forward log-sum-exp partials per point: one per group of >= 2 components.
inline int64_t fwd_max_slots(int64_t K) { return (K + 1) / 2; }
// beta rows: K rounded up to whole passes of 32 components (the padding rows
// take the stores of the padding components of the last group or pass)
inline int64_t beta_rows(int64_t K) { return (K + 31) / 32 * 32; }
// Reverse partial slots per component over the 8 XCDs (a multiple of 8, at
// least 2 per XCD); the launch keeps each XCD's waves within its share.
inline int64_t bwd_max_slots(int64_t Npad, int64_t K) {
  (void)Npad;
  return std::max<int64_t>(16, 9600 / K / 8 * 8);
}

template <int PREC>
void mfma_prep(const GmmGeom& g, const float* x, const float* alphas, const float* means,
               const float* qd, const float* l, void* xh, void* xl, void* xhT, void* xlT, void* Qh,
               void* Ql, float* negc, float* kappa, float* shift, hipStream_t st);
template <int PREC>
FlatSplit mfma_fwd(const GmmGeom& g, const FwdCfg& c, const dexk::MfmaOps& o, float* beta,
                   float2* ml, hipStream_t st);
template <int PREC>
FlatSplit mfma_bwd(const GmmGeom& g, const BwdCfg& c, const dexk::MfmaOps& o, const float* beta,
                   const float* f, const float* ct, float* part, hipStream_t st);

// Feature-product forward (BF16 variant, D = 64; defined with the BF16 kernels).
// qf_prep: the origin (shift), x~^T, the per-tile scaled FP16 copy of x and
// its exponents, the coefficient operand, kappa' and rescale factors. qf_fwd: beta and the per-pass
// log-sum-exp partials (FlatSplit::sk passes; W holds the block count).
void qf_prep(const GmmGeom& g, const float* x, const float* alphas, const float* means,
             const float* qd, const float* l, void* xhT, void* x16, int* tile_exp, void* W16,
             float* kq, float* isc, float* shift, hipStream_t st);
FlatSplit qf_fwd(const GmmGeom& g, const FwdCfg& c, const void* x16, const void* W16,
                 const float* kq, const float* isc, const int* tile_exp, float* beta, float2* ml,
                 hipStream_t st);
inline bool qf_eligible(const GmmGeom& g, int prec) { return prec == dexk::PREC_BF16 && g.D == 64; }
// Forward mode of the feature-product form: qf_tan_prep writes the scaled FP16
// copy of x~ (about the forward's origin `shift`), its tile exponents and the
// tangent coefficient operand with dkq' and its rescale factors; qf_jvp writes
// one FP64 partial of sum_{i,k} exp(beta_ik - f_i) dbeta_ik per (pass, 64-point
// tile), qf_tan_parts(g) of them.
void qf_tan_prep(const GmmGeom& g, const float* x, const float* means, const float* qd,
                 const float* l, const float* da, const float* dm, const float* dq,
                 const float* dl, const float* shift, void* x16, int* tile_exp, void* dW16,
                 float* dkq, float* disc, hipStream_t st);
int64_t qf_tan_parts(const GmmGeom& g);
void qf_jvp(const GmmGeom& g, const void* x16, const void* dW16, const float* dkq,
            const float* disc, const int* tile_exp, const float* beta, const float* f,
            double* part, hipStream_t st);

template <>
void mfma_prep<dexk::PREC_F32>(const GmmGeom&, const float*, const float*, const float*,
                               const float*, const float*, void*, void*, void*, void*, void*,
                               void*, float*, float*, float*, hipStream_t);
template <>
void mfma_prep<dexk::PREC_BF16>(const GmmGeom&, const float*, const float*, const float*,
                                const float*, const float*, void*, void*, void*, void*, void*,
                                void*, float*, float*, float*, hipStream_t);
template <>
void mfma_prep<dexk::PREC_BF16X3>(const GmmGeom&, const float*, const float*, const float*,
                                  const float*, const float*, void*, void*, void*, void*, void*,
                                  void*, float*, float*, float*, hipStream_t);
template <>
FlatSplit mfma_fwd<dexk::PREC_F32>(const GmmGeom&, const FwdCfg&, const dexk::MfmaOps&, float*,
                              float2*, hipStream_t);
template <>
FlatSplit mfma_fwd<dexk::PREC_BF16>(const GmmGeom&, const FwdCfg&, const dexk::MfmaOps&, float*,
                               float2*, hipStream_t);
template <>
FlatSplit mfma_fwd<dexk::PREC_BF16X3>(const GmmGeom&, const FwdCfg&, const dexk::MfmaOps&, float*,
                                 float2*, hipStream_t);
template <>
FlatSplit mfma_bwd<dexk::PREC_F32>(const GmmGeom&, const BwdCfg&, const dexk::MfmaOps&, const float*,
                              const float*, const float*, float*, hipStream_t);
template <>
FlatSplit mfma_bwd<dexk::PREC_BF16>(const GmmGeom&, const BwdCfg&, const dexk::MfmaOps&, const float*,
                               const float*, const float*, float*, hipStream_t);
template <>
FlatSplit mfma_bwd<dexk::PREC_BF16X3>(const GmmGeom&, const BwdCfg&, const dexk::MfmaOps&,
                                 const float*, const float*, const float*, float*, hipStream_t);

}  // namespace dexi
