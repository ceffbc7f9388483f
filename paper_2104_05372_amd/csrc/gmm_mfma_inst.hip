// Grid kernels of the single-instance GMM matrix-core path for one operand
// precision, selected at compile time by DEX_PREC (0 FP32, 1 BF16, 2 split-BF16).
#include <algorithm>

#include "gmm_host.h"
#include "internal.h"

#ifndef DEX_PREC
#error "compile with -DDEX_PREC=0|1|2"
#endif

namespace dexk {

template <int PREC, int DP>
__global__ void __launch_bounds__(256) k_prep_x(const float* __restrict__ x, int N, int D, int Npad,
                                                typename Store<PREC>::S* xh,
                                                typename Store<PREC>::S* xl,
                                                typename MomT<MomOf<PREC>::MP>::S* xhT,
                                                typename MomT<MomOf<PREC>::MP>::S* xlT) {
  prep_x_tile<PREC, DP>(x, N, D, Npad, blockIdx.x * 64, xh, xl, xhT, xlT);
}

template <int PREC, int DP>
__global__ void __launch_bounds__(256) k_prep_q(const float* __restrict__ alphas,
                                                const float* __restrict__ means,
                                                const float* __restrict__ qd,
                                                const float* __restrict__ l, int D,
                                                typename Store<PREC>::S* Qh,
                                                typename Store<PREC>::S* Ql, float* negc,
                                                float* kappa) {
  prep_q_comp<PREC, DP>(alphas, means, qd, l, D, blockIdx.x, Qh, Ql, negc, kappa);
}

// Both grid kernels split their work evenly over W waves (split_lo), so every
// wave does the same amount of work whatever N, K and the CU count are, and no
// partly filled second wave of blocks trails the launch. Forward units are
// (group of NKQ components, 16-point tile), group-major: a wave loads a
// group's operands once and streams its tiles; its range covers at most a few
// groups.
template <int DP, int PREC, int NKQ, int CK, int PD>
__global__ void __launch_bounds__(256) k_gmm_fwd(MfmaOps ops, int Npad, int K, int64_t T, int W,
                                                 float* __restrict__ beta,
                                                 float2* __restrict__ ml) {
  // wave index, made explicitly uniform so the split arithmetic and the loop
  // control stay in scalar registers
  const int w = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (w >= W) return;
  const int64_t ntiles = Npad / 16;
  int64_t pos = split_lo(w, T, W);
  const int64_t hi = split_lo(w + 1, T, W);
  while (pos < hi) {
    const int64_t grp = pos / ntiles;
    const int64_t ta = pos - grp * ntiles;
    const int64_t tb = min<int64_t>(ntiles, ta + (hi - pos));
    fwd_unit_kq<DP, PREC, NKQ, CK, PD>(ops, Npad, K, (int)grp * NKQ, (int)ta, (int)tb, beta,
                                   ml + (size_t)grp * Npad);
    pos += tb - ta;
  }
}

// Reverse units are (group of GW components, 32-point step), group-major; for
// each group it touches a wave writes one partial moment slot.
template <int DP, int PREC, int GW>
__global__ void __launch_bounds__(256) k_gmm_bwd(MfmaOps ops, int N, int Npad, int K, int64_t T,
                                                 int W, const float* __restrict__ beta,
                                                 const float* __restrict__ f,
                                                 const float* __restrict__ ct,
                                                 float* __restrict__ part) {
  // wave index, made explicitly uniform so the split arithmetic and the loop
  // control stay in scalar registers
  const int w = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (w >= W) return;
  const size_t E = mom_slot(DP);
  const int64_t nsteps = Npad / 32;
  int64_t pos = split_lo(w, T, W);
  const int64_t hi = split_lo(w + 1, T, W);
  while (pos < hi) {
    const int64_t kg = pos / nsteps;
    const int64_t s0 = pos - kg * nsteps;
    const int64_t s1 = min<int64_t>(nsteps, s0 + (hi - pos));
    const int slot = (int)(w - split_owner(kg * nsteps, T, W));
    bwd_mom_unit<DP, MomOf<PREC>::MP, GW>(ops.xhT, ops.xlT, N, Npad, K, (int)kg * GW,
                                          (int)(s0 * 32), (int)(s1 * 32), beta, f, ct[0],
                                          part + (size_t)slot * K * E, E);
    pos += s1 - s0;
  }
}

}  // namespace dexk

namespace dexi {
using namespace dexk;

constexpr int P = DEX_PREC;
using S = typename Store<P>::S;
using SM = typename MomT<MomOf<P>::MP>::S;

template <int DP>
static void prep_dp(const GmmGeom& g, const float* x, const float* alphas, const float* means,
                    const float* qd, const float* l, void* xh, void* xl, void* xhT, void* xlT,
                    void* Qh, void* Ql, float* negc, float* kappa, hipStream_t st) {
  hipLaunchKernelGGL((k_prep_x<P, DP>), dim3((unsigned)(g.Npad / 64)), dim3(256), 0, st, x, (int)g.N,
                     (int)g.D, (int)g.Npad, (S*)xh, (S*)xl, (SM*)xhT, (SM*)xlT);
  hipLaunchKernelGGL((k_prep_q<P, DP>), dim3((unsigned)g.K), dim3(256), 0, st, alphas, means, qd, l,
                     (int)g.D, (S*)Qh, (S*)Ql, negc, kappa);
}

template <>
void mfma_prep<P>(const GmmGeom& g, const float* x, const float* alphas, const float* means,
                  const float* qd, const float* l, void* xh, void* xl, void* xhT, void* xlT,
                  void* Qh, void* Ql, float* negc, float* kappa, hipStream_t st) {
  if (g.DP == 16)
    prep_dp<16>(g, x, alphas, means, qd, l, xh, xl, xhT, xlT, Qh, Ql, negc, kappa, st);
  else if (g.DP == 32)
    prep_dp<32>(g, x, alphas, means, qd, l, xh, xl, xhT, xlT, Qh, Ql, negc, kappa, st);
  else
    prep_dp<64>(g, x, alphas, means, qd, l, xh, xl, xhT, xlT, Qh, Ql, negc, kappa, st);
}

// Resident 256-thread blocks of `kernel` per CU.
template <typename Kern>
static int blocks_per_cu(Kern kernel) {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kernel, 256, 0) != hipSuccess ||
      blocks < 1)
    blocks = 1;
  return blocks;
}

// Waves to launch: all that can be resident (one block puts one wave on each
// SIMD of a CU), capped by wps waves per SIMD when wps > 0.
static int launch_waves(int bpc, int wps) {
  int w = bpc * 4;
  if (wps > 0) w = std::min(w, 4 * wps);
  return std::min(kMaxWaves, w * num_cus());
}

template <int DP, int NKQ, int CK, int PD>
static FlatSplit fwd_launch(const GmmGeom& g, const FwdCfg& c, const MfmaOps& o, float* beta,
                            float2* ml, hipStream_t st) {
  static const int bpc = blocks_per_cu(k_gmm_fwd<DP, P, NKQ, CK, PD>);
  FlatSplit sp{};
  sp.sk = (int)((g.K + NKQ - 1) / NKQ);
  sp.T = (int64_t)sp.sk * (g.Npad / 16);
  sp.W = (int)std::min<int64_t>(sp.T, launch_waves(bpc, c.wps));
  hipLaunchKernelGGL((k_gmm_fwd<DP, P, NKQ, CK, PD>), dim3((unsigned)((sp.W + 3) / 4)), dim3(256),
                     0, st, o, (int)g.Npad, (int)g.K, sp.T, sp.W, beta, ml);
  return sp;
}

// operand chunk depth: 32 for the 16-bit products when DP >= 32, else 16
template <int DP>
static FlatSplit fwd_dp(const GmmGeom& g, const FwdCfg& c, const MfmaOps& o, float* beta,
                        float2* ml, hipStream_t st) {
  constexpr int CK = (P != PREC_F32 && DP >= 32) ? 32 : 16;
  if constexpr (P == PREC_BF16) {
    if (c.nkq == 4)
      return c.pd == 2 ? fwd_launch<DP, 4, CK, 2>(g, c, o, beta, ml, st)
                       : fwd_launch<DP, 4, CK, 1>(g, c, o, beta, ml, st);
  }
  return c.pd == 2 ? fwd_launch<DP, 2, CK, 2>(g, c, o, beta, ml, st)
                   : fwd_launch<DP, 2, CK, 1>(g, c, o, beta, ml, st);
}

template <>
FlatSplit mfma_fwd<P>(const GmmGeom& g, const FwdCfg& c, const MfmaOps& o, float* beta,
                      float2* ml, hipStream_t st) {
  if (g.DP == 16) return fwd_dp<16>(g, c, o, beta, ml, st);
  if (g.DP == 32) return fwd_dp<32>(g, c, o, beta, ml, st);
  return fwd_dp<64>(g, c, o, beta, ml, st);
}

template <int DP, int GW>
static FlatSplit bwd_launch(const GmmGeom& g, const BwdCfg& c, const MfmaOps& o, const float* beta,
                            const float* f, const float* ct, float* part, hipStream_t st) {
  FlatSplit sp{};
  sp.gw = GW;
  sp.nsteps = g.Npad / 32;
  const int64_t groups = (g.K + GW - 1) / GW;
  sp.T = groups * sp.nsteps;
  // at most bwd_max_slots partial slots per group: W <= (slots - 1) * groups
  const int64_t wcap = (bwd_max_slots(g.Npad, g.K) - 1) * groups;
  static const int bpc = blocks_per_cu(k_gmm_bwd<DP, P, GW>);
  sp.W = (int)std::min<int64_t>(std::min<int64_t>(sp.T, wcap), launch_waves(bpc, c.wps));
  hipLaunchKernelGGL((k_gmm_bwd<DP, P, GW>), dim3((unsigned)((sp.W + 3) / 4)), dim3(256), 0, st, o,
                     (int)g.N, (int)g.Npad, (int)g.K, sp.T, sp.W, beta, f, ct, part);
  return sp;
}

template <int DP>
static FlatSplit bwd_dp(const GmmGeom& g, const BwdCfg& c, const MfmaOps& o, const float* beta,
                        const float* f, const float* ct, float* part, hipStream_t st) {
  if (c.gw == 4) return bwd_launch<DP, 4>(g, c, o, beta, f, ct, part, st);
  if (c.gw == 2) return bwd_launch<DP, 2>(g, c, o, beta, f, ct, part, st);
  return bwd_launch<DP, 1>(g, c, o, beta, f, ct, part, st);
}

template <>
FlatSplit mfma_bwd<P>(const GmmGeom& g, const BwdCfg& c, const MfmaOps& o, const float* beta,
                      const float* f, const float* ct, float* part, hipStream_t st) {
  if (g.DP == 16) return bwd_dp<16>(g, c, o, beta, f, ct, part, st);
  if (g.DP == 32) return bwd_dp<32>(g, c, o, beta, f, ct, part, st);
  return bwd_dp<64>(g, c, o, beta, f, ct, part, st);
}

}  // namespace dexi
