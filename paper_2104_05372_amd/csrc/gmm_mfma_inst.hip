// Grid kernels of the single-instance GMM matrix-core path for one operand
// precision, selected at compile time by DEX_PREC (0 FP32, 1 BF16, 2 split-BF16).
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

template <int DP, int PREC, int CB, int CK>
__global__ void __launch_bounds__(256) k_gmm_fwd(MfmaOps ops, int N, int Npad, int K, int kchunk,
                                                 float* __restrict__ beta, float2* __restrict__ ml) {
  const int k0 = blockIdx.y * kchunk, k1 = min(K, k0 + kchunk);
  fwd_unit<DP, PREC, CB, CK>(ops, N, Npad, blockIdx.x * 64 * CB, k0, k1, beta,
                             ml + (size_t)blockIdx.y * Npad);
}

template <int DP, int PREC, int GW>
__global__ void __launch_bounds__(256) k_gmm_bwd(MfmaOps ops, int N, int Npad, int K, int chunk,
                                                 const float* __restrict__ beta,
                                                 const float* __restrict__ f,
                                                 const float* __restrict__ ct,
                                                 float* __restrict__ part) {
  const int pbeg = blockIdx.y * chunk, pend = min(Npad, pbeg + chunk);
  const size_t E = mom_slot(DP);
  bwd_mom_unit<DP, MomOf<PREC>::MP, GW>(ops.xhT, ops.xlT, N, Npad, K, blockIdx.x * 4 * GW, pbeg,
                                        pend, beta, f, ct[0], part + (size_t)blockIdx.y * K * E, E);
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

template <int DP, int CB, int CK>
static void fwd_launch(const GmmGeom& g, const FwdCfg& c, const MfmaOps& o, float* beta, float2* ml,
                       hipStream_t st) {
  const int kchunk = (int)((g.K + c.sk - 1) / c.sk);
  dim3 grid((unsigned)(g.Npad / (64 * CB)), (unsigned)c.sk);
  hipLaunchKernelGGL((k_gmm_fwd<DP, P, CB, CK>), grid, dim3(256), 0, st, o, (int)g.N, (int)g.Npad,
                     (int)g.K, kchunk, beta, ml);
}

template <int DP>
static void fwd_dp(const GmmGeom& g, const FwdCfg& c, const MfmaOps& o, float* beta, float2* ml,
                   hipStream_t st) {
  const int ck = DP == 16 ? 16 : c.ck;
  if (c.cb == 4) {
    if (ck == 32) fwd_launch<DP, 4, (DP >= 32 ? 32 : 16)>(g, c, o, beta, ml, st);
    else fwd_launch<DP, 4, 16>(g, c, o, beta, ml, st);
  } else {
    if (ck == 32) fwd_launch<DP, 2, (DP >= 32 ? 32 : 16)>(g, c, o, beta, ml, st);
    else fwd_launch<DP, 2, 16>(g, c, o, beta, ml, st);
  }
}

template <>
void mfma_fwd<P>(const GmmGeom& g, const FwdCfg& c, const MfmaOps& o, float* beta, float2* ml,
                 hipStream_t st) {
  if (g.DP == 16)
    fwd_dp<16>(g, c, o, beta, ml, st);
  else if (g.DP == 32)
    fwd_dp<32>(g, c, o, beta, ml, st);
  else
    fwd_dp<64>(g, c, o, beta, ml, st);
}

template <int DP, int GW>
static void bwd_launch(const GmmGeom& g, const BwdCfg& c, const MfmaOps& o, const float* beta,
                       const float* f, const float* ct, float* part, hipStream_t st) {
  int64_t chunk;
  int n;
  bwd_chunks(g.Npad, c.s, &chunk, &n);
  dim3 grid((unsigned)((g.K + 4 * GW - 1) / (4 * GW)), (unsigned)n);
  hipLaunchKernelGGL((k_gmm_bwd<DP, P, GW>), grid, dim3(256), 0, st, o, (int)g.N, (int)g.Npad,
                     (int)g.K, (int)chunk, beta, f, ct, part);
}

template <int DP>
static void bwd_dp(const GmmGeom& g, const BwdCfg& c, const MfmaOps& o, const float* beta,
                   const float* f, const float* ct, float* part, hipStream_t st) {
  if (c.gw == 4)
    bwd_launch<DP, 4>(g, c, o, beta, f, ct, part, st);
  else if (c.gw == 2)
    bwd_launch<DP, 2>(g, c, o, beta, f, ct, part, st);
  else
    bwd_launch<DP, 1>(g, c, o, beta, f, ct, part, st);
}

template <>
void mfma_bwd<P>(const GmmGeom& g, const BwdCfg& c, const MfmaOps& o, const float* beta,
                 const float* f, const float* ct, float* part, hipStream_t st) {
  if (g.DP == 16)
    bwd_dp<16>(g, c, o, beta, f, ct, part, st);
  else if (g.DP == 32)
    bwd_dp<32>(g, c, o, beta, f, ct, part, st);
  else
    bwd_dp<64>(g, c, o, beta, f, ct, part, st);
}

}  // namespace dexi
