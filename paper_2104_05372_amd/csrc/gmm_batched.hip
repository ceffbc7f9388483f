// Many independent GMM instances of uneven size, FP32 matrix-core form.
//
// The nested parallel loop `for b. for i k. ...` is flattened into work items
// (Sec. 6.1.1: parallelism is allocated at the top level only). A host-side
// plan lists, per phase, the items (instance, point block[, component group])
// ordered longest first; the forward and reverse phases each run as one
// persistent launch whose blocks take items from an atomic counter until the
// list is exhausted, so the smallest instances do not pay a launch each.
// Tiles: 16-deep contraction chunks (D = 9..16 padded to 16, 17..32 to 32);
// D <= 8 runs on the vector units.
#include <string.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "gmm_host.h"
#include "internal.h"

namespace dexk {

struct BInst {
  int32_t N, D, K, DP;
  int64_t Npad;
  int64_t a_off, m_off, l_off, x_off, f_off;       // packed inputs / f (elements)
  int64_t xh_off, xhT_off, Q_off, negc_off, kappa_off, beta_off;  // cache (bytes)
  int64_t ml_off;     // ws float2 elements
  int64_t fpart_off;  // ws float pairs
  int64_t part_off;   // ws floats
  int32_t nblk;       // Npad / 256
  int32_t split;      // forward operands in split FP16 (variant DEX_GMM_F16X3, D > 8)
  int64_t xl_off, ts_off, Ql_off;  // cache (bytes): split form: low parts, per-tile x scales
  int64_t sh_off;     // cache (bytes): origin shift[DP], the factor scale, max |mu - shift|
};

struct BItem {
  int32_t inst, a, b, c;
};

constexpr int kBFwdCfgs = 2;
constexpr int kBBwdCfgs = 4;
struct BBwd {
  int gw;
  int64_t chunk;
};
__host__ __device__ inline BBwd bbwd_cfg(int i) {
  const BBwd t[kBBwdCfgs] = {{2, 4096}, {1, 4096}, {2, 2048}, {4, 8192}};
  return t[i];
}
__host__ __device__ inline int bfwd_cb(int i) { return i == 0 ? 4 : 2; }

struct PlanHeader {
  int64_t B;
  int64_t inst_off;
  int64_t prepx_off, n_prepx;
  int64_t prepq_off, n_prepq;
  int64_t merge_off, n_merge;
  int64_t fwd_off[kBFwdCfgs], n_fwd[kBFwdCfgs];
  int64_t bwd_off[kBBwdCfgs], n_bwd[kBBwdCfgs];
  int64_t nch_off;  // int32 [kBBwdCfgs][B]: point chunks per instance
  int64_t cache_bytes, ws_bytes;
  int64_t ws_ml, ws_fpart, ws_counter, ws_part;  // byte offsets into ws
};

__device__ inline const PlanHeader* hdr(const char* plan) { return (const PlanHeader*)plan; }

__device__ inline MfmaOps bops(const BInst& I, const char* cache) {
  MfmaOps o;
  o.xh = cache + I.xh_off;
  o.xl = I.split ? cache + I.xl_off : nullptr;
  o.xhT = cache + I.xhT_off;
  o.xlT = nullptr;
  o.Qh = cache + I.Q_off;
  o.Ql = I.split ? cache + I.Ql_off : nullptr;
  o.negc = (const float*)(cache + I.negc_off);
  o.kappa = (const float*)(cache + I.kappa_off);
  return o;
}

// ---------------------------------------------------------------------------
// D <= 8: the 16x16 matrix-core tiles would be mostly padding, so these
// instances run on the vector units. Q~, -c~ and kappa come from the same
// operand cache (DP = 16, row-major, zero padded).
//
// Forward. The block's npts points are split in two halves and its 256 lanes
// in G = 512 / npts component groups: a lane takes points pi and pi + npts/2
// for the components of its group (one group per wave). Each component's
// triangular factor, offset and constant are staged in LDS, 64 components at a
// time, and read back as wave-wide broadcasts; the groups' running
// log-sum-exps are merged through LDS at the end. All 256 lanes must call it.
template <int DV>
DEX_DEV void fwd_unit_valu(const MfmaOps& o, int N, int Npad, int p0blk, int npts, int K,
                           float* __restrict__ beta, float2* __restrict__ ml) {
  constexpr int NQ = DV * (DV + 1) / 2;  // lower-triangular entries of Q~
  constexpr int CW = 64;                 // floats per staged component
  constexpr int KS = 64;                 // components staged at a time
  constexpr int NT = (NQ + DV + 1 + 3) / 4;  // float4 reads per component
  static_assert(NQ + DV + 1 <= CW, "staged component does not fit");
  __shared__ __attribute__((aligned(16))) float tab[KS * CW];
  __shared__ float2 mls[512];
  (void)N;
  const float* xh = (const float*)o.xh;
  const float* Q = (const float*)o.Qh;
  const int tid = (int)threadIdx.x;
  const int half = npts >> 1, G = 256 / half, JC = KS / G;
  const int pi = tid % half, g = tid / half;
  const int Kg = (K + G - 1) / G;
  const int pa = p0blk + pi, pb = pa + half;
  float xa[DV], xb[DV];
#pragma unroll
  for (int b = 0; b < DV; ++b) {
    xa[b] = xh[(size_t)pa * 16 + b];
    xb[b] = xh[(size_t)pb * 16 + b];
  }
  // this lane stages entry r of components tid / CW + 4 i: its source is
  // base[k * stride] (Q~ row entry, -c~ entry or kappa), or zero padding
  const int r = tid % CW;
  const float* base = nullptr;
  int stride = 0;
  if (r < NQ) {
    int a = 0, e = r;
    while (e > a) {
      e -= a + 1;
      ++a;
    }
    base = Q + a * 16 + e;
    stride = 256;
  } else if (r < NQ + DV) {
    base = o.negc + (r - NQ);
    stride = 16;
  } else if (r == NQ + DV) {
    base = o.kappa;
    stride = 1;
  }
  constexpr int SV = KS * CW / 256;  // staged values per lane
  float sv[SV];
  // the global loads of a stage are issued one stage ahead of its use
  auto stage_load = [&](int j0) {
#pragma unroll
    for (int i = 0; i < SV; ++i) {
      const int slot = tid / CW + (256 / CW) * i;
      const int j = j0 + slot % JC, k = (slot / JC) * Kg + j;
      sv[i] = (base && j < Kg && k < K) ? base[(size_t)k * stride] : 0.f;
    }
  };
  stage_load(0);
  float ma = -INFINITY, la = 0.f, mb = -INFINITY, lb = 0.f;
  // running log-sum-exp: one exponential of -|bv - m| serves both cases
  auto lse = [](float& m, float& l, float bv) {
    const float d = bv - m;
    const float ex = __expf(-fabsf(d));
    l = d > 0.f ? fmaf(l, ex, 1.f) : l + ex;
    m = fmaxf(m, bv);
  };
  for (int j0 = 0; j0 < Kg; j0 += JC) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < SV; ++i) tab[(tid / CW + (256 / CW) * i) * CW + r] = sv[i];
    __syncthreads();
    if (j0 + JC < Kg) stage_load(j0 + JC);
    const int jn = std::min(JC, Kg - j0);
    for (int jj = 0; jj < jn; ++jj) {
      const int k = g * Kg + j0 + jj;
      if (k >= K) break;  // the same for the whole wave
      const float4* T4 = (const float4*)(tab + (g * JC + jj) * CW);
      float t[4 * NT];
#pragma unroll
      for (int i = 0; i < NT; ++i) {
        const float4 v = T4[i];
        t[4 * i] = v.x;
        t[4 * i + 1] = v.y;
        t[4 * i + 2] = v.z;
        t[4 * i + 3] = v.w;
      }
      float sa = 0.f, sb = 0.f;
      int e = 0;
#pragma unroll
      for (int a = 0; a < DV; ++a) {
        float ya = t[NQ + a], yb = t[NQ + a];
#pragma unroll
        for (int b = 0; b <= a; ++b) {
          ya = fmaf(t[e], xa[b], ya);
          yb = fmaf(t[e], xb[b], yb);
          ++e;
        }
        sa = fmaf(ya, ya, sa);
        sb = fmaf(yb, yb, sb);
      }
      const float kap = t[NQ + DV];
      const float ba = kap - 0.5f * sa, bb = kap - 0.5f * sb;
      // padded points (N <= p < Npad) get a value too; nothing reads it
      beta[(size_t)k * Npad + pa] = ba;
      beta[(size_t)k * Npad + pb] = bb;
      lse(ma, la, ba);
      lse(mb, lb, bb);
    }
  }
  mls[g * npts + pi] = make_float2(ma, la);
  mls[g * npts + pi + half] = make_float2(mb, lb);
  __syncthreads();
  if (tid < npts) {
    float m = -INFINITY;
    for (int gg = 0; gg < G; ++gg) m = fmaxf(m, mls[gg * npts + tid].x);
    float l = 0.f;
    for (int gg = 0; gg < G; ++gg) {
      const float2 v = mls[gg * npts + tid];
      l += v.y * __expf(v.x - m);
    }
    ml[p0blk + tid] = make_float2(m, l);
  }
}

// Reverse for D <= 8: wave wv accumulates, per component, the lane-private sums
// of w x_a x_b (a >= b), w x_a and w over the points [pbeg, pend), reduces them
// across the wave and writes them in the partial-slot layout of bwd_mom_unit
// (DP = 16, one 16x16 block).
template <int DV, int GW>
DEX_DEV void bwd_unit_valu(const float* __restrict__ xh, int N, int Npad, int K, int kbase,
                           int pbeg, int pend, const float* __restrict__ beta,
                           const float* __restrict__ f, float ctv, float* __restrict__ part,
                           size_t pstride) {
  constexpr int NS = DV * (DV + 1) / 2;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int kw = kbase + wv * GW;
  if (kw >= K) return;
  float sacc[GW][NS], uacc[GW][DV], aacc[GW];
#pragma unroll
  for (int gk = 0; gk < GW; ++gk) {
#pragma unroll
    for (int e = 0; e < NS; ++e) sacc[gk][e] = 0.f;
#pragma unroll
    for (int a = 0; a < DV; ++a) uacc[gk][a] = 0.f;
    aacc[gk] = 0.f;
  }
  // The next tile's point, log-density and weights are loaded before the
  // current tile's products, to cover the load latency.
  float xn[DV], fn = 0.f, bn[GW];
  auto load = [&](int t0) {
    const int p = t0 + lane;
    const bool valid = t0 < pend && p < N;
    const int pc = valid ? p : 0;
#pragma unroll
    for (int b = 0; b < DV; ++b) xn[b] = xh[(size_t)pc * 16 + b];
    fn = valid ? f[pc] : 0.f;
#pragma unroll
    for (int gk = 0; gk < GW; ++gk)
      bn[gk] = valid ? beta[(size_t)std::min(kw + gk, K - 1) * Npad + pc] : -INFINITY;
  };
  load(pbeg);
  for (int t0 = pbeg; t0 < pend; t0 += 64) {
    float x[DV], bt[GW];
#pragma unroll
    for (int b = 0; b < DV; ++b) x[b] = xn[b];
#pragma unroll
    for (int gk = 0; gk < GW; ++gk) bt[gk] = bn[gk];
    const float fp = fn;
    load(t0 + 64);
#pragma unroll
    for (int gk = 0; gk < GW; ++gk) {
      const int k = kw + gk;
      if (k >= K) break;
      // beta is -inf past the last point, so w = 0 there
      const float w = __expf(bt[gk] - fp) * ctv;
      aacc[gk] += w;
      float wx[DV];
#pragma unroll
      for (int a = 0; a < DV; ++a) {
        wx[a] = w * x[a];
        uacc[gk][a] += wx[a];
      }
      int e = 0;
#pragma unroll
      for (int a = 0; a < DV; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
          sacc[gk][e] = fmaf(wx[a], x[b], sacc[gk][e]);
          ++e;
        }
    }
  }
#pragma unroll
  for (int gk = 0; gk < GW; ++gk) {
    const int k = kw + gk;
    if (k >= K) break;
    float* P = part + (size_t)k * pstride;
    int e = 0;
#pragma unroll
    for (int a = 0; a < DV; ++a) {
#pragma unroll
      for (int b = 0; b <= a; ++b) {
        const float v = wave_sum(sacc[gk][e++]);
        // entry (r = b, s = a) of the 16x16 block, in matrix-core output order
        if (lane == 0) P[(16 * (a >> 2) + b) * 4 + (a & 3)] = v;
      }
      const float uv = wave_sum(uacc[gk][a]);
      if (lane == 0) P[256 + a] = uv;
    }
    const float av = wave_sum(aacc[gk]);
    if (lane == 0) P[256 + 16] = av;
  }
}

// One block per instance: the origin shift, the mean of the first min(K, 16)
// means (every operand is taken about it, so data far from the origin loses
// nothing to cancellation: only x - mu enters). Split instances also get the
// power of two that brings the largest factor entry (exp(qd) or |l|) to
// [2^13, 2^14), and the largest |mu_k - shift|, which bounds every tile's
// point scale (the points are scaled per 64-point tile in the preparation):
// scaled means then stay inside the FP16 range in every tile.
__global__ void __launch_bounds__(256) k_bscale(const char* __restrict__ plan,
                                                const float* __restrict__ means,
                                                const float* __restrict__ qd,
                                                const float* __restrict__ l, char* cache) {
  const PlanHeader* h = hdr(plan);
  const BInst I = ((const BInst*)(plan + h->inst_off))[blockIdx.x];
  __shared__ float csh[64];
  __shared__ float red[8];
  block_shift(means + I.m_off, I.K, I.D, csh);
  const int t = threadIdx.x;
  float* sh = (float*)(cache + I.sh_off);
  if (t < I.DP) sh[t] = csh[t];
  if (!I.split) {
    if (t == 0) sh[I.DP] = sh[I.DP + 1] = 1.f;
    return;
  }
  float mq = 0.f, mm = 0.f;
  const int64_t nd = (int64_t)I.K * I.D, nl = (int64_t)I.K * I.D * (I.D - 1) / 2;
  for (int64_t e = t; e < nd; e += 256) {
    mq = fmaxf(mq, expf(qd[I.m_off + e]));
    mm = fmaxf(mm, fabsf(means[I.m_off + e] - csh[(int)(e % I.D)]));
  }
  for (int64_t e = t; e < nl; e += 256) mq = fmaxf(mq, fabsf(l[I.l_off + e]));
  mq = wave_max(mq);
  mm = wave_max(mm);
  if ((t & 63) == 0) {
    red[t >> 6] = mq;
    red[4 + (t >> 6)] = mm;
  }
  __syncthreads();
  if (t == 0) {
    mq = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    int eq = 0;
    if (mq > 0.f && mq <= 3.0e38f) (void)frexpf(mq, &eq);
    sh[I.DP] = ldexpf(1.f, 14 - eq);
    sh[I.DP + 1] = fmaxf(fmaxf(red[4], red[5]), fmaxf(red[6], red[7]));
  }
}

// Split form, one 64-point tile: x - shift in FP32 for the reverse (x~^T, as in
// the FP32 form) and, scaled by the power of two that brings the larger of the
// tile's largest |x - shift| and the instance's largest |mu - shift| (shift[DP
// + 1]) to [2^13, 2^14), in split FP16 for the forward (row layout); the tile's
// scale goes to ts[p0 / 64]. (256 threads; the loads are all issued before the
// first is used.)
template <int DP>
DEX_DEV void prep_x_tile_split(const float* __restrict__ x, int N, int D, int Npad, int p0,
                               const float* __restrict__ shift, _Float16* xh, _Float16* xl,
                               float* xhT, float* ts) {
  constexpr int NL = 64 * DP / 256;
  __shared__ float tile[64][DP + 1];
  __shared__ float red[4];
  __syncthreads();
  float v[NL], mx = 0.f;
  // branch-free loads at clamped addresses, selected afterwards
  float sv[NL];  // (the shift has DP entries, zero past D)
#pragma unroll
  for (int r = 0; r < NL; ++r) {
    const int e = threadIdx.x + 256 * r, pp = e / DP, b = e % DP, p = p0 + pp;
    v[r] = x[(size_t)min(p, N - 1) * D + min(b, D - 1)];
    sv[r] = shift[b];
  }
#pragma unroll
  for (int r = 0; r < NL; ++r) {
    const int e = threadIdx.x + 256 * r, pp = e / DP, b = e % DP, p = p0 + pp;
    v[r] = p < N && b < D ? v[r] - sv[r] : 0.f;
  }
#pragma unroll
  for (int r = 0; r < NL; ++r) {
    const int e = threadIdx.x + 256 * r;
    tile[e / DP][e % DP] = v[r];
    mx = fmaxf(mx, fabsf(v[r]));
  }
  mx = wave_max(mx);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  mx = fmaxf(fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3])), shift[DP + 1]);
  int ex = 0;
  if (mx > 0.f && mx <= 3.0e38f) (void)frexpf(mx, &ex);
  const float sc = ldexpf(1.f, 14 - ex);
  if (threadIdx.x == 0) ts[p0 / 64] = sc;
  for (int e = threadIdx.x; e < 8 * DP; e += blockDim.x) {
    const int pp = e / (DP / 8), b0 = 8 * (e % (DP / 8));
    float w[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) w[i] = tile[pp][b0 + i] * sc;
    store8_split<PREC_F16X3>(xh, xl, (size_t)(p0 + pp) * DP + b0, w);
  }
  // x~^T in the matrix-core step order of the moment products (as prep_x_tile)
  for (int e = threadIdx.x; e < 8 * DP; e += blockDim.x) {
    const int b = e / 8, s0 = 8 * (e % 8);
    float w[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int sp = s0 + i, st = sp & 32, q = sp & 31;
      w[i] = tile[st + 4 * (q >> 3) + (q & 3) + 16 * ((q >> 2) & 1)][b];
    }
    mom_store8<MP_F32>(xhT, nullptr, (size_t)b * Npad + p0 + s0, w);
  }
}

__global__ void __launch_bounds__(256) k_bprep_x(const char* __restrict__ plan,
                                                 const float* __restrict__ x, char* cache) {
  const PlanHeader* h = hdr(plan);
  const BItem w = ((const BItem*)(plan + h->prepx_off))[blockIdx.x];
  const BInst I = ((const BInst*)(plan + h->inst_off))[w.inst];
  if (I.split) {
    const float* sh = (const float*)(cache + I.sh_off);
    _Float16* xh = (_Float16*)(cache + I.xh_off);
    _Float16* xl = (_Float16*)(cache + I.xl_off);
    float* xhT = (float*)(cache + I.xhT_off);
    float* ts = (float*)(cache + I.ts_off);
    if (I.DP == 16)
      prep_x_tile_split<16>(x + I.x_off, I.N, I.D, (int)I.Npad, w.a * 64, sh, xh, xl, xhT, ts);
    else
      prep_x_tile_split<32>(x + I.x_off, I.N, I.D, (int)I.Npad, w.a * 64, sh, xh, xl, xhT, ts);
    return;
  }
  const float* sh = (const float*)(cache + I.sh_off);
  float* xh = (float*)(cache + I.xh_off);
  float* xhT = (float*)(cache + I.xhT_off);
  if (I.DP == 16)
    prep_x_tile<PREC_F32, 16>(x + I.x_off, I.N, I.D, (int)I.Npad, w.a * 64, xh, nullptr, xhT, nullptr,
                              nullptr, sh);
  else
    prep_x_tile<PREC_F32, 32>(x + I.x_off, I.N, I.D, (int)I.Npad, w.a * 64, xh, nullptr, xhT, nullptr,
                              nullptr, sh);
}

__global__ void __launch_bounds__(256) k_bprep_q(const char* __restrict__ plan,
                                                 const float* __restrict__ alphas,
                                                 const float* __restrict__ means,
                                                 const float* __restrict__ qd,
                                                 const float* __restrict__ l, char* cache) {
  const PlanHeader* h = hdr(plan);
  const BItem w = ((const BItem*)(plan + h->prepq_off))[blockIdx.x];
  const BInst I = ((const BInst*)(plan + h->inst_off))[w.inst];
  float* negc = (float*)(cache + I.negc_off);
  float* kappa = (float*)(cache + I.kappa_off);
  if (I.split) {
    using H = Store<PREC_F16X3>::S;
    const float* sh = (const float*)(cache + I.sh_off);
    H* Qh = (H*)(cache + I.Q_off);
    H* Ql = (H*)(cache + I.Ql_off);
    if (I.DP == 16)
      prep_q_comp<PREC_F16X3, 16>(alphas + I.a_off, means + I.m_off, qd + I.m_off, l + I.l_off, I.D,
                                  w.a, Qh, Ql, negc, kappa, sh, sh[I.DP]);
    else
      prep_q_comp<PREC_F16X3, 32>(alphas + I.a_off, means + I.m_off, qd + I.m_off, l + I.l_off, I.D,
                                  w.a, Qh, Ql, negc, kappa, sh, sh[I.DP]);
    return;
  }
  float* Q = (float*)(cache + I.Q_off);
  const float* sh = (const float*)(cache + I.sh_off);
  if (I.DP == 16)
    prep_q_comp<PREC_F32, 16>(alphas + I.a_off, means + I.m_off, qd + I.m_off, l + I.l_off, I.D, w.a,
                              Q, nullptr, negc, kappa, sh);
  else
    prep_q_comp<PREC_F32, 32>(alphas + I.a_off, means + I.m_off, qd + I.m_off, l + I.l_off, I.D, w.a,
                              Q, nullptr, negc, kappa, sh);
}

__global__ void fill_counters(int* c, int n) {
  if ((int)threadIdx.x < n) c[threadIdx.x] = 0;
}

// Take the next item index for the whole block.
DEX_DEV int next_item(int* counter) {
  __shared__ int cur;
  __syncthreads();
  if (threadIdx.x == 0) cur = atomicAdd(counter, 1);
  __syncthreads();
  return __builtin_amdgcn_readfirstlane(cur);
}

// SPLIT: the plan's instances with D > 8 carry split FP16 operands.
template <int CB, bool SPLIT>
__global__ void __launch_bounds__(256) k_bgmm_fwd(const char* __restrict__ plan, int cfg,
                                                  const char* cache, char* ws) {
  const PlanHeader* h = hdr(plan);
  const BInst* inst = (const BInst*)(plan + h->inst_off);
  const BItem* items = (const BItem*)(plan + h->fwd_off[cfg]);
  const int n = (int)h->n_fwd[cfg];
  int* counter = (int*)(ws + h->ws_counter);
  float2* ml = (float2*)(ws + h->ws_ml);
  for (;;) {
    const int it = next_item(counter);
    if (it >= n) break;
    const BItem w = items[it];
    const BInst I = inst[w.inst];
    const MfmaOps o = bops(I, cache);
    float* beta = (float*)(cache + I.beta_off);
    if (I.D <= 8) {
      fwd_unit_valu<8>(o, I.N, (int)I.Npad, w.a * 64 * CB, 64 * CB, I.K, beta, ml + I.ml_off);
    } else if constexpr (SPLIT) {
      // the wave's points lie in one 64-point tile, whose x scale applies
      const int p0 = w.a * 64 * CB + (threadIdx.x >> 6) * 16 * CB;
      const float xs = ((const float*)(cache + I.ts_off))[p0 / 64];
      const float sc = xs * ((const float*)(cache + I.sh_off))[I.DP], sfac = 1.f / (sc * sc);
      if (I.DP == 16)
        fwd_unit<16, PREC_F16X3, CB, 16>(o, I.N, (int)I.Npad, p0, 0, I.K, beta, ml + I.ml_off, sfac,
                                         xs);
      else
        fwd_unit<32, PREC_F16X3, CB, 16>(o, I.N, (int)I.Npad, p0, 0, I.K, beta, ml + I.ml_off, sfac,
                                         xs);
    } else if (I.DP == 16)
      fwd_unit<16, PREC_F32, CB, 16>(o, I.N, (int)I.Npad, w.a * 64 * CB + (threadIdx.x >> 6) * 16 * CB,
                                     0, I.K, beta, ml + I.ml_off);
    else
      fwd_unit<32, PREC_F32, CB, 16>(o, I.N, (int)I.Npad, w.a * 64 * CB + (threadIdx.x >> 6) * 16 * CB,
                                     0, I.K, beta, ml + I.ml_off);
  }
}

__global__ void __launch_bounds__(256) k_bmerge(const char* __restrict__ plan, float* __restrict__ f,
                                                char* ws) {
  const PlanHeader* h = hdr(plan);
  const BItem w = ((const BItem*)(plan + h->merge_off))[blockIdx.x];
  const BInst I = ((const BInst*)(plan + h->inst_off))[w.inst];
  const float2* ml = (const float2*)(ws + h->ws_ml) + I.ml_off;
  float* fpart = (float*)(ws + h->ws_fpart) + 2 * I.fpart_off;
  float s = 0.f, e = 0.f;
  merge_lse_block<float>(ml, 1, I.N, (int)I.Npad, w.a * 256, f + I.f_off, s, e);
  if (threadIdx.x == 0) {
    fpart[2 * w.a] = s;
    fpart[2 * w.a + 1] = e;
  }
}

__global__ void __launch_bounds__(256) k_bfinalize_F(const char* __restrict__ plan,
                                                     const float* __restrict__ alphas,
                                                     const char* ws, float* __restrict__ F) {
  const PlanHeader* h = hdr(plan);
  const BInst I = ((const BInst*)(plan + h->inst_off))[blockIdx.x];
  const float* fpart = (const float*)(ws + h->ws_fpart) + 2 * I.fpart_off;
  finalize_F_block<float>(fpart, I.nblk, alphas + I.a_off, I.K, I.N, F + blockIdx.x);
}

template <int GW, bool SPLIT>
__global__ void __launch_bounds__(256) k_bgmm_bwd(const char* __restrict__ plan, int cfg,
                                                  const char* cache, const float* __restrict__ f,
                                                  const float* __restrict__ ct, char* ws) {
  const PlanHeader* h = hdr(plan);
  const BInst* inst = (const BInst*)(plan + h->inst_off);
  const BItem* items = (const BItem*)(plan + h->bwd_off[cfg]);
  const int n = (int)h->n_bwd[cfg];
  const int64_t chunk = bbwd_cfg(cfg).chunk;
  int* counter = (int*)(ws + h->ws_counter) + 1;
  float* part = (float*)(ws + h->ws_part);
  for (;;) {
    const int it = next_item(counter);
    if (it >= n) break;
    const BItem w = items[it];
    const BInst I = inst[w.inst];
    const float* beta = (const float*)(cache + I.beta_off);
    const int pbeg = (int)(w.b * chunk);
    const int pend = (int)std::min<int64_t>(I.Npad, pbeg + chunk);
    const size_t E = mom_slot(I.DP);
    float* P = part + I.part_off + (size_t)w.b * I.K * E;
    if (I.D <= 8) {
      bwd_unit_valu<8, GW>((const float*)(cache + I.xh_off), I.N, (int)I.Npad, I.K, w.a * 4 * GW,
                           pbeg, pend, beta, f + I.f_off, ct[w.inst], P, E);
    } else if constexpr (SPLIT) {
      // FP32 moments of x - shift; the cotangent is applied in the assembly
      if (I.DP == 16)
        bwd_mom_unit<16, MP_F32, GW>(cache + I.xhT_off, nullptr, I.N, (int)I.Npad, I.K,
                                     w.a * 4 * GW + (threadIdx.x >> 6) * GW, pbeg, pend, beta,
                                     f + I.f_off, 1.f, P, E);
      else
        bwd_mom_unit<32, MP_F32, GW>(cache + I.xhT_off, nullptr, I.N, (int)I.Npad, I.K,
                                     w.a * 4 * GW + (threadIdx.x >> 6) * GW, pbeg, pend, beta,
                                     f + I.f_off, 1.f, P, E);
    } else if (I.DP == 16)
      bwd_mom_unit<16, MP_F32, GW>(cache + I.xhT_off, nullptr, I.N, (int)I.Npad, I.K,
                                   w.a * 4 * GW + (threadIdx.x >> 6) * GW,
                                   pbeg, pend, beta, f + I.f_off, ct[w.inst], P, E);
    else
      bwd_mom_unit<32, MP_F32, GW>(cache + I.xhT_off, nullptr, I.N, (int)I.Npad, I.K,
                                   w.a * 4 * GW + (threadIdx.x >> 6) * GW,
                                   pbeg, pend, beta, f + I.f_off, ct[w.inst], P, E);
  }
}

__global__ void __launch_bounds__(256) k_bbwd_finalize(const char* __restrict__ plan, int cfg,
                                                       const char* ws, const char* cache,
                                                       const float* __restrict__ alphas,
                                                       const float* __restrict__ qd,
                                                       const float* __restrict__ l,
                                                       const float* __restrict__ means,
                                                       const float* __restrict__ ct,
                                                       float* __restrict__ d_alphas,
                                                       float* __restrict__ d_means,
                                                       float* __restrict__ d_qd,
                                                       float* __restrict__ d_l, int accumulate) {
  const PlanHeader* h = hdr(plan);
  const BItem w = ((const BItem*)(plan + h->prepq_off))[blockIdx.x];  // (instance, k)
  const BInst I = ((const BInst*)(plan + h->inst_off))[w.inst];
  const int nch = ((const int32_t*)(plan + h->nch_off))[cfg * h->B + w.inst];
  const size_t E = mom_slot(I.DP);
  const float* part = (const float*)(ws + h->ws_part) + I.part_off + (size_t)w.a * E;
  if (I.split) {
    // moments of x - shift without the cotangent
    const float* sh = (const float*)(cache + I.sh_off);
    const float c = ct[w.inst];
    bwd_finalize_mom<32>(part, (size_t)I.K * E, nch, w.a, I.K, I.D, I.DP, I.N, alphas + I.a_off,
                     means + I.m_off, qd + I.m_off, l + I.l_off, c, d_alphas + I.a_off,
                     d_means + I.m_off, d_qd + I.m_off, d_l + I.l_off, accumulate, sh, c, c, c);
    return;
  }
  bwd_finalize_mom<32>(part, (size_t)I.K * E, nch, w.a, I.K, I.D, I.DP, I.N, alphas + I.a_off,
                   means + I.m_off, qd + I.m_off, l + I.l_off, ct[w.inst], d_alphas + I.a_off,
                   d_means + I.m_off, d_qd + I.m_off, d_l + I.l_off, accumulate,
                   (const float*)(cache + I.sh_off));
}

}  // namespace dexk

// ===========================================================================
namespace dexi {
using namespace dexk;

namespace {

struct PlanBuild {
  PlanHeader h{};
  std::vector<BInst> inst;
  std::vector<BItem> prepx, prepq, merge;
  std::vector<BItem> fwd[kBFwdCfgs], bwd[kBBwdCfgs];
  std::vector<int32_t> nch;  // [cfg][B]
  size_t bytes = 0;
};

int64_t dp_cost(int DP) { return DP == 16 ? 1 : 3; }  // 16-deep chunks per 16 points per k

PlanBuild build_plan(const int64_t* shapes, int64_t B, int32_t variant) {
  PlanBuild p;
  p.h.B = B;
  p.inst.resize(B);
  int64_t a = 0, m = 0, lo = 0, xo = 0, fo = 0, ml = 0, fp = 0, cache = 0, part = 0;
  auto take = [&](int64_t bytes) {
    int64_t at = cache;
    cache += (int64_t)align256((size_t)bytes);
    return at;
  };
  for (int64_t b = 0; b < B; ++b) {
    BInst& I = p.inst[b];
    I.N = (int32_t)shapes[3 * b];
    I.D = (int32_t)shapes[3 * b + 1];
    I.K = (int32_t)shapes[3 * b + 2];
    I.DP = I.D <= 16 ? 16 : 32;
    I.Npad = (I.N + 255) / 256 * 256;
    I.nblk = (int32_t)(I.Npad / 256);
    I.a_off = a;
    I.m_off = m;
    I.l_off = lo;
    I.x_off = xo;
    I.f_off = fo;
    a += I.K;
    m += (int64_t)I.K * I.D;
    lo += (int64_t)I.K * I.D * (I.D - 1) / 2;
    xo += (int64_t)I.N * I.D;
    fo += I.N;
    I.split = variant == DEX_GMM_F16X3 && I.D > 8;
    const int64_t es = I.split ? 2 : 4;  // forward operand element bytes
    I.xh_off = take(I.Npad * I.DP * es);
    I.xhT_off = take(I.Npad * I.DP * 4);
    I.Q_off = take((int64_t)I.K * I.DP * I.DP * es);
    if (I.split) {
      I.xl_off = take(I.Npad * I.DP * es);
      I.Ql_off = take((int64_t)I.K * I.DP * I.DP * es);
      I.ts_off = take(I.Npad / 64 * 4);
    }
    I.sh_off = take((int64_t)(I.DP + 2) * 4);
    I.negc_off = take((int64_t)I.K * I.DP * 4);
    I.kappa_off = take((int64_t)I.K * 4);
    I.beta_off = take((int64_t)I.K * I.Npad * 4);
    I.ml_off = ml;
    ml += I.Npad;
    I.fpart_off = fp;
    fp += I.nblk;
    int64_t maxch = 0;
    for (int c = 0; c < kBBwdCfgs; ++c) {
      const int64_t ch = (I.Npad + bbwd_cfg(c).chunk - 1) / bbwd_cfg(c).chunk;
      maxch = std::max(maxch, ch);
    }
    I.part_off = part;
    part += maxch * I.K * (int64_t)mom_slot(I.DP);
    part = (part + 63) / 64 * 64;
    for (int t = 0; t < I.Npad / 64; ++t) p.prepx.push_back({(int32_t)b, t, 0, 0});
    for (int k = 0; k < I.K; ++k) p.prepq.push_back({(int32_t)b, k, 0, 0});
    for (int t = 0; t < I.nblk; ++t) p.merge.push_back({(int32_t)b, t, 0, 0});
  }
  // forward work lists, longest first
  for (int c = 0; c < kBFwdCfgs; ++c) {
    const int pts = 64 * bfwd_cb(c);
    std::vector<std::pair<int64_t, BItem>> v;
    for (int64_t b = 0; b < B; ++b) {
      const BInst& I = p.inst[b];
      for (int t = 0; t < I.Npad / pts; ++t)
        v.push_back({(int64_t)I.K * dp_cost(I.DP) * pts, BItem{(int32_t)b, t, 0, 0}});
    }
    std::stable_sort(v.begin(), v.end(), [](auto& x, auto& y) { return x.first > y.first; });
    for (auto& e : v) p.fwd[c].push_back(e.second);
  }
  p.nch.assign((size_t)kBBwdCfgs * B, 0);
  for (int c = 0; c < kBBwdCfgs; ++c) {
    const BBwd bc = bbwd_cfg(c);
    std::vector<std::pair<int64_t, BItem>> v;
    for (int64_t b = 0; b < B; ++b) {
      const BInst& I = p.inst[b];
      const int nch = (int)((I.Npad + bc.chunk - 1) / bc.chunk);
      p.nch[(size_t)c * B + b] = nch;
      const int kg = 4 * bc.gw;
      const int ngroups = (I.K + kg - 1) / kg;
      for (int g = 0; g < ngroups; ++g) {
        const int kk = std::min(kg, I.K - g * kg);
        for (int s = 0; s < nch; ++s) {
          const int64_t pts = std::min<int64_t>(bc.chunk, I.Npad - s * bc.chunk);
          // the busiest wave of the block bounds the item's time
          const int64_t per_wave = std::min(bc.gw, kk);
          // moment blocks per 32 points: 1 (DP = 16) or 3 (DP = 32)
          v.push_back({per_wave * pts * (I.DP == 16 ? 1 : 3),
                       BItem{(int32_t)b, g, s, 0}});
        }
      }
    }
    std::stable_sort(v.begin(), v.end(), [](auto& x, auto& y) { return x.first > y.first; });
    for (auto& e : v) p.bwd[c].push_back(e.second);
  }
  // layout of the plan bytes
  size_t o = align256(sizeof(PlanHeader));
  auto place = [&](size_t bytes) {
    size_t at = o;
    o += align256(bytes);
    return (int64_t)at;
  };
  p.h.inst_off = place(p.inst.size() * sizeof(BInst));
  p.h.prepx_off = place(p.prepx.size() * sizeof(BItem));
  p.h.n_prepx = (int64_t)p.prepx.size();
  p.h.prepq_off = place(p.prepq.size() * sizeof(BItem));
  p.h.n_prepq = (int64_t)p.prepq.size();
  p.h.merge_off = place(p.merge.size() * sizeof(BItem));
  p.h.n_merge = (int64_t)p.merge.size();
  for (int c = 0; c < kBFwdCfgs; ++c) {
    p.h.fwd_off[c] = place(p.fwd[c].size() * sizeof(BItem));
    p.h.n_fwd[c] = (int64_t)p.fwd[c].size();
  }
  for (int c = 0; c < kBBwdCfgs; ++c) {
    p.h.bwd_off[c] = place(p.bwd[c].size() * sizeof(BItem));
    p.h.n_bwd[c] = (int64_t)p.bwd[c].size();
  }
  p.h.nch_off = place(p.nch.size() * sizeof(int32_t));
  p.bytes = o;
  p.h.cache_bytes = cache;
  size_t w = 0;
  p.h.ws_counter = (int64_t)w;  // fixed at offset 0: the host clears it before each phase
  w += 256;
  p.h.ws_ml = (int64_t)w;
  w += align256((size_t)ml * sizeof(float2));
  p.h.ws_fpart = (int64_t)w;
  w += align256((size_t)fp * 2 * sizeof(float));
  p.h.ws_part = (int64_t)w;
  w += align256((size_t)part * sizeof(float));
  p.h.ws_bytes = (int64_t)w;
  return p;
}

// host copy of the header fields the launcher needs, recovered from the
// descriptor (the plan itself lives on the device)
struct HostPlan {
  int64_t B, n_prepx, n_prepq, n_merge, n_fwd[kBFwdCfgs], n_bwd[kBBwdCfgs], cache, ws;
};

}  // namespace

size_t gmm_batched_plan_bytes(int64_t B, const int64_t* shapes, int32_t variant) {
  return build_plan(shapes, B, variant).bytes;
}

// Descriptor dims: {B, sum N, sum K, sum K*D, sum K*L, sum N*D, plan bytes, cache bytes}.
// The item counts and workspace size are recovered from the plan header on
// the host by dex_gmm_batched_plan only; launches use the counts stored in
// fparams (exact integers below 2^53).
dex_status gmm_batched_plan(const int64_t* shapes, int64_t B, int32_t variant, dex_desc* d,
                            void* plan, size_t plan_bytes) {
  PlanBuild p = build_plan(shapes, B, variant);
  int64_t sumN = 0, sumK = 0, sumKD = 0, sumKL = 0, sumND = 0;
  for (int64_t b = 0; b < B; ++b) {
    const int64_t N = shapes[3 * b], D = shapes[3 * b + 1], K = shapes[3 * b + 2];
    sumN += N;
    sumK += K;
    sumKD += K * D;
    sumKL += K * D * (D - 1) / 2;
    sumND += N * D;
  }
  memset(d, 0, sizeof(*d));
  d->kind = DEX_GMM_BATCHED;
  d->dtype = DEX_F32;
  d->variant = variant;
  d->dims[0] = B;
  d->dims[1] = sumN;
  d->dims[2] = sumK;
  d->dims[3] = sumKD;
  d->dims[4] = sumKL;
  d->dims[5] = sumND;
  d->dims[6] = (int64_t)p.bytes;
  d->dims[7] = p.h.cache_bytes;
  // item counts for the launches: prepx, merge, ws bytes, and the persistent
  // lists' lengths are read on the device; the host needs grid sizes
  d->fparams[0] = (double)p.h.n_prepx;
  d->fparams[1] = (double)p.h.n_merge;
  d->fparams[2] = (double)p.h.ws_bytes;
  d->fparams[3] = 0.0;
  if (!plan) return DEX_OK;
  if (plan_bytes < p.bytes) return fail(DEX_ERR_INVALID_ARG, "plan buffer too small");
  char* o = (char*)plan;
  memset(o, 0, p.bytes);
  memcpy(o, &p.h, sizeof(PlanHeader));
  memcpy(o + p.h.inst_off, p.inst.data(), p.inst.size() * sizeof(BInst));
  memcpy(o + p.h.prepx_off, p.prepx.data(), p.prepx.size() * sizeof(BItem));
  memcpy(o + p.h.prepq_off, p.prepq.data(), p.prepq.size() * sizeof(BItem));
  memcpy(o + p.h.merge_off, p.merge.data(), p.merge.size() * sizeof(BItem));
  for (int c = 0; c < kBFwdCfgs; ++c)
    memcpy(o + p.h.fwd_off[c], p.fwd[c].data(), p.fwd[c].size() * sizeof(BItem));
  for (int c = 0; c < kBBwdCfgs; ++c)
    memcpy(o + p.h.bwd_off[c], p.bwd[c].data(), p.bwd[c].size() * sizeof(BItem));
  memcpy(o + p.h.nch_off, p.nch.data(), p.nch.size() * sizeof(int32_t));
  return DEX_OK;
}

size_t gmm_batched_ws_bytes(const dex_desc& d, int role) {
  if (role == DEX_WS_RESID) return (size_t)d.dims[7];
  return (size_t)d.fparams[2];
}

int gmm_batched_num_configs(const dex_desc& d, int role) {
  (void)d;
  return role == DEX_WS_VJP ? kBBwdCfgs : kBFwdCfgs;
}

// Blocks of the persistent launches, per CU: the reverse kernels hide their
// load latency with more resident blocks; the forward ones do best with two.
static int persistent_blocks(bool reverse) { return num_cus() * (reverse ? 4 : 2); }

dex_status gmm_batched_fwd(const dex_desc& d, int cfg, const void* plan, const GmmPtrs& in,
                           void* F, void* f, void* cache, void* ws, hipStream_t st) {
  if (cfg < 0 || cfg >= kBFwdCfgs) return fail(DEX_ERR_INVALID_ARG, "batched forward config");
  const int64_t B = d.dims[0], sumK = d.dims[2];
  const int64_t n_prepx = (int64_t)d.fparams[0], n_merge = (int64_t)d.fparams[1];
  const char* pl = (const char*)plan;
  char* cc = (char*)cache;
  char* w = (char*)ws;
  const bool split = d.variant == DEX_GMM_F16X3;
  hipLaunchKernelGGL(k_bscale, dim3((unsigned)B), dim3(256), 0, st, pl, (const float*)in.means,
                     (const float*)in.qd, (const float*)in.l, cc);
  hipLaunchKernelGGL(k_bprep_x, dim3((unsigned)n_prepx), dim3(256), 0, st, pl, (const float*)in.x, cc);
  hipLaunchKernelGGL(k_bprep_q, dim3((unsigned)sumK), dim3(256), 0, st, pl, (const float*)in.alphas,
                     (const float*)in.means, (const float*)in.qd, (const float*)in.l, cc);
  hipLaunchKernelGGL(fill_counters, dim3(1), dim3(64), 0, st, (int*)w, 64);
  ProfRange pr(DEX_PROF_BGMM_FWD, st);
#define DEX_BF(CB_, S_)                                                                    \
  hipLaunchKernelGGL((k_bgmm_fwd<CB_, S_>), dim3(persistent_blocks(false)), dim3(256), 0, st, pl, \
                     cfg, (const char*)cc, w)
  if (bfwd_cb(cfg) == 4) {
    if (split)
      DEX_BF(4, true);
    else
      DEX_BF(4, false);
  } else {
    if (split)
      DEX_BF(2, true);
    else
      DEX_BF(2, false);
  }
#undef DEX_BF
  pr.end(1);
  hipLaunchKernelGGL(k_bmerge, dim3((unsigned)n_merge), dim3(256), 0, st, pl, (float*)f, w);
  hipLaunchKernelGGL(k_bfinalize_F, dim3((unsigned)B), dim3(256), 0, st, pl, (const float*)in.alphas,
                     (const char*)w, (float*)F);
  return check_hip(hipGetLastError(), "gmm_batched_fwd");
}

dex_status gmm_batched_vjp(const dex_desc& d, int cfg, const void* plan, const GmmPtrs& in,
                           const void* f, const void* cache, const void* ct, const GmmGrads& out,
                           bool accumulate, void* ws, hipStream_t st) {
  if (cfg < 0 || cfg >= kBBwdCfgs) return fail(DEX_ERR_INVALID_ARG, "batched reverse config");
  const int64_t sumK = d.dims[2];
  const char* pl = (const char*)plan;
  char* w = (char*)ws;
  const BBwd bc = bbwd_cfg(cfg);
  hipLaunchKernelGGL(fill_counters, dim3(1), dim3(64), 0, st, (int*)w, 64);
  const bool split = d.variant == DEX_GMM_F16X3;
#define DEX_BB(GW_)                                                                          \
  do {                                                                                       \
    if (split)                                                                               \
      hipLaunchKernelGGL((k_bgmm_bwd<GW_, true>), dim3(persistent_blocks(true)), dim3(256), 0, \
                         st, pl, cfg, (const char*)cache, (const float*)f, (const float*)ct, w); \
    else                                                                                     \
      hipLaunchKernelGGL((k_bgmm_bwd<GW_, false>), dim3(persistent_blocks(true)), dim3(256), 0, \
                         st, pl, cfg, (const char*)cache, (const float*)f, (const float*)ct, w); \
  } while (0)
  ProfRange pr(DEX_PROF_BGMM_VJP, st);
  if (bc.gw == 1)
    DEX_BB(1);
  else if (bc.gw == 2)
    DEX_BB(2);
  else
    DEX_BB(4);
#undef DEX_BB
  pr.end(1);
  hipLaunchKernelGGL(k_bbwd_finalize, dim3((unsigned)sumK), dim3(256), 0, st, pl, cfg,
                     (const char*)w, (const char*)cache, (const float*)in.alphas, (const float*)in.qd,
                     (const float*)in.l, (const float*)in.means, (const float*)ct,
                     (float*)out.d_alphas,
                     (float*)out.d_means, (float*)out.d_qd, (float*)out.d_l, accumulate ? 1 : 0);
  return check_hip(hipGetLastError(), "gmm_batched_vjp");
}

}  // namespace dexi
