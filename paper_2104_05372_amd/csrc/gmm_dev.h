// GMM device code shared by the single-instance and the batched launches.
//
// Objective (one instance), with Q_k = diag(exp(qd_k)) + strict-lower(l_k):
//   beta[i,k] = alphas[k] + sum_d qd[k,d] - 1/2 ||Q_k (x_i - mu_k)||^2
//   f[i] = logsumexp_k beta[i,k],   F = sum_i f[i] - N logsumexp_k alphas[k]
//
// Reverse pass (transpose of the linearized loop `for i k`, Sec. 5.2): the
// cotangent of beta[i,k] is w[i,k] = ct exp(beta[i,k] - f[i]); the indexed reads
// of the component-k parameters transpose into accumulations over i
// (LetIndexingTranspose, Fig. "transposition rules"), a regular segmented
// reduction (Sec. 6.1.3):
//   A_k = sum_i w_ik,  b_k = sum_i w_ik y_ik,  M_k = sum_i w_ik y_ik r_ik^T,
// with r_ik = x_i - mu_k and y_ik = Q_k r_ik, from which
//   d_alphas[k] = A_k - ct N softmax(alphas)_k,   d_means[k] = Q_k^T b_k,
//   d_qd[k,d] = A_k - exp(qd[k,d]) M_k[d,d],       d_l[k](a,b) = -M_k[a,b] (a > b).
//
// Matrix-core form (FP32 storage): Y = Q~ X~^T - c~ is a triangular-block
// product on 16x16 output tiles with BF16, split-BF16 or FP32 operands and FP32
// accumulation; c~_k = Q~_k mu_k, so y = Q~(x~ - mu). The contraction over the
// feature index is cut into chunks of CK (16 or 32) and a chunk is skipped when
// it lies wholly above the diagonal. Padded dimension DP in {16, 32, 64}.
// beta is kept as a residual (it is the input of the non-linear exp in the
// reverse pass, Sec. 5.3.2), so the reverse pass recomputes Y but not its norm.
//
// Lane layout of a 16x16 matrix-core tile (wave64): lane = 16 g + c holds
// column c and rows 4g..4g+3 of the output; for the operands, lane 16 g + c
// supplies row (A) or column (B) c and the contraction values of group g.
// Which contraction index a group's values stand for is our choice as long as
// A and B agree, which the kernels below use to avoid register transposes.
#pragma once

#include <math.h>

#include "common.h"

namespace dexk {

enum { PREC_F32 = 0, PREC_BF16 = 1, PREC_BF16X3 = 2 };

template <int PREC>
struct Store {
  using S = __bf16;
};
template <>
struct Store<PREC_F32> {
  using S = float;
};

template <int PREC, int NV>
struct VecT;
template <int NV>
struct VecT<PREC_F32, NV> {
  typedef __attribute__((__vector_size__(NV * sizeof(float)))) float V;
};
template <int NV>
struct VecT<PREC_BF16, NV> {
  typedef __attribute__((__vector_size__(NV * sizeof(__bf16)))) __bf16 V;
};
template <int NV>
struct VecT<PREC_BF16X3, NV> {
  typedef __attribute__((__vector_size__(NV * sizeof(__bf16)))) __bf16 V;
};

// One lane's NV contraction values (hi [, lo]).
template <int PREC, int NV>
struct Op {
  static constexpr int NS = PREC == PREC_BF16X3 ? 2 : 1;
  typename VecT<PREC, NV>::V v[NS];
};

template <int PREC, int NV>
DEX_DEV f32x4 mma_chunk(const typename VecT<PREC, NV>::V& a, const typename VecT<PREC, NV>::V& b,
                        f32x4 c) {
  if constexpr (PREC == PREC_F32) {
    // NV steps of 16x16x4; step j takes element j of every lane
#pragma unroll
    for (int j = 0; j < NV; ++j) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j], b[j], c, 0, 0, 0);
  } else if constexpr (NV == 8) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  } else {
    static_assert(NV == 4, "BF16 operands hold 4 or 8 values per lane");
    typedef __attribute__((__vector_size__(4 * sizeof(short)))) short s4;
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4, a), __builtin_bit_cast(s4, b),
                                                  c, 0, 0, 0);
  }
  return c;
}

template <int PREC, int NV>
DEX_DEV f32x4 mma(const Op<PREC, NV>& a, const Op<PREC, NV>& b, f32x4 c) {
  if constexpr (PREC == PREC_BF16X3) {
    c = mma_chunk<PREC, NV>(a.v[1], b.v[0], c);  // small cross terms first
    c = mma_chunk<PREC, NV>(a.v[0], b.v[1], c);
    c = mma_chunk<PREC, NV>(a.v[0], b.v[0], c);
  } else {
    c = mma_chunk<PREC, NV>(a.v[0], b.v[0], c);
  }
  return c;
}

// NV contiguous elements at element offset `off` of the hi (and lo) arrays.
template <int PREC, int NV>
DEX_DEV Op<PREC, NV> load_op(const typename Store<PREC>::S* hi, const typename Store<PREC>::S* lo,
                             size_t off) {
  using V = typename VecT<PREC, NV>::V;
  Op<PREC, NV> o;
  o.v[0] = *reinterpret_cast<const V*>(hi + off);
  if constexpr (Op<PREC, NV>::NS == 2) o.v[1] = *reinterpret_cast<const V*>(lo + off);
  return o;
}

// Two runs of 4 contiguous elements, at off and off + 16.
template <int PREC>
DEX_DEV Op<PREC, 8> load_op_split(const typename Store<PREC>::S* hi,
                                  const typename Store<PREC>::S* lo, size_t off) {
  using V4 = typename VecT<PREC, 4>::V;
  Op<PREC, 8> o;
#pragma unroll
  for (int s = 0; s < Op<PREC, 8>::NS; ++s) {
    const typename Store<PREC>::S* base = (s == 0 ? hi : lo) + off;
    V4 a = *reinterpret_cast<const V4*>(base);
    V4 b = *reinterpret_cast<const V4*>(base + 16);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      o.v[s][e] = a[e];
      o.v[s][e + 4] = b[e];
    }
  }
  return o;
}

template <int PREC>
DEX_DEV Op<PREC, 8> to_op(const float (&v)[8]) {
  Op<PREC, 8> o;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    if constexpr (PREC == PREC_F32) {
      o.v[0][e] = v[e];
    } else {
      __bf16 h = (__bf16)v[e];
      o.v[0][e] = h;
      if constexpr (PREC == PREC_BF16X3) o.v[1][e] = (__bf16)(v[e] - (float)h);
    }
  }
  return o;
}

template <int PREC>
DEX_DEV void store_split(typename Store<PREC>::S* hi, typename Store<PREC>::S* lo, size_t off,
                         float v) {
  if constexpr (PREC == PREC_F32) {
    hi[off] = v;
  } else {
    __bf16 h = (__bf16)v;
    hi[off] = h;
    if constexpr (PREC == PREC_BF16X3) lo[off] = (__bf16)(v - (float)h);
  }
}

// The value the products actually use for v (hi, or hi + lo).
template <int PREC>
DEX_DEV float rounded(float v) {
  if constexpr (PREC == PREC_F32) {
    return v;
  } else {
    __bf16 h = (__bf16)v;
    float r = (float)h;
    if constexpr (PREC == PREC_BF16X3) r += (float)(__bf16)(v - r);
    return r;
  }
}

// Error-free transformation of a + b (Knuth's TwoSum).
template <typename T>
DEX_DEV void two_sum(T a, T b, T& s, T& e) {
  s = a + b;
  T bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Compensated sum of one value per thread over the block, fixed tree; the
// result (s, e) is valid in thread 0.
template <typename T>
DEX_DEV void block_comp_sum(T v, T& out_s, T& out_e) {
  __shared__ T sh_s[16], sh_e[16];
  T s = v, e = 0;
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    T os = xor_lane(s, m), oe = xor_lane(e, m);
    T ns, ne;
    two_sum(s, os, ns, ne);
    s = ns;
    e = e + oe + ne;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) {
    sh_s[w] = s;
    sh_e[w] = e;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    T S = sh_s[0], E = sh_e[0];
    for (int i = 1; i < nw; ++i) {
      T ns, ne;
      two_sum(S, sh_s[i], ns, ne);
      S = ns;
      E += sh_e[i] + ne;
    }
    out_s = S;
    out_e = E;
  }
}

template <typename T>
DEX_DEV T dexp(T v);
template <>
DEX_DEV float dexp<float>(float v) { return expf(v); }
template <>
DEX_DEV double dexp<double>(double v) { return exp(v); }
template <typename T>
DEX_DEV T dlog(T v);
template <>
DEX_DEV float dlog<float>(float v) { return logf(v); }
template <>
DEX_DEV double dlog<double>(double v) { return log(v); }

// Reduce per-lane partial values over the 4 lane groups (lane bits 5 and 4);
// for NV = 4 lane group g ends up owning entry g, for NV = 2 groups {0,1} own
// entry 0 and {2,3} entry 1, for NV = 1 every group owns the total.
template <int NV>
DEX_DEV void treduce_groups(float (&v)[NV]) {
  const int lane = threadIdx.x & 63;
  if constexpr (NV == 4) {
    const bool h5 = lane & 32;
    float s0 = h5 ? v[0] : v[2], s1 = h5 ? v[1] : v[3];
    float k0 = h5 ? v[2] : v[0], k1 = h5 ? v[3] : v[1];
    k0 += xor_lane(s0, 32);
    k1 += xor_lane(s1, 32);
    const bool h4 = lane & 16;
    float s = h4 ? k0 : k1, kk = h4 ? k1 : k0;
    v[0] = kk + xor_lane(s, 16);
  } else if constexpr (NV == 2) {
    const bool h5 = lane & 32;
    float s = h5 ? v[0] : v[1], kk = h5 ? v[1] : v[0];
    v[0] = kk + xor_lane(s, 32);
    v[0] += xor_lane(v[0], 16);
  } else {
    v[0] += xor_lane(v[0], 32);
    v[0] += xor_lane(v[0], 16);
  }
}

// Operand cache of one instance (FP32 storage, matrix-core forms).
struct MfmaOps {
  const void *xh, *xl;    // x~   [Npad x DP]
  const void *xhT, *xlT;  // x~^T [DP x Npad]
  const void *Qh, *Ql;    // Q~   [K x DP x DP]
  const float* negc;      // -c~  [K x DP]
  const float* kappa;     // alphas[k] + sum_d qd[k,d]   [K]
};

// ---------------------------------------------------------------------------
// Operand preparation for 64 points starting at p0: x~ (row-major) and x~^T,
// zero padded to DP features and Npad points.
template <int PREC, int DP>
DEX_DEV void prep_x_tile(const float* __restrict__ x, int N, int D, int Npad, int p0,
                         typename Store<PREC>::S* xh, typename Store<PREC>::S* xl,
                         typename Store<PREC>::S* xhT, typename Store<PREC>::S* xlT) {
  __shared__ float tile[64][DP + 1];
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * DP; e += blockDim.x) {
    int pp = e / DP, b = e % DP, p = p0 + pp;
    tile[pp][b] = (p < N && b < D) ? x[(size_t)p * D + b] : 0.f;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * DP; e += blockDim.x) {
    int pp = e / DP, b = e % DP;
    store_split<PREC>(xh, xl, (size_t)(p0 + pp) * DP + b, tile[pp][b]);
  }
  for (int e = threadIdx.x; e < 64 * DP; e += blockDim.x) {
    int b = e / 64, pp = e % 64;
    store_split<PREC>(xhT, xlT, (size_t)b * Npad + p0 + pp, tile[pp][b]);
  }
}

// Q~_k (dense DP x DP, zero above the diagonal and in the padding), -c~_k and
// kappa_k for one component k.
template <int PREC, int DP>
DEX_DEV void prep_q_comp(const float* __restrict__ alphas, const float* __restrict__ means,
                         const float* __restrict__ qd, const float* __restrict__ l, int D, int k,
                         typename Store<PREC>::S* Qh, typename Store<PREC>::S* Ql, float* negc,
                         float* kappa) {
  __shared__ float qs[DP][DP + 1];
  const int L = D * (D - 1) / 2;
  __syncthreads();
  for (int e = threadIdx.x; e < DP * DP; e += blockDim.x) {
    int a = e / DP, b = e % DP;
    float q = 0.f;
    if (a < D && b < D) {
      if (a == b)
        q = expf(qd[(size_t)k * D + a]);
      else if (a > b)
        q = l[(size_t)k * L + a * (a - 1) / 2 + b];
    }
    store_split<PREC>(Qh, Ql, (size_t)k * DP * DP + e, q);
    qs[a][b] = rounded<PREC>(q);
  }
  __syncthreads();
  if (threadIdx.x < DP) {
    const int a = threadIdx.x;
    float c = 0.f;
    for (int b = 0; b < D; ++b) c = fmaf(qs[a][b], means[(size_t)k * D + b], c);
    negc[(size_t)k * DP + a] = -c;
  }
  if (threadIdx.x == 0) {
    float s = alphas[k];
    for (int d = 0; d < D; ++d) s += qd[(size_t)k * D + d];
    kappa[k] = s;
  }
}

// ---------------------------------------------------------------------------
// Forward unit: 4 waves x 16*CB points from p0, components [k0, k1).
// Each wave builds Y^T (DP x 16*CB) = Q~_k X~^T - c~ from 16x16 tiles (row
// block rb of Q, column block cb of points). A point's squared norm reduces
// across the 4 lane groups, after which each lane owns one point and keeps its
// running log-sum-exp over the k-range.
template <int DP, int PREC, int CB, int CK>
DEX_DEV void fwd_unit(const MfmaOps& ops, int N, int Npad, int p0blk, int k0, int k1,
                      float* __restrict__ beta, float2* __restrict__ ml) {
  using S = typename Store<PREC>::S;
  constexpr int NV = CK / 4;
  constexpr int NRB = DP / 16, NCH = DP / CK;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;
  const int p0 = p0blk + wv * (16 * CB);
  const S* xh = (const S*)ops.xh;
  const S* xl = (const S*)ops.xl;
  const S* Qh = (const S*)ops.Qh;
  const S* Ql = (const S*)ops.Ql;

  Op<PREC, NV> xb[CB][NCH];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb)
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
      xb[cb][ch] = load_op<PREC, NV>(xh, xl, (size_t)(p0 + 16 * cb + c) * DP + CK * ch + NV * g);

  int p;
  bool owner;
  if constexpr (CB == 4) {
    p = p0 + lane;
    owner = true;
  } else if constexpr (CB == 2) {
    p = p0 + 16 * (g >> 1) + c;
    owner = (g & 1) == 0;
  } else {
    p = p0 + c;
    owner = g == 0;
  }
  float m = -INFINITY, lsum = 0.f;

  for (int k = k0; k < k1; ++k) {
    const size_t qoff = (size_t)k * DP * DP;
    f32x4 acc[CB][NRB];
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) {
      const f32x4 ci = *reinterpret_cast<const f32x4*>(ops.negc + (size_t)k * DP + 16 * rb + 4 * g);
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) acc[cb][rb] = ci;
    }
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) {
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) {
        if (CK * ch > 16 * rb + 15) continue;  // chunk wholly above the diagonal
        const Op<PREC, NV> qa =
            load_op<PREC, NV>(Qh + qoff, Ql ? Ql + qoff : nullptr, (size_t)(16 * rb + c) * DP + CK * ch + NV * g);
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[cb][rb] = mma<PREC, NV>(qa, xb[cb][ch], acc[cb][rb]);
      }
    }
    float s[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
      float t = 0.f;
#pragma unroll
      for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) t = fmaf(acc[cb][rb][i], acc[cb][rb][i], t);
      s[cb] = t;
    }
    treduce_groups<CB>(s);
    const float b = ops.kappa[k] - 0.5f * s[0];
    if (owner && p < N) beta[(size_t)k * Npad + p] = b;
    const float d = b - m;
    if (d > 0.f) {
      lsum = lsum * __expf(-d) + 1.f;
      m = b;
    } else {
      lsum += __expf(d);
    }
  }
  if (owner) ml[p] = make_float2(m, lsum);
}

// ---------------------------------------------------------------------------
// Reverse unit: wave wv handles components kbase+wv*GW .. +GW-1 over the points
// [pbeg, pend), in tiles of 16*PB. Y (points x DP) = X~ Q~_k^T - c~ is
// recomputed with points as rows, so a lane holds column a = 16 ab + c of rows
// p = 16 pb + 4 g + i. Scaled by w, these registers are directly the B operand
// of the weighted outer product
//   M_k^T (DP x DP) += X~^T (DP x 32) (w Y) (32 x DP)
// over 32-point chunks, where lane group g's contraction values are the points
// {4g..4g+3, 16+4g..16+4g+3}; the A operand X~^T is loaded to match.
// Partials per component: M (row stride DP, rows a >= b written), b at DP*DP,
// A at DP*DP + DP; `part` points at the (chunk, component 0) slot, `pstride`
// floats apart per component.
template <int DP, int PREC, int PB, int GW, int CK>
DEX_DEV void bwd_unit(const MfmaOps& ops, int N, int Npad, int K, int kbase, int pbeg, int pend,
                      const float* __restrict__ beta, const float* __restrict__ f, float ctv,
                      float* __restrict__ part, size_t pstride) {
  using S = typename Store<PREC>::S;
  constexpr int NV = CK / 4;
  constexpr int NAB = DP / 16, NCH = DP / CK, NJ = PB / 2;
  constexpr int NBLK = NAB * (NAB + 1) / 2;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;
  const int kw = kbase + wv * GW;
  if (kw >= K) return;
  const S* xh = (const S*)ops.xh;
  const S* xl = (const S*)ops.xl;
  const S* xhT = (const S*)ops.xhT;
  const S* xlT = (const S*)ops.xlT;
  const S* Qh = (const S*)ops.Qh;
  const S* Ql = (const S*)ops.Ql;
  __shared__ float wsh[4][64];

  f32x4 macc[GW][NBLK];
  float bacc[GW][NAB];
  float aacc[GW];
#pragma unroll
  for (int gk = 0; gk < GW; ++gk) {
#pragma unroll
    for (int q = 0; q < NBLK; ++q) macc[gk][q] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ab = 0; ab < NAB; ++ab) bacc[gk][ab] = 0.f;
    aacc[gk] = 0.f;
  }

  for (int t0 = pbeg; t0 < pend; t0 += 16 * PB) {
    Op<PREC, NV> xa[PB][NCH];
#pragma unroll
    for (int pb = 0; pb < PB; ++pb)
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch)
        xa[pb][ch] = load_op<PREC, NV>(xh, xl, (size_t)(t0 + 16 * pb + c) * DP + CK * ch + NV * g);
    Op<PREC, 8> xt[NAB][NJ];
#pragma unroll
    for (int bb = 0; bb < NAB; ++bb)
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        xt[bb][j] = load_op_split<PREC>(xhT, xlT, (size_t)(16 * bb + c) * Npad + t0 + 32 * j + 4 * g);
    const int pown = t0 + lane;
    const bool vown = lane < 16 * PB && pown < N;
    const float fown = vown ? f[pown] : 0.f;

#pragma unroll
    for (int gk = 0; gk < GW; ++gk) {
      const int k = kw + gk;
      if (k >= K) break;
      const size_t qoff = (size_t)k * DP * DP;
      f32x4 acc[PB][NAB];
#pragma unroll
      for (int ab = 0; ab < NAB; ++ab) {
        const float nc = ops.negc[(size_t)k * DP + 16 * ab + c];
#pragma unroll
        for (int pb = 0; pb < PB; ++pb) acc[pb][ab] = f32x4{nc, nc, nc, nc};
      }
#pragma unroll
      for (int ab = 0; ab < NAB; ++ab) {
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
          if (CK * ch > 16 * ab + 15) continue;
          const Op<PREC, NV> qb =
              load_op<PREC, NV>(Qh + qoff, Ql ? Ql + qoff : nullptr, (size_t)(16 * ab + c) * DP + CK * ch + NV * g);
#pragma unroll
          for (int pb = 0; pb < PB; ++pb) acc[pb][ab] = mma<PREC, NV>(xa[pb][ch], qb, acc[pb][ab]);
        }
      }
      // w for the point this lane owns, then broadcast through LDS to the
      // lanes holding that point's row of Y
      float w = 0.f;
      if (vown) w = __expf(beta[(size_t)k * Npad + pown] - fown) * ctv;
      aacc[gk] += w;
      wsh[wv][lane] = w;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      f32x4 wr[PB];
#pragma unroll
      for (int pb = 0; pb < PB; ++pb) wr[pb] = *reinterpret_cast<const f32x4*>(&wsh[wv][16 * pb + 4 * g]);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
#pragma unroll
        for (int ab = 0; ab < NAB; ++ab) {
          float v[8];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            v[e] = acc[2 * j][ab][e] * wr[2 * j][e];
            v[e + 4] = acc[2 * j + 1][ab][e] * wr[2 * j + 1][e];
          }
          float t = 0.f;
#pragma unroll
          for (int e = 0; e < 8; ++e) t += v[e];
          bacc[gk][ab] += t;
          const Op<PREC, 8> wy = to_op<PREC>(v);
          const int q = ab * (ab + 1) / 2;
#pragma unroll
          for (int bb = 0; bb <= ab; ++bb) macc[gk][q + bb] = mma<PREC, 8>(xt[bb][j], wy, macc[gk][q + bb]);
        }
      }
    }
  }

#pragma unroll
  for (int gk = 0; gk < GW; ++gk) {
    const int k = kw + gk;
    if (k >= K) break;
    float* P = part + (size_t)k * pstride;
#pragma unroll
    for (int ab = 0; ab < NAB; ++ab) {
      const int q = ab * (ab + 1) / 2;
#pragma unroll
      for (int bb = 0; bb <= ab; ++bb)
        *reinterpret_cast<f32x4*>(&P[(size_t)(16 * ab + c) * DP + 16 * bb + 4 * g]) = macc[gk][q + bb];
      float bv = bacc[gk][ab];
      bv += xor_lane(bv, 16);
      bv += xor_lane(bv, 32);
      if (g == 0) P[DP * DP + 16 * ab + c] = bv;
    }
    const float av = wave_sum(aacc[gk]);
    if (lane == 0) P[DP * DP + DP] = av;
  }
}

// ---------------------------------------------------------------------------
// Merge the per-k-range (max, sum) pairs of the points [p0, p0 + 256) into f,
// and a compensated partial sum of f over them (valid in thread 0).
template <typename T>
DEX_DEV void merge_lse_block(const float2* __restrict__ ml, int Sk, int N, int Npad, int p0,
                             T* __restrict__ f, T& ps, T& pe) {
  const int p = p0 + threadIdx.x;
  T v = 0;
  if (p < N) {
    float M = -INFINITY;
    for (int s = 0; s < Sk; ++s) M = fmaxf(M, ml[(size_t)s * Npad + p].x);
    float L = 0.f;
    for (int s = 0; s < Sk; ++s) {
      const float2 e = ml[(size_t)s * Npad + p];
      if (e.y > 0.f) L += e.y * __expf(e.x - M);
    }
    v = (T)(M + logf(L));
    f[p] = v;
  }
  block_comp_sum<T>(v, ps, pe);
}

// F = (sum of compensated partials, fixed order) - N logsumexp(alphas); the
// result is written by thread 0.
template <typename T>
DEX_DEV void finalize_F_block(const T* __restrict__ fpart, int nparts, const T* __restrict__ alphas,
                              int K, int64_t N, T* __restrict__ F) {
  T v = 0, ve = 0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
    T ns, ne;
    two_sum(v, fpart[2 * i], ns, ne);
    v = ns;
    ve += fpart[2 * i + 1] + ne;
  }
  T s = 0, e = 0;
  block_comp_sum<T>(v + ve, s, e);
  if (threadIdx.x == 0) {
    T m = -INFINITY;
    for (int k = 0; k < K; ++k) m = alphas[k] > m ? alphas[k] : m;
    T z = 0;
    for (int k = 0; k < K; ++k) z += dexp<T>(alphas[k] - m);
    const T lse = m + dlog<T>(z);
    F[0] = (s - (T)N * lse) + e;
  }
}

// Reverse, final step for component k: fixed-order compensated sum over the
// S partial slots (stride `sstride` elements), then the gradient assembly.
// Slot layout: M[a*ld + b] (a >= b), b[ld*ld + a], A at ld*ld + ld.
// With `means` non-null the slots hold sum_i w y x~^T instead of M, and
// M = that - b mu^T is formed here (the matrix-core reverse pass contracts
// against x~, which does not depend on the component).
template <typename T, typename TP>
DEX_DEV void bwd_finalize_comp(const TP* __restrict__ part, size_t sstride, int S, int k, int K,
                               int D, int ld, int64_t N, const T* __restrict__ alphas,
                               const T* __restrict__ qd, const T* __restrict__ l,
                               const T* __restrict__ means, T ctv, T* __restrict__ d_alphas,
                               T* __restrict__ d_means, T* __restrict__ d_qd, T* __restrict__ d_l,
                               int accumulate) {
  __shared__ T bsh[64], mdiag[64], Ash;
  const int L = D * (D - 1) / 2;
  const int nM = D * (D + 1) / 2;
  auto comp_sum = [&](size_t off) {
    T s = 0, err = 0;
    for (int sp = 0; sp < S; ++sp) {
      T ns, ne;
      two_sum<T>(s, (T)part[(size_t)sp * sstride + off], ns, ne);
      s = ns;
      err += ne;
    }
    return s + err;
  };
  __syncthreads();
  for (int e = threadIdx.x; e <= D; e += blockDim.x) {
    if (e < D)
      bsh[e] = comp_sum((size_t)ld * ld + e);
    else
      Ash = comp_sum((size_t)ld * ld + ld);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nM; e += blockDim.x) {
    int a = (int)((sqrtf(8.f * e + 1.f) - 1.f) * 0.5f);
    while (a * (a + 1) / 2 > e) --a;
    while ((a + 1) * (a + 2) / 2 <= e) ++a;
    const int b = e - a * (a + 1) / 2;
    T val = comp_sum((size_t)a * ld + b);
    if (means) val -= bsh[a] * means[(size_t)k * D + b];
    if (a > b) {
      T* o = d_l + (size_t)k * L + a * (a - 1) / 2 + b;
      *o = accumulate ? *o - val : -val;
    } else {
      mdiag[a] = val;
    }
  }
  __syncthreads();
  const T A = Ash;
  for (int d = threadIdx.x; d < D; d += blockDim.x) {
    const T eq = dexp<T>(qd[(size_t)k * D + d]);
    const T gq = A - eq * mdiag[d];
    T gm = eq * bsh[d];
    for (int a = d + 1; a < D; ++a) gm += l[(size_t)k * L + a * (a - 1) / 2 + d] * bsh[a];
    T* oq = d_qd + (size_t)k * D + d;
    T* om = d_means + (size_t)k * D + d;
    *oq = accumulate ? *oq + gq : gq;
    *om = accumulate ? *om + gm : gm;
  }
  if (threadIdx.x == 0) {
    T m = -INFINITY;
    for (int j = 0; j < K; ++j) m = alphas[j] > m ? alphas[j] : m;
    T z = 0;
    for (int j = 0; j < K; ++j) z += dexp<T>(alphas[j] - m);
    const T sm = dexp<T>(alphas[k] - m) / z;
    const T ga = A - ctv * (T)N * sm;
    d_alphas[k] = accumulate ? d_alphas[k] + ga : ga;
  }
  __syncthreads();
}

}  // namespace dexk
