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

#include <type_traits>

#include "common.h"

namespace dexk {

// PREC_F16X3: split FP16 operands (hi + lo, 22 significant bits) of values
// the caller has brought into the FP16 range by powers of two.
enum { PREC_F32 = 0, PREC_BF16 = 1, PREC_BF16X3 = 2, PREC_F16X3 = 3 };
constexpr bool prec_split(int PREC) { return PREC == PREC_BF16X3 || PREC == PREC_F16X3; }

template <int PREC>
struct Store {
  using S = __bf16;
};
template <>
struct Store<PREC_F32> {
  using S = float;
};
template <>
struct Store<PREC_F16X3> {
  using S = _Float16;
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
template <int NV>
struct VecT<PREC_F16X3, NV> {
  typedef __attribute__((__vector_size__(NV * sizeof(_Float16)))) _Float16 V;
};

// One lane's NV contraction values (hi [, lo]).
template <int PREC, int NV>
struct Op {
  static constexpr int NS = prec_split(PREC) ? 2 : 1;
  typename VecT<PREC, NV>::V v[NS];
};

template <int PREC, int NV>
DEX_DEV f32x4 mma_chunk(const typename VecT<PREC, NV>::V& a, const typename VecT<PREC, NV>::V& b,
                        f32x4 c) {
  if constexpr (PREC == PREC_F32) {
    // NV steps of 16x16x4; step j takes element j of every lane
#pragma unroll
    for (int j = 0; j < NV; ++j) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j], b[j], c, 0, 0, 0);
  } else if constexpr (PREC == PREC_F16X3) {
    static_assert(NV == 4 || NV == 8, "FP16 operands hold 4 or 8 values per lane");
    if constexpr (NV == 8)
      c = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    else
      c = __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
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
  if constexpr (prec_split(PREC)) {
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
      using H = typename Store<PREC>::S;
      H h = (H)v[e];
      o.v[0][e] = h;
      if constexpr (prec_split(PREC)) o.v[1][e] = (H)(v[e] - (float)h);
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
    using H = typename Store<PREC>::S;
    H h = (H)v;
    hi[off] = h;
    if constexpr (prec_split(PREC)) lo[off] = (H)(v - (float)h);
  }
}

// The value the products actually use for v (hi, or hi + lo).
template <int PREC>
DEX_DEV float rounded(float v) {
  if constexpr (PREC == PREC_F32) {
    return v;
  } else {
    using H = typename Store<PREC>::S;
    H h = (H)v;
    float r = (float)h;
    if constexpr (prec_split(PREC)) r += (float)(H)(v - r);
    return r;
  }
}

// Eight consecutive operand elements (one 16-byte store per array in 16 bits,
// two in FP32); `off` is a multiple of 8.
template <int PREC>
DEX_DEV void store8_split(typename Store<PREC>::S* hi, typename Store<PREC>::S* lo, size_t off,
                          const float (&v)[8]) {
  if constexpr (PREC == PREC_F32) {
    *reinterpret_cast<f32x4*>(hi + off) = f32x4{v[0], v[1], v[2], v[3]};
    *reinterpret_cast<f32x4*>(hi + off + 4) = f32x4{v[4], v[5], v[6], v[7]};
  } else {
    using H = typename Store<PREC>::S;
    typedef __attribute__((__vector_size__(8 * sizeof(H)))) H H8;
    H8 h, l;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      h[i] = (H)v[i];
      if constexpr (prec_split(PREC)) l[i] = (H)(v[i] - (float)h[i]);
    }
    *reinterpret_cast<H8*>(hi + off) = h;
    if constexpr (prec_split(PREC)) *reinterpret_cast<H8*>(lo + off) = l;
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
  if constexpr (NV == 4) {
    // entries 0 / 2 summed over lane pairs 32 apart (lower half keeps entry 0,
    // upper half entry 2), likewise 1 / 3; then over rows 16 apart, row g
    // keeping entry g
    const LanePair a = swap32(v[0], v[2]);
    const LanePair b = swap32(v[1], v[3]);
    const LanePair r = swap16(a.first + a.second, b.first + b.second);
    v[0] = r.first + r.second;
  } else if constexpr (NV == 2) {
    const LanePair a = swap32(v[0], v[1]);
    v[0] = pair_sum16(a.first + a.second);
  } else {
    v[0] = pair_sum16(pair_sum32(v[0]));
  }
}

// Reverse pass as weighted moments. With y = Q~(x~ - mu) and r = x~ - mu, the
// accumulated cotangent of Q_k is M_k = sum_i w y r^T = Q~_k C_k with
// C_k = sum_i w (x~ - mu)(x~ - mu)^T = S_k - u mu^T - mu u^T + A mu mu^T, where
//   S_k = sum_i w_ik x~_i x~_i^T,  u_k = sum_i w_ik x~_i,  A_k = sum_i w_ik.
// So the per-point work of the reverse pass is the symmetric weighted second
// moment S_k (a regular segmented reduction over i for each k, Sec. 6.1.3) plus
// u_k and A_k; Y is not recomputed. The D x D products with Q_k are done once
// per component in the final step.
enum { MP_F32 = 0, MP_F16 = 1, MP_F16X3 = 2 };
template <int PREC>
struct MomOf {
  // (the split-FP16 forward form keeps FP32 moments in the reverse)
  static constexpr int MP =
      PREC == PREC_F32 || PREC == PREC_F16X3 ? MP_F32 : PREC == PREC_BF16 ? MP_F16 : MP_F16X3;
};
template <int MP>
struct MomT {
  using S = _Float16;
  typedef _Float16 V8 __attribute__((ext_vector_type(8)));
  typedef _Float16 V4 __attribute__((ext_vector_type(4)));
  typedef _Float16 V2 __attribute__((ext_vector_type(2)));
  static constexpr int NS = MP == MP_F16X3 ? 2 : 1;
};
template <>
struct MomT<MP_F32> {
  using S = float;
  typedef float V8 __attribute__((ext_vector_type(8)));
  typedef float V4 __attribute__((ext_vector_type(4)));
  typedef float V2 __attribute__((ext_vector_type(2)));
  static constexpr int NS = 1;
};

// Position of point j (0..31) of a 32-point step in the x~^T layout: the 8
// points lane group g contracts over ({4g..4g+3} and {16+4g..16+4g+3}, in the
// order the matrix cores pair them) are stored contiguously at 8g.
__host__ __device__ inline int mom_pos(int j) { return 8 * ((j & 15) >> 2) + (j & 3) + 4 * (j >> 4); }

template <int MP>
DEX_DEV void mom_store(typename MomT<MP>::S* hi, typename MomT<MP>::S* lo, size_t off, float v) {
  if constexpr (MP == MP_F32) {
    hi[off] = v;
  } else {
    const _Float16 h = (_Float16)v;
    hi[off] = h;
    if constexpr (MP == MP_F16X3) lo[off] = (_Float16)(v - (float)h);
  }
}

template <int MP>
DEX_DEV void mom_store8(typename MomT<MP>::S* hi, typename MomT<MP>::S* lo, size_t off,
                        const float (&v)[8]) {
  if constexpr (MP == MP_F32) {
    *reinterpret_cast<f32x4*>(hi + off) = f32x4{v[0], v[1], v[2], v[3]};
    *reinterpret_cast<f32x4*>(hi + off + 4) = f32x4{v[4], v[5], v[6], v[7]};
  } else {
    typename MomT<MP>::V8 h, l;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      h[i] = (_Float16)v[i];
      if constexpr (MP == MP_F16X3) l[i] = (_Float16)(v[i] - (float)h[i]);
    }
    *reinterpret_cast<typename MomT<MP>::V8*>(hi + off) = h;
    if constexpr (MP == MP_F16X3) *reinterpret_cast<typename MomT<MP>::V8*>(lo + off) = l;
  }
}

template <int MP>
DEX_DEV f32x4 mom_mma1(const typename MomT<MP>::V8& a, const typename MomT<MP>::V8& b, f32x4 c) {
  if constexpr (MP == MP_F32) {
#pragma unroll
    for (int j = 0; j < 8; ++j) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j], b[j], c, 0, 0, 0);
  } else {
    c = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
  return c;
}

// Even split of T equal work units over W waves (W <= T, so no wave is idle):
// wave w owns the units [split_lo(w), split_lo(w + 1)).
__host__ __device__ inline int64_t split_lo(int64_t w, int64_t T, int64_t W) { return T * w / W; }
// The wave that owns unit i.
__host__ __device__ inline int64_t split_owner(int64_t i, int64_t T, int64_t W) {
  return ((i + 1) * W - 1) / T;
}
// Number of waves owning part of the units [a, a + len): the partial results
// a segment of that length is split into.
__host__ __device__ inline int split_slots(int64_t a, int64_t len, int64_t T, int64_t W) {
  return (int)(split_owner(a + len - 1, T, W) - split_owner(a, T, W) + 1);
}

// Number of Q~ contraction chunks (depth CK) that meet the lower triangle.
__host__ __device__ constexpr int fwd_nq(int DP, int CK) {
  int n = 0;
  for (int rb = 0; rb < DP / 16; ++rb)
    for (int ch = 0; ch < DP / CK; ++ch)
      if (CK * ch <= 16 * rb + 15) ++n;
  return n;
}

// Operand cache of one instance (FP32 storage, matrix-core forms).
struct MfmaOps {
  const void *xh, *xl;    // x~   [Npad x DP]
  const void *xhT, *xlT;  // x~^T [DP x Npad], moment precision (FP16 or FP32)
  const void *Qh, *Ql;    // Q~   [K x DP x DP]
  const float* negc;      // -c~  [K x DP]
  const float* kappa;     // alphas[k] + sum_d qd[k,d]   [K]
};

// ---------------------------------------------------------------------------
// The origin about which the matrix-core forms take their operands: the mean
// of the first min(K, 16) component means, c[d] = (1/K') sum_{k<K'} means[k][d]
// (a fixed-order sum, the same in every block), zero for d >= D, into csh[64]
// (LDS). Every term of the objective and of its gradient depends on x_i and
// mu_k only through x_i - mu_k = (x_i - c) - (mu_k - c), so moving the origin
// changes no result; a point among the means keeps the 16-bit operands, and
// the expansion ||Q(x - mu)||^2 = x^T P x - 2 (P mu)^T x + mu^T P mu of the
// feature-product form, free of the cancellation that data far from the
// origin would cause. Sixteen means (4 KiB, one load per thread) keep the cost
// per block small: every block of the preparation launch computes it.
// For 256-thread blocks; every thread must call it.
DEX_DEV void block_shift(const float* __restrict__ means, int K, int D, float* csh) {
  constexpr int kMeans = 16;
  __shared__ float part[kMeans][64];
  const int t = threadIdx.x, Kc = K < kMeans ? K : kMeans;
  // thread t: mean t / 16, dimensions 4 (t % 16) .. + 3
  const int k = t >> 4, d0 = 4 * (t & 15);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int d = d0 + i;
    part[k][d] = k < Kc && d < D ? means[(size_t)k * D + d] : 0.f;
  }
  __syncthreads();
  if (t < 64) {
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < kMeans; ++q) s += part[q][t];
    csh[t] = t < D ? s / (float)Kc : 0.f;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Operand preparation for 64 points starting at p0: x~ (row-major) and x~^T,
// zero padded to DP features and Npad points.
// Optional outputs: xh == nullptr skips x~; tmax != nullptr receives the
// largest |x| of the tile (for the scaling of the feature-product forward).
// shift != nullptr: every coordinate of a real point has shift[b] subtracted
// (the origin moved among the means, so 16-bit operands carry
// x - c, not x; every quadratic form in x - mu is unchanged). The result is
// then multiplied by `scale` (a power of two for the split-FP16 form).
template <int PREC, int DP>
DEX_DEV void prep_x_tile(const float* __restrict__ x, int N, int D, int Npad, int p0,
                         typename Store<PREC>::S* xh, typename Store<PREC>::S* xl,
                         typename MomT<MomOf<PREC>::MP>::S* xhT,
                         typename MomT<MomOf<PREC>::MP>::S* xlT, float* tmax = nullptr,
                         const float* __restrict__ shift = nullptr, float scale = 1.f) {
  // (256 threads) the tile's loads are all issued before the first is used
  constexpr int NL = 64 * DP / 256;
  __shared__ float tile[64][DP + 1];
  __shared__ float red[16];
  __syncthreads();
  float mx = 0.f;
  float v[NL];
  // branch-free: every load at a clamped, valid address, selected afterwards
  // (a load under a branch would be waited for before the next is issued)
  // (the shift has DP entries, zero past D)
  float sv[NL];
#pragma unroll
  for (int r = 0; r < NL; ++r) {
    const int e = threadIdx.x + 256 * r, pp = e / DP, b = e % DP, p = p0 + pp;
    v[r] = x[(size_t)min(p, N - 1) * D + min(b, D - 1)];
    sv[r] = shift ? shift[b] : 0.f;
  }
#pragma unroll
  for (int r = 0; r < NL; ++r) {
    const int e = threadIdx.x + 256 * r, pp = e / DP, b = e % DP, p = p0 + pp;
    const bool in = p < N && b < D;
    v[r] = in ? (v[r] - sv[r]) * scale : 0.f;
  }
#pragma unroll
  for (int r = 0; r < NL; ++r) {
    const int e = threadIdx.x + 256 * r;
    tile[e / DP][e % DP] = v[r];
    mx = fmaxf(mx, fabsf(v[r]));
  }
  if (tmax) {
    mx = wave_max(mx);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  }
  __syncthreads();
  if (tmax && threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) mx = fmaxf(mx, red[w]);
    tmax[p0 / 64] = mx;
  }
  // x~: eight consecutive features of a point per store
  for (int e = threadIdx.x; xh && e < 8 * DP; e += blockDim.x) {
    const int pp = e / (DP / 8), b0 = 8 * (e % (DP / 8));
    float v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = tile[pp][b0 + i];
    store8_split<PREC>(xh, xl, (size_t)(p0 + pp) * DP + b0, v);
  }
  // x~^T: eight consecutive storage positions of a feature row per store (p0
  // is a multiple of 64, so the 32-point steps align); position s of a step
  // holds point 4(s/8) + s%4 + 16((s/4)%2)
  for (int e = threadIdx.x; e < 8 * DP; e += blockDim.x) {
    const int b = e / 8, s0 = 8 * (e % 8);
    float v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int sp = s0 + i, st = sp & 32, q = sp & 31;
      v[i] = tile[st + 4 * (q >> 3) + (q & 3) + 16 * ((q >> 2) & 1)][b];
    }
    mom_store8<MomOf<PREC>::MP>(xhT, xlT, (size_t)b * Npad + p0 + s0, v);
  }
}

// Q~_k (dense DP x DP, zero above the diagonal and in the padding), -c~_k and
// kappa_k for one component k (means shifted by shift[] when it is given, as
// the points are in prep_x_tile). Scaled form: Q~ is multiplied by qscale and
// the shifted mean by xscale, so -c~ carries qscale * xscale; kappa is not
// scaled.
template <int PREC, int DP>
DEX_DEV void prep_q_comp(const float* __restrict__ alphas, const float* __restrict__ means,
                         const float* __restrict__ qd, const float* __restrict__ l, int D, int k,
                         typename Store<PREC>::S* Qh, typename Store<PREC>::S* Ql, float* negc,
                         float* kappa, const float* __restrict__ shift = nullptr,
                         float qscale = 1.f, float xscale = 1.f) {
  __shared__ float qs[DP][DP + 1];
  __shared__ float mus[DP], qds[DP];
  const int L = D * (D - 1) / 2;
  __syncthreads();
  if (threadIdx.x < DP) {
    const int a = threadIdx.x;
    mus[a] = a < D ? (means[(size_t)k * D + a] - (shift ? shift[a] : 0.f)) * xscale : 0.f;
    qds[a] = a < D ? qd[(size_t)k * D + a] : 0.f;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < DP * DP; e += blockDim.x) {
    const int a = e / DP, b = e % DP;
    float q = 0.f;
    if (a < D && b < D) {
      if (a == b)
        q = expf(qds[a]);
      else if (a > b)
        q = l[(size_t)k * L + a * (a - 1) / 2 + b];
    }
    qs[a][b] = q * qscale;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < DP * DP / 8; e += blockDim.x) {
    const int a = e / (DP / 8), b0 = 8 * (e % (DP / 8));
    float v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = qs[a][b0 + i];
    store8_split<PREC>(Qh, Ql, (size_t)k * DP * DP + (size_t)a * DP + b0, v);
  }
  if (threadIdx.x < DP) {
    // -c~ with the operand values the products use
    const int a = threadIdx.x;
    float c = 0.f;
    for (int b = 0; b < D; ++b) c = fmaf(rounded<PREC>(qs[a][b]), mus[b], c);
    negc[(size_t)k * DP + a] = -c;
  }
  if (threadIdx.x < 64) {
    float s = 0.f;
    for (int d = threadIdx.x; d < D; d += 64) s += qds[d];
    s = wave_sum(s);
    if (threadIdx.x == 0) kappa[k] = alphas[k] + s;
  }
}

// ---------------------------------------------------------------------------
// Forward unit of one wave: 16*CB points from p0, components [k0, k1).
// The wave builds Y^T (DP x 16*CB) = Q~_k X~^T - c~ from 16x16 tiles (row
// block rb of Q, column block cb of points). A point's squared norm reduces
// across the 4 lane groups, after which each lane owns one point and keeps its
// running log-sum-exp over the k-range. With scaled operands -c~ is multiplied
// by cscale (the points' scale where it differs from the means') and the
// squared norm by sfac (the inverse square of the operands' scale product).
template <int DP, int PREC, int CB, int CK>
DEX_DEV void fwd_unit(const MfmaOps& ops, int N, int Npad, int p0, int k0, int k1,
                      float* __restrict__ beta, float2* __restrict__ ml, float sfac = 1.f,
                      float cscale = 1.f) {
  using S = typename Store<PREC>::S;
  constexpr int NV = CK / 4;
  constexpr int NRB = DP / 16, NCH = DP / CK;
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
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
  if (k0 >= k1) {
    if (owner) ml[p] = make_float2(m, lsum);
    return;
  }

  // operands of component k: the Q~ chunks that meet the lower triangle, -c~
  // and kappa; those of k+1 are loaded while k is computed
  constexpr int NQ = fwd_nq(DP, CK);
  Op<PREC, NV> qa[NQ];
  f32x4 ci[NRB];
  float kap;
  auto load_k = [&](int k, Op<PREC, NV>(&q)[NQ], f32x4(&cc)[NRB], float& kp) {
    const size_t qoff = (size_t)k * DP * DP;
    int n = 0;
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch)
        if (CK * ch <= 16 * rb + 15)
          q[n++] = load_op<PREC, NV>(Qh + qoff, Ql ? Ql + qoff : nullptr,
                                     (size_t)(16 * rb + c) * DP + CK * ch + NV * g);
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
      cc[rb] = *reinterpret_cast<const f32x4*>(ops.negc + (size_t)k * DP + 16 * rb + 4 * g);
    kp = ops.kappa[k];
  };
  auto compute_k = [&](int k, const Op<PREC, NV>(&q)[NQ], const f32x4(&cc)[NRB], float kp) {
    f32x4 acc[CB][NRB];
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) acc[cb][rb] = cc[rb] * cscale;
    int n = 0;
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) {
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) {
        if (CK * ch > 16 * rb + 15) continue;  // chunk wholly above the diagonal
        const Op<PREC, NV>& qq = q[n++];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[cb][rb] = mma<PREC, NV>(qq, xb[cb][ch], acc[cb][rb]);
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
    const float b = kp - 0.5f * (s[0] * sfac);
    // every lane stores: lanes that share a point hold bit-identical totals,
    // and the padded points (p < Npad) have finite residuals nobody reads.
    // No branch here keeps the operand prefetch of the next component alive.
    // The residual streams out (read again only by the reverse pass), so it
    // is stored non-temporally and does not evict the Q~ operands from L2.
    __builtin_nontemporal_store(b, &beta[(size_t)k * Npad + p]);
    const float d = b - m;
    const float e = __expf(-fabsf(d));
    lsum = d > 0.f ? fmaf(lsum, e, 1.f) : lsum + e;
    m = fmaxf(m, b);
  };

  // two operand sets in turn: the next component's loads are in flight while
  // the current one is computed, without register copies. The scheduling
  // barriers keep the issue order loads(k+1), compute(k), store(k),
  // loads(k+2), ...: the wait for a set then never covers the loads issued
  // after it, and the residual store before it has had a whole component's
  // compute to complete (vector memory operations retire in issue order).
  Op<PREC, NV> qb[NQ];
  f32x4 cb2[NRB];
  float kb;
  load_k(k0, qa, ci, kap);
  int k = k0;
  for (; k + 1 < k1; k += 2) {
    load_k(k + 1, qb, cb2, kb);
    __builtin_amdgcn_sched_barrier(0);
    compute_k(k, qa, ci, kap);
    __builtin_amdgcn_sched_barrier(0);
    load_k(min(k + 2, k1 - 1), qa, ci, kap);  // unconditional: no branch between loads and use
    __builtin_amdgcn_sched_barrier(0);
    compute_k(k + 1, qb, cb2, kb);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (k < k1) compute_k(k, qa, ci, kap);
  if (owner) ml[p] = make_float2(m, lsum);
}

// ---------------------------------------------------------------------------
// Forward unit of one wave, components resident: the Q~ operands, -c~ and
// kappa of the NKQ components k0 .. k0+NKQ-1 stay in registers while the
// 16-point tiles t0 .. t1-1 of x~ stream through them (tile t + PD is loaded
// while tile t is computed). Every Q~ chunk load thus serves all the
// wave's tiles, instead of one tile set per load. Per tile, the squared norms
// of the NKQ components reduce across the 4 lane groups so that lane group
// jown(g) owns component k0 + jown of point c; it stores beta (rows padded to
// a multiple of 4 components, so the padding components of the last group
// need no mask) and the tile's (max, sum) log-sum-exp partial over the
// group's valid components.
template <int DP, int PREC, int NKQ, int CK, int PD>
DEX_DEV void fwd_unit_kq(const MfmaOps& ops, int Npad, int K, int k0, int t0, int t1,
                         float* __restrict__ beta, float2* __restrict__ mlg) {
  static_assert(NKQ == 2 || NKQ == 4, "components per wave");
  using S = typename Store<PREC>::S;
  constexpr int NV = CK / 4;
  constexpr int NRB = DP / 16, NCH = DP / CK;
  constexpr int NQ = fwd_nq(DP, CK);
  const int lane = threadIdx.x & 63, g = lane >> 4, c = lane & 15;
  const S* xh = (const S*)ops.xh;
  const S* xl = (const S*)ops.xl;
  const S* Qh = (const S*)ops.Qh;
  const S* Ql = (const S*)ops.Ql;

  Op<PREC, NV> q[NKQ][NQ];
  f32x4 nc[NKQ][NRB];
#pragma unroll
  for (int j = 0; j < NKQ; ++j) {
    const int k = min(k0 + j, K - 1);  // past K: computed, stored in padding rows, not merged
    const size_t qoff = (size_t)k * DP * DP;
    int n = 0;
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch)
        if (CK * ch <= 16 * rb + 15)
          q[j][n++] = load_op<PREC, NV>(Qh + qoff, Ql ? Ql + qoff : nullptr,
                                        (size_t)(16 * rb + c) * DP + CK * ch + NV * g);
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
      nc[j][rb] = *reinterpret_cast<const f32x4*>(ops.negc + (size_t)k * DP + 16 * rb + 4 * g);
  }
  const int jown = NKQ == 4 ? g : g >> 1;
  const int kown = k0 + jown;
  const bool vown = kown < K;
  const float kap = ops.kappa[min(kown, K - 1)];
  float* brow = beta + (size_t)kown * Npad;

  auto load_x = [&](int t, Op<PREC, NV>(&xb)[NCH]) {
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
      xb[ch] = load_op<PREC, NV>(xh, xl, (size_t)(16 * t + c) * DP + CK * ch + NV * g);
  };
  auto products = [&](int j, const Op<PREC, NV>(&xb)[NCH], f32x4(&acc)[NRB]) {
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb) acc[rb] = nc[j][rb];
    int n = 0;
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch)
        if (CK * ch <= 16 * rb + 15) acc[rb] = mma<PREC, NV>(q[j][n++], xb[ch], acc[rb]);
  };
  auto sumsq = [&](const f32x4(&acc)[NRB]) {
    float t2 = 0.f;
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
      for (int i = 0; i < 4; ++i) t2 = fmaf(acc[rb][i], acc[rb][i], t2);
    return t2;
  };
  auto compute = [&](int t, const Op<PREC, NV>(&xb)[NCH]) {
    // the products of component j+1 are issued while the squared norm of
    // component j is summed, so the matrix cores and the vector ALU overlap
    float sq[NKQ];
    f32x4 acc[2][NRB];
    products(0, xb, acc[0]);
#pragma unroll
    for (int j = 0; j < NKQ; ++j) {
      if (j + 1 < NKQ) products(j + 1, xb, acc[(j + 1) & 1]);
      sq[j] = sumsq(acc[j & 1]);
      if (j + 1 < NKQ) {
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one matrix-core op
          __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);  // then three vector ALU ops
        }
      }
    }
    treduce_groups<NKQ>(sq);
    const float b = kap - 0.5f * sq[0];
    const int p = 16 * t + c;
    // lanes that own the same (component, point) hold bit-identical values
    __builtin_nontemporal_store(b, &brow[p]);
    // log-sum-exp over the group's valid components of point p
    float m = pair_max32(vown ? b : -INFINITY);
    if constexpr (NKQ == 4) m = pair_max16(m);
    float e = pair_sum32(vown ? __expf(b - m) : 0.f);
    if constexpr (NKQ == 4) e = pair_sum16(e);
    mlg[p] = make_float2(m, e);
  };

  // ring of PD + 1 tile buffers: tile t + PD is loaded while tile t is
  // computed. Tile indices past t1 - 1 are clamped to it: the last tile is then
  // computed again and stores the same values, which keeps the loop free of
  // branches between loads and their use.
  Op<PREC, NV> xr[PD + 1][NCH];
  if (t0 >= t1) return;
#pragma unroll
  for (int i = 0; i < PD; ++i) load_x(min(t0 + i, t1 - 1), xr[i]);
  for (int t = t0; t < t1; t += PD + 1) {
#pragma unroll
    for (int r = 0; r <= PD; ++r) {
      load_x(min(t + r + PD, t1 - 1), xr[(r + PD) % (PD + 1)]);
      __builtin_amdgcn_sched_barrier(0);
      compute(min(t + r, t1 - 1), xr[r]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// ---------------------------------------------------------------------------
// Partial slot of one (point chunk, component): the lower 16x16 blocks of S in
// matrix-core output order (block q = ab(ab+1)/2 + bb, then lane, then row i),
// u at NBLK*256, A at NBLK*256 + DP; padded to a multiple of 4 floats.
__host__ __device__ inline size_t mom_slot(int DP) {
  const int nb = DP / 16;
  return (size_t)(nb * (nb + 1) / 2) * 256 + DP + 4;
}

// FP16 moments with the point weights computed ahead (software pipelined).
// Step s (32 points) computes the weights of step s + 2 from beta and f loaded
// two steps earlier and writes them to LDS buffer s % 2, reads back those of
// step s + 1 (written during step s - 1) from the other buffer, and runs its
// own products with the weights read during step s - 1. So neither the
// exponentials nor the LDS round trip sit between two steps' products, and
// the scheduler interleaves them with the matrix-core instructions. Within a
// wave LDS instructions execute in issue order; the fence at the end of every
// step keeps the compiler from moving a step's LDS accesses past it. Same
// operands, sums and slot layout as the other moment forms.
template <int DP, int GW>
DEX_DEV void bwd_mom_unit_f16p(const void* xT_hi, int N, int Npad, int K, int kw, int pbeg,
                               int pend, const float* __restrict__ beta,
                               const float* __restrict__ f, float ctv, float* __restrict__ part,
                               size_t pstride) {
  using V8 = typename MomT<MP_F16>::V8;
  constexpr int NB = DP / 16, NBLK = NB * (NB + 1) / 2;
  constexpr int NP = (GW + 1) / 2;  // component pairs
  constexpr int SP = 32;            // points per step
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;
  const int half = lane >> 5, j = lane & 31;
  if (kw >= K) return;
  const _Float16* xh = (const _Float16*)xT_hi;
  __shared__ __attribute__((aligned(16))) _Float16 wsh[2][4][2 * NP][32];

  f32x4 sacc[GW][NBLK];
  f32x4 uq[NB];  // u = x~^T W: 16 dims x 16 component columns per row block
  float aacc[NP];
#pragma unroll
  for (int gk = 0; gk < GW; ++gk)
#pragma unroll
    for (int q = 0; q < NBLK; ++q) sacc[gk][q] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ab = 0; ab < NB; ++ab) uq[ab] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int pp = 0; pp < NP; ++pp) aacc[pp] = 0.f;

  // every load is in bounds: steps past the end reload the last one, f is
  // clamped to N - 1, components past K to K - 1
  // x~^T rows and beta by buffer loads: a wave-uniform resource and step offset
  // (scalar registers) plus a 32-bit per-lane byte offset fixed for the whole
  // unit, so a load needs no vector address arithmetic (the host guarantees
  // DP * Npad * 2 < 2^32; the resources' ranges are not used for clamping)
  const __amdgpu_buffer_rsrc_t xr_ = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<_Float16*>(xh), (short)0, -1, 0x00020000);
  const __amdgpu_buffer_rsrc_t br_ = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(beta + (size_t)kw * Npad), (short)0, -1, 0x00020000);
  uint32_t xoff[NB], boff[NP];
#pragma unroll
  for (int bb = 0; bb < NB; ++bb) xoff[bb] = (uint32_t)((16 * bb + c) * Npad + 8 * g) * 2u;
#pragma unroll
  for (int pp = 0; pp < NP; ++pp)
    boff[pp] = (uint32_t)((min(kw + 2 * pp + half, K - 1) - kw) * Npad + j) * 4u;
  auto load_x = [&](int t, V8(&xt)[NB]) {
#pragma unroll
    for (int bb = 0; bb < NB; ++bb)
      xt[bb] = __builtin_bit_cast(
          V8, __builtin_amdgcn_raw_buffer_load_b128(xr_, xoff[bb], (uint32_t)t * 2u, 0));
  };
  auto load_w = [&](int t, float(&bt)[NP], float& ft) {
    const int p = t + j;
    ft = f[min(p, N - 1)];
#pragma unroll
    for (int pp = 0; pp < NP; ++pp)
      bt[pp] = __builtin_bit_cast(
          float, __builtin_amdgcn_raw_buffer_load_b32(br_, boff[pp], (uint32_t)t * 4u, 0));
  };
  // weights of the step at t (lanes 0-31: component kw + 2pp, lanes 32-63:
  // kw + 2pp + 1, point t + j) into LDS buffer b; zero past N, K or pend
  auto weights = [&](int t, const float(&bt)[NP], float ft, int b) {
    const bool vown = t < pend && t + j < N;
#pragma unroll
    for (int pp = 0; pp < NP; ++pp) {
      const bool vk = kw + 2 * pp + half < K && (GW > 1 || half == 0);
      const float w = vown && vk ? __expf(bt[pp] - ft) * ctv : 0.f;
      aacc[pp] += w;
      wsh[b][wv][2 * pp + half][mom_pos(j)] = (_Float16)w;
    }
  };
  // lane (c, g): the weights of its 8 points for every component (A-operand
  // scaling), and component c's weights of those points (u product)
  auto readw = [&](int b, V8(&wq)[GW], V8& wc) {
#pragma unroll
    for (int gk = 0; gk < GW; ++gk) wq[gk] = *reinterpret_cast<const V8*>(&wsh[b][wv][gk][8 * g]);
    wc = c < GW ? *reinterpret_cast<const V8*>(&wsh[b][wv][c < GW ? c : 0][8 * g]) : V8{};
  };
  auto wave_fence = [] {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  // step at t0 with parity b (= step index % 2): x rows xt (loaded during the
  // previous step), next step's rows into xn, beta/f slot (bs, fs) holding the
  // step at t0 + 2 SP, weights wc / wcc of this step, wn / wnc receive the next
  auto step = [&](int t0, V8(&xt)[NB], V8(&xn)[NB], float(&bs)[NP], float& fs, V8(&wq)[GW],
                  V8& wcc, V8(&wn)[GW], V8& wnc, int b) {
    load_x(t0 + SP < pend ? t0 + SP : t0, xn);
    weights(t0 + 2 * SP, bs, fs, b);
    load_w(min(t0 + 4 * SP, pend - SP), bs, fs);
    readw(b ^ 1, wn, wnc);
#pragma unroll
    for (int bb = 0; bb < NB; ++bb) uq[bb] = mom_mma1<MP_F16>(xt[bb], wcc, uq[bb]);
    // scaled rows of component gk + 1 are formed while component gk's
    // products run (two buffers)
    V8 sa[2][NB];
#pragma unroll
    for (int ab = 0; ab < NB; ++ab) sa[0][ab] = xt[ab] * wq[0];
#pragma unroll
    for (int gk = 0; gk < GW; ++gk) {
      if (gk + 1 < GW) {
#pragma unroll
        for (int ab = 0; ab < NB; ++ab) sa[(gk + 1) & 1][ab] = xt[ab] * wq[gk + 1];
      }
#pragma unroll
      for (int ab = 0; ab < NB; ++ab) {
        const int q0 = ab * (ab + 1) / 2;
#pragma unroll
        for (int bb = 0; bb <= ab; ++bb)
          sacc[gk][q0 + bb] = mom_mma1<MP_F16>(sa[gk & 1][ab], xt[bb], sacc[gk][q0 + bb]);
      }
#pragma unroll
      for (int i = 0; i < NBLK; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one matrix-core op
        __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);  // then two vector ALU ops
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    wave_fence();
  };

  V8 xA[NB], xB[NB], wqA[GW], wqB[GW], wcA, wcB;
  float bA[NP], fA, bB[NP], fB;
  if (pbeg >= pend) return;
  // prologue: weights of steps 0 and 1 into buffers 0 and 1, slots refilled
  // with steps 2 and 3, weights of step 0 read back
  load_x(pbeg, xA);
  load_w(pbeg, bA, fA);
  load_w(min(pbeg + SP, pend - SP), bB, fB);
  weights(pbeg, bA, fA, 0);
  weights(pbeg + SP, bB, fB, 1);
  load_w(min(pbeg + 2 * SP, pend - SP), bA, fA);
  load_w(min(pbeg + 3 * SP, pend - SP), bB, fB);
  wave_fence();
  readw(0, wqA, wcA);
  int t0 = pbeg;
  for (; t0 + SP < pend; t0 += 2 * SP) {
    step(t0, xA, xB, bA, fA, wqA, wcA, wqB, wcB, 0);
    step(t0 + SP, xB, xA, bB, fB, wqB, wcB, wqA, wcA, 1);
  }
  if (t0 < pend) step(t0, xA, xB, bA, fA, wqA, wcA, wqB, wcB, 0);

  // A: lanes 0-31 hold component kw + 2pp, lanes 32-63 component kw + 2pp + 1
  float asum[NP];
#pragma unroll
  for (int pp = 0; pp < NP; ++pp) {
    float v = aacc[pp];
#pragma unroll
    for (int m = 16; m >= 1; m >>= 1) v += xor_lane(v, m);
    asum[pp] = v;
  }
#pragma unroll
  for (int gk = 0; gk < GW; ++gk) {
    const int k = kw + gk;
    if (k >= K) break;
    float* P = part + (size_t)k * pstride;
#pragma unroll
    for (int q = 0; q < NBLK; ++q) *reinterpret_cast<f32x4*>(&P[q * 256 + lane * 4]) = sacc[gk][q];
    // uq[ab] lane (c, g): u of component kw + c, dims 16 ab + 4 g + i
    if (c == gk) {
#pragma unroll
      for (int ab = 0; ab < NB; ++ab)
        *reinterpret_cast<f32x4*>(&P[NBLK * 256 + 16 * ab + 4 * g]) = uq[ab];
    }
    if (lane == 32 * (gk & 1)) P[NBLK * 256 + DP] = asum[gk >> 1];
  }
}

// One wave accumulates S, u, A for components kw .. kw+GW-1 over the points
// [pbeg, pend), 32 per step. Both operands come from x~^T: lane 16 g + c
// holds feature row 16 bb + c and the 8 points of group g (one 16-byte load
// per row block in FP16); the A operand is that row scaled by the point
// weights, the B operand the unscaled row. The weights of a step are computed
// two components at a time (lanes 0-31 one component, 32-63 the next) and
// exchanged through LDS in the same point order (FP16 for the FP16 moments).
template <int DP, int MP, int GW, bool DB = true>
DEX_DEV void bwd_mom_unit_gen(const void* xT_hi, const void* xT_lo, int N, int Npad, int K, int kw,
                              int pbeg, int pend, const float* __restrict__ beta,
                              const float* __restrict__ f, float ctv, float* __restrict__ part,
                              size_t pstride) {
  using MT = MomT<MP>;
  using S = typename MT::S;
  using V8 = typename MT::V8;
  using WT = typename std::conditional<MP == MP_F16, _Float16, float>::type;
  constexpr int NB = DP / 16, NBLK = NB * (NB + 1) / 2, NS = MT::NS;
  constexpr int NP = (GW + 1) / 2;  // component pairs
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, g = lane >> 4, c = lane & 15;
  const int half = lane >> 5, j = lane & 31;
  if (kw >= K) return;
  const S* xh = (const S*)xT_hi;
  const S* xl = (const S*)xT_lo;
  __shared__ __attribute__((aligned(16))) WT wsh[4][2 * NP][32];

  // FP32 form with few blocks: the products of 8 steps go into a tile of their
  // own (sinn), which is then added to sacc, so no FP32 sum runs through more
  // than 16 matrix-core additions plus one per 8 steps (instead of two per
  // step over the whole point range): the rounding error of the weighted
  // moments drops several-fold, which matters where the gradient cancels
  // (dqd = A - exp(qd) M_dd).
  constexpr bool kBlk = MP == MP_F32 && NBLK <= 3;
  f32x4 sacc[GW][NBLK];
  f32x4 sinn[kBlk ? GW : 1][kBlk ? NBLK : 1];
  int nstep = 0;
  float uacc[GW][NB];  // FP32 and split forms: u by lane dot products
  f32x4 uq[NB];        // FP16 form: u = x~^T W, 16 dims x 16 component columns per block
  float aacc[NP];
#pragma unroll
  for (int gk = 0; gk < GW; ++gk) {
#pragma unroll
    for (int q = 0; q < NBLK; ++q) sacc[gk][q] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ab = 0; ab < NB; ++ab) uacc[gk][ab] = 0.f;
  }
  auto fold = [&] {
    if constexpr (kBlk) {
#pragma unroll
      for (int gk = 0; gk < GW; ++gk)
#pragma unroll
        for (int q = 0; q < NBLK; ++q) {
          sacc[gk][q] += sinn[gk][q];
          sinn[gk][q] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
    }
  };
  if constexpr (kBlk) {
#pragma unroll
    for (int gk = 0; gk < GW; ++gk)
#pragma unroll
      for (int q = 0; q < NBLK; ++q) sinn[gk][q] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
#pragma unroll
  for (int ab = 0; ab < NB; ++ab) uq[ab] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int pp = 0; pp < NP; ++pp) aacc[pp] = 0.f;

  // Steps of 32 points; [pbeg, pend) is a multiple of 32 long. The loop runs
  // two steps per iteration with two register sets, so nothing is copied
  // between steps: DB loads the next step's x~^T rows into the other set while
  // the current one is computed (otherwise a step loads its own rows, and the
  // other wave on the SIMD covers the wait); beta and f, which stream from HBM,
  // are loaded two steps ahead into the slot just consumed. Every load is in
  // bounds: steps past the end reload the last one, f is clamped to N-1,
  // components past K to K-1.
  auto load_x = [&](int t, V8(&xt)[NB][NS]) {
#pragma unroll
    for (int bb = 0; bb < NB; ++bb)
#pragma unroll
      for (int s = 0; s < NS; ++s)
        xt[bb][s] = *reinterpret_cast<const V8*>((s == 0 ? xh : xl) +
                                                 (size_t)(16 * bb + c) * Npad + t + 8 * g);
  };
  auto load_w = [&](int t, float(&bt)[NP], float& ft) {
    const int p = t + j;
    ft = f[min(p, N - 1)];
#pragma unroll
    for (int pp = 0; pp < NP; ++pp)
      bt[pp] = __builtin_nontemporal_load(
          &beta[(size_t)min(kw + 2 * pp + half, K - 1) * Npad + p]);
  };
  auto step = [&](int t0, V8(&xt)[NB][NS], V8(&xn)[NB][NS], float(&bc)[NP], float& fc) {
    if constexpr (DB)
      load_x(t0 + 32 < pend ? t0 + 32 : t0, xn);
    else
      load_x(t0, xt);
    __builtin_amdgcn_sched_barrier(0);
    const bool vown = t0 + j < N;
#pragma unroll
    for (int pp = 0; pp < NP; ++pp) {
      const bool vk = kw + 2 * pp + half < K && (GW > 1 || half == 0);
      const float w = vown && vk ? __expf(bc[pp] - fc) * ctv : 0.f;
      aacc[pp] += w;
      wsh[wv][2 * pp + half][mom_pos(j)] = (WT)w;
    }
    load_w(min(t0 + 64, pend - 32), bc, fc);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    typedef WT W8 __attribute__((ext_vector_type(8)));
    // (the lean FP16 form reads each component's weights where it uses them)
    constexpr bool kWq = DB || MP != MP_F16;
    W8 wq[kWq ? GW : 1];
    if constexpr (kWq) {
#pragma unroll
      for (int gk = 0; gk < GW; ++gk) wq[gk] = *reinterpret_cast<const W8*>(&wsh[wv][gk][8 * g]);
    }
    W8 wcol{};  // FP16 form: lane (c, g) holds component c's weights of its 8 points
    if constexpr (MP == MP_F16) {
      if (c < GW) wcol = *reinterpret_cast<const W8*>(&wsh[wv][c][8 * g]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if constexpr (MP == MP_F16) {
#pragma unroll
      for (int bb = 0; bb < NB; ++bb) uq[bb] = mom_mma1<MP>(xt[bb][0], wcol, uq[bb]);
      // DB: scaled rows of component gk + 1 are formed while component gk's
      // products run (two buffers); otherwise each row block is scaled just
      // before its products (fewer registers: more waves per SIMD hide the
      // dependency). Components past K have zero weights, so their products
      // add nothing and no branch is needed.
      V8 sa[DB ? 2 : 1][NB];
      if constexpr (DB) {
#pragma unroll
        for (int ab = 0; ab < NB; ++ab) sa[0][ab] = xt[ab][0] * wq[0];
      }
#pragma unroll
      for (int gk = 0; gk < GW; ++gk) {
        if constexpr (DB) {
          if (gk + 1 < GW) {
#pragma unroll
            for (int ab = 0; ab < NB; ++ab) sa[(gk + 1) & 1][ab] = xt[ab][0] * wq[gk + 1];
          }
        }
#pragma unroll
        for (int ab = 0; ab < NB; ++ab) {
          const int q0 = ab * (ab + 1) / 2;
          if constexpr (!DB)
            sa[0][ab] = xt[ab][0] * *reinterpret_cast<const W8*>(&wsh[wv][gk][8 * g]);
#pragma unroll
          for (int bb = 0; bb <= ab; ++bb)
            sacc[gk][q0 + bb] =
                mom_mma1<MP>(sa[DB ? (gk & 1) : 0][ab], xt[bb][0], sacc[gk][q0 + bb]);
        }
#pragma unroll
        for (int i = 0; i < NBLK; ++i) {
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);
        }
      }
    }
#pragma unroll
    for (int gk = 0; gk < (MP == MP_F16 ? 0 : GW); ++gk) {
      const int k = kw + gk;
      if (k >= K) break;
#pragma unroll
      for (int ab = 0; ab < NB; ++ab) {
        V8 sa[NS];
        if constexpr (MP == MP_F32) {
          float ut = 0.f;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            sa[0][e] = xt[ab][0][e] * wq[gk][e];
            ut = fmaf(xt[ab][0][e], wq[gk][e], ut);
          }
          uacc[gk][ab] += ut;
        } else if constexpr (MP == MP_F16X3) {
          float ut = 0.f;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const float xv = (float)xt[ab][0][e] + (float)xt[ab][1][e];
            const float v = xv * wq[gk][e];
            ut = fmaf(xv, wq[gk][e], ut);
            const _Float16 h = (_Float16)v;
            sa[0][e] = h;
            sa[1][e] = (_Float16)(v - (float)h);
          }
          uacc[gk][ab] += ut;
        }
        const int q0 = ab * (ab + 1) / 2;
#pragma unroll
        for (int bb = 0; bb <= ab; ++bb) {
          if constexpr (kBlk) {
            sinn[gk][q0 + bb] = mom_mma1<MP>(sa[0], xt[bb][0], sinn[gk][q0 + bb]);
          } else {
            f32x4 acc = sacc[gk][q0 + bb];
            if constexpr (MP == MP_F16X3) {
              acc = mom_mma1<MP>(sa[1], xt[bb][0], acc);
              acc = mom_mma1<MP>(sa[0], xt[bb][1], acc);
            }
            sacc[gk][q0 + bb] = mom_mma1<MP>(sa[0], xt[bb][0], acc);
          }
        }
      }
      // the scaling of the next row block overlaps this block's products
#pragma unroll
      for (int i = 0; i < NBLK; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (kBlk) {
      if ((++nstep & 7) == 0) fold();
    }
  };
  V8 xA[NB][NS], xB[NB][NS];
  float bA[NP], fA, bB[NP], fB;
  if (pbeg < pend) {
    if constexpr (DB) load_x(pbeg, xA);
    load_w(pbeg, bA, fA);
    load_w(min(pbeg + 32, pend - 32), bB, fB);
  }
  int t0 = pbeg;
  for (; t0 + 32 < pend; t0 += 64) {
    step(t0, xA, xB, bA, fA);
    step(t0 + 32, xB, xA, bB, fB);
  }
  if (t0 < pend) step(t0, xA, xB, bA, fA);
  fold();

  // A: lanes 0-31 hold component kw + 2pp, lanes 32-63 component kw + 2pp + 1
  float asum[NP];
#pragma unroll
  for (int pp = 0; pp < NP; ++pp) {
    float v = aacc[pp];
#pragma unroll
    for (int m = 16; m >= 1; m >>= 1) v += xor_lane(v, m);
    asum[pp] = v;
  }
#pragma unroll
  for (int gk = 0; gk < GW; ++gk) {
    const int k = kw + gk;
    if (k >= K) break;
    float* P = part + (size_t)k * pstride;
#pragma unroll
    for (int q = 0; q < NBLK; ++q) *reinterpret_cast<f32x4*>(&P[q * 256 + lane * 4]) = sacc[gk][q];
    if constexpr (MP == MP_F16) {
      // uq[ab] lane (c, g): u of component kw + c, dims 16 ab + 4 g + i
      if (c == gk) {
#pragma unroll
        for (int ab = 0; ab < NB; ++ab)
          *reinterpret_cast<f32x4*>(&P[NBLK * 256 + 16 * ab + 4 * g]) = uq[ab];
      }
    } else {
#pragma unroll
      for (int ab = 0; ab < NB; ++ab) {
        float uv = uacc[gk][ab];
        uv += xor_lane(uv, 16);
        uv += xor_lane(uv, 32);
        if (g == 0) P[NBLK * 256 + 16 * ab + c] = uv;
      }
    }
    if (lane == 32 * (gk & 1)) P[NBLK * 256 + DP] = asum[gk >> 1];
  }
}

// The FP16 form with double-buffered rows takes the pipelined-weights unit
// (whose 32-bit row offsets need DP * Npad * 2 < 2^32: the host launches the
// form without double-buffered rows beyond that).
template <int DP, int MP, int GW, bool DB = true>
DEX_DEV void bwd_mom_unit(const void* xT_hi, const void* xT_lo, int N, int Npad, int K, int kw,
                          int pbeg, int pend, const float* __restrict__ beta,
                          const float* __restrict__ f, float ctv, float* __restrict__ part,
                          size_t pstride) {
  if constexpr (MP == MP_F16 && DB)
    bwd_mom_unit_f16p<DP, GW>(xT_hi, N, Npad, K, kw, pbeg, pend, beta, f, ctv, part, pstride);
  else
    bwd_mom_unit_gen<DP, MP, GW, DB>(xT_hi, xT_lo, N, Npad, K, kw, pbeg, pend, beta, f, ctv, part,
                                     pstride);
}

// Final step of the moment form for component k: fixed-order compensated sums
// over the S partial slots, C_k, then M_k = Q_k C_k and the gradient assembly
// (FP32 Q_k from qd and l). shift: the origin the moments were taken about
// (nullptr: zero), subtracted from the means here as from the points. The
// summed second moments, first moments and weight sum are multiplied by m2, m1
// and m0 (the undoing of a scaled form's operand scales and a cotangent left
// out of its weights).
template <int DPM = 64>
DEX_DEV void bwd_finalize_mom(const float* __restrict__ part, size_t sstride, int S, int k, int K,
                              int D, int DP, int64_t N, const float* __restrict__ alphas,
                              const float* __restrict__ means, const float* __restrict__ qd,
                              const float* __restrict__ l, float ctv, float* __restrict__ d_alphas,
                              float* __restrict__ d_means, float* __restrict__ d_qd,
                              float* __restrict__ d_l, int accumulate,
                              const float* __restrict__ shift = nullptr, float m2 = 1.f,
                              float m1 = 1.f, float m0 = 1.f) {
  // Called with 256 threads. C is symmetric; QT holds Q transposed (row
  // stride 68 floats keeps 16-byte rows aligned for vector reads).
  // DPM: the largest DP the caller passes (LDS and registers are sized for it)
  static_assert(DPM == 32 || DPM == 64, "assembly sized for DP <= 32 or <= 64");
  constexpr int NBM = DPM / 16, NBLKM = NBM * (NBM + 1) / 2;
  constexpr int NPV = (NBLKM * 256 + DPM + 1 + 255) / 256;  // slot elements per thread
  constexpr int NQV = DPM * DPM / 256;                       // Q elements per thread
  __shared__ __attribute__((aligned(16))) float C[DPM][DPM + 1];
  __shared__ __attribute__((aligned(16))) float QT[DPM][DPM + 4];
  __shared__ float us[DPM], mus[DPM], vq[DPM], bq[DPM], Ash;
  const int NB = DP / 16, NBLK = NB * (NB + 1) / 2;
  const int L = D * (D - 1) / 2;
  const int t = threadIdx.x;
  // slots in a fixed order; the loads of 8 slots are issued together
  auto comp_sum = [&](size_t off) {
    float s = 0.f, err = 0.f;
    int sp = 0;
    for (; sp + 8 <= S; sp += 8) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(sp + u) * sstride + off];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        float ns, ne;
        two_sum<float>(s, v[u], ns, ne);
        s = ns;
        err += ne;
      }
    }
    for (; sp < S; ++sp) {
      float ns, ne;
      two_sum<float>(s, part[(size_t)sp * sstride + off], ns, ne);
      s = ns;
      err += ne;
    }
    return s + err;
  };
  __shared__ float red[8];
  __shared__ float Ps[NBLKM * 256 + DPM + 4];  // summed slot: S blocks, u, A
  // Every global input is loaded first, each thread's loads issued together,
  // so the block waits for memory once instead of once per phase.
  const int NE = NBLK * 256 + DP + 1;
  float pv[NPV], qv[NQV], av[4];
  if (S == 1) {  // one slot (already reduced): plain loads, issued together
#pragma unroll
    for (int i = 0; i < NPV; ++i) {
      const int e = t + 256 * i;
      pv[i] = e < NE ? part[e] : 0.f;
    }
  } else if (S <= 8) {
    // up to 8 slots (the batched launch's point chunks): every load of the
    // thread's NPV elements issued before the first sum, then the same
    // fixed-order compensated sums
    float v[NPV][8];
#pragma unroll
    for (int i = 0; i < NPV; ++i) {
      const int e = t + 256 * i;
#pragma unroll
      for (int u = 0; u < 8; ++u) v[i][u] = u < S && e < NE ? part[(size_t)u * sstride + e] : 0.f;
    }
#pragma unroll
    for (int i = 0; i < NPV; ++i) {
      float sm = 0.f, err = 0.f;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (u < S) {
          float ns, ne;
          two_sum<float>(sm, v[i][u], ns, ne);
          sm = ns;
          err += ne;
        }
      }
      pv[i] = sm + err;
    }
  } else {
#pragma unroll
    for (int i = 0; i < NPV; ++i) {
      const int e = t + 256 * i;
      pv[i] = e < NE ? comp_sum((size_t)e) : 0.f;
    }
  }
  {
    // element e = t + 256 i of Q (row-major D x D): (a, b) advanced
    // incrementally, no division per element. Both candidate values are loaded
    // (at clamped, valid addresses) and the diagonal exp is always evaluated,
    // so the selection is branch-free and the 32 loads are in flight together.
    const int q256 = 256 / D, r256 = 256 - q256 * D;
    int a = t / D, b = t - (t / D) * D;
    // with D = 1 there is no strict lower part (L = 0, l may be empty): the
    // unused load then reads qd instead
    const float* lsrc = L > 0 ? l + (size_t)k * L : qd + (size_t)k * D;
    float dv[NQV], lv[NQV];
    int sel[NQV];  // 0: zero, 1: diagonal, 2: strict lower
#pragma unroll
    for (int i = 0; i < NQV; ++i) {
      const int e = t + 256 * i;
      const bool in = e < D * D;
      sel[i] = !in ? 0 : a == b ? 1 : a > b ? 2 : 0;
      dv[i] = qd[(size_t)k * D + min(a, D - 1)];
      lv[i] = lsrc[sel[i] == 2 ? a * (a - 1) / 2 + b : 0];
      a += q256;
      b += r256;
      if (b >= D) {
        b -= D;
        ++a;
      }
    }
#pragma unroll
    for (int i = 0; i < NQV; ++i) {
      const float ev = expf(dv[i]);
      qv[i] = sel[i] == 1 ? ev : sel[i] == 2 ? lv[i] : 0.f;
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int j = t + 256 * i;
    av[i] = j < K ? alphas[j] : -INFINITY;
  }
  const float mu_t = t < D ? means[(size_t)k * D + t] - (shift ? shift[t] : 0.f) : 0.f;
  // softmax normaliser of alpha (components past 1024 read in a second pass)
  float am = fmaxf(fmaxf(av[0], av[1]), fmaxf(av[2], av[3]));
  for (int j = t + 1024; j < K; j += 256) am = fmaxf(am, alphas[j]);
  am = wave_max(am);
#pragma unroll
  for (int i = 0; i < NPV; ++i) {
    const int e = t + 256 * i;
    pv[i] *= e < NBLK * 256 ? m2 : e < NBLK * 256 + DP ? m1 : m0;
    if (e < NE) Ps[e] = pv[i];
  }
  // QT and C: rows and columns past D stay zero
  for (int e = t; e < DPM * (DPM + 4); e += 256) (&QT[0][0])[e] = 0.f;
  for (int e = t; e < DPM * (DPM + 1); e += 256) (&C[0][0])[e] = 0.f;
  if ((t & 63) == 0) red[t >> 6] = am;
  if (t < D) mus[t] = mu_t;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NQV; ++i) {
    const int e = t + 256 * i;
    if (e < D * D) QT[e % D][e / D] = qv[i];
  }
  am = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  float az = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i) az += av[i] > -INFINITY ? expf(av[i] - am) : 0.f;
  for (int j = t + 1024; j < K; j += 256) az += expf(alphas[j] - am);
  az = wave_sum(az);
  if ((t & 63) == 0) red[4 + (t >> 6)] = az;
  if (t < D) us[t] = Ps[NBLK * 256 + t];
  if (t == 0) Ash = Ps[NBLK * 256 + DP];
  __syncthreads();
  az = red[4] + red[5] + red[6] + red[7];
  const float A = Ash;
  {
    // C = S - u mu^T - mu u^T + A mu mu^T over the stored lower blocks: the
    // thread's entry of block q = (ab, bb) is pv[q] (element t of the block),
    // at row r = 16 bb + (t/4 % 16) and column s = 16 ab + 4 (t/64) + t % 4
    const int rl = (t >> 2) & 15, sl = 4 * (t >> 6) + (t & 3);
    float ur[NBM], mr[NBM], usv[NBM], msv[NBM];
#pragma unroll
    for (int j = 0; j < NBM; ++j) {
      ur[j] = us[16 * j + rl];
      mr[j] = mus[16 * j + rl];
      usv[j] = us[16 * j + sl];
      msv[j] = mus[16 * j + sl];
    }
#pragma unroll
    for (int q = 0; q < NBLKM; ++q) {
      const int ab = q < 1 ? 0 : q < 3 ? 1 : q < 6 ? 2 : 3;
      const int bb = q - ab * (ab + 1) / 2;
      const int r = 16 * bb + rl, s2 = 16 * ab + sl;
      if (q >= NBLK || r >= D || s2 >= D || r > s2) continue;
      const float v = pv[q] - ur[bb] * msv[ab] - mr[bb] * usv[ab] + A * mr[bb] * msv[ab];
      C[r][s2] = v;
      C[s2][r] = v;
    }
  }
  if (t < D) vq[t] = us[t] - A * mus[t];
  __syncthreads();
  // M = Q C on the matrix cores (FP32 products, FP32 accumulation): wave w
  // computes rows 16w..16w+15 as four 16x16 tiles; Q is lower triangular, so
  // the contraction runs over cc < 16w + 16, four at a time. Lane 16g + c
  // supplies A = Q[16w + c][cc + g] and B = C[cc + g][16n + c], and holds
  // M[16w + 4g + i][16n + c]. Entries past D are zero in QT and C.
  if (DPM == 64 || 16 * (t >> 6) < DPM) {  // (256 threads: waves past DPM / 16 have no rows)
    const int w = t >> 6, lane = t & 63, c = lane & 15, g = lane >> 4;
    const int ce = min(DP, 16 * w + 16);
    f32x4 mt[NBM];
#pragma unroll
    for (int n = 0; n < NBM; ++n) mt[n] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
    for (int cc = 0; cc < ce; cc += 4) {
      const float qa = QT[cc + g][16 * w + c];
#pragma unroll
      for (int n = 0; n < NBM; ++n)
        mt[n] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa, C[cc + g][16 * n + c], mt[n], 0, 0, 0);
    }
#pragma unroll
    for (int n = 0; n < NBM; ++n) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int a = 16 * w + 4 * g + i, b = 16 * n + c;
        if (a >= D || b >= D || a < b) continue;
        const float mv = mt[n][i];
        if (a > b) {
          float* o = d_l + (size_t)k * L + a * (a - 1) / 2 + b;
          *o = accumulate ? *o - mv : -mv;
        } else {
          float* o = d_qd + (size_t)k * D + a;
          const float gq = A - QT[a][a] * mv;
          *o = accumulate ? *o + gq : gq;
        }
      }
    }
  }
  // bq = Q (u - A mu), then d_means = Q^T bq: four threads per row, the
  // partial sums combined over the quad
  {
    const int a = t >> 2, r = t & 3;
    float v = 0.f;
    if (a < D)
      for (int cc = r; cc <= a; cc += 4) v = fmaf(QT[cc][a], vq[cc], v);
    v += xor_lane(v, 1);
    v += xor_lane(v, 2);
    if (a < D && r == 0) bq[a] = v;
  }
  __syncthreads();
  {
    const int d = t >> 2, r = t & 3;
    float gm = 0.f;
    if (d < D)
      for (int a = d + r; a < D; a += 4) gm = fmaf(QT[d][a], bq[a], gm);
    gm += xor_lane(gm, 1);
    gm += xor_lane(gm, 2);
    if (d < D && r == 0) {
      float* om = d_means + (size_t)k * D + d;
      *om = accumulate ? *om + gm : gm;
    }
  }
  if (t == 0) {
    const float ga = A - ctv * (float)N * (expf(alphas[k] - am) / az);
    d_alphas[k] = accumulate ? d_alphas[k] + ga : ga;
  }
  __syncthreads();
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
    // partials in groups of 8, each group's loads issued together, folded in
    // order (online log-sum-exp)
    float M = -INFINITY, L = 0.f;
    for (int s0 = 0; s0 < Sk; s0 += 8) {
      float2 e[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        e[u] = s0 + u < Sk ? ml[(size_t)(s0 + u) * Npad + p] : make_float2(-INFINITY, 0.f);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (e[u].y == 0.f) continue;
        const float d = e[u].x - M;
        const float x = __expf(-fabsf(d));
        L = d > 0.f ? fmaf(L, x, e[u].y) : fmaf(e[u].y, x, L);
        M = fmaxf(M, e[u].x);
      }
    }
    v = (T)(M + logf(L));
    f[p] = v;
  }
  block_comp_sum<T>(v, ps, pe);
}

// Merge of many (max, sum) partials per point: four threads per point (64
// points per 256-thread block), each folding every fourth partial in order
// (online log-sum-exp, loads issued 8 at a time); the four results are then
// combined in thread order. f[p] and a compensated partial sum of f over the
// block's points (valid in thread 0).
template <typename T>
DEX_DEV void merge_lse_quad(const float2* __restrict__ ml, int Sk, int N, int Npad, int p0,
                            T* __restrict__ f, T& ps, T& pe) {
  const int p = p0 + (threadIdx.x >> 2), q = threadIdx.x & 3;
  float M = -INFINITY, L = 0.f;
  if (p < N) {
    for (int s0 = q; s0 < Sk; s0 += 32) {
      float2 e[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int sl = s0 + 4 * u;
        e[u] = sl < Sk ? ml[(size_t)sl * Npad + p] : make_float2(-INFINITY, 0.f);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (e[u].y == 0.f) continue;
        const float d = e[u].x - M;
        const float x = __expf(-fabsf(d));
        L = d > 0.f ? fmaf(L, x, e[u].y) : fmaf(e[u].y, x, L);
        M = fmaxf(M, e[u].x);
      }
    }
  }
  const int base = threadIdx.x & ~3;
  float Mq[4], Lq[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    Mq[i] = __shfl(M, base + i, 64);
    Lq[i] = __shfl(L, base + i, 64);
  }
  float Mt = fmaxf(fmaxf(Mq[0], Mq[1]), fmaxf(Mq[2], Mq[3]));
  float Lt = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (Lq[i] > 0.f) Lt += Lq[i] * __expf(Mq[i] - Mt);
  T v = 0;
  if (p < N && q == 0) {
    v = (T)(Mt + logf(Lt));
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
  // logsumexp(alphas) by the whole block: max, then the sum in a fixed order
  __shared__ T red[16];
  T m = -INFINITY;
  for (int k = threadIdx.x; k < K; k += blockDim.x) m = alphas[k] > m ? alphas[k] : m;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const T om = xor_lane(m, o);
    m = om > m ? om : m;
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  m = red[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = red[w] > m ? red[w] : m;
  T z = 0;
  for (int k = threadIdx.x; k < K; k += blockDim.x) z += dexp<T>(alphas[k] - m);
  T zs = 0, ze = 0;
  block_comp_sum<T>(z, zs, ze);
  if (threadIdx.x == 0) {
    const T lse = m + dlog<T>(zs + ze);
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
