// GMM forward as one matrix product over second-order features (D = 64,
// FP16 products, FP32 accumulation).
//
// With P_k = Q_k^T Q_k (Q_k lower triangular, diagonal exp(qd_k)),
//   ||Q_k (x - mu_k)||^2 = sum_{a<=b} c_ab P_k[a][b] x_a x_b
//                          - 2 sum_a (P_k mu_k)_a x_a + mu_k^T P_k mu_k,
// c_ab = 1 on the diagonal and 2 off it. The 2080 products x_a x_b and the 64
// values x_a are the features of a point, the coefficients a column of one
// component, so the Mahalanobis terms of all (i, k) are one product of an
// N x 2144 feature matrix with a 2144 x K coefficient matrix, and
//   beta_ik = (kappa_k - mu^T P mu / 2) - (feature_i . coef_k) / 2.
// The feature matrix is never stored: each wave forms its operand chunks from
// the x rows it holds in registers (one packed FP16 multiply per two features).
//
// Feature slots. A lane of group g (lanes 16g .. 16g+15) holds its point's x
// rotated by 16g: xr[j] = x[(j + 16g) mod 64]. The 2144 features are 272
// packed ops, op o = 17 A + i (A < 16, i < 17), each giving two features:
//   i < 16: xr[A] * xr[B], xr[A] * xr[B+1], B = A + 2i (A even) or A + 1 + 2i
//   i = 16: xr[A] * xr[B*], xr[A] * one,     B* = A + 32 (A even) or A (A odd)
// The rotation maps the same op to a different pair in each lane group; over
// the four groups every unordered pair {a, b} and every x_a appears exactly
// once, except pairs 32 apart, which groups 2 and 3 repeat: their coefficient
// is zero there. Chunk ch (32 contraction values = 8 per lane group) holds the
// ops 4ch .. 4ch+3. The coefficient operand is laid out to match, per lane
// group.
//
// Scaling: the x of each 64-point tile is multiplied by sx = 2^-ex
// (|x sx| < 2^7, ex >= -6, so products and linear features stay below 2^14)
// and "one" is sx, so every feature carries sx^2; the coefficients of
// component k are multiplied by sw_k = 2^ew (largest in [2^13, 2^14)). The
// product is rescaled by 2^(2 ex) / sw_k, exactly.
#pragma once

#include "gmm_dev.h"

namespace dexk {
namespace qf {

constexpr int kOps = 272;
constexpr int kChunks = 68;
constexpr int kPass = 32;  // components per pass (two 16-wide tiles)

typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

__host__ __device__ constexpr int op_a(int o) { return o / 17; }
__host__ __device__ constexpr int op_i(int o) { return o % 17; }
__host__ __device__ constexpr int op_b(int o) {
  return op_i(o) < 16 ? (op_a(o) % 2 == 0 ? op_a(o) + 2 * op_i(o) : op_a(o) + 1 + 2 * op_i(o))
                      : (op_a(o) % 2 == 0 ? op_a(o) + 32 : op_a(o));
}

// Coefficient of slot (op o, half h) in lane group g for P (row-major 64x64)
// and Pmu = P mu; zero for the repeated pairs.
DEX_DEV float coef(int o, int h, int g, const float (*P)[65], const float* Pmu) {
  const int A = op_a(o), i = op_i(o), B = op_b(o);
  if (i == 16 && h == 1) return -2.f * Pmu[(A + 16 * g) & 63];
  const int bb = i < 16 ? B + h : B;
  const int d = bb - A;  // 0 .. 32, no wrap before the rotation
  if (d == 32 && g >= 2) return 0.f;
  const int a = (A + 16 * g) & 63, b = (bb + 16 * g) & 63;
  return (a == b ? 1.f : 2.f) * P[a][b];
}

// The 8 FP16 features of chunk ch for a lane whose rotated x is xr2 (packed
// pairs, xr2[j] = (xr[2j], xr[2j+1])) and one = sx.
template <int CH>
DEX_DEV h8 features(const h2 (&xr2)[32], _Float16 one) {
  h8 z;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    constexpr int o0 = 4 * CH;
    const int o = o0 + q;
    const int A = op_a(o), B = op_b(o);
    const _Float16 xa = (A & 1) ? xr2[A >> 1][1] : xr2[A >> 1][0];
    const h2 av = {xa, xa};
    h2 bv;
    if (op_i(o) < 16) {
      bv = xr2[B >> 1];
    } else {
      const _Float16 xb = (B & 1) ? xr2[B >> 1][1] : xr2[B >> 1][0];
      bv = h2{xb, one};
    }
    const h2 p = av * bv;
    z[2 * q] = p[0];
    z[2 * q + 1] = p[1];
  }
  return z;
}

}  // namespace qf
}  // namespace dexk
