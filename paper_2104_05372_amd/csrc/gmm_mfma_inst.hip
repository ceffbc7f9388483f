// Grid kernels of the single-instance GMM matrix-core path for one operand
// precision, selected at compile time by DEX_PREC (0 FP32, 1 BF16, 2 split-BF16).
#include <algorithm>

#include <utility>

#include "gmm_host.h"
#include "gmm_qf.h"
#include "internal.h"

#ifndef DEX_PREC
#error "compile with -DDEX_PREC=0|1|2"
#endif

namespace dexk {

// Operand preparation in one launch: blocks 0 .. K-1 prepare component k
// (Q~, -c~, kappa), the others one 64-point tile of x~ and x~^T each.
template <int PREC, int DP>
__global__ void __launch_bounds__(256) k_prep(const float* __restrict__ x, int N, int D, int Npad,
                                              int K, const float* __restrict__ alphas,
                                              const float* __restrict__ means,
                                              const float* __restrict__ qd,
                                              const float* __restrict__ l,
                                              typename Store<PREC>::S* xh,
                                              typename Store<PREC>::S* xl,
                                              typename MomT<MomOf<PREC>::MP>::S* xhT,
                                              typename MomT<MomOf<PREC>::MP>::S* xlT,
                                              typename Store<PREC>::S* Qh,
                                              typename Store<PREC>::S* Ql, float* negc,
                                              float* kappa, float* __restrict__ shift) {
  // every block computes the origin itself (one launch less); block 0 keeps it
  // for the reverse pass
  __shared__ float csh[64];
  block_shift(means, K, D, csh);
  if (blockIdx.x == 0 && threadIdx.x < 64) shift[threadIdx.x] = csh[threadIdx.x];
  if ((int)blockIdx.x < K)
    prep_q_comp<PREC, DP>(alphas, means, qd, l, D, blockIdx.x, Qh, Ql, negc, kappa, csh);
  else
    prep_x_tile<PREC, DP>(x, N, D, Npad, (blockIdx.x - K) * 64, xh, xl, xhT, xlT, nullptr, csh);
}

// The grid kernels split their work evenly over the waves (split_lo), so every
// wave does the same amount of work whatever N, K and the CU count are, and no
// partly filled second wave of blocks trails the launch. Workgroups are
// dispatched to the 8 XCDs round-robin, each XCD with its own L2: XCD x
// (blocks b with b % 8 == x) takes the x-th eighth of the point tiles for all
// component groups, so the x~ tiles it streams (1/8 of x~) stay in its L2
// while every group reads them. Forward units on an XCD are (group of NKQ
// components, 16-point tile), group-major: a wave loads a group's operands
// once and streams its tiles; its range covers at most a few groups. The grid
// is a multiple of 8 blocks.
template <int DP, int PREC, int NKQ, int CK, int PD>
__global__ void __launch_bounds__(256) k_gmm_fwd(MfmaOps ops, int Npad, int K, int ngroups,
                                                 float* __restrict__ beta,
                                                 float2* __restrict__ ml) {
  // wave index, made explicitly uniform so the split arithmetic and the loop
  // control stay in scalar registers
  const int xcd = blockIdx.x & 7;
  const int wl = (blockIdx.x >> 3) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int Wx = (gridDim.x >> 3) * 4;
  const int64_t ntiles = Npad / 16;
  const int64_t t0 = xcd * ntiles / 8, nix = (xcd + 1) * ntiles / 8 - t0;
  const int64_t Tx = (int64_t)ngroups * nix;
  int64_t pos = split_lo(wl, Tx, Wx);
  const int64_t hi = split_lo(wl + 1, Tx, Wx);
  while (pos < hi) {
    const int64_t grp = pos / nix;
    const int64_t ta = pos - grp * nix;
    const int64_t tb = min<int64_t>(nix, ta + (hi - pos));
    fwd_unit_kq<DP, PREC, NKQ, CK, PD>(ops, Npad, K, (int)grp * NKQ, (int)(t0 + ta),
                                       (int)(t0 + tb), beta, ml + (size_t)grp * Npad);
    pos += tb - ta;
  }
}

// Reverse units are (group of GW components, 32-point step); XCD x takes the
// x-th eighth of the steps for all groups (its slice of x~^T stays in its L2),
// group-major on the XCD. For each group it touches a wave writes one partial
// moment slot: slot x * SX + (rank of the wave among the XCD's waves on that
// group). Only the first min(Wx, units of the XCD) waves of an XCD take part,
// so each of them owns at least one unit and the ranks of a group's waves are
// contiguous (no unwritten slot between them). Waves share no LDS and meet at
// no barrier, so the others leave at once.
template <int DP, int PREC, int GW, bool DB>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(DB ? 1 : 2)))
k_gmm_bwd(MfmaOps ops, int N, int Npad, int K, int SX,
                                                 const float* __restrict__ beta,
                                                 const float* __restrict__ f,
                                                 const float* __restrict__ ct,
                                                 float* __restrict__ part) {
  // wave index, made explicitly uniform so the split arithmetic and the loop
  // control stay in scalar registers
  const int xcd = blockIdx.x & 7;
  const int wl = (blockIdx.x >> 3) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const size_t E = mom_slot(DP);
  const int64_t nsteps = Npad / 32, nkg = (K + GW - 1) / GW;
  const int64_t s0x = xcd * nsteps / 8, nsx = (xcd + 1) * nsteps / 8 - s0x;
  const int64_t Tx = nkg * nsx;
  const int64_t Wx = min<int64_t>((gridDim.x >> 3) * 4, Tx);
  if (wl >= Wx) return;
  int64_t pos = split_lo(wl, Tx, Wx);
  const int64_t hi = split_lo(wl + 1, Tx, Wx);
  while (pos < hi) {
    const int64_t kg = pos / nsx;
    const int64_t s0 = pos - kg * nsx;
    const int64_t s1 = min<int64_t>(nsx, s0 + (hi - pos));
    const int slot = xcd * SX + (int)(wl - split_owner(kg * nsx, Tx, Wx));
    bwd_mom_unit<DP, MomOf<PREC>::MP, GW, DB>(ops.xhT, ops.xlT, N, Npad, K, (int)kg * GW,
                                          (int)((s0x + s0) * 32), (int)((s0x + s1) * 32), beta,
                                          f, ct[0], part + (size_t)slot * K * E, E);
    pos += s1 - s0;
  }
}

#if DEX_PREC == 1
// ---------------------------------------------------------------------------
// Feature-product forward (see gmm_qf.h). qf_x_tile: per 64-point tile, x~^T
// for the reverse pass and the scaled FP16 copy of x with its exponent.
// qf_w_comp: per component k < Kp, P = Q^T Q, the coefficient operand, kappa'
// and the rescale factor. LDS of the two parts (they share one buffer):
constexpr size_t kQfXLds = 64 * 65 * 4 + 16;  // per tile (a block holds two)
constexpr size_t kQfWLds = 64 * 68 * 4 + 64 * 65 * 4 + (64 + 64 + 12) * 4;

// Two tiles per 256-thread block, 128 threads each (x-tile blocks then fit in
// one round of resident blocks next to the coefficient blocks); a half whose
// tile is past the end only joins the barriers.
DEX_DEV void qf_x_tile(int tix0, int ntiles, char* smem, const float* __restrict__ x, int N,
                       int Npad, _Float16* __restrict__ xhT, _Float16* __restrict__ x16,
                       int* __restrict__ tile_exp, const float* __restrict__ means, int K,
                       float* csh) {
  // x~^T for the reverse pass, and x scaled by the tile's 2^-ex (|x| 2^-ex <
  // 2^7) in FP16, row-major, for the feature products
  const int hf = threadIdx.x >> 7, t = threadIdx.x & 127, tix = tix0 + hf;
  const bool live = tix < ntiles;
  float(*tile)[65] = reinterpret_cast<float(*)[65]>(smem + hf * kQfXLds);
  float* red = reinterpret_cast<float*>(smem + hf * kQfXLds + 64 * 65 * 4);
  const int p0 = tix * 64;
  float mx = 0.f;
  // the tile's x first, then the origin (its loads overlap these)
  float v[32];
#pragma unroll
  for (int i = 0; i < 32; ++i) {
    const int e = t + 128 * i, p = p0 + (e >> 6);
    v[i] = live && p < N ? x[(size_t)p * 64 + (e & 63)] : 0.f;
  }
  block_shift(means, K, 64, csh);
  if (live) {
    // x - c: thread t always meets coordinate t & 63
    const float cs = csh[t & 63];
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      const int e = t + 128 * i, p = p0 + (e >> 6);
      v[i] = p < N ? v[i] - cs : 0.f;
    }
#pragma unroll
    for (int i = 0; i < 32; ++i) {
      const int e = t + 128 * i;
      tile[e >> 6][e & 63] = v[i];
      mx = fmaxf(mx, fabsf(v[i]));
    }
  }
  mx = wave_max(mx);
  if ((t & 63) == 0) red[t >> 6] = mx;
  __syncthreads();
  if (!live) return;  // no barrier follows
  mx = fmaxf(red[0], red[1]);
  // ex >= -6 keeps the linear features (x 2^-ex)(2^-ex) below 2^13 as well
  int ex = -6;
  if (mx > 0.f) {
    int E;
    frexpf(mx, &E);  // mx < 2^E
    ex = max(-6, E - 7);
  }
  if (t == 0) tile_exp[tix] = ex;
  const float sx = ldexpf(1.f, -ex);
  for (int e = t; e < 8 * 64; e += 128) {
    const int pp = e >> 3, b0 = 8 * (e & 7);
    qf::h8 h;
#pragma unroll
    for (int i = 0; i < 8; ++i) h[i] = (_Float16)(tile[pp][b0 + i] * sx);
    *reinterpret_cast<qf::h8*>(x16 + (size_t)(p0 + pp) * 64 + b0) = h;
  }
  for (int e = t; xhT && e < 8 * 64; e += 128) {  // (xhT == nullptr: no reverse operand)
    const int b = e / 8, s0 = 8 * (e % 8);
    float v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int sp = s0 + i, st = sp & 32, q = sp & 31;
      v[i] = tile[st + 4 * (q >> 3) + (q & 3) + 16 * ((q >> 2) & 1)][b];
    }
    mom_store8<MP_F16>(xhT, nullptr, (size_t)b * Npad + p0 + s0, v);
  }
}

DEX_DEV void qf_w_comp(int k, char* smem, const float* __restrict__ alphas,
                       const float* __restrict__ means, const float* __restrict__ qd,
                       const float* __restrict__ l, int K, _Float16* __restrict__ W16,
                       float* __restrict__ kq, float* __restrict__ isc, float* csh,
                       float* __restrict__ keep) {
  constexpr int D = 64, L = D * (D - 1) / 2;
  // Qs: row stride 68 floats keeps 16-byte row pieces aligned for vector reads
  float(*Qs)[68] = reinterpret_cast<float(*)[68]>(smem);
  float(*P)[65] = reinterpret_cast<float(*)[65]>(smem + 64 * 68 * 4);
  float* mus = reinterpret_cast<float*>(smem + 64 * 68 * 4 + 64 * 65 * 4);
  float* Pmu = mus + 64;
  float* red = Pmu + 64;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const size_t ct = (size_t)(k >> 4), c = (size_t)(k & 15);
  auto wpos = [&](int ch, int g, int e) {
    return (((ct * qf::kChunks + ch) * 4 + g) * 16 + c) * 8 + e;
  };
  if (k >= K) {  // padding component: zero coefficients
    for (int s = t; s < qf::kChunks * 32; s += 256)
      W16[wpos(s / 32, (s / 8) & 3, s & 7)] = (_Float16)0.f;
    if (t == 0) {
      kq[k] = 0.f;
      isc[k] = 0.f;
    }
    return;
  }
  // global loads first, issued together
  // branch-free (both loads issued at valid addresses), so all 32 loads are
  // in flight together
  float qv[16], dv[16], lv[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int e = t + 256 * i;
    const int a = e / D, b = e % D;
    dv[i] = qd[(size_t)k * D + a];
    lv[i] = l[(size_t)k * L + (a > b ? a * (a - 1) / 2 + b : 0)];
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int e = t + 256 * i;
    const int a = e / D, b = e % D;
    const float ev = expf(dv[i]);
    qv[i] = a == b ? ev : a > b ? lv[i] : 0.f;
  }
  const float mu_raw = t < D ? means[(size_t)k * D + t] : 0.f;
  const float qd_t = t < D ? qd[(size_t)k * D + t] : 0.f;
  // the origin, once the component's loads are in flight (block 0 keeps it for
  // the reverse pass and forward mode)
  block_shift(means, K, 64, csh);
  if (keep && t < 64) keep[t] = csh[t];
  const float mu_t = t < D ? mu_raw - csh[t] : 0.f;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int e = t + 256 * i;
    Qs[e / D][e % D] = qv[i];
  }
  if (t < D) mus[t] = mu_t;
  const float sqd = wave_sum(qd_t);  // sum of qd_k, complete in wave 0
  __syncthreads();
  // P = Q^T Q: thread t owns column b = t % 64 and rows a = 16 (t / 64) + j;
  // Q[r][a] = 0 for r < a, so the sum starts at r = 16 (t / 64). The 16
  // Q values of a step are 4 broadcast vector reads.
  {
    const int b = t & 63, a0 = 16 * wv;
    float acc[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[j] = 0.f;
#pragma unroll 4
    for (int r = a0; r < D; ++r) {
      const float qb = Qs[r][b];
      const f32x4* qrow = reinterpret_cast<const f32x4*>(&Qs[r][a0]);
#pragma unroll
      for (int j4 = 0; j4 < 4; ++j4) {
        const f32x4 q = qrow[j4];
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[4 * j4 + i] = fmaf(q[i], qb, acc[4 * j4 + i]);
      }
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) P[a0 + j][b] = acc[j];
  }
  __syncthreads();
  // P mu: four threads per row, combined over the quad
  {
    const int a = t >> 2, r = t & 3;
    float v = 0.f;
#pragma unroll 4
    for (int b = r; b < D; b += 4) v = fmaf(P[a][b], mus[b], v);
    v += xor_lane(v, 1);
    v += xor_lane(v, 2);
    if (r == 0) Pmu[a] = v;
  }
  __syncthreads();
  // coefficients (kept in registers), their largest magnitude, then the scaled
  // FP16 operand
  constexpr int kPer = qf::kChunks * 32 / 256;  // 8.5 -> 9 per thread
  float cv[kPer + 1];
  float cm = 0.f;
#pragma unroll
  for (int i = 0; i <= kPer; ++i) {
    const int s = t + 256 * i;
    float v = 0.f;
    if (s < qf::kChunks * 32) {
      const int ch = s / 32, g = (s / 8) & 3, e = s & 7;
      v = qf::coef(4 * ch + (e >> 1), e & 1, g, P, Pmu);
    }
    cv[i] = v;
    cm = fmaxf(cm, fabsf(v));
  }
  const float mpm = wave_sum(t < D ? mus[t] * Pmu[t] : 0.f);
  cm = wave_max(cm);
  if (lane == 0) red[wv] = cm;
  if (t == 0) {
    red[4] = mpm;
    red[5] = sqd;
  }
  __syncthreads();
  cm = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  int ew = 0;
  if (cm > 0.f) {
    int E;
    frexpf(cm, &E);  // cm < 2^E: cm * 2^(14-E) in [2^13, 2^14)
    ew = 14 - E;
  }
  const float sw = ldexpf(1.f, ew);
#pragma unroll
  for (int i = 0; i <= kPer; ++i) {
    const int s = t + 256 * i;
    if (s < qf::kChunks * 32) {
      const int ch = s / 32, g = (s / 8) & 3, e = s & 7;
      W16[wpos(ch, g, e)] = (_Float16)(sw * cv[i]);
    }
  }
  if (t == 0) {
    kq[k] = alphas[k] + red[5] - 0.5f * red[4];
    isc[k] = ldexpf(1.f, -ew);  // 1 / sw
  }
}

// Tangent coefficients of component k for forward mode (the slot layout and
// the power-of-two scaling of qf_w_comp). dQ, the tangent of Q, has diagonal
// exp(qd) dqd and strict lower part dl; the tangent of P = Q^T Q is
// dP = G + G^T with G = Q^T dQ. With r = x~ - mu~ (both about the origin c,
// which the tangent leaves fixed) and dy = dQ r - Q dmu,
//   y . dy = r^T dP r / 2 - r^T P dmu = (feature . dcoef) / 2 + const,
// where dcoef is built from (dP, v = dP mu~ + P dmu) exactly as coef is from
// (P, P mu~), and const = mu~ . (dP mu~ / 2 + P dmu). Hence
//   dbeta = dkq' - (feature . dcoef) / 2,  dkq' = dalpha + sum_d dqd - const.
constexpr size_t kQfTLds = 2 * 64 * 68 * 4 + 2 * 64 * 65 * 4 + (5 * 64 + 8) * 4;

DEX_DEV void qf_tan_comp(int k, char* smem, const float* __restrict__ means,
                         const float* __restrict__ qd, const float* __restrict__ l,
                         const float* __restrict__ da, const float* __restrict__ dm,
                         const float* __restrict__ dq, const float* __restrict__ dl, int K,
                         const float* __restrict__ shift, _Float16* __restrict__ dW16,
                         float* __restrict__ dkq, float* __restrict__ disc) {
  constexpr int D = 64, L = D * (D - 1) / 2;
  float(*Qs)[68] = reinterpret_cast<float(*)[68]>(smem);
  float(*dQs)[68] = reinterpret_cast<float(*)[68]>(smem + 64 * 68 * 4);
  float(*P)[65] = reinterpret_cast<float(*)[65]>(smem + 2 * 64 * 68 * 4);
  float(*G)[65] = reinterpret_cast<float(*)[65]>(smem + 2 * 64 * 68 * 4 + 64 * 65 * 4);
  float* mus = reinterpret_cast<float*>(smem + 2 * 64 * 68 * 4 + 2 * 64 * 65 * 4);
  float* dms = mus + 64;
  float* v = dms + 64;
  float* Pdm = v + 64;
  float* dPm = Pdm + 64;
  float* red = dPm + 64;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const size_t ct = (size_t)(k >> 4), c = (size_t)(k & 15);
  auto wpos = [&](int ch, int g, int e) {
    return (((ct * qf::kChunks + ch) * 4 + g) * 16 + c) * 8 + e;
  };
  if (k >= K) {  // padding component: zero tangent coefficients
    for (int s = t; s < qf::kChunks * 32; s += 256)
      dW16[wpos(s / 32, (s / 8) & 3, s & 7)] = (_Float16)0.f;
    if (t == 0) {
      dkq[k] = 0.f;
      disc[k] = 0.f;
    }
    return;
  }
  // every global load first, issued together (branch-free, valid addresses)
  float dv[16], lv[16], ddv[16], dlv[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int e = t + 256 * i;
    const int a = e / D, b = e % D;
    const size_t li = (size_t)k * L + (a > b ? a * (a - 1) / 2 + b : 0);
    dv[i] = qd[(size_t)k * D + a];
    ddv[i] = dq[(size_t)k * D + a];
    lv[i] = l[li];
    dlv[i] = dl[li];
  }
  const float mu_t = t < D ? means[(size_t)k * D + t] - shift[t] : 0.f;
  const float dm_t = t < D ? dm[(size_t)k * D + t] : 0.f;
  const float dq_t = t < D ? dq[(size_t)k * D + t] : 0.f;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int e = t + 256 * i;
    const int a = e / D, b = e % D;
    const float ev = expf(dv[i]);
    Qs[a][b] = a == b ? ev : a > b ? lv[i] : 0.f;
    dQs[a][b] = a == b ? ev * ddv[i] : a > b ? dlv[i] : 0.f;
  }
  if (t < D) {
    mus[t] = mu_t;
    dms[t] = dm_t;
  }
  const float sdq = wave_sum(dq_t);  // sum of dqd_k, complete in wave 0
  __syncthreads();
  // P = Q^T Q and G = Q^T dQ: thread t owns column b = t % 64 and rows
  // a = 16 (t / 64) + j; Q[r][a] = 0 for r < a, so the sums start at r = a0
  const int b = t & 63, a0 = 16 * wv;
  {
    float accP[16], accG[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) accP[j] = accG[j] = 0.f;
#pragma unroll 4
    for (int r = a0; r < D; ++r) {
      const float qb = Qs[r][b], dqb = dQs[r][b];
      const f32x4* qrow = reinterpret_cast<const f32x4*>(&Qs[r][a0]);
#pragma unroll
      for (int j4 = 0; j4 < 4; ++j4) {
        const f32x4 q = qrow[j4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          accP[4 * j4 + i] = fmaf(q[i], qb, accP[4 * j4 + i]);
          accG[4 * j4 + i] = fmaf(q[i], dqb, accG[4 * j4 + i]);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      P[a0 + j][b] = accP[j];
      G[a0 + j][b] = accG[j];
    }
  }
  __syncthreads();
  // dP = G + G^T, into G (read all, then write)
  {
    float dp[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) dp[j] = G[a0 + j][b] + G[b][a0 + j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) G[a0 + j][b] = dp[j];
  }
  __syncthreads();
  // P dmu and dP mu~: four threads per row, combined over the quad
  {
    const int a = t >> 2, r = t & 3;
    float s1 = 0.f, s2 = 0.f;
#pragma unroll 4
    for (int bb = r; bb < D; bb += 4) {
      s1 = fmaf(P[a][bb], dms[bb], s1);
      s2 = fmaf(G[a][bb], mus[bb], s2);
    }
    s1 += xor_lane(s1, 1);
    s1 += xor_lane(s1, 2);
    s2 += xor_lane(s2, 1);
    s2 += xor_lane(s2, 2);
    if (r == 0) {
      Pdm[a] = s1;
      dPm[a] = s2;
      v[a] = s1 + s2;
    }
  }
  __syncthreads();
  constexpr int kPer = qf::kChunks * 32 / 256;
  float cv[kPer + 1];
  float cm = 0.f;
#pragma unroll
  for (int i = 0; i <= kPer; ++i) {
    const int s = t + 256 * i;
    float val = 0.f;
    if (s < qf::kChunks * 32) {
      const int ch = s / 32, g = (s / 8) & 3, e = s & 7;
      val = qf::coef(4 * ch + (e >> 1), e & 1, g, G, v);
    }
    cv[i] = val;
    cm = fmaxf(cm, fabsf(val));
  }
  const float cst = wave_sum(t < D ? mus[t] * (0.5f * dPm[t] + Pdm[t]) : 0.f);
  cm = wave_max(cm);
  if (lane == 0) red[wv] = cm;
  if (t == 0) {
    red[4] = cst;
    red[5] = sdq;
  }
  __syncthreads();
  cm = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
  int ew = 0;
  if (cm > 0.f) {
    int E;
    frexpf(cm, &E);
    ew = 14 - E;
  }
  const float sw = ldexpf(1.f, ew);
#pragma unroll
  for (int i = 0; i <= kPer; ++i) {
    const int s = t + 256 * i;
    if (s < qf::kChunks * 32) {
      const int ch = s / 32, g = (s / 8) & 3, e = s & 7;
      dW16[wpos(ch, g, e)] = (_Float16)(sw * cv[i]);
    }
  }
  if (t == 0) {
    dkq[k] = da[k] + red[5] - red[4];
    disc[k] = ldexpf(1.f, -ew);
  }
}

// Forward-mode preparation in one launch: blocks [0, Kp) the tangent
// coefficients of one component each, the others two 64-point tiles of the
// scaled FP16 copy of x~ each (no reverse operand).
__global__ void __launch_bounds__(256) k_qf_tan_prep(
    const float* __restrict__ x, int N, int Npad, _Float16* __restrict__ x16,
    int* __restrict__ tile_exp, const float* __restrict__ means, const float* __restrict__ qd,
    const float* __restrict__ l, const float* __restrict__ da, const float* __restrict__ dm,
    const float* __restrict__ dq, const float* __restrict__ dl, int K, int Kp,
    const float* __restrict__ shift, _Float16* __restrict__ dW16, float* __restrict__ dkq,
    float* __restrict__ disc) {
  __shared__ __attribute__((aligned(16))) char smem[kQfTLds > 2 * kQfXLds ? kQfTLds : 2 * kQfXLds];
  // (the x tiles recompute the forward's origin: the same fixed-order sum of
  // the same means, so the same bits as the stored one)
  __shared__ float csh[64];
  if ((int)blockIdx.x < Kp)
    qf_tan_comp(blockIdx.x, smem, means, qd, l, da, dm, dq, dl, K, shift, dW16, dkq, disc);
  else
    qf_x_tile(2 * (blockIdx.x - Kp), Npad / 64, smem, x, N, Npad, nullptr, x16, tile_exp, means, K,
              csh);
}

// One launch for both parts of the preparation: blocks [0, Kp) build the
// coefficient operand of one component each (latency-bound), the others two
// 64-point x tiles each (bandwidth-bound), so the two overlap.
__global__ void __launch_bounds__(256) k_qf_prep(const float* __restrict__ x, int N, int Npad,
                                                 _Float16* __restrict__ xhT,
                                                 _Float16* __restrict__ x16,
                                                 int* __restrict__ tile_exp,
                                                 const float* __restrict__ alphas,
                                                 const float* __restrict__ means,
                                                 const float* __restrict__ qd,
                                                 const float* __restrict__ l, int K, int Kp,
                                                 _Float16* __restrict__ W16,
                                                 float* __restrict__ kq, float* __restrict__ isc,
                                                 float* __restrict__ shift) {
  __shared__ __attribute__((aligned(16))) char smem[kQfWLds > 2 * kQfXLds ? kQfWLds : 2 * kQfXLds];
  // every block computes the origin itself (one launch less); block 0 keeps it
  // for the reverse pass and forward mode
  // (each part issues its own global loads first, so their latency and that of
  // the origin's loads overlap)
  __shared__ float csh[64];
  float* keep = blockIdx.x == 0 ? shift : nullptr;
  if ((int)blockIdx.x < Kp)
    qf_w_comp(blockIdx.x, smem, alphas, means, qd, l, K, W16, kq, isc, csh, keep);
  else
    qf_x_tile(2 * (blockIdx.x - Kp), Npad / 64, smem, x, N, Npad, xhT, x16, tile_exp, means, K,
              csh);
}

// Sum / max over the 16 lanes of a row (DPP: quad swaps, half-row and row
// mirrors); every lane of the row gets the same bits.
template <int CTRL>
DEX_DEV float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
DEX_DEV float row_max16(float v) {
  v = fmaxf(v, dpp<0xB1>(v));
  v = fmaxf(v, dpp<0x4E>(v));
  v = fmaxf(v, dpp<0x141>(v));
  return fmaxf(v, dpp<0x140>(v));
}
// Max over the 16 lanes of a row on order-preserving integer keys of the
// floats (integer max needs no NaN canonicalisation and fuses with DPP).
DEX_DEV int fkey(float v) {
  const int b = __float_as_int(v);
  return b ^ ((b >> 31) & 0x7fffffff);
}
DEX_DEV float funkey(int k) { return __int_as_float(k ^ ((k >> 31) & 0x7fffffff)); }
template <int CTRL>
DEX_DEV int dppi(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
DEX_DEV float row_max16k(int k) {
  k = max(k, dppi<0xB1>(k));
  k = max(k, dppi<0x4E>(k));
  k = max(k, dppi<0x141>(k));
  return funkey(max(k, dppi<0x140>(k)));
}
DEX_DEV float row_sum16(float v) {
  v = v + dpp<0xB1>(v);
  v = v + dpp<0x4E>(v);
  v = v + dpp<0x141>(v);
  return v + dpp<0x140>(v);
}

// One block per CU, 8 waves (2 per SIMD). A unit is (pass of 32 components,
// 64-point tile); XCD x takes the x-th eighth of the tiles for all passes
// (its x copies stay in its L2), pass-major, and a block a contiguous range
// of the XCD's units. The block holds the coefficient operand of its current
// pass in LDS (68 chunks x 2 component tiles x 64 lanes x 16 B = 136 KiB), so
// the waves run their units with no barrier; the block meets only to load the
// next pass. A wave computes its tile as 4 point tiles x NT component tiles:
// per chunk 4 feature sets (4 packed multiplies each) and 4 NT products. NT
// is 2, except in a last pass with at most 16 real components (K = 200: the
// seventh pass holds 8), which runs one component tile: half the products and
// half the coefficient operand.
constexpr int kQfWaves = 8;

template <int CH, int NT, bool TR>
DEX_DEV void qf_chunk(const qf::h2 (&xr)[4][32], _Float16 one, const qf::h8 (&w)[2],
                      f32x4 (&acc)[4][2]) {
  // TR: coefficients as the A operand and features as B (the A and B register
  // layouts of this product are the same): the result is component x point, so
  // a lane holds 4 components of one point (lane (c, g): point c, components
  // 4g .. 4g + 3 of the tile). Otherwise point x component: lane (c, g) holds
  // points 4g .. 4g + 3 of component c.
#pragma unroll
  for (int tt = 0; tt < 4; ++tt) {
    const qf::h8 z = qf::features<CH>(xr[tt], one);
#pragma unroll
    for (int n = 0; n < NT; ++n)
      acc[tt][n] = TR ? __builtin_amdgcn_mfma_f32_16x16x32_f16(w[n], z, acc[tt][n], 0, 0, 0)
                      : __builtin_amdgcn_mfma_f32_16x16x32_f16(z, w[n], acc[tt][n], 0, 0, 0);
  }
#pragma unroll
  for (int tt = 0; tt < 4; ++tt) {
    __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);   // a feature set (4 packed muls)
    __builtin_amdgcn_sched_group_barrier(0x008, NT, 0);  // its products
  }
}

// chunks CH.. with the operands of chunk CH + 1 read from LDS during chunk CH
template <int NT, bool TR, int... CH>
DEX_DEV void qf_chunks(const qf::h2 (&xr)[4][32], _Float16 one, const qf::h8 (*wsh)[2][64],
                       int lane, f32x4 (&acc)[4][2], std::integer_sequence<int, CH...>) {
  qf::h8 w[2][2];
#pragma unroll
  for (int n = 0; n < NT; ++n) w[0][n] = wsh[0][n][lane];
  (
      [&] {
        if constexpr (CH + 1 < qf::kChunks) {
#pragma unroll
          for (int n = 0; n < NT; ++n) w[(CH + 1) & 1][n] = wsh[CH + 1][n][lane];
        }
        qf_chunk<CH, NT, TR>(xr, one, w[CH & 1], acc);
        __builtin_amdgcn_sched_barrier(0);
      }(),
      ...);
}

// x rows of the 64-point tile at pb, rotated by 16g (8 halves per load)
DEX_DEV void qf_load_x(const _Float16* __restrict__ x16, int pb, int c, int g,
                       qf::h2 (&xr)[4][32]) {
#pragma unroll
  for (int tt = 0; tt < 4; ++tt) {
    const _Float16* row = x16 + (size_t)(pb + 16 * tt + c) * 64;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const qf::h8 v = *reinterpret_cast<const qf::h8*>(row + ((8 * j + 16 * g) & 63));
#pragma unroll
      for (int e = 0; e < 4; ++e) xr[tt][4 * j + e] = qf::h2{v[2 * e], v[2 * e + 1]};
    }
  }
}

// TAN = false: the forward (beta and log-sum-exp partials). TAN = true: forward
// mode with the tangent coefficient operand: the same products give dbeta, and
// each (pass, tile) unit writes sum_{i, k} exp(beta_ik - f_i) dbeta_ik over its
// 64 points and 32 components into part[pass * ntiles + tile] (FP64), beta and
// f being the forward's residuals.
template <bool TAN>
__global__ void __launch_bounds__(64 * kQfWaves) k_gmm_fwd_qf(
    const _Float16* __restrict__ x16, int N, int Npad, int K, const _Float16* __restrict__ W16,
    const float* __restrict__ kq, const float* __restrict__ isc, const int* __restrict__ tile_exp,
    int npass, float* __restrict__ beta, float2* __restrict__ ml, const float* __restrict__ fres,
    double* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) qf::h8 wsh[qf::kChunks][2][64];
  const int t = threadIdx.x, lane = t & 63, g = lane >> 4, c = lane & 15;
  const int wv = __builtin_amdgcn_readfirstlane(t >> 6);
  const int64_t ntiles = Npad / 64;
  const int xcd = blockIdx.x & 7, lb = blockIdx.x >> 3, Gx = gridDim.x >> 3;
  const int64_t t0 = xcd * ntiles / 8, ntx = (xcd + 1) * ntiles / 8 - t0;
  // the XCD's units split over its blocks by cost: a unit of a full pass
  // weighs 3, one of a last pass with a single component tile 2 (half the
  // products, the same feature work)
  const bool half_last = K - (npass - 1) * qf::kPass <= 16;
  const int64_t wh = half_last ? 2 : 3, Wfull = 3 * (int64_t)(npass - 1) * ntx,
                Wtot = Wfull + wh * ntx;
  auto unit_at = [&](int64_t w) {  // the first unit that starts at weight >= w
    return w <= Wfull ? (w + 2) / 3 : (int64_t)(npass - 1) * ntx + (w - Wfull + wh - 1) / wh;
  };
  const int64_t ua = unit_at(split_lo(lb, Wtot, Gx)), ub = unit_at(split_lo(lb + 1, Wtot, Gx));
  qf::h2 xr[4][32];
  f32x4 acc[4][2];
  for (int64_t cur = ua; cur < ub;) {
    const int pass = (int)(cur / ntx);
    const int64_t seg = min<int64_t>(ub, (int64_t)(pass + 1) * ntx);
    // the pass's units with NT component tiles
    auto run = [&](auto ntc) {
      constexpr int NT = decltype(ntc)::value;
      // the pass's coefficient operand into LDS (component tiles 2 pass + n,
      // n < NT) by direct loads (global_load_lds_dwordx4: a wave moves one
      // 1 KiB (chunk, tile) piece per instruction, lane i's 16 bytes to the
      // piece's base + 16 i), all of a wave's pieces in flight together and no
      // registers used
      constexpr int kPieces = qf::kChunks * NT;
      __syncthreads();
#pragma unroll
      for (int i = 0; i < (kPieces + kQfWaves - 1) / kQfWaves; ++i) {
        const int q = kQfWaves * i + wv, ch = q / NT, n = q % NT;
        if (kPieces % kQfWaves == 0 || q < kPieces)
          __builtin_amdgcn_global_load_lds(
              W16 + ((((size_t)(2 * pass + n) * qf::kChunks + ch) * 64 + lane) * 8),
              (__attribute__((address_space(3))) void*)&wsh[ch][n][0], 16, 0, 0);
      }
      __syncthreads();  // (waits for the loads: vmcnt(0))
      // the pass's kappa' and rescale factors of the lane's components
      // (16 n + 4 g + i), loaded once per pass (not after every unit's products)
      // (forward: components 16 n + 4 g + i; forward mode: component 16 n + c)
      float kqv[NT][4], iscv[NT][4];
#pragma unroll
      for (int n = 0; n < NT; ++n)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int kc = pass * qf::kPass + 16 * n + (TAN ? c : 4 * g + i);
          kqv[n][i] = kq[kc];
          iscv[n][i] = isc[kc];
        }
      for (int64_t u = cur + wv; u < seg; u += kQfWaves) {
        const int pb = (int)(t0 + (u - (int64_t)pass * ntx)) * 64;  // the tile's first point
        // one prep tile: one scale 2^-ex, and "one" = 2^-ex
        const int ex = tile_exp[pb >> 6];
        const _Float16 one = (_Float16)ldexpf(1.f, -ex);
        qf_load_x(x16, pb, c, g, xr);
#pragma unroll
        for (int tt = 0; tt < 4; ++tt)
#pragma unroll
          for (int n = 0; n < NT; ++n) acc[tt][n] = f32x4{0.f, 0.f, 0.f, 0.f};
        // the products at a higher wave priority than the loads and epilogues,
        // so the two waves of a SIMD drift apart and one's epilogue overlaps
        // the other's products
        __builtin_amdgcn_s_setprio(2);
        qf_chunks<NT, !TAN>(xr, one, wsh, lane, acc,
                            std::make_integer_sequence<int, qf::kChunks>{});
        __builtin_amdgcn_s_setprio(0);
        if constexpr (TAN) {
          // lane (c, g) holds acc[tt][n][i] of point pb + 16 tt + 4 g + i and
          // component pass * 32 + 16 n + c: dbeta = dkq' - disc 2^(2 ex) / 2 *
          // product, weighted by exp(beta - f) (beta read 4 points at a time)
          float lsum = 0.f;
#pragma unroll
          for (int n = 0; n < NT; ++n) {
            const int k = pass * qf::kPass + 16 * n + c;  // < Kp: beta has the row
            const bool vk = k < K;
            const float kk = kqv[n][0], is = ldexpf(iscv[n][0], 2 * ex);
#pragma unroll
            for (int tt = 0; tt < 4; ++tt) {
              const int p0 = pb + 16 * tt + 4 * g;
              const f32x4 bv = *reinterpret_cast<const f32x4*>(beta + (size_t)k * Npad + p0);
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const int p = p0 + i;
                const float fv = fres[min(p, N - 1)];
                const float w = vk && p < N ? __expf(bv[i] - fv) : 0.f;
                lsum = fmaf(w, kk - 0.5f * is * acc[tt][n][i], lsum);
              }
            }
          }
          const double ds = wave_sum((double)lsum);
          if (lane == 0) part[(size_t)pass * ntiles + (pb >> 6)] = ds;
          continue;
        }
        // lane (c, g) holds, for point pb + 16 tt + c, acc[tt][n][i] of
        // component pass * 32 + 16 n + 4 g + i.
        // epilogue: beta = kappa' - isc 2^(2 ex) / 2 * product, stored per
        // component row; the pass's log-sum-exp of each point: the lane's 4 NT
        // components, then the 4 lanes of the point (lanes c, c + 16, c + 32,
        // c + 48) by two lane-pair exchanges; exp(b - M) as exp2(b log2 e -
        // M log2 e). Passes whose components are all real skip the masks.
        auto lse = [&](auto full_t) {
          constexpr bool FULL = decltype(full_t)::value;
          constexpr float kL2e = 1.4426950408889634f;
#pragma unroll
          for (int tt = 0; tt < 4; ++tt) {
            const int p = pb + 16 * tt + c;
            float m = -INFINITY;
#pragma unroll
            for (int n = 0; n < NT; ++n)
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const int k = pass * qf::kPass + 16 * n + 4 * g + i;
                const float b = kqv[n][i] - 0.5f * ldexpf(iscv[n][i], 2 * ex) * acc[tt][n][i];
                acc[tt][n][i] = b;
                beta[(size_t)k * Npad + p] = b;
                if (FULL || k < K) m = fmaxf(m, b);
              }
            m = pair_max32(pair_max16(m));
            const float m2 = m * kL2e;
            float e = 0.f;
#pragma unroll
            for (int n = 0; n < NT; ++n)
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const int k = pass * qf::kPass + 16 * n + 4 * g + i;
                const float ev = __builtin_amdgcn_exp2f(fmaf(acc[tt][n][i], kL2e, -m2));
                e += FULL || k < K ? ev : 0.f;
              }
            e = pair_sum32(pair_sum16(e));
            if (g == 0) ml[(size_t)pass * Npad + p] = make_float2(m, e);
          }
        };
        if (pass * qf::kPass + 16 * NT <= K)
          lse(std::true_type{});
        else
          lse(std::false_type{});
      }
    };
    if (pass == npass - 1 && half_last)
      run(std::integral_constant<int, 1>{});
    else
      run(std::integral_constant<int, 2>{});
    cur = seg;
  }
}
#endif
}  // namespace dexk

namespace dexi {
using namespace dexk;

constexpr int P = DEX_PREC;
using S = typename Store<P>::S;
using SM = typename MomT<MomOf<P>::MP>::S;

template <int DP>
static void prep_dp(const GmmGeom& g, const float* x, const float* alphas, const float* means,
                    const float* qd, const float* l, void* xh, void* xl, void* xhT, void* xlT,
                    void* Qh, void* Ql, float* negc, float* kappa, float* shift,
                    hipStream_t st) {
  hipLaunchKernelGGL((k_prep<P, DP>), dim3((unsigned)(g.K + g.Npad / 64)), dim3(256), 0, st, x,
                     (int)g.N, (int)g.D, (int)g.Npad, (int)g.K, alphas, means, qd, l, (S*)xh,
                     (S*)xl, (SM*)xhT, (SM*)xlT, (S*)Qh, (S*)Ql, negc, kappa, shift);
}

template <>
void mfma_prep<P>(const GmmGeom& g, const float* x, const float* alphas, const float* means,
                  const float* qd, const float* l, void* xh, void* xl, void* xhT, void* xlT,
                  void* Qh, void* Ql, float* negc, float* kappa, float* shift,
                  hipStream_t st) {
  if (g.DP == 16)
    prep_dp<16>(g, x, alphas, means, qd, l, xh, xl, xhT, xlT, Qh, Ql, negc, kappa, shift, st);
  else if (g.DP == 32)
    prep_dp<32>(g, x, alphas, means, qd, l, xh, xl, xhT, xlT, Qh, Ql, negc, kappa, shift, st);
  else
    prep_dp<64>(g, x, alphas, means, qd, l, xh, xl, xhT, xlT, Qh, Ql, negc, kappa, shift, st);
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
  const int blocks = std::max(8, launch_waves(bpc, c.wps) / 4 / 8 * 8);
  sp.W = 4 * blocks;
  hipLaunchKernelGGL((k_gmm_fwd<DP, P, NKQ, CK, PD>), dim3((unsigned)blocks), dim3(256), 0, st, o,
                     (int)g.Npad, (int)g.K, sp.sk, beta, ml);
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

template <int DP, int GW, bool DB>
static FlatSplit bwd_launch(const GmmGeom& g, const BwdCfg& c, const MfmaOps& o, const float* beta,
                            const float* f, const float* ct, float* part, hipStream_t st) {
  FlatSplit sp{};
  sp.gw = GW;
  sp.nsteps = g.Npad / 32;
  const int64_t groups = (g.K + GW - 1) / GW;
  // waves per XCD: as many as resident, at most (slots per XCD - 1) per group,
  // and no more than the units of the smallest XCD slice
  const int64_t sx_cap = bwd_max_slots(g.Npad, g.K) / 8;
  static const int bpc = blocks_per_cu(k_gmm_bwd<DP, P, GW, DB>);
  int64_t wx = launch_waves(bpc, c.wps) / 8 / 4 * 4;
  wx = std::min<int64_t>(wx, (sx_cap - 1) * groups);
  wx = std::min<int64_t>(wx, groups * (sp.nsteps / 8)) / 4 * 4;
  wx = std::max<int64_t>(wx, 4);
  sp.W = (int)wx;  // waves per XCD
  // A group's waves on one XCD are fewer than wx / groups + 2, so SX slots
  // suffice; SX <= sx_cap since wx <= (sx_cap - 1) * groups (the floor of 4
  // waves only applies when groups < 4, i.e. K <= 12, where sx_cap >= 100).
  sp.T = (wx + groups - 1) / groups + 1;  // slots per XCD (SX)
  hipLaunchKernelGGL((k_gmm_bwd<DP, P, GW, DB>), dim3((unsigned)(2 * wx)), dim3(256), 0, st, o,
                     (int)g.N, (int)g.Npad, (int)g.K, (int)sp.T, beta, f, ct, part);
  return sp;
}

template <int DP>
static FlatSplit bwd_dp(const GmmGeom& g, const BwdCfg& c, const MfmaOps& o, const float* beta,
                        const float* f, const float* ct, float* part, hipStream_t st) {
  // the FP16 form with double-buffered rows addresses x~^T rows by 32-bit byte
  // offsets (DP * Npad * 2 < 2^32); beyond that the form without runs
  const bool wide = P == PREC_BF16 && (uint64_t)DP * (uint64_t)g.Npad * 2u >= (1ull << 32);
  if (c.gw == 4 && !c.db) return bwd_launch<DP, 4, false>(g, c, o, beta, f, ct, part, st);
  if (wide) return bwd_launch<DP, 4, false>(g, BwdCfg{4, c.wps, 0}, o, beta, f, ct, part, st);
  if (c.gw == 4) return bwd_launch<DP, 4, true>(g, c, o, beta, f, ct, part, st);
  if (c.gw == 3) return bwd_launch<DP, 3, true>(g, c, o, beta, f, ct, part, st);
  if (c.gw == 2) return bwd_launch<DP, 2, true>(g, c, o, beta, f, ct, part, st);
  return bwd_launch<DP, 1, true>(g, c, o, beta, f, ct, part, st);
}

template <>
FlatSplit mfma_bwd<P>(const GmmGeom& g, const BwdCfg& c, const MfmaOps& o, const float* beta,
                      const float* f, const float* ct, float* part, hipStream_t st) {
  if (g.DP == 16) return bwd_dp<16>(g, c, o, beta, f, ct, part, st);
  if (g.DP == 32) return bwd_dp<32>(g, c, o, beta, f, ct, part, st);
  return bwd_dp<64>(g, c, o, beta, f, ct, part, st);
}


#if DEX_PREC == 1
void qf_prep(const GmmGeom& g, const float* x, const float* alphas, const float* means,
             const float* qd, const float* l, void* xhT, void* x16, int* tile_exp, void* W16,
             float* kq, float* isc, float* shift, hipStream_t st) {
  const int ntiles = (int)(g.Npad / 64);
  const int Kp = (int)((g.K + qf::kPass - 1) / qf::kPass * qf::kPass);
  hipLaunchKernelGGL(k_qf_prep, dim3((unsigned)(Kp + (ntiles + 1) / 2)), dim3(256), 0, st, x,
                     (int)g.N, (int)g.Npad, (_Float16*)xhT, (_Float16*)x16, tile_exp, alphas, means, qd, l,
                     (int)g.K, Kp, (_Float16*)W16, kq, isc, shift);
}

FlatSplit qf_fwd(const GmmGeom& g, const FwdCfg& c, const void* x16, const void* W16,
                 const float* kq, const float* isc, const int* tile_exp, float* beta, float2* ml,
                 hipStream_t st) {
  (void)c;
  FlatSplit sp{};
  sp.sk = (int)((g.K + qf::kPass - 1) / qf::kPass);
  sp.T = (int64_t)sp.sk * (g.Npad / 64);
  sp.W = std::max(8, num_cus() / 8 * 8);  // one block per CU, a multiple of 8
  hipLaunchKernelGGL(k_gmm_fwd_qf<false>, dim3((unsigned)sp.W), dim3(64 * kQfWaves), 0, st,
                     (const _Float16*)x16, (int)g.N, (int)g.Npad, (int)g.K, (const _Float16*)W16,
                     kq, isc, tile_exp, sp.sk, beta, ml, (const float*)nullptr, (double*)nullptr);
  return sp;
}

void qf_tan_prep(const GmmGeom& g, const float* x, const float* means, const float* qd,
                 const float* l, const float* da, const float* dm, const float* dq,
                 const float* dl, const float* shift, void* x16, int* tile_exp, void* dW16,
                 float* dkq, float* disc, hipStream_t st) {
  const int ntiles = (int)(g.Npad / 64);
  const int Kp = (int)((g.K + qf::kPass - 1) / qf::kPass * qf::kPass);
  hipLaunchKernelGGL(k_qf_tan_prep, dim3((unsigned)(Kp + (ntiles + 1) / 2)), dim3(256), 0, st, x,
                     (int)g.N, (int)g.Npad, (_Float16*)x16, tile_exp, means, qd, l, da, dm, dq, dl,
                     (int)g.K, Kp, shift, (_Float16*)dW16, dkq, disc);
}

int64_t qf_tan_parts(const GmmGeom& g) {
  return (g.K + qf::kPass - 1) / qf::kPass * (g.Npad / 64);
}

void qf_jvp(const GmmGeom& g, const void* x16, const void* dW16, const float* dkq,
            const float* disc, const int* tile_exp, const float* beta, const float* f,
            double* part, hipStream_t st) {
  const int npass = (int)((g.K + qf::kPass - 1) / qf::kPass);
  const int blocks = std::max(8, num_cus() / 8 * 8);
  hipLaunchKernelGGL(k_gmm_fwd_qf<true>, dim3((unsigned)blocks), dim3(64 * kQfWaves), 0, st,
                     (const _Float16*)x16, (int)g.N, (int)g.Npad, (int)g.K, (const _Float16*)dW16,
                     dkq, disc, tile_exp, npass, const_cast<float*>(beta), (float2*)nullptr, f,
                     part);
}
#endif

}  // namespace dexi
