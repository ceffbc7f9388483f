// GMM log-likelihood, one instance: host dispatch, the VALU forms (FP64 or
// FP32, one thread per point) and the merge / finalize kernels shared with the
// matrix-core forms (gmm_dev.h, gmm_mfma_inst.hip).
#include "gmm_host.h"
#include "internal.h"

namespace dexk {

// Forward, VALU: one thread per point, D <= DB. beta is stored [K][N].
template <typename T, int DB>
__global__ void __launch_bounds__(256) gmm_fwd_valu(const T* __restrict__ alphas,
                                                    const T* __restrict__ means,
                                                    const T* __restrict__ qd,
                                                    const T* __restrict__ l,
                                                    const T* __restrict__ x, int N, int D, int K,
                                                    T* __restrict__ beta, T* __restrict__ f,
                                                    T* __restrict__ fpart) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  const bool valid = p < N;
  const int L = D * (D - 1) / 2;
  T xr[DB];
#pragma unroll
  for (int b = 0; b < DB; ++b) xr[b] = (valid && b < D) ? x[(size_t)p * D + b] : T(0);
  T m = -INFINITY, ls = 0;
  for (int k = 0; k < K; ++k) {
    T r[DB];
    T kap = alphas[k];
#pragma unroll
    for (int b = 0; b < DB; ++b) {
      if (b < D) {
        r[b] = xr[b] - means[(size_t)k * D + b];
        kap += qd[(size_t)k * D + b];
      } else {
        r[b] = 0;
      }
    }
    T s = 0;
#pragma unroll
    for (int a = 0; a < DB; ++a) {
      if (a < D) {
        T y = dexp<T>(qd[(size_t)k * D + a]) * r[a];
#pragma unroll
        for (int b = 0; b < a; ++b) y += l[(size_t)k * L + a * (a - 1) / 2 + b] * r[b];
        s += y * y;
      }
    }
    const T bv = kap - T(0.5) * s;
    if (valid) beta[(size_t)k * N + p] = bv;
    const T d = bv - m;
    if (d > 0) {
      ls = ls * dexp<T>(-d) + 1;
      m = bv;
    } else {
      ls += dexp<T>(d);
    }
  }
  T v = 0;
  if (valid) {
    v = m + dlog<T>(ls);
    f[p] = v;
  }
  T s = 0, e = 0;
  block_comp_sum<T>(v, s, e);
  if (threadIdx.x == 0) {
    fpart[2 * blockIdx.x] = s;
    fpart[2 * blockIdx.x + 1] = e;
  }
}

// Reverse, VALU: block (k, point chunk), 64-point tiles. Threads 0..63 put
// w y and r of one point each in LDS; then every thread accumulates its share
// of the D(D+1)/2 + D + 1 sums over the tile.
template <typename T, int DB>
__global__ void __launch_bounds__(256) gmm_bwd_valu(const T* __restrict__ means,
                                                    const T* __restrict__ qd,
                                                    const T* __restrict__ l,
                                                    const T* __restrict__ x, int N, int D, int K,
                                                    int chunk_pts, const T* __restrict__ beta,
                                                    const T* __restrict__ f,
                                                    const T* __restrict__ ct,
                                                    T* __restrict__ part) {
  constexpr int MAXE = (DB * (DB + 1) / 2 + DB + 1 + 255) / 256;
  __shared__ T wy[64][DB + 1], rr[64][DB + 1], wsh[64];
  const int k = blockIdx.x;
  const int L = D * (D - 1) / 2;
  const int nM = D * (D + 1) / 2, nE = nM + D + 1;
  const int pbeg = blockIdx.y * chunk_pts, pend = min(N, pbeg + chunk_pts);
  const T ctv = ct[0];
  int ea[MAXE], eb[MAXE], kind[MAXE];
  T acc[MAXE];
#pragma unroll
  for (int q = 0; q < MAXE; ++q) {
    const int e = threadIdx.x + 256 * q;
    acc[q] = 0;
    kind[q] = 3;
    ea[q] = eb[q] = 0;
    if (e < nM) {
      int a = 0;
      while ((a + 1) * (a + 2) / 2 <= e) ++a;
      ea[q] = a;
      eb[q] = e - a * (a + 1) / 2;
      kind[q] = 0;
    } else if (e < nM + D) {
      ea[q] = e - nM;
      kind[q] = 1;
    } else if (e < nE) {
      kind[q] = 2;
    }
  }
  for (int t0 = pbeg; t0 < pend; t0 += 64) {
    __syncthreads();
    if (threadIdx.x < 64) {
      const int p = t0 + threadIdx.x;
      const bool valid = p < pend;
      T r[DB];
      T w = 0;
#pragma unroll
      for (int b = 0; b < DB; ++b)
        r[b] = (valid && b < D) ? x[(size_t)p * D + b] - means[(size_t)k * D + b] : T(0);
      if (valid) w = dexp<T>(beta[(size_t)k * N + p] - f[p]) * ctv;
#pragma unroll
      for (int a = 0; a < DB; ++a) {
        if (a < D) {
          T y = dexp<T>(qd[(size_t)k * D + a]) * r[a];
#pragma unroll
          for (int b = 0; b < a; ++b) y += l[(size_t)k * L + a * (a - 1) / 2 + b] * r[b];
          wy[threadIdx.x][a] = w * y;
          rr[threadIdx.x][a] = r[a];
        }
      }
      wsh[threadIdx.x] = w;
    }
    __syncthreads();
    const int np = min(64, pend - t0);
#pragma unroll
    for (int q = 0; q < MAXE; ++q) {
      if (kind[q] == 0) {
        for (int pp = 0; pp < np; ++pp) acc[q] += wy[pp][ea[q]] * rr[pp][eb[q]];
      } else if (kind[q] == 1) {
        for (int pp = 0; pp < np; ++pp) acc[q] += wy[pp][ea[q]];
      } else if (kind[q] == 2) {
        for (int pp = 0; pp < np; ++pp) acc[q] += wsh[pp];
      }
    }
  }
  T* P = part + ((size_t)blockIdx.y * K + k) * ((size_t)D * D + D + 1);
#pragma unroll
  for (int q = 0; q < MAXE; ++q) {
    if (kind[q] == 0)
      P[(size_t)ea[q] * D + eb[q]] = acc[q];
    else if (kind[q] == 1)
      P[(size_t)D * D + ea[q]] = acc[q];
    else if (kind[q] == 2)
      P[(size_t)D * D + D] = acc[q];
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_merge_lse(const float2* __restrict__ ml, int Sk, int N,
                                                   int Npad, T* __restrict__ f,
                                                   T* __restrict__ fpart) {
  T s = 0, e = 0;
  merge_lse_block<T>(ml, Sk, N, Npad, blockIdx.x * 256, f, s, e);
  if (threadIdx.x == 0) {
    fpart[2 * blockIdx.x] = s;
    fpart[2 * blockIdx.x + 1] = e;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_merge_lse_quad(const float2* __restrict__ ml, int Sk,
                                                        int N, int Npad, T* __restrict__ f,
                                                        T* __restrict__ fpart) {
  T s = 0, e = 0;
  merge_lse_quad<T>(ml, Sk, N, Npad, blockIdx.x * 64, f, s, e);
  if (threadIdx.x == 0) {
    fpart[2 * blockIdx.x] = s;
    fpart[2 * blockIdx.x + 1] = e;
  }
}

// s + err += a, compensated (two_sum)
DEX_DEV void comp_add(float& s, float& err, float a) {
  float ns, ne;
  two_sum<float>(s, a, ns, ne);
  s = ns;
  err += ne;
}

// Fixed-order compensated sum of each component's partial moment slots (the
// waves that owned part of its group's points), written back into slot 0, so
// the per-component finalize reads a single slot. One thread per element.
// Slots of component k: on each XCD x the waves that owned part of its
// group's steps, in slots x * SX + rank; summed in (x, rank) order.
DEX_DEV int mom_slots(int64_t kg, int x, int64_t nkg, int64_t nsteps, int Wx) {
  const int64_t nsx = (x + 1) * nsteps / 8 - x * nsteps / 8;
  return nsx == 0 ? 0 : split_slots(kg * nsx, nsx, nkg * nsx, min<int64_t>(Wx, nkg * nsx));
}

__global__ void __launch_bounds__(256) k_mom_reduce(float* __restrict__ part, int64_t E, int K,
                                                    int gw, int64_t nsteps, int Wx, int SX) {
  const int64_t i0 = (int64_t)blockIdx.x * 256, i = i0 + threadIdx.x;
  const int64_t nkg = (K + gw - 1) / gw;
  // slot counts: with E >= 256 a block meets at most two components, whose
  // counts 16 threads compute once (64-bit divisions) and share
  __shared__ int Ssh[2][8];
  const int k0 = (int)(i0 / E);
  const bool shared_counts = E >= 256;
  if (shared_counts) {
    if (threadIdx.x < 16) {
      const int kk = k0 + (int)(threadIdx.x >> 3);
      Ssh[threadIdx.x >> 3][threadIdx.x & 7] =
          kk < K ? mom_slots(kk / gw, threadIdx.x & 7, nkg, nsteps, Wx) : 0;
    }
    __syncthreads();
  }
  if (i >= (int64_t)K * E) return;
  const int k = (int)(i / E);
  const int64_t kg = k / gw;
  const size_t stride = (size_t)K * E;
  // the first 5 slots of every XCD are loaded together (one round trip for
  // the usual case: a group's waves on one XCD leave at most wx / groups + 2
  // slots), then summed in (x, rank) order; slots past 5 follow in batches of 4
  int S[8];
  float v[8][5];
#pragma unroll
  for (int x = 0; x < 8; ++x) {
    S[x] = shared_counts ? Ssh[k - k0][x] : mom_slots(kg, x, nkg, nsteps, Wx);
    const float* base = part + (size_t)x * SX * stride + i;
#pragma unroll
    for (int u = 0; u < 5; ++u) v[x][u] = u < S[x] ? base[(size_t)u * stride] : 0.f;
  }
  float s = 0.f, err = 0.f;
#pragma unroll
  for (int x = 0; x < 8; ++x) {
#pragma unroll
    for (int u = 0; u < 5; ++u)
      if (u < S[x]) comp_add(s, err, v[x][u]);
    const float* base = part + (size_t)x * SX * stride + i;
    for (int sp = 5; sp < S[x]; sp += 4) {
      float w[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) w[u] = sp + u < S[x] ? base[(size_t)(sp + u) * stride] : 0.f;
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (sp + u < S[x]) comp_add(s, err, w[u]);
    }
  }
  part[i] = s + err;
}

// Forward mode of the objective on the vector ALU (every D <= 64; FP64, or
// FP32 with x - mu formed exactly in FP64 and rounded once). Block
// (256 points, chunk of kJvpKC components); the components of the chunk are
// staged in LDS in turn. For point i and component k, with r = x_i - mu_k,
//   y = Q_k r, dy = dQ_k r - Q_k dmu_k (dQ: diagonal exp(qd) dqd, strict lower
//   dl), beta = kappa_k - |y|^2 / 2, dbeta = dalpha_k + sum_d dqd_kd - y . dy,
// and the tangent of f_i = LSE_k beta_ik is sum_k exp(beta_ik - f_i) dbeta_ik.
// Each block writes its FP64 sum of these to part[blockIdx.y * gridDim.x +
// blockIdx.x].
constexpr int kJvpKC = 8;

template <typename T, int DB>
__global__ void __launch_bounds__(256) gmm_jvp_valu(
    const T* __restrict__ alphas, const T* __restrict__ means, const T* __restrict__ qd,
    const T* __restrict__ l, const T* __restrict__ x, const T* __restrict__ f, int N, int D, int K,
    const T* __restrict__ da, const T* __restrict__ dm, const T* __restrict__ dq,
    const T* __restrict__ dl, double* __restrict__ part) {
  __shared__ T Qs[DB][DB + 1], dQs[DB][DB + 1];
  __shared__ T mus[DB], qdm[DB], kap[2];
  __shared__ double sh[32];
  const int t = threadIdx.x, p = blockIdx.x * 256 + t;
  const bool valid = p < N;
  const int L = D * (D - 1) / 2;
  T xr[DB];
#pragma unroll
  for (int b = 0; b < DB; ++b) xr[b] = (valid && b < D) ? x[(size_t)p * D + b] : T(0);
  const T fp = valid ? f[p] : T(0);
  double acc = 0.0;
  const int k0 = blockIdx.y * kJvpKC, k1 = min(K, k0 + kJvpKC);
  for (int k = k0; k < k1; ++k) {
    __syncthreads();
    for (int e = t; e < DB * DB; e += 256) {
      const int a = e / DB, b = e % DB;
      T q = 0, dqv = 0;
      if (a < D && b < D) {
        if (a == b) {
          const T ev = dexp<T>(qd[(size_t)k * D + a]);
          q = ev;
          dqv = ev * dq[(size_t)k * D + a];
        } else if (a > b) {
          const size_t li = (size_t)k * L + a * (a - 1) / 2 + b;
          q = l[li];
          dqv = dl[li];
        }
      }
      Qs[a][b] = q;
      dQs[a][b] = dqv;
    }
    if (t < DB) mus[t] = t < D ? means[(size_t)k * D + t] : T(0);
    if (t < 64) {
      T s = 0, ds = 0;
      for (int d = t; d < D; d += 64) {
        s += qd[(size_t)k * D + d];
        ds += dq[(size_t)k * D + d];
      }
      s = wave_sum(s);
      ds = wave_sum(ds);
      if (t == 0) {
        kap[0] = alphas[k] + s;
        kap[1] = da[k] + ds;
      }
    }
    __syncthreads();
    if (t < DB) {  // Q_k dmu_k
      T v = 0;
      for (int b = 0; b <= t && b < D; ++b) v += Qs[t][b] * dm[(size_t)k * D + b];
      qdm[t] = v;
    }
    __syncthreads();
    T r[DB];
#pragma unroll
    for (int b = 0; b < DB; ++b) r[b] = b < D ? (T)((double)xr[b] - (double)mus[b]) : T(0);
    T s = 0, sd = 0;
#pragma unroll
    for (int a = 0; a < DB; ++a) {
      if (a < D) {
        T y = 0, dy = -qdm[a];
#pragma unroll
        for (int b = 0; b <= a; ++b) {
          y += Qs[a][b] * r[b];
          dy += dQs[a][b] * r[b];
        }
        s += y * y;
        sd += y * dy;
      }
    }
    if (valid) acc += (double)(dexp<T>(kap[0] - T(0.5) * s - fp) * (kap[1] - sd));
  }
  acc = block_sum(acc, sh);
  if (t == 0) part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = acc;
}

// dF = (sum of the partials, fixed order) - N sum_k softmax(alpha)_k dalpha_k,
// in FP64.
template <typename T>
__global__ void __launch_bounds__(256) k_jvp_final(const double* __restrict__ part, int64_t np,
                                                   const T* __restrict__ alphas,
                                                   const T* __restrict__ da, int K, int64_t N,
                                                   T* __restrict__ out) {
  __shared__ double sh[32];
  double s = 0.0, am = -INFINITY;
  for (int64_t i = threadIdx.x; i < np; i += 256) s += part[i];
  for (int k = threadIdx.x; k < K; k += 256) am = fmax(am, (double)alphas[k]);
  s = block_sum(s, sh);
  // max over the block (every thread's am), through the same LDS slots
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = -INFINITY;
  __syncthreads();
  {
    double m = am;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  }
  __syncthreads();
  am = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
  double z = 0.0, zd = 0.0;
  for (int k = threadIdx.x; k < K; k += 256) {
    const double e = exp((double)alphas[k] - am);
    z += e;
    zd += e * (double)da[k];
  }
  z = block_sum(z, sh);
  zd = block_sum(zd, sh);
  if (threadIdx.x == 0) out[0] = (T)(s - (double)N * zd / z);
}

template <typename T>
__global__ void __launch_bounds__(256) k_finalize_F(const T* __restrict__ fpart, int nparts,
                                                    const T* __restrict__ alphas, int K, int64_t N,
                                                    T* __restrict__ F) {
  finalize_F_block<T>(fpart, nparts, alphas, K, N, F);
}

template <typename T, typename TP>
__global__ void __launch_bounds__(256) k_bwd_finalize(const TP* __restrict__ part, size_t E, int S,
                                                      int K, int D, int ld, int64_t N,
                                                      const T* __restrict__ alphas,
                                                      const T* __restrict__ qd,
                                                      const T* __restrict__ l,
                                                      const T* __restrict__ means,
                                                      const T* __restrict__ ct,
                                                      T* __restrict__ d_alphas,
                                                      T* __restrict__ d_means, T* __restrict__ d_qd,
                                                      T* __restrict__ d_l, int accumulate) {
  const int k = blockIdx.x;
  bwd_finalize_comp<T, TP>(part + (size_t)k * E, (size_t)K * E, S, k, K, D, ld, N, alphas, qd, l,
                           means, ct[0], d_alphas, d_means, d_qd, d_l, accumulate);
}

// Component k's moment partials, already summed into slot 0 (S = 1); the
// moments were taken about the origin `shift`.
__global__ void __launch_bounds__(256) k_bwd_finalize_mom(
    const float* __restrict__ part, size_t E, int S, int K, int D, int DP, int64_t N,
    const float* __restrict__ alphas, const float* __restrict__ means, const float* __restrict__ qd,
    const float* __restrict__ l, const float* __restrict__ ct, float* __restrict__ d_alphas,
    float* __restrict__ d_means, float* __restrict__ d_qd, float* __restrict__ d_l, int accumulate,
    const float* __restrict__ shift) {
  const int k = blockIdx.x;
  bwd_finalize_mom(part + (size_t)k * E, (size_t)K * E, S, k, K, D, DP, N, alphas, means, qd, l,
                   ct[0], d_alphas, d_means, d_qd, d_l, accumulate, shift);
}

}  // namespace dexk

// ===========================================================================
namespace dexi {
using namespace dexk;

namespace {

struct Shape {
  GmmGeom g;
  int dtype, variant, prec;
  bool mfma;
  size_t tsize;
};

Shape shape_of(const dex_desc& d) {
  Shape s{};
  s.g.N = d.dims[0];
  s.g.D = d.dims[1];
  s.g.K = d.dims[2];
  s.g.DP = s.g.D <= 16 ? 16 : s.g.D <= 32 ? 32 : 64;
  s.g.Npad = (s.g.N + 255) / 256 * 256;
  s.dtype = d.dtype;
  s.variant = d.variant;
  s.tsize = d.dtype == DEX_F64 ? 8 : 4;
  s.mfma = d.dtype == DEX_F32;
  s.prec = d.variant == DEX_GMM_BF16 ? PREC_BF16 : d.variant == DEX_GMM_BF16X3 ? PREC_BF16X3 : PREC_F32;
  return s;
}

// forward candidates: (components resident per wave, waves per SIMD (0: all
// resident), x~ tiles loaded ahead); BF16 config 0 is the feature-product form
// (D = 64 only; other D run config 1 in its place)
const FwdCfg kFwdBF[] = {{0, 0, 0}, {4, 0, 1}, {4, 0, 2}, {2, 0, 1},
                         {2, 0, 2}, {4, 1, 2}, {2, 2, 2}, {0, 1, 0}};
const FwdCfg kFwdF32[] = {{2, 0, 1}, {2, 0, 2}, {2, 2, 1}, {2, 1, 2}};
// reverse candidates: (components per wave, waves per SIMD (0: all resident),
// FP16 form: scaled rows double-buffered (default) or not)
const BwdCfg kBwdBF[] = {{2, 0}, {3, 0}, {4, 0}, {2, 2}, {3, 2}, {4, 0, 0}, {2, 1}, {4, 1}};
const BwdCfg kBwdF32[] = {{2, 0}, {1, 0}, {4, 0}, {2, 2}, {1, 2}};
constexpr int kValuS = 16;

int nfwd(const Shape& s) { return s.prec == PREC_BF16 ? 8 : 4; }
int nbwd(const Shape& s) { return s.prec == PREC_F32 ? 5 : 8; }
size_t mom_es(const Shape& s) { return s.prec == PREC_F32 ? 4 : 2; }
FwdCfg fwd_cfg(const Shape& s, int i) { return s.prec == PREC_BF16 ? kFwdBF[i] : kFwdF32[i]; }
BwdCfg bwd_cfg(const Shape& s, int i) { return s.prec == PREC_F32 ? kBwdF32[i] : kBwdBF[i]; }

struct CacheLayout {
  size_t xh, xl, xhT, xlT, Qh, Ql, negc, kappa, beta, shift, total;
  // feature-product forward (BF16, D = 64): coefficient operand, kappa',
  // rescale factors, scaled FP16 copy of x, per-tile scale exponents
  size_t W16, kq, isc, x16, texp;
};

CacheLayout cache_layout(const Shape& s) {
  CacheLayout c{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align256(bytes);
    return at;
  };
  const GmmGeom& g = s.g;
  if (s.mfma) {
    const size_t es = s.prec == PREC_F32 ? 4 : 2;
    const bool lo = s.prec == PREC_BF16X3;
    c.xh = take(g.Npad * g.DP * es);
    c.xl = lo ? take(g.Npad * g.DP * es) : 0;
    c.xhT = take(g.Npad * g.DP * mom_es(s));
    c.xlT = lo ? take(g.Npad * g.DP * mom_es(s)) : 0;
    c.Qh = take(g.K * g.DP * g.DP * es);
    c.Ql = lo ? take(g.K * g.DP * g.DP * es) : 0;
    c.negc = take(g.K * g.DP * 4);
    c.kappa = take(g.K * 4);
    c.shift = take(64 * 4);
    c.beta = take(beta_rows(g.K) * g.Npad * 4);
    if (qf_eligible(g, s.prec)) {
      const size_t Kp = (size_t)beta_rows(g.K);
      c.W16 = take(Kp / 16 * 68 * 64 * 8 * 2);
      c.kq = take(Kp * 4);
      c.isc = take(Kp * 4);
      c.x16 = take((size_t)g.Npad * 64 * 2);
      c.texp = take((size_t)(g.Npad / 64) * 4);
    }
  } else {
    c.beta = take(g.K * g.N * s.tsize);
  }
  c.total = o;
  return c;
}

MfmaOps ops_of(const Shape& s, const CacheLayout& cl, const char* cache) {
  MfmaOps o;
  const bool lo = s.prec == PREC_BF16X3;
  o.xh = cache + cl.xh;
  o.xl = lo ? cache + cl.xl : nullptr;
  o.xhT = cache + cl.xhT;
  o.xlT = lo ? cache + cl.xlT : nullptr;
  o.Qh = cache + cl.Qh;
  o.Ql = lo ? cache + cl.Ql : nullptr;
  o.negc = (const float*)(cache + cl.negc);
  o.kappa = (const float*)(cache + cl.kappa);
  return o;
}

template <typename T>
void launch_fwd_valu(const Shape& s, const GmmPtrs& in, T* beta, T* f, T* fpart, hipStream_t st) {
  dim3 grid((unsigned)((s.g.N + 255) / 256));
#define DEX_FV(DB)                                                                         \
  hipLaunchKernelGGL((gmm_fwd_valu<T, DB>), grid, dim3(256), 0, st, (const T*)in.alphas, \
                     (const T*)in.means, (const T*)in.qd, (const T*)in.l, (const T*)in.x,  \
                     (int)s.g.N, (int)s.g.D, (int)s.g.K, beta, f, fpart)
  if (s.g.D <= 4)
    DEX_FV(4);
  else if (s.g.D <= 8)
    DEX_FV(8);
  else if (s.g.D <= 16)
    DEX_FV(16);
  else if (s.g.D <= 32)
    DEX_FV(32);
  else
    DEX_FV(64);
#undef DEX_FV
}

template <typename T>
void launch_bwd_valu(const Shape& s, const GmmPtrs& in, const T* beta, const T* f, const T* ct,
                     T* part, int chunk, hipStream_t st) {
  dim3 grid((unsigned)s.g.K, (unsigned)((s.g.N + chunk - 1) / chunk));
#define DEX_BV(DB)                                                                          \
  hipLaunchKernelGGL((gmm_bwd_valu<T, DB>), grid, dim3(256), 0, st, (const T*)in.means,   \
                     (const T*)in.qd, (const T*)in.l, (const T*)in.x, (int)s.g.N,         \
                     (int)s.g.D, (int)s.g.K, chunk, beta, f, ct, part)
  if (s.g.D <= 4)
    DEX_BV(4);
  else if (s.g.D <= 8)
    DEX_BV(8);
  else if (s.g.D <= 16)
    DEX_BV(16);
  else if (s.g.D <= 32)
    DEX_BV(32);
  else
    DEX_BV(64);
#undef DEX_BV
}

bool valid_shape(const Shape& s) {
  const GmmGeom& g = s.g;
  if (g.N < 1 || g.D < 1 || g.K < 1 || g.D > 64) return false;
  if (s.dtype != DEX_F32 && s.dtype != DEX_F64) return false;
  if (s.variant != DEX_GMM_PLAIN && s.dtype != DEX_F32) return false;
  if (s.variant > DEX_GMM_BF16X3) return false;  // the split-FP16 form is batched only
  return true;
}

}  // namespace

size_t gmm_cache_bytes(const dex_desc& d) {
  Shape s = shape_of(d);
  if (!valid_shape(s)) return 0;
  return cache_layout(s).total;
}

// Forward-mode workspace. Feature-product form (16-bit variant, D = 64): the
// scaled FP16 x~ and its tile exponents, the tangent coefficient operand,
// dkq' and rescale factors, one FP64 partial per (pass, tile). Vector-ALU
// form: one FP64 partial per (point block, component chunk).
struct JvpLayout {
  size_t x16, texp, dW16, dkq, disc, part, total;
  int64_t nparts;
};
static JvpLayout jvp_layout(const Shape& s) {
  JvpLayout j{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align256(bytes);
    return at;
  };
  if (s.mfma && qf_eligible(s.g, s.prec)) {
    const size_t Kp = (size_t)beta_rows(s.g.K);
    j.x16 = take((size_t)s.g.Npad * 64 * 2);
    j.texp = take((size_t)(s.g.Npad / 64) * 4);
    j.dW16 = take(Kp / 16 * 68 * 64 * 8 * 2);
    j.dkq = take(Kp * 4);
    j.disc = take(Kp * 4);
    j.nparts = qf_tan_parts(s.g);
  } else {
    j.nparts = ((s.g.N + 255) / 256) * ((s.g.K + kJvpKC - 1) / kJvpKC);
  }
  j.part = take((size_t)j.nparts * 8);
  j.total = o;
  return j;
}

size_t gmm_ws_bytes(const dex_desc& d, int role) {
  Shape s = shape_of(d);
  if (!valid_shape(s)) return 0;
  if (role == DEX_WS_RESID) return cache_layout(s).total;
  if (role == DEX_WS_JVP) return jvp_layout(s).total;
  const size_t nparts = (size_t)(s.g.Npad / 64);  // objective partials (one per 64 points)
  if (role == DEX_WS_FWD) {
    size_t b = align256(nparts * 2 * s.tsize);
    if (s.mfma) b += align256((size_t)fwd_max_slots(s.g.K) * s.g.Npad * sizeof(float2));
    return b;
  }
  if (s.mfma)
    return align256((size_t)bwd_max_slots(s.g.Npad, s.g.K) * s.g.K * mom_slot(s.g.DP) * 4);
  return align256((size_t)kValuS * s.g.K * (s.g.D * s.g.D + s.g.D + 1) * s.tsize);
}

int gmm_num_configs(const dex_desc& d, int role) {
  Shape s = shape_of(d);
  if (!s.mfma) return 1;
  return role == DEX_WS_VJP ? nbwd(s) : nfwd(s);
}

dex_status gmm_fwd(const dex_desc& d, int cfg, const GmmPtrs& in, void* F, void* f, void* cache,
                   void* ws, hipStream_t st) {
  Shape s = shape_of(d);
  if (!valid_shape(s)) return fail(DEX_ERR_UNSUPPORTED, "GMM shape/dtype/variant not supported");
  CacheLayout cl = cache_layout(s);
  char* cc = (char*)cache;
  const size_t nparts = (size_t)(s.g.Npad / 64);
  if (!s.mfma) {
    double* fpart = (double*)ws;
    launch_fwd_valu<double>(s, in, (double*)(cc + cl.beta), (double*)f, fpart, st);
    hipLaunchKernelGGL((k_finalize_F<double>), dim3(1), dim3(256), 0, st, fpart,
                       (int)((s.g.N + 255) / 256), (const double*)in.alphas, (int)s.g.K, s.g.N,
                       (double*)F);
    return check_hip(hipGetLastError(), "gmm_fwd (VALU)");
  }
  if (cfg < 0 || cfg >= nfwd(s)) return fail(DEX_ERR_INVALID_ARG, "GMM forward config %d out of range", cfg);
  const FwdCfg c = fwd_cfg(s, cfg);
  float* fpart = (float*)ws;
  float2* ml = (float2*)((char*)ws + align256(nparts * 2 * 4));
  float* beta = (float*)(cc + cl.beta);
  const MfmaOps o = ops_of(s, cl, cc);
  const float* x = (const float*)in.x;
  const float *al = (const float*)in.alphas, *mu = (const float*)in.means,
              *qd = (const float*)in.qd, *l = (const float*)in.l;
  void *xh = cc + cl.xh, *xl = cc + cl.xl, *xhT = cc + cl.xhT, *xlT = cc + cl.xlT, *Qh = cc + cl.Qh,
       *Ql = cc + cl.Ql;
  float *negc = (float*)(cc + cl.negc), *kappa = (float*)(cc + cl.kappa);
  float* shift = (float*)(cc + cl.shift);  // written by the preparation launch
  FlatSplit sp{};
  switch (s.prec) {
    case PREC_BF16:
      if (c.nkq == 0 && qf_eligible(s.g, s.prec)) {
        qf_prep(s.g, x, al, mu, qd, l, xhT, cc + cl.x16, (int*)(cc + cl.texp), cc + cl.W16,
                (float*)(cc + cl.kq), (float*)(cc + cl.isc), shift, st);
        ProfRange pr(DEX_PROF_GMM_FWD, st);
        sp = qf_fwd(s.g, c, cc + cl.x16, cc + cl.W16, (const float*)(cc + cl.kq),
                    (const float*)(cc + cl.isc), (const int*)(cc + cl.texp), beta, ml, st);
        pr.end(1);
      } else {
        const FwdCfg ck = c.nkq == 0 ? kFwdBF[1] : c;
        mfma_prep<PREC_BF16>(s.g, x, al, mu, qd, l, xh, xl, xhT, xlT, Qh, Ql, negc, kappa, shift,
                             st);
        ProfRange pr(DEX_PROF_GMM_FWD, st);
        sp = mfma_fwd<PREC_BF16>(s.g, ck, o, beta, ml, st);
        pr.end(1);
      }
      break;
    case PREC_BF16X3:
      mfma_prep<PREC_BF16X3>(s.g, x, al, mu, qd, l, xh, xl, xhT, xlT, Qh, Ql, negc, kappa, shift,
                             st);
      {
        ProfRange pr(DEX_PROF_GMM_FWD, st);
        sp = mfma_fwd<PREC_BF16X3>(s.g, c, o, beta, ml, st);
        pr.end(1);
      }
      break;
    default:
      mfma_prep<PREC_F32>(s.g, x, al, mu, qd, l, xh, xl, xhT, xlT, Qh, Ql, negc, kappa, shift,
                          st);
      {
        ProfRange pr(DEX_PROF_GMM_FWD, st);
        sp = mfma_fwd<PREC_F32>(s.g, c, o, beta, ml, st);
        pr.end(1);
      }
  }
  // few partials per point: one thread per point; many: four
  const bool quad = sp.sk > 16;
  const unsigned nq = (unsigned)(s.g.Npad / (quad ? 64 : 256));
  if (quad)
    hipLaunchKernelGGL((k_merge_lse_quad<float>), dim3(nq), dim3(256), 0, st, ml, sp.sk,
                       (int)s.g.N, (int)s.g.Npad, (float*)f, fpart);
  else
    hipLaunchKernelGGL((k_merge_lse<float>), dim3(nq), dim3(256), 0, st, ml, sp.sk, (int)s.g.N,
                       (int)s.g.Npad, (float*)f, fpart);
  hipLaunchKernelGGL((k_finalize_F<float>), dim3(1), dim3(256), 0, st, fpart, (int)nq, al,
                     (int)s.g.K, s.g.N, (float*)F);
  return check_hip(hipGetLastError(), "gmm_fwd (MFMA)");
}

dex_status gmm_vjp(const dex_desc& d, int cfg, const GmmPtrs& in, const void* f,
                   const void* cache, const void* ct, const GmmGrads& out, bool accumulate,
                   void* ws, hipStream_t st) {
  Shape s = shape_of(d);
  if (!valid_shape(s)) return fail(DEX_ERR_UNSUPPORTED, "GMM shape/dtype/variant not supported");
  CacheLayout cl = cache_layout(s);
  const char* cc = (const char*)cache;
  if (!s.mfma) {
    const int chunk = (int)(((s.g.N + kValuS - 1) / kValuS + 63) / 64 * 64);
    const int S = (int)((s.g.N + chunk - 1) / chunk);
    launch_bwd_valu<double>(s, in, (const double*)(cc + cl.beta), (const double*)f,
                            (const double*)ct, (double*)ws, chunk, st);
    const size_t E = (size_t)s.g.D * s.g.D + s.g.D + 1;
    hipLaunchKernelGGL((k_bwd_finalize<double, double>), dim3((unsigned)s.g.K), dim3(256), 0, st,
                       (const double*)ws, E, S, (int)s.g.K, (int)s.g.D, (int)s.g.D, s.g.N,
                       (const double*)in.alphas, (const double*)in.qd, (const double*)in.l,
                       (const double*)nullptr, (const double*)ct, (double*)out.d_alphas, (double*)out.d_means,
                       (double*)out.d_qd, (double*)out.d_l, accumulate ? 1 : 0);
    return check_hip(hipGetLastError(), "gmm_vjp (VALU)");
  }
  if (cfg < 0 || cfg >= nbwd(s)) return fail(DEX_ERR_INVALID_ARG, "GMM reverse config %d out of range", cfg);
  const BwdCfg c = bwd_cfg(s, cfg);
  const MfmaOps o = ops_of(s, cl, cc);
  const float* beta = (const float*)(cc + cl.beta);
  float* part = (float*)ws;
  ProfRange pr(DEX_PROF_GMM_VJP, st);
  FlatSplit sp{};
  switch (s.prec) {
    case PREC_BF16:
      sp = mfma_bwd<PREC_BF16>(s.g, c, o, beta, (const float*)f, (const float*)ct, part, st);
      break;
    case PREC_BF16X3:
      sp = mfma_bwd<PREC_BF16X3>(s.g, c, o, beta, (const float*)f, (const float*)ct, part, st);
      break;
    default:
      sp = mfma_bwd<PREC_F32>(s.g, c, o, beta, (const float*)f, (const float*)ct, part, st);
  }
  pr.end(1);
  const int64_t E = (int64_t)mom_slot(s.g.DP);
  hipLaunchKernelGGL(k_mom_reduce, dim3((unsigned)((s.g.K * E + 255) / 256)), dim3(256), 0, st,
                     part, E, (int)s.g.K, sp.gw, sp.nsteps, sp.W, (int)sp.T);
  hipLaunchKernelGGL(k_bwd_finalize_mom, dim3((unsigned)s.g.K), dim3(256), 0, st, (const float*)part,
                     (size_t)E, 1, (int)s.g.K,
                     (int)s.g.D, s.g.DP, s.g.N, (const float*)in.alphas, (const float*)in.means,
                     (const float*)in.qd, (const float*)in.l, (const float*)ct,
                     (float*)out.d_alphas, (float*)out.d_means, (float*)out.d_qd, (float*)out.d_l,
                     accumulate ? 1 : 0, (const float*)(cc + cl.shift));
  return check_hip(hipGetLastError(), "gmm_vjp (MFMA)");
}

template <typename T>
static void launch_jvp_valu(const Shape& s, const GmmPtrs& in, const void* f, const GmmGrads& t,
                            double* part, hipStream_t st) {
  dim3 grid((unsigned)((s.g.N + 255) / 256), (unsigned)((s.g.K + kJvpKC - 1) / kJvpKC));
#define DEX_JV(DB)                                                                            \
  hipLaunchKernelGGL((gmm_jvp_valu<T, DB>), grid, dim3(256), 0, st, (const T*)in.alphas,     \
                     (const T*)in.means, (const T*)in.qd, (const T*)in.l, (const T*)in.x,     \
                     (const T*)f, (int)s.g.N, (int)s.g.D, (int)s.g.K, (const T*)t.d_alphas,   \
                     (const T*)t.d_means, (const T*)t.d_qd, (const T*)t.d_l, part)
  if (s.g.D <= 4)
    DEX_JV(4);
  else if (s.g.D <= 8)
    DEX_JV(8);
  else if (s.g.D <= 16)
    DEX_JV(16);
  else if (s.g.D <= 32)
    DEX_JV(32);
  else
    DEX_JV(64);
#undef DEX_JV
}

dex_status gmm_jvp(const dex_desc& d, int cfg, const GmmPtrs& in, const void* f,
                   const void* cache, const GmmGrads& t, void* dF, void* ws, hipStream_t st) {
  (void)cfg;
  Shape s = shape_of(d);
  if (!valid_shape(s)) return fail(DEX_ERR_UNSUPPORTED, "GMM shape/dtype/variant not supported");
  const JvpLayout jl = jvp_layout(s);
  char* w = (char*)ws;
  double* part = (double*)(w + jl.part);
  if (s.mfma && qf_eligible(s.g, s.prec)) {
    // tangent products over the same second-order features as the forward
    const CacheLayout cl = cache_layout(s);
    const char* cc = (const char*)cache;
    const float* shift = (const float*)(cc + cl.shift);
    qf_tan_prep(s.g, (const float*)in.x, (const float*)in.means, (const float*)in.qd,
                (const float*)in.l, (const float*)t.d_alphas, (const float*)t.d_means,
                (const float*)t.d_qd, (const float*)t.d_l, shift, w + jl.x16, (int*)(w + jl.texp),
                w + jl.dW16, (float*)(w + jl.dkq), (float*)(w + jl.disc), st);
    ProfRange pr(DEX_PROF_GMM_JVP, st);
    qf_jvp(s.g, w + jl.x16, w + jl.dW16, (const float*)(w + jl.dkq), (const float*)(w + jl.disc),
           (const int*)(w + jl.texp), (const float*)(cc + cl.beta), (const float*)f, part, st);
    pr.end(1);
  } else {
    ProfRange pr(DEX_PROF_GMM_JVP, st);
    if (s.tsize == 8)
      launch_jvp_valu<double>(s, in, f, t, part, st);
    else
      launch_jvp_valu<float>(s, in, f, t, part, st);
    pr.end(1);
  }
  if (s.tsize == 8)
    hipLaunchKernelGGL((k_jvp_final<double>), dim3(1), dim3(256), 0, st, (const double*)part,
                       jl.nparts, (const double*)in.alphas, (const double*)t.d_alphas, (int)s.g.K,
                       s.g.N, (double*)dF);
  else
    hipLaunchKernelGGL((k_jvp_final<float>), dim3(1), dim3(256), 0, st, (const double*)part,
                       jl.nparts, (const float*)in.alphas, (const float*)t.d_alphas, (int)s.g.K,
                       s.g.N, (float*)dF);
  return check_hip(hipGetLastError(), "gmm_jvp");
}

}  // namespace dexi
