// In-place periodic five-point diffusion loop and its reverse pass, gfx950.
//
// Forward (a State loop, Sec. 2.3.1): for t in 0..T-1,
//   u <- u + c (u[y+1,x] + u[y-1,x] + u[y,x+1] + u[y,x-1] - 4u) + rho sin(u)
// where every read is of the previous field (`get` yields a value, Sec. 5.3.2),
// so each step is a Jacobi sweep into a second buffer. Every `every`-th state
// (t = 0, every, 2 every, ...) is copied out as a checkpoint.
// Loss L = 1/2 ||u_T - target||^2.
//
// Reverse (ForTranspose runs the loop backwards; GetTranspose/PutTranspose carry
// the cotangent of the state): lam_T = dL (u_T - target), then for t = T-1..0
//   lam_t = S^T lam_{t+1} + rho cos(u_t) lam_{t+1},
// S being the linear diffusion step. The gather form computes S^T lam at each
// cell from its neighbours (S is symmetric); the scatter form is the literal
// transposed loop body, in which every cell adds its weighted cotangent into the
// cells it read (LetIndexingTranspose), with atomics. With the recompute
// variant the states of a checkpoint segment are rebuilt before its adjoint
// steps; only the non-linear term reads them (Sec. 5.3.2).
#include "common.h"
#include "internal.h"

namespace dexk {

// One forward step, 4 cells per thread (W % 4 == 0, W >= 8).
__global__ void __launch_bounds__(256) stencil_step_vec(const float* __restrict__ u,
                                                        float* __restrict__ un,
                                                        float* __restrict__ snap, int H, int W,
                                                        float c, float rho) {
  const int W4 = W >> 2;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)H * W4) return;
  const int y = (int)(t / W4), x4 = (int)(t % W4);
  const int yn = y == 0 ? H - 1 : y - 1, ys = y == H - 1 ? 0 : y + 1;
  const int x0 = 4 * x4;
  const float4 cc = *reinterpret_cast<const float4*>(u + (int64_t)y * W + x0);
  const float4 nn = *reinterpret_cast<const float4*>(u + (int64_t)yn * W + x0);
  const float4 ss = *reinterpret_cast<const float4*>(u + (int64_t)ys * W + x0);
  const float lf = u[(int64_t)y * W + (x0 == 0 ? W - 1 : x0 - 1)];
  const float rt = u[(int64_t)y * W + (x0 + 4 == W ? 0 : x0 + 4)];
  float4 o;
  o.x = cc.x + c * (((ss.x + nn.x) + cc.y) + lf - 4.f * cc.x);
  o.y = cc.y + c * (((ss.y + nn.y) + cc.z) + cc.x - 4.f * cc.y);
  o.z = cc.z + c * (((ss.z + nn.z) + cc.w) + cc.y - 4.f * cc.z);
  o.w = cc.w + c * (((ss.w + nn.w) + rt) + cc.z - 4.f * cc.w);
  if (rho != 0.f) {
    o.x += rho * sinf(cc.x);
    o.y += rho * sinf(cc.y);
    o.z += rho * sinf(cc.z);
    o.w += rho * sinf(cc.w);
  }
  *reinterpret_cast<float4*>(un + (int64_t)y * W + x0) = o;
  if (snap) *reinterpret_cast<float4*>(snap + (int64_t)y * W + x0) = cc;
}

// Strip form (W % 256 == 0, H % (4 RB) == 0): each wave owns 256 columns
// (4 per lane) of RB consecutive rows. The RB + 2 input rows it needs are
// loaded once into registers; left and right neighbours come from the
// adjacent lanes, and only the two strip-edge cells are read separately. In
// the adjoint (ADJ) the same body computes S^T g + rho cos(u) g.
template <int RB, bool ADJ>
__global__ void __launch_bounds__(256) stencil_strip(const float* __restrict__ u,
                                                     float* __restrict__ out,
                                                     float* __restrict__ snap,
                                                     const float* __restrict__ ustate, int H, int W,
                                                     float c, float rho, int accumulate) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int x0 = blockIdx.x * 256;
  const int y0 = (blockIdx.y * 4 + wv) * RB;
  const int xl = x0 == 0 ? W - 1 : x0 - 1;
  const int xr = x0 + 256 == W ? 0 : x0 + 256;
  f32x4 r[RB + 2];
  float el[RB + 2], er[RB + 2];
#pragma unroll
  for (int q = 0; q < RB + 2; ++q) {
    int y = y0 - 1 + q;
    y = y < 0 ? y + H : (y >= H ? y - H : y);
    const float* row = u + (int64_t)y * W;
    r[q] = *reinterpret_cast<const f32x4*>(row + x0 + 4 * lane);
    el[q] = row[xl];
    er[q] = row[xr];
  }
  const float a = 1.f - 4.f * c;
  // a compile-time row index (static_for): r, el and er stay in registers
  static_for<RB>([&](auto qc) {
    constexpr int q = decltype(qc)::value + 1;
    const f32x4 cc = r[q], nn = r[q - 1], ss = r[q + 1];
    float lf = __shfl_up(cc[3], 1, 64);
    float rt = __shfl_down(cc[0], 1, 64);
    if (lane == 0) lf = el[q];
    if (lane == 63) rt = er[q];
    const int64_t off = (int64_t)(y0 + q - 1) * W + x0 + 4 * lane;
    f32x4 o;
    if constexpr (!ADJ) {
      o[0] = cc[0] + c * (((ss[0] + nn[0]) + cc[1]) + lf - 4.f * cc[0]);
      o[1] = cc[1] + c * (((ss[1] + nn[1]) + cc[2]) + cc[0] - 4.f * cc[1]);
      o[2] = cc[2] + c * (((ss[2] + nn[2]) + cc[3]) + cc[1] - 4.f * cc[2]);
      o[3] = cc[3] + c * (((ss[3] + nn[3]) + rt) + cc[2] - 4.f * cc[3]);
      if (rho != 0.f) {
#pragma unroll
        for (int e = 0; e < 4; ++e) o[e] += rho * sinf(cc[e]);
      }
      if (snap) *reinterpret_cast<f32x4*>(snap + off) = cc;
    } else {
      o[0] = a * cc[0] + c * (((ss[0] + nn[0]) + cc[1]) + lf);
      o[1] = a * cc[1] + c * (((ss[1] + nn[1]) + cc[2]) + cc[0]);
      o[2] = a * cc[2] + c * (((ss[2] + nn[2]) + cc[3]) + cc[1]);
      o[3] = a * cc[3] + c * (((ss[3] + nn[3]) + rt) + cc[2]);
      if (rho != 0.f) {
        const f32x4 us = *reinterpret_cast<const f32x4*>(ustate + off);
#pragma unroll
        for (int e = 0; e < 4; ++e) o[e] += rho * cosf(us[e]) * cc[e];
      }
      if (accumulate) {
        const f32x4 p = *reinterpret_cast<const f32x4*>(out + off);
#pragma unroll
        for (int e = 0; e < 4; ++e) o[e] += p[e];
      }
    }
    *reinterpret_cast<f32x4*>(out + off) = o;
  });
}

__global__ void __launch_bounds__(256) stencil_step_scalar(const float* __restrict__ u,
                                                           float* __restrict__ un,
                                                           float* __restrict__ snap, int H,
                                                           int W, float c, float rho) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)H * W) return;
  const int y = (int)(t / W), x = (int)(t % W);
  const int yn = y == 0 ? H - 1 : y - 1, ys = y == H - 1 ? 0 : y + 1;
  const int xl = x == 0 ? W - 1 : x - 1, xr = x == W - 1 ? 0 : x + 1;
  const float cc = u[t];
  float o = cc + c * (((u[(int64_t)ys * W + x] + u[(int64_t)yn * W + x]) + u[(int64_t)y * W + xr]) +
                      u[(int64_t)y * W + xl] - 4.f * cc);
  if (rho != 0.f) o += rho * sinf(cc);
  un[t] = o;
  if (snap) snap[t] = cc;
}

// Adjoint step, gather form: lam = S^T g + rho cos(u) g  (=|+= into out).
__global__ void __launch_bounds__(256) stencil_adj_gather(const float* __restrict__ g,
                                                          const float* __restrict__ u,
                                                          float* __restrict__ out, int H, int W,
                                                          float c, float rho, int accumulate) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)H * W) return;
  const int y = (int)(t / W), x = (int)(t % W);
  const int yn = y == 0 ? H - 1 : y - 1, ys = y == H - 1 ? 0 : y + 1;
  const int xl = x == 0 ? W - 1 : x - 1, xr = x == W - 1 ? 0 : x + 1;
  const float gc = g[t];
  // cell (y+1, x) read u[y, x] as its north neighbour, etc.
  float v = (1.f - 4.f * c) * gc +
            c * (((g[(int64_t)ys * W + x] + g[(int64_t)yn * W + x]) + g[(int64_t)y * W + xr]) +
                 g[(int64_t)y * W + xl]);
  if (rho != 0.f) v += rho * cosf(u[t]) * gc;
  out[t] = accumulate ? out[t] + v : v;
}

// Vectorised gather-form adjoint (W % 4 == 0, W >= 8); same arithmetic order.
__global__ void __launch_bounds__(256) stencil_adj_gather_vec(const float* __restrict__ g,
                                                              const float* __restrict__ u,
                                                              float* __restrict__ out, int H,
                                                              int W, float c, float rho,
                                                              int accumulate) {
  const int W4 = W >> 2;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)H * W4) return;
  const int y = (int)(t / W4), x4 = (int)(t % W4);
  const int yn = y == 0 ? H - 1 : y - 1, ys = y == H - 1 ? 0 : y + 1;
  const int x0 = 4 * x4;
  const float4 cc = *reinterpret_cast<const float4*>(g + (int64_t)y * W + x0);
  const float4 nn = *reinterpret_cast<const float4*>(g + (int64_t)yn * W + x0);
  const float4 ss = *reinterpret_cast<const float4*>(g + (int64_t)ys * W + x0);
  const float lf = g[(int64_t)y * W + (x0 == 0 ? W - 1 : x0 - 1)];
  const float rt = g[(int64_t)y * W + (x0 + 4 == W ? 0 : x0 + 4)];
  const float a = 1.f - 4.f * c;
  float4 v;
  v.x = a * cc.x + c * (((ss.x + nn.x) + cc.y) + lf);
  v.y = a * cc.y + c * (((ss.y + nn.y) + cc.z) + cc.x);
  v.z = a * cc.z + c * (((ss.z + nn.z) + cc.w) + cc.y);
  v.w = a * cc.w + c * (((ss.w + nn.w) + rt) + cc.z);
  if (rho != 0.f) {
    const float4 uu = *reinterpret_cast<const float4*>(u + (int64_t)y * W + x0);
    v.x += rho * cosf(uu.x) * cc.x;
    v.y += rho * cosf(uu.y) * cc.y;
    v.z += rho * cosf(uu.z) * cc.z;
    v.w += rho * cosf(uu.w) * cc.w;
  }
  float4* o = reinterpret_cast<float4*>(out + (int64_t)y * W + x0);
  if (accumulate) {
    float4 p = *o;
    v.x += p.x;
    v.y += p.y;
    v.z += p.z;
    v.w += p.w;
  }
  *o = v;
}

// Adjoint step, scatter form: the transposed loop body literally, each cell
// accumulating its weighted cotangent into the five cells it read. `out`
// must hold zero (or the value to accumulate onto) on entry.
__global__ void __launch_bounds__(256) stencil_adj_scatter(const float* __restrict__ g,
                                                           const float* __restrict__ u,
                                                           float* __restrict__ out, int H,
                                                           int W, float c, float rho) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)H * W) return;
  const int y = (int)(t / W), x = (int)(t % W);
  const int yn = y == 0 ? H - 1 : y - 1, ys = y == H - 1 ? 0 : y + 1;
  const int xl = x == 0 ? W - 1 : x - 1, xr = x == W - 1 ? 0 : x + 1;
  const float gc = g[t];
  float self = (1.f - 4.f * c) * gc;
  if (rho != 0.f) self += rho * cosf(u[t]) * gc;
  atomicAdd(&out[t], self);
  atomicAdd(&out[(int64_t)ys * W + x], c * gc);
  atomicAdd(&out[(int64_t)yn * W + x], c * gc);
  atomicAdd(&out[(int64_t)y * W + xr], c * gc);
  atomicAdd(&out[(int64_t)y * W + xl], c * gc);
}

// Forward mode, one step of the primal and its tangent together (the
// linearized step, Sec. 5.1: the diffusion part is linear, the non-linear term
// linearizes to rho cos(u) du, which reads the primal state of the same step):
//   un  = u  + c (sum of the 4 neighbours of u  - 4 u ) + rho sin(u)
//   dun = du + c (sum of the 4 neighbours of du - 4 du) + rho cos(u) du
// One cell per thread, periodic indices.
__global__ void __launch_bounds__(256) stencil_tan_step(const float* __restrict__ u,
                                                        const float* __restrict__ du,
                                                        float* __restrict__ un,
                                                        float* __restrict__ dun, int H, int W,
                                                        float c, float rho) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)H * W) return;
  const int y = (int)(t / W), x = (int)(t % W);
  const int yn = y == 0 ? H - 1 : y - 1, ys = y == H - 1 ? 0 : y + 1;
  const int xl = x == 0 ? W - 1 : x - 1, xr = x == W - 1 ? 0 : x + 1;
  const int64_t is = (int64_t)ys * W + x, in = (int64_t)yn * W + x;
  const int64_t ir = (int64_t)y * W + xr, il = (int64_t)y * W + xl;
  const float cc = u[t], dc = du[t];
  float o = cc + c * (((u[is] + u[in]) + u[ir]) + u[il] - 4.f * cc);
  float d = dc + c * (((du[is] + du[in]) + du[ir]) + du[il] - 4.f * dc);
  if (rho != 0.f) {
    o += rho * sinf(cc);
    d += rho * cosf(cc) * dc;
  }
  un[t] = o;
  dun[t] = d;
}

// Per-block partial sums of (u - target)(du - dtarget) in FP64: the tangent of
// L = 1/2 ||u - target||^2.
__global__ void __launch_bounds__(256) stencil_tan_loss_partial(const float* __restrict__ u,
                                                                const float* __restrict__ tg,
                                                                const float* __restrict__ du,
                                                                const float* __restrict__ dtg,
                                                                int64_t n,
                                                                double* __restrict__ part) {
  __shared__ double sh[16];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    s += ((double)u[i] - (double)tg[i]) * ((double)du[i] - (double)dtg[i]);
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void stencil_sum_final(const double* __restrict__ part, int nb, float* __restrict__ out) {
  __shared__ double sh[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) s += part[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[0] = (float)s;
}

// Per-block partial sums of (u - target)^2 in FP64.
__global__ void __launch_bounds__(256) stencil_loss_partial(const float* __restrict__ u,
                                                            const float* __restrict__ tg,
                                                            int64_t n, double* __restrict__ part) {
  __shared__ double sh[16];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double d = (double)u[i] - (double)tg[i];
    s += d * d;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void stencil_loss_final(const double* __restrict__ part, int nb, float* __restrict__ L) {
  __shared__ double sh[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) s += part[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) L[0] = (float)(0.5 * s);
}

// lam = dL * (u - target)
__global__ void __launch_bounds__(256) stencil_lam_init(const float* __restrict__ u,
                                                        const float* __restrict__ tg,
                                                        const float* __restrict__ dL, int64_t n,
                                                        float* __restrict__ lam) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) lam[i] = dL[0] * (u[i] - tg[i]);
}

__global__ void __launch_bounds__(256) copy_f32(const float* __restrict__ a, float* __restrict__ b,
                                                int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) b[i] = a[i];
}

}  // namespace dexk

// ===========================================================================
namespace dexi {
using namespace dexk;

namespace {
constexpr int kLossBlocks = 1024;

struct St {
  int H, W, T, every, nck;
  float c, rho;
  int64_t n;
  bool vec;
};

St st_of(const dex_desc& d) {
  St s;
  s.H = (int)d.dims[0];
  s.W = (int)d.dims[1];
  s.T = (int)d.dims[2];
  s.every = (int)d.dims[3];
  s.nck = s.every > 0 ? (s.T + s.every - 1) / s.every : 0;
  s.c = (float)d.fparams[0];
  s.rho = (float)d.fparams[1];
  s.n = (int64_t)s.H * s.W;
  s.vec = (s.W % 4) == 0 && s.W >= 8;
  return s;
}

// Rows per wave of the strip kernels (0: the grid does not allow the strip
// form). Taller strips re-read fewer halo rows (RB + 2 rows read per RB
// written) but 16 rows measured no faster than 8 at 4096^2 (fewer waves per
// SIMD, 170 registers).
constexpr int kRB = 8;
int strip_rb(const St& s) { return s.W % 256 == 0 && s.H % (4 * kRB) == 0 ? kRB : 0; }

template <bool ADJ>
void launch_strip(const St& s, const float* in, float* out, float* snap, const float* ustate,
                  int accumulate, hipStream_t st) {
  hipLaunchKernelGGL((stencil_strip<kRB, ADJ>), dim3(s.W / 256, s.H / (4 * kRB)), dim3(256), 0, st,
                     in, out, snap, ustate, s.H, s.W, s.c, s.rho, accumulate);
}

// strip: use the strip kernels where the grid allows them (a tuning config).
void step(const St& s, const float* u, float* un, float* snap, bool strip, hipStream_t st) {
  const int rb = strip ? strip_rb(s) : 0;
  if (rb) {
    launch_strip<false>(s, u, un, snap, nullptr, 0, st);
  } else if (s.vec) {
    const int64_t nt = s.n / 4;
    hipLaunchKernelGGL(stencil_step_vec, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st, u,
                       un, snap, s.H, s.W, s.c, s.rho);
  } else {
    hipLaunchKernelGGL(stencil_step_scalar, dim3((unsigned)((s.n + 255) / 256)), dim3(256), 0, st,
                       u, un, snap, s.H, s.W, s.c, s.rho);
  }
}

// form: 0 gather (strip kernel where the grid allows), 1 scatter, 2 gather (vector kernel).
void adj(const St& s, int form, const float* g, const float* u, float* out, bool accumulate,
         hipStream_t st) {
  const unsigned nb = (unsigned)((s.n + 255) / 256);
  if (form == 1) {
    if (!accumulate) fill_zero(out, (size_t)s.n * 4, st);
    hipLaunchKernelGGL(stencil_adj_scatter, dim3(nb), dim3(256), 0, st, g, u, out, s.H, s.W, s.c,
                       s.rho);
  } else if (form == 0 && strip_rb(s)) {
    launch_strip<true>(s, g, out, nullptr, u, accumulate ? 1 : 0, st);
  } else if (s.vec) {
    hipLaunchKernelGGL(stencil_adj_gather_vec, dim3((unsigned)((s.n / 4 + 255) / 256)), dim3(256),
                       0, st, g, u, out, s.H, s.W, s.c, s.rho, accumulate ? 1 : 0);
  } else {
    hipLaunchKernelGGL(stencil_adj_gather, dim3(nb), dim3(256), 0, st, g, u, out, s.H, s.W, s.c,
                       s.rho, accumulate ? 1 : 0);
  }
}
}  // namespace

size_t stencil_ws_bytes(const dex_desc& d, int role) {
  St s = st_of(d);
  const size_t fb = align256((size_t)s.n * 4);
  if (role == DEX_WS_FWD) return fb + align256(kLossBlocks * 8);
  if (role == DEX_WS_JVP) return 4 * fb + align256(kLossBlocks * 8);  // (u, du) ping-pong
  if (role == DEX_WS_VJP) {
    size_t b = 2 * fb;  // cotangent ping-pong
    if (d.variant == DEX_STENCIL_RECOMPUTE) b += (size_t)(s.every > 1 ? s.every - 1 : 0) * fb + fb;
    return b;
  }
  return 0;
}

int stencil_num_configs(const dex_desc& d, int role) {
  (void)d;
  // fwd: 0 strip kernel (where the grid allows), 1 vector kernel; vjp: 0 gather
  // form (strip kernels where allowed), 1 scatter form, 2 gather form with
  // vector kernels
  return role == DEX_WS_VJP ? 3 : 2;
}

dex_status stencil_fwd(const dex_desc& d, int cfg, const float* u0, const float* target, float* L,
                       float* uT, float* ckpt, void* ws, hipStream_t st) {
  St s = st_of(d);
  float* other = (float*)ws;
  double* part = (double*)((char*)ws + align256((size_t)s.n * 4));
  // step t writes into uT when (T-1-t) is even, so the last step lands in uT
  const float* cur = u0;
  ProfRange pr(DEX_PROF_STENCIL_FWD, st);
  for (int t = 0; t < s.T; ++t) {
    float* dst = ((s.T - 1 - t) % 2 == 0) ? uT : other;
    float* snap = (t % s.every == 0) ? ckpt + (int64_t)(t / s.every) * s.n : nullptr;
    step(s, cur, dst, snap, cfg == 0, st);
    cur = dst;
  }
  pr.end(s.T);
  if (s.T == 0) {
    hipLaunchKernelGGL(copy_f32, dim3((unsigned)((s.n + 255) / 256)), dim3(256), 0, st, u0, uT, s.n);
  }
  hipLaunchKernelGGL(stencil_loss_partial, dim3(kLossBlocks), dim3(256), 0, st, uT, target, s.n, part);
  hipLaunchKernelGGL(stencil_loss_final, dim3(1), dim3(256), 0, st, part, kLossBlocks, L);
  return check_hip(hipGetLastError(), "stencil_fwd");
}

// Forward mode: tL = <u_T - target, du_T - dtarget>, the primal and tangent
// states stepped together through the workspace ping-pong buffers.
dex_status stencil_jvp(const dex_desc& d, const float* u0, const float* target, const float* du0,
                       const float* dtarget, float* tL, void* ws, hipStream_t st) {
  St s = st_of(d);
  const size_t fb = align256((size_t)s.n * 4);
  float* buf[2][2] = {{(float*)ws, (float*)((char*)ws + fb)},
                      {(float*)((char*)ws + 2 * fb), (float*)((char*)ws + 3 * fb)}};
  double* part = (double*)((char*)ws + 4 * fb);
  const float *u = u0, *du = du0;
  const unsigned nb = (unsigned)((s.n + 255) / 256);
  for (int t = 0; t < s.T; ++t) {
    float* un = buf[t & 1][0];
    float* dun = buf[t & 1][1];
    hipLaunchKernelGGL(stencil_tan_step, dim3(nb), dim3(256), 0, st, u, du, un, dun, s.H, s.W, s.c,
                       s.rho);
    u = un;
    du = dun;
  }
  hipLaunchKernelGGL(stencil_tan_loss_partial, dim3(kLossBlocks), dim3(256), 0, st, u, target, du,
                     dtarget, s.n, part);
  hipLaunchKernelGGL(stencil_sum_final, dim3(1), dim3(256), 0, st, part, kLossBlocks, tL);
  return check_hip(hipGetLastError(), "stencil_jvp");
}

// uT_in: the forward's final state (second residual).
dex_status stencil_vjp(const dex_desc& d, int cfg, const float* u0, const float* target,
                       const float* ckpt, const float* uT_in, const float* dL, float* du0,
                       bool accumulate, void* ws, hipStream_t st) {
  (void)u0;
  St s = st_of(d);
  const int form = cfg;
  const size_t fb = align256((size_t)s.n * 4);
  float* lamA = (float*)ws;
  float* lamB = (float*)((char*)ws + fb);
  float* seg = (float*)((char*)ws + 2 * fb);  // states u_{s0+1} .. u_{s0+len-1}
  const unsigned nb = (unsigned)((s.n + 255) / 256);
  if (s.T == 0) {
    if (accumulate) {
      // du0 += dL (u0 - target)
      hipLaunchKernelGGL(stencil_lam_init, dim3(nb), dim3(256), 0, st, uT_in, target, dL, s.n, lamA);
      hipLaunchKernelGGL(stencil_adj_gather, dim3(nb), dim3(256), 0, st, lamA, nullptr, du0, s.H,
                         s.W, 0.f, 0.f, 1);
    } else {
      hipLaunchKernelGGL(stencil_lam_init, dim3(nb), dim3(256), 0, st, uT_in, target, dL, s.n, du0);
    }
    return check_hip(hipGetLastError(), "stencil_vjp");
  }
  hipLaunchKernelGGL(stencil_lam_init, dim3(nb), dim3(256), 0, st, uT_in, target, dL, s.n, lamA);
  float* g = lamA;
  float* o = lamB;
  const bool recompute = d.variant == DEX_STENCIL_RECOMPUTE;
  if (!recompute && s.rho != 0.f)
    return fail(DEX_ERR_INVALID_ARG, "the no-recompute reverse pass needs rho == 0");
  ProfRange pr(DEX_PROF_STENCIL_VJP, st);
  int64_t launches = 0;
  for (int sg = s.nck - 1; sg >= 0; --sg) {
    const int s0 = sg * s.every;
    const int len = std::min(s.every, s.T - s0);
    const float* ck = ckpt + (int64_t)sg * s.n;
    if (recompute) {
      // rebuild u_{s0+1} .. u_{s0+len-1} from the checkpoint
      const float* cur = ck;
      for (int q = 1; q < len; ++q) {
        float* dst = seg + (int64_t)(q - 1) * (fb / 4);
        step(s, cur, dst, nullptr, form == 0, st);
        cur = dst;
        ++launches;
      }
    }
    for (int q = len - 1; q >= 0; --q) {
      const int t = s0 + q;
      const float* ut = nullptr;
      if (recompute) ut = q == 0 ? ck : seg + (int64_t)(q - 1) * (fb / 4);
      const bool last = (t == 0);
      float* dst = last ? du0 : o;
      adj(s, form, g, ut, dst, last && accumulate, st);
      ++launches;
      if (!last) std::swap(g, o);
    }
  }
  pr.end(launches);
  return check_hip(hipGetLastError(), "stencil_vjp");
}

}  // namespace dexi
