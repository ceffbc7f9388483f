/*
 * dex.h -- C ABI of libdexmi, the MI355X (gfx950) reverse-mode path for
 * pointful, index-set-typed loops.
 *
 * Paper: "Getting to the Point. Index Sets and Parallelism-Preserving Autodiff
 * for Pointful Array Programming" (arXiv 2104.05372).
 *
 * The calls follow the paper's statement of the problem:
 *   linearize : (a -> b) -> a -> (b, a -o b)            (Sec. 5.1)
 *   transpose : (a -o b) -> (b -o a)                     (Sec. 5.2)
 *   grad f x  = transpose (snd (linearize f x)) 1.0      (Sec. 5.2)
 *   (+=)      : Ref h w -> w -> {Accum h} Unit, runAccum (Sec. 2.3.2)
 *   (!)       : Ref h (n=>a) -> n -> Ref h a             (Sec. 2.3.3)
 *
 *   dex_fwd            = the primal half of `linearize f x`: the output and the
 *                        residuals the linear map closes over.
 *   dex_vjp            = `transpose (snd (linearize f x)) ct`.
 *   dex_accum_scatter  = `runAccum \acc. for j. acc!(idx.j) += scale.j * vals.j`.
 *
 * General rules for every entry point
 *   - Pointers named *_dev, and every dex_buf.ptr, are device pointers on the
 *     current HIP device, owned by the caller. dex_fwd, dex_vjp and
 *     dex_accum_scatter never allocate device memory; scratch comes from the
 *     caller's `workspace` (size from dex_workspace_bytes /
 *     dex_accum_scatter_workspace_bytes).
 *   - Work is enqueued on `hip_stream` (a hipStream_t; NULL = default stream)
 *     and the call returns after the launches. Argument errors are detected on
 *     the host and returned before anything is enqueued. A failed launch
 *     returns DEX_ERR_HIP. dex_last_error() gives a message for the last
 *     non-OK status on the calling thread.
 *   - Arrays are dense, row-major, with no padding (the flat unboxed layout of
 *     Sec. 6.3). Float arrays of a descriptor share its `dtype`.
 *   - A device that is not gfx950 gives DEX_ERR_UNSUPPORTED.
 */
#ifndef DEX_H
#define DEX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dex_status;
#define DEX_OK                0
#define DEX_ERR_INVALID_ARG  (-1) /* null pointer, bad size, dtype mismatch */
#define DEX_ERR_OUT_OF_RANGE (-2) /* DEX_SYNC_CHECK found an index outside its set */
#define DEX_ERR_UNSUPPORTED  (-3) /* kind/dtype/variant/shape not built, or not gfx950 */
#define DEX_ERR_HIP          (-4) /* a HIP runtime call or launch failed */
#define DEX_ERR_WORKSPACE    (-5) /* workspace missing or smaller than required */

/* element types */
#define DEX_F64 1
#define DEX_F32 2
#define DEX_I32 3
#define DEX_U32 4
#define DEX_I64 5
#define DEX_U8  6

/* function kinds (dex_desc.kind) */
#define DEX_GMM          1 /* GMM log-likelihood, one instance            */
#define DEX_GMM_BATCHED  2 /* many independent GMM instances, one launch  */
#define DEX_GATHER_SCALE 3 /* out[j,:] = w[j] * T[idx[j],:]                */
#define DEX_STENCIL5     4 /* in-place periodic 5-point diffusion loop     */

/* GMM arithmetic variants (dex_desc.variant) */
#define DEX_GMM_PLAIN  0 /* every product and sum in the descriptor dtype            */
#define DEX_GMM_BF16   1 /* 16-bit matrix-core operands, FP32 accumulation, FP32
                            storage only. Forward at D = 64: one FP16 product over
                            the second-order features of x (||Q_k r||^2 expanded
                            through P_k = Q_k^T Q_k, per-tile power-of-two scaling);
                            forward at other D: BF16 Q_k (x_i - mu_k) products;
                            reverse (weighted moments) FP16 at every D. All operands
                            are taken about the mean of the first min(K, 16)
                            component means, which changes no result (only x - mu
                            enters) but keeps the 16-bit values small for data far
                            from the origin.                                      */
#define DEX_GMM_BF16X3 2 /* split-BF16 operands, hi*hi + hi*lo + lo*hi per product   */
#define DEX_GMM_F16X3  3 /* DEX_GMM_BATCHED only: the forward of instances with D > 8
                            takes split-FP16 operands (hi + lo, 22 significant bits;
                            hi*hi + hi*lo + lo*hi per product, FP32 accumulation) of
                            x - c and Q_k, c the mean of the instance's first
                            min(K, 16) means, each scaled by a power of two so its
                            largest entry lies in [2^13, 2^14); the reverse keeps
                            FP32 moments. FP32-class results (about 1e-6 relative).
                            D <= 8 instances run as in PLAIN.                     */

/* stencil variants */
#define DEX_STENCIL_RECOMPUTE 0 /* reverse pass recomputes each checkpoint segment */
#define DEX_STENCIL_LINEAR    1 /* reverse pass uses no primal state (step linear) */

/* flags */
#define DEX_ACCUMULATE   1u /* dex_vjp: ct_in += result (VarTranspose); else ct_in = result */
#define DEX_CHECK_BOUNDS 2u /* count indices outside [0, n_rows) into *oob_count_dev
                               (int64, added to) and skip them                        */
#define DEX_SYNC_CHECK   4u /* with DEX_CHECK_BOUNDS: wait for the stream and return
                               DEX_ERR_OUT_OF_RANGE if this call found any           */
#define DEX_NO_DW        8u /* DEX_GATHER_SCALE dex_vjp: skip the cotangent of w      */
#define DEX_DETERMINISTIC 16u /* dex_accum_scatter, float: sort-based form whose rounding
                                order is fixed (bit-reproducible), no atomics        */

/* workspace roles for dex_workspace_bytes */
#define DEX_WS_FWD   0 /* scratch for dex_fwd                           */
#define DEX_WS_VJP   1 /* scratch for dex_vjp                           */
#define DEX_WS_RESID 2 /* bytes of the second (operand-cache) residual  */
#define DEX_WS_JVP   3 /* scratch for dex_jvp                           */

/*
 * Descriptor of the function being differentiated.
 *   kind     DEX_GMM | DEX_GMM_BATCHED | DEX_GATHER_SCALE | DEX_STENCIL5
 *   dtype    DEX_F64 or DEX_F32: storage type of all float buffers
 *   variant  arithmetic variant (see above), 0 for kinds without variants
 *   config   0 = tuned or default tile configuration; c > 0 forces candidate c
 *            (see dex_num_configs); used by the autotuner and by tests
 *   dims     DEX_GMM:          {N, D, K}
 *            DEX_GMM_BATCHED:  filled by dex_gmm_batched_plan
 *            DEX_GATHER_SCALE: {V (rows of T), R (row length), n (indices)}
 *            DEX_STENCIL5:     {H, W, steps, every (checkpoint interval)}
 *   fparams  DEX_STENCIL5: {c (diffusion weight), rho (weight of the
 *            non-linear term rho*sin(u); 0 for the pure diffusion loop)}
 */
typedef struct dex_desc {
  int32_t kind;
  int32_t dtype;
  int32_t variant;
  int32_t config;
  int64_t dims[8];
  double fparams[4];
} dex_desc;

/* A device array: ptr (may be NULL only when numel == 0), element count, dtype. */
typedef struct dex_buf {
  void* ptr;
  int64_t numel;
  int32_t dtype;
  int32_t reserved;
} dex_buf;

/*
 * Buffer lists per kind (in / out / resid / ct_out / ct_in, in this order):
 *
 * DEX_GMM (dims {N, D, K}, L = D(D-1)/2). Objective, with
 *   Q_k = diag(exp(qd[k])) + strict-lower(l[k]), Q_k[a,b] (a > b) at l[k, a(a-1)/2 + b]:
 *     beta[i,k] = alphas[k] + sum_d qd[k,d] - 1/2 || Q_k (x[i] - means[k]) ||^2
 *     f[i]      = logsumexp_k beta[i,k]                (max-shifted)
 *     F         = sum_i f[i] - N logsumexp_k alphas[k]
 *   in     = alphas[K], means[K*D], qd[K*D], l[K*L], x[N*D]
 *   out    = F[1]
 *   resid  = f[N] (dtype), cache[DEX_WS_RESID bytes, DEX_U8] (may be numel 0
 *            when DEX_WS_RESID is 0)
 *   ct_out = dF[1] (device scalar)
 *   ct_in  = d_alphas[K], d_means[K*D], d_qd[K*D], d_l[K*L]
 *   The reverse pass is the transposed loop: for the reads of alphas.k, means.k
 *   and Q.k inside `for i k` (rule LetIndexingTranspose, Fig. "transposition
 *   rules"), each cotangent is a regular segmented reduction over i
 *   (Sec. 6.1.3), done as per-block partial sums and a fixed-order compensated
 *   final sum (so the result does not depend on scheduling).
 *
 * DEX_GMM_BATCHED (dims from dex_gmm_batched_plan; FP32, variant PLAIN or F16X3):
 *   in     = plan[bytes, DEX_U8, device copy of the plan], alphas, means, qd, l, x
 *            (instances concatenated in order; instance b's arrays have the
 *            DEX_GMM sizes of its (N_b, D_b, K_b))
 *   out    = F[B];  resid = f[sum N_b];  ct_out = dF[B]
 *   ct_in  = d_alphas, d_means, d_qd, d_l (packed like the inputs)
 *
 * DEX_GATHER_SCALE (dims {V, R, n}; FP32):
 *   in     = T[V*R], idx[n] (DEX_I32), w[n]
 *   out    = out[n*R];  resid = none;  ct_out = g[n*R]
 *   ct_in  = dT[V*R], dw[n] (dw may be numel 0 with DEX_NO_DW)
 *   dT is the transposed gather: dT!(idx.j) += w.j * g.j (Sec. 5.3.3).
 *   config 1 (default): the (row, position) pairs are radix sorted and every
 *   row's sum is formed by one owner in index order and written once -- no
 *   atomics, bit-reproducible (needs DEX_WS_VJP workspace); config 2: block-local
 *   sort + run sums + float atomics (rounding order unspecified).
 *
 * DEX_STENCIL5 (dims {H, W, steps, every}; FP32): the State loop
 *     for t in 0..steps-1:  u := u + c (u[y+1,x]+u[y-1,x]+u[y,x+1]+u[y,x-1]-4u) + rho sin(u)
 *   (periodic; each step reads only the previous field), then
 *     L = 1/2 || u_T - target ||^2.
 *   in     = u0[H*W], target[H*W]
 *   out    = L[1], uT[H*W]
 *   resid  = checkpoints[ceil(steps/every) * H*W]  (u_0, u_every, u_2every, ...)
 *   ct_out = dL[1] (device scalar)
 *   ct_in  = du0[H*W]
 *   The reverse pass runs the time loop backwards (ForTranspose); with
 *   DEX_STENCIL_RECOMPUTE it rebuilds each segment's states from its
 *   checkpoint first (only non-linear terms read them, Sec. 5.3.2).
 *   configs: fwd 1 row-strip kernel (default; used where W % 256 == 0 and
 *   H % 32 == 0, else the vector kernel), 2 vector kernel; vjp 1 gather-form
 *   adjoint with row-strip kernels where allowed (default), 2 scatter-form
 *   adjoint (atomics), 3 gather form with vector kernels. All configs compute
 *   the same values.
 */

/* Message for a status code (static storage). */
const char* dex_status_string(dex_status s);

/* Message describing the last non-OK status returned on this thread. */
const char* dex_last_error(void);

/* Library version string, e.g. "dexmi 0.1 gfx950". */
const char* dex_version(void);

/* Check the current device (must be gfx950) and set up per-device state.
 * Called implicitly by every entry point; safe to call repeatedly. */
dex_status dex_init(void);

/* Bytes of caller-provided scratch that `role` (DEX_WS_*) needs for `d`. */
dex_status dex_workspace_bytes(const dex_desc* d, int32_t role, size_t* bytes);

/* Number of tile configurations that `config` may select for (d, role). */
dex_status dex_num_configs(const dex_desc* d, int32_t role, int32_t* count);

/* Forward: out = f(in) and the residuals for dex_vjp. */
dex_status dex_fwd(const dex_desc* d,
                   const dex_buf* in, int32_t n_in,
                   dex_buf* out, int32_t n_out,
                   dex_buf* resid, int32_t n_resid,
                   void* workspace, size_t ws_bytes,
                   void* hip_stream);

/* Reverse: ct_in (=|+=) transpose(linearize f in) applied to ct_out.
 * `resid` must come from dex_fwd with an identical descriptor and inputs. */
dex_status dex_vjp(const dex_desc* d,
                   const dex_buf* in, int32_t n_in,
                   const dex_buf* resid, int32_t n_resid,
                   const dex_buf* ct_out, int32_t n_ct_out,
                   dex_buf* ct_in, int32_t n_ct_in,
                   uint32_t flags,
                   void* workspace, size_t ws_bytes,
                   void* hip_stream);

/* Forward mode: t_out = the linear map of `linearize f in` (Sec. 5.1, the
 * linearization rules of its figure, e.g. LinFor for the loop over j) applied
 * to the tangents t_in, i.e. the directional derivative of f at `in` along
 * t_in. The transpose of the same map is dex_vjp, so for every t_in and ct_out
 * <t_out, ct_out> = <t_in, ct_in> up to rounding.
 *   DEX_GATHER_SCALE: in = T[V*R], idx[n] (DEX_I32), w[n] (as for dex_fwd);
 *     t_in = tT[V*R], tw[n];  t_out = tout[n*R],
 *     tout[j, :] = tw[j] T[idx[j], :] + w[j] tT[idx[j], :]
 *     (idx is an integer and has no tangent; rows whose index is outside [0, V)
 *     give zeros, as in dex_fwd).
 *   DEX_STENCIL5: in = u0[H*W], target[H*W] (as for dex_fwd);
 *     t_in = du0[H*W], dtarget[H*W];  t_out = dL[1]: the loop is run forward
 *     with each state's tangent beside it (du_{t+1} = S du_t + rho cos(u_t) du_t,
 *     S the linear diffusion step), then dL = <u_T - target, du_T - dtarget>
 *     (summed in FP64, fixed order). Workspace: four H*W fields and the sum's
 *     partials (DEX_WS_JVP).
 *   DEX_GMM: in = alphas, means, qd, l, x (as for dex_fwd); resid = f, cache from
 *     dex_fwd with the same descriptor and inputs; t_in = dalphas[K], dmeans[K*D],
 *     dqd[K*D], dl[K*L]; t_out = dF[1]. The linearized loop is run forward: per
 *     point i and component k, dy = dQ_k r_ik - Q_k dmu_k (dQ_k: diagonal
 *     exp(qd) dqd, strict lower dl), dbeta = dalpha_k + sum_d dqd_kd - y.dy,
 *     dF = sum_i sum_k exp(beta_ik - f_i) dbeta_ik - N softmax(alphas).dalphas.
 *     16-bit variant at D = 64: dbeta comes from one FP16 matrix-core product
 *     of the forward's second-order features with tangent coefficients (built
 *     from dP = dQ^T Q + Q^T dQ), weighted by the forward's beta residual.
 *     Every other form: one vector-ALU pass in the descriptor dtype (FP32 forms
 *     compute in FP32). The per-block sums and the final sum are FP64 in a
 *     fixed order. Workspace: DEX_WS_JVP bytes.
 *   Other kinds: DEX_ERR_UNSUPPORTED.
 * All buffers are device memory owned by the caller; t_out is overwritten.
 * Argument errors are reported before anything is enqueued; the call enqueues
 * on hip_stream and returns. resid is empty (n_resid = 0) except for DEX_GMM.
 * Workspace: DEX_WS_JVP bytes (0 for the gather). */
dex_status dex_jvp(const dex_desc* d,
                   const dex_buf* in, int32_t n_in,
                   const dex_buf* resid, int32_t n_resid,
                   const dex_buf* t_in, int32_t n_t_in,
                   dex_buf* t_out, int32_t n_t_out,
                   void* workspace, size_t ws_bytes,
                   void* hip_stream);

/* Regular segmented reduction (Sec. 6.1.3: the accumulator indexed by a subset
 * of the loop indices, `for i j. acc!i += values.i.j`):
 *   out[i] (= or, with DEX_ACCUMULATE, +=) sum_j values[i, j],  i < rows, j < cols
 * values: device, rows x cols FP32 row-major; out: device, rows FP32. Each row
 * is summed by a fixed group of lanes in FP64 in a fixed order (bit-reproducible). rows = 0
 * does nothing; cols = 0 gives zero sums. Negative sizes or null pointers with
 * rows > 0: DEX_ERR_INVALID_ARG, before anything is enqueued. */
dex_status dex_reduce_rows(float* out, const float* values, int64_t rows, int64_t cols,
                           uint32_t flags, void* hip_stream);

/* Complete reduction (Sec. 6.1.3: the accumulator never indexed,
 * `for i. acc += values.i`): out[0] (= or += with DEX_ACCUMULATE) sum_i values[i].
 * values: device, n FP32; out: device, one FP32. Per-block FP64 partial sums over
 * a fixed grid, then one block adds them in order (bit-reproducible).
 * workspace: device scratch of at least DEX_REDUCE_WS_BYTES bytes. */
#define DEX_REDUCE_WS_BYTES 8192
dex_status dex_reduce_all(float* out, const float* values, int64_t n, uint32_t flags,
                          void* workspace, size_t ws_bytes, void* hip_stream);

/* dex_reduce_all without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). It allocates nothing: the per-block FP64
 * partials go to a fixed 8 KiB array (1024 doubles) that the library holds in
 * each GPU's memory from the first call on that GPU (or dex_init) until the
 * process ends. That size does not depend on n, so any n >= 0 is accepted;
 * arguments and flags otherwise as for dex_reduce_all, and the result is bit
 * for bit the same. Calls that overlap on one GPU (other streams, other host
 * threads) share the array and race; calls on one stream are ordered. */
dex_status dex_reduce_all_noalloc(float* out, const float* values, int64_t n, uint32_t flags,
                                  void* hip_stream);

/*
 * acc!(idx[j]) += scale[j] * vals[j, :]  for j in [0, n)      (Sec. 2.3.2-2.3.3)
 *
 *   acc        device, n_rows x row_len, DEX_F32 or DEX_I32; accumulated into,
 *              never overwritten; not to be read until the stream reaches the
 *              end of this call (the write-only Ref of `runAccum`).
 *   idx        device, n entries, DEX_I32 or DEX_U32.
 *   vals       device, n x row_len of acc's type, or NULL meaning all ones.
 *   scale      device, n floats, or NULL meaning all ones (DEX_F32 only).
 *   flags      DEX_CHECK_BOUNDS / DEX_SYNC_CHECK. Without DEX_CHECK_BOUNDS an
 *              out-of-range index is still skipped (never written), but not counted.
 *   oob_count_dev  device int64, required with DEX_CHECK_BOUNDS; the number of
 *              out-of-range indices is added to it.
 * Integer accumulation is exact, hence identical under every schedule. Float
 * accumulation is associative only up to rounding (Sec. 2.3.2): duplicate
 * indices are first summed in registers/LDS within a block, then added with
 * global atomics, so the rounding order is unspecified.
 * With DEX_DETERMINISTIC (float only) the (index, position) pairs are radix
 * sorted and each run of equal indices is summed in index order by one owner,
 * so the result is bit-identical from run to run; needs the workspace below.
 * Integer with row_len == 1, vals == NULL and n_rows <= 65536 is the
 * histogram of Sec. 6.1.2 and uses LDS-private counters.
 */
dex_status dex_accum_scatter(void* acc, int32_t acc_dtype, int64_t n_rows, int64_t row_len,
                             const void* idx, int32_t idx_dtype,
                             const void* vals, const float* scale, int64_t n,
                             uint32_t flags, int64_t* oob_count_dev,
                             void* workspace, size_t ws_bytes,
                             void* hip_stream);

/* Scratch bytes that dex_accum_scatter needs for these arguments. */
dex_status dex_accum_scatter_workspace_bytes(int32_t acc_dtype, int64_t n_rows,
                                             int64_t row_len, int64_t n, int32_t has_vals,
                                             uint32_t flags, size_t* bytes);

/*
 * Host-side plan for DEX_GMM_BATCHED. `shapes` is host memory, B rows of
 * (N, D, K) int64 with 1 <= D <= 32, N >= 1, K >= 1 (D <= 8 runs on the vector
 * units, 9..16 and 17..32 on matrix-core tiles padded to 16 and 32); variant
 * DEX_GMM_PLAIN or DEX_GMM_F16X3 (fixed in the plan and the descriptor; the
 * operand cache of F16X3 holds the split parts). Fills *desc_out and
 * writes the plan (instance table and work lists, longest work first) into
 * host memory `plan` of *plan_bytes bytes. Call with plan == NULL to query
 * *plan_bytes. The caller copies the plan to the device and passes it as in[0].
 */
dex_status dex_gmm_batched_plan(const int64_t* shapes, int64_t B, int32_t variant,
                                dex_desc* desc_out, void* plan, size_t* plan_bytes);

/*
 * Autotuner: times every tile configuration of (d, role) on the caller's
 * buffers (arguments as for dex_fwd / dex_vjp) with HIP events, keeps the
 * fastest for the descriptor's shape class in a process-wide table that
 * dex_fwd / dex_vjp consult when d->config == 0, and returns it in *best.
 * The buffers' contents are overwritten. Enqueues on hip_stream and waits.
 */
dex_status dex_autotune(const dex_desc* d, int32_t role,
                        const dex_buf* in, int32_t n_in,
                        dex_buf* out, int32_t n_out,
                        dex_buf* resid, int32_t n_resid,
                        const dex_buf* ct_out, int32_t n_ct_out,
                        dex_buf* ct_in, int32_t n_ct_in,
                        void* workspace, size_t ws_bytes,
                        void* hip_stream, int32_t* best);

/* Drop every tuned configuration (the process-wide table). */
void dex_autotune_reset(void);

/*
 * Live kernel timing. When enabled, the library records a pair of HIP events on
 * the launching stream around each launch (or launch sequence) of the main
 * kernel of a path, identified as below; dex_profile_read waits for the
 * recorded events and returns their summed duration and the number of kernel
 * launches they cover. Disabled by default; enabling adds two event records
 * per covered launch.
 */
#define DEX_PROF_GMM_FWD      0 /* matrix-core forward tile kernel            */
#define DEX_PROF_GMM_VJP      1 /* matrix-core reverse tile kernel            */
#define DEX_PROF_SCATTER      2 /* float row scatter (sort + segmented sum)   */
#define DEX_PROF_HIST         3 /* LDS-private histogram kernel               */
#define DEX_PROF_GATHER       4 /* gather-scale forward                       */
#define DEX_PROF_GATHER_DW    5 /* cotangent of the gather weights            */
#define DEX_PROF_BGMM_FWD     6 /* batched forward persistent kernel          */
#define DEX_PROF_BGMM_VJP     7 /* batched reverse persistent kernel          */
#define DEX_PROF_STENCIL_FWD  8 /* forward steps (one range per dex_fwd)      */
#define DEX_PROF_STENCIL_VJP  9 /* reverse steps incl. recompute (per dex_vjp) */
#define DEX_PROF_GATHER_JVP  10 /* gather-scale forward mode (dex_jvp)        */
#define DEX_PROF_REDUCE_ROWS 11 /* regular segmented reduction                */
#define DEX_PROF_REDUCE_ALL  12 /* complete reduction (both passes)           */
#define DEX_PROF_GMM_JVP     13 /* GMM forward-mode tangent kernel (dex_jvp)   */
#define DEX_PROF_COUNT       14
void dex_profile_enable(int32_t on);
dex_status dex_profile_read(int32_t id, double* total_ms, int64_t* launches);
void dex_profile_reset(void);

#ifdef __cplusplus
}
#endif

#endif /* DEX_H */
