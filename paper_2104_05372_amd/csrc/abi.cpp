// The C ABI of libdexmi: argument checking, dispatch to the kernel files,
// status reporting, the tuned-configuration table and the autotuner.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "internal.h"

namespace dexi {

static thread_local char g_err[512] = "";

dex_status fail(dex_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

dex_status check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return DEX_OK;
  return fail(DEX_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

namespace {
struct DevInfo {
  bool checked = false;
  bool ok = false;
  bool scratch_ready = false;
  int cus = 0;
  char arch[64] = "";
};
std::mutex g_mu;
std::map<int, DevInfo> g_dev;

// tuned configurations: (kind, dtype, variant, role, dims...) -> config
using TuneKey = std::tuple<int, int, int, int, int64_t, int64_t, int64_t, int64_t>;
std::map<TuneKey, int> g_tuned;

TuneKey tune_key(const dex_desc& d, int role) {
  return TuneKey(d.kind, d.dtype, d.variant, role, d.dims[0], d.dims[1], d.dims[2], d.dims[3]);
}
}  // namespace

// ---- live kernel timing ----------------------------------------------------
namespace {
struct ProfRec {
  hipEvent_t e0, e1;
  int64_t launches;
};
std::mutex g_pmu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof[DEX_PROF_COUNT];
double g_prof_ms[DEX_PROF_COUNT] = {};
int64_t g_prof_n[DEX_PROF_COUNT] = {};
}  // namespace

ProfRange::ProfRange(int id_, hipStream_t s_) : id(id_), s(s_) {
  bool on;
  {
    std::lock_guard<std::mutex> lk(g_pmu);
    on = g_prof_on;
  }
  if (on && hipEventCreate(&e0) == hipSuccess) {
    if (hipEventRecord(e0, s) != hipSuccess) {
      hipEventDestroy(e0);
      e0 = nullptr;
    }
  } else {
    e0 = nullptr;
  }
}

void ProfRange::end(int64_t launches) {
  if (!e0) return;
  hipEvent_t e1;
  if (hipEventCreate(&e1) != hipSuccess) return;
  hipEventRecord(e1, s);
  std::lock_guard<std::mutex> lk(g_pmu);
  g_prof[id].push_back({e0, e1, launches});
  e0 = nullptr;
}

static void prof_collect(int id) {
  for (auto& r : g_prof[id]) {
    hipEventSynchronize(r.e1);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.e0, r.e1) == hipSuccess) {
      g_prof_ms[id] += ms;
      g_prof_n[id] += r.launches;
    }
    hipEventDestroy(r.e0);
    hipEventDestroy(r.e1);
  }
  g_prof[id].clear();
}

int num_cus() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  std::lock_guard<std::mutex> lk(g_mu);
  DevInfo& di = g_dev[dev];
  if (!di.cus) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) == hipSuccess) di.cus = p.multiProcessorCount;
    if (!di.cus) di.cus = 256;
  }
  return di.cus;
}

static dex_status ensure_device() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return check_hip(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_mu);
  DevInfo& di = g_dev[dev];
  if (!di.checked) {
    hipDeviceProp_t p;
    e = hipGetDeviceProperties(&p, dev);
    if (e != hipSuccess) return check_hip(e, "hipGetDeviceProperties");
    snprintf(di.arch, sizeof(di.arch), "%s", p.gcnArchName);
    di.cus = p.multiProcessorCount;
    di.ok = strncmp(p.gcnArchName, "gfx950", 6) == 0;
    di.checked = true;
  }
  if (!di.ok) return fail(DEX_ERR_UNSUPPORTED, "device %d is %s, libdexmi is built for gfx950", dev, di.arch);
  if (!di.scratch_ready) {  // per-device address of the library's own scratch array
    const dex_status st = reduce_scratch_init();
    if (st != DEX_OK) return st;
    di.scratch_ready = true;
  }
  return DEX_OK;
}

static int pick_config(const dex_desc& d, int role) {
  if (d.config > 0) return d.config - 1;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_tuned.find(tune_key(d, role));
  return it == g_tuned.end() ? 0 : it->second;
}

static size_t dtype_size(int32_t dt) {
  switch (dt) {
    case DEX_F64:
    case DEX_I64:
      return 8;
    case DEX_F32:
    case DEX_I32:
    case DEX_U32:
      return 4;
    case DEX_U8:
      return 1;
    default:
      return 0;
  }
}

// Check a buffer list entry: dtype, numel, non-null pointer when numel > 0.
static dex_status want(const dex_buf* b, int i, const char* role, int32_t dtype, int64_t numel) {
  const dex_buf& x = b[i];
  if (x.dtype != dtype)
    return fail(DEX_ERR_INVALID_ARG, "%s[%d]: dtype %d, expected %d", role, i, x.dtype, dtype);
  if (x.numel != numel)
    return fail(DEX_ERR_INVALID_ARG, "%s[%d]: %lld elements, expected %lld", role, i,
                (long long)x.numel, (long long)numel);
  if (numel > 0 && !x.ptr) return fail(DEX_ERR_INVALID_ARG, "%s[%d]: null pointer", role, i);
  return DEX_OK;
}

#define DEX_TRY(expr)              \
  do {                             \
    dex_status _s = (expr);        \
    if (_s != DEX_OK) return _s;   \
  } while (0)

static dex_status check_count(int32_t got, int32_t need, const char* role) {
  if (got != need) return fail(DEX_ERR_INVALID_ARG, "%s: %d buffers, expected %d", role, got, need);
  return DEX_OK;
}

static dex_status check_desc(const dex_desc* d) {
  if (!d) return fail(DEX_ERR_INVALID_ARG, "null descriptor");
  if (d->config < 0) return fail(DEX_ERR_INVALID_ARG, "negative config");
  switch (d->kind) {
    case DEX_GMM: {
      const int64_t N = d->dims[0], D = d->dims[1], K = d->dims[2];
      if (N < 1 || D < 1 || K < 1) return fail(DEX_ERR_INVALID_ARG, "GMM dims must be positive");
      if (D > 64) return fail(DEX_ERR_UNSUPPORTED, "GMM with D > 64 is not built");
      if (N > (int64_t(1) << 30) || K > (int64_t(1) << 20))
        return fail(DEX_ERR_UNSUPPORTED, "GMM too large");
      if (d->dtype != DEX_F32 && d->dtype != DEX_F64)
        return fail(DEX_ERR_INVALID_ARG, "GMM dtype must be F32 or F64");
      if (d->variant < DEX_GMM_PLAIN || d->variant > DEX_GMM_BF16X3)
        return fail(DEX_ERR_INVALID_ARG, "unknown GMM variant %d", d->variant);
      if (d->variant != DEX_GMM_PLAIN && d->dtype != DEX_F32)
        return fail(DEX_ERR_UNSUPPORTED, "BF16 variants take FP32 storage");
      return DEX_OK;
    }
    case DEX_GMM_BATCHED:
      if (d->dtype != DEX_F32) return fail(DEX_ERR_UNSUPPORTED, "batched GMM is FP32");
      if (d->dims[0] < 1) return fail(DEX_ERR_INVALID_ARG, "batched GMM: no instances");
      return DEX_OK;
    case DEX_GATHER_SCALE:
      if (d->dtype != DEX_F32) return fail(DEX_ERR_UNSUPPORTED, "gather is FP32");
      if (d->dims[0] < 1 || d->dims[1] < 1 || d->dims[2] < 0)
        return fail(DEX_ERR_INVALID_ARG, "gather dims");
      if (d->dims[0] > (int64_t(1) << 31) - 1)
        return fail(DEX_ERR_UNSUPPORTED, "gather: at most 2^31-1 rows (int32 indices)");
      if (d->dims[1] > (1 << 20)) return fail(DEX_ERR_UNSUPPORTED, "gather: row too long");
      return DEX_OK;
    case DEX_STENCIL5:
      if (d->dtype != DEX_F32) return fail(DEX_ERR_UNSUPPORTED, "stencil is FP32");
      if (d->dims[0] < 1 || d->dims[1] < 1 || d->dims[2] < 0 || d->dims[3] < 1)
        return fail(DEX_ERR_INVALID_ARG, "stencil dims {H, W, steps>=0, every>=1}");
      if (d->dims[0] * d->dims[1] > (int64_t(1) << 31))
        return fail(DEX_ERR_UNSUPPORTED, "stencil grid too large");
      if (d->variant != DEX_STENCIL_RECOMPUTE && d->variant != DEX_STENCIL_LINEAR)
        return fail(DEX_ERR_INVALID_ARG, "unknown stencil variant %d", d->variant);
      if (d->variant == DEX_STENCIL_LINEAR && d->fparams[1] != 0.0)
        return fail(DEX_ERR_INVALID_ARG, "the linear reverse pass needs rho == 0");
      return DEX_OK;
    default:
      return fail(DEX_ERR_INVALID_ARG, "unknown kind %d", d->kind);
  }
}

static size_t ws_bytes(const dex_desc& d, int role) {
  if (role == DEX_WS_JVP && d.kind == DEX_GATHER_SCALE) return 0;  // (the gather needs none)
  switch (d.kind) {
    case DEX_GMM:
      return gmm_ws_bytes(d, role);
    case DEX_GMM_BATCHED:
      return gmm_batched_ws_bytes(d, role);
    case DEX_STENCIL5:
      return stencil_ws_bytes(d, role);
    case DEX_GATHER_SCALE:
      return role == DEX_WS_VJP ? scatter_ws_bytes(DEX_F32, d.dims[0], d.dims[1], d.dims[2], true, true)
                                : 0;
    default:
      return 0;
  }
}

static dex_status check_ws(const dex_desc& d, int role, void* ws, size_t wsb) {
  const size_t need = ws_bytes(d, role);
  if (need && (!ws || wsb < need))
    return fail(DEX_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, wsb);
  return DEX_OK;
}

}  // namespace dexi

using namespace dexi;

extern "C" {

const char* dex_status_string(dex_status s) {
  switch (s) {
    case DEX_OK:
      return "ok";
    case DEX_ERR_INVALID_ARG:
      return "invalid argument";
    case DEX_ERR_OUT_OF_RANGE:
      return "index out of range";
    case DEX_ERR_UNSUPPORTED:
      return "unsupported";
    case DEX_ERR_HIP:
      return "HIP error";
    case DEX_ERR_WORKSPACE:
      return "workspace too small";
    default:
      return "unknown status";
  }
}

const char* dex_last_error(void) { return g_err; }

const char* dex_version(void) { return "dexmi 0.1 gfx950"; }

dex_status dex_init(void) { return ensure_device(); }

dex_status dex_workspace_bytes(const dex_desc* d, int32_t role, size_t* bytes) {
  DEX_TRY(check_desc(d));
  if (!bytes) return fail(DEX_ERR_INVALID_ARG, "null output");
  if (role < DEX_WS_FWD || role > DEX_WS_JVP) return fail(DEX_ERR_INVALID_ARG, "bad role");
  *bytes = ws_bytes(*d, role);
  return DEX_OK;
}

dex_status dex_num_configs(const dex_desc* d, int32_t role, int32_t* count) {
  DEX_TRY(check_desc(d));
  if (!count) return fail(DEX_ERR_INVALID_ARG, "null output");
  switch (d->kind) {
    case DEX_GMM:
      *count = gmm_num_configs(*d, role);
      break;
    case DEX_GMM_BATCHED:
      *count = gmm_batched_num_configs(*d, role);
      break;
    case DEX_STENCIL5:
      *count = stencil_num_configs(*d, role);
      break;
    case DEX_GATHER_SCALE:
      *count = role == DEX_WS_VJP ? 2 : 1;
      break;
    default:
      *count = 1;
  }
  return DEX_OK;
}

dex_status dex_fwd(const dex_desc* d, const dex_buf* in, int32_t n_in, dex_buf* out, int32_t n_out,
                   dex_buf* resid, int32_t n_resid, void* workspace, size_t ws_bytes_,
                   void* hip_stream) {
  DEX_TRY(check_desc(d));
  if ((n_in && !in) || (n_out && !out) || (n_resid && !resid))
    return fail(DEX_ERR_INVALID_ARG, "null buffer list");
  // every argument is checked on the host first; the device is set up (and
  // checked to be gfx950) only before the launches
  hipStream_t s = (hipStream_t)hip_stream;
  const int cfg = pick_config(*d, DEX_WS_FWD);
  int32_t nc = 1;
  dex_num_configs(d, DEX_WS_FWD, &nc);
  if (cfg >= nc) return fail(DEX_ERR_INVALID_ARG, "config %d out of range (%d configs)", cfg + 1, nc);
  DEX_TRY(check_ws(*d, DEX_WS_FWD, workspace, ws_bytes_));
  switch (d->kind) {
    case DEX_GMM: {
      const int64_t N = d->dims[0], D = d->dims[1], K = d->dims[2], L = D * (D - 1) / 2;
      const int32_t t = d->dtype;
      DEX_TRY(check_count(n_in, 5, "in"));
      DEX_TRY(want(in, 0, "in", t, K));
      DEX_TRY(want(in, 1, "in", t, K * D));
      DEX_TRY(want(in, 2, "in", t, K * D));
      DEX_TRY(want(in, 3, "in", t, K * L));
      DEX_TRY(want(in, 4, "in", t, N * D));
      DEX_TRY(check_count(n_out, 1, "out"));
      DEX_TRY(want(out, 0, "out", t, 1));
      DEX_TRY(check_count(n_resid, 2, "resid"));
      DEX_TRY(want(resid, 0, "resid", t, N));
      DEX_TRY(want(resid, 1, "resid", DEX_U8, (int64_t)gmm_cache_bytes(*d)));
      GmmPtrs p{in[0].ptr, in[1].ptr, in[2].ptr, in[3].ptr, in[4].ptr};
      DEX_TRY(ensure_device());
      return gmm_fwd(*d, cfg, p, out[0].ptr, resid[0].ptr, resid[1].ptr, workspace, s);
    }
    case DEX_GMM_BATCHED: {
      const int64_t B = d->dims[0], sumN = d->dims[1], sumK = d->dims[2], sumKD = d->dims[3],
                    sumKL = d->dims[4], sumND = d->dims[5], plan_bytes = d->dims[6];
      DEX_TRY(check_count(n_in, 6, "in"));
      DEX_TRY(want(in, 0, "in", DEX_U8, plan_bytes));
      DEX_TRY(want(in, 1, "in", DEX_F32, sumK));
      DEX_TRY(want(in, 2, "in", DEX_F32, sumKD));
      DEX_TRY(want(in, 3, "in", DEX_F32, sumKD));
      DEX_TRY(want(in, 4, "in", DEX_F32, sumKL));
      DEX_TRY(want(in, 5, "in", DEX_F32, sumND));
      DEX_TRY(check_count(n_out, 1, "out"));
      DEX_TRY(want(out, 0, "out", DEX_F32, B));
      DEX_TRY(check_count(n_resid, 2, "resid"));
      DEX_TRY(want(resid, 0, "resid", DEX_F32, sumN));
      DEX_TRY(want(resid, 1, "resid", DEX_U8, d->dims[7]));
      GmmPtrs p{in[1].ptr, in[2].ptr, in[3].ptr, in[4].ptr, in[5].ptr};
      DEX_TRY(ensure_device());
      return gmm_batched_fwd(*d, cfg, in[0].ptr, p, out[0].ptr, resid[0].ptr, resid[1].ptr,
                             workspace, s);
    }
    case DEX_GATHER_SCALE: {
      const int64_t V = d->dims[0], R = d->dims[1], n = d->dims[2];
      DEX_TRY(check_count(n_in, 3, "in"));
      DEX_TRY(want(in, 0, "in", DEX_F32, V * R));
      DEX_TRY(want(in, 1, "in", DEX_I32, n));
      DEX_TRY(want(in, 2, "in", DEX_F32, n));
      DEX_TRY(check_count(n_out, 1, "out"));
      DEX_TRY(want(out, 0, "out", DEX_F32, n * R));
      DEX_TRY(ensure_device());
      return gather_fwd((const float*)in[0].ptr, (const int32_t*)in[1].ptr, (const float*)in[2].ptr,
                        V, R, n, (float*)out[0].ptr, false, nullptr, s);
    }
    case DEX_STENCIL5: {
      const int64_t n = d->dims[0] * d->dims[1];
      const int64_t nck = (d->dims[2] + d->dims[3] - 1) / d->dims[3];
      DEX_TRY(check_count(n_in, 2, "in"));
      DEX_TRY(want(in, 0, "in", DEX_F32, n));
      DEX_TRY(want(in, 1, "in", DEX_F32, n));
      DEX_TRY(check_count(n_out, 2, "out"));
      DEX_TRY(want(out, 0, "out", DEX_F32, 1));
      DEX_TRY(want(out, 1, "out", DEX_F32, n));
      DEX_TRY(check_count(n_resid, 2, "resid"));
      DEX_TRY(want(resid, 0, "resid", DEX_F32, nck * n));
      DEX_TRY(want(resid, 1, "resid", DEX_F32, n));
      if (out[1].ptr == in[0].ptr) return fail(DEX_ERR_INVALID_ARG, "uT must not alias u0");
      DEX_TRY(ensure_device());
      DEX_TRY(stencil_fwd(*d, cfg, (const float*)in[0].ptr, (const float*)in[1].ptr,
                          (float*)out[0].ptr, (float*)out[1].ptr, (float*)resid[0].ptr, workspace, s));
      if (resid[1].ptr != out[1].ptr) {
        hipError_t e = hipMemcpyAsync(resid[1].ptr, out[1].ptr, (size_t)n * 4,
                                      hipMemcpyDeviceToDevice, s);
        return check_hip(e, "stencil residual copy");
      }
      return DEX_OK;
    }
  }
  return fail(DEX_ERR_INVALID_ARG, "unknown kind");
}

dex_status dex_jvp(const dex_desc* d, const dex_buf* in, int32_t n_in, const dex_buf* resid,
                   int32_t n_resid, const dex_buf* t_in, int32_t n_t_in, dex_buf* t_out,
                   int32_t n_t_out, void* workspace, size_t ws_bytes_, void* hip_stream) {
  DEX_TRY(check_desc(d));
  if ((n_in && !in) || (n_resid && !resid) || (n_t_in && !t_in) || (n_t_out && !t_out))
    return fail(DEX_ERR_INVALID_ARG, "null buffer list");
  if (d->kind == DEX_GMM) {
    const int64_t N = d->dims[0], D = d->dims[1], K = d->dims[2], L = D * (D - 1) / 2;
    const int32_t t = d->dtype;
    DEX_TRY(check_count(n_in, 5, "in"));
    DEX_TRY(want(in, 0, "in", t, K));
    DEX_TRY(want(in, 1, "in", t, K * D));
    DEX_TRY(want(in, 2, "in", t, K * D));
    DEX_TRY(want(in, 3, "in", t, K * L));
    DEX_TRY(want(in, 4, "in", t, N * D));
    DEX_TRY(check_count(n_resid, 2, "resid"));
    DEX_TRY(want(resid, 0, "resid", t, N));
    DEX_TRY(want(resid, 1, "resid", DEX_U8, (int64_t)gmm_cache_bytes(*d)));
    DEX_TRY(check_count(n_t_in, 4, "t_in"));
    DEX_TRY(want(t_in, 0, "t_in", t, K));
    DEX_TRY(want(t_in, 1, "t_in", t, K * D));
    DEX_TRY(want(t_in, 2, "t_in", t, K * D));
    DEX_TRY(want(t_in, 3, "t_in", t, K * L));
    DEX_TRY(check_count(n_t_out, 1, "t_out"));
    DEX_TRY(want(t_out, 0, "t_out", t, 1));
    DEX_TRY(check_ws(*d, DEX_WS_JVP, workspace, ws_bytes_));
    DEX_TRY(ensure_device());
    const int cfg = pick_config(*d, DEX_WS_VJP);
    GmmPtrs p{in[0].ptr, in[1].ptr, in[2].ptr, in[3].ptr, in[4].ptr};
    GmmGrads tg{t_in[0].ptr, t_in[1].ptr, t_in[2].ptr, t_in[3].ptr};
    return gmm_jvp(*d, cfg, p, resid[0].ptr, resid[1].ptr, tg, t_out[0].ptr, workspace,
                   (hipStream_t)hip_stream);
  }
  if (n_resid != 0) return fail(DEX_ERR_INVALID_ARG, "no residuals for this kind");
  if (d->kind == DEX_STENCIL5) {
    const int64_t n = d->dims[0] * d->dims[1];
    DEX_TRY(check_count(n_in, 2, "in"));
    DEX_TRY(want(in, 0, "in", DEX_F32, n));
    DEX_TRY(want(in, 1, "in", DEX_F32, n));
    DEX_TRY(check_count(n_t_in, 2, "t_in"));
    DEX_TRY(want(t_in, 0, "t_in", DEX_F32, n));
    DEX_TRY(want(t_in, 1, "t_in", DEX_F32, n));
    DEX_TRY(check_count(n_t_out, 1, "t_out"));
    DEX_TRY(want(t_out, 0, "t_out", DEX_F32, 1));
    DEX_TRY(check_ws(*d, DEX_WS_JVP, workspace, ws_bytes_));
    DEX_TRY(ensure_device());
    return stencil_jvp(*d, (const float*)in[0].ptr, (const float*)in[1].ptr,
                       (const float*)t_in[0].ptr, (const float*)t_in[1].ptr,
                       (float*)t_out[0].ptr, workspace, (hipStream_t)hip_stream);
  }
  if (d->kind != DEX_GATHER_SCALE)
    return fail(DEX_ERR_UNSUPPORTED,
                "forward mode is implemented for DEX_GMM, DEX_GATHER_SCALE and DEX_STENCIL5");
  const int64_t V = d->dims[0], R = d->dims[1], n = d->dims[2];
  DEX_TRY(check_count(n_in, 3, "in"));
  DEX_TRY(want(in, 0, "in", DEX_F32, V * R));
  DEX_TRY(want(in, 1, "in", DEX_I32, n));
  DEX_TRY(want(in, 2, "in", DEX_F32, n));
  DEX_TRY(check_count(n_t_in, 2, "t_in"));
  DEX_TRY(want(t_in, 0, "t_in", DEX_F32, V * R));
  DEX_TRY(want(t_in, 1, "t_in", DEX_F32, n));
  DEX_TRY(check_count(n_t_out, 1, "t_out"));
  DEX_TRY(want(t_out, 0, "t_out", DEX_F32, n * R));
  DEX_TRY(check_ws(*d, DEX_WS_JVP, workspace, ws_bytes_));
  DEX_TRY(ensure_device());
  hipStream_t s = (hipStream_t)hip_stream;
  return gather_jvp((const float*)in[0].ptr, (const float*)t_in[0].ptr, (const int32_t*)in[1].ptr,
                    (const float*)in[2].ptr, (const float*)t_in[1].ptr, V, R, n,
                    (float*)t_out[0].ptr, s);
}

dex_status dex_reduce_rows(float* out, const float* values, int64_t rows, int64_t cols,
                           uint32_t flags, void* hip_stream) {
  if (rows < 0 || cols < 0) return fail(DEX_ERR_INVALID_ARG, "negative size");
  if (rows > 0 && (!out || (cols > 0 && !values))) return fail(DEX_ERR_INVALID_ARG, "null buffer");
  if (flags & ~DEX_ACCUMULATE) return fail(DEX_ERR_INVALID_ARG, "unknown flags");
  if (rows == 0) return DEX_OK;
  DEX_TRY(ensure_device());
  return reduce_rows(out, values, rows, cols, flags & DEX_ACCUMULATE, (hipStream_t)hip_stream);
}

dex_status dex_reduce_all(float* out, const float* values, int64_t n, uint32_t flags,
                          void* workspace, size_t ws_bytes_, void* hip_stream) {
  if (n < 0) return fail(DEX_ERR_INVALID_ARG, "negative size");
  if (!out || (n > 0 && !values)) return fail(DEX_ERR_INVALID_ARG, "null buffer");
  if (flags & ~DEX_ACCUMULATE) return fail(DEX_ERR_INVALID_ARG, "unknown flags");
  static_assert(kReduceBlocks * 8 <= DEX_REDUCE_WS_BYTES, "partials fit the documented workspace");
  if (!workspace || ws_bytes_ < DEX_REDUCE_WS_BYTES)
    return fail(DEX_ERR_WORKSPACE, "workspace of %d bytes needed", DEX_REDUCE_WS_BYTES);
  DEX_TRY(ensure_device());
  return reduce_all(out, values, n, flags & DEX_ACCUMULATE, workspace, (hipStream_t)hip_stream);
}

dex_status dex_reduce_all_noalloc(float* out, const float* values, int64_t n, uint32_t flags,
                                  void* hip_stream) {
  if (n < 0) return fail(DEX_ERR_INVALID_ARG, "negative size");
  if (!out || (n > 0 && !values)) return fail(DEX_ERR_INVALID_ARG, "null buffer");
  if (flags & ~DEX_ACCUMULATE) return fail(DEX_ERR_INVALID_ARG, "unknown flags");
  DEX_TRY(ensure_device());
  return reduce_all_noalloc(out, values, n, flags & DEX_ACCUMULATE, (hipStream_t)hip_stream);
}

dex_status dex_vjp(const dex_desc* d, const dex_buf* in, int32_t n_in, const dex_buf* resid,
                   int32_t n_resid, const dex_buf* ct_out, int32_t n_ct_out, dex_buf* ct_in,
                   int32_t n_ct_in, uint32_t flags, void* workspace, size_t ws_bytes_,
                   void* hip_stream) {
  DEX_TRY(check_desc(d));
  if ((n_in && !in) || (n_resid && !resid) || (n_ct_out && !ct_out) || (n_ct_in && !ct_in))
    return fail(DEX_ERR_INVALID_ARG, "null buffer list");
  // every argument is checked on the host first; the device is set up (and
  // checked to be gfx950) only before the launches
  hipStream_t s = (hipStream_t)hip_stream;
  const bool acc = flags & DEX_ACCUMULATE;
  const int cfg = pick_config(*d, DEX_WS_VJP);
  int32_t nc = 1;
  dex_num_configs(d, DEX_WS_VJP, &nc);
  if (cfg >= nc) return fail(DEX_ERR_INVALID_ARG, "config %d out of range (%d configs)", cfg + 1, nc);
  DEX_TRY(check_ws(*d, DEX_WS_VJP, workspace, ws_bytes_));
  switch (d->kind) {
    case DEX_GMM: {
      const int64_t N = d->dims[0], D = d->dims[1], K = d->dims[2], L = D * (D - 1) / 2;
      const int32_t t = d->dtype;
      DEX_TRY(check_count(n_in, 5, "in"));
      DEX_TRY(want(in, 0, "in", t, K));
      DEX_TRY(want(in, 1, "in", t, K * D));
      DEX_TRY(want(in, 2, "in", t, K * D));
      DEX_TRY(want(in, 3, "in", t, K * L));
      DEX_TRY(want(in, 4, "in", t, N * D));
      DEX_TRY(check_count(n_resid, 2, "resid"));
      DEX_TRY(want(resid, 0, "resid", t, N));
      DEX_TRY(want(resid, 1, "resid", DEX_U8, (int64_t)gmm_cache_bytes(*d)));
      DEX_TRY(check_count(n_ct_out, 1, "ct_out"));
      DEX_TRY(want(ct_out, 0, "ct_out", t, 1));
      DEX_TRY(check_count(n_ct_in, 4, "ct_in"));
      DEX_TRY(want(ct_in, 0, "ct_in", t, K));
      DEX_TRY(want(ct_in, 1, "ct_in", t, K * D));
      DEX_TRY(want(ct_in, 2, "ct_in", t, K * D));
      DEX_TRY(want(ct_in, 3, "ct_in", t, K * L));
      GmmPtrs p{in[0].ptr, in[1].ptr, in[2].ptr, in[3].ptr, in[4].ptr};
      GmmGrads g{ct_in[0].ptr, ct_in[1].ptr, ct_in[2].ptr, ct_in[3].ptr};
      DEX_TRY(ensure_device());
      return gmm_vjp(*d, cfg, p, resid[0].ptr, resid[1].ptr, ct_out[0].ptr, g, acc, workspace, s);
    }
    case DEX_GMM_BATCHED: {
      const int64_t B = d->dims[0], sumN = d->dims[1], sumK = d->dims[2], sumKD = d->dims[3],
                    sumKL = d->dims[4], sumND = d->dims[5], plan_bytes = d->dims[6];
      DEX_TRY(check_count(n_in, 6, "in"));
      DEX_TRY(want(in, 0, "in", DEX_U8, plan_bytes));
      DEX_TRY(want(in, 1, "in", DEX_F32, sumK));
      DEX_TRY(want(in, 2, "in", DEX_F32, sumKD));
      DEX_TRY(want(in, 3, "in", DEX_F32, sumKD));
      DEX_TRY(want(in, 4, "in", DEX_F32, sumKL));
      DEX_TRY(want(in, 5, "in", DEX_F32, sumND));
      DEX_TRY(check_count(n_resid, 2, "resid"));
      DEX_TRY(want(resid, 0, "resid", DEX_F32, sumN));
      DEX_TRY(want(resid, 1, "resid", DEX_U8, d->dims[7]));
      DEX_TRY(check_count(n_ct_out, 1, "ct_out"));
      DEX_TRY(want(ct_out, 0, "ct_out", DEX_F32, B));
      DEX_TRY(check_count(n_ct_in, 4, "ct_in"));
      DEX_TRY(want(ct_in, 0, "ct_in", DEX_F32, sumK));
      DEX_TRY(want(ct_in, 1, "ct_in", DEX_F32, sumKD));
      DEX_TRY(want(ct_in, 2, "ct_in", DEX_F32, sumKD));
      DEX_TRY(want(ct_in, 3, "ct_in", DEX_F32, sumKL));
      GmmPtrs p{in[1].ptr, in[2].ptr, in[3].ptr, in[4].ptr, in[5].ptr};
      GmmGrads g{ct_in[0].ptr, ct_in[1].ptr, ct_in[2].ptr, ct_in[3].ptr};
      DEX_TRY(ensure_device());
      return gmm_batched_vjp(*d, cfg, in[0].ptr, p, resid[0].ptr, resid[1].ptr, ct_out[0].ptr, g,
                             acc, workspace, s);
    }
    case DEX_GATHER_SCALE: {
      const int64_t V = d->dims[0], R = d->dims[1], n = d->dims[2];
      DEX_TRY(check_count(n_in, 3, "in"));
      DEX_TRY(want(in, 0, "in", DEX_F32, V * R));
      DEX_TRY(want(in, 1, "in", DEX_I32, n));
      DEX_TRY(want(in, 2, "in", DEX_F32, n));
      if (n_resid != 0) return fail(DEX_ERR_INVALID_ARG, "gather has no residuals");
      DEX_TRY(check_count(n_ct_out, 1, "ct_out"));
      DEX_TRY(want(ct_out, 0, "ct_out", DEX_F32, n * R));
      DEX_TRY(check_count(n_ct_in, 2, "ct_in"));
      DEX_TRY(want(ct_in, 0, "ct_in", DEX_F32, V * R));
      const bool with_dw = !(flags & DEX_NO_DW);
      DEX_TRY(want(ct_in, 1, "ct_in", DEX_F32, with_dw ? n : 0));
      DEX_TRY(ensure_device());
      // config 1 (default): radix sort + one owner per row; config 2: block sort +
      // run sums + atomics
      const int path = cfg == 0 ? kScatterSorted : kScatterAtomic;
      if (!acc) DEX_TRY(fill_zero(ct_in[0].ptr, (size_t)(V * R) * 4, s));
      DEX_TRY(accum_scatter(ct_in[0].ptr, DEX_F32, V, R, in[1].ptr, DEX_I32, ct_out[0].ptr,
                            (const float*)in[2].ptr, n, false, nullptr, workspace, ws_bytes_, path,
                            s, !acc));
      if (with_dw)
        DEX_TRY(gather_dw((const float*)in[0].ptr, (const int32_t*)in[1].ptr,
                          (const float*)ct_out[0].ptr, V, R, n, (float*)ct_in[1].ptr, acc, s));
      return DEX_OK;
    }
    case DEX_STENCIL5: {
      const int64_t n = d->dims[0] * d->dims[1];
      const int64_t nck = (d->dims[2] + d->dims[3] - 1) / d->dims[3];
      DEX_TRY(check_count(n_in, 2, "in"));
      DEX_TRY(want(in, 0, "in", DEX_F32, n));
      DEX_TRY(want(in, 1, "in", DEX_F32, n));
      DEX_TRY(check_count(n_resid, 2, "resid"));
      DEX_TRY(want(resid, 0, "resid", DEX_F32, nck * n));
      DEX_TRY(want(resid, 1, "resid", DEX_F32, n));
      DEX_TRY(check_count(n_ct_out, 1, "ct_out"));
      DEX_TRY(want(ct_out, 0, "ct_out", DEX_F32, 1));
      DEX_TRY(check_count(n_ct_in, 1, "ct_in"));
      DEX_TRY(want(ct_in, 0, "ct_in", DEX_F32, n));
      DEX_TRY(ensure_device());
      return stencil_vjp(*d, cfg, (const float*)in[0].ptr, (const float*)in[1].ptr,
                         (const float*)resid[0].ptr, (const float*)resid[1].ptr,
                         (const float*)ct_out[0].ptr, (float*)ct_in[0].ptr, acc, workspace, s);
    }
  }
  return fail(DEX_ERR_INVALID_ARG, "unknown kind");
}

dex_status dex_accum_scatter_workspace_bytes(int32_t acc_dtype, int64_t n_rows, int64_t row_len,
                                             int64_t n, int32_t has_vals, uint32_t flags,
                                             size_t* bytes) {
  if (!bytes) return fail(DEX_ERR_INVALID_ARG, "null output");
  *bytes = scatter_ws_bytes(acc_dtype, n_rows, row_len, n, has_vals != 0,
                            (flags & DEX_DETERMINISTIC) != 0);
  return DEX_OK;
}

dex_status dex_accum_scatter(void* acc, int32_t acc_dtype, int64_t n_rows, int64_t row_len,
                             const void* idx, int32_t idx_dtype, const void* vals,
                             const float* scale, int64_t n, uint32_t flags,
                             int64_t* oob_count_dev, void* workspace, size_t ws_bytes_,
                             void* hip_stream) {
  if (acc_dtype != DEX_F32 && acc_dtype != DEX_I32)
    return fail(DEX_ERR_INVALID_ARG, "acc dtype must be F32 or I32");
  if (idx_dtype != DEX_I32 && idx_dtype != DEX_U32)
    return fail(DEX_ERR_INVALID_ARG, "idx dtype must be I32 or U32");
  if (n_rows < 1 || row_len < 1 || n < 0) return fail(DEX_ERR_INVALID_ARG, "bad sizes");
  if (n_rows > (int64_t(1) << 40) || row_len > (int64_t(1) << 24))
    return fail(DEX_ERR_UNSUPPORTED, "table too large");
  if (n > 0 && (!acc || !idx)) return fail(DEX_ERR_INVALID_ARG, "null acc or idx");
  if (acc_dtype == DEX_I32 && scale) return fail(DEX_ERR_INVALID_ARG, "integer accumulation takes no scale");
  const bool check = flags & DEX_CHECK_BOUNDS;
  if (check && !oob_count_dev) return fail(DEX_ERR_INVALID_ARG, "DEX_CHECK_BOUNDS needs oob_count_dev");
  if ((flags & DEX_DETERMINISTIC) && acc_dtype != DEX_F32)
    return fail(DEX_ERR_INVALID_ARG, "DEX_DETERMINISTIC applies to float accumulation");
  {
    const size_t need = scatter_ws_bytes(acc_dtype, n_rows, row_len, n, vals != nullptr,
                                         (flags & DEX_DETERMINISTIC) != 0);
    if (need && (!workspace || ws_bytes_ < need))
      return fail(DEX_ERR_WORKSPACE, "this accumulation needs %zu workspace bytes, got %zu", need,
                  workspace ? ws_bytes_ : (size_t)0);
  }
  DEX_TRY(ensure_device());
  hipStream_t s = (hipStream_t)hip_stream;
  long long before = 0, after = 0;
  const bool sync = check && (flags & DEX_SYNC_CHECK);
  if (sync) {
    DEX_TRY(check_hip(hipMemcpyAsync(&before, oob_count_dev, 8, hipMemcpyDeviceToHost, s), "oob read"));
    DEX_TRY(check_hip(hipStreamSynchronize(s), "sync"));
  }
  const int path = (flags & DEX_DETERMINISTIC) ? kScatterSorted : kScatterAtomic;
  if (path == 1 && acc_dtype != DEX_F32)
    return fail(DEX_ERR_INVALID_ARG, "DEX_DETERMINISTIC applies to float accumulation");
  DEX_TRY(accum_scatter(acc, acc_dtype, n_rows, row_len, idx, idx_dtype, vals, scale, n, check,
                        oob_count_dev, workspace, ws_bytes_, path, s));
  if (sync) {
    DEX_TRY(check_hip(hipMemcpyAsync(&after, oob_count_dev, 8, hipMemcpyDeviceToHost, s), "oob read"));
    DEX_TRY(check_hip(hipStreamSynchronize(s), "sync"));
    if (after != before)
      return fail(DEX_ERR_OUT_OF_RANGE, "%lld indices outside [0, %lld)", after - before, (long long)n_rows);
  }
  return DEX_OK;
}

dex_status dex_gmm_batched_plan(const int64_t* shapes, int64_t B, int32_t variant,
                                dex_desc* desc_out, void* plan, size_t* plan_bytes) {
  if (!shapes || B < 1 || !plan_bytes || !desc_out)
    return fail(DEX_ERR_INVALID_ARG, "batched plan: null argument or B < 1");
  if (variant != DEX_GMM_PLAIN && variant != DEX_GMM_F16X3)
    return fail(DEX_ERR_UNSUPPORTED, "batched GMM: variant PLAIN or F16X3");
  for (int64_t b = 0; b < B; ++b) {
    const int64_t N = shapes[3 * b], D = shapes[3 * b + 1], K = shapes[3 * b + 2];
    if (N < 1 || K < 1 || D < 1 || D > 32)
      return fail(DEX_ERR_UNSUPPORTED, "instance %lld: N>=1, K>=1, 1<=D<=32", (long long)b);
    if (N > (int64_t(1) << 26) || K > 4096) return fail(DEX_ERR_UNSUPPORTED, "instance too large");
  }
  const size_t need = gmm_batched_plan_bytes(B, shapes, variant);
  if (!plan) {
    *plan_bytes = need;
    return gmm_batched_plan(shapes, B, variant, desc_out, nullptr, need);
  }
  if (*plan_bytes < need) return fail(DEX_ERR_INVALID_ARG, "plan buffer too small");
  return gmm_batched_plan(shapes, B, variant, desc_out, plan, need);
}

dex_status dex_autotune(const dex_desc* d, int32_t role, const dex_buf* in, int32_t n_in,
                        dex_buf* out, int32_t n_out, dex_buf* resid, int32_t n_resid,
                        const dex_buf* ct_out, int32_t n_ct_out, dex_buf* ct_in, int32_t n_ct_in,
                        void* workspace, size_t ws_bytes_, void* hip_stream, int32_t* best) {
  DEX_TRY(check_desc(d));
  if (role != DEX_WS_FWD && role != DEX_WS_VJP) return fail(DEX_ERR_INVALID_ARG, "role");
  DEX_TRY(ensure_device());
  int32_t nc = 1;
  DEX_TRY(dex_num_configs(d, role, &nc));
  hipStream_t s = (hipStream_t)hip_stream;
  hipEvent_t e0, e1;
  DEX_TRY(check_hip(hipEventCreate(&e0), "event"));
  DEX_TRY(check_hip(hipEventCreate(&e1), "event"));
  float best_ms = 1e30f;
  int best_c = 0;
  dex_status last = DEX_OK;
  for (int c = 0; c < nc; ++c) {
    dex_desc dc = *d;
    dc.config = c + 1;
    auto run = [&]() -> dex_status {
      if (role == DEX_WS_FWD)
        return dex_fwd(&dc, in, n_in, out, n_out, resid, n_resid, workspace, ws_bytes_, hip_stream);
      return dex_vjp(&dc, in, n_in, resid, n_resid, ct_out, n_ct_out, ct_in, n_ct_in, 0, workspace,
                     ws_bytes_, hip_stream);
    };
    dex_status st = run();  // warm-up
    if (st != DEX_OK) {
      last = st;
      continue;
    }
    std::vector<float> ts;
    for (int r = 0; r < 3; ++r) {
      hipEventRecord(e0, s);
      st = run();
      hipEventRecord(e1, s);
      hipEventSynchronize(e1);
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      if (st == DEX_OK) ts.push_back(ms);
    }
    if (ts.empty()) continue;
    std::sort(ts.begin(), ts.end());
    if (ts[ts.size() / 2] < best_ms) {
      best_ms = ts[ts.size() / 2];
      best_c = c;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (best_ms >= 1e30f) return last != DEX_OK ? last : fail(DEX_ERR_HIP, "no configuration ran");
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_tuned[tune_key(*d, role)] = best_c;
  }
  if (best) *best = best_c + 1;
  return DEX_OK;
}

void dex_autotune_reset(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_tuned.clear();
}

void dex_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_pmu);
  g_prof_on = on != 0;
}

dex_status dex_profile_read(int32_t id, double* total_ms, int64_t* launches) {
  if (id < 0 || id >= DEX_PROF_COUNT || !total_ms || !launches)
    return fail(DEX_ERR_INVALID_ARG, "profile id %d", id);
  std::lock_guard<std::mutex> lk(g_pmu);
  prof_collect(id);
  *total_ms = g_prof_ms[id];
  *launches = g_prof_n[id];
  return DEX_OK;
}

void dex_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_pmu);
  for (int i = 0; i < DEX_PROF_COUNT; ++i) {
    prof_collect(i);
    g_prof_ms[i] = 0.0;
    g_prof_n[i] = 0;
  }
}

}  // extern "C"
