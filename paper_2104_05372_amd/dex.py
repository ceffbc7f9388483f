"""ctypes binding of libdexmi (include/dex.h): argument marshalling only.

Every function here forwards to the C entry point of the same name; all
arithmetic runs in the library's HIP kernels. PyTorch supplies device memory
and the current HIP stream. If the shared library is missing or cannot be
loaded, every call raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdexmi.so")

# status codes
DEX_OK = 0
DEX_ERR_INVALID_ARG = -1
DEX_ERR_OUT_OF_RANGE = -2
DEX_ERR_UNSUPPORTED = -3
DEX_ERR_HIP = -4
DEX_ERR_WORKSPACE = -5
# dtypes
DEX_F64, DEX_F32, DEX_I32, DEX_U32, DEX_I64, DEX_U8 = 1, 2, 3, 4, 5, 6
# kinds
DEX_GMM, DEX_GMM_BATCHED, DEX_GATHER_SCALE, DEX_STENCIL5 = 1, 2, 3, 4
# variants
DEX_GMM_PLAIN, DEX_GMM_BF16, DEX_GMM_BF16X3, DEX_GMM_F16X3 = 0, 1, 2, 3
DEX_STENCIL_RECOMPUTE, DEX_STENCIL_LINEAR = 0, 1
# flags
DEX_ACCUMULATE, DEX_CHECK_BOUNDS, DEX_SYNC_CHECK, DEX_NO_DW, DEX_DETERMINISTIC = 1, 2, 4, 8, 16
# workspace roles
DEX_WS_FWD, DEX_WS_VJP, DEX_WS_RESID, DEX_WS_JVP = 0, 1, 2, 3

EXPORTS = (
    "dex_status_string", "dex_last_error", "dex_version", "dex_init", "dex_workspace_bytes",
    "dex_num_configs", "dex_fwd", "dex_vjp", "dex_jvp", "dex_reduce_rows", "dex_reduce_all",
    "dex_reduce_all_noalloc", "dex_accum_scatter",
    "dex_accum_scatter_workspace_bytes", "dex_gmm_batched_plan", "dex_autotune",
    "dex_autotune_reset", "dex_profile_enable", "dex_profile_read", "dex_profile_reset",
)


class DexDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("config", ctypes.c_int32),
                ("dims", ctypes.c_int64 * 8), ("fparams", ctypes.c_double * 4)]


class DexBuf(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p), ("numel", ctypes.c_int64),
                ("dtype", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class DexError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"dex status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libdexmi.so (once); raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2104_05372_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        S, P, I32, I64, SZ = ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        DP, BP = ctypes.POINTER(DexDesc), ctypes.POINTER(DexBuf)
        L.dex_status_string.restype = ctypes.c_char_p
        L.dex_status_string.argtypes = [S]
        L.dex_last_error.restype = ctypes.c_char_p
        L.dex_version.restype = ctypes.c_char_p
        L.dex_init.restype = S
        L.dex_workspace_bytes.argtypes = [DP, I32, ctypes.POINTER(SZ)]
        L.dex_workspace_bytes.restype = S
        L.dex_num_configs.argtypes = [DP, I32, ctypes.POINTER(I32)]
        L.dex_num_configs.restype = S
        L.dex_fwd.argtypes = [DP, BP, I32, BP, I32, BP, I32, P, SZ, P]
        L.dex_fwd.restype = S
        L.dex_vjp.argtypes = [DP, BP, I32, BP, I32, BP, I32, BP, I32, ctypes.c_uint32, P, SZ, P]
        L.dex_vjp.restype = S
        L.dex_jvp.argtypes = [DP, BP, I32, BP, I32, BP, I32, BP, I32, P, SZ, P]
        L.dex_jvp.restype = S
        L.dex_reduce_rows.argtypes = [P, P, I64, I64, ctypes.c_uint32, P]
        L.dex_reduce_rows.restype = S
        L.dex_reduce_all.argtypes = [P, P, I64, ctypes.c_uint32, P, SZ, P]
        L.dex_reduce_all.restype = S
        L.dex_reduce_all_noalloc.argtypes = [P, P, I64, ctypes.c_uint32, P]
        L.dex_reduce_all_noalloc.restype = S
        L.dex_accum_scatter.argtypes = [P, I32, I64, I64, P, I32, P, P, I64, ctypes.c_uint32, P, P, SZ, P]
        L.dex_accum_scatter.restype = S
        L.dex_accum_scatter_workspace_bytes.argtypes = [I32, I64, I64, I64, I32, ctypes.c_uint32,
                                                        ctypes.POINTER(SZ)]
        L.dex_accum_scatter_workspace_bytes.restype = S
        L.dex_gmm_batched_plan.argtypes = [P, I64, I32, DP, P, ctypes.POINTER(SZ)]
        L.dex_gmm_batched_plan.restype = S
        L.dex_autotune.argtypes = [DP, I32, BP, I32, BP, I32, BP, I32, BP, I32, BP, I32, P, SZ, P,
                                   ctypes.POINTER(I32)]
        L.dex_autotune.restype = S
        L.dex_autotune_reset.restype = None
        L.dex_profile_enable.argtypes = [I32]
        L.dex_profile_enable.restype = None
        L.dex_profile_read.argtypes = [I32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I64)]
        L.dex_profile_read.restype = S
        L.dex_profile_reset.restype = None
        _lib = L
    return _lib


def check(status: int):
    if status != DEX_OK:
        L = lib()
        raise DexError(status, f"{L.dex_status_string(status).decode()}: {L.dex_last_error().decode()}")


_DT = {torch.float64: DEX_F64, torch.float32: DEX_F32, torch.int32: DEX_I32,
       torch.int64: DEX_I64, torch.uint8: DEX_U8}
try:
    _DT[torch.uint32] = DEX_U32
except AttributeError:  # older torch
    pass


def dtype_code(t: torch.Tensor) -> int:
    return _DT[t.dtype]


def _check_device(t: torch.Tensor, name: str = "buffer"):
    """Device buffers must live on the GPU. Without a visible GPU the library
    itself reports the missing device (after its host-side argument checks)."""
    if t.numel() and not t.is_cuda and torch.cuda.is_available():
        raise ValueError(f"dex {name} must be a GPU tensor (got device {t.device})")


def buf(t: torch.Tensor | None, dtype: int | None = None) -> DexBuf:
    if t is None:
        return DexBuf(None, 0, dtype or DEX_F32, 0)
    if not t.is_contiguous():
        raise ValueError("dex buffers must be contiguous")
    _check_device(t)
    return DexBuf(t.data_ptr() if t.numel() else None, t.numel(),
                  dtype if dtype is not None else dtype_code(t), 0)


def bufs(ts, dtypes=None):
    arr = (DexBuf * max(1, len(ts)))()
    for i, t in enumerate(ts):
        arr[i] = buf(t, None if dtypes is None else dtypes[i])
    return arr, len(ts)


def stream_ptr(stream=None):
    """The HIP stream to enqueue on: the given torch stream, else torch's current
    one. Without a visible GPU this is the null stream, and the library then
    reports the missing device itself."""
    if stream is None and not torch.cuda.is_available():
        return None
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# ---- descriptors --------------------------------------------------------------

def desc(kind, dtype, dims, variant=0, config=0, fparams=()):
    d = DexDesc()
    d.kind, d.dtype, d.variant, d.config = kind, dtype, variant, config
    for i, v in enumerate(dims):
        d.dims[i] = int(v)
    for i, v in enumerate(fparams):
        d.fparams[i] = float(v)
    return d


def gmm_desc(N, D, K, dtype=DEX_F32, variant=DEX_GMM_BF16, config=0):
    return desc(DEX_GMM, dtype, (N, D, K), variant, config)


def gather_desc(V, R, n):
    return desc(DEX_GATHER_SCALE, DEX_F32, (V, R, n))


def stencil_desc(H, W, steps, every, c=0.2, rho=0.0, variant=DEX_STENCIL_RECOMPUTE, config=0):
    return desc(DEX_STENCIL5, DEX_F32, (H, W, steps, every), variant, config, (c, rho))


# ---- entry points ---------------------------------------------------------------

def dex_version() -> str:
    return lib().dex_version().decode()


def dex_init():
    check(lib().dex_init())


def dex_workspace_bytes(d: DexDesc, role: int) -> int:
    n = ctypes.c_size_t(0)
    check(lib().dex_workspace_bytes(ctypes.byref(d), role, ctypes.byref(n)))
    return n.value


def dex_num_configs(d: DexDesc, role: int) -> int:
    n = ctypes.c_int32(0)
    check(lib().dex_num_configs(ctypes.byref(d), role, ctypes.byref(n)))
    return n.value


def workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def dex_fwd(d: DexDesc, ins, outs, resid, ws: torch.Tensor | None = None, stream=None,
            dtypes=None):
    """ins/outs/resid: lists of tensors. dtypes: optional override per list."""
    a, na = bufs(ins, dtypes and dtypes.get("in"))
    o, no = bufs(outs, dtypes and dtypes.get("out"))
    r, nr = bufs(resid, dtypes and dtypes.get("resid"))
    wp = ctypes.c_void_p(ws.data_ptr()) if ws is not None else None
    wb = ws.numel() if ws is not None else 0
    check(lib().dex_fwd(ctypes.byref(d), a, na, o, no, r, nr, wp, wb, stream_ptr(stream)))


def dex_jvp(d: DexDesc, ins, t_in, t_out, ws: torch.Tensor | None = None, stream=None,
            resid=(), dtypes=None):
    """Forward mode: t_out = the linearization of f at ins applied to t_in
    (resid: dex_fwd's residuals, for DEX_GMM)."""
    a, na = bufs(ins, dtypes and dtypes.get("in"))
    r, nr = bufs(list(resid), dtypes and dtypes.get("resid"))
    ti, nti = bufs(t_in)
    to, nto = bufs(t_out)
    wp = ctypes.c_void_p(ws.data_ptr()) if ws is not None else None
    wb = ws.numel() if ws is not None else 0
    check(lib().dex_jvp(ctypes.byref(d), a, na, r, nr, ti, nti, to, nto, wp, wb,
                        stream_ptr(stream)))


DEX_REDUCE_WS_BYTES = 8192


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _f32_buffer(t, name):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float32:
        raise ValueError(f"{name} must be float32 (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    _check_device(t, name)


def dex_reduce_rows(out: torch.Tensor, values: torch.Tensor, flags=0, stream=None):
    """out[i] (=|+=) sum_j values[i, j] for a 2-D float32 `values`; `out` holds
    one float32 per row."""
    _f32_buffer(values, "values")
    _f32_buffer(out, "out")
    if values.dim() != 2:
        raise ValueError(f"values must be 2-D (rows x cols), got shape {tuple(values.shape)}")
    rows, cols = values.shape
    if out.numel() != rows:
        raise ValueError(f"out must hold {rows} values (one per row), got {out.numel()}")
    check(lib().dex_reduce_rows(_ptr(out), _ptr(values), rows, cols, flags, stream_ptr(stream)))


def dex_reduce_all(out: torch.Tensor, values: torch.Tensor, ws: torch.Tensor, flags=0,
                   stream=None):
    """out[0] (=|+=) sum of all of float32 `values`; ws: at least
    DEX_REDUCE_WS_BYTES bytes of uint8 device memory."""
    _f32_buffer(values, "values")
    _f32_buffer(out, "out")
    if out.numel() != 1:
        raise ValueError(f"out must hold one value, got {out.numel()}")
    if not isinstance(ws, torch.Tensor) or ws.dtype != torch.uint8 or not ws.is_contiguous():
        raise ValueError("ws must be a contiguous uint8 tensor")
    if ws.numel() < DEX_REDUCE_WS_BYTES:
        raise ValueError(f"ws must hold at least {DEX_REDUCE_WS_BYTES} bytes, got {ws.numel()}")
    _check_device(ws, "ws")
    check(lib().dex_reduce_all(_ptr(out), _ptr(values), values.numel(), flags, _ptr(ws),
                               ws.numel(), stream_ptr(stream)))


def dex_reduce_all_noalloc(out: torch.Tensor, values: torch.Tensor, flags=0, stream=None):
    """out[0] (=|+=) sum of all of float32 `values`, with no workspace: the
    library's own per-GPU scratch holds the partials (calls that overlap on one
    GPU race)."""
    _f32_buffer(values, "values")
    _f32_buffer(out, "out")
    if out.numel() != 1:
        raise ValueError(f"out must hold one value, got {out.numel()}")
    check(lib().dex_reduce_all_noalloc(_ptr(out), _ptr(values), values.numel(), flags,
                                       stream_ptr(stream)))


def dex_vjp(d: DexDesc, ins, resid, ct_out, ct_in, flags=0, ws: torch.Tensor | None = None,
            stream=None, dtypes=None):
    a, na = bufs(ins, dtypes and dtypes.get("in"))
    r, nr = bufs(resid, dtypes and dtypes.get("resid"))
    co, nco = bufs(ct_out)
    ci, nci = bufs(ct_in, dtypes and dtypes.get("ct_in"))
    wp = ctypes.c_void_p(ws.data_ptr()) if ws is not None else None
    wb = ws.numel() if ws is not None else 0
    check(lib().dex_vjp(ctypes.byref(d), a, na, r, nr, co, nco, ci, nci, flags, wp, wb,
                        stream_ptr(stream)))


def dex_accum_scatter_workspace_bytes(acc_dtype, n_rows, row_len, n, has_vals, flags=0) -> int:
    b = ctypes.c_size_t(0)
    check(lib().dex_accum_scatter_workspace_bytes(acc_dtype, n_rows, row_len, n, int(bool(has_vals)),
                                                  flags, ctypes.byref(b)))
    return b.value


def dex_accum_scatter(acc: torch.Tensor, idx: torch.Tensor, vals: torch.Tensor | None = None,
                      scale: torch.Tensor | None = None, flags: int = 0,
                      oob: torch.Tensor | None = None, ws: torch.Tensor | None = None,
                      stream=None, idx_dtype: int | None = None):
    """acc!(idx[j]) += scale[j] * vals[j]  (acc: [n_rows] or [n_rows, row_len])."""
    n_rows = acc.shape[0]
    row_len = acc.numel() // max(1, n_rows)
    acc_dt = dtype_code(acc)
    idt = idx_dtype if idx_dtype is not None else dtype_code(idx)
    n = idx.numel()
    if ws is None:
        nb = dex_accum_scatter_workspace_bytes(acc_dt, n_rows, row_len, n, vals is not None, flags)
        ws = workspace(nb, acc.device) if nb else None
    for t in (acc, idx, vals, scale, oob, ws):
        if t is not None:
            if not t.is_contiguous():
                raise ValueError("dex buffers must be contiguous")
            _check_device(t)
    check(lib().dex_accum_scatter(
        ctypes.c_void_p(acc.data_ptr()), acc_dt, n_rows, row_len, ctypes.c_void_p(idx.data_ptr()),
        idt, ctypes.c_void_p(vals.data_ptr()) if vals is not None else None,
        ctypes.c_void_p(scale.data_ptr()) if scale is not None else None, n, flags,
        ctypes.c_void_p(oob.data_ptr()) if oob is not None else None,
        ctypes.c_void_p(ws.data_ptr()) if ws is not None else None,
        ws.numel() if ws is not None else 0, stream_ptr(stream)))


def dex_gmm_batched_plan(shapes: np.ndarray, variant: int = DEX_GMM_PLAIN):
    """Returns (descriptor, plan bytes as a uint8 numpy array)."""
    shapes = np.ascontiguousarray(shapes, dtype=np.int64)
    B = shapes.shape[0]
    d = DexDesc()
    nb = ctypes.c_size_t(0)
    check(lib().dex_gmm_batched_plan(shapes.ctypes.data, B, variant, ctypes.byref(d), None,
                                     ctypes.byref(nb)))
    plan = np.zeros(nb.value, dtype=np.uint8)
    check(lib().dex_gmm_batched_plan(shapes.ctypes.data, B, variant, ctypes.byref(d),
                                     plan.ctypes.data, ctypes.byref(nb)))
    return d, plan


def dex_autotune(d: DexDesc, role: int, ins, outs, resid, ct_out, ct_in, ws, stream=None,
                 dtypes=None) -> int:
    a, na = bufs(ins, dtypes and dtypes.get("in"))
    o, no = bufs(outs)
    r, nr = bufs(resid, dtypes and dtypes.get("resid"))
    co, nco = bufs(ct_out)
    ci, nci = bufs(ct_in)
    best = ctypes.c_int32(0)
    check(lib().dex_autotune(ctypes.byref(d), role, a, na, o, no, r, nr, co, nco, ci, nci,
                             ctypes.c_void_p(ws.data_ptr()), ws.numel(), stream_ptr(stream),
                             ctypes.byref(best)))
    return best.value


def dex_autotune_reset():
    lib().dex_autotune_reset()


DEX_PROF = dict(GMM_FWD=0, GMM_VJP=1, SCATTER=2, HIST=3, GATHER=4, GATHER_DW=5, BGMM_FWD=6,
                BGMM_VJP=7, STENCIL_FWD=8, STENCIL_VJP=9, GATHER_JVP=10, REDUCE_ROWS=11,
                REDUCE_ALL=12, GMM_JVP=13)


def dex_profile_enable(on: bool = True):
    lib().dex_profile_enable(1 if on else 0)


def dex_profile_read(which) -> tuple[float, int]:
    """(total milliseconds, kernel launches) recorded for a path's main kernel."""
    i = DEX_PROF[which] if isinstance(which, str) else int(which)
    ms, n = ctypes.c_double(0), ctypes.c_int64(0)
    check(lib().dex_profile_read(i, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def dex_profile_reset():
    lib().dex_profile_reset()
