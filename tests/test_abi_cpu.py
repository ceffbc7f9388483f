"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/dex.h declares, rejects bad arguments before touching a
device, sizes its workspaces, and builds batched plans."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dex.h")


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dex_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def dex():
    from paper_2104_05372_amd import dex as d
    d.lib()
    return d


def test_library_exports_every_declared_function(dex):
    names = header_functions()
    assert len(names) >= 12
    L = ctypes.CDLL(dex.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(dex.EXPORTS)


def test_status_strings(dex):
    L = dex.lib()
    for s in (0, -1, -2, -3, -4, -5):
        assert L.dex_status_string(s).decode() not in ("", "unknown status")
    assert "gfx950" in dex.dex_version()


def _status(fn, *a):
    try:
        fn(*a)
    except dex_error() as e:
        return e.status
    return 0


def dex_error():
    from paper_2104_05372_amd.dex import DexError
    return DexError


def test_invalid_descriptors_rejected_on_host(dex):
    bad = [dex.gmm_desc(0, 2, 3), dex.gmm_desc(10, 65, 3), dex.gmm_desc(10, 2, 3, dex.DEX_F64, dex.DEX_GMM_BF16),
           dex.desc(99, dex.DEX_F32, (1, 1, 1)), dex.stencil_desc(8, 8, 10, 0),
           dex.stencil_desc(8, 8, 10, 2, rho=0.1, variant=dex.DEX_STENCIL_LINEAR),
           dex.gather_desc(0, 4, 4)]
    for d in bad:
        s = _status(dex.dex_workspace_bytes, d, dex.DEX_WS_FWD)
        assert s in (dex.DEX_ERR_INVALID_ARG, dex.DEX_ERR_UNSUPPORTED), s
        s = _status(dex.dex_fwd, d, [], [], [], None)
        assert s in (dex.DEX_ERR_INVALID_ARG, dex.DEX_ERR_UNSUPPORTED), s
        s = _status(dex.dex_jvp, d, [], [], [], None)
        assert s in (dex.DEX_ERR_INVALID_ARG, dex.DEX_ERR_UNSUPPORTED), s


def test_forward_mode_argument_checks(dex):
    """dex_jvp: missing or mis-sized buffers are rejected on the host, before any
    device work; residuals are refused where the kind has none."""
    # the GMM form needs the forward's residuals and four tangents
    assert _status(dex.dex_jvp, dex.gmm_desc(100, 4, 3), [], [], [], None) == dex.DEX_ERR_INVALID_ARG
    d = dex.gather_desc(10, 4, 5)
    assert _status(dex.dex_jvp, d, [], [], [], None) == dex.DEX_ERR_INVALID_ARG
    import torch
    T, idx, w = torch.zeros(10, 4), torch.zeros(5, dtype=torch.int32), torch.zeros(5)
    tT, tw, out = torch.zeros(10, 4), torch.zeros(5), torch.zeros(5, 4)
    assert _status(dex.dex_jvp, d, [T, idx, w], [tT], [out], None) == dex.DEX_ERR_INVALID_ARG
    assert _status(dex.dex_jvp, d, [T, idx, w], [tT, tw], [torch.zeros(5, 3)], None) \
        == dex.DEX_ERR_INVALID_ARG
    assert dex.dex_workspace_bytes(d, dex.DEX_WS_JVP) == 0
    assert _status(lambda: dex.dex_jvp(d, [T, idx, w], [tT, tw], [out], None, resid=[out])) \
        == dex.DEX_ERR_INVALID_ARG
    # the matrix-core tangent pass holds its own FP16 copy of x (N_pad x 64) and
    # the tangent coefficient operand; the vector-ALU pass only its partial sums
    gd = dex.gmm_desc(100_000, 64, 200, dex.DEX_F32, dex.DEX_GMM_BF16)
    assert dex.dex_workspace_bytes(gd, dex.DEX_WS_JVP) >= 100_096 * 64 * 2 + 224 * 2176 * 2
    gv = dex.gmm_desc(1000, 5, 20, dex.DEX_F32, dex.DEX_GMM_PLAIN)
    assert 0 < dex.dex_workspace_bytes(gv, dex.DEX_WS_JVP) < 1 << 16


def test_accum_scatter_argument_checks(dex):
    L = dex.lib()
    # bad dtypes / sizes return before any device work
    assert L.dex_accum_scatter(None, 7, 10, 1, None, dex.DEX_I32, None, None, 0, 0, None, None, 0, None) \
        == dex.DEX_ERR_INVALID_ARG
    assert L.dex_accum_scatter(None, dex.DEX_F32, 0, 1, None, dex.DEX_I32, None, None, 0, 0, None, None, 0,
                               None) == dex.DEX_ERR_INVALID_ARG
    assert L.dex_accum_scatter(None, dex.DEX_F32, 10, 1, None, dex.DEX_I32, None, None, 5, 0, None, None, 0,
                               None) == dex.DEX_ERR_INVALID_ARG
    # bounds checking needs a counter
    assert L.dex_accum_scatter(ctypes.c_void_p(16), dex.DEX_I32, 10, 1, ctypes.c_void_p(16), dex.DEX_I32, None,
                               None, 5, dex.DEX_CHECK_BOUNDS, None, None, 0, None) == dex.DEX_ERR_INVALID_ARG


def test_workspace_sizes(dex):
    d = dex.gmm_desc(100_000, 64, 200, dex.DEX_F32, dex.DEX_GMM_BF16)
    cache = dex.dex_workspace_bytes(d, dex.DEX_WS_RESID)
    # bf16 x (both layouts) + bf16 Q + beta, at least
    assert cache >= 100_096 * 64 * 2 * 2 + 200 * 64 * 64 * 2 + 200 * 100_096 * 4
    assert dex.dex_workspace_bytes(d, dex.DEX_WS_VJP) > 0
    d64 = dex.gmm_desc(1000, 2, 5, dex.DEX_F64, dex.DEX_GMM_PLAIN)
    assert dex.dex_workspace_bytes(d64, dex.DEX_WS_RESID) >= 1000 * 5 * 8
    st = dex.stencil_desc(64, 64, 100, 32)
    assert dex.dex_workspace_bytes(st, dex.DEX_WS_VJP) >= (2 + 31) * 64 * 64 * 4
    lin = dex.stencil_desc(64, 64, 100, 32, variant=dex.DEX_STENCIL_LINEAR)
    assert dex.dex_workspace_bytes(lin, dex.DEX_WS_VJP) < dex.dex_workspace_bytes(st, dex.DEX_WS_VJP)
    hist = dex.dex_accum_scatter_workspace_bytes(dex.DEX_I32, 65536, 1, 1 << 26, False)
    assert hist >= 32768 * 4
    assert dex.dex_num_configs(d, dex.DEX_WS_FWD) >= 2
    assert dex.dex_num_configs(d, dex.DEX_WS_VJP) >= 2


def test_batched_plan(dex):
    shapes = workloads.batched_shapes(64, seed=3)
    d, plan = dex.dex_gmm_batched_plan(shapes)
    B = shapes.shape[0]
    N, D, K = shapes[:, 0], shapes[:, 1], shapes[:, 2]
    assert d.kind == dex.DEX_GMM_BATCHED and d.dims[0] == B
    assert d.dims[1] == N.sum() and d.dims[2] == K.sum()
    assert d.dims[3] == (K * D).sum() and d.dims[4] == (K * D * (D - 1) // 2).sum()
    assert d.dims[5] == (N * D).sum() and d.dims[6] == plan.size
    # header: int64 fields; instance table follows at inst_off
    hdr = plan[:8 * 40].view(np.int64)
    assert hdr[0] == B
    inst_off = hdr[1]
    rec = np.dtype([("N", "<i4"), ("D", "<i4"), ("K", "<i4"), ("DP", "<i4"), ("Npad", "<i8"),
                    ("offs", "<i8", (14,)), ("nblk", "<i4"), ("split", "<i4"),
                    ("offs2", "<i8", (4,))])
    inst = plan[inst_off: inst_off + B * rec.itemsize].view(rec)
    assert np.array_equal(inst["N"], N) and np.array_equal(inst["D"], D) and np.array_equal(inst["K"], K)
    assert np.all(inst["Npad"] % 256 == 0) and np.all(inst["Npad"] >= N)
    # packed input offsets are prefix sums in instance order
    assert np.array_equal(inst["offs"][:, 0], np.concatenate([[0], np.cumsum(K)[:-1]]))
    assert np.array_equal(inst["offs"][:, 3], np.concatenate([[0], np.cumsum(N * D)[:-1]]))
    assert np.all(inst["split"] == 0)
    ws = dex.dex_workspace_bytes(d, dex.DEX_WS_FWD)
    assert ws > 0 and dex.dex_workspace_bytes(d, dex.DEX_WS_RESID) == d.dims[7]
    # the split-FP16 variant: D > 8 instances flagged, their operands in 2-byte
    # hi and lo parts (plus the shift and scales)
    d2, plan2 = dex.dex_gmm_batched_plan(shapes, dex.DEX_GMM_F16X3)
    assert d2.variant == dex.DEX_GMM_F16X3 and list(d2.dims[:6]) == list(d.dims[:6])
    inst2 = plan2[inst_off: inst_off + B * rec.itemsize].view(rec)
    assert np.array_equal(inst2["split"], (D > 8).astype(np.int32))
    lows = inst2["offs2"][:, [0, 2]]  # xl, Ql; the shift block (offs2[3]) is everyone's
    assert np.all(lows[D > 8] > 0) and np.all(lows[D <= 8] == 0) and np.all(inst2["offs2"][:, 3] > 0)


def test_batched_plan_rejects_bad_shapes(dex):
    for bad in ([[100, 33, 5]], [[100, 0, 5]], [[0, 8, 5]], [[100, 8, 0]]):
        with pytest.raises(dex_error()):
            dex.dex_gmm_batched_plan(np.array(bad))
    for variant in (dex.DEX_GMM_BF16, dex.DEX_GMM_BF16X3, 7):
        with pytest.raises(dex_error()):
            dex.dex_gmm_batched_plan(np.array([[100, 16, 5]]), variant)


def test_package_has_no_oracle_dependency():
    """The product package never imports the oracle."""
    pkg = os.path.join(ROOT, "paper_2104_05372_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".cpp", ".h")):
                src = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in src and "from oracle" not in src, fn


def test_reduction_argument_checks(dex):
    """Bad sizes, null buffers, unknown flags and a short workspace are rejected on
    the host; an empty segmented reduction is a no-op that needs no device."""
    L = dex.lib()
    assert L.dex_reduce_rows(None, None, -1, 4, 0, None) == dex.DEX_ERR_INVALID_ARG
    assert L.dex_reduce_rows(None, None, 3, 4, 0, None) == dex.DEX_ERR_INVALID_ARG
    assert L.dex_reduce_rows(ctypes.c_void_p(16), ctypes.c_void_p(16), 3, 4, 64, None) \
        == dex.DEX_ERR_INVALID_ARG
    assert L.dex_reduce_rows(None, None, 0, 4, 0, None) == dex.DEX_OK
    assert L.dex_reduce_all(None, None, 5, 0, None, 0, None) == dex.DEX_ERR_INVALID_ARG
    assert L.dex_reduce_all(ctypes.c_void_p(16), ctypes.c_void_p(16), 5, 0, ctypes.c_void_p(16), 16,
                            None) == dex.DEX_ERR_WORKSPACE


def test_reduction_binding_rejects_bad_tensors(dex):
    """The Python reductions check dtype, contiguity, rank, output size and the
    workspace before any pointer reaches the library (a wrong dtype, a
    transposed view or a short output would otherwise be read or written past
    its end on the device)."""
    import torch
    v = torch.zeros(6, 4)
    out = torch.zeros(6)
    ws = torch.zeros(dex.DEX_REDUCE_WS_BYTES, dtype=torch.uint8)
    bad_rows = [
        (out, v.double()),                 # float64 values
        (out, v.to(torch.bfloat16)),       # bf16 values
        (out, torch.zeros(4, 6).t()),      # transposed view (not contiguous)
        (out, torch.zeros(24)),            # not 2-D
        (torch.zeros(5), v),               # short output
        (out.double(), v),                 # float64 output
    ]
    for o, x in bad_rows:
        with pytest.raises(ValueError):
            dex.dex_reduce_rows(o, x)
    one = torch.zeros(1)
    bad_all = [
        (one, v.double(), ws),
        (one, torch.zeros(4, 6).t(), ws),
        (torch.zeros(2), v, ws),
        (one, v, ws[:100]),                                   # short workspace
        (one, v, torch.zeros(dex.DEX_REDUCE_WS_BYTES // 4)),  # float workspace
    ]
    for o, x, w in bad_all:
        with pytest.raises(ValueError):
            dex.dex_reduce_all(o, x, w)


def test_undersized_workspace_rejected_on_host(dex):
    """Every entry point that takes a workspace refuses a missing or one-byte
    short one with DEX_ERR_WORKSPACE, on the host, before any device work."""
    import torch
    u8 = torch.uint8

    def short(n):
        return torch.zeros(max(n - 1, 0), dtype=u8)

    N, D, K = 300, 8, 4
    L = D * (D - 1) // 2
    for variant in (dex.DEX_GMM_PLAIN, dex.DEX_GMM_BF16):
        d = dex.gmm_desc(N, D, K, dex.DEX_F32, variant)
        ins = [torch.zeros(K), torch.zeros(K, D), torch.zeros(K, D), torch.zeros(K, L), torch.zeros(N, D)]
        resid = [torch.zeros(N), torch.zeros(dex.dex_workspace_bytes(d, dex.DEX_WS_RESID), dtype=u8)]
        grads = [torch.zeros_like(t) for t in ins[:4]]
        calls = {
            dex.DEX_WS_FWD: lambda ws: dex.dex_fwd(d, ins, [torch.zeros(1)], resid, ws),
            dex.DEX_WS_VJP: lambda ws: dex.dex_vjp(d, ins, resid, [torch.ones(1)], grads, 0, ws),
            dex.DEX_WS_JVP: lambda ws: dex.dex_jvp(d, ins, grads, [torch.zeros(1)], ws, resid=resid),
        }
        for role, call in calls.items():
            need = dex.dex_workspace_bytes(d, role)
            assert need > 0, (variant, role)
            for ws in (None, short(need)):
                assert _status(call, ws) == dex.DEX_ERR_WORKSPACE, (variant, role, need)
    # the checkpointed loop's reverse pass and forward mode
    st = dex.stencil_desc(32, 32, 10, 4, rho=0.1)
    u = [torch.zeros(32, 32), torch.zeros(32, 32)]
    ck = [torch.zeros(3 * 32 * 32), torch.zeros(32, 32)]
    for role, call in ((dex.DEX_WS_VJP, lambda ws: dex.dex_vjp(st, u, ck, [torch.ones(1)],
                                                                [torch.zeros(32, 32)], 0, ws)),
                       (dex.DEX_WS_JVP, lambda ws: dex.dex_jvp(st, u, u, [torch.zeros(1)], ws))):
        need = dex.dex_workspace_bytes(st, role)
        assert need > 0
        for ws in (None, short(need)):
            assert _status(call, ws) == dex.DEX_ERR_WORKSPACE, role
    # the deterministic (sorted) transposed gather
    gd = dex.gather_desc(100, 8, 1000)
    gd.config = 2
    T, idx, w = torch.zeros(100, 8), torch.zeros(1000, dtype=torch.int32), torch.zeros(1000)
    need = dex.dex_workspace_bytes(gd, dex.DEX_WS_VJP)
    assert need > 0
    for ws in (None, short(need)):
        assert _status(dex.dex_vjp, gd, [T, idx, w], [], [torch.zeros(1000, 8)],
                       [torch.zeros(100, 8), torch.zeros(1000)], 0, ws) == dex.DEX_ERR_WORKSPACE
    # dex_accum_scatter: the histogram's private counters and the sorted float form
    h = torch.zeros(65536, dtype=torch.int32)
    keys = torch.zeros(1 << 12, dtype=torch.int32)
    need = dex.dex_accum_scatter_workspace_bytes(dex.DEX_I32, 65536, 1, 1 << 12, False)
    assert _status(lambda: dex.dex_accum_scatter(h, keys, ws=short(need))) == dex.DEX_ERR_WORKSPACE
    acc, vals = torch.zeros(100, 8), torch.zeros(1000, 8)
    need = dex.dex_accum_scatter_workspace_bytes(dex.DEX_F32, 100, 8, 1000, True, dex.DEX_DETERMINISTIC)
    assert need > 0
    assert _status(lambda: dex.dex_accum_scatter(acc, idx, vals, flags=dex.DEX_DETERMINISTIC,
                                                 ws=short(need))) == dex.DEX_ERR_WORKSPACE
    # the complete reduction (its allocation-free form takes none)
    L_ = dex.lib()
    assert L_.dex_reduce_all(ctypes.c_void_p(16), ctypes.c_void_p(16), 5, 0, None, 0, None) \
        == dex.DEX_ERR_WORKSPACE
