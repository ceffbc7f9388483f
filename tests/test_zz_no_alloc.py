"""The allocation-free complete reduction (dex_reduce_all_noalloc) against the
workspace form (dex_reduce_all) through the C ABI: the same kernels and
summation order, so the results must agree bit for bit, on consecutive calls
that share the library's scratch array (the second on a smaller input), with
and without accumulation."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _pair(dex, v, flags=0, init=0.0):
    dev = v.device
    a = torch.full((1,), init, device=dev)
    b = torch.full((1,), init, device=dev)
    ws = torch.empty(dex.DEX_REDUCE_WS_BYTES, dtype=torch.uint8, device=dev)
    dex.dex_reduce_all(a, v, ws, flags)
    dex.dex_reduce_all_noalloc(b, v, flags)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy()


def test_noalloc_matches_workspace_form_on_consecutive_calls(dev):
    from paper_2104_05372_amd import dex
    gen = torch.Generator(device=dev).manual_seed(11)
    big = torch.randn(5_000_003, device=dev, generator=gen)
    small = torch.randn(777, device=dev, generator=gen)
    for name, v in (("first call, 5000003 values", big), ("second call, 777 values", small)):
        print(f"  noalloc {name}", flush=True)
        a, b = _pair(dex, v)
        assert a.tobytes() == b.tobytes(), (name, a, b)
        exact = float(np.sum(v.cpu().numpy().astype(np.float64)))
        assert abs(float(b[0]) - exact) <= 1e-6 * max(1.0, float(np.sum(np.abs(v.cpu().numpy()))))
    # accumulate, and an empty input (the partials of the previous call must not leak)
    a, b = _pair(dex, small, dex.DEX_ACCUMULATE, init=2.5)
    assert a.tobytes() == b.tobytes()
    a, b = _pair(dex, torch.empty(0, device=dev))
    assert float(a[0]) == 0.0 and float(b[0]) == 0.0


def test_noalloc_ordered_on_one_stream(dev):
    """Several calls queued on one stream, each reading the scratch its own
    first kernel wrote: every result matches the workspace form."""
    from paper_2104_05372_amd import dex
    gen = torch.Generator(device=dev).manual_seed(12)
    vs = [torch.randn(n, device=dev, generator=gen) for n in (1 << 20, 4099, 1 << 16, 3)]
    outs = [torch.empty(1, device=dev) for _ in vs]
    for o, v in zip(outs, vs):
        dex.dex_reduce_all_noalloc(o, v)
    torch.cuda.synchronize()
    ws = torch.empty(dex.DEX_REDUCE_WS_BYTES, dtype=torch.uint8, device=dev)
    for o, v in zip(outs, vs):
        r = torch.empty(1, device=dev)
        dex.dex_reduce_all(r, v, ws)
        torch.cuda.synchronize()
        assert r.cpu().numpy().tobytes() == o.cpu().numpy().tobytes()
