"""GPU parity of the regular segmented and the complete reduction against the
oracle (FP64 exact sums): within 1e-6 relative (the results are FP32), and
bit-identical from run to run."""
import numpy as np
import pytest
import torch

from oracle import reduce as ored

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("rows,cols,seed", [(1000, 128, 0), (7, 3, 1), (513, 1000, 2), (64, 1, 3),
                                            (10, 0, 4), (0, 16, 5), (3, 100_003, 6), (20_000, 52, 7)])
def test_segmented(dev, rows, cols, seed):
    from paper_2104_05372_amd import dex
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((rows, cols)).astype(np.float32)
    print(f"  reduce_rows {rows}x{cols}", flush=True)
    tv = torch.tensor(v, device=dev)
    out = torch.full((rows,), 7.0, device=dev)
    dex.dex_reduce_rows(out, tv)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    want = ored.reduce_rows(v)
    assert np.all(np.abs(got - want) <= 1e-6 * np.maximum(np.abs(v).sum(axis=1), 1e-30))
    again = torch.empty_like(out)
    dex.dex_reduce_rows(again, tv)
    assert torch.equal(again, out)
    dex.dex_reduce_rows(out, tv, dex.DEX_ACCUMULATE)  # out += sums
    torch.cuda.synchronize()
    assert np.allclose(out.cpu().numpy(), 2 * want, rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("n,seed", [(1, 0), (1000, 1), (1 << 20, 2), (12_345_677, 3), (0, 4)])
def test_complete(dev, n, seed):
    from paper_2104_05372_amd import dex
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(n).astype(np.float32)
    print(f"  reduce_all n={n}", flush=True)
    tv = torch.tensor(v, device=dev)
    ws = torch.empty(dex.DEX_REDUCE_WS_BYTES, dtype=torch.uint8, device=dev)
    out = torch.full((1,), 3.0, device=dev)
    dex.dex_reduce_all(out, tv, ws)
    torch.cuda.synchronize()
    want = ored.reduce_all(v)
    assert abs(out.item() - want) <= 1e-6 * max(float(np.abs(v).sum()), 1e-30)
    again = torch.empty_like(out)
    dex.dex_reduce_all(again, tv, ws)
    assert torch.equal(again, out)
    dex.dex_reduce_all(out, tv, ws, dex.DEX_ACCUMULATE)
    torch.cuda.synchronize()
    assert abs(out.item() - 2 * want) <= 2e-6 * max(float(np.abs(v).sum()), 1e-30)
