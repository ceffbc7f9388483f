"""GPU parity of the batched (persistent, one launch per phase) GMM against the
FP64 oracle, instance by instance (FP32: 1e-5 relative L2)."""
import numpy as np
import pytest
import torch

import workloads
from oracle import gmm as ogmm

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def run_batched(shapes, insts, fcfg=0, bcfg=0, ct=None, dev="cuda", variant=0):
    from paper_2104_05372_amd import dex
    d, plan = dex.dex_gmm_batched_plan(shapes, variant)
    packed = [torch.tensor(a, device=dev) for a in workloads.pack_batched(insts)]
    tplan = torch.tensor(plan, device=dev)
    B = shapes.shape[0]
    F = torch.empty(B, device=dev)
    f = torch.empty(int(d.dims[1]), device=dev)
    cache = torch.empty(int(d.dims[7]), dtype=torch.uint8, device=dev)
    ws = dex.workspace(dex.dex_workspace_bytes(d, dex.DEX_WS_FWD), dev)
    d.config = fcfg
    print(f"  batched B={B} variant={variant} fwd cfg={fcfg}", flush=True)
    dex.dex_fwd(d, [tplan, *packed], [F], [f, cache], ws)
    d.config = bcfg
    ctt = torch.tensor(np.ones(B, np.float32) if ct is None else ct, device=dev)
    grads = [torch.empty_like(p) for p in packed[:4]]
    print(f"  batched vjp cfg={bcfg}", flush=True)
    dex.dex_vjp(d, [tplan, *packed], [f, cache], [ctt], grads, 0, ws)
    torch.cuda.synchronize()
    return F.cpu().numpy(), f.cpu().numpy(), [x.cpu().numpy() for x in grads]


def split(shapes, arr, per):
    out, o = [], 0
    for row in shapes:
        m = per(*row)
        out.append(arr[o:o + m])
        o += m
    return out


def check_instances(shapes, insts, got, which, ct=None, tol=1e-5):
    F, f, grads = got
    fs = split(shapes, f, lambda N, D, K: N)
    ga = split(shapes, grads[0], lambda N, D, K: K)
    gm = split(shapes, grads[1], lambda N, D, K: K * D)
    gq = split(shapes, grads[2], lambda N, D, K: K * D)
    gl = split(shapes, grads[3], lambda N, D, K: K * D * (D - 1) // 2)
    for b in which:
        g = insts[b]
        Fo, fo = ogmm.objective(*g.params(), g.x)
        c = 1.0 if ct is None else float(ct[b])
        go = ogmm.vjp(*g.params(), g.x, fo, c)
        assert abs(F[b] - Fo) <= tol * abs(Fo), b
        assert rel(fs[b], fo) <= tol, b
        for a, o in zip((ga[b], gm[b], gq[b], gl[b]), go):
            assert rel(a, o.ravel()) <= tol, b


def small_batch():
    shapes = np.array([[1000, 8, 10], [1537, 16, 3], [2049, 32, 7], [256, 8, 1],
                       [3001, 32, 12], [999, 16, 25], [4100, 8, 2], [600, 8, 77]], np.int64)
    return shapes, workloads.batched_inputs(shapes, seed=30)


@pytest.mark.parametrize("fcfg,bcfg", [(0, 0), (1, 1), (2, 2), (1, 3), (2, 4)])
def test_small_batch_all_configs(dev, fcfg, bcfg):
    shapes, insts = small_batch()
    got = run_batched(shapes, insts, fcfg, bcfg)
    check_instances(shapes, insts, got, range(len(insts)))


@pytest.mark.parametrize("fcfg,bcfg", [(0, 0), (2, 4)])
def test_any_dimension(dev, fcfg, bcfg):
    """Dimensions other than 8, 16 and 32: D <= 8 on the vector units (D = 1
    has no off-diagonal factor entries), 9..16 and 17..32 on padded tiles."""
    shapes = np.array([[700, 1, 9], [513, 3, 20], [900, 5, 70], [1100, 7, 33], [300, 2, 1],
                       [600, 12, 15], [800, 20, 11], [1000, 31, 6], [450, 9, 40]], np.int64)
    insts = workloads.batched_inputs(shapes, seed=41)
    got = run_batched(shapes, insts, fcfg, bcfg)
    check_instances(shapes, insts, got, range(len(insts)))


SPLIT_SHAPES = np.array([[1000, 8, 10], [1537, 16, 3], [2049, 32, 7], [600, 12, 15], [800, 20, 11],
                         [1000, 31, 6], [450, 9, 40], [3001, 32, 12], [999, 16, 25], [300, 2, 1]],
                        np.int64)


@pytest.mark.parametrize("fcfg,bcfg", [(0, 0), (1, 1), (2, 4)])
def test_split_fp16_variant(dev, fcfg, bcfg):
    """DEX_GMM_F16X3: split-FP16 operands for D > 8 (D <= 8 as in PLAIN), held
    to the FP32 bound."""
    from paper_2104_05372_amd import dex
    insts = workloads.batched_inputs(SPLIT_SHAPES, seed=52)
    got = run_batched(SPLIT_SHAPES, insts, fcfg, bcfg, variant=dex.DEX_GMM_F16X3)
    check_instances(SPLIT_SHAPES, insts, got, range(len(insts)))


def test_split_fp16_cotangents(dev):
    """Per-instance cotangents, negative ones included (the split form applies
    them in the assembly, not in the weights)."""
    from paper_2104_05372_amd import dex
    insts = workloads.batched_inputs(SPLIT_SHAPES, seed=53)
    ct = np.linspace(-3, 2, len(insts)).astype(np.float32)
    got = run_batched(SPLIT_SHAPES, insts, ct=ct, variant=dex.DEX_GMM_F16X3)
    check_instances(SPLIT_SHAPES, insts, got, range(len(insts)), ct)


@pytest.mark.parametrize("variant", [0, 3])
@pytest.mark.parametrize("offset,scale", [(100.0, 1.0), (1000.0, 1.0), (0.0, 2.0 ** 20),
                                          (0.0, 1e-5), (50.0, 3.0e3)])
def test_shifted_and_rescaled_data(dev, offset, scale, variant):
    """x and the means moved by `offset` and scaled by `scale` (Q by 1/scale):
    the same Mahalanobis terms, with raw values far from the origin (where x
    itself would lose the FP32 digits of x - mu to cancellation) or far outside
    what FP16 holds unscaled. Every instance's operands are taken about the
    mean of its first means; the split form also scales them by powers of two."""
    shapes = SPLIT_SHAPES
    base = workloads.batched_inputs(shapes, seed=54)
    insts = [workloads.GMMInputs(g.alphas, (g.means + offset) * scale, g.qd - np.log(scale),
                                 g.l / scale, (g.x + offset) * scale).astype(np.float32)
             for g in base]
    got = run_batched(shapes, insts, variant=variant)
    check_instances(shapes, insts, got, range(len(insts)))


def test_split_fp16_points_at_the_origin_shift(dev):
    """A tile whose points sit (almost) on the origin shift while the means are
    spread: a tile scale taken from the points alone would blow the scaled
    offsets -c~ out of range. The scale is bounded by the means' spread."""
    from paper_2104_05372_amd import dex
    shapes = np.array([[600, 16, 12], [700, 24, 9]], np.int64)
    insts = []
    for g, (N, D, K) in zip(workloads.batched_inputs(shapes, seed=61), shapes):
        c = np.mean(g.means[:min(K, 16)].astype(np.float32), axis=0, dtype=np.float32)
        x = g.x.copy()
        x[:128] = c + np.float32(1e-12) * g.x[:128]
        insts.append(workloads.GMMInputs(g.alphas, g.means, g.qd, g.l, x).astype(np.float32))
    got = run_batched(shapes, insts, variant=dex.DEX_GMM_F16X3)
    check_instances(shapes, insts, got, range(len(insts)))


@pytest.mark.parametrize("variant", [0, 3])
def test_accumulate_into_gradients(dev, variant):
    """DEX_ACCUMULATE adds the batch's gradients to what the buffers hold: a
    second reverse call into the first call's output gives twice the gradient."""
    from paper_2104_05372_amd import dex
    shapes, insts = small_batch()
    d, plan = dex.dex_gmm_batched_plan(shapes, variant)
    packed = [torch.tensor(a, device=dev) for a in workloads.pack_batched(insts)]
    ins = [torch.tensor(plan, device=dev), *packed]
    B = shapes.shape[0]
    F = torch.empty(B, device=dev)
    f = torch.empty(int(d.dims[1]), device=dev)
    cache = torch.empty(int(d.dims[7]), dtype=torch.uint8, device=dev)
    ws = dex.workspace(dex.dex_workspace_bytes(d, dex.DEX_WS_FWD), dev)
    ct = torch.ones(B, device=dev)
    dex.dex_fwd(d, ins, [F], [f, cache], ws)
    once = [torch.empty_like(p) for p in packed[:4]]
    dex.dex_vjp(d, ins, [f, cache], [ct], once, 0, ws)
    twice = [g.clone() for g in once]
    dex.dex_vjp(d, ins, [f, cache], [ct], twice, dex.DEX_ACCUMULATE, ws)
    torch.cuda.synchronize()
    for a, b in zip(once, twice):
        assert torch.allclose(2 * a, b, rtol=1e-6, atol=0), variant


def test_per_instance_cotangents(dev):
    shapes, insts = small_batch()
    ct = np.linspace(-2, 2, len(insts)).astype(np.float32)
    got = run_batched(shapes, insts, ct=ct)
    check_instances(shapes, insts, got, range(len(insts)), ct)


def _oracle_instance(args):
    """Objective, f and gradient of one instance (regenerated from its seed)."""
    b, (N, D, K), seed_base = args
    g = workloads.gmm_inputs(int(N), int(D), int(K), seed_base + 1 + b, np.float32)
    Fo, fo = ogmm.objective(*g.params(), g.x)
    return b, Fo, fo, ogmm.vjp(*g.params(), g.x, fo)


@pytest.mark.timeout(600)
def test_full_batch_every_instance(dev):
    """512 instances, N ~ U[1000, 50000], D in {8,16,32}, K ~ U[10,100], in the
    benchmark's single launch per phase; every instance's F, f and gradient
    against the oracle (the oracle runs on a pool of host threads)."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    from threadpoolctl import threadpool_limits
    shapes = workloads.batched_shapes()
    insts = workloads.batched_inputs(shapes)
    F, f, grads = run_batched(shapes, insts)
    del insts
    fs = split(shapes, f, lambda N, D, K: N)
    ga = split(shapes, grads[0], lambda N, D, K: K)
    gm = split(shapes, grads[1], lambda N, D, K: K * D)
    gq = split(shapes, grads[2], lambda N, D, K: K * D)
    gl = split(shapes, grads[3], lambda N, D, K: K * D * (D - 1) // 2)
    base = workloads.BATCHED["seed"]
    cost = shapes[:, 0] * shapes[:, 2] * shapes[:, 1] ** 2
    order = [int(b) for b in np.argsort(-cost)]  # largest first
    workers = max(1, min(16, os.cpu_count() or 1))
    print(f"  oracle for {len(order)} instances on {workers} threads", flush=True)
    bad = []
    with threadpool_limits(1), ThreadPoolExecutor(workers) as ex:
        for done, (b, Fo, fo, go) in enumerate(
                ex.map(_oracle_instance, [(b, shapes[b], base) for b in order])):
            errs = [abs(F[b] - Fo) / abs(Fo), rel(fs[b], fo)] + \
                [rel(a, o.ravel()) for a, o in zip((ga[b], gm[b], gq[b], gl[b]), go)]
            if max(errs) > 1e-5:
                bad.append((b, errs))
            if done % 128 == 127:
                print(f"  {done + 1} instances checked", flush=True)
    assert not bad, bad[:5]
