"""GPU parity of the GMM objective and its reverse pass against the FP64 oracle.

Tolerances (relative L2 per output block, FP64 on the host):
  FP64 form            1e-10
  FP32 form            1e-5
  16-bit products      TOL_MIXED16 (derived below)
  split-BF16 products  TOL_BF16X3
The 16-bit variant (DEX_GMM_BF16) rounds its matrix-core operands to 16 bits:
at D = 64 the forward is one FP16 product over second-order features (unit
roundoff 2^-11, per-tile power-of-two scaling), at other D the forward takes
BF16 operands (2^-9); the reverse moments take FP16 operands at every D.
beta_ik = kappa_k - ||y_ik||^2 / 2 sums about D^2 rounded terms of total size
of order ||y||^2 ~ 2D, so beta carries absolute errors of order 2D u and the
weights w = exp(beta - f) relative errors of that order (6e-2 at D = 64,
u = 2^-11), which cancel in part across the N points of each sum; measured
gradient errors are 4-8e-3, and the bound is 1e-2. All operands are taken
about a point among the means (the results do not depend on the origin), so
the same bound holds for data far from the origin. Split-BF16 drops only the
lo*lo terms (about 2^-16 relative); bound 2e-4.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import gmm as ogmm

pytestmark = pytest.mark.gpu

TOL_MIXED16 = 1e-2
TOL_BF16X3 = 2e-4


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def run_gmm(g, dtype, variant, fcfg=0, bcfg=0, ct=1.0, accumulate_into=None, dev="cuda"):
    from paper_2104_05372_amd import dex
    tdt = torch.float64 if dtype == dex.DEX_F64 else torch.float32
    t = [torch.tensor(np.ascontiguousarray(a), dtype=tdt, device=dev).contiguous()
         for a in (g.alphas, g.means, g.qd, g.l, g.x)]
    N, D, K = g.N, g.D, g.K
    d = dex.gmm_desc(N, D, K, dtype, variant, fcfg)
    F = torch.empty(1, dtype=tdt, device=dev)
    f = torch.empty(N, dtype=tdt, device=dev)
    cache = torch.empty(dex.dex_workspace_bytes(d, dex.DEX_WS_RESID), dtype=torch.uint8, device=dev)
    ws = dex.workspace(dex.dex_workspace_bytes(d, dex.DEX_WS_FWD), dev)
    print(f"  gmm fwd N={N} D={D} K={K} dtype={dtype} variant={variant} cfg={fcfg}", flush=True)
    dex.dex_fwd(d, t, [F], [f, cache], ws)
    d.config = bcfg
    grads = ([torch.zeros_like(x) for x in t[:4]] if accumulate_into is None
             else [torch.tensor(a, dtype=tdt, device=dev) for a in accumulate_into])
    ctt = torch.tensor([ct], dtype=tdt, device=dev)
    wsv = dex.workspace(dex.dex_workspace_bytes(d, dex.DEX_WS_VJP), dev)
    print(f"  gmm vjp cfg={bcfg}", flush=True)
    dex.dex_vjp(d, t, [f, cache], [ctt], grads,
                dex.DEX_ACCUMULATE if accumulate_into is not None else 0, wsv)
    torch.cuda.synchronize()
    return float(F.item()), f.cpu().numpy(), [x.cpu().numpy() for x in grads]


def oracle_gmm(g, ct=1.0):
    F, f = ogmm.objective(*g.params(), g.x)
    return F, f, ogmm.vjp(*g.params(), g.x, f, ct)


def check(got, want, tol, what=""):
    F, f, grads = got
    Fo, fo, go = want
    assert abs(F - Fo) <= tol * max(1.0, abs(Fo)), (what, F, Fo)
    assert rel(f, fo) <= tol, (what, rel(f, fo))
    for name, a, b in zip(("d_alphas", "d_means", "d_qd", "d_l"), grads, go):
        if b.size:
            assert rel(a, b) <= tol, (what, name, rel(a, b))


def test_small_fp64_matches_oracle_and_golden(dev):
    import json
    import os
    from paper_2104_05372_amd import dex
    g = workloads.gmm_small()
    got = run_gmm(g, dex.DEX_F64, dex.DEX_GMM_PLAIN)
    check(got, oracle_gmm(g), 1e-10, "S0 fp64")
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "gmm_small_f64.json")))
    assert abs(got[0] - gold["F"]) <= 1e-10 * abs(gold["F"])
    assert rel(got[2][0], gold["d_alphas"]) <= 1e-10
    assert rel(got[2][3], gold["d_l"]) <= 1e-10


@pytest.mark.parametrize("N,D,K", [(257, 1, 3), (1000, 3, 4), (700, 7, 1), (1500, 16, 5),
                                   (999, 17, 6), (2048, 32, 3), (640, 33, 4), (1100, 64, 5)])
def test_fp64_shapes(dev, N, D, K):
    from paper_2104_05372_amd import dex
    g = workloads.gmm_inputs(N, D, K, 100 + D)
    check(run_gmm(g, dex.DEX_F64, dex.DEX_GMM_PLAIN), oracle_gmm(g), 1e-10, f"fp64 {N},{D},{K}")


@pytest.mark.parametrize("N,D,K", [(257, 1, 3), (1000, 2, 5), (700, 7, 1), (1500, 16, 5),
                                   (999, 17, 6), (2048, 32, 3), (640, 33, 4), (3000, 64, 7),
                                   (513, 63, 2)])
def test_fp32_matrix_core_shapes(dev, N, D, K):
    from paper_2104_05372_amd import dex
    g = workloads.gmm_inputs(N, D, K, 200 + D, np.float32)
    check(run_gmm(g, dex.DEX_F32, dex.DEX_GMM_PLAIN), oracle_gmm(g), 1e-5, f"fp32 {N},{D},{K}")


@pytest.mark.parametrize("variant,tol", [(1, TOL_MIXED16), (2, TOL_BF16X3)])
@pytest.mark.parametrize("N,D,K", [(1000, 2, 5), (1500, 16, 5), (999, 17, 6), (3000, 64, 7),
                                   (640, 33, 4)])
def test_bf16_shapes(dev, variant, tol, N, D, K):
    g = workloads.gmm_inputs(N, D, K, 300 + D, np.float32)
    got = run_gmm(g, 2, variant)
    want = oracle_gmm(g)
    errs = [rel(a, b) for a, b in zip(got[2], want[2]) if b.size]
    print(f"  variant {variant} N={N} D={D} K={K} grad rel-L2 per block: {errs}", flush=True)
    check(got, want, tol, f"bf16 v{variant} {N},{D},{K}")


@pytest.mark.parametrize("offset", [100.0, 1000.0])
@pytest.mark.parametrize("D,variant", [(64, 1), (16, 1), (33, 1), (64, 0), (20, 2)])
def test_data_far_from_origin(dev, offset, D, variant):
    """x and the means ~ offset + N(0, 1): the objective and its gradient depend
    only on x - mu, but 16-bit operands of x itself, or the expansion
    x^T P x - 2 (P mu)^T x + mu^T P mu, would lose everything to cancellation.
    The kernels first move the origin to the mean of the first 16 means."""
    tol = {0: 1e-5, 1: TOL_MIXED16, 2: TOL_BF16X3}[variant]
    g = workloads.gmm_inputs(2000, D, 7, 50 + D)
    g = workloads.GMMInputs(g.alphas, g.means + offset, g.qd, g.l, g.x + offset).astype(np.float32)
    got = run_gmm(g, 2, variant)
    want = oracle_gmm(g)
    errs = [rel(a, b) for a, b in zip(got[2], want[2]) if b.size]
    print(f"  offset {offset} D={D} variant {variant}: grad rel-L2 per block {errs}", flush=True)
    check(got, want, tol, f"offset {offset} D={D} v{variant}")


@pytest.mark.parametrize("scale", [2.0 ** 10, 2.0 ** 8, 2.0 ** -6])
def test_feature_product_forward_under_rescaling(dev, scale):
    """x and the means scaled by s, Q by 1/s: the same distribution of
    Mahalanobis terms at large or small |x|, which moves the FP16 scale of the
    feature-product forward (BF16 variant, D = 64)."""
    g = workloads.gmm_inputs(3000, 64, 9, 21, np.float32)
    g = workloads.GMMInputs(g.alphas, (g.means * scale).astype(np.float32),
                            (g.qd - np.log(scale)).astype(np.float32),
                            (g.l / scale).astype(np.float32), (g.x * scale).astype(np.float32))
    check(run_gmm(g, 2, 1), oracle_gmm(g), TOL_MIXED16, f"bf16 rescaled by {scale}")


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_every_tile_configuration(dev, variant):
    from paper_2104_05372_amd import dex
    g = workloads.gmm_inputs(2500, 64, 9, 7, np.float32)
    want = oracle_gmm(g)
    tol = {0: 1e-5, 1: TOL_MIXED16, 2: TOL_BF16X3}[variant]
    d = dex.gmm_desc(g.N, g.D, g.K, dex.DEX_F32, variant)
    nf, nb = dex.dex_num_configs(d, dex.DEX_WS_FWD), dex.dex_num_configs(d, dex.DEX_WS_VJP)
    ref = None
    for c in range(1, max(nf, nb) + 1):
        got = run_gmm(g, dex.DEX_F32, variant, min(c, nf), min(c, nb))
        check(got, want, tol, f"config {c}")
        if ref is None:
            ref = got
        else:  # every configuration computes the same function
            assert rel(got[2][3], ref[2][3]) <= tol


def test_cotangent_scaling_and_accumulate(dev):
    from paper_2104_05372_amd import dex
    g = workloads.gmm_inputs(1200, 16, 4, 9, np.float32)
    want = oracle_gmm(g, ct=-2.5)
    got = run_gmm(g, dex.DEX_F32, dex.DEX_GMM_PLAIN, ct=-2.5)
    check(got, want, 1e-5, "ct=-2.5")
    base = [np.full_like(a, 0.25, dtype=np.float32) for a in want[2]]
    acc = run_gmm(g, dex.DEX_F32, dex.DEX_GMM_PLAIN, ct=-2.5, accumulate_into=base)
    for a, b in zip(acc[2], want[2]):
        if b.size:
            assert rel(a - 0.25, b) <= 1e-5


def test_autograd_function(dev):
    from paper_2104_05372_amd import autograd
    g = workloads.gmm_inputs(800, 8, 3, 13, np.float32)
    t = [torch.tensor(a, device=dev, requires_grad=(i < 4)) for i, a in enumerate(
        (g.alphas, g.means, g.qd, g.l, g.x))]
    F = autograd.gmm_loglik(*t, variant=0)
    F.backward()
    Fo, fo, go = oracle_gmm(g)
    assert abs(F.item() - Fo) <= 1e-5 * abs(Fo)
    for x, b in zip(t[:4], go):
        assert rel(x.grad.cpu().numpy(), b) <= 1e-5


def test_full_size_bf16_and_fp32(dev):
    """N=1e5, D=64, K=200 in the launch configuration the benchmark uses."""
    g = workloads.gmm_large()
    want = oracle_gmm(g)
    for variant, tol in ((1, TOL_MIXED16), (0, 1e-5)):
        got = run_gmm(g, 2, variant)
        errs = {n: rel(a, b) for n, a, b in zip(("alphas", "means", "qd", "l"), got[2], want[2])}
        print(f"  full size variant {variant}: F rel {abs(got[0]-want[0])/abs(want[0]):.3e} "
              f"f rel {rel(got[1], want[1]):.3e} grads {errs}", flush=True)
        check(got, want, tol, f"full size v{variant}")


def run_gmm_jvp(g, dtype, variant, tangent, dev="cuda"):
    """dex_fwd, then dex_jvp along `tangent`; returns (dF, the forward's F)."""
    from paper_2104_05372_amd import dex
    tdt = torch.float64 if dtype == dex.DEX_F64 else torch.float32
    t = [torch.tensor(np.ascontiguousarray(a), dtype=tdt, device=dev).contiguous()
         for a in (g.alphas, g.means, g.qd, g.l, g.x)]
    tt = [torch.tensor(np.ascontiguousarray(a), dtype=tdt, device=dev).reshape(-1)
          for a in tangent]
    N, D, K = g.N, g.D, g.K
    d = dex.gmm_desc(N, D, K, dtype, variant)
    F = torch.empty(1, dtype=tdt, device=dev)
    f = torch.empty(N, dtype=tdt, device=dev)
    cache = torch.empty(dex.dex_workspace_bytes(d, dex.DEX_WS_RESID), dtype=torch.uint8, device=dev)
    print(f"  gmm jvp N={N} D={D} K={K} dtype={dtype} variant={variant}", flush=True)
    dex.dex_fwd(d, t, [F], [f, cache], dex.workspace(dex.dex_workspace_bytes(d, dex.DEX_WS_FWD), dev))
    dF = torch.empty(1, dtype=tdt, device=dev)
    dex.dex_jvp(d, t, tt, [dF], dex.workspace(dex.dex_workspace_bytes(d, dex.DEX_WS_JVP), dev),
                resid=[f, cache])
    torch.cuda.synchronize()
    return float(dF.item()), float(F.item())


def along_gradient(g, seed, mix=0.5):
    """A tangent mostly along the oracle gradient (unit gradient direction plus
    `mix` times a unit random direction), so that dF = <grad F, t> is of the
    size of |grad F| and a relative error bound on dF is meaningful."""
    go = ogmm.vjp(*g.params(), g.x)
    rng = np.random.default_rng(seed)
    noise = [rng.standard_normal(np.shape(a)) for a in go]
    ng = np.sqrt(sum(float(np.sum(a * a)) for a in go))
    nn = np.sqrt(sum(float(np.sum(a * a)) for a in noise))
    return [(a / ng + mix * b / nn).astype(g.x.dtype) for a, b in zip(go, noise)]


# (16-bit variant at D = 64: the matrix-core tangent products; every other
# case: the vector-ALU tangent pass in FP32. The weights exp(beta - f) use the
# forward's residual f, so the forward mode of a variant carries that
# variant's forward error: its bound is the variant's.)
@pytest.mark.parametrize("N,D,K,variant,tol", [(3000, 8, 5, 0, 1e-5), (2500, 64, 9, 1, TOL_MIXED16),
                                                (2000, 20, 7, 2, TOL_BF16X3), (1500, 64, 33, 0, 1e-5),
                                                (3100, 64, 40, 1, TOL_MIXED16),
                                                (1100, 16, 5, 1, TOL_MIXED16), (700, 1, 3, 0, 1e-5)])
def test_forward_mode(dev, N, D, K, variant, tol):
    """dex_jvp of the objective (the linearized loop run forward, no reverse
    pass) against the oracle's forward mode, relative to |dF|."""
    from paper_2104_05372_amd import dex
    g = workloads.gmm_inputs(N, D, K, 40 + D, np.float32)
    tangent = along_gradient(g, D + K)
    got, _ = run_gmm_jvp(g, dex.DEX_F32, variant, tangent)
    want = ogmm.jvp(*g.params(), g.x, tangent)
    print(f"  jvp N={N} D={D} K={K} v{variant}: dF {got:.9g} oracle {want:.9g} "
          f"rel {abs(got - want) / abs(want):.3e}", flush=True)
    assert abs(got - want) <= tol * abs(want), (got, want)


@pytest.mark.parametrize("D,variant,tol", [(64, 1, TOL_MIXED16), (64, 0, 1e-5), (12, 1, TOL_MIXED16)])
def test_forward_mode_far_from_origin(dev, D, variant, tol):
    from paper_2104_05372_amd import dex
    g = workloads.gmm_inputs(2000, D, 6, 60 + D)
    g = workloads.GMMInputs(g.alphas, g.means + 100.0, g.qd, g.l, g.x + 100.0).astype(np.float32)
    tangent = along_gradient(g, 7)
    got, _ = run_gmm_jvp(g, dex.DEX_F32, variant, tangent)
    want = ogmm.jvp(*g.params(), g.x, tangent)
    assert abs(got - want) <= tol * abs(want), (got, want)


@pytest.mark.parametrize("variant,tol", [(1, TOL_MIXED16), (0, 1e-5)])
def test_forward_mode_transposes_to_reverse_mode(dev, variant, tol):
    """<J t, 1> = <t, J^T 1>: dex_jvp (forward pass over tangents) against the
    inner product of t with dex_vjp's gradient (reverse pass), two different
    kernels, for random tangents."""
    from paper_2104_05372_amd import dex
    g = workloads.gmm_inputs(2600, 64, 11, 71, np.float32)
    _, _, grads = run_gmm(g, dex.DEX_F32, variant)
    rng = np.random.default_rng(5)
    for trial in range(3):
        tangent = [rng.standard_normal(np.shape(a)).astype(np.float32) for a in grads]
        if trial == 2:
            tangent = along_gradient(g, 9)
        jv, _ = run_gmm_jvp(g, dex.DEX_F32, variant, tangent)
        vj = sum(float(np.dot(a.ravel().astype(np.float64), b.ravel().astype(np.float64)))
                 for a, b in zip(grads, tangent))
        scale = sum(float(np.dot(np.abs(a.ravel()), np.abs(b.ravel()))) for a, b in zip(grads, tangent))
        print(f"  trial {trial}: jvp {jv:.9g} <t, vjp> {vj:.9g} scale {scale:.4g}", flush=True)
        assert abs(jv - vj) <= 2 * tol * scale, (trial, jv, vj, scale)


def test_forward_mode_full_size(dev):
    """N=1e5, D=64, K=200, 16-bit variant (the matrix-core tangent products)."""
    from paper_2104_05372_amd import dex
    g = workloads.gmm_large()
    tangent = along_gradient(g, 3)
    got, _ = run_gmm_jvp(g, dex.DEX_F32, dex.DEX_GMM_BF16, tangent)
    want = ogmm.jvp(*g.params(), g.x, tangent)
    print(f"  full-size jvp: {got:.9g} oracle {want:.9g} rel {abs(got - want) / abs(want):.3e}",
          flush=True)
    assert abs(got - want) <= TOL_MIXED16 * abs(want)


def test_forward_mode_fp64(dev):
    from paper_2104_05372_amd import dex
    g = workloads.gmm_inputs(400, 3, 4, 9, np.float64)
    rng = np.random.default_rng(3)
    tangent = [rng.standard_normal(np.shape(a)) for a in (g.alphas, g.means, g.qd, g.l)]
    got, _ = run_gmm_jvp(g, dex.DEX_F64, 0, tangent)
    want = ogmm.jvp(*g.params(), g.x, tangent)
    assert abs(got - want) <= 1e-10 * max(1.0, abs(want))


@pytest.mark.parametrize("variant,D", [(0, 16), (1, 64), (0, 64), (1, 20)])
def test_nan_point_propagates_and_leaves_no_state(dev, variant, D):
    """One NaN coordinate: F, that point's f and every gradient entry are NaN
    (each component's sums take that point with a NaN weight), as in the
    oracle; every other point's f is unaffected; the call reports success and a
    following call on clean data is exact."""
    tol = {0: 1e-5, 1: TOL_MIXED16}[variant]
    g = workloads.gmm_inputs(1000, D, 5, 77, np.float32)
    x = g.x.copy()
    x[123, 3] = np.nan
    got = run_gmm(workloads.GMMInputs(g.alphas, g.means, g.qd, g.l, x), 2, variant)
    Fo, fo, go = oracle_gmm(workloads.GMMInputs(g.alphas, g.means, g.qd, g.l, x))
    assert np.isnan(got[0]) and np.isnan(Fo)
    assert np.isnan(got[1][123]) and np.isnan(fo[123])
    others = np.delete(np.arange(1000), 123)
    assert np.all(np.isfinite(got[1][others]))
    assert rel(got[1][others], fo[others]) <= tol
    for a, b in zip(got[2], go):
        assert np.array_equal(np.isnan(a), np.isnan(np.asarray(b).reshape(a.shape)))
    check(run_gmm(g, 2, variant), oracle_gmm(g), tol, "clean call after a NaN call")
