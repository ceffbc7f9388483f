"""The torch.autograd.Function wrappers: each backward is the library's adjoint
kernel (dex_vjp), reached through torch's autograd, and compared with the FP64
oracle's reverse pass (grad f x = transpose (snd (linearize f x)) applied to
the output cotangent, Sec. 5.2)."""
import numpy as np
import pytest
import torch

import workloads
from oracle import gmm as ogmm
from oracle import scatter as osc
from oracle import stencil as ost

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("V,R,n,seed", [(300, 100, 4097, 3), (1000, 128, 50_000, 1), (7, 3, 5000, 2)])
def test_gather_scale_backward(dev, V, R, n, seed):
    from paper_2104_05372_amd import autograd
    si = workloads.scatter_inputs(V, R, n, 1.1, seed)
    T = torch.tensor(si.table, device=dev, requires_grad=True)
    w = torch.tensor(si.w, device=dev, requires_grad=True)
    idx = torch.tensor(si.idx, device=dev)
    out = autograd.gather_scale(T, idx, w)
    assert rel(out.detach().cpu().numpy(), osc.gather(si.table, si.idx, si.w)) <= 1e-6
    out.backward(torch.tensor(si.g, device=dev))
    assert rel(T.grad.cpu().numpy(), osc.scatter(V, si.idx, si.w, si.g)) <= 1e-5
    assert rel(w.grad.cpu().numpy(), osc.scatter_dw(si.table, si.idx, si.g)) <= 1e-5


def test_gather_scale_backward_without_weight_gradient(dev):
    """w without requires_grad: the backward skips dw (DEX_NO_DW) and dT is
    unchanged."""
    from paper_2104_05372_amd import autograd
    si = workloads.scatter_inputs(500, 64, 20_000, 1.1, 8)
    T = torch.tensor(si.table, device=dev, requires_grad=True)
    w = torch.tensor(si.w, device=dev)
    out = autograd.gather_scale(T, torch.tensor(si.idx, device=dev), w)
    (out * torch.tensor(si.g, device=dev)).sum().backward()
    assert w.grad is None
    assert rel(T.grad.cpu().numpy(), osc.scatter(500, si.idx, si.w, si.g)) <= 1e-5


@pytest.mark.parametrize("steps,every,rho", [(40, 32, 0.0), (40, 7, 0.3), (25, 1, 0.3), (33, 33, -0.2)])
def test_diffusion_backward(dev, steps, every, rho):
    from paper_2104_05372_amd import autograd
    u0, tg = workloads.stencil_inputs(64, 96, 9)
    tu = torch.tensor(u0, device=dev, requires_grad=True)
    L, uT = autograd.diffusion_loss(tu, torch.tensor(tg, device=dev), steps, every, rho=rho)
    (2.0 * L).backward()  # an output cotangent of 2
    Lo, uTo, go = ost.loss_and_grad(u0, tg, steps, rho=rho)
    assert abs(L.item() - Lo) <= 1e-5 * abs(Lo)
    assert rel(uT.cpu().numpy(), uTo) <= 1e-5
    assert rel(tu.grad.cpu().numpy(), 2.0 * go) <= 1e-5


def test_diffusion_checkpoint_interval_through_autograd(dev):
    """The recompute interval is invisible in the gradient (rho != 0, so the
    reverse pass reads the recomputed states)."""
    from paper_2104_05372_amd import autograd
    u0, tg = workloads.stencil_inputs(32, 64, 4)
    grads = []
    for every in (1, 6, 50):
        tu = torch.tensor(u0, device=dev, requires_grad=True)
        L, _ = autograd.diffusion_loss(tu, torch.tensor(tg, device=dev), 50, every, rho=0.25)
        L.backward()
        grads.append(tu.grad.cpu().numpy())
    assert np.array_equal(grads[0], grads[1]) and np.array_equal(grads[0], grads[2])


@pytest.mark.parametrize("dtype,variant,tol", [(np.float64, 0, 1e-10), (np.float32, 1, 1e-2),
                                               (np.float32, 2, 2e-4)])
def test_gmm_loglik_backward_variants(dev, dtype, variant, tol):
    from paper_2104_05372_amd import autograd
    g = workloads.gmm_inputs(1200, 64 if variant == 1 else 12, 6, 17, dtype)
    t = [torch.tensor(a, device=dev, requires_grad=(i < 4)) for i, a in enumerate(
        (g.alphas, g.means, g.qd, g.l, g.x))]
    F = autograd.gmm_loglik(*t, variant=variant)
    (-3.0 * F).backward()
    Fo, fo = ogmm.objective(*g.params(), g.x)
    go = ogmm.vjp(*g.params(), g.x, fo, -3.0)
    assert abs(F.item() - Fo) <= tol * abs(Fo)
    assert t[4].grad is None
    for x, b in zip(t[:4], go):
        assert rel(x.grad.cpu().numpy(), b) <= tol
