"""Pins for the in-place stencil loop oracle: the FFT closed form (the periodic
five-point step is diagonal in the Fourier basis), the adjoint identity of a
single step, and central finite differences of the loss."""
import numpy as np
import pytest

import workloads
from oracle import stencil


def fft_symbol(H, W, c=0.2):
    p = np.arange(H)[:, None]
    q = np.arange(W)[None, :]
    return 1.0 + c * (2 * np.cos(2 * np.pi * p / H) + 2 * np.cos(2 * np.pi * q / W) - 4.0)


def fft_power(v, H, W, steps):
    lam = fft_symbol(H, W) ** steps
    return np.real(np.fft.ifft2(lam * np.fft.fft2(v)))


@pytest.mark.parametrize("H,W,steps", [(16, 16, 50), (32, 24, 7), (8, 40, 1)])
def test_forward_and_gradient_match_fft_closed_form(H, W, steps):
    u0, target = workloads.stencil_inputs(H, W, 9)
    L, uT, grad = stencil.loss_and_grad(u0, target, steps)
    want_uT = fft_power(u0.astype(np.float64), H, W, steps)
    assert np.max(np.abs(uT - want_uT)) < 1e-12
    want_grad = fft_power(want_uT - target.astype(np.float64), H, W, steps)
    assert np.max(np.abs(grad - want_grad)) < 1e-12
    assert np.isclose(L, 0.5 * np.sum((want_uT - target) ** 2), rtol=1e-12)


def test_step_adjoint_identity():
    rng = np.random.default_rng(0)
    u, v = rng.standard_normal((2, 12, 20))
    assert np.isclose(np.sum(stencil.step(u) * v), np.sum(u * stencil.step_transpose(v)),
                      rtol=1e-13)


def test_step_transpose_is_not_forward_for_asymmetric_weights():
    """With direction-dependent weights the transpose differs from the forward,
    so the symmetric case is not hiding an index mistake: rebuild the scatter
    form with an asymmetric kernel and check the adjoint identity."""
    rng = np.random.default_rng(1)
    u, v = rng.standard_normal((2, 9, 11))
    fwd = lambda z: z + 0.3 * np.roll(z, -1, 0) - 0.1 * np.roll(z, 1, 1)
    # transpose: cell (y,x) read z[y+1,x] -> accumulate at y+1; read z[y,x-1] -> at x-1
    tr = lambda g: g + 0.3 * np.roll(g, 1, 0) - 0.1 * np.roll(g, -1, 1)
    assert np.isclose(np.sum(fwd(u) * v), np.sum(u * tr(v)), rtol=1e-13)


def test_gradient_central_differences():
    u0, target = workloads.stencil_inputs(10, 10, 3)
    u0 = u0.astype(np.float64)
    _, _, grad = stencil.loss_and_grad(u0, target, 12)
    for (y, x) in [(0, 0), (3, 7), (9, 9)]:
        e = np.zeros_like(u0)
        e[y, x] = 1e-6
        up = stencil.loss_and_grad(u0 + e, target, 12)[0]
        dn = stencil.loss_and_grad(u0 - e, target, 12)[0]
        assert np.isclose((up - dn) / 2e-6, grad[y, x], rtol=1e-6, atol=1e-8)


def test_planted_gauss_seidel_is_caught():
    """An in-place update that reads already-updated neighbours (not the value
    semantics of `get`) disagrees with the closed form."""
    u0, _ = workloads.stencil_inputs(8, 8, 2)
    u = u0.astype(np.float64).copy()
    H, W = u.shape
    for y in range(H):
        for x in range(W):
            u[y, x] = u[y, x] + 0.2 * (u[(y + 1) % H, x] + u[y - 1, x] + u[y, (x + 1) % W]
                                       + u[y, x - 1] - 4 * u[y, x])
    assert np.max(np.abs(u - fft_power(u0.astype(np.float64), H, W, 1))) > 1e-3


@pytest.mark.parametrize("rho", [0.05, -0.3])
def test_nonlinear_term_gradient_central_differences(rho):
    u0, target = workloads.stencil_inputs(9, 12, 5)
    u0 = u0.astype(np.float64)
    _, _, grad = stencil.loss_and_grad(u0, target, 15, rho=rho)
    for (y, x) in [(0, 0), (4, 7), (8, 11)]:
        e = np.zeros_like(u0)
        e[y, x] = 1e-6
        up = stencil.loss_and_grad(u0 + e, target, 15, rho=rho)[0]
        dn = stencil.loss_and_grad(u0 - e, target, 15, rho=rho)[0]
        assert np.isclose((up - dn) / 2e-6, grad[y, x], rtol=1e-6, atol=1e-8)


def test_nonlinear_step_adjoint_identity():
    """The transposed step at state u is the adjoint of the linearized step."""
    rng = np.random.default_rng(4)
    u, du, v = rng.standard_normal((3, 10, 14))
    # linearized step applied to du: diffusion part is linear, sin part gives cos(u) du
    lin = stencil.step(du) + 0.2 * np.cos(u) * du
    assert np.isclose(np.sum(lin * v), np.sum(du * stencil.step_transpose(v, u=u, rho=0.2)),
                      rtol=1e-13)


@pytest.mark.parametrize("rho", [0.0, 0.3])
def test_loss_jvp_central_differences(rho):
    rng = np.random.default_rng(21)
    u0, tg = rng.standard_normal((10, 12)), rng.standard_normal((10, 12))
    du0, dtg = rng.standard_normal((10, 12)), rng.standard_normal((10, 12))
    h = 1e-5
    up = stencil.loss_and_grad(u0 + h * du0, tg + h * dtg, 9, rho=rho)[0]
    dn = stencil.loss_and_grad(u0 - h * du0, tg - h * dtg, 9, rho=rho)[0]
    got = stencil.loss_jvp(u0, tg, du0, dtg, 9, rho=rho)
    assert np.isclose((up - dn) / (2 * h), got, rtol=1e-7, atol=1e-9)


@pytest.mark.parametrize("rho", [0.0, -0.2])
def test_loss_jvp_vjp_dot_product_identity(rho):
    """<grad_u0, du0> - <u_T - target, dtarget> = dL, against the pinned reverse pass."""
    rng = np.random.default_rng(22)
    u0, tg = rng.standard_normal((8, 9)), rng.standard_normal((8, 9))
    du0, dtg = rng.standard_normal((8, 9)), rng.standard_normal((8, 9))
    _, uT, g = stencil.loss_and_grad(u0, tg, 13, rho=rho)
    want = float(np.sum(g * du0) - np.sum((uT - tg) * dtg))
    assert np.isclose(stencil.loss_jvp(u0, tg, du0, dtg, 13, rho=rho), want, rtol=1e-12)


def test_loss_jvp_linear_loop_is_the_loop_of_the_tangent():
    """With rho = 0 the loop is linear, so the tangent state is the forward loop
    applied to du0 (and to nothing else)."""
    rng = np.random.default_rng(23)
    u0, tg, du0 = (rng.standard_normal((6, 10)) for _ in range(3))
    uT = stencil.forward(u0, 7)
    want = float(np.sum((uT - tg) * stencil.forward(du0, 7)))
    got = stencil.loss_jvp(u0, tg, du0, np.zeros_like(tg), 7)
    assert np.isclose(got, want, rtol=1e-12)
    assert stencil.loss_jvp(u0, tg, np.zeros_like(u0), np.zeros_like(tg), 7, rho=0.4) == 0.0
