"""Pins for the FP64 GMM oracle, against things other than itself:
scipy's Gaussian log-density, torch autograd, central finite differences,
complex-step derivatives, invariants, and planted mistakes that must be caught."""
import numpy as np
import pytest
import scipy.special
import scipy.stats

import workloads
from oracle import gmm


def _Q_independent(qd_k, l_k):
    """Q built from the packing convention by explicit enumeration of the
    strictly-lower entries in row-major order (independent of oracle.build_Q)."""
    D = qd_k.shape[0]
    Q = np.zeros((D, D))
    it = iter(l_k)
    for a in range(D):
        for b in range(a):
            Q[a, b] = next(it)
        Q[a, a] = np.exp(qd_k[a])
    return Q


def scipy_objective(g):
    """F through scipy: beta[i,k] = alphas[k] + logpdf_k(x_i) + D/2 log(2 pi), the
    Gaussian with precision Q^T Q has log det(Q) = sum qd (Q is triangular)."""
    N, D, K = g.N, g.D, g.K
    beta = np.empty((N, K))
    for k in range(K):
        Q = _Q_independent(g.qd[k], g.l[k])
        cov = np.linalg.inv(Q.T @ Q)
        lp = scipy.stats.multivariate_normal.logpdf(g.x, mean=g.means[k], cov=cov)
        beta[:, k] = g.alphas[k] + lp + 0.5 * D * np.log(2 * np.pi)
    return (scipy.special.logsumexp(beta, axis=1).sum()
            - N * scipy.special.logsumexp(g.alphas))


def params_flat(g):
    return np.concatenate([g.alphas.ravel(), g.means.ravel(), g.qd.ravel(), g.l.ravel()])


def unflat(g, v):
    K, D = g.K, g.D
    s = [K, K * D, K * D, K * workloads.n_lower(D)]
    parts = np.split(v, np.cumsum(s)[:-1])
    return workloads.GMMInputs(parts[0], parts[1].reshape(K, D), parts[2].reshape(K, D),
                               parts[3].reshape(K, -1), g.x)


def F_of(g, v):
    h = unflat(g, v)
    return gmm.objective(h.alphas, h.means, h.qd, h.l, h.x)[0]


def grad_flat(g, ct=1.0):
    return np.concatenate([a.ravel() for a in gmm.vjp(g.alphas, g.means, g.qd, g.l, g.x, ct=ct)])


@pytest.mark.parametrize("N,D,K,seed", [(1000, 2, 5, 0), (300, 3, 4, 11), (200, 6, 3, 12)])
def test_objective_matches_scipy(N, D, K, seed):
    g = workloads.gmm_inputs(N, D, K, seed)
    F, f = gmm.objective(*g.params(), g.x)
    ref = scipy_objective(g)
    assert abs(F - ref) <= 1e-10 * max(1.0, abs(ref))


def test_single_component_closed_form():
    g = workloads.gmm_inputs(50, 4, 1, 21)
    F, _ = gmm.objective(*g.params(), g.x)
    # with one component, the log-sum-exps are the identity and alphas cancel
    Q = _Q_independent(g.qd[0], g.l[0])
    r = g.x - g.means[0]
    want = g.N * g.qd[0].sum() - 0.5 * np.einsum("ia,ia->", r @ Q.T, r @ Q.T)
    assert abs(F - want) <= 1e-11 * abs(want)
    d_alphas = gmm.vjp(*g.params(), g.x)[0]
    assert abs(d_alphas[0]) <= 1e-9


def test_alpha_shift_invariance():
    g = workloads.gmm_small()
    F0, _ = gmm.objective(*g.params(), g.x)
    F1, _ = gmm.objective(g.alphas + 3.7, g.means, g.qd, g.l, g.x)
    assert abs(F1 - F0) <= 1e-10 * abs(F0)
    d_alphas = gmm.vjp(*g.params(), g.x)[0]
    assert abs(d_alphas.sum()) <= 1e-9


def test_scalar_closed_form_D1_K1():
    # N points, D = 1, K = 1: F = N*qd - 1/2 sum (e^qd (x - mu))^2,
    # dF/dmu = e^{2 qd} sum (x - mu), dF/dqd = N - e^{2 qd} sum (x - mu)^2.
    x = np.array([[0.3], [-1.2], [2.0]])
    qd, mu = 0.25, -0.4
    g = workloads.GMMInputs(np.array([0.7]), np.array([[mu]]), np.array([[qd]]),
                            np.zeros((1, 0)), x)
    F, _ = gmm.objective(*g.params(), g.x)
    r = x[:, 0] - mu
    assert np.isclose(F, 3 * qd - 0.5 * np.exp(2 * qd) * np.sum(r * r), rtol=1e-14)
    da, dm, dq, dl = gmm.vjp(*g.params(), g.x)
    assert np.isclose(dm[0, 0], np.exp(2 * qd) * r.sum(), rtol=1e-13)
    assert np.isclose(dq[0, 0], 3 - np.exp(2 * qd) * np.sum(r * r), rtol=1e-13)
    assert abs(da[0]) < 1e-14 and dl.shape == (1, 0)


def test_grad_central_differences():
    g = workloads.gmm_small()
    v = params_flat(g)
    gr = grad_flat(g)
    rng = np.random.default_rng(5)
    sel = rng.choice(v.size, 20, replace=False)
    fd = np.empty(sel.size)
    for n, j in enumerate(sel):
        h = 1e-6 * max(1.0, abs(v[j]))
        e = np.zeros_like(v)
        e[j] = h
        fd[n] = (F_of(g, v + e) - F_of(g, v - e)) / (2 * h)
    err = np.linalg.norm(fd - gr[sel]) / np.linalg.norm(gr[sel])
    assert err < 1e-6, err


def _F_complex(g, v):
    """The objective evaluated in complex arithmetic (for the complex-step
    derivative); the max shift of each log-sum-exp uses real parts."""
    h = unflat(g, v)
    N, D, K = h.x.shape[0], h.x.shape[1], h.alphas.shape[0]
    beta = np.empty((N, K), dtype=complex)
    for k in range(K):
        Q = np.zeros((D, D), dtype=complex)
        p = 0
        for a in range(D):
            for b in range(a):
                Q[a, b] = h.l[k][p]
                p += 1
            Q[a, a] = np.exp(h.qd[k][a])
        y = (h.x - h.means[k]) @ Q.T
        beta[:, k] = h.alphas[k] + h.qd[k].sum() - 0.5 * np.sum(y * y, axis=1)

    def lse(z, axis=None):
        m = np.max(z.real, axis=axis, keepdims=True)
        s = np.log(np.sum(np.exp(z - m), axis=axis, keepdims=True)) + m
        return s

    return np.sum(lse(beta, 1)) - N * lse(h.alphas)[0]


@pytest.mark.parametrize("N,D,K,seed", [(1000, 2, 5, 0), (120, 5, 3, 31)])
def test_grad_complex_step(N, D, K, seed):
    g = workloads.gmm_inputs(N, D, K, seed)
    v = params_flat(g).astype(complex)
    gr = grad_flat(g)
    h = 1e-30
    cs = np.empty(v.size)
    for j in range(v.size):
        e = np.zeros_like(v)
        e[j] = 1j * h
        cs[j] = _F_complex(g, v + e).imag / h
    assert np.max(np.abs(cs - gr) / np.maximum(1.0, np.abs(gr))) < 1e-11


def test_grad_torch_autograd():
    torch = pytest.importorskip("torch")
    g = workloads.gmm_inputs(400, 4, 6, 41)
    t = {n: torch.tensor(getattr(g, n), dtype=torch.float64, requires_grad=(n != "x"))
         for n in ("alphas", "means", "qd", "l", "x")}
    D = g.D
    rows, cols = torch.tril_indices(D, D, offset=-1)
    Fsum = 0.0
    betas = []
    for k in range(g.K):
        Q = torch.diag(torch.exp(t["qd"][k]))
        L = torch.zeros(D, D, dtype=torch.float64).index_put((rows, cols), t["l"][k])
        Q = Q + L
        y = (t["x"] - t["means"][k]) @ Q.T
        betas.append(t["alphas"][k] + t["qd"][k].sum() - 0.5 * (y * y).sum(1))
    B = torch.stack(betas, 1)
    Fsum = torch.logsumexp(B, 1).sum() - g.N * torch.logsumexp(t["alphas"], 0)
    Fsum.backward()
    ours = gmm.vjp(*g.params(), g.x)
    for name, o in zip(("alphas", "means", "qd", "l"), ours):
        ref = t[name].grad.numpy()
        assert np.linalg.norm(o - ref) <= 1e-12 * np.linalg.norm(ref), name


def test_vjp_is_linear_in_cotangent():
    g = workloads.gmm_inputs(100, 3, 4, 51)
    a = grad_flat(g, 1.0)
    b = grad_flat(g, -2.5)
    assert np.allclose(b, -2.5 * a, rtol=1e-13, atol=1e-13)


def test_jvp_vjp_dot_product():
    """<vjp(1), v> equals the directional derivative along v (complex step)."""
    g = workloads.gmm_inputs(150, 4, 3, 61)
    v0 = params_flat(g)
    rng = np.random.default_rng(0)
    dv = rng.standard_normal(v0.size)
    jvp = _F_complex(g, v0 + 1e-30j * dv).imag / 1e-30
    assert abs(np.dot(grad_flat(g), dv) - jvp) <= 1e-11 * max(1.0, abs(jvp))


def test_suff_stats_assemble_to_gradient():
    g = workloads.gmm_inputs(200, 4, 3, 71)
    F, f = gmm.objective(*g.params(), g.x)
    da, dm, dq, dl = gmm.vjp(*g.params(), g.x, f)
    st = gmm.suff_stats(*g.params(), g.x, f)
    sm = np.exp(g.alphas - scipy.special.logsumexp(g.alphas))
    for k, (A, b, M) in st.items():
        Q = _Q_independent(g.qd[k], g.l[k])
        assert np.isclose(da[k], A - g.N * sm[k], atol=1e-10)
        assert np.allclose(dm[k], Q.T @ b, atol=1e-10)
        assert np.allclose(dq[k], A - np.exp(g.qd[k]) * np.diag(M), atol=1e-10)
        assert np.allclose(dl[k], -M[np.tril_indices(g.D, -1)], atol=1e-10)


# --- planted mistakes: each must make one of the pins above fail -------------

def test_planted_transposed_Q_is_caught(monkeypatch):
    g = workloads.gmm_inputs(300, 3, 4, 11)
    good = gmm.build_Q
    monkeypatch.setattr(gmm, "build_Q", lambda qd, l: good(qd, l).T)
    F, _ = gmm.objective(*g.params(), g.x)
    assert abs(F - scipy_objective(g)) > 1e-6 * abs(F)


def test_planted_linear_diagonal_is_caught(monkeypatch):
    g = workloads.gmm_inputs(300, 3, 4, 11)
    good = gmm.build_Q

    def bad(qd, l):
        Q = good(qd, l)
        np.fill_diagonal(Q, 1.0 + np.asarray(qd))   # exp(qd) replaced by 1 + qd
        return Q

    monkeypatch.setattr(gmm, "build_Q", bad)
    F, _ = gmm.objective(*g.params(), g.x)
    assert abs(F - scipy_objective(g)) > 1e-6 * abs(F)


def _tangent(g, seed):
    rng = np.random.default_rng(seed)
    return tuple(rng.standard_normal(np.shape(a)) for a in (g.alphas, g.means, g.qd, g.l))


@pytest.mark.parametrize("N,D,K,seed", [(40, 3, 4, 1), (25, 5, 2, 2), (30, 1, 3, 3)])
def test_jvp_central_differences(N, D, K, seed):
    g = workloads.gmm_inputs(N, D, K, seed, np.float64)
    t = _tangent(g, seed)
    h = 1e-6
    args = (g.alphas, g.means, g.qd, g.l)
    up = gmm.objective(*(a + h * b for a, b in zip(args, t)), g.x)[0]
    dn = gmm.objective(*(a - h * b for a, b in zip(args, t)), g.x)[0]
    got = gmm.jvp(*args, g.x, t)
    assert np.isclose((up - dn) / (2 * h), got, rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("N,D,K,seed", [(50, 4, 3, 4), (20, 6, 5, 5)])
def test_jvp_vjp_dot_product_identity(N, D, K, seed):
    """<J t, 1> = <t, J^T 1>: forward mode against the pinned reverse pass."""
    g = workloads.gmm_inputs(N, D, K, seed, np.float64)
    t = _tangent(g, seed + 10)
    grads = gmm.vjp(g.alphas, g.means, g.qd, g.l, g.x)
    rhs = sum(float(np.sum(np.asarray(a) * b)) for a, b in zip(grads, t))
    assert np.isclose(gmm.jvp(g.alphas, g.means, g.qd, g.l, g.x, t), rhs, rtol=1e-10)


def test_jvp_along_a_uniform_alpha_shift_is_zero():
    """F is invariant under alphas -> alphas + c (the log-sum-exp terms and the
    normaliser move together), so the derivative along (1, .., 1) vanishes."""
    g = workloads.gmm_inputs(30, 3, 4, 6, np.float64)
    t = (np.ones(4), np.zeros_like(g.means), np.zeros_like(g.qd), np.zeros_like(g.l))
    assert abs(gmm.jvp(g.alphas, g.means, g.qd, g.l, g.x, t)) < 1e-9
