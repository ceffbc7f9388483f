"""GMM log-likelihood objective and its reverse-mode derivative, in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The objective is a pointful loop over the index sets i:N (points) and k:K
(components):

    beta[i, k] = alphas[k] + sum_d qd[k, d] - 1/2 * || Q_k (x[i] - means[k]) ||^2
    f[i]       = logsumexp_k beta[i, k]
    F          = sum_i f[i] - N * logsumexp_k alphas[k]

with Q_k = diag(exp(qd[k])) + L_k and L_k strictly lower-triangular, L_k[a, b]
(a > b) stored at l[k, a*(a-1)/2 + b]. The paper does not contain this objective;
it supplies the mechanism by which its gradient is obtained:

  * grad f x = transpose (snd (linearize f x)) 1.0 (Sec. 5.2, definition of
    `grad`): the gradient is the transposed linear map applied to the output
    cotangent.
  * Inside `for i k`, the parameter reads `alphas.k`, `means.k` and `Q.k` are
    indexed reads; rule LetIndexingTranspose (Fig. "transposition rules")
    turns each into an accumulation `dparam!k += ...` into a sliced cotangent
    reference, which is a regular segmented reduction over i (Sec. 6.1.3).
  * `sum` over i and the log-sum-exp reductions are complete reductions; their
    transposes broadcast the cotangent (AddTranspose, Fig. "transposition
    rules").
  * Non-linear intermediates (beta and f) are kept from the forward pass, or
    recomputed, as LetNonlinearTranspose keeps non-linear lets forward.

log-sum-exp uses the max shift: m + log(sum exp(v - m)), m = max v.
"""
from __future__ import annotations

import numpy as np


def lower_index(a: int, b: int) -> int:
    """Position of Q[a, b] (a > b) in the packed strictly-lower vector."""
    return a * (a - 1) // 2 + b


def build_Q(qd_k: np.ndarray, l_k: np.ndarray) -> np.ndarray:
    """Q_k = diag(exp(qd_k)) + strict-lower(l_k), as a dense D x D FP64 matrix."""
    D = qd_k.shape[0]
    Q = np.diag(np.exp(np.asarray(qd_k, dtype=np.float64)))
    for a in range(1, D):
        for b in range(a):
            Q[a, b] = float(l_k[lower_index(a, b)])
    return Q


def logsumexp(v: np.ndarray, axis=None) -> np.ndarray:
    """Max-shifted log-sum-exp."""
    m = np.max(v, axis=axis, keepdims=True)
    s = np.log(np.sum(np.exp(v - m), axis=axis, keepdims=True)) + m
    return np.squeeze(s, axis=axis) if axis is not None else s.reshape(())


def _f64(*arrays):
    return tuple(np.asarray(a, dtype=np.float64) for a in arrays)


def beta(alphas, means, qd, l, x) -> np.ndarray:
    """beta[i, k] for all points and components, as an [N, K] FP64 array."""
    alphas, means, qd, l, x = _f64(alphas, means, qd, l, x)
    N, K = x.shape[0], alphas.shape[0]
    out = np.empty((N, K))
    for k in range(K):
        Q = build_Q(qd[k], l[k])
        r = x - means[k]                    # r[i] = x[i] - means[k]
        y = r @ Q.T                         # y[i] = Q_k r[i]
        out[:, k] = alphas[k] + qd[k].sum() - 0.5 * np.sum(y * y, axis=1)
    return out


def objective(alphas, means, qd, l, x):
    """Forward pass. Returns (F, f) with f[i] = logsumexp_k beta[i, k]."""
    b = beta(alphas, means, qd, l, x)
    f = logsumexp(b, axis=1)
    N = b.shape[0]
    F = float(np.sum(f) - N * logsumexp(np.asarray(alphas, np.float64)))
    return F, f


def vjp(alphas, means, qd, l, x, f=None, ct: float = 1.0):
    """Reverse pass: cotangents of (alphas, means, qd, l) for output cotangent ct.

    Follows the transposed loop: for each component k, the cotangent of
    beta[i, k] is w[i, k] = ct * exp(beta[i, k] - f[i]) (transpose of the
    log-sum-exp over k, then of the sum over i); each read of a component-k
    parameter inside the loop over i becomes an accumulation over i into that
    parameter's cotangent slot k.
    """
    alphas, means, qd, l, x = _f64(alphas, means, qd, l, x)
    N, D = x.shape
    K = alphas.shape[0]
    if f is None:
        _, f = objective(alphas, means, qd, l, x)
    f = np.asarray(f, dtype=np.float64)
    d_alphas = np.zeros(K)
    d_means = np.zeros((K, D))
    d_qd = np.zeros((K, D))
    d_l = np.zeros((K, D * (D - 1) // 2))
    for k in range(K):
        Q = build_Q(qd[k], l[k])
        r = x - means[k]
        y = r @ Q.T
        bk = alphas[k] + qd[k].sum() - 0.5 * np.sum(y * y, axis=1)
        w = ct * np.exp(bk - f)                       # cotangent of beta[:, k]
        # beta = alphas.k + sum qd.k - 1/2 y.y : accumulate each read's cotangent
        d_alphas[k] += w.sum()
        d_qd[k] += w.sum()                            # from sum_d qd[k, d]
        wy = w[:, None] * y                           # cotangent of y is -w y
        dQ = -(wy.T @ r)                              # y = Q r  =>  dQ += ct_y r^T
        d_means[k] += Q.T @ wy.sum(axis=0)            # r = x - means.k, ct_r = Q^T ct_y
        d_qd[k] += np.diag(dQ) * np.exp(qd[k])        # Q[d, d] = exp(qd[k, d])
        for a in range(1, D):
            for b in range(a):
                d_l[k, lower_index(a, b)] += dQ[a, b]
    # - N * logsumexp(alphas): its transpose adds -ct * N * softmax(alphas)
    sm = np.exp(alphas - logsumexp(alphas))
    d_alphas -= ct * N * sm
    return d_alphas, d_means, d_qd, d_l


def jvp(alphas, means, qd, l, x, t, f=None) -> float:
    """Forward mode: the derivative of F along the tangent t = (dalphas, dmeans,
    dqd, dl), written as the linearized loop (Sec. 5.1): for each component k,
    Q = build_Q(qd.k, l.k) has tangent dQ (diagonal exp(qd) dqd, strict lower
    part dl), y = Q r with r = x - mean.k has tangent dy = dQ r - Q dmean.k,
    beta.k = alpha.k + sum qd.k - 1/2 y.y has tangent
    dbeta = dalpha.k + sum dqd.k - y.dy, and the log-sum-exp over k passes on
    the softmax weights exp(beta - f); the last term of F contributes
    -N softmax(alphas).dalphas."""
    alphas, means, qd, l, x = _f64(alphas, means, qd, l, x)
    da, dm, dq, dl = (np.asarray(a, dtype=np.float64) for a in t)
    N, D = x.shape
    K = alphas.shape[0]
    if f is None:
        _, f = objective(alphas, means, qd, l, x)
    f = np.asarray(f, dtype=np.float64)
    dF = 0.0
    for k in range(K):
        Q = build_Q(qd[k], l[k])
        # strict lower part dl (build_Q with qd = 0 puts ones on the diagonal)
        dQ = build_Q(np.zeros(D), dl[k]) - np.eye(D) + np.diag(np.exp(qd[k]) * dq[k])
        r = x - means[k]
        y = r @ Q.T
        dy = r @ dQ.T - Q @ dm[k]
        bk = alphas[k] + qd[k].sum() - 0.5 * np.sum(y * y, axis=1)
        dbk = da[k] + dq[k].sum() - np.sum(y * dy, axis=1)
        dF += float(np.sum(np.exp(bk - f) * dbk))
    sm = np.exp(alphas - logsumexp(alphas))
    return dF - N * float(np.dot(sm, da))


def suff_stats(alphas, means, qd, l, x, f, ct: float = 1.0, ks=None):
    """Per-component weighted sums behind the gradient, for sampled checks:
    A_k = sum_i w_ik, b_k = sum_i w_ik y_ik, M_k = sum_i w_ik y_ik r_ik^T."""
    alphas, means, qd, l, x = _f64(alphas, means, qd, l, x)
    f = np.asarray(f, dtype=np.float64)
    ks = range(alphas.shape[0]) if ks is None else ks
    out = {}
    for k in ks:
        Q = build_Q(qd[k], l[k])
        r = x - means[k]
        y = r @ Q.T
        bk = alphas[k] + qd[k].sum() - 0.5 * np.sum(y * y, axis=1)
        w = ct * np.exp(bk - f)
        out[k] = (w.sum(), (w[:, None] * y).sum(0), (w[:, None] * y).T @ r)
    return out
