"""torch.autograd.Function wrappers over the C ABI.

Each forward calls dex_fwd (the primal half of `linearize`, Sec. 5.1) and keeps
the residuals it returns; each backward calls dex_vjp (`transpose` of the
linear map applied to the output cotangent, Sec. 5.2). No arithmetic of the
path happens in PyTorch.
"""
from __future__ import annotations

import torch

from . import dex


def _ws(d, role, device):
    return dex.workspace(dex.dex_workspace_bytes(d, role), device)


class GMMLogLik(torch.autograd.Function):
    """F = sum_i logsumexp_k beta[i,k] - N logsumexp(alphas) (see include/dex.h).

    Inputs alphas [K], means [K,D], qd [K,D], l [K, D(D-1)/2], x [N,D]; all FP32
    or all FP64. `variant` is dex.DEX_GMM_PLAIN / DEX_GMM_BF16 / DEX_GMM_BF16X3.
    Returns a 0-d tensor. x gets no gradient.
    """

    @staticmethod
    def forward(ctx, alphas, means, qd, l, x, variant=dex.DEX_GMM_BF16, config=0):
        N, D = x.shape
        K = alphas.shape[0]
        dt = dex.dtype_code(x)
        d = dex.gmm_desc(N, D, K, dt, variant, config)
        dev = x.device
        F = torch.empty(1, dtype=x.dtype, device=dev)
        f = torch.empty(N, dtype=x.dtype, device=dev)
        cache = torch.empty(max(1, dex.dex_workspace_bytes(d, dex.DEX_WS_RESID)), dtype=torch.uint8,
                            device=dev)
        cache_v = cache[: dex.dex_workspace_bytes(d, dex.DEX_WS_RESID)]
        ins = [t.contiguous() for t in (alphas, means, qd, l, x)]
        dex.dex_fwd(d, ins, [F], [f, cache_v], _ws(d, dex.DEX_WS_FWD, dev))
        ctx.save_for_backward(*ins, f, cache_v)
        ctx.d = d
        return F.reshape(())

    @staticmethod
    def backward(ctx, dF):
        alphas, means, qd, l, x, f, cache = ctx.saved_tensors
        d = ctx.d
        ct = dF.reshape(1).to(x.dtype).contiguous()
        grads = [torch.empty_like(t) for t in (alphas, means, qd, l)]
        dex.dex_vjp(d, [alphas, means, qd, l, x], [f, cache], [ct], grads, 0,
                    _ws(d, dex.DEX_WS_VJP, x.device))
        return (*grads, None, None, None)


class GatherScale(torch.autograd.Function):
    """out[j,:] = w[j] * T[idx[j],:]; backward: dT by scatter-accumulate, dw by dot products."""

    @staticmethod
    def forward(ctx, T, idx, w):
        V, R = T.shape
        n = idx.shape[0]
        d = dex.gather_desc(V, R, n)
        out = torch.empty(n, R, dtype=T.dtype, device=T.device)
        ins = [T.contiguous(), idx.contiguous(), w.contiguous()]
        dex.dex_fwd(d, ins, [out], [])
        ctx.save_for_backward(*ins)
        ctx.d = d
        return out

    @staticmethod
    def backward(ctx, g):
        T, idx, w = ctx.saved_tensors
        dT = torch.empty_like(T)
        want_dw = ctx.needs_input_grad[2]
        dw = torch.empty_like(w) if want_dw else None
        flags = 0 if want_dw else dex.DEX_NO_DW
        dex.dex_vjp(ctx.d, [T, idx, w], [], [g.contiguous()], [dT, dw], flags,
                    _ws(ctx.d, dex.DEX_WS_VJP, T.device))
        return dT, None, dw


class Diffusion(torch.autograd.Function):
    """L = 1/2 ||u_T - target||^2 after `steps` in-place diffusion steps.

    Checkpoints every `every` steps; with variant DEX_STENCIL_RECOMPUTE the
    reverse pass rebuilds each segment from its checkpoint. Returns (L, u_T);
    only L carries a gradient (to u0).
    """

    @staticmethod
    def forward(ctx, u0, target, steps, every=32, c=0.2, rho=0.0,
                variant=dex.DEX_STENCIL_RECOMPUTE, config=0):
        H, W = u0.shape
        d = dex.stencil_desc(H, W, steps, every, c, rho, variant, config)
        dev = u0.device
        nck = (steps + every - 1) // every
        L = torch.empty(1, dtype=torch.float32, device=dev)
        uT = torch.empty_like(u0)
        ck = torch.empty(max(nck, 0) * H * W, dtype=torch.float32, device=dev)
        u0c, tc = u0.contiguous(), target.contiguous()
        dex.dex_fwd(d, [u0c, tc], [L, uT], [ck, uT], _ws(d, dex.DEX_WS_FWD, dev))
        ctx.save_for_backward(u0c, tc, ck, uT)
        ctx.d = d
        ctx.mark_non_differentiable(uT)
        return L.reshape(()), uT

    @staticmethod
    def backward(ctx, dL, duT):
        u0, target, ck, uT = ctx.saved_tensors
        du0 = torch.empty_like(u0)
        ct = dL.reshape(1).contiguous()
        dex.dex_vjp(ctx.d, [u0, target], [ck, uT], [ct], [du0], 0,
                    _ws(ctx.d, dex.DEX_WS_VJP, u0.device))
        return du0, None, None, None, None, None, None, None


def gmm_loglik(alphas, means, qd, l, x, variant=dex.DEX_GMM_BF16, config=0):
    return GMMLogLik.apply(alphas, means, qd, l, x, variant, config)


def gather_scale(T, idx, w):
    return GatherScale.apply(T, idx, w)


def diffusion_loss(u0, target, steps, every=32, c=0.2, rho=0.0,
                   variant=dex.DEX_STENCIL_RECOMPUTE, config=0):
    return Diffusion.apply(u0, target, steps, every, c, rho, variant, config)


def histogram(keys: torch.Tensor, bins: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """int32 counts of keys in [0, bins), accumulated into `out` (zeros if None)."""
    h = torch.zeros(bins, dtype=torch.int32, device=keys.device) if out is None else out
    idt = dex.DEX_U32 if keys.dtype != torch.int32 else dex.DEX_I32
    dex.dex_accum_scatter(h, keys, idx_dtype=idt)
    return h


def accum_scatter(acc, idx, vals=None, scale=None, check_bounds=False):
    """acc!(idx[j]) += scale[j] * vals[j], in place. Returns the number of
    out-of-range indices when check_bounds is set (synchronises)."""
    if check_bounds:
        oob = torch.zeros(1, dtype=torch.int64, device=acc.device)
        dex.dex_accum_scatter(acc, idx, vals, scale, dex.DEX_CHECK_BOUNDS, oob)
        return int(oob.item())
    dex.dex_accum_scatter(acc, idx, vals, scale)
    return None
