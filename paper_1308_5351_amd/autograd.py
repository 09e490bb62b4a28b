"""torch.autograd Functions over libgnk: FBIE with reverse-mode derivatives with
respect to the right-hand side gamma and the boundary data (eta, eta', A), and
Fourier boundary curves with the chain rule to their coefficients.

Every forward and backward step runs in the HIP library (GMRES, the transposed
products of the adjoint solve, the geometric Cauchy sums, the Fourier sums);
this module only passes tensors and cotangents through. Complex gradients
follow torch's convention (dL/dRe z + i dL/dIm z).

Example (gradient of L = sum_k h_k^2 with respect to Fourier coefficients):

    eta, etap, _ = fourier_curve(coef, kmin, n)                 # coef.requires_grad
    mu, h = fbie(eta, etap, torch.ones_like(eta), gam, m1, n)
    loss = (h.view(m1, n).mean(1) ** 2).sum(); loss.backward()    # coef.grad
"""
from __future__ import annotations

from typing import Optional

import torch

from . import gnk

_CTX: dict = {}


def default_context(device: Optional[int] = None) -> gnk.Context:
    dev = torch.cuda.current_device() if device is None else device
    if dev not in _CTX:
        _CTX[dev] = gnk.Context(dev)
    return _CTX[dev]


class FourierCurve(torch.autograd.Function):
    """(coef) -> (eta, eta', eta''), eta_j(t_p) = sum_k coef[j, k - kmin] e^{i s k t_p}."""

    @staticmethod
    def forward(ctx, coef, kmin, n, ccw, gctx):
        ctx.set_materialize_grads(False)
        ctx.meta = (coef.shape[0], coef.shape[1], kmin, n, ccw, gctx)
        return gctx.fourier_curve(coef.detach(), kmin, n, ccw)

    @staticmethod
    def backward(ctx, g_eta, g_etap, g_etapp):
        m1, nk, kmin, n, ccw, gctx = ctx.meta
        if g_eta is None and g_etap is None and g_etapp is None:
            return None, None, None, None, None
        g = gctx.fourier_vjp(g_eta, g_etap, g_etapp, m1, nk, kmin, n, ccw)
        return g, None, None, None, None


class FBIESolve(torch.autograd.Function):
    """(eta, eta', A, gamma) -> (mu, h) of (I - N) mu = -M gamma, h = [M mu - (I - N) gamma]/2.

    Backward: one adjoint GMRES solve for all columns (lam and dL/dgamma), then
    one geometric pass over the four bilinear terms per column
    (g_h/2)^T dCop mu - (g_h/2)^T dAop gamma - lam^T dAop mu - lam^T dCop gamma."""

    @staticmethod
    def forward(ctx, eta, etap, A, gam, m1, n, opts, gctx):
        ctx.set_materialize_grads(False)
        dom = gnk.DeviceDomain(m1, n, eta.detach().contiguous(), etap.detach().contiguous(),
                               A.detach().contiguous())
        mu, h, infos, st = gctx.fbie(dom, gam.detach(), **opts)
        if st != gnk.OK:
            raise gnk.GnkError(st, f"FBIE did not converge: {infos}")
        ctx.dom, ctx.opts, ctx.gctx = dom, opts, gctx
        ctx.save_for_backward(gam, mu)
        return mu, h

    @staticmethod
    def backward(ctx, g_mu, g_h):
        gam, mu = ctx.saved_tensors
        dom, opts, gctx = ctx.dom, ctx.opts, ctx.gctx
        if g_mu is None and g_h is None:
            return (None,) * 8
        o = dict(opts)
        lam, g_gam, infos, st = gctx.fbie_adjoint(dom, g_mu, g_h, **o)
        if st != gnk.OK:
            raise gnk.GnkError(st, f"adjoint GMRES did not converge: {infos}")
        need_geom = any(ctx.needs_input_grad[:3])
        g_eta = g_etap = g_A = None
        if need_geom:
            cols = lambda x: x.unsqueeze(1) if x.dim() == 1 else x
            L, M, G = cols(lam).t().contiguous(), cols(mu).t().contiguous(), cols(gam).t().contiguous()
            H = cols(g_h).t().contiguous() if g_h is not None else None
            terms = []
            for r in range(L.shape[0]):
                if H is not None:
                    terms += [(gnk.OP_FC, 0.5, H[r], M[r]), (gnk.OP_FB, -0.5, H[r], G[r])]
                terms += [(gnk.OP_FB, -1.0, L[r], M[r]), (gnk.OP_FC, -1.0, L[r], G[r])]
            want = tuple(bool(x) for x in ctx.needs_input_grad[:3])
            g_eta, g_etap, g_A = gctx.geom_vjp(dom, terms, want)
        return g_eta, g_etap, g_A, (g_gam if ctx.needs_input_grad[3] else None), None, None, None, None


def fourier_curve(coef: torch.Tensor, kmin: int, n: int, ccw: bool = False, context: Optional[gnk.Context] = None):
    gctx = context or default_context(coef.device.index)
    return FourierCurve.apply(coef, kmin, n, ccw, gctx)


_SOLVE_OPTS = ("restart", "maxit", "tol", "prec", "inner_tol", "max_refine")


def fbie(eta, etap, A, gam, m1: int, n: int, context: Optional[gnk.Context] = None, **opts):
    """Differentiable FBIE; opts: restart, maxit, tol, prec, inner_tol, max_refine
    (as Context.fbie). The forward and the adjoint solve use the same options.
    Options that change the discrete map (far_tol > 0: the treecode's truncated
    sums; subtract=False: the equation without singularity subtraction) have no
    matching adjoint and are rejected."""
    bad = sorted(k for k in opts if k not in _SOLVE_OPTS)
    if bad:
        raise ValueError(f"autograd.fbie does not take {bad}: only {list(_SOLVE_OPTS)} (the adjoint solve "
                         "differentiates the FBIE map with directly summed products and singularity subtraction)")
    gctx = context or default_context(eta.device.index)
    return FBIESolve.apply(eta, etap, A, gam, m1, n, opts, gctx)
