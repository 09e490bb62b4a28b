"""GPU parity of the differentiation path (adjoint GMRES, geometric Cauchy
sums, Fourier chain rule, autograd Functions) against the gradient oracle, and
central finite differences of the GPU forward solve at the full
perturbed-circles size (129 curves x 16 Fourier coefficients, n = 2048).

Tolerances: operator-level results (no solve) to 1e-11 relative L-infinity;
results through a GMRES solve at tol 1e-13 to 1e-8 relative (the CPU
reference-gradient bar); finite differences of solves at step 1e-6 to 2e-5
relative to the largest gradient entry (their own noise is about
kappa * tol / step plus O(step^2))."""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import gradient as og
from oracle import nystrom as orc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gk():
    from paper_1308_5351_amd import gnk
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return gnk


@pytest.fixture(scope="module")
def ctx(gk):
    c = gk.Context(0)
    yield c
    c.close()


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _rel(x, ref):
    return float(np.max(np.abs(np.asarray(x) - ref)) / np.max(np.abs(ref)))


def _reduced(m1=9, n=256, seed=0):
    coeffs, kmin = wl.fourier_perturbed_circles(m1, n, [wl.SEED, 41, seed], side=4.0, dmin=1.0)
    return coeffs, kmin, n


def _dev_domain(gk, eta, etap, A, m1, n):
    return gk.DeviceDomain(m1, n, _cuda(eta), _cuda(etap), _cuda(A))


# ------------------------------------------------------------ Fourier curves
def test_fourier_curve_and_vjp_match_oracle(ctx):
    print("[grad] fourier curve m1=9 n=256", flush=True)
    coeffs, kmin, n = _reduced()
    e, ep, epp = ctx.fourier_curve(_cuda(coeffs), kmin, n)
    re, rep, repp = og.fourier_nodes(coeffs, kmin, n)
    assert _rel(e.cpu().numpy(), re) < 1e-13
    assert _rel(ep.cpu().numpy(), rep) < 1e-13
    assert _rel(epp.cpu().numpy(), repp) < 1e-13
    ccw = og.fourier_nodes(coeffs, kmin, n, ccw=True)[1]
    assert _rel(ctx.fourier_curve(_cuda(coeffs), kmin, n, ccw=True)[1].cpu().numpy(), ccw) < 1e-13
    rng = np.random.default_rng(5)
    N = coeffs.shape[0] * n
    gs = [rng.normal(size=N) + 1j * rng.normal(size=N) for _ in range(3)]
    g = ctx.fourier_vjp(*[_cuda(x) for x in gs], coeffs.shape[0], coeffs.shape[1], kmin, n)
    ref = og.fourier_coef_grad(*gs, kmin, coeffs.shape[1], n)
    assert _rel(g.cpu().numpy(), ref) < 1e-12
    g2 = ctx.fourier_vjp(_cuda(gs[0]), None, None, coeffs.shape[0], coeffs.shape[1], kmin, n)
    assert _rel(g2.cpu().numpy(), og.fourier_coef_grad(gs[0], None, None, kmin, coeffs.shape[1], n)) < 1e-12


# ------------------------------------------------------- geometric gradients
@pytest.mark.parametrize("m1,n", [(9, 256), (3, 70), (1, 64)])
def test_geom_vjp_matches_oracle(gk, ctx, m1, n):
    print(f"[grad] geom_vjp m1={m1} n={n}", flush=True)
    coeffs, kmin, _ = _reduced(m1, n, seed=m1)
    eta, etap, _ = og.fourier_nodes(coeffs, kmin, n)
    rng = np.random.default_rng([m1, n])
    N = eta.shape[0]
    A = 1.0 + 0.3 * (rng.normal(size=N) + 1j * rng.normal(size=N))
    v1, v2 = rng.normal(size=N), rng.normal(size=N)
    u = [rng.normal(size=N) for _ in range(4)]
    terms_np = [("FB", 0.7, u[0], v1), ("FC", -1.3, u[1], v2), ("FC", 0.5, u[2], v1), ("FB", 2.0, u[3], v2)]
    ref = og.bilinear_geom_grad(eta, etap, A, n, [(op, c * uu, vv) for op, c, uu, vv in terms_np])
    dom = _dev_domain(gk, eta, etap, A, m1, n)
    V1, V2 = _cuda(v1), _cuda(v2)          # shared v pointers form groups
    U = [_cuda(x) for x in u]
    opmap = {"FB": gk.OP_FB, "FC": gk.OP_FC}
    terms = [(opmap[op], c, U[k], V1 if vv is v1 else V2) for k, (op, c, _, vv) in enumerate(terms_np)]
    got = ctx.geom_vjp(dom, terms)
    for name, gg, rr in zip(("eta", "etap", "A"), got, ref):
        err = _rel(gg.cpu().numpy(), rr)
        print(f"  g_{name} rel err {err:.2e}", flush=True)
        assert err < 1e-11
    # only some outputs
    g_only = ctx.geom_vjp(dom, terms, want=(False, True, False))
    assert g_only[0] is None and g_only[2] is None
    assert torch.equal(g_only[1], got[1])


def test_geom_vjp_full_size_sampled(gk, ctx):
    """129 perturbed circles, n = 2048 (N = 264,192): sampled entries against
    the oracle's row-and-column evaluation."""
    print("[grad] geom_vjp full size", flush=True)
    dom_h, _ = wl.config4()
    N = dom_h.N
    rng = np.random.default_rng(11)
    u1, u2, v1, v2 = (rng.normal(size=N) for _ in range(4))
    terms_np = [("FB", 1.0, u1, v1), ("FC", 1.0, u2, v2)]
    dom = gk.DeviceDomain.from_host(dom_h)
    terms = [(gk.OP_FB, 1.0, _cuda(u1), _cuda(v1)), (gk.OP_FC, 1.0, _cuda(u2), _cuda(v2))]
    got = [g.cpu().numpy() for g in ctx.geom_vjp(dom, terms)]
    idx = np.concatenate([[0, 1, 2047, 2048, N - 1], rng.choice(N, 19, replace=False)])
    ref = og.bilinear_geom_grad_rows(dom_h.eta, dom_h.etap, dom_h.A, dom_h.n,
                                     [(op, u, v) for op, _, u, v in terms_np], idx)
    for gg, rr in zip(got, ref):
        err = float(np.max(np.abs(gg[idx] - rr)) / np.max(np.abs(rr)))
        assert err < 1e-10, err


# ------------------------------------------------------------- adjoint solve
def test_fbie_adjoint_matches_oracle(gk, ctx):
    print("[grad] adjoint solve m1=9 n=256", flush=True)
    coeffs, kmin, n = _reduced()
    eta, etap, _ = og.fourier_nodes(coeffs, kmin, n)
    A = np.ones_like(eta)
    N = eta.shape[0]
    rng = np.random.default_rng(2)
    gam = (eta ** 2).real
    g_mu, g_h = rng.normal(size=N), rng.normal(size=N)
    ref = og.fbie_vjp(eta, etap, A, gam, n, g_mu=g_mu, g_h=g_h)
    dom = _dev_domain(gk, eta, etap, A, coeffs.shape[0], n)
    lam, g_gam, infos, st = ctx.fbie_adjoint(dom, _cuda(g_mu), _cuda(g_h), tol=1e-13, restart=50)
    assert st == gk.OK and infos[0]["flag"] == 0
    assert _rel(lam.cpu().numpy(), ref["lam"]) < 1e-9
    assert _rel(g_gam.cpu().numpy(), ref["g_gam"]) < 1e-9
    # only g_h, and two columns at once
    G = np.stack([g_h, -2.0 * g_mu], 1)
    lam2, g_gam2, _, st = ctx.fbie_adjoint(dom, None, _cuda(G), tol=1e-13, restart=50)
    assert st == gk.OK
    for r in range(2):
        rr = og.fbie_vjp(eta, etap, A, gam, n, g_h=G[:, r])
        assert _rel(lam2[:, r].cpu().numpy(), rr["lam"]) < 1e-9
        assert _rel(g_gam2[:, r].cpu().numpy(), rr["g_gam"]) < 1e-9


def test_fbie_adjoint_errors(gk, ctx):
    coeffs, kmin, n = _reduced(2, 64)
    eta, etap, _ = og.fourier_nodes(coeffs, kmin, n)
    dom = _dev_domain(gk, eta, etap, np.ones_like(eta), 2, n)
    with pytest.raises(ValueError):
        ctx.fbie_adjoint(dom, None, None)
    bad = torch.full((eta.shape[0],), float("nan"), dtype=torch.float64, device="cuda")
    with pytest.raises(gk.GnkError) as e:
        ctx.fbie_adjoint(dom, bad, None)
    assert e.value.status == gk.ERR_NONFINITE


# ------------------------------------------------------------------ autograd
def _loss(h, m1, n):
    return (h.reshape(m1, n).mean(dim=1) ** 2).sum()


def test_autograd_matches_oracle_gradient(gk, ctx):
    """L = sum_k h_k^2 through FourierCurve and FBIESolve; dL/dcoef and dL/dgamma
    against the dense CPU reference gradient."""
    print("[grad] autograd vs oracle m1=9 n=256", flush=True)
    from paper_1308_5351_amd import autograd as ga
    coeffs, kmin, n = _reduced()
    m1 = coeffs.shape[0]
    eta0, _, _ = og.fourier_nodes(coeffs, kmin, n)
    gam_np = (eta0 ** 2).real
    L_ref, g_gam_ref, g_c_ref = og.fbie_loss_and_grad(coeffs, kmin, n, gam_np)
    coef = _cuda(coeffs).requires_grad_(True)
    gam = _cuda(gam_np).requires_grad_(True)
    eta, etap, _ = ga.fourier_curve(coef, kmin, n, context=ctx)
    mu, h = ga.fbie(eta, etap, torch.ones_like(eta), gam, m1, n, context=ctx, tol=1e-13, restart=50)
    L = _loss(h, m1, n)
    L.backward()
    assert abs(L.item() - L_ref) <= 1e-9 * L_ref
    e_c = _rel(coef.grad.cpu().numpy(), g_c_ref)
    e_g = _rel(gam.grad.cpu().numpy(), g_gam_ref)
    print(f"  dL/dcoef rel err {e_c:.2e}, dL/dgamma rel err {e_g:.2e}", flush=True)
    assert e_c < 1e-8 and e_g < 1e-8


def test_autograd_mu_cotangent_and_A(gk, ctx):
    """A loss on mu alone, with A a non-constant leaf: dL/dA, dL/deta' against
    the oracle (the g_mu path of the adjoint and the A terms of the geometry)."""
    from paper_1308_5351_amd import autograd as ga
    coeffs, kmin, n = _reduced(4, 128, seed=3)
    m1 = coeffs.shape[0]
    eta_np, etap_np, _ = og.fourier_nodes(coeffs, kmin, n)
    rng = np.random.default_rng(9)
    N = eta_np.shape[0]
    A_np = 1.0 + 0.2 * (rng.normal(size=N) + 1j * rng.normal(size=N))
    gam_np = rng.normal(size=N)
    w = rng.normal(size=N)
    eta = _cuda(eta_np).requires_grad_(True)
    etap = _cuda(etap_np).requires_grad_(True)
    A = _cuda(A_np).requires_grad_(True)
    mu, h = ga.fbie(eta, etap, A, _cuda(gam_np), m1, n, context=ctx, tol=1e-13, restart=60)
    (mu * _cuda(w)).sum().backward()
    ref = og.fbie_vjp(eta_np, etap_np, A_np, gam_np, n, g_mu=w)
    for name, t, r in (("eta", eta, ref["g_eta"]), ("etap", etap, ref["g_etap"]), ("A", A, ref["g_A"])):
        err = _rel(t.grad.cpu().numpy(), r)
        print(f"  g_{name} rel err {err:.2e}", flush=True)
        assert err < 1e-8


def test_autograd_full_size_finite_differences(gk, ctx):
    """129 curves x 16 coefficients, n = 2048: the autograd gradient of
    L = sum_k h_k^2 against central differences of the GPU forward solve on 16
    random coefficients (real and imaginary parts) and 2 random directions."""
    print("[grad] full-size finite differences", flush=True)
    from paper_1308_5351_amd import autograd as ga
    dom_h, gam_h = wl.config4()
    coeffs, kmin = dom_h.meta["coeffs"], dom_h.meta["kmin"]
    m1, n = dom_h.m1, dom_h.n
    gam = _cuda(gam_h[:, 0])
    opts = dict(tol=1e-13, restart=60, maxit=10)

    def loss_of(c):
        eta, etap, _ = ctx.fourier_curve(c, kmin, n)
        dom = gk.DeviceDomain(m1, n, eta, etap, torch.ones_like(eta))
        _, h, infos, st = ctx.fbie(dom, gam, **opts)
        assert st == gk.OK
        return _loss(h, m1, n).item()

    coef = _cuda(coeffs).requires_grad_(True)
    eta, etap, _ = ga.fourier_curve(coef, kmin, n, context=ctx)
    _, h = ga.fbie(eta, etap, torch.ones_like(eta), gam, m1, n, context=ctx, **opts)
    _loss(h, m1, n).backward()
    g = coef.grad.detach()
    scale = g.abs().max().item()
    assert scale > 0
    rng = np.random.default_rng(17)
    base = coef.detach()
    step = 1e-6
    worst = 0.0
    for q in range(16):
        j, k = int(rng.integers(m1)), int(rng.integers(coeffs.shape[1]))
        for part in (1.0, 1j):
            d = torch.zeros_like(base)
            d[j, k] = part * step
            fd = (loss_of(base + d) - loss_of(base - d)) / (2 * step)
            an = g[j, k].real.item() if part == 1.0 else g[j, k].imag.item()
            worst = max(worst, abs(fd - an) / scale)
    for _ in range(2):
        d = torch.from_numpy(rng.normal(size=coeffs.shape) + 1j * rng.normal(size=coeffs.shape)).cuda()
        fd = (loss_of(base + step * d) - loss_of(base - step * d)) / (2 * step)
        an = torch.sum(g.real * d.real + g.imag * d.imag).item()
        worst = max(worst, abs(fd - an) / (scale * d.abs().sum().item()))
    print(f"  worst FD mismatch / max|g| = {worst:.2e}", flush=True)
    assert worst < 2e-5
