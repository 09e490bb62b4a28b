"""Full-size parity of the large workloads against the oracle's stored
solutions (matrix-free FP64 route, tests/golden/make_golden_large.py), element
by element: the close-boundary workload (N = 133120) in FP64 and in mixed
precision, the perturbed-circles workload (N = 264192) forward and its
gradient, and every domain of the 64-domain batched workload (sampled rows of
every stored column), FP64 and mixed. Bar: relative L-infinity 1e-10 on mu and
h (reading: max|x - x_oracle| / max(max|x_oracle|, max|gamma|)), 1e-8 on the
gradient."""
import os

import numpy as np
import pytest
import torch

import workloads as wl

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    path = os.path.join(GOLDEN, f"{name}_oracle.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written")
    return np.load(path)


@pytest.fixture(scope="module")
def gk():
    from paper_1308_5351_amd import gnk
    assert torch.cuda.is_available()
    return gnk


@pytest.fixture(scope="module")
def ctx(gk):
    c = gk.Context(0)
    yield c
    c.close()


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _rel(x, ref, s):
    return float(np.max(np.abs(x - ref)) / max(float(np.max(np.abs(ref))), s))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_close_boundaries_full_size(gk, ctx, prec):
    """65 close boundaries (gaps 1e-3..1e-2 of size, Kress-graded corners), n = 2048."""
    z = _golden("cfg2")
    dom, gam = wl.config2()
    g = gam[:, 0]
    dd = gk.DeviceDomain.from_host(dom)
    p = gk.MIXED if prec == "mixed" else gk.FP64
    print(f"[golden] close boundaries N={dom.N} {prec}", flush=True)
    mu, h, infos, st = ctx.fbie(dd, _cuda(g), tol=1e-14, restart=256, maxit=8, prec=p)
    s = float(np.max(np.abs(g)))
    e_mu, e_h = _rel(mu.cpu().numpy(), z["mu"], s), _rel(h.cpu().numpy(), z["h"], s)
    print(f"  {infos[0]}\n  err mu {e_mu:.2e} h {e_h:.2e} (oracle relres {float(z['relres'][0]):.1e})", flush=True)
    assert st == 0 and e_mu < 1e-10 and e_h < 1e-10


def test_perturbed_circles_forward(gk, ctx):
    """129 perturbed circles, n = 2048: FP64 FBIE as the benchmark runs it."""
    z = _golden("cfg4")
    dom, gam = wl.config4()
    g = gam[:, 0]
    dd = gk.DeviceDomain.from_host(dom)
    print(f"[golden] perturbed circles N={dom.N}", flush=True)
    mu, h, infos, st = ctx.fbie(dd, _cuda(g), tol=1e-13, restart=60, maxit=10)
    s = float(np.max(np.abs(g)))
    e_mu, e_h = _rel(mu.cpu().numpy(), z["mu"], s), _rel(h.cpu().numpy(), z["h"], s)
    print(f"  {infos[0]}\n  err mu {e_mu:.2e} h {e_h:.2e}", flush=True)
    assert st == 0 and e_mu < 1e-10 and e_h < 1e-10


def test_perturbed_circles_gradient(gk, ctx):
    """L = sum_k h_k^2 through the autograd wrapper (Fourier curves -> FBIE ->
    adjoint GMRES -> geometric pass -> chain rule): the loss, dL/dgamma on every
    node and dL/dcoef of the oracle's four components against the oracle's
    reverse-mode gradient (matrix-free adjoint solve, geometric rows from the
    kernel derivatives)."""
    z = _golden("cfg4")
    if "g_coef" not in z.files:
        pytest.skip("gradient not written")
    from paper_1308_5351_amd import autograd as ag
    dom, gam = wl.config4()
    coeffs, kmin = dom.meta["coeffs"], dom.meta["kmin"]
    coef = _cuda(coeffs).requires_grad_(True)
    g = _cuda(gam[:, 0]).requires_grad_(True)
    print("[golden] gradient N=264192", flush=True)
    eta, etap, _ = ag.fourier_curve(coef, kmin, dom.n, context=ctx)
    _, h = ag.fbie(eta, etap, torch.ones_like(eta), g, dom.m1, dom.n, context=ctx, tol=1e-13, restart=60,
                   maxit=10)
    L = (h.view(dom.m1, dom.n).mean(1) ** 2).sum()
    L.backward()
    comps = z["g_coef_components"]
    gc = coef.grad.cpu().numpy()[comps]
    e_c = float(np.max(np.abs(gc - z["g_coef"])) / np.max(np.abs(z["g_coef"])))
    e_g = float(np.max(np.abs(g.grad.cpu().numpy() - z["g_gam"])) / np.max(np.abs(z["g_gam"])))
    e_L = abs(L.item() - float(z["loss"])) / abs(float(z["loss"]))
    print(f"  loss {L.item():.6e} rel {e_L:.2e}; dL/dcoef rel {e_c:.2e}; dL/dgamma rel {e_g:.2e}", flush=True)
    assert e_L < 1e-9 and e_c < 1e-8 and e_g < 1e-8


@pytest.fixture(scope="module")
def batch():
    return wl.config3()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batched_every_domain(gk, ctx, batch, prec):
    """The 64-domain batched workload in one call (FP64: restart 50; mixed: every
    Arnoldi product mixed, FP64 residual per restart of 10, as the benchmark runs
    it): for every domain, every stored column's mu and h on the oracle's sampled
    rows, and the component means of h."""
    z = _golden("cfg3")
    if f"d{len(batch) - 1}_cols" not in z.files:
        pytest.skip("the batched golden file holds only some of the domains")
    doms = [gk.DeviceDomain.from_host(d) for d, _ in batch]
    gams = [_cuda(g) for _, g in batch]
    if prec == "fp64":
        kw = dict(restart=50, maxit=20, tol=1e-13)
    else:
        kw = dict(restart=10, maxit=40, tol=1e-13, prec=gk.MIXED, inner_tol=1.0)
    print(f"[golden] batched {prec}", flush=True)
    mus, hs, infos, st = ctx.fbie_batched(doms, gams, **kw)
    assert st == 0
    worst = (0.0, None)
    ncols = 0
    for d, ((dom, gam), mu, h) in enumerate(zip(batch, mus, hs)):
        cols, rows = z[f"d{d}_cols"], z[f"d{d}_rows"]
        M = mu.cpu().numpy()
        H = h.cpu().numpy()
        M = M[:, None] if M.ndim == 1 else M
        H = H[:, None] if H.ndim == 1 else H
        for k, c in enumerate(cols):
            s = float(z[f"d{d}_gam_max"][k])
            e_mu = float(np.max(np.abs(M[rows, c] - z[f"d{d}_mu"][:, k]))) / max(float(z[f"d{d}_mu_max"][k]), s)
            e_h = float(np.max(np.abs(H[rows, c] - z[f"d{d}_h"][:, k]))) / max(float(z[f"d{d}_h_max"][k]), s)
            hk = H[:, c].reshape(dom.m1, dom.n).mean(axis=1)
            e_hk = float(np.max(np.abs(hk - z[f"d{d}_hk"][:, k]))) / max(float(z[f"d{d}_h_max"][k]), s)
            e = max(e_mu, e_h, e_hk)
            if e > worst[0]:
                worst = (e, (d, int(c), str(z[f"d{d}_route"])))
            ncols += 1
    print(f"  {ncols} columns of 64 domains; worst rel err {worst[0]:.2e} at {worst[1]}", flush=True)
    assert worst[0] < 1e-10
