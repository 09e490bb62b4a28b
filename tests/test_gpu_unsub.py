"""GPU parity of the equations without singularity subtraction (Example 2's
comparison) against the oracle: the operators GNK_OP_FB_U and GNK_OP_GB_U,
and gnk_fbie / gnk_fbie_ad with no_subtraction = 1.

Tolerances as in test_gpu_parity.py: products 1e-12, solves 1e-10 relative
L-infinity (error / max(|ref|, |gamma|))."""
import numpy as np
import pytest
import torch

import workloads as wl
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


def _dense(d):
    N = d.eta.shape[0]
    B = orc.kernel_matrix(d.eta, d.etap, d.A, d.n).imag
    nd = orc.n_diagonal(d.etap, d.etapp, d.A, d.Ap, d.n)
    P = orc.block_diag_repeat(np.full((d.n, d.n), 1.0 / d.n), d.m1)
    return np.eye(N) - B - np.diag(nd), np.eye(N) + B.T + np.diag(nd) + P


def _domains():
    return [("ex2-eps0.05", wl.example2_circles(64, 0.05)),
            ("annulus", wl.annulus(96)),
            ("unbounded", wl.circles_unbounded(64, [0.0, 2.5, -1.0 + 2.0j], [1.0, 0.6, 0.4]))]


@pytest.mark.parametrize("name,dom", _domains(), ids=lambda v: v if isinstance(v, str) else "")
def test_operators_without_subtraction(gk, ctx, name, dom):
    print(f"[unsub] operators {name}", flush=True)
    FBu, GBu = _dense(dom)
    rng = np.random.default_rng([wl.SEED, 81, dom.eta.shape[0]])
    x = rng.normal(size=(dom.eta.shape[0], 3))
    dd = gk.DeviceDomain.from_host(dom)
    for op, M in ((gk.OP_FB_U, FBu), (gk.OP_GB_U, GBu)):
        y = ctx.apply(dd, op, _cuda(x)).cpu().numpy()
        ref = M @ x
        assert np.max(np.abs(y - ref)) < 1e-12 * np.max(np.abs(ref)), op


@pytest.mark.parametrize("name,dom", _domains(), ids=lambda v: v if isinstance(v, str) else "")
def test_fbie_without_subtraction_matches_oracle(gk, ctx, name, dom):
    print(f"[unsub] fbie {name}", flush=True)
    f = (lambda z: 1.0 / (z - 2.0) + np.sin(z)) if dom.bounded else (lambda z: 1.0 / (z - 0.1) + 0.3 / z ** 2)
    gam, _ = wl.closed_form_rhs(dom, f)
    mu_r, h_r = orc.fbie_unsubtracted(dom.eta, dom.etap, dom.etapp, dom.A, dom.Ap, gam, dom.n)
    dd = gk.DeviceDomain.from_host(dom)
    mu, h, infos, st = ctx.fbie(dd, _cuda(gam), restart=40, maxit=40, tol=1e-13, subtract=False)
    assert st == gk.OK, infos
    s = max(np.max(np.abs(mu_r)), np.max(np.abs(gam)))
    assert np.max(np.abs(mu.cpu().numpy() - mu_r)) / s < 1e-10
    assert np.max(np.abs(h.cpu().numpy() - h_r)) / s < 1e-10


@pytest.mark.parametrize("name,dom", _domains(), ids=lambda v: v if isinstance(v, str) else "")
def test_fbiead_without_subtraction_matches_oracle(gk, ctx, name, dom):
    print(f"[unsub] fbiead {name}", flush=True)
    rng = np.random.default_rng([wl.SEED, 82])
    gam = np.cos(2 * np.angle(dom.eta)) + 0.1 * rng.normal(size=dom.eta.shape[0])
    mu_r = orc.fbiead_unsubtracted(dom.eta, dom.etap, dom.etapp, dom.A, dom.Ap, gam, dom.n)
    dd = gk.DeviceDomain.from_host(dom)
    mu, infos, st = ctx.fbie_ad(dd, _cuda(gam), restart=40, maxit=40, tol=1e-13, subtract=False)
    assert st == gk.OK, infos
    s = max(np.max(np.abs(mu_r)), np.max(np.abs(gam)))
    assert np.max(np.abs(mu.cpu().numpy() - mu_r)) / s < 1e-10


def test_example2_effect_on_the_gpu(gk, ctx):
    # the paper's observation: with close circles the subtracted solve stays exact,
    # the plain trapezoidal rule does not
    dom = wl.example2_circles(128, 0.01)
    gam, mu_ex = wl.closed_form_rhs(dom, lambda z: 1.0 / (z - 2.0) + np.sin(z))
    dd = gk.DeviceDomain.from_host(dom)
    mu_s, _, _, st_s = ctx.fbie(dd, _cuda(gam), restart=40, maxit=40, tol=1e-13)
    mu_u, _, _, st_u = ctx.fbie(dd, _cuda(gam), restart=40, maxit=40, tol=1e-13, subtract=False)
    assert st_s == gk.OK and st_u == gk.OK
    assert np.max(np.abs(mu_s.cpu().numpy() - mu_ex)) < 1e-11
    assert np.max(np.abs(mu_u.cpu().numpy() - mu_ex)) > 1e-2


def test_no_subtraction_argument_errors(gk, ctx):
    dom = wl.annulus(32)
    gam, _ = wl.closed_form_rhs(dom, lambda z: z)
    no2 = gk.DeviceDomain(dom.m1, dom.n, _cuda(dom.eta), _cuda(dom.etap), _cuda(dom.A))
    with pytest.raises(gk.GnkError) as e:
        ctx.fbie(no2, _cuda(gam), subtract=False)
    assert e.value.status == gk.ERR_ARG
    dd = gk.DeviceDomain.from_host(dom)
    with pytest.raises(gk.GnkError) as e:
        ctx.fbie_batched([dd], [_cuda(gam[:, None])], subtract=False)
    assert e.value.status == gk.ERR_ARG
    # the subtracted solve still works afterwards
    mu, h, infos, st = ctx.fbie(dd, _cuda(gam))
    assert st == gk.OK
