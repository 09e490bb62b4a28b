"""Far-field compression (treecode) of the Cauchy sums against the direct sum.

The treecode replaces the sum over a far box b by its p-term expansion about
the box centre, with r_b/|z - c_b| <= rho = 0.4 and p = log(far_tol)/log(rho);
the truncation error of box b is at most rho^p (1 + rho)/(1 - rho) times
sum_{j in b} |w_j|/|z - eta_j|. So per target i

    |S_tree_i - S_i| <= 2.4 far_tol A_i + rounding,   A_i = sum_{j != i} |w_j|/|eta_i - eta_j|,

which is what these tests check (rounding allowance 1e-13 A_i), on dense
sums for moderate N and on sampled rows of the direct sum for large N. Solves
with far_tol = 1e-13 must meet the 1e-10 parity bound against the oracle."""
import os

import numpy as np
import pytest
import torch

import workloads as wl
from oracle import nystrom as orc

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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


def _direct_rows(eta, w, rows):
    """S_i and A_i for the given rows (direct sums, FP64)."""
    d = eta[rows][:, None] - eta[None, :]
    d[np.arange(rows.shape[0]), rows] = 1.0
    inv = 1.0 / d
    inv[np.arange(rows.shape[0]), rows] = 0.0
    return inv @ w, np.abs(inv) @ np.abs(w)


def _check(got, S, A, far_tol):
    err = np.abs(got - S)
    bound = (2.4 * far_tol + 1e-13) * A
    assert np.all(err <= bound), float(np.max(err / bound))


@pytest.mark.parametrize("far_tol", [1e-6, 1e-10, 1e-14])
def test_tree_config1_dense(ctx, far_tol):
    dom, _ = wl.config1()
    rng = np.random.default_rng([wl.SEED, 91])
    w = rng.normal(size=(dom.eta.shape[0], 2)) + 1j * rng.normal(size=(dom.eta.shape[0], 2))
    print(f"[tree] config1 far_tol={far_tol}", flush=True)
    got = ctx.cauchy_sum(_cuda(dom.eta), _cuda(w), far_tol=far_tol).cpu().numpy()
    rows = np.arange(dom.eta.shape[0])
    for q in range(2):
        S, A = _direct_rows(dom.eta, w[:, q], rows)
        _check(got[:, q], S, A, far_tol)


@pytest.mark.parametrize("N", [1, 3, 255, 256, 257, 1000, 5003])
def test_tree_small_and_ragged(ctx, N):
    rng = np.random.default_rng([wl.SEED, 92, N])
    eta = rng.uniform(-1, 1, N) + 1j * rng.uniform(-1, 1, N)
    w = rng.normal(size=N) + 1j * rng.normal(size=N)
    print(f"[tree] random N={N}", flush=True)
    got = ctx.cauchy_sum(_cuda(eta), _cuda(w), far_tol=1e-12).cpu().numpy()
    S, A = _direct_rows(eta, w, np.arange(N))
    _check(got, S, A, 1e-12)


def test_tree_config4_sampled(ctx):
    # 129 perturbed circles, N = 264192: sampled rows of the direct sum
    dom, _ = wl.config4()
    N = dom.eta.shape[0]
    rng = np.random.default_rng([wl.SEED, 93])
    w = np.cos(3 * np.angle(dom.eta)) * dom.etap
    print(f"[tree] config4 N={N}", flush=True)
    got = ctx.cauchy_sum(_cuda(dom.eta), _cuda(w), far_tol=1e-12).cpu().numpy()
    rows = np.concatenate([rng.choice(N - 1, 95, replace=False), [N - 1]])
    S, A = _direct_rows(dom.eta, w, rows)
    _check(got[rows], S, A, 1e-12)


def test_tree_fbie_config1_against_golden(gk, ctx):
    g = np.load(os.path.join(GOLDEN, "cfg1_oracle.npz"))
    dom, gam = wl.config1()
    dd = gk.DeviceDomain.from_host(dom)
    mu, h, infos, st = ctx.fbie(dd, _cuda(gam[:, 0]), restart=25, tol=1e-12, far_tol=1e-13)
    assert st == gk.OK, infos
    s = max(np.max(np.abs(g["mu"])), np.max(np.abs(gam)))
    assert np.max(np.abs(mu.cpu().numpy() - g["mu"])) / s < 1e-10
    assert np.max(np.abs(h.cpu().numpy() - g["h"])) / s < 1e-10
    mu_ad, infos, st = ctx.fbie_ad(dd, _cuda(gam[:, 0]), restart=25, tol=1e-12, far_tol=1e-13)
    assert st == gk.OK, infos
    assert np.max(np.abs(mu_ad.cpu().numpy() - g["mu_ad"])) / s < 1e-10


def test_tree_fbie_closed_form_unbounded(gk, ctx):
    # exterior of circles: gamma = Re[A f], mu = Im[A f], h = 0 (eq. (e:ex-gam))
    dom = wl.circles_unbounded(256, [0.0, 3.0, -2.0 + 2.5j, 1.5 - 3.0j], [1.0, 0.7, 0.5, 0.8])
    gam, mu_ex = wl.closed_form_rhs(dom, lambda z: 1.0 / (z - 0.2) + 0.5 / (z - 3.1))
    dd = gk.DeviceDomain.from_host(dom)
    mu, h, infos, st = ctx.fbie(dd, _cuda(gam), restart=40, tol=1e-13, far_tol=1e-13)
    assert st == gk.OK, infos
    mu_r, h_r = orc.fbie(dom.eta, dom.etap, dom.A, gam, dom.n)
    s = max(np.max(np.abs(mu_r)), np.max(np.abs(gam)))
    assert np.max(np.abs(mu.cpu().numpy() - mu_r)) / s < 1e-10
    assert np.max(np.abs(mu.cpu().numpy() - mu_ex)) < 1e-9


def test_tree_argument_errors(gk, ctx):
    dom = wl.annulus(32)
    gam, _ = wl.closed_form_rhs(dom, lambda z: z)
    dd = gk.DeviceDomain.from_host(dom)
    for kw in (dict(far_tol=1.0), dict(far_tol=1e-17), dict(far_tol=1e-8, prec=gk.MIXED)):
        with pytest.raises(gk.GnkError) as e:
            ctx.fbie(dd, _cuda(gam), **kw)
        assert e.value.status == gk.ERR_ARG
    eta = _cuda(np.exp(1j * np.linspace(0, 6, 50)))
    with pytest.raises(gk.GnkError) as e:
        ctx.cauchy_sum(eta, eta, far_tol=0.5)
    assert e.value.status == gk.ERR_ARG
    mu, h, infos, st = ctx.fbie(dd, _cuda(gam))
    assert st == gk.OK


def test_tree_profile_counts(gk, ctx):
    # the profile separates the treecode products and counts the work of their lists:
    # at most the direct sum's 16 N(N-1) flops per column, and well below it for large N
    dom, _ = wl.config4()
    N = dom.eta.shape[0]
    w = np.cos(3 * np.angle(dom.eta)) * dom.etap
    ctx.profile(True)
    ctx.profile_read(reset=True)
    ctx.cauchy_sum(_cuda(dom.eta), _cuda(w), far_tol=1e-12)
    p = ctx.profile_read(reset=True)
    ctx.profile(False)
    assert p["launches_tree"] == 1 and p["ms_tree"] > 0.0
    direct = 16.0 * N * (N - 1)
    assert 0.0 < p["flops_tree"] < 0.2 * direct
    ctx.profile(True)
    ctx.cauchy_sum(_cuda(dom.eta[:20000]), _cuda(w[:20000]))
    p = ctx.profile_read(reset=True)
    ctx.profile(False)
    assert p["launches_tree"] == 0 and p["flops_tree"] == 0.0 and p["launches"] >= 1
