"""The library's HIP-event profile (gnk_profile / gnk_profile_read): circulant
products are reported on their own, with 24 algorithmic bytes per unknown and
column, and stay out of the Cauchy-sum totals; Cauchy sums count N(N-1) pairs
per column."""
import numpy as np
import pytest
import torch

import workloads as wl

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


def test_profile_separates_circulant_products(gk, ctx):
    dom = wl.annulus(256)
    dd = gk.DeviceDomain.from_host(dom)
    N = dom.eta.shape[0]
    x = torch.from_numpy(np.random.default_rng([wl.SEED, 61]).normal(size=(N, 3))).cuda()
    ctx.profile(True)
    ctx.profile_read(reset=True)
    ctx.apply(dd, gk.OP_LHAT, x)
    p = ctx.profile_read(reset=True)
    assert p["launches_fft"] == 1 and p["ms_fft"] > 0.0
    assert p["bytes_fft"] == 24.0 * N * 3
    assert p["launches"] == 0 and p["pair_cols"] == 0.0
    eta = torch.from_numpy(dom.eta).cuda()
    ctx.cauchy_sum(eta, eta)
    p = ctx.profile_read(reset=True)
    ctx.profile(False)
    assert p["launches_fft"] == 0 and p["launches"] >= 1
    assert p["pair_cols"] == float(N) * (N - 1)


def test_profile_leaves_out_speculative_steps(gk, ctx):
    # GMRES runs a few fully masked steps after its column stops (up to four steps per
    # graph launch, one launch ahead); the profile counts only the products that do work, so
    # products minus Arnoldi steps is the same for solves of different lengths
    dom, gam = wl.config1(n=256)
    dd = gk.DeviceDomain.from_host(dom)
    g = torch.from_numpy(gam[:, 0].copy()).cuda()
    extra = []
    for tol in (1e-6, 1e-9, 1e-12):
        ctx.profile(True)
        ctx.profile_read(reset=True)
        mu, h, infos, st = ctx.fbie(dd, g, restart=40, tol=tol)
        p = ctx.profile_read(reset=True)
        ctx.profile(False)
        assert st == gk.OK
        extra.append(p["launches1"] - infos[0]["inner_it"])
    assert len(set(extra)) == 1, extra
