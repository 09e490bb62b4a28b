"""Scale invariance of the discrete system (GPU): with A = 1 the kernel
K_ij = (2/n) eta'_j/(eta_j - eta_i) (eqs. (e:N), (e:M)) is unchanged by
eta -> s eta, so mu and h of FBIE are those of the unscaled domain for the
same gamma. Solved at s = 1e6, 1e-6, 1e15 and 1e-15 in FP64 and in mixed
precision (the FP32 far tiles: one column on the VALU, several on the matrix
cores) and compared with the oracle's unscaled solution at 1e-10. At 1e-15
the closest nodes of the close-boundary case are about 1e-20 apart: the FP64
loops share one reciprocal among four pairs, so they invert products of four
squared distances (about 1e-160 there, 1e127 at the far end of 1e15), which
must stay in the normal FP64 range."""
import copy

import numpy as np
import pytest
import torch

import workloads as wl
from oracle import nystrom as orc

pytestmark = pytest.mark.gpu


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


def _scaled(dom, s):
    d = copy.copy(dom)
    d.eta, d.etap, d.etapp = dom.eta * s, dom.etap * s, dom.etapp * s
    return d


@pytest.fixture(scope="module")
def close_one():
    """9 close boundaries (gaps 1e-3..1e-2 of size, graded corners), n = 256, one column."""
    dom, gam = wl.config2(n=256, m1=9)
    mu, h = orc.fbie(dom.eta, dom.etap, dom.A, gam, dom.n)
    return dom, gam, mu, h


@pytest.fixture(scope="module")
def sep_many():
    """A domain of the batched generator with 8 right-hand sides (matrix-core far tiles)."""
    dom, gam = wl.batch_domain(11, m1_range=(8, 8), ns=(256,))
    mu, h = orc.fbie(dom.eta, dom.etap, dom.A, gam, dom.n)
    return dom, gam, mu, h


@pytest.mark.parametrize("s", [1e6, 1e-6, 1e15, 1e-15])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("case", ["close_one", "sep_many"])
def test_scaled_domain_matches_unscaled_oracle(gk, ctx, request, s, prec, case):
    dom, gam, mu_o, h_o = request.getfixturevalue(case)
    sd = _scaled(dom, s)
    dd = gk.DeviceDomain.from_host(sd)
    p = gk.MIXED if prec == "mixed" else gk.FP64
    print(f"[scale] {case} s={s:g} {prec}", flush=True)
    mu, h, infos, st = ctx.fbie(dd, _cuda(gam), tol=1e-13, restart=100, maxit=10, prec=p)
    sc = float(np.max(np.abs(gam)))
    e_mu = orc.rel_linf(mu.cpu().numpy(), mu_o, sc)
    e_h = orc.rel_linf(h.cpu().numpy(), h_o, sc)
    print(f"  err mu {e_mu:.2e} h {e_h:.2e} mixed steps {[i['mixed_steps'] for i in infos]}", flush=True)
    assert st == 0 and e_mu < 1e-10 and e_h < 1e-10
    if prec == "mixed":
        assert all(i["mixed_steps"] >= 1 for i in infos)
