"""Solver options of the C ABI: the residual history, refinement steps and
max_refine of mixed solves, and the options the autograd wrapper rejects."""
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


@pytest.fixture(scope="module")
def small_close():
    return wl.config2(n=256, m1=9)


@pytest.fixture(scope="module")
def separated():
    """A domain of the batched generator (well-separated holes), two columns."""
    dom, gam = wl.batch_domain(5, m1_range=(5, 8), ns=(256,))
    return dom, np.ascontiguousarray(gam[:, :2])


def test_residual_history_fp64(gk, ctx, separated):
    """Per column: 1 + inner_it + outer_it entries (the true residual at each
    cycle start, then one estimate per Arnoldi step, and the final true
    residual); it starts at 1 (x0 = 0) and ends at the reported true residual."""
    dom, g = separated
    dd = gk.DeviceDomain.from_host(dom)
    R = 6
    mu, h, infos, st = ctx.fbie(dd, _cuda(g), tol=1e-12, restart=R, maxit=40, hist_len=2000)
    assert st == 0
    for inf in infos:
        hs = inf["hist"]
        print(f"[hist] outer {inf['outer_it']} inner {inf['inner_it']} count {inf['hist_count']} "
              f"first {hs[0]:.3e} last {hs[-1]:.3e}", flush=True)
        assert inf["hist_count"] == 1 + inf["inner_it"] + inf["outer_it"] == len(hs)
        assert hs[0] == pytest.approx(1.0, rel=1e-12)
        assert hs[-1] == inf["true_relres"] and hs[-1] <= 1e-12
        assert inf["refine_steps"] == 0
        # cycles of R steps (the last one shorter): [true, est x R, true, est x R, ..., true];
        # within a cycle the estimates do not increase (GMRES minimises the residual)
        k = 0
        for cyc in range(inf["outer_it"]):
            steps = min(R, inf["inner_it"] - R * cyc)
            est = hs[k + 1:k + 1 + steps]
            assert all(b <= a * (1 + 1e-12) for a, b in zip(est, est[1:]))
            k += 1 + steps
        assert k == len(hs) - 1
    mu_o, h_o = orc.fbie(dom.eta, dom.etap, dom.A, g, dom.n)
    assert orc.rel_linf(mu.cpu().numpy(), mu_o, np.max(np.abs(g))) < 1e-10


def test_residual_history_truncated(gk, ctx, separated):
    dom, gam = separated
    dd = gk.DeviceDomain.from_host(dom)
    _, _, infos, st = ctx.fbie(dd, _cuda(gam[:, 0]), tol=1e-12, restart=64, hist_len=5)
    assert st == 0 and infos[0]["hist_count"] == 5 and len(infos[0]["hist"]) == 5


def test_mixed_refinement_steps_and_cap(gk, ctx, separated):
    """inner_tol = 1 makes every Arnoldi product mixed: each restart cycle (4
    steps) is one refinement step (refine_steps = outer_it). With max_refine = 2 only the
    first two cycles are mixed and the rest take FP64 products; the result
    meets the same 1e-10 bar against the oracle."""
    dom, gam = separated
    g = gam[:, 0]
    dd = gk.DeviceDomain.from_host(dom)
    kw = dict(prec=gk.MIXED, inner_tol=1.0, restart=4, maxit=200, tol=1e-13)
    mu1, _, inf1, st1 = ctx.fbie(dd, _cuda(g), **kw)
    mu2, _, inf2, st2 = ctx.fbie(dd, _cuda(g), max_refine=2, **kw)
    i1, i2 = inf1[0], inf2[0]
    print(f"[refine] uncapped {i1}\n[refine] capped {i2}", flush=True)
    assert st1 == 0 and st2 == 0
    assert i1["outer_it"] > 2 and i1["refine_steps"] == i1["outer_it"]
    assert i2["refine_steps"] == 2 and i2["mixed_steps"] <= 2 * 4
    mu_o, _ = orc.fbie(dom.eta, dom.etap, dom.A, g, dom.n)
    s = np.max(np.abs(g))
    for mu in (mu1, mu2):
        assert orc.rel_linf(mu.cpu().numpy(), mu_o, s) < 1e-10


def test_bad_option_values_rejected(gk, ctx, small_close):
    dom, gam = small_close
    dd = gk.DeviceDomain.from_host(dom)
    with pytest.raises(gk.GnkError) as e:
        ctx.fbie(dd, _cuda(gam[:, 0]), max_refine=-1)
    assert e.value.status == gk.ERR_ARG


def test_autograd_rejects_options_without_adjoint(gk, ctx):
    from paper_1308_5351_amd import autograd as ag
    dom = wl.disk(32, "eta-alpha")
    cu = lambda a: _cuda(a)
    args = (cu(dom.eta), cu(dom.etap), cu(dom.A), cu(np.ones(dom.N)), dom.m1, dom.n)
    for bad in (dict(far_tol=1e-10), dict(subtract=False), dict(hist_len=10)):
        with pytest.raises(ValueError):
            ag.fbie(*args, context=ctx, **bad)
