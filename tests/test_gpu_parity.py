"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Tolerances: relative L-infinity <= 1e-10 on mu and h for the solves
(error / max(|ref|_inf, |gamma|_inf)); operator products and Cauchy sums are
compared tighter (they involve no solve).
"""
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


def _rel(x, ref, scale=None):
    return orc.rel_linf(x, ref, scale)


def _dense_E(eta):
    N = eta.shape[0]
    d = eta[:, None] - eta[None, :]
    d[np.arange(N), np.arange(N)] = 1.0
    E = 1.0 / d
    E[np.arange(N), np.arange(N)] = 0.0
    return E


# ------------------------------------------------------------- Cauchy sums
@pytest.mark.parametrize("N,nrhs", [(1, 1), (2, 1), (63, 2), (257, 1), (1000, 3), (2311, 9), (4096, 1)])
def test_cauchy_sum_matches_dense(ctx, N, nrhs):
    print(f"[cauchy] N={N} nrhs={nrhs}", flush=True)
    rng = np.random.default_rng([7, N, nrhs])
    eta = rng.uniform(-1, 1, N) + 1j * rng.uniform(-1, 1, N)
    w = rng.normal(size=(N, nrhs)) + 1j * rng.normal(size=(N, nrhs))
    E = _dense_E(eta)
    ref = E @ w
    scale = (np.abs(E) @ np.abs(w)).max()
    S = ctx.cauchy_sum(_cuda(eta), _cuda(w)).cpu().numpy()
    if N == 1:                      # empty sum
        assert np.all(S == 0)
        return
    err = np.max(np.abs(S - ref)) / scale
    print(f"  err/scale = {err:.2e}")
    assert err < 1e-13


@pytest.mark.parametrize("tpt,splits", [("1", "1"), ("2", "1"), ("2", "3"), ("1", "7"), ("2", "64")])
def test_cauchy_sum_launch_shapes(ctx, monkeypatch, tpt, splits):
    """Every launch shape (targets per lane, source splits) gives the same sums,
    including ragged tails, the masked self window and whole waves past N."""
    monkeypatch.setenv("GNK_CAUCHY_TPT", tpt)
    monkeypatch.setenv("GNK_CAUCHY_SPLITS", splits)
    for N, nrhs in ((131, 1), (1030, 5), (2049, 2)):
        print(f"[shape] tpt={tpt} splits={splits} N={N} nrhs={nrhs}", flush=True)
        rng = np.random.default_rng([8, N])
        eta = rng.uniform(-1, 1, N) + 1j * rng.uniform(-1, 1, N)
        w = rng.normal(size=(N, nrhs)) + 1j * rng.normal(size=(N, nrhs))
        E = _dense_E(eta)
        ref = E @ w
        scale = (np.abs(E) @ np.abs(w)).max()
        S = ctx.cauchy_sum(_cuda(eta), _cuda(w)).cpu().numpy()
        assert np.max(np.abs(S - ref)) / scale < 1e-13


def test_cauchy_sum_deterministic(ctx):
    N = 3001
    rng = np.random.default_rng(11)
    eta = _cuda(rng.uniform(-1, 1, N) + 1j * rng.uniform(-1, 1, N))
    w = _cuda(rng.normal(size=N) + 1j * rng.normal(size=N))
    a = ctx.cauchy_sum(eta, w)
    b = ctx.cauchy_sum(eta, w)
    assert torch.equal(a, b)


# -------------------------------------------------------- operator products
def _ops_dense(d):
    Aop, Cop = orc.fbie_operators(d.eta, d.etap, d.A, d.n)
    return Aop, Cop


def _domains_small():
    out = []
    dom0, _ = wl.config0("eta-alpha")
    out.append(("cfg0b", dom0))
    # ragged: three components, n = 70 (not a power of two: direct circulant path)
    out.append(("ragged", wl.circles_unbounded(70, [0j, 1.6 + 0.3j, -1.2 + 1.0j], [0.5, 0.4, 0.45])))
    out.append(("ex2", wl.example2_circles(128, 0.05)))
    return out


@pytest.mark.parametrize("name,dom", _domains_small(), ids=lambda v: v if isinstance(v, str) else "")
def test_operators_match_oracle(gk, ctx, name, dom):
    print(f"[ops] {name} N={dom.N}", flush=True)
    dd = gk.DeviceDomain.from_host(dom)
    Aop, Cop = _ops_dense(dom)
    G = orc.fbiead_operator(dom.eta, dom.etap, dom.etapp, dom.A, dom.Ap, dom.n, dom.c)
    Lhat = orc.block_diag_repeat(orc.circulant_L(dom.n), dom.m1)
    rng = np.random.default_rng(3)
    x = rng.normal(size=(dom.N, 3))
    xt = _cuda(x)
    cases = {gk.OP_FB: Aop, gk.OP_FC: Cop, gk.OP_GB: G, gk.OP_FB_T: Aop.T, gk.OP_FC_T: Cop.T,
             gk.OP_GB_T: G.T, gk.OP_LHAT: Lhat}
    for op, M in cases.items():
        y = ctx.apply(dd, op, xt).cpu().numpy()
        ref = M @ x
        scale = (np.abs(M) @ np.abs(x)).max()
        err = np.max(np.abs(y - ref)) / scale
        print(f"  op {op}: err/scale {err:.2e}")
        assert err < 1e-13, (name, op, err)


def test_adjoint_dot_product(gk, ctx):
    """<u, Op v> = <Op^T u, v> through the ABI."""
    dom = wl.circles_unbounded(128, [0j, 1.3 + 0.4j], [0.5, 0.4])
    dd = gk.DeviceDomain.from_host(dom)
    rng = np.random.default_rng(5)
    u, v = rng.normal(size=dom.N), rng.normal(size=dom.N)
    for op, opt in ((gk.OP_FB, gk.OP_FB_T), (gk.OP_FC, gk.OP_FC_T), (gk.OP_GB, gk.OP_GB_T)):
        a = u @ ctx.apply(dd, op, _cuda(v)).cpu().numpy()
        b = ctx.apply(dd, opt, _cuda(u)).cpu().numpy() @ v
        assert abs(a - b) < 1e-12 * max(1, abs(a))


# ------------------------------------------------------------------ solves
def _solve_and_compare(gk, ctx, dom, gam, tol=1e-12, restart=25, maxit=40):
    dd = gk.DeviceDomain.from_host(dom)
    g = _cuda(gam)
    mu, h, infos, st = ctx.fbie(dd, g, restart=restart, maxit=maxit, tol=tol)
    mu_o, h_o = orc.fbie(dom.eta, dom.etap, dom.A, gam, dom.n)
    gs = np.max(np.abs(gam))
    e_mu = _rel(mu.cpu().numpy(), mu_o, gs)
    e_h = _rel(h.cpu().numpy(), h_o, gs)
    return st, infos, e_mu, e_h


@pytest.mark.parametrize("kind", ["one", "eta-alpha"])
def test_fbie_config0(gk, ctx, kind):
    dom, gam = wl.config0(kind)
    print(f"[fbie] cfg0 A={kind}", flush=True)
    st, infos, e_mu, e_h = _solve_and_compare(gk, ctx, dom, gam)
    print(f"  status {st} infos {infos[0]} err mu {e_mu:.2e} h {e_h:.2e}")
    assert st == 0 and infos[0]["flag"] == 0
    assert infos[0]["true_relres"] <= 1e-12
    assert e_mu < 1e-10 and e_h < 1e-10


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_fbie_initial_guess(gk, ctx, prec):
    """The options' initial guess x0. Started at the oracle's mu the solve stops at
    the first cycle start; started at a perturbed mu it reaches the oracle's mu and
    h in fewer Arnoldi steps than from zero. In mixed precision a start from x0
    first prepares FP64 steps, and the cycle start (residual below inner_tol)
    switches to mixed ones."""
    dom, gam = wl.config0("eta-alpha")
    dd = gk.DeviceDomain.from_host(dom)
    g = _cuda(gam)
    mu_o, h_o = orc.fbie(dom.eta, dom.etap, dom.A, gam, dom.n)
    gs = np.max(np.abs(gam))
    p = gk.MIXED if prec == "mixed" else gk.FP64
    _, _, inf0, st0 = ctx.fbie(dd, g, prec=p)
    assert st0 == 0
    mu, h, inf1, st1 = ctx.fbie(dd, g, prec=p, x0=_cuda(mu_o))
    print(f"[x0] {prec}: from zero {inf0[0]}, from the solution {inf1[0]}", flush=True)
    assert st1 == 0 and inf1[0]["inner_it"] <= 1
    assert _rel(mu.cpu().numpy(), mu_o, gs) < 1e-10 and _rel(h.cpu().numpy(), h_o, gs) < 1e-10
    rng = np.random.default_rng(17)
    x0 = mu_o + 1e-6 * gs * rng.standard_normal(mu_o.shape)
    mu, h, inf2, st2 = ctx.fbie(dd, g, prec=p, x0=_cuda(x0))
    print(f"[x0] {prec}: from a perturbed solution {inf2[0]}", flush=True)
    assert st2 == 0 and inf2[0]["inner_it"] < inf0[0]["inner_it"]
    if prec == "mixed":
        assert inf2[0]["mixed_steps"] >= 1
    assert _rel(mu.cpu().numpy(), mu_o, gs) < 1e-10 and _rel(h.cpu().numpy(), h_o, gs) < 1e-10


def test_solves_follow_the_current_stream(gk, ctx):
    """A solve issued while a side torch stream is current is enqueued on that
    stream (its Arnoldi steps captured there) and equals the solve on the
    default stream; back on the default stream the context follows again."""
    dom = wl.example4_circles(128, 1e-1)
    gam = (dom.eta ** 2).real
    dd = gk.DeviceDomain.from_host(dom)
    g = _cuda(gam)
    mu0, h0, _, st0 = ctx.fbie(dd, g)
    ad0, _, sa0 = ctx.fbie_ad(dd, g)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        mu1, h1, _, st1 = ctx.fbie(dd, g)
        ad1, _, sa1 = ctx.fbie_ad(dd, g)
        done = torch.cuda.Event()
        done.record(side)
    torch.cuda.current_stream().wait_stream(side)
    mu2, h2, _, st2 = ctx.fbie(dd, g)
    torch.cuda.synchronize()
    assert done.query()
    assert st0 == st1 == st2 == 0 and sa0 == sa1 == 0
    s = np.max(np.abs(gam))
    for a, b in ((mu1, mu0), (h1, h0), (mu2, mu0), (h2, h0), (ad1, ad0)):
        assert _rel(a.cpu().numpy(), b.cpu().numpy(), s) < 1e-13


def test_fbie_multi_rhs_ragged(gk, ctx):
    """Several right-hand sides at once on a ragged mesh equal the oracle column by column."""
    dom = wl.circles_unbounded(70, [0j, 1.6 + 0.3j, -1.2 + 1.0j], [0.5, 0.4, 0.45])
    rng = np.random.default_rng(9)
    gam = np.stack([(dom.eta ** k).real for k in (1, 2)] + [rng.normal(size=dom.N)], axis=1)
    st, infos, e_mu, e_h = _solve_and_compare(gk, ctx, dom, gam)
    print(f"  multi-rhs err mu {e_mu:.2e} h {e_h:.2e} infos {infos}")
    assert st == 0 and e_mu < 1e-10 and e_h < 1e-10


def test_fbie_closed_form(gk, ctx):
    """gamma = Re[A f(eta)] => mu = Im[A f], h = 0 (Example 1 form), on the GPU."""
    dom = wl.example2_circles(256, 0.1)
    f = lambda z: np.sin(z) + 1.0 / (z - 2.0)
    gam, mu_ex = wl.closed_form_rhs(dom, f)
    dd = gk.DeviceDomain.from_host(dom)
    mu, h, infos, st = ctx.fbie(dd, _cuda(gam))
    assert st == 0
    assert np.max(np.abs(mu.cpu().numpy() - mu_ex)) < 1e-9
    assert np.max(np.abs(h.cpu().numpy())) < 1e-9


def test_gmres_disk_two_iterations(gk, ctx):
    """On the unit disk with A = eta the matrix is I + 11^T/n: GMRES needs two steps."""
    dom = wl.disk(64)
    f = lambda z: 1.0 + 0.5 * z ** 3
    gam, mu_ex = wl.closed_form_rhs(dom, f)
    dd = gk.DeviceDomain.from_host(dom)
    mu, h, infos, st = ctx.fbie(dd, _cuda(gam))
    assert st == 0 and infos[0]["inner_it"] <= 2
    assert np.max(np.abs(mu.cpu().numpy() - mu_ex)) < 1e-12


@pytest.mark.parametrize("which", ["cfg0b", "annulus", "unbounded"])
def test_fbiead_matches_oracle(gk, ctx, which):
    if which == "cfg0b":
        dom, gam = wl.config0("eta-alpha")
        gam = gam[:, 0]
    elif which == "annulus":
        dom = wl.annulus(128)
        gam = np.ones(dom.N)
    else:
        dom = wl.circles_unbounded(96, [0j, 1.4 + 0.3j], [0.5, 0.45])
        gam = (dom.eta ** 2).real
    print(f"[fbiead] {which}", flush=True)
    dd = gk.DeviceDomain.from_host(dom)
    mu, infos, st = ctx.fbie_ad(dd, _cuda(gam))
    ref = orc.fbiead(dom.eta, dom.etap, dom.etapp, dom.A, dom.Ap, gam, dom.n, dom.c)
    err = _rel(mu.cpu().numpy(), ref, np.max(np.abs(gam)))
    print(f"  err {err:.2e} infos {infos[0]}")
    assert st == 0 and err < 1e-10


def test_config1_full_size_against_golden(gk, ctx):
    """17 components, n = 1024 (N = 17408): FBIE and FBIEad vs the stored oracle solution."""
    dom, gam = wl.config1()
    ref = np.load(os.path.join(GOLDEN, "cfg1_oracle.npz"))
    assert np.allclose(ref["eta_checksum"], [dom.eta.real.sum(), dom.eta.imag.sum()], rtol=0, atol=1e-9)
    dd = gk.DeviceDomain.from_host(dom)
    g = _cuda(gam[:, 0])
    print("[cfg1] fbie", flush=True)
    mu, h, infos, st = ctx.fbie(dd, g)
    gs = np.max(np.abs(gam))
    e_mu = _rel(mu.cpu().numpy(), ref["mu"], gs)
    e_h = _rel(h.cpu().numpy(), ref["h"], gs)
    print(f"  fbie err mu {e_mu:.2e} h {e_h:.2e} infos {infos[0]}")
    assert st == 0 and e_mu < 1e-10 and e_h < 1e-10
    print("[cfg1] fbie_ad", flush=True)
    mua, infa, sta = ctx.fbie_ad(dd, g)
    e_ad = _rel(mua.cpu().numpy(), ref["mu_ad"], gs)
    print(f"  fbiead err {e_ad:.2e} infos {infa[0]}")
    assert sta == 0 and e_ad < 1e-10


# ------------------------------------------------------------ error paths
def test_error_paths(gk, ctx):
    dom, gam = wl.config0("eta-alpha")
    dd = gk.DeviceDomain.from_host(dom)
    g = _cuda(gam[:, 0])
    # odd n
    bad = gk.DeviceDomain(dom.m1, dom.n - 1, dd.eta[: dom.m1 * (dom.n - 1)], dd.etap[: dom.m1 * (dom.n - 1)],
                          dd.A[: dom.m1 * (dom.n - 1)])
    with pytest.raises(gk.GnkError) as e:
        ctx.fbie(bad, g[: dom.m1 * (dom.n - 1)])
    assert e.value.status == gk.ERR_ODD_N
    # NaN in gamma
    g2 = g.clone()
    g2[5] = float("nan")
    with pytest.raises(gk.GnkError) as e:
        ctx.fbie(dd, g2)
    assert e.value.status == gk.ERR_NONFINITE
    # A = 0 at a node
    A2 = dd.A.clone()
    A2[3] = 0
    with pytest.raises(gk.GnkError) as e:
        ctx.fbie(gk.DeviceDomain(dom.m1, dom.n, dd.eta, dd.etap, A2), g)
    assert e.value.status == gk.ERR_ZERO_A
    # eta' = 0 for the adjoint equation
    ep2 = dd.etap.clone()
    ep2[0] = 0
    with pytest.raises(gk.GnkError) as e:
        ctx.fbie_ad(gk.DeviceDomain(dom.m1, dom.n, dd.eta, ep2, dd.A, dd.etapp, dd.Ap, dom.c), g)
    assert e.value.status == gk.ERR_ZERO_ETAP
    # not converged with a tiny iteration budget: best iterate written, flag 1
    mu, h, infos, st = ctx.fbie(dd, g, restart=1, maxit=1)
    assert st == gk.NOT_CONVERGED and infos[0]["flag"] == 1
    assert torch.isfinite(mu).all()
    # the state after the last cycle: one cycle of one step; from a zero start
    # one step cannot raise the residual, and at a restart the Givens estimate
    # equals the true residual up to rounding
    inf = infos[0]
    assert inf["outer_it"] == 1 and inf["inner_it"] == 1
    assert 0.0 < inf["true_relres"] <= 1.0
    assert abs(inf["relres"] - inf["true_relres"]) <= 1e-8 * inf["true_relres"]
    # two cycles of one step: the counts follow the cycles
    _, _, infos2, st2 = ctx.fbie(dd, g, restart=1, maxit=2)
    assert st2 == gk.NOT_CONVERGED and infos2[0]["outer_it"] == 2 and infos2[0]["inner_it"] == 2
    assert infos2[0]["true_relres"] <= inf["true_relres"] * (1 + 1e-12)
    # bad options
    with pytest.raises(gk.GnkError) as e:
        ctx.fbie(dd, g, restart=0)
    assert e.value.status == gk.ERR_ARG


def test_failed_checks_write_nothing(gk, ctx):
    """Through the C ABI: a call whose inputs fail the device checks (a
    non-finite gamma, A = 0 at a node) returns the error and leaves the
    caller's mu and h as they were, although the checks' result is read only
    after the right-hand side product has been queued."""
    import ctypes as C
    dom, gam = wl.config0("eta-alpha")
    dd = gk.DeviceDomain.from_host(dom)
    ctx._bind_stream()
    o = ctx._opts(25, 40, 1e-12, gk.FP64, 0.0, 0, None)
    g_bad = _cuda(gam[:, 0].copy())
    g_bad[7] = float("nan")
    A0 = dd.A.clone()
    A0[3] = 0
    cases = [(dd, g_bad, gk.ERR_NONFINITE),
             (gk.DeviceDomain(dom.m1, dom.n, dd.eta, dd.etap, A0), _cuda(gam[:, 0].copy()), gk.ERR_ZERO_A)]
    for dom_dev, g, want in cases:
        mu = torch.full((dom.N,), 123.0, dtype=torch.float64, device="cuda")
        h = torch.full((dom.N,), -7.0, dtype=torch.float64, device="cuda")
        infos = (gk.Info * 1)()
        d = dom_dev._struct()
        st = ctx.lib.gnk_fbie(ctx.h, C.byref(d), g.data_ptr(), 1, C.byref(o), mu.data_ptr(), h.data_ptr(), infos)
        torch.cuda.synchronize()
        assert st == want
        assert bool((mu == 123.0).all()) and bool((h == -7.0).all())
    # FBIEad: eta' = 0 at a node
    ep0 = dd.etap.clone()
    ep0[5] = 0
    d = gk.DeviceDomain(dom.m1, dom.n, dd.eta, ep0, dd.A, dd.etapp, dd.Ap, dom.c)._struct()
    mu = torch.full((dom.N,), 123.0, dtype=torch.float64, device="cuda")
    infos = (gk.Info * 1)()
    g = _cuda(gam[:, 0].copy())
    st = ctx.lib.gnk_fbie_ad(ctx.h, C.byref(d), g.data_ptr(), 1, C.byref(o), mu.data_ptr(), infos)
    torch.cuda.synchronize()
    assert st == gk.ERR_ZERO_ETAP and bool((mu == 123.0).all())


def test_workspace_cap(gk, monkeypatch):
    monkeypatch.setenv("GNK_WORKSPACE_MB", "1")
    c = gk.Context(0)
    dom, gam = wl.config1(n=256)
    dd = gk.DeviceDomain.from_host(dom)
    with pytest.raises(gk.GnkError) as e:
        c.fbie(dd, _cuda(gam[:, 0]))
    assert e.value.status == gk.ERR_OOM
    c.close()


@pytest.mark.parametrize("n", [2, 4, 8, 16, 64, 256, 512, 1024, 2048, 4096])
def test_circulant_every_fft_length(gk, ctx, n):
    # L-hat by FFT against the dense circulant blocks L_pq = (-1)^(p-q) (1/n) cot((p-q) pi/n):
    # an odd number of real columns (m1 * nrhs), several vectors per workgroup for short n and
    # a partly filled last workgroup
    m1 = 1 if n == 2 else 3
    nrhs = 7 if n <= 256 else 3
    centres = [0j, 3.0 + 0.5j, -2.5 + 2.0j][:m1]
    dom = wl.circles_unbounded(n, centres, [1.0, 0.7, 0.5][:m1])
    print(f"[circulant] n={n} m1={m1} nrhs={nrhs}", flush=True)
    dd = gk.DeviceDomain.from_host(dom)
    rng = np.random.default_rng([wl.SEED, 62, n])
    x = rng.normal(size=(dom.N, nrhs))
    y = ctx.apply(dd, gk.OP_LHAT, _cuda(x)).cpu().numpy()
    L = orc.circulant_L(n)
    for k in range(m1):
        blk = slice(k * n, (k + 1) * n)
        ref = L @ x[blk]
        # (for n = 2, L = 0 exactly; the dense form holds cot(pi/2) rounded, 6e-17)
        scale = max((np.abs(L) @ np.abs(x[blk])).max(), np.abs(x[blk]).max() / n)
        assert np.max(np.abs(y[blk] - ref)) / scale < 1e-13, k
