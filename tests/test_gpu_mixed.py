"""Mixed precision (FP32 far tiles, FP64 near tiles, FP64 refinement) through the C ABI.

Bar: the refined solution matches the FP64 oracle to the same 1e-10 relative
L-infinity as the FP64 path."""
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


def test_mixed_products_close_to_fp64(gk, ctx, small_close):
    """Mixed products differ from FP64 by about FP32 rounding (and the FP32
    branch is really taken)."""
    dom, _ = small_close
    dd = gk.DeviceDomain.from_host(dom)
    rng = np.random.default_rng(4)
    x = _cuda(rng.normal(size=(dom.N, 2)))
    for op in (gk.OP_FB, gk.OP_FC, gk.OP_FB_T, gk.OP_FC_T):
        y64 = ctx.apply(dd, op, x).cpu().numpy()
        y32 = ctx.apply(dd, op, x, prec=gk.MIXED).cpu().numpy()
        err = np.max(np.abs(y32 - y64)) / np.max(np.abs(y64))
        print(f"[mixed] op {op} rel err {err:.2e}", flush=True)
        assert 1e-12 < err < 1e-5


@pytest.mark.parametrize("nrhs", [4, 8, 13, 21])
def test_mixed_products_matrix_cores(gk, ctx, small_close, nrhs):
    """Products with 4-16 column groups take their far tiles on the matrix cores
    (13 columns = groups of 8, 4 and 1; 21 = 16 and a padded group of 5):
    every column against the FP64 product, and against the oracle's kernel
    rows on sampled targets."""
    dom, _ = small_close
    dd = gk.DeviceDomain.from_host(dom)
    rng = np.random.default_rng([5, nrhs])
    x = rng.normal(size=(dom.N, nrhs))
    xd = _cuda(x)
    for op in (gk.OP_FB, gk.OP_FC_T):
        y64 = ctx.apply(dd, op, xd).cpu().numpy()
        y32 = ctx.apply(dd, op, xd, prec=gk.MIXED).cpu().numpy()
        err = np.max(np.abs(y32 - y64), axis=0) / np.max(np.abs(y64), axis=0)
        print(f"[mixed] nrhs {nrhs} op {op} per-column rel err max {err.max():.2e} min {err.min():.2e}", flush=True)
        assert np.all(err < 1e-6) and np.all(err > 1e-13)
    # FB on sampled rows from the kernel definition: y = 2x + diag(B1)x - Bx
    rows = slice(0, dom.N, 37)
    K = orc.kernel_rows(dom.eta, dom.etap, dom.A, dom.n, rows)
    idx = np.arange(dom.N)[rows]
    B = K.imag
    ref = 2.0 * x[idx] + B.sum(axis=1)[:, None] * x[idx] - B @ x
    y32 = ctx.apply(dd, gk.OP_FB, xd, prec=gk.MIXED).cpu().numpy()[idx]
    assert np.max(np.abs(y32 - ref)) / np.max(np.abs(ref)) < 1e-6


@pytest.mark.parametrize("nrhs", [8, 13, 20])
def test_mixed_matrix_cores_short_tiles(gk, ctx, nrhs):
    """n = 100 (N = 100 (m+1), not a multiple of 64): the last source and target
    tiles of the domain are short, so the matrix-core far kernel stages zero
    weights past their end. Products against the FP64 ones and the oracle's
    kernel rows; a mixed solve with every Arnoldi product mixed against the
    dense oracle at 1e-10."""
    dom, gam = wl.batch_domain(7, m1_range=(nrhs, nrhs), ns=(100,))
    assert dom.N % 64 != 0 and gam.shape[1] == nrhs
    dd = gk.DeviceDomain.from_host(dom)
    rng = np.random.default_rng([8, nrhs])
    x = rng.normal(size=(dom.N, nrhs))
    xd = _cuda(x)
    print(f"[mixed] short tiles: N = {dom.N}, nrhs {nrhs}", flush=True)
    y64 = ctx.apply(dd, gk.OP_FB, xd).cpu().numpy()
    y32 = ctx.apply(dd, gk.OP_FB, xd, prec=gk.MIXED).cpu().numpy()
    err = np.max(np.abs(y32 - y64), axis=0) / np.max(np.abs(y64), axis=0)
    print(f"  per-column rel err max {err.max():.2e} min {err.min():.2e}", flush=True)
    assert np.all(err < 1e-6) and np.all(err > 1e-13)
    K = orc.kernel_rows(dom.eta, dom.etap, dom.A, dom.n, slice(dom.N - 70, dom.N))
    idx = np.arange(dom.N - 70, dom.N)
    B = K.imag
    ref = 2.0 * x[idx] + B.sum(axis=1)[:, None] * x[idx] - B @ x
    assert np.max(np.abs(y32[idx] - ref)) / np.max(np.abs(ref)) < 1e-6
    mu, h, infos, st = ctx.fbie(dd, _cuda(gam), tol=1e-13, restart=10, maxit=40, prec=gk.MIXED, inner_tol=1.0)
    mu_o, h_o = orc.fbie(dom.eta, dom.etap, dom.A, gam, dom.n)
    s = np.max(np.abs(gam))
    e_mu = orc.rel_linf(mu.cpu().numpy(), mu_o, s)
    e_h = orc.rel_linf(h.cpu().numpy(), h_o, s)
    print(f"  solve: err mu {e_mu:.2e} h {e_h:.2e} mixed steps {[i['mixed_steps'] for i in infos]}", flush=True)
    assert st == 0 and all(i["mixed_steps"] >= 1 for i in infos)
    assert e_mu < 1e-10 and e_h < 1e-10


@pytest.mark.parametrize("restart,inner_tol", [(50, 0.0), (10, 1.0)])
def test_batched_mixed_matrix_cores_matches_oracle(gk, ctx, restart, inner_tol):
    """Batched mixed solve of domains with 8-13 right-hand sides (matrix-core far
    tiles) against the dense oracle, 1e-10 relative L-infinity: relaxed
    switching (inner_tol default) and outer refinement (every product mixed,
    FP64 residual at each restart of 10)."""
    batch = [wl.batch_domain(d, m1_range=(8, 13), ns=(128, 256)) for d in range(3)]
    doms = [gk.DeviceDomain.from_host(d) for d, _ in batch]
    gams = [_cuda(g) for _, g in batch]
    print(f"[mixed] batched sizes {[(d.m1, d.n) for d, _ in batch]} restart {restart}", flush=True)
    mus, hs, infos, st = ctx.fbie_batched(doms, gams, tol=1e-13, prec=gk.MIXED, restart=restart,
                                          inner_tol=inner_tol)
    assert st == 0
    assert max(i["mixed_steps"] for inf in infos for i in inf) >= 1
    if inner_tol >= 1.0:   # every Arnoldi step mixed
        assert all(i["mixed_steps"] == i["inner_it"] for inf in infos for i in inf)
    worst = 0.0
    for (dom, gam), mu, h in zip(batch, mus, hs):
        mu_o, h_o = orc.fbie(dom.eta, dom.etap, dom.A, gam, dom.n)
        s = np.max(np.abs(gam))
        worst = max(worst, orc.rel_linf(mu.cpu().numpy(), mu_o, s), orc.rel_linf(h.cpu().numpy(), h_o, s))
    print(f"  worst rel err {worst:.2e}", flush=True)
    assert worst < 1e-10


@pytest.mark.parametrize("nrhs", [1, 2])
def test_fbie_mixed_matches_oracle_reduced(gk, ctx, small_close, nrhs):
    """9 close boundaries (3 graded polygons), n = 256: mixed + refinement vs the dense oracle."""
    dom, gam = small_close
    if nrhs == 2:
        gam = np.concatenate([gam, (dom.eta ** 3).real[:, None] * 0.1], axis=1)
    dd = gk.DeviceDomain.from_host(dom)
    mu, h, infos, st = ctx.fbie(dd, _cuda(gam), prec=gk.MIXED, tol=1e-13, restart=64)
    mu_o, h_o = orc.fbie(dom.eta, dom.etap, dom.A, gam, dom.n)
    s = np.max(np.abs(gam))
    e_mu = orc.rel_linf(mu.cpu().numpy(), mu_o, s)
    e_h = orc.rel_linf(h.cpu().numpy(), h_o, s)
    print(f"[mixed] reduced close: err mu {e_mu:.2e} h {e_h:.2e} infos {infos}", flush=True)
    assert st == 0 and all(i["mixed_steps"] >= 1 for i in infos)
    assert e_mu < 1e-10 and e_h < 1e-10


def test_fbiead_mixed_matches_oracle(gk, ctx):
    dom = wl.example4_circles(256, 1e-2)
    gam = (dom.eta ** 2).real
    dd = gk.DeviceDomain.from_host(dom)
    mu, infos, st = ctx.fbie_ad(dd, _cuda(gam), prec=gk.MIXED, tol=1e-13, restart=64)
    ref = orc.fbiead(dom.eta, dom.etap, dom.etapp, dom.A, dom.Ap, gam, dom.n, dom.c)
    err = orc.rel_linf(mu.cpu().numpy(), ref, np.max(np.abs(gam)))
    print(f"[mixed] fbiead ex4: err {err:.2e} infos {infos}", flush=True)
    assert st == 0 and err < 1e-10


def test_close_boundary_full_size(gk, ctx):
    """65 close boundaries, n = 2048 (N = 133120): mixed and FP64 GPU solves agree
    to 1e-10, and the oracle's residual on sampled rows is at the solver tolerance."""
    dom, gam = wl.config2()
    g = gam[:, 0]
    dd = gk.DeviceDomain.from_host(dom)
    gt = _cuda(g)
    print("[full] fp64 solve", flush=True)
    mu64, h64, inf64, st64 = ctx.fbie(dd, gt, tol=1e-14, restart=256, maxit=8)
    print(f"  {inf64}", flush=True)
    print("[full] mixed solve", flush=True)
    mu32, h32, inf32, st32 = ctx.fbie(dd, gt, tol=1e-14, restart=256, maxit=8, prec=gk.MIXED)
    print(f"  {inf32}", flush=True)
    assert st64 == 0 and st32 == 0
    a64, a32 = mu64.cpu().numpy(), mu32.cpu().numpy()
    s = np.max(np.abs(g))
    assert orc.rel_linf(a32, a64, s) < 1e-10
    assert orc.rel_linf(h32.cpu().numpy(), h64.cpu().numpy(), s) < 1e-10
    rng = np.random.default_rng(21)
    rows = np.sort(rng.choice(dom.N, 48, replace=False))
    res, y = orc.fbie_residual_rows(dom.eta, dom.etap, dom.A, g, a32, dom.n, rows)
    rel = np.max(np.abs(res)) / np.max(np.abs(y))
    print(f"[full] oracle residual on {len(rows)} rows: {rel:.2e}", flush=True)
    assert rel < 1e-9
