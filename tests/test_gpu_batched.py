"""Batched FBIE (many domains, ragged sizes, several right-hand sides each)
through the C ABI, against the CPU oracle and against single-domain solves."""
import os

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


def _small_batch():
    return [wl.batch_domain(d, m1_range=(2, 5), ns=(64, 128, 256)) for d in range(6)]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batched_matches_oracle(gk, ctx, prec):
    batch = _small_batch()
    doms = [gk.DeviceDomain.from_host(d) for d, _ in batch]
    gams = [_cuda(g) for _, g in batch]
    p = gk.MIXED if prec == "mixed" else gk.FP64
    print(f"[batched] small {prec}: sizes {[(d.m1, d.n) for d, _ in batch]}", flush=True)
    mus, hs, infos, st = ctx.fbie_batched(doms, gams, tol=1e-13, prec=p, restart=50)
    assert st == 0
    worst = 0.0
    for (dom, gam), mu, h, inf in zip(batch, mus, hs, infos):
        assert all(i["flag"] == 0 for i in inf)
        mu_o, h_o = orc.fbie(dom.eta, dom.etap, dom.A, gam, dom.n)
        s = np.max(np.abs(gam))
        e = max(orc.rel_linf(mu.cpu().numpy(), mu_o, s), orc.rel_linf(h.cpu().numpy(), h_o, s))
        worst = max(worst, e)
    print(f"  worst rel err {worst:.2e}", flush=True)
    assert worst < 1e-10


def test_batched_equals_single_domain_solves(gk, ctx):
    batch = _small_batch()
    doms = [gk.DeviceDomain.from_host(d) for d, _ in batch]
    gams = [_cuda(g) for _, g in batch]
    mus, hs, infos, st = ctx.fbie_batched(doms, gams, tol=1e-13, restart=50)
    for dd, g, mu, h in zip(doms, gams, mus, hs):
        mu1, h1, _, st1 = ctx.fbie(dd, g, tol=1e-13, restart=50)
        assert st1 == 0
        s = float(g.abs().max())
        assert float((mu1 - mu).abs().max()) / s < 1e-11
        assert float((h1 - h).abs().max()) / s < 1e-11


def test_batched_tune_cache(gk, monkeypatch, tmp_path):
    """The autotuner writes its choice to GNK_TUNE_CACHE and a new context reuses it."""
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("GNK_TUNE_CACHE", str(path))
    batch = _small_batch()[:3]
    doms = [gk.DeviceDomain.from_host(d) for d, _ in batch]
    gams = [_cuda(g) for _, g in batch]
    c1 = gk.Context(0)
    m1, _, _, st1 = c1.fbie_batched(doms, gams, want_h=False)
    c1.close()
    lines = path.read_text().strip().splitlines()
    assert len(lines) == 1 and len(lines[0].split()) == 3
    c2 = gk.Context(0)
    m2, _, _, st2 = c2.fbie_batched(doms, gams, want_h=False)
    c2.close()
    assert st1 == 0 and st2 == 0
    assert len(path.read_text().strip().splitlines()) == 1      # reused, not re-tuned
    for a, b in zip(m1, m2):
        assert torch.equal(a, b)


def test_batched_full_workload(gk, ctx):
    """64 domains (m+1 in 2..40, n in 256..2048, m+1 right-hand sides each):
    every column converges; sampled domains equal single-domain solves; the
    oracle's residual on sampled rows is at the tolerance."""
    batch = wl.config3()
    doms = [gk.DeviceDomain.from_host(d) for d, _ in batch]
    gams = [_cuda(g) for _, g in batch]
    print(f"[batched] full: {len(batch)} domains, N total {sum(d.N for d, _ in batch)}", flush=True)
    mus, hs, infos, st = ctx.fbie_batched(doms, gams, tol=1e-12, restart=50)
    print(f"  status {st}; max iters {max(i['inner_it'] for inf in infos for i in inf)}", flush=True)
    assert st == 0
    Ns = [d.N for d, _ in batch]
    pick = [int(np.argmax(Ns)), int(np.argsort(Ns)[len(Ns) // 2]), int(np.argmin(Ns))]
    for d in pick:
        dom, gam = batch[d]
        mu1, h1, _, st1 = ctx.fbie(doms[d], gams[d], tol=1e-12, restart=50)
        s = np.max(np.abs(gam))
        e = float((mu1 - mus[d]).abs().max()) / s
        print(f"  domain {d} N={dom.N} k={gam.shape[1]}: batched vs single {e:.2e}", flush=True)
        assert st1 == 0 and e < 1e-10
        rows = np.sort(np.random.default_rng(d).choice(dom.N, 16, replace=False))
        col = gam.shape[1] // 2
        res, y = orc.fbie_residual_rows(dom.eta, dom.etap, dom.A, gam[:, col], mus[d][:, col].cpu().numpy(),
                                        dom.n, rows)
        rel = np.max(np.abs(res)) / np.max(np.abs(y))
        print(f"  domain {d}: oracle residual rows {rel:.2e}", flush=True)
        assert rel < 1e-9
