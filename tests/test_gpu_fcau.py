"""GPU parity of the Cauchy integral formula at interior points (gnk_fcau,
Sec. 7) against the CPU oracle (oracle/fcau.py), through the C ABI.

Tolerance: relative L-infinity <= 1e-10 of the oracle's values (scale: the
largest |f| of the case); both sides sum every node in FP64 and differ only in
summation order and in the reciprocal (one Newton step from v_rcp_f64, a few
ulp). Points within 1e-4 of the boundary make the two sums large, but their
ratio is well conditioned, so the same bound holds there.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads as wl
from oracle.fcau import fcau as fcau_ref

pytestmark = pytest.mark.gpu

TOL = 1e-10


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


def _gpu(ctx, eta, etap, f, z, m1, n, finf=None):
    return ctx.fcau(_cuda(eta), _cuda(etap), _cuda(f), _cuda(z), m1, n, finf=finf).cpu().numpy()


def _rel(x, ref):
    return np.max(np.abs(x - ref)) / np.max(np.abs(ref))


def _circle(c, r, n, ccw=True):
    t = 2 * np.pi * np.arange(n) / n
    s = 1.0 if ccw else -1.0
    e = np.exp(1j * s * t)
    return c + r * e, 1j * s * r * e


def _domain(parts, n):
    eta, etap = zip(*(_circle(c, r, n, ccw) for c, r, ccw in parts))
    return np.concatenate(eta), np.concatenate(etap)


CASES = {
    # name: (components, n, f, points, f(inf) or None)
    "disk": ([(0.0, 1.0, True)], 64, np.exp,
             np.array([0.0, 0.3 + 0.2j, -0.5j, 0.9, 0.999 * np.exp(0.7j)]), None),
    "annulus": ([(0.0, 1.0, True), (0.0, 0.3, False)], 96, lambda z: z ** 2 + 1.0 / (z - 0.1),
                np.array([0.6, -0.5 + 0.2j, 0.31, 0.995j, -0.7 - 0.3j]), None),
    "exterior1": ([(0.0, 1.0, False)], 64, lambda z: 1.0 / (z - 0.2) + 2.0,
                  np.array([2.0, 1.5j, 1.001, -1.01 + 0.1j, 30.0 - 40.0j]), 2.0),
    "exterior2": ([(-1.5, 0.5, False), (1.5, 0.7, False)], 64,
                  lambda z: 1.0 / (z + 1.4) + 0.5 / (z - 1.6) - 0.3j,
                  np.array([0.0, 3j, -1.5 + 0.55, 2.21, -4.0 + 1.0j]), -0.3j),
}


@pytest.mark.parametrize("name", list(CASES))
def test_fcau_closed_forms(ctx, name):
    parts, n, f, z, finf = CASES[name]
    print(f"[fcau] closed form {name}", flush=True)
    eta, etap = _domain(parts, n)
    got = _gpu(ctx, eta, etap, f(eta), z, len(parts), n, finf)
    ref = fcau_ref(eta, etap, f(eta), z, n, finf)
    assert _rel(got, ref) < TOL
    assert np.max(np.abs(got - f(z))) < 1e-11 * max(1.0, np.max(np.abs(f(z))))


def _cfg1_functions(dom):
    cen = [c for c, _, _, _ in dom.meta["ellipses"]]
    fs = [lambda z: z ** 2 + sum(1.0 / (z - c) for c in cen),
          np.exp,
          lambda z: 1.0 / (z - cen[0]) ** 3]
    return fs


def test_fcau_config1_interior_points(ctx):
    # 17 components, N = 17408; 3001 points (ragged last tile), a quarter of
    # them 1e-4..1e-2 inside G next to a node; three columns
    dom, _ = wl.config1()
    z = wl.interior_points_config1(dom, 3001, [wl.SEED, 71])
    fs = _cfg1_functions(dom)
    F = np.stack([f(dom.eta) for f in fs], axis=1)
    print(f"[fcau] config1 N={dom.eta.shape[0]} nz={z.shape[0]} nrhs=3", flush=True)
    got = _gpu(ctx, dom.eta, dom.etap, F, z, dom.m1, dom.n)
    ref = fcau_ref(dom.eta, dom.etap, F, z, dom.n)
    for q in range(3):
        assert _rel(got[:, q], ref[:, q]) < TOL, q
    exact = np.stack([f(z) for f in fs], axis=1)
    assert _rel(got, exact) < 1e-8


def test_fcau_target_on_nodes(ctx):
    dom, _ = wl.config1(n=256)
    F = np.exp(dom.eta)[:, None]
    idx = np.array([0, 5, 255, 256, 1000, dom.eta.shape[0] - 1])
    z = np.concatenate([dom.eta[idx], [0.1 + 0.1j, -0.2j]])
    got = _gpu(ctx, dom.eta, dom.etap, F, z, dom.m1, dom.n)
    assert np.array_equal(got[:idx.shape[0], 0], F[idx, 0])
    assert np.max(np.abs(got[idx.shape[0]:, 0] - np.exp(z[idx.shape[0]:]))) < 1e-12


def test_fcau_many_columns_unbounded(ctx):
    # nine columns: weight columns 10 = one 8-column group + one 2-column group
    parts = [(-1.5, 0.5, False), (1.5, 0.7, False), (0.2, 0.3, False)]
    n = 160
    eta, etap = _domain(parts, n)
    alphas = [-1.5 + 0.1j, 1.6, 0.2 - 0.05j]
    cols, finf = [], []
    for q in range(9):
        a = alphas[q % 3]
        cols.append(1.0 / (eta - a) ** (1 + q // 3) + 0.1 * q)
        finf.append(0.1 * q)
    F = np.stack(cols, axis=1)
    rng = np.random.default_rng([wl.SEED, 72])
    z = rng.uniform(-3, 3, 700) + 1j * rng.uniform(-2, 2, 700)
    keep = np.ones(z.shape, bool)
    for c, r, _ in parts:
        keep &= np.abs(z - c) > 1.02 * r
    z = z[keep]
    print(f"[fcau] 9 columns nz={z.shape[0]}", flush=True)
    got = _gpu(ctx, eta, etap, F, z, len(parts), n, finf=np.array(finf))
    ref = fcau_ref(eta, etap, F, z, n, finf=np.array(finf))
    for q in range(9):
        assert _rel(got[:, q], ref[:, q]) < TOL, q


@pytest.mark.parametrize("n,nz", [(8, 1), (8, 65), (6, 129), (1, 3)])
def test_fcau_tiny(ctx, n, nz):
    eta, etap = _domain([(0.0, 1.0, True)], n)
    rng = np.random.default_rng([wl.SEED, 73, n, nz])
    z = 0.5 * (rng.uniform(-1, 1, nz) + 1j * rng.uniform(-1, 1, nz))
    f = eta ** 2 + 0.5
    got = _gpu(ctx, eta, etap, f, z, 1, n)
    ref = fcau_ref(eta, etap, f, z, n)
    assert _rel(got, ref) < TOL


def test_fcau_large_sampled(ctx):
    # config 4 geometry (129 perturbed circles, N = 264192), 100003 exterior
    # points; the oracle evaluates a sample of them, including the last one
    dom, _ = wl.config4()
    z = wl.exterior_points_fourier(dom, 100003, [wl.SEED, 74])
    cen = dom.meta["coeffs"][:, -dom.meta["kmin"]]
    f = lambda w: 1.0 / (w - cen[0]) + 1.0 / (w - cen[64]) ** 2 + 3.0
    print(f"[fcau] config4 N={dom.eta.shape[0]} nz={z.shape[0]}", flush=True)
    got = _gpu(ctx, dom.eta, dom.etap, f(dom.eta), z, dom.m1, dom.n, finf=3.0)
    rng = np.random.default_rng([wl.SEED, 75])
    sample = np.concatenate([rng.choice(z.shape[0] - 1, 47, replace=False), [z.shape[0] - 1]])
    ref = fcau_ref(dom.eta, dom.etap, f(dom.eta), z[sample], dom.n, finf=3.0)
    assert _rel(got[sample], ref) < TOL
    assert _rel(got, f(z)) < 1e-8


def test_fcau_argument_errors(gk, ctx):
    lib = gk.load_library()
    eta = _cuda(np.exp(1j * np.linspace(0, 6, 8)))
    out = torch.empty(4, dtype=torch.complex128, device="cuda")
    z = _cuda(np.array([0.1j, 0.2, 0.3, 0.0]))
    p = lambda t: t.data_ptr()
    assert lib.gnk_fcau(ctx.h, 0, 8, p(eta), p(eta), p(eta), 1, p(z), 4, None, p(out)) == gk.ERR_ARG
    assert lib.gnk_fcau(ctx.h, 1, 8, p(eta), p(eta), p(eta), 0, p(z), 4, None, p(out)) == gk.ERR_ARG
    assert lib.gnk_fcau(ctx.h, 1, 8, p(eta), p(eta), p(eta), 1, p(z), 0, None, p(out)) == gk.ERR_ARG
    assert lib.gnk_fcau(ctx.h, 1, 8, p(eta), p(eta), p(eta), 1, p(z), 4, None, p(z)) == gk.ERR_ARG
    assert lib.gnk_fcau(ctx.h, 1, 8, p(eta), None, p(eta), 1, p(z), 4, None, p(out)) == gk.ERR_ARG
    # a valid call still works after the errors
    assert lib.gnk_fcau(ctx.h, 1, 8, p(eta), p(eta), p(eta), 1, p(z), 4, None, p(out)) == gk.OK


# ------------------------------------------------------------------ treecode sums (gnk_fcau_tree)
def test_fcau_tree_config1_matches_oracle_and_direct(ctx):
    dom, _ = wl.config1()
    z = wl.interior_points_config1(dom, 3001, [wl.SEED, 71])
    fs = _cfg1_functions(dom)
    F = np.stack([f(dom.eta) for f in fs], axis=1)
    print(f"[fcau-tree] config1 N={dom.eta.shape[0]} nz={z.shape[0]}", flush=True)
    e, p, Fc, zc = _cuda(dom.eta), _cuda(dom.etap), _cuda(F), _cuda(z)
    got = ctx.fcau(e, p, Fc, zc, dom.m1, dom.n, far_tol=1e-13).cpu().numpy()
    direct = ctx.fcau(e, p, Fc, zc, dom.m1, dom.n).cpu().numpy()
    ref = fcau_ref(dom.eta, dom.etap, F, z, dom.n)
    for q in range(3):
        assert _rel(got[:, q], ref[:, q]) < TOL, q
        assert _rel(got[:, q], direct[:, q]) < TOL, q


def test_fcau_tree_large_sampled(ctx):
    # 264192 nodes, 100003 exterior points, f(inf) given; a sample against the oracle
    dom, _ = wl.config4()
    z = wl.exterior_points_fourier(dom, 100003, [wl.SEED, 74])
    cen = dom.meta["coeffs"][:, -dom.meta["kmin"]]
    f = lambda w: 1.0 / (w - cen[0]) + 1.0 / (w - cen[64]) ** 2 + 3.0
    print(f"[fcau-tree] config4 N={dom.eta.shape[0]} nz={z.shape[0]}", flush=True)
    got = ctx.fcau(_cuda(dom.eta), _cuda(dom.etap), _cuda(f(dom.eta)), _cuda(z), dom.m1, dom.n, finf=3.0,
                   far_tol=1e-12).cpu().numpy()
    rng = np.random.default_rng([wl.SEED, 76])
    sample = np.concatenate([rng.choice(z.shape[0] - 1, 47, replace=False), [z.shape[0] - 1]])
    ref = fcau_ref(dom.eta, dom.etap, f(dom.eta), z[sample], dom.n, finf=3.0)
    assert _rel(got[sample], ref) < TOL
    assert _rel(got, f(z)) < 1e-8


def test_fcau_tree_node_hits_and_tiny(ctx):
    dom, _ = wl.config1(n=256)
    Fv = np.exp(dom.eta)
    idx = np.array([0, 5, 255, 256, 1000, dom.eta.shape[0] - 1])
    z = np.concatenate([dom.eta[idx], [0.1 + 0.1j, -0.2j]])
    got = ctx.fcau(_cuda(dom.eta), _cuda(dom.etap), _cuda(Fv), _cuda(z), dom.m1, dom.n, far_tol=1e-13).cpu().numpy()
    assert np.array_equal(got[:idx.shape[0]], Fv[idx])
    assert np.max(np.abs(got[idx.shape[0]:] - np.exp(z[idx.shape[0]:]))) < 1e-12
    for n, nz in ((8, 1), (6, 129)):
        eta, etap = _domain([(0.0, 1.0, True)], n)
        rng = np.random.default_rng([wl.SEED, 77, n, nz])
        zz = 0.5 * (rng.uniform(-1, 1, nz) + 1j * rng.uniform(-1, 1, nz))
        fv = eta ** 2 + 0.5
        g = ctx.fcau(_cuda(eta), _cuda(etap), _cuda(fv), _cuda(zz), 1, n, far_tol=1e-13).cpu().numpy()
        assert _rel(g, fcau_ref(eta, etap, fv, zz, n)) < TOL


def test_fcau_tree_argument_errors(gk, ctx):
    lib = gk.load_library()
    eta = _cuda(np.exp(1j * np.linspace(0, 6, 8)))
    out = torch.empty(4, dtype=torch.complex128, device="cuda")
    z = _cuda(np.array([0.1j, 0.2, 0.3, 0.0]))
    p = lambda t: t.data_ptr()
    for ft in (0.0, 0.5, 1e-17):
        assert lib.gnk_fcau_tree(ctx.h, 1, 8, p(eta), p(eta), p(eta), 1, p(z), 4, None, ft, p(out)) == gk.ERR_ARG
    assert lib.gnk_fcau_tree(ctx.h, 1, 8, p(eta), p(eta), p(eta), 1, p(z), 4, None, 1e-12, p(out)) == gk.OK
