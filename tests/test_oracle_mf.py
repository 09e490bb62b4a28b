"""The oracle's matrix-free route (oracle/mf.c, oracle/mf.py) against its dense
LU route on the same seeded geometries at reduced sizes, and against closed
forms; the stored reference solutions of the large workloads against their
generators. CPU only."""
import os

import numpy as np
import pytest

import workloads as wl
from oracle import gradient as og
from oracle import mf
from oracle import nystrom as orc

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.fixture(scope="module")
def close9():
    """9 close boundaries (3 Kress-graded rounded polygons), n = 128."""
    dom, gam = wl.config2(n=128, m1=9)
    return dom, gam


def _random_A(dom, seed=3):
    rng = np.random.default_rng(seed)
    return 1.0 + 0.3 * (rng.normal(size=dom.N) + 1j * rng.normal(size=dom.N))


@pytest.mark.parametrize("ncols", [1, 3])
@pytest.mark.parametrize("trans", [False, True])
@pytest.mark.parametrize("kind", ["A=1", "random A"])
def test_products_match_dense(close9, ncols, trans, kind):
    """(2I + diag(B1) - B) x and (D - diag(D1) + Lhat) x, and the transposes,
    equal the dense matrices of oracle.nystrom (a complex A exercises A_i/A_j)."""
    dom, _ = close9
    A = dom.A if kind == "A=1" else _random_A(dom)
    geo = mf.Geometry(dom.eta, dom.etap, A, dom.n)
    Aop, Cop = orc.fbie_operators(dom.eta, dom.etap, A, dom.n)
    x = np.random.default_rng(ncols).normal(size=(dom.N, ncols))
    ya, yc = mf.fbie_ops(geo, x, trans=trans)
    ra, rc = (Aop.T @ x, Cop.T @ x) if trans else (Aop @ x, Cop @ x)
    assert _rel(ya, ra) < 1e-13 and _rel(yc, rc) < 1e-13


def test_row_ranges_match_full_product(close9):
    dom, _ = close9
    geo = mf.Geometry(dom.eta, dom.etap, _random_A(dom), dom.n)
    x = np.random.default_rng(1).normal(size=(dom.N, 2))
    ya, yc = mf.fbie_ops(geo, x)
    L = orc.block_diag_repeat(geo.L, geo.m1)
    for i0, i1 in ((0, 17), (100, 613), (dom.N - 5, dom.N)):
        ra, rc = mf.fbie_rows(geo, x, i0, i1)
        assert np.allclose(ra, ya[i0:i1], rtol=0, atol=1e-13 * np.abs(ya).max())
        assert np.allclose(rc, (yc - L @ x)[i0:i1], rtol=0, atol=1e-13 * np.abs(yc).max())
    with pytest.raises(ValueError):
        mf.fbie_rows(geo, x, 10, dom.N + 1)


def test_kernel_rows_match_definition(close9):
    dom, _ = close9
    A = _random_A(dom)
    geo = mf.Geometry(dom.eta, dom.etap, A, dom.n)
    K = mf.kernel_rows(geo, 50, 90)
    assert _rel(K, orc.kernel_matrix(dom.eta, dom.etap, A, dom.n)[50:90]) < 1e-14


def test_gmres_on_the_disk_takes_two_steps():
    """Unit disk, A = eta: 2I + diag(B1) - B = I + 11^T/n, whose minimal polynomial
    has degree 2, so GMRES ends in at most two Arnoldi steps."""
    dom = wl.disk(64, "eta-alpha")
    geo = mf.Geometry(dom.eta, dom.etap, dom.A, dom.n)
    b = np.random.default_rng(0).normal(size=(dom.N, 2))
    x, info = mf.gmres(lambda v: mf.fbie_ops(geo, v)[0], b, tol=1e-14, restart=10)
    assert np.all(info["iters"] <= 2) and np.all(info["relres"] <= 1e-14)
    ref = np.linalg.solve(np.eye(dom.N) + np.ones((dom.N, dom.N)) / dom.n, b)
    assert _rel(x, ref) < 1e-13


def test_gmres_zero_rhs_gives_zero():
    dom = wl.disk(32, "eta-alpha")
    geo = mf.Geometry(dom.eta, dom.etap, dom.A, dom.n)
    b = np.zeros((dom.N, 2))
    b[:, 1] = 1.0
    x, info = mf.gmres(lambda v: mf.fbie_ops(geo, v)[0], b, tol=1e-14, restart=10)
    assert np.all(x[:, 0] == 0.0) and info["iters"][0] == 0


def test_gmres_restarts_reach_the_tolerance(close9):
    """A short restart: the true residual of every cycle is recomputed and the
    solve still reaches the tolerance (and the dense solution)."""
    dom, gam = close9
    geo = mf.Geometry(dom.eta, dom.etap, dom.A, dom.n)
    Aop, Cop = orc.fbie_operators(dom.eta, dom.etap, dom.A, dom.n)
    b = -(Cop @ gam)
    x, info = mf.gmres(lambda v: mf.fbie_ops(geo, v)[0], b, tol=1e-13, restart=8, maxit=200)
    assert info["cycles"] > 1 and info["relres"][0] <= 1e-13
    assert _rel(x[:, 0], np.linalg.solve(Aop, b[:, 0])) < 1e-10


def test_fbie_matches_dense_lu_close_boundaries():
    """The close-boundary generator at n = 256 (9 boundaries, gaps 1e-3..1e-2 of
    size, graded corners): matrix-free mu, h equal the dense LU solution."""
    dom, gam = wl.config2(n=256, m1=9)
    g = gam[:, 0]
    mu, h = orc.fbie(dom.eta, dom.etap, dom.A, g, dom.n)
    geo = mf.Geometry(dom.eta, dom.etap, dom.A, dom.n)
    mu2, h2, info = mf.fbie(geo, g, tol=1e-15, restart=300, maxit=2)
    s = np.max(np.abs(g))
    assert info["relres"][0] < 1e-14
    assert orc.rel_linf(mu2, mu, s) < 1e-12 and orc.rel_linf(h2, h, s) < 1e-12


def test_fbie_matches_dense_lu_batched_domain():
    """A domain of the batched generator with all its right-hand sides at once."""
    dom, gam = wl.batch_domain(7, ns=(128,))
    mu, h = orc.fbie(dom.eta, dom.etap, dom.A, gam, dom.n)
    geo = mf.Geometry(dom.eta, dom.etap, dom.A, dom.n)
    mu2, h2, info = mf.fbie(geo, gam, tol=1e-15, restart=100, maxit=2)
    s = np.max(np.abs(gam))
    assert np.all(info["relres"] < 1e-14)
    assert orc.rel_linf(mu2, mu, s) < 1e-12 and orc.rel_linf(h2, h, s) < 1e-12


def test_fbie_closed_form_annulus():
    """gamma = Re[A f] with f analytic in G gives mu = Im[A f] and h = 0 (Example
    1's closed form), here through the matrix-free route alone."""
    dom = wl.annulus(128)
    gam, mu_ex = wl.closed_form_rhs(dom, lambda z: 1.0 / (z - 2.0) + z ** 2)
    geo = mf.Geometry(dom.eta, dom.etap, dom.A, dom.n)
    mu, h, info = mf.fbie(geo, gam, tol=1e-15, restart=100, maxit=2)
    assert np.max(np.abs(mu - mu_ex)) < 1e-12 and np.max(np.abs(h)) < 1e-12


def test_adjoint_and_gradient_match_dense():
    """Perturbed circles at reduced size (9 curves, n = 256): lam, dL/dgamma and
    dL/dcoef of L = sum_k h_k^2 through the matrix-free route and the sampled
    geometric rows equal the dense reverse-mode oracle."""
    coeffs, kmin = wl.fourier_perturbed_circles(9, 256, [wl.SEED, 4])
    n = 256
    eta, etap, _ = og.fourier_nodes(coeffs, kmin, n)
    A = np.ones_like(eta)
    gam = (eta ** 2).real
    L_ref, g_gam_ref, g_c_ref = og.fbie_loss_and_grad(coeffs, kmin, n, gam)
    geo = mf.Geometry(eta, etap, A, n)
    mu, h, _ = mf.fbie(geo, gam, tol=1e-15, restart=100, maxit=2)
    L, g_h = og.mean_square_loss(h, n)
    lam, g_gam, info = mf.fbie_adjoint(geo, g_h=g_h, tol=1e-15, restart=100, maxit=2)
    ref = og.fbie_vjp(eta, etap, A, gam, n, g_h=g_h)
    assert abs(L - L_ref) <= 1e-12 * L_ref
    assert _rel(lam, ref["lam"]) < 1e-12 and _rel(g_gam, g_gam_ref) < 1e-12
    j = 5
    idx = np.arange(j * n, (j + 1) * n)
    ge, gp, _ = og.bilinear_geom_grad_rows(eta, etap, A, n, og.fbie_geom_terms(g_h, lam, mu, gam), idx)
    g_c = og.fourier_coef_grad(ge, gp, None, kmin, coeffs.shape[1], n)[0]
    assert float(np.max(np.abs(g_c - g_c_ref[j])) / np.max(np.abs(g_c_ref))) < 1e-11


# ------------------------------------------------------------------ stored reference solutions
def _golden(name):
    path = os.path.join(GOLDEN, f"{name}_oracle.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written yet")
    return np.load(path)


@pytest.mark.parametrize("name,gen", [("cfg2", wl.config2), ("cfg4", wl.config4)])
def test_golden_matches_generator_and_tolerance(name, gen):
    """The stored solutions belong to the current seeded geometry, reached the
    solver tolerance, and have the sizes of the workload."""
    z = _golden(name)
    dom, gam = gen()
    assert np.allclose(z["eta_checksum"], [dom.eta.real.sum(), dom.eta.imag.sum(), dom.N], rtol=0, atol=1e-9)
    assert z["mu"].shape == (dom.N,) and z["h"].shape == (dom.N,)
    assert float(np.max(z["relres"])) < 1e-14
    assert np.all(np.isfinite(z["mu"])) and np.all(np.isfinite(z["h"]))


def test_golden_cfg4_gradient_consistent():
    """dL/dgamma of the stored gradient: L is quadratic in h, and the stored loss
    equals sum_k h_k^2 of the stored h."""
    z = _golden("cfg4")
    if "g_coef" not in z.files:
        pytest.skip("gradient not written yet")
    n = 2048
    L, _ = og.mean_square_loss(z["h"], n)
    assert abs(L - float(z["loss"])) <= 1e-14 * abs(L)
    assert float(np.max(z["lam_relres"])) < 1e-14
    assert z["g_coef"].shape == (4, 16) and np.all(np.isfinite(z["g_gam"]))


def test_golden_cfg3_matches_generator():
    z = _golden("cfg3")
    for d in range(64):
        if f"d{d}_checksum" not in z.files:
            pytest.skip("batched reference incomplete")
        dom, gam = wl.batch_domain(d)
        assert np.allclose(z[f"d{d}_checksum"], [dom.eta.real.sum(), dom.eta.imag.sum(), dom.N], rtol=0, atol=1e-9)
        cols = z[f"d{d}_cols"]
        assert np.allclose(z[f"d{d}_gam_max"], np.max(np.abs(gam[:, cols]), axis=0), rtol=1e-15, atol=0)
        if str(z[f"d{d}_route"]) == "mf":
            assert float(np.max(z[f"d{d}_relres"])) < 1e-14
