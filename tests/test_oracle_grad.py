"""Pins of the gradient oracle (oracle.gradient) against central finite
differences of the dense forward computation (LU solves, no adjoint): the
bilinear-form geometry gradients for each operator, the gamma gradient, the
mu cotangent, and the full chain to the Fourier coefficients."""
import numpy as np
import pytest

import workloads as wl
from oracle import gradient as og
from oracle import nystrom as ny


def _small_fourier(m1=4, n=64, seed=7):
    coeffs, kmin = wl.fourier_perturbed_circles(m1, n, [wl.SEED, 40, seed], side=3.0, dmin=1.0)
    return coeffs, kmin


def _rand_geom(seed=0, n=32, m1=3):
    coeffs, kmin = _small_fourier(m1, n, seed)
    eta, etap, _ = og.fourier_nodes(coeffs, kmin, n)
    rng = np.random.default_rng(seed)
    A = 1.0 + 0.3 * (rng.normal(size=eta.shape) + 1j * rng.normal(size=eta.shape))
    return eta, etap, A, n, rng


def _bilinear(op, u, v, eta, etap, A, n):
    Aop, Cop = ny.fbie_operators(eta, etap, A, n)
    return float(u @ ((Aop if op == "FB" else Cop) @ v))


@pytest.mark.parametrize("op", ["FB", "FC"])
def test_bilinear_geom_grad_matches_fd(op):
    eta, etap, A, n, rng = _rand_geom(1)
    N = eta.shape[0]
    u, v = rng.normal(size=N), rng.normal(size=N)
    ge, gp, ga = og.bilinear_geom_grad(eta, etap, A, n, [(op, u, v)])
    h = 1e-6
    for which in range(3):
        d = rng.normal(size=N) + 1j * rng.normal(size=N)
        args = [eta, etap, A]
        plus = list(args)
        minus = list(args)
        plus[which] = args[which] + h * d
        minus[which] = args[which] - h * d
        fd = (_bilinear(op, u, v, *plus, n) - _bilinear(op, u, v, *minus, n)) / (2 * h)
        g = (ge, gp, ga)[which]
        an = float(np.real(np.sum(np.conj(g) * d)))
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an)), (op, which, fd, an)


def test_bilinear_rows_match_dense():
    eta, etap, A, n, rng = _rand_geom(2)
    N = eta.shape[0]
    terms = [("FB", rng.normal(size=N), rng.normal(size=N)), ("FC", rng.normal(size=N), rng.normal(size=N)),
             ("FB", rng.normal(size=N), rng.normal(size=N))]
    dense = og.bilinear_geom_grad(eta, etap, A, n, terms)
    idx = [0, 5, 31, 32, 77, N - 1]
    rows = og.bilinear_geom_grad_rows(eta, etap, A, n, terms, idx)
    for a, b in zip(dense, rows):
        assert np.max(np.abs(a[idx] - b)) <= 1e-13 * np.max(np.abs(a))


def test_fbie_vjp_gamma_and_mu_cotangent():
    coeffs, kmin = _small_fourier()
    n = 64
    eta, etap, _ = og.fourier_nodes(coeffs, kmin, n)
    A = np.ones_like(eta)
    N = eta.shape[0]
    rng = np.random.default_rng(3)
    gam = (eta ** 2).real
    g_mu = rng.normal(size=N)
    g_h = rng.normal(size=N)

    def L(g):
        mu, h = ny.fbie(eta, etap, A, g, n)
        return float(g_mu @ mu + g_h @ h)

    r = og.fbie_vjp(eta, etap, A, gam, n, g_mu=g_mu, g_h=g_h)
    for _ in range(4):
        d = rng.normal(size=N)
        fd = (L(gam + 1e-6 * d) - L(gam - 1e-6 * d)) / 2e-6
        an = float(r["g_gam"] @ d)
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))
    # L is linear in gamma, so the gradient is exactly -(Aop^-T g_mu ...) composed:
    # check against the explicit dense inverse as well
    Aop, Cop = ny.fbie_operators(eta, etap, A, n)
    Ai = np.linalg.inv(Aop)
    dmu = -Ai @ Cop                                   # dmu/dgam
    dh = 0.5 * (Cop @ dmu - Aop)                      # dh/dgam
    assert np.allclose(r["g_gam"], dmu.T @ g_mu + dh.T @ g_h, rtol=0, atol=1e-10 * np.max(np.abs(r["g_gam"])))


def test_fbie_loss_coefficient_gradient_fd():
    coeffs, kmin = _small_fourier()
    n = 64
    eta, _, _ = og.fourier_nodes(coeffs, kmin, n)
    gam = (eta ** 2).real
    L0, g_gam, g_c = og.fbie_loss_and_grad(coeffs, kmin, n, gam)
    assert L0 > 0
    rng = np.random.default_rng(4)
    scale = np.max(np.abs(g_c))
    h = 1e-6
    picks = [(j, k) for j in range(coeffs.shape[0]) for k in rng.choice(coeffs.shape[1], 3, replace=False)]
    for j, k in picks:
        for part in (1.0, 1j):
            cp = coeffs.copy()
            cm = coeffs.copy()
            cp[j, k] += h * part
            cm[j, k] -= h * part
            fd = (og.fbie_loss(cp, kmin, n, gam) - og.fbie_loss(cm, kmin, n, gam)) / (2 * h)
            an = g_c[j, k].real if part == 1.0 else g_c[j, k].imag
            assert abs(fd - an) <= 2e-7 * scale, (j, k, part, fd, an)


def test_fourier_nodes_match_generator():
    coeffs, kmin = _small_fourier(3, 32)
    dom = wl.domain_from_fourier(coeffs, kmin, 32)
    eta, etap, etapp = og.fourier_nodes(coeffs, kmin, 32)
    assert np.max(np.abs(eta - dom.eta)) < 1e-13
    assert np.max(np.abs(etap - dom.etap)) < 1e-13
    assert np.max(np.abs(etapp - dom.etapp)) < 1e-12
