"""Pins of the no-subtraction variant of the oracle (Example 2's comparison).

The diagonal limit (e:N-tt) is checked against the kernel (e:N) itself at
parameters next to the diagonal; on the disk both variants are exact and
equal; on a smooth annulus both converge to the closed-form solution; and on
the paper's Example 2 geometry with close circles the subtracted form stays
accurate while the plain trapezoidal rule loses all accuracy (the effect the
paper reports)."""
import numpy as np

import workloads as wl
from oracle import nystrom as orc
from workloads import geometry as geo


def test_n_diagonal_is_the_kernel_limit():
    c, a, b, phi, alpha = 0.1 + 0.2j, 1.0, 0.6, 0.3, 0.05

    def ev(t):
        e, d1, d2 = geo.ellipse(np.array([t]), c, a, b, phi, ccw=True)
        return e[0], d1[0], d2[0]

    def kernel(s, t):            # N(s, t) of eq. (e:N) with A = eta - alpha
        es, ps, _ = ev(s)
        et, pt, _ = ev(t)
        return (1 / np.pi) * ((es - alpha) / (et - alpha) * pt / (et - es)).imag

    n = 100
    for t in (0.0, 0.7, 2.9, 5.1):
        e, p, pp = ev(t)
        lim = orc.n_diagonal(np.array([p]), np.array([pp]), np.array([e - alpha]), np.array([p]), n)[0]
        # the symmetric mean removes the O(h) term; at h = 1e-4 the O(h^2) term and
        # the cancellation in the kernel are both below 1e-9 (a wrong factor 1/2 on
        # either part of (e:N-tt) would be off by 1e-4..1e-3)
        h = 1e-4
        near = 0.5 * (kernel(t + h, t) + kernel(t - h, t)) * (2 * np.pi / n)
        assert abs(near - lim) < 1e-9


def test_disk_both_variants_agree():
    n = 32
    d = wl.disk(n)
    gam, mu_ex = wl.closed_form_rhs(d, lambda z: z ** 3 + 0.5)
    mu_s, h_s = orc.fbie(d.eta, d.etap, d.A, gam, n)
    mu_u, h_u = orc.fbie_unsubtracted(d.eta, d.etap, d.etapp, d.A, d.Ap, gam, n)
    assert np.max(np.abs(mu_u - mu_s)) < 1e-13
    assert np.max(np.abs(h_u - h_s)) < 1e-13


def test_annulus_converges_without_subtraction():
    # smooth, well separated boundaries: the plain trapezoidal rule is accurate too
    for n in (64, 128):
        d = wl.annulus(n)
        gam, mu_ex = wl.closed_form_rhs(d, lambda z: 1.0 / (z - 0.1) + z)
        mu_u, h_u = orc.fbie_unsubtracted(d.eta, d.etap, d.etapp, d.A, d.Ap, gam, n)
        assert np.max(np.abs(mu_u - mu_ex)) < 1e-12
        assert np.max(np.abs(h_u)) < 1e-10   # h = 0 for gamma = Re[A f] (eq. (e:ex-gam))


def test_example2_close_circles_need_the_subtraction():
    n = 128
    d = wl.example2_circles(n, 0.01)
    f = lambda z: 1.0 / (z - 2.0) + np.sin(z)
    gam, mu_ex = wl.closed_form_rhs(d, f)
    mu_s, _ = orc.fbie(d.eta, d.etap, d.A, gam, n)
    mu_u, _ = orc.fbie_unsubtracted(d.eta, d.etap, d.etapp, d.A, d.Ap, gam, n)
    assert np.max(np.abs(mu_s - mu_ex)) < 1e-12
    assert np.max(np.abs(mu_u - mu_ex)) > 1e-2


def test_fbiead_unsubtracted_invariant():
    # (I + N* + J) phi = 1 has J phi = 1 (phi the constant-mode solution, Example 1's
    # invariant) for the exact operator; the discrete one approaches it as n grows
    errs = []
    for n in (64, 128):
        d = wl.annulus(n)
        phi = orc.fbiead_unsubtracted(d.eta, d.etap, d.etapp, d.A, d.Ap, np.ones(d.eta.shape[0]), n)
        errs.append(np.max(np.abs(orc.component_means(phi, n) - 1.0)))
    assert errs[1] < 1e-10 and errs[1] <= errs[0]
