"""Checks of the seeded input generators: derivatives, orientation, grading,
non-overlap and determinism."""
import numpy as np
import pytest

import workloads as wl
from workloads import geometry as geo


def _fd_check(curve, tol=1e-6):
    t = np.linspace(0.1, 6.1, 37)
    h = 1e-5
    e0, d1, d2 = curve(t)
    ep, d1p, _ = curve(t + h)
    em, d1m, _ = curve(t - h)
    assert np.max(np.abs((ep - em) / (2 * h) - d1)) < tol * max(1, np.max(np.abs(d1)))
    assert np.max(np.abs((d1p - d1m) / (2 * h) - d2)) < tol * max(1, np.max(np.abs(d2)))


def _signed_area(eta, etap, n):
    # (1/2) int Im(conj(eta) eta') dt by the trapezoidal rule
    return 0.5 * np.sum((np.conj(eta) * etap).imag) * 2 * np.pi / n


def test_curve_derivatives():
    _fd_check(lambda t: geo.circle(t, 0.3 + 0.1j, 0.7, True))
    _fd_check(lambda t: geo.ellipse(t, 0.1j, 0.4, 0.2, 0.7, ccw=False))
    rng = np.random.default_rng(0)
    c = (rng.normal(size=16) + 1j * rng.normal(size=16)) * 0.01
    c[7] = 0.5
    c[8] = 1.0
    _fd_check(lambda t: geo.fourier_curve(t, c, -7, ccw=False))


@pytest.mark.parametrize("p", [2, 3, 5])
def test_kress_omega(p):
    t = np.linspace(0, 2 * np.pi, 2001)
    om, dom, ddom = geo.kress_omega(t, p)
    assert abs(om[0]) < 1e-15 and abs(om[-1] - 2 * np.pi) < 1e-12
    assert np.all(np.diff(om) > 0)                 # strictly increasing
    assert abs(dom[0]) < 1e-12 and abs(dom[-1]) < 1e-12
    h = 1e-6
    tt = np.linspace(0.2, 6.0, 29)
    for f, df in ((lambda x: geo.kress_omega(x, p)[0], lambda x: geo.kress_omega(x, p)[1]),
                  (lambda x: geo.kress_omega(x, p)[1], lambda x: geo.kress_omega(x, p)[2])):
        fd = (f(tt + h) - f(tt - h)) / (2 * h)
        assert np.max(np.abs(fd - df(tt))) < 1e-6 * max(1, np.max(np.abs(df(tt))))


def test_graded_polygon():
    verts = np.exp(1j * (2 * np.pi * np.arange(5) / 5 + 0.1))
    poly = geo.RoundedPolygon(verts, rad=0.1, ccw=False)
    _fd_check(lambda t: poly(t), tol=1e-4)
    n = 512
    t = geo.nodes(n)
    eta, etap, etapp = geo.graded_polygon(t, poly, 3)
    # closed curve, clockwise (negative signed area), eta' = 0 at the corner parameter t = 0
    assert abs(eta[0] - poly(np.array([0.0]))[0][0]) < 1e-14
    assert _signed_area(eta, etap, n) < 0
    assert abs(etap[0]) < 1e-12
    # the graded derivative is consistent with finite differences away from corners
    _fd_check(lambda s: geo.graded_polygon(s, poly, 3), tol=1e-4)


def test_config_orientation_and_determinism():
    d0, g0 = wl.config0()
    d0b, _ = wl.config0()
    assert np.array_equal(d0.eta, d0b.eta)
    areas = [_signed_area(d0.eta[d0.comp(k)], d0.etap[d0.comp(k)], d0.n) for k in range(d0.m1)]
    assert areas[0] > 0 and areas[1] < 0          # outer ccw, inner cw (G on the left)
    d1, g1 = wl.config1(n=64)
    assert d1.m1 == 17 and d1.N == 17 * 64
    for k in range(1, 17):
        assert _signed_area(d1.eta[d1.comp(k)], d1.etap[d1.comp(k)], 64) < 0
    # inner ellipses disjoint from each other and from alpha = 0
    for (c, a, b, _) in d1.meta["ellipses"]:
        assert abs(c) > max(a, b)
    assert np.all(np.isfinite(g1))


def test_close_boundary_workload_prefix():
    """Close-boundary generator: clockwise components, true gaps in
    [1e-3, 1e-2] x size to the anchor, no overlaps, graded polygons with eta' = 0
    at the corner parameter t = 0."""
    d9, g9 = wl.config2(n=256, m1=9)
    assert d9.m1 == 9 and d9.N == 9 * 256 and not d9.bounded
    for k in range(9):
        assert _signed_area(d9.eta[d9.comp(k)], d9.etap[d9.comp(k)], 256) < 0
    kinds = d9.meta["kinds"]
    assert kinds[0] == "poly" and kinds[4] == "poly" and kinds[1] == "ellipse"
    assert abs(d9.etap[0]) < 1e-12               # corner at t = 0 of a graded polygon
    from scipy.spatial import cKDTree
    e = d9.eta.reshape(9, 256)
    for k in range(1, 9):
        others = np.concatenate([e[:k], e[k + 1:]]).ravel()
        dmin, _ = cKDTree(np.c_[others.real, others.imag]).query(np.c_[e[k].real, e[k].imag])
        assert dmin.min() > 3e-4
    shapes = wl.close_shapes(9, [wl.SEED, 2])
    for s in shapes:
        assert s.size > 0.3
