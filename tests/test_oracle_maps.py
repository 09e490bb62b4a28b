"""Pins of the circular-slit map oracle (oracle/maps.py).

On the five-circle domain of Example 2 (alpha = 0 in G): the boundary values
must be those of a function analytic in G (their Cauchy integral vanishes
outside G), with its zero at alpha and a positive derivative there, which the
Cauchy integral formula of Sec. 7 (an independent oracle) recovers from the
boundary values alone; h must be constant on each component; and the domain's
symmetry under z -> i z gives the four slits one radius."""
import numpy as np
import pytest

import workloads as wl
from oracle import nystrom as orc
from oracle.fcau import cauchy_sums, fcau
from oracle.maps import circular_slit_map


def test_boundary_values_are_those_of_an_analytic_function():
    # for f analytic in G, the Cauchy integral of its boundary values vanishes at
    # every point outside the closure of G (outside the unit circle, inside the holes)
    n = 256
    d = wl.example2_circles(n, 0.1)
    f, R, mu, h = circular_slit_map(d.eta, d.etap, 0.0, n)
    s2 = 2.0 + 2.0 * np.sqrt(2.0)
    off = (2.0 - 0.1) / s2
    holes = [off * (1 + 1j), off * (-1 + 1j), off * (-1 - 1j), off * (1 - 1j)]
    zout = np.array([1.5, -2.0j, 1.2 + 1.2j] + holes)
    P = cauchy_sums(d.eta, f * d.etap, zout) / (n * 1j)
    assert np.max(np.abs(P)) < 1e-10
    # a slip in the formula (the sign of mu) breaks it
    g = np.exp(-orc.component_means(h, n)[0]) * d.eta * np.exp(-np.log(np.abs(d.eta)) +
                                                                np.repeat(orc.component_means(h, n), n) - 1j * mu)
    assert np.max(np.abs(cauchy_sums(d.eta, g * d.etap, zout) / (n * 1j))) > 1e-3


def test_symmetric_domain_has_equal_radii():
    # Example 2's domain is invariant under z -> i z and alpha = 0 is fixed, so the
    # four inner circles map to slits of one radius
    n = 256
    d = wl.example2_circles(n, 0.1)
    f, R, mu, h = circular_slit_map(d.eta, d.etap, 0.0, n)
    assert np.max(np.abs(R[1:] - R[1])) < 1e-12


def test_example2_map_is_analytic_with_zero_at_alpha():
    n = 256
    d = wl.example2_circles(n, 0.1)
    alpha = 0.0
    f, R, mu, h = circular_slit_map(d.eta, d.etap, alpha, n)
    # h constant on every component, radii inside the unit disc
    spread = np.max(np.abs(h - np.repeat(orc.component_means(h, n), n)))
    assert spread < 1e-10
    assert np.all(R[1:] < 1.0) and np.all(R[1:] > 0.0)
    # |f| = 1 on the outer circle and R_j on the others (by construction), and the
    # Cauchy integral of the boundary values reproduces f(alpha) = 0 and, at
    # interior points, values of modulus below 1
    assert np.max(np.abs(np.abs(f[:n]) - 1.0)) < 1e-12
    z = np.array([alpha, 0.05 + 0.02j, -0.3j, 0.6])
    fz = fcau(d.eta, d.etap, f, z, n)
    assert abs(fz[0]) < 1e-10
    assert np.all(np.abs(fz[1:]) < 1.0)


def test_map_derivative_at_alpha_is_positive():
    # f(z)/(z - alpha) is analytic and equals f'(alpha) > 0 at alpha
    n = 256
    d = wl.example2_circles(n, 0.1)
    f, R, mu, h = circular_slit_map(d.eta, d.etap, 0.0, n)
    q = fcau(d.eta, d.etap, f / d.eta, np.array([0.0]), n)[0]
    assert abs(q.imag) < 1e-10 and q.real > 0.0


# ---------------------------------------------------------------- circular and radial slits
# Example 3's second target: theta = (pi/2, 0, pi/2, 0, pi/2) on Example 2's domain.
# The domain and this theta are invariant under z -> -z and under the reflection
# z -> i conj(z) (across the line y = x), and alpha = 0 is fixed by both; the map is
# unique under f(0) = 0, f'(0) > 0, so f(-z) = -f(z) and f(i conj z) = i conj f(z).
# The radial slits of the circles centred on y = x therefore lie on that line, at
# angles pi/4 and -3 pi/4, and the two circular slits share one radius.
from oracle.maps import slit_map  # noqa: E402

THETA_EX3 = np.array([np.pi / 2, 0.0, np.pi / 2, 0.0, np.pi / 2])


def _holes(eps):
    s2 = 2.0 + 2.0 * np.sqrt(2.0)
    off = (2.0 - eps) / s2
    return [off * (1 + 1j), off * (-1 + 1j), off * (-1 - 1j), off * (1 - 1j)]


def test_radial_slit_angles_and_radii_from_symmetry():
    n = 256
    d = wl.example2_circles(n, 0.1)
    f, level, mu, h = slit_map(d.eta, d.etap, 0.0, THETA_EX3, n)
    assert level[0] == 0.0
    # radial slits: arg f is constant, at the angle the symmetry fixes
    for k, ang in ((1, np.pi / 4), (3, -3 * np.pi / 4)):
        seg = f[k * n:(k + 1) * n]
        assert np.max(np.abs(np.angle(seg * np.exp(-1j * ang)))) < 1e-12
        assert abs(np.angle(np.exp(-1j * level[k]) * np.exp(-1j * ang))) < 1e-12
        assert np.all(np.abs(seg) < 1.0)
    # circular slits: one radius, |f| equal to it along the component
    assert abs(level[2] - level[4]) < 1e-12
    for k in (2, 4):
        assert np.max(np.abs(np.abs(f[k * n:(k + 1) * n]) - np.exp(level[k]))) < 1e-12
    assert np.max(np.abs(np.abs(f[:n]) - 1.0)) < 1e-12
    # f(-z) = -f(z): node p of circle 1 and node p + n/2 of circle 3 are z and -z
    f1, f3 = f[n:2 * n], f[3 * n:4 * n]
    assert np.max(np.abs(f3 - (-np.roll(f1, -n // 2)))) < 1e-12
    # h constant on every component
    assert np.max(np.abs(h - np.repeat(orc.component_means(h, n), n))) < 1e-10


def test_radial_slit_map_is_analytic_with_zero_at_alpha():
    n = 256
    d = wl.example2_circles(n, 0.1)
    f, level, mu, h = slit_map(d.eta, d.etap, 0.0, THETA_EX3, n)
    zout = np.array([1.5, -2.0j, 1.2 + 1.2j] + _holes(0.1))
    assert np.max(np.abs(cauchy_sums(d.eta, f * d.etap, zout) / (n * 1j))) < 1e-10
    fz = fcau(d.eta, d.etap, f, np.array([0.0, 0.3j, -0.5 + 0.1j]), n)
    assert abs(fz[0]) < 1e-10 and np.all(np.abs(fz[1:]) < 1.0)
    q = fcau(d.eta, d.etap, f / d.eta, np.array([0.0]), n)[0]
    assert abs(q.imag) < 1e-10 and q.real > 0.0
    # dividing by rot instead of multiplying (a plausible slip) breaks analyticity
    rot = np.repeat(np.exp(1j * (np.pi / 2 - THETA_EX3)), n)
    hb = np.repeat(orc.component_means(h, n), n)
    gam = -np.real(rot * (np.log(np.abs(d.eta)) + 1j * np.concatenate(
        [np.unwrap(np.angle(d.eta[k * n:(k + 1) * n])) for k in range(5)])))
    g = np.exp(-hb[0]) * d.eta * np.exp((gam + hb + 1j * mu) * rot)
    assert np.max(np.abs(cauchy_sums(d.eta, g * d.etap, zout) / (n * 1j))) > 1e-3


def test_all_radial_slits_point_at_the_centres():
    # theta = 0 on every inner circle: the disc with four radial slits; the domain's
    # rotation by pi/2 and its reflections put each slit on the ray through its circle's centre
    n = 256
    d = wl.example2_circles(n, 0.1)
    theta = np.array([np.pi / 2, 0.0, 0.0, 0.0, 0.0])
    f, level, mu, h = slit_map(d.eta, d.etap, 0.0, theta, n)
    for k, c in enumerate(_holes(0.1), start=1):
        seg = f[k * n:(k + 1) * n]
        assert np.max(np.abs(np.angle(seg / c))) < 1e-12
        assert np.all(np.abs(seg) < 1.0)


def test_theta_pi_over_2_is_the_circular_slit_map():
    n = 128
    d = wl.example2_circles(n, 0.05)
    f, level, _, _ = slit_map(d.eta, d.etap, 0.0, np.full(5, np.pi / 2), n)
    fc, R, _, _ = circular_slit_map(d.eta, d.etap, 0.0, n)
    assert np.max(np.abs(f - fc)) < 1e-14 and np.max(np.abs(np.exp(level) - R)) < 1e-14


# ------------------------------------------------------------ closed forms, one circle
def _circle_nodes(n, ccw):
    t = 2 * np.pi * np.arange(n) / n
    e = np.exp(1j * t) if ccw else np.exp(-1j * t)
    return e, (1j if ccw else -1j) * e


def test_disc_map_is_the_moebius_map():
    # the unit disc: f(z) = (z - alpha) / (1 - conj(alpha) z) (f(alpha) = 0, f'(alpha) > 0)
    n = 128
    eta, etap = _circle_nodes(n, True)
    for alpha in (0.0, 0.3 + 0.4j, -0.6j):
        f, level, _, _ = slit_map(eta, etap, alpha, np.array([np.pi / 2]), n)
        assert np.max(np.abs(f - (eta - alpha) / (1 - np.conj(alpha) * eta))) < 1e-12
        assert level[0] == 0.0


@pytest.mark.parametrize("alpha", [2.0, 1.5 - 0.7j, -3.0j])
def test_exterior_of_the_circle_closed_forms(alpha):
    # |z| > 1 onto the plane with one slit, F(alpha) = 0, F(z) = z + O(1):
    #   circular slit: F = z (z - alpha) / (z - 1/conj(alpha)), radius |alpha|
    #   radial slit:   F = z + e^{2 i phi} / z - e^{i phi} (|alpha| + 1/|alpha|), alpha = |alpha| e^{i phi}
    #                  (a Joukowski map), on the ray at angle phi + pi
    n = 256
    eta, etap = _circle_nodes(n, False)
    F, level, _, _ = slit_map(eta, etap, alpha, np.array([np.pi / 2]), n, bounded=False)
    assert np.max(np.abs(F - eta * (eta - alpha) / (eta - 1 / np.conj(alpha)))) < 1e-11
    assert abs(level[0] - np.log(abs(alpha))) < 1e-12
    F, level, _, _ = slit_map(eta, etap, alpha, np.array([0.0]), n, bounded=False)
    ph = np.angle(alpha)
    ex = eta + np.exp(2j * ph) / eta - np.exp(1j * ph) * (abs(alpha) + 1 / abs(alpha))
    assert np.max(np.abs(F - ex)) < 1e-11
    assert abs(np.angle(np.exp(-1j * level[0]) * np.exp(-1j * (ph + np.pi)))) < 1e-12


# ------------------------------------------------------------ Example 4 (unbounded)
EX4_CENTRES = np.array([0.0, 1 + 1j, -1 + 1j, -1 - 1j, 1 - 1j])


def _hole_sums(d, F, z):
    # (1/2 pi i) int_Gamma (F - eta)/(eta - z) d eta at points z inside the holes: for F - z
    # analytic in the unbounded G (bounded at infinity) this is -(F - z)(infinity), one
    # constant for every hole
    return -cauchy_sums(d.eta, (F - d.eta) * d.etap, z) / (d.n * 1j)


def test_example4_map_is_analytic_with_zero_at_alpha():
    n = 256
    d = wl.example4_circles(n, 0.1)
    alpha = 2.0 + 2.0j
    F, level, mu, h = slit_map(d.eta, d.etap, alpha, THETA_EX3, n, bounded=False)
    P = _hole_sums(d, F, EX4_CENTRES + 0.05)
    assert np.max(np.abs(P - P[0])) < 1e-10
    # Cauchy's formula at alpha with (F - z)(infinity) = -P: F(alpha) = 0
    Fa = alpha - P[0] - cauchy_sums(d.eta, (F - d.eta) * d.etap, np.array([alpha]))[0] / (n * 1j)
    assert abs(Fa) < 1e-10
    # the slit conditions, and h constant on every component
    for k in range(5):
        seg = F[k * n:(k + 1) * n]
        if THETA_EX3[k] == 0.0:
            assert np.max(np.abs(np.angle(seg * np.exp(1j * level[k])))) < 1e-10
        else:
            assert np.max(np.abs(np.log(np.abs(seg)) - level[k])) < 1e-10
    assert np.max(np.abs(h - np.repeat(orc.component_means(h, n), n))) < 1e-9
    # multiplying by rot instead of dividing breaks analyticity
    rot = np.repeat(np.exp(1j * (np.pi / 2 - THETA_EX3)), n)
    dz = d.eta - alpha
    arg = np.concatenate([np.unwrap(np.angle(dz[k * n:(k + 1) * n])) for k in range(5)])
    gam = -np.real(rot * (np.log(np.abs(dz)) + 1j * arg))
    G = dz * np.exp((gam + np.repeat(orc.component_means(h, n), n) + 1j * mu) * rot)
    Q = _hole_sums(d, G, EX4_CENTRES + 0.05)
    assert np.max(np.abs(Q - Q[0])) > 1e-3


def test_example4_symmetry():
    # z -> i conj(z) fixes alpha = 2 + 2i, the domain and this theta, and F(z) = z + O(1):
    # so F(i conj z) = i conj F(z): the radial slits of the circles on y = x lie on that
    # line, and the circular slits of -1 + i and 1 - i share one radius. With
    # theta = pi/2 everywhere and alpha = 2 (fixed by z -> conj z), conjugate circles
    # share a radius.
    n = 256
    d = wl.example4_circles(n, 0.1)
    F, level, _, _ = slit_map(d.eta, d.etap, 2.0 + 2.0j, THETA_EX3, n, bounded=False)
    assert abs(level[2] - level[4]) < 1e-10
    for k in (1, 3):
        assert abs(np.exp(-2j * level[k]) - 1j) < 1e-10      # 2 arg F = pi/2 (mod 2 pi)
    F, level, _, _ = slit_map(d.eta, d.etap, 2.0, np.full(5, np.pi / 2), n, bounded=False)
    assert abs(level[1] - level[4]) < 1e-10 and abs(level[2] - level[3]) < 1e-10
