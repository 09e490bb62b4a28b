"""Pins of the circular-slit map oracle (oracle/maps.py).

On the five-circle domain of Example 2 (alpha = 0 in G): the boundary values
must be those of a function analytic in G (their Cauchy integral vanishes
outside G), with its zero at alpha and a positive derivative there, which the
Cauchy integral formula of Sec. 7 (an independent oracle) recovers from the
boundary values alone; h must be constant on each component; and the domain's
symmetry under z -> i z gives the four slits one radius."""
import numpy as np

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
