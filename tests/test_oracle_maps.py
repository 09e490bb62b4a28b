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
