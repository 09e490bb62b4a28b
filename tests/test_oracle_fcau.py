"""Pins of the Cauchy-integral oracle (oracle/fcau.py) against closed forms.

The formula of Sec. 7 (eqs. (e:cauchy5)/(e:cauchy6)) must reproduce a function
analytic in G at interior points, to the accuracy of the trapezoidal rule for
the subtracted integrand, which is analytic in eta. The cases are chosen so
that a plausible slip fails one of them: a dropped eta' or wrong F fails every
closed form; a sign error in F or the wrong weight 1/(N i) instead of 1/(n i)
fails the unbounded cases (the bounded ratio cancels both); the plain,
unsubtracted sum fails the points next to the boundary.
"""
import numpy as np

from oracle.fcau import cauchy_sums, fcau


def circle(c, r, n, ccw=True):
    t = 2 * np.pi * np.arange(n) / n
    s = 1.0 if ccw else -1.0
    e = np.exp(1j * s * t)
    return c + r * e, 1j * s * r * e


def domain(parts, n):
    eta, etap = zip(*(circle(c, r, n, ccw) for c, r, ccw in parts))
    return np.concatenate(eta), np.concatenate(etap)


def test_disk_entire_function():
    n = 64
    eta, etap = domain([(0.0, 1.0, True)], n)
    f = np.exp
    z = np.array([0.0, 0.3 + 0.2j, -0.5j, 0.9, 0.999 * np.exp(0.7j), 1e-12 + 0.99999j])
    got = fcau(eta, etap, f(eta), z, n)
    assert np.max(np.abs(got - f(z))) < 1e-13


def test_plain_sum_is_not_enough_near_the_boundary():
    # the unsubtracted trapezoidal Cauchy sum (1/(2 pi i)) sum f eta' / (eta - z) (2 pi / n)
    # loses all accuracy next to the boundary; the ratio form of (e:cauchy4-b) does not
    n = 64
    eta, etap = domain([(0.0, 1.0, True)], n)
    z = np.array([0.999 * np.exp(0.05j)])
    plain = -cauchy_sums(eta, np.exp(eta) * etap, z) / (n * 1j)
    assert abs(plain[0] - np.exp(z[0])) > 1e-3
    assert abs(fcau(eta, etap, np.exp(eta), z, n)[0] - np.exp(z[0])) < 1e-12


def test_annulus_bounded():
    n = 96
    eta, etap = domain([(0.0, 1.0, True), (0.0, 0.3, False)], n)
    f = lambda z: z ** 2 + 1.0 / (z - 0.1)        # pole inside the hole
    z = np.array([0.6, -0.5 + 0.2j, 0.31, 0.995j, -0.7 - 0.3j])
    got = fcau(eta, etap, f(eta), z, n)
    assert np.max(np.abs(got - f(z))) < 1e-12 * np.max(np.abs(f(z)))


def test_exterior_one_hole():
    n = 64
    eta, etap = domain([(0.0, 1.0, False)], n)
    f = lambda z: 1.0 / (z - 0.2) + 2.0
    z = np.array([2.0, 1.5j, 1.001, -1.01 + 0.1j, 30.0 - 40.0j])
    got = fcau(eta, etap, f(eta), z, n, finf=2.0)
    assert np.max(np.abs(got - f(z))) < 1e-12


def test_exterior_two_holes():
    # two components: the weight is 1/(n i) with n nodes per component, not 1/((m+1) n i)
    n = 64
    eta, etap = domain([(-1.5, 0.5, False), (1.5, 0.7, False)], n)
    f = lambda z: 1.0 / (z + 1.4) + 0.5 / (z - 1.6) - 0.3j
    z = np.array([0.0, 3j, -1.5 + 0.55, 2.21, -4.0 + 1.0j])
    got = fcau(eta, etap, f(eta), z, n, finf=-0.3j)
    assert np.max(np.abs(got - f(z))) < 1e-11
    wrong = fcau(eta, etap, f(eta), z, 2 * n, finf=-0.3j)
    assert np.max(np.abs(wrong - f(z))) > 1e-2


def test_constant_function():
    n = 48
    c = 0.7 - 0.2j
    eta, etap = domain([(0.0, 1.0, True), (0.2, 0.25, False)], n)
    z = np.array([0.5, -0.6j, 0.2 + 0.26])
    assert np.max(np.abs(fcau(eta, etap, np.full(eta.shape, c), z, n) - c)) < 1e-14
    eta, etap = domain([(0.0, 1.0, False)], n)
    z = np.array([1.5, 2j, 1.0001])
    assert np.max(np.abs(fcau(eta, etap, np.full(eta.shape, c), z, n, finf=c) - c)) < 1e-14


def test_target_on_a_node_takes_the_node_value():
    n = 32
    eta, etap = domain([(0.0, 1.0, True), (0.0, 0.4, False)], n)
    f = np.exp(eta) + 1j * eta
    z = np.array([eta[5], 0.6, eta[40]])
    got = fcau(eta, etap, f, z, n)
    assert got[0] == f[5] and got[2] == f[40]
    assert abs(got[1] - (np.exp(0.6) + 0.6j)) < 1e-12


def test_columns_are_independent():
    n = 40
    eta, etap = domain([(0.0, 1.0, False), (2.5, 0.5, False)], n)
    F = np.stack([1.0 / (eta - 0.1), eta ** -2, 1.0 / (eta - 2.4) + 1.0], axis=1)
    z = np.array([1.7, -2.0j, 4.0])
    finf = np.array([0.0, 0.0, 1.0])
    got = fcau(eta, etap, F, z, n, finf=finf)
    for q in range(3):
        one = fcau(eta, etap, F[:, q], z, n, finf=finf[q])
        assert np.max(np.abs(got[:, q] - one)) <= 1e-14 * np.max(np.abs(one))
    ref = np.stack([1.0 / (z - 0.1), z ** -2, 1.0 / (z - 2.4) + 1.0], axis=1)
    assert np.max(np.abs(got - ref)) < 1e-10
