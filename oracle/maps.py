"""CPU FP64 oracle for the conformal map onto the disc with circular slits.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call, link or
execute anything under ``oracle/``; only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.

The paper (Example 3) computes this map from FBIE with theta = pi/2 by a method
it cites; the steps below are derived from the Riemann-Hilbert problem that
FBIE solves (Sec. 2: given gamma, find g analytic in G and h piecewise
constant with Re[A g] = gamma + h; mu = Im[A g] on the boundary):

  * G bounded, outer boundary Gamma_0, alpha in G (A = eta - alpha is then
    the admissible choice of eq. (e:A) with theta = pi/2). Write the map as
    f(z) = c (z - alpha) exp((z - alpha) g(z)), c > 0, g analytic in G.
  * |f| = R_j on Gamma_j (R_0 = 1) becomes, with A = eta - alpha (theta = pi/2
    in eq. (e:A)) and gamma = -log|eta - alpha|,
        Re[A g] = gamma + (log R_j - log c) = gamma + h_j.
  * So A g = gamma + h + i mu on the boundary, and
        f(eta) = c (eta - alpha) exp(gamma + h + i mu),  c = exp(-h_0),
        R_j = exp(h_j - h_0).

The discrete h is only approximately constant on each component; the map
takes h_j as its mean over component j (the reading used for h_k elsewhere).

The disc with circular and radial slits (Example 3, theta = (pi/2, 0, pi/2, 0,
pi/2)) follows the same way with a piecewise constant theta, theta_0 = pi/2:
write rot = exp(i (pi/2 - theta)), so A = rot (eta - alpha) (eq. (e:A)), and
ask Re[rot log f] to be constant on each Gamma_j. With
f = c (z - alpha) exp((z - alpha) g) that is Re[A g] = gamma + h_j with

    gamma = -Re[rot log(eta - alpha)],

log(eta - alpha) taken continuous along each component (alpha lies in G, so
its argument returns to its start around every inner component and gains 2 pi
around Gamma_0). Then (eta - alpha) g = (gamma + h + i mu) / rot,

    f(eta) = exp(-h_0) (eta - alpha) exp((gamma + h + i mu) / rot),

and Re[rot log f] = h_j - h_0 sin(theta_j) =: level_j on Gamma_j. For
theta_j = pi/2 that is log R_j (a circular slit of radius R_j); for
theta_j = 0 it is -arg f (a radial slit at angle -level_j); any other constant
gives an arc of a logarithmic spiral. The integral identity behind the
discrete FBIE (eq. (e:NM-const)) holds for piecewise constant theta as well:
the contribution of a component other than the one holding s cancels by
residues, whatever its phase.

Unbounded G (Example 4): A = rot (eq. (e:A)) and the solution of the
Riemann-Hilbert problem vanishes at infinity. Write the map onto the extended
plane with slits as F(z) = (z - alpha) exp(g(z)), g analytic in G with
g(infinity) = 0, so F(alpha) = 0 and F(z) = z + O(1) at infinity; then
Re[rot g] = gamma + h_j with the same gamma (alpha lies outside every hole,
so log(eta - alpha) is continuous along every component), and

    F(eta) = (eta - alpha) exp((gamma + h + i mu) / rot),  level_j = h_j.

Every component becomes a slit; theta_0 is free.
"""
from __future__ import annotations

import numpy as np

from . import nystrom as orc


def circular_slit_map(eta, etap, alpha, n):
    """Boundary values f(eta_i) of the map onto the unit disc with circular
    slits (f(alpha) = 0, f'(alpha) > 0) and the slit radii R_j (R_0 = 1).

    eta, etap: (N,) complex, component-major, Gamma_0 (ccw) first. Returns
    (f, R, mu, h) with h the per-node values of FBIE's h."""
    eta = np.asarray(eta, np.complex128)
    etap = np.asarray(etap, np.complex128)
    A = eta - alpha
    gam = -np.log(np.abs(eta - alpha))
    mu, h = orc.fbie(eta, etap, A, gam, n)
    hbar = orc.component_means(h, n)
    hn = np.repeat(hbar, n)
    f = np.exp(-hbar[0]) * (eta - alpha) * np.exp(gam + hn + 1j * mu)
    R = np.exp(hbar - hbar[0])
    return f, R, mu, h


def slit_map(eta, etap, alpha, theta, n, bounded=True):
    """Boundary values of the map onto the unit disc (bounded G; theta_0 = pi/2,
    f(alpha) = 0, f'(alpha) > 0) or the extended plane (unbounded G; F(alpha) = 0,
    F(z) = z + O(1) at infinity) with slits on the curves
    Re[exp(i (pi/2 - theta_j)) log w] = level_j (circular for theta_j = pi/2,
    radial for theta_j = 0).

    theta: (m1,) real. Returns (f, level, mu, h); level_0 = 0 for bounded G."""
    eta = np.asarray(eta, np.complex128)
    etap = np.asarray(etap, np.complex128)
    theta = np.asarray(theta, np.float64)
    m1 = eta.shape[0] // n
    d = eta - alpha
    arg = np.concatenate([np.unwrap(np.angle(d[k * n:(k + 1) * n])) for k in range(m1)])
    rot = np.repeat(np.exp(1j * (np.pi / 2 - theta)), n)
    A = rot * d if bounded else rot
    gam = -np.real(rot * (np.log(np.abs(d)) + 1j * arg))
    mu, h = orc.fbie(eta, etap, A, gam, n)
    hbar = orc.component_means(h, n)
    if not bounded:
        return d * np.exp((gam + np.repeat(hbar, n) + 1j * mu) / rot), hbar, mu, h
    f = np.exp(-hbar[0]) * d * np.exp((gam + np.repeat(hbar, n) + 1j * mu) / rot)
    level = hbar - hbar[0] * np.sin(theta)
    return f, level, mu, h
