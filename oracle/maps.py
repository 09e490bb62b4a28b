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
