"""CPU FP64 oracle for the Cauchy integral formula at interior points.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call, link or
execute anything under ``oracle/``; only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.

What it computes (Sec. 7 of the paper, "Computing the Cauchy integral
formula"): the values f(z_i) of a function analytic in G at points z_i of G,
from the boundary values f_j = f(eta_j) at the trapezoidal nodes, by the
subtracted form of the Cauchy integral (eqs. (e:cauchy2)-(e:cauchy6)). With the
matrix F_ij = 1/(z_i - eta_j) of eq. (e:F),

    P_f = F [f eta'],   P_1 = F [eta']

and

    bounded G:    f(z) = P_f / P_1                                   (e:cauchy6-b)
    unbounded G:  f(z) = (f(inf) - P_f/(n i)) / (1 - P_1/(n i))     (e:cauchy6-u)

where n is the number of nodes on each boundary component (the trapezoidal
weight 2 pi/n times the 1/(2 pi i) of the Cauchy formula). The subtraction of
f(z) under the integral, which makes the integrand analytic at eta = z, is what
turns the plain sums into these ratios.

Readings where the text is silent or garbled:
  * the integrand of eq. (e:cau-2) is printed as (f(eta) - z)/(eta - z); it is
    (f(eta) - f(z))/(eta - z), the integrand of (e:cauchy2);
  * a target equal to a node eta_k (the formula's two sums are infinite there)
    takes the limit of the ratio, f_k.
"""
from __future__ import annotations

import numpy as np


def cauchy_sums(eta, w, z, block=2048):
    """(F w)_i = sum_j w_j / (z_i - eta_j) for every target, eq. (e:F).

    w: (N,) or (N, q). Targets are taken in blocks of `block` rows; each
    row's sum is one matrix-vector product (a library primitive)."""
    eta = np.asarray(eta, np.complex128)
    z = np.asarray(z, np.complex128)
    w = np.asarray(w, np.complex128)
    out = np.zeros((z.shape[0],) + w.shape[1:], np.complex128)
    with np.errstate(divide="ignore", invalid="ignore"):
        for a in range(0, z.shape[0], block):
            F = 1.0 / (z[a:a + block, None] - eta[None, :])
            out[a:a + block] = F @ w
    return out


def fcau(eta, etap, f, z, n, finf=None):
    """f at the points z by eqs. (e:cauchy5)/(e:cauchy6).

    eta, etap: (N,) complex nodes and derivatives (N = (m+1) n, component-major).
    f: (N,) or (N, q) complex boundary values. z: (nz,) complex targets in G.
    finf: None for bounded G, else f(infinity) (scalar or (q,)) for unbounded G.
    Returns (nz,) or (nz, q)."""
    eta = np.asarray(eta, np.complex128)
    etap = np.asarray(etap, np.complex128)
    f = np.asarray(f, np.complex128)
    z = np.asarray(z, np.complex128)
    one = f.ndim == 1
    fm = f[:, None] if one else f
    Pf = cauchy_sums(eta, fm * etap[:, None], z)
    P1 = cauchy_sums(eta, etap, z)[:, None]
    with np.errstate(divide="ignore", invalid="ignore"):
        if finf is None:
            out = Pf / P1
        else:
            fi = np.broadcast_to(np.asarray(finf, np.complex128), (fm.shape[1],))
            out = (fi[None, :] - Pf / (n * 1j)) / (1.0 - P1 / (n * 1j))
    # targets on a node: the limit of the ratio is the node's value
    for i in range(z.shape[0]):
        hit = np.nonzero(eta == z[i])[0]
        if hit.size:
            out[i] = fm[hit[0]]
    return out[:, 0] if one else out
