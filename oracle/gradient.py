"""CPU FP64 oracle for derivatives of the FBIE outputs.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call, link or
execute anything under ``oracle/``; only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.

Setting. With Aop = 2I + diag(B1) - B (eq. (e:sys)) and
Cop = D - diag(D1) + Lhat (eqs. (e:y), (e:bh)), FBIE computes
    mu = -Aop^{-1} Cop gamma,        h = (Cop mu - Aop gamma) / 2.
For a real function L(mu, h) with cotangents g_mu = dL/dmu, g_h = dL/dh,
differentiating both relations gives the reverse-mode rules used here:
    lam     = Aop^{-T} (Cop^T g_h / 2 + g_mu)          (adjoint solve)
    dL/dgam = -Aop^T g_h / 2 - Cop^T lam
    dL      = (g_h/2)^T dCop mu - (g_h/2)^T dAop gamma - lam^T dAop mu - lam^T dCop gamma
for the dependence on the boundary data (eta, eta', A) through B = Im K and
D = Re K, K_ij = (2/n)(A_i/A_j) eta'_j/(eta_j - eta_i) (Lhat depends on n only).

K is holomorphic in each of eta_i, eta_j, eta'_j, A_i, A_j, with
    dK_ij/deta_i = K_ij/(eta_j - eta_i),   dK_ij/deta_j = -K_ij/(eta_j - eta_i),
    dK_ij/deta'_j = (2/n)(A_i/A_j)/(eta_j - eta_i),
    dK_ij/dA_i = K_ij/A_i,                 dK_ij/dA_j = -K_ij/A_j.
A real quantity s = Re F(z) of a complex input z has the gradient
g = ds/dRe z + i ds/dIm z = conj(dF/dz) (the convention of torch.autograd).

Everything is dense (N x N matrices, LAPACK LU), so it is meant for N up to a
few thousand; ``bilinear_geom_grad_rows`` evaluates chosen entries of the
geometric gradient one by one for larger N.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .nystrom import circulant_L, block_diag_repeat, fbie_operators, kernel_matrix, kernel_rows


def _coupling(terms, N):
    """Gamma = dS/dD - i dS/dB for S = sum_t u_t^T Op_t v_t, treating the off-diagonal
    entries of B and D as independent (Op = FB: Aop, Op = FC: Cop).

    u^T (diag(B1) - B) v = sum_{i != j} B_ij u_i (v_i - v_j)
    u^T (D - diag(D1)) v = sum_{i != j} D_ij u_i (v_j - v_i)."""
    GB = np.zeros((N, N))
    GD = np.zeros((N, N))
    for op, u, v in terms:
        if op == "FB":
            GB += u[:, None] * (v[:, None] - v[None, :])
        elif op == "FC":
            GD += u[:, None] * (v[None, :] - v[:, None])
        else:
            raise ValueError(op)
    G = GD - 1j * GB
    np.fill_diagonal(G, 0.0)
    return G


def bilinear_geom_grad(eta, etap, A, n, terms):
    """Gradients of S = sum_t u_t^T Op_t(eta, eta', A) v_t with respect to eta,
    eta' and A (complex, conj-Wirtinger convention). terms: (op, u, v) with op in
    {"FB", "FC"} and real u, v. Since B = Im K = Re(-i K) and D = Re K,
    S = const + Re sum_{i != j} Gamma_ij K_ij with Gamma from ``_coupling``."""
    N = eta.shape[0]
    G = _coupling(terms, N)
    K = kernel_matrix(eta, etap, A, n)
    diff = eta[None, :] - eta[:, None]                 # eta_j - eta_i
    np.fill_diagonal(diff, 1.0)
    GK = G * K
    Q = GK / diff
    dF_deta = Q.sum(axis=1) - Q.sum(axis=0)            # target role (row) and source role (column)
    dKdetap = (2.0 / n) * (A[:, None] / A[None, :]) / diff
    np.fill_diagonal(dKdetap, 0.0)
    dF_detap = (G * dKdetap).sum(axis=0)               # eta'_j enters column j only
    dF_dA = (GK.sum(axis=1) - GK.sum(axis=0)) / A
    return np.conj(dF_deta), np.conj(dF_detap), np.conj(dF_dA)


def bilinear_geom_grad_rows(eta, etap, A, n, terms, idx):
    """Entries idx of the three gradients of ``bilinear_geom_grad``, each from
    row p and column p of Gamma * K alone (O(N) work per entry)."""
    N = eta.shape[0]
    ge = np.zeros(len(idx), np.complex128)
    gp = np.zeros(len(idx), np.complex128)
    ga = np.zeros(len(idx), np.complex128)
    for q, p in enumerate(idx):
        # row p: Gamma_pj K_pj ; column p: Gamma_ip K_ip
        Kr = kernel_rows(eta, etap, A, n, slice(p, p + 1))[0]
        dcol = eta[p] - eta                              # eta_p - eta_i (source p, targets i)
        dcol[p] = 1.0
        Kc = (2.0 / n) * (A / A[p]) * etap[p] / dcol
        Kc[p] = 0.0
        Gr = np.zeros(N, np.complex128)
        Gc = np.zeros(N, np.complex128)
        for op, u, v in terms:
            if op == "FB":
                Gr += -1j * u[p] * (v[p] - v)
                Gc += -1j * u * (v - v[p])
            else:
                Gr += u[p] * (v - v[p])
                Gc += u * (v[p] - v)
        Gr[p] = 0.0
        Gc[p] = 0.0
        drow = eta - eta[p]                              # eta_j - eta_p
        drow[p] = 1.0
        dF_deta = np.sum(Gr * Kr / drow) - np.sum(Gc * Kc / dcol)
        dk = (2.0 / n) * (A / A[p]) / dcol
        dk[p] = 0.0
        dF_detap = np.sum(Gc * dk)
        dF_dA = (np.sum(Gr * Kr) - np.sum(Gc * Kc)) / A[p]
        ge[q], gp[q], ga[q] = np.conj(dF_deta), np.conj(dF_detap), np.conj(dF_dA)
    return ge, gp, ga


def fbie_vjp(eta, etap, A, gam, n, g_mu=None, g_h=None):
    """Reverse-mode derivatives of (mu, h) = FBIE(eta, eta', A, gamma) for one
    right-hand side: returns dict(mu, h, lam, g_gam, g_eta, g_etap, g_A)."""
    N = eta.shape[0]
    g_mu = np.zeros(N) if g_mu is None else g_mu
    g_h = np.zeros(N) if g_h is None else g_h
    Aop, Cop = fbie_operators(eta, etap, A, n)
    lu = sla.lu_factor(Aop)
    mu = sla.lu_solve(lu, -(Cop @ gam))
    h = (Cop @ mu - Aop @ gam) / 2.0
    lam = sla.lu_solve(lu, 0.5 * (Cop.T @ g_h) + g_mu, trans=1)
    g_gam = -0.5 * (Aop.T @ g_h) - Cop.T @ lam
    terms = fbie_geom_terms(g_h, lam, mu, gam)
    g_eta, g_etap, g_A = bilinear_geom_grad(eta, etap, A, n, terms)
    return dict(mu=mu, h=h, lam=lam, g_gam=g_gam, g_eta=g_eta, g_etap=g_etap, g_A=g_A)


def fbie_geom_terms(g_h, lam, mu, gam):
    """The four bilinear terms of the geometric differential of L."""
    return [("FC", 0.5 * g_h, mu), ("FB", -0.5 * g_h, gam), ("FB", -lam, mu), ("FC", -lam, gam)]


def mean_square_loss(h, n):
    """L = sum_k h_k^2 with h_k the mean of h over component k; returns (L, dL/dh)."""
    hk = h.reshape(-1, n).mean(axis=1)
    return float(np.sum(hk ** 2)), np.repeat(2.0 * hk / n, n)


def fourier_nodes(coeffs, kmin, n, ccw=False):
    """eta, eta', eta'' of eta_j(t) = sum_k c_{j,k} e^{i s k t} (s = +1 ccw, -1 cw)
    at t_p = 2 pi p / n, component-major."""
    s = 1.0 if ccw else -1.0
    t = 2.0 * np.pi * np.arange(n) / n
    ks = np.arange(kmin, kmin + coeffs.shape[1], dtype=np.float64)
    ph = np.exp(1j * s * np.outer(t, ks))                      # n x nk
    eta = (ph @ coeffs.T).T.ravel()
    etap = (ph @ (coeffs * (1j * s * ks)).T).T.ravel()
    etapp = (ph @ (coeffs * (-(ks ** 2))).T).T.ravel()
    return eta, etap, etapp


def fourier_coef_grad(g_eta, g_etap, g_etapp, kmin, nk, n, ccw=False):
    """Chain rule to the coefficients: g_c = sum_p sum_z g_z,p conj(dz_p/dc), with
    d eta_p/dc_k = e^{i s k t_p}, d eta'_p/dc_k = i s k e^{i s k t_p},
    d eta''_p/dc_k = -k^2 e^{i s k t_p}. Returns an (m+1) x nk array."""
    s = 1.0 if ccw else -1.0
    t = 2.0 * np.pi * np.arange(n) / n
    ks = np.arange(kmin, kmin + nk, dtype=np.float64)
    phc = np.exp(-1j * s * np.outer(t, ks))                    # conj of the basis
    ge = g_eta.reshape(-1, n)
    out = ge @ phc
    if g_etap is not None:
        out = out + (g_etap.reshape(-1, n) @ phc) * (-1j * s * ks)[None, :]
    if g_etapp is not None:
        out = out + (g_etapp.reshape(-1, n) @ phc) * (-(ks ** 2))[None, :]
    return out


def fbie_loss_and_grad(coeffs, kmin, n, gam):
    """L = sum_k h_k^2 for the unbounded domain exterior to the Fourier curves
    (clockwise, A = 1) and right-hand side gam (held fixed); returns
    (L, dL/dgam, dL/dcoeffs)."""
    eta, etap, _ = fourier_nodes(coeffs, kmin, n)
    A = np.ones_like(eta)
    Aop, Cop = fbie_operators(eta, etap, A, n)
    mu = sla.lu_solve(sla.lu_factor(Aop), -(Cop @ gam))
    h = (Cop @ mu - Aop @ gam) / 2.0
    L, g_h = mean_square_loss(h, n)
    r = fbie_vjp(eta, etap, A, gam, n, g_h=g_h)
    g_c = fourier_coef_grad(r["g_eta"], r["g_etap"], None, kmin, coeffs.shape[1], n)
    return L, r["g_gam"], g_c


def fbie_loss(coeffs, kmin, n, gam):
    """Forward only: L = sum_k h_k^2 (for finite differences)."""
    eta, etap, _ = fourier_nodes(coeffs, kmin, n)
    A = np.ones_like(eta)
    Aop, Cop = fbie_operators(eta, etap, A, n)
    mu = sla.lu_solve(sla.lu_factor(Aop), -(Cop @ gam))
    h = (Cop @ mu - Aop @ gam) / 2.0
    return mean_square_loss(h, n)[0]


__all__ = ["bilinear_geom_grad", "bilinear_geom_grad_rows", "fbie_vjp", "fbie_geom_terms", "mean_square_loss",
           "fourier_nodes", "fourier_coef_grad", "fbie_loss_and_grad", "fbie_loss", "circulant_L",
           "block_diag_repeat"]
