"""CPU FP64 oracle for the Nystrom discretisation with the generalized Neumann kernel.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call, link or
execute anything under ``oracle/``; only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.

What it computes: the dense trapezoidal-rule Nystrom systems of the paper,
assembled element by element from the kernel definitions (never through the
factored Cauchy-matrix form the GPU path uses), solved by LAPACK LU.

  * kernel_matrix      -- K_ij = (2 pi/n)(1/pi)(A_i/A_j) eta'_j/(eta_j-eta_i), i != j
                          so that B = Im K (eq. (e:B), kernel (e:N)) and
                          D = Re K (matrix D of Sec. 3.3, kernel (e:M)).
  * circulant_L        -- the n x n matrix L of Sec. 3.3 (defined just before (e:K-L)).
  * wittich_K          -- Wittich's matrix K of Sec. 3.3 (used in (e:phi-kp)).
  * fbie_operators     -- 2I + diag(B1) - B (eq. (e:sys)) and D - diag(D1) + Lhat
                          (eqs. (e:y), (e:bh)).
  * fbie               -- y, mu, h of Sec. 3.3-3.6.
  * rhs_wittich        -- y by the other route, eq. (e:phi-kp) with Wittich's matrix
                          and the kernel M_1 of (e:M-M1).
  * fbiead_e           -- the vector e of eq. (e:ei) with r(t_i) from (e:ri) and the
                          kernel N_g of (e:Ng), (e:Ng-tt) (direct form, not (e:bve)).
  * fbiead             -- (diag(e) + B^T + Phat) mu = gamma, eq. (e:sys*).
  * n_diagonal, fbie_unsubtracted, fbiead_unsubtracted
                       -- the same equations without singularity subtraction
                          (Example 2): the kernel N with its diagonal limit (e:N-tt).

Arrays: complex128 / float64 vectors of length N = (m+1) n in component-major
order (node i = k n + p, eq. (e:ti-skp)).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def kernel_matrix(eta, etap, A, n):
    """K_ij = (2/n) (A_i/A_j) eta'_j / (eta_j - eta_i) for i != j, K_ii = 0.

    (2 pi / n) * N(t_i, t_j) = Im K_ij   (eq. (e:N) times the trapezoidal weight)
    (2 pi / n) * M(t_i, t_j) = Re K_ij   (eq. (e:M) times the trapezoidal weight)
    """
    eta = np.asarray(eta, np.complex128)
    N = eta.shape[0]
    diff = eta[None, :] - eta[:, None]          # eta_j - eta_i
    diff[np.arange(N), np.arange(N)] = 1.0
    K = (2.0 / n) * (A[:, None] / A[None, :]) * (etap[None, :] / diff)
    K[np.arange(N), np.arange(N)] = 0.0
    return K


def circulant_L(n):
    """L_pq = (-1)^(p-q) (1/n) cot((p-q) pi / n) for p != q, 0 on the diagonal (Sec. 3.3)."""
    p = np.arange(n)
    d = p[:, None] - p[None, :]
    L = np.zeros((n, n))
    off = d != 0
    sign = np.where(d % 2 == 0, 1.0, -1.0)
    L[off] = sign[off] * (1.0 / n) / np.tan(d[off] * np.pi / n)
    return L


def wittich_K(n):
    """Wittich's matrix: K_pq = (2/n) cot((p-q) pi / n) if p-q odd, 0 if even (Sec. 3.3)."""
    p = np.arange(n)
    d = p[:, None] - p[None, :]
    K = np.zeros((n, n))
    odd = (d % 2) != 0
    K[odd] = (2.0 / n) / np.tan(d[odd] * np.pi / n)
    return K


def block_diag_repeat(M, m1):
    """I_{m+1} (x) M: the block-diagonal matrices Lhat and Phat."""
    return np.kron(np.eye(m1), M)


def fbie_operators(eta, etap, A, n):
    """Dense (2I + diag(B1) - B) and (D - diag(D1) + Lhat)."""
    N = eta.shape[0]
    m1 = N // n
    K = kernel_matrix(eta, etap, A, n)
    B = K.imag
    D = K.real
    one = np.ones(N)
    Aop = 2.0 * np.eye(N) + np.diag(B @ one) - B           # eq. (e:sys)
    Cop = D - np.diag(D @ one) + block_diag_repeat(circulant_L(n), m1)   # eq. (e:y)/(e:bh)
    return Aop, Cop


def fbie(eta, etap, A, gam, n, return_ops=False):
    """Solve (2I + diag(B1) - B) mu = -y, y = (D - diag(D1) + Lhat) gamma  (Sec. 3.2-3.5),
    then h = [(D - diag(D1) + Lhat) mu - (2I + diag(B1) - B) gamma] / 2  (eq. (e:bh)).

    gam: (N,) or (N, nrhs). Returns mu, h with the shape of gam."""
    Aop, Cop = fbie_operators(eta, etap, A, n)
    y = Cop @ gam
    lu = sla.lu_factor(Aop)
    mu = sla.lu_solve(lu, -y)
    h = (Cop @ mu - Aop @ gam) / 2.0
    if return_ops:
        return mu, h, Aop, Cop
    return mu, h


def rhs_wittich(eta, etap, A, gam, n):
    """y = phi(t) by eq. (e:phi-kp): Wittich's matrix for the cotangent part, the
    trapezoidal rule for M_1 on the same component and for M on the others.

    (2 pi/n) M_1(s_kp, s_kq) = (1/n) cot((p-q) pi/n) + (2 pi/n) M(s_kp, s_kq), p != q,
    from the split (e:M-M1)."""
    N = eta.shape[0]
    m1 = N // n
    D = kernel_matrix(eta, etap, A, n).real          # (2 pi/n) M(t_i, t_j), i != j
    Kw = wittich_K(n)
    p = np.arange(n)
    d = p[:, None] - p[None, :]
    cotn = np.zeros((n, n))
    cotn[d != 0] = (1.0 / n) / np.tan(d[d != 0] * np.pi / n)
    y = np.zeros(N)
    for k in range(m1):
        sk = slice(k * n, (k + 1) * n)
        gk = gam[sk]
        diff_k = gk[None, :] - gk[:, None]            # gamma_k(s_q) - gamma_k(s_p)
        M1w = cotn + D[sk, sk]                        # (2 pi/n) M_1, p != q
        np.fill_diagonal(M1w, 0.0)
        yk = np.sum(-Kw * diff_k, axis=1) + np.sum(M1w * diff_k, axis=1)
        for l in range(m1):
            if l == k:
                continue
            sl_ = slice(l * n, (l + 1) * n)
            diff_kl = gam[sl_][None, :] - gk[:, None]
            yk = yk + np.sum(D[sk, sl_] * diff_kl, axis=1)
        y[sk] = yk
    return y


def fbiead_e(eta, etap, etapp, A, Ap, n, c):
    """e_i = 1 - c + r(t_i) - sum_{j != i} (2 pi/n) N(t_j, t_i)      (eq. (e:ei))
    r(t_i) = (2 pi/n) sum_{j != i} N_g(t_i, t_j) + (2 pi/n) N_g(t_i, t_i)   (eq. (e:ri))
    N_g(s,t) = (1/pi) Im[(A(s) eta'(t) - A(t) eta'(s)) / (A(s)(eta(t) - eta(s)))]  (e:Ng)
    N_g(t,t) = (1/pi) Im[eta''/eta' - A'/A]                            (e:Ng-tt)."""
    N = eta.shape[0]
    idx = np.arange(N)
    diff = eta[None, :] - eta[:, None]           # eta_j - eta_i
    diff[idx, idx] = 1.0
    Ng = (A[:, None] * etap[None, :] - A[None, :] * etap[:, None]) / (A[:, None] * diff)
    Ng = (2.0 / n) * Ng.imag
    Ng[idx, idx] = 0.0
    r = Ng.sum(axis=1) + (2.0 / n) * (etapp / etap - Ap / A).imag
    B = kernel_matrix(eta, etap, A, n).imag      # B_ij = (2 pi/n) N(t_i, t_j)
    return 1.0 - c + r - B.sum(axis=0)           # sum_j B_ji


def fbiead_operator(eta, etap, etapp, A, Ap, n, c):
    """diag(e) + B^T + Phat, eq. (e:sys*)."""
    N = eta.shape[0]
    m1 = N // n
    e = fbiead_e(eta, etap, etapp, A, Ap, n, c)
    B = kernel_matrix(eta, etap, A, n).imag
    P = np.full((n, n), 1.0 / n)
    return np.diag(e) + B.T + block_diag_repeat(P, m1)


def fbiead(eta, etap, etapp, A, Ap, gam, n, c, return_op=False):
    """Solve (diag(e) + B^T + Phat) mu = gamma (Sec. 4.2-4.5)."""
    G = fbiead_operator(eta, etap, etapp, A, Ap, n, c)
    mu = sla.lu_solve(sla.lu_factor(G), gam)
    if return_op:
        return mu, G
    return mu


def n_diagonal(etap, etapp, A, Ap, n):
    """(2 pi/n) N(t_i, t_i) from the diagonal limit (e:N-tt):
    (2 pi/n)(1/pi)(1/2 Im(eta''/eta') - Im(A'/A))."""
    return (2.0 / n) * (0.5 * (etapp / etap).imag - (Ap / A).imag)


def fbie_unsubtracted(eta, etap, etapp, A, Ap, gam, n):
    """FBIE without singularity subtraction (Example 2's comparison): the
    trapezoidal rule for the continuous kernel N with its diagonal limit,
    (I - N_n) mu = -y, N_n = B + diag((2 pi/n) N(t_i, t_i)), instead of
    2I + diag(B1) - B. The right-hand side y and h use the discretization of M of
    eq. (e:y) in both variants (its other form, eq. (e:phi-kp), gives the same
    vector to rounding), so the two differ only in the treatment of N:
    h = [(D - diag(D1) + Lhat) mu - (I - N_n) gamma] / 2."""
    N = eta.shape[0]
    _, Cop = fbie_operators(eta, etap, A, n)
    B = kernel_matrix(eta, etap, A, n).imag
    Aop = np.eye(N) - B - np.diag(n_diagonal(etap, etapp, A, Ap, n))
    mu = sla.lu_solve(sla.lu_factor(Aop), -(Cop @ gam))
    h = (Cop @ mu - Aop @ gam) / 2.0
    return mu, h


def fbiead_unsubtracted(eta, etap, etapp, A, Ap, gam, n):
    """FBIEad without singularity subtraction: (I + N*_n + J) mu = gamma with
    (N*_n)_ij = (2 pi/n) N(t_j, t_i) (= B^T off the diagonal, the limit (e:N-tt)
    on it) and J = Phat, instead of diag(e) + B^T + Phat of eq. (e:sys*)."""
    N = eta.shape[0]
    m1 = N // n
    B = kernel_matrix(eta, etap, A, n).imag
    G = np.eye(N) + B.T + np.diag(n_diagonal(etap, etapp, A, Ap, n)) + \
        block_diag_repeat(np.full((n, n), 1.0 / n), m1)
    return sla.lu_solve(sla.lu_factor(G), gam)


def component_means(x, n):
    """(1/n) sum over each component: the Phat / J average (eq. (e:bJ2), trapezoidal)."""
    x = np.asarray(x)
    return x.reshape(-1, n, *x.shape[1:]).mean(axis=1)


def rel_linf(x, ref, scale=None):
    """max|x - ref| / max(max|ref|, scale)."""
    den = np.max(np.abs(ref))
    if scale is not None:
        den = max(den, scale)
    return float(np.max(np.abs(np.asarray(x) - ref)) / den)


def kernel_rows(eta, etap, A, n, rows):
    """Rows `rows` (a slice) of K_ij = (2/n)(A_i/A_j) eta'_j/(eta_j - eta_i), K_ii = 0:
    the same definition as kernel_matrix, restricted to a block of targets."""
    idx = np.arange(eta.shape[0])[rows]
    diff = eta[None, :] - eta[idx][:, None]
    self_ = idx[:, None] == np.arange(eta.shape[0])[None, :]
    diff[self_] = 1.0
    K = (2.0 / n) * (A[idx][:, None] / A[None, :]) * (etap[None, :] / diff)
    K[self_] = 0.0
    return K


def fbie_residual_rows(eta, etap, A, gam, mu, n, rows):
    """Rows `rows` of r = (2I + diag(B1) - B) mu + (D - diag(D1) + Lhat) gamma,
    the residual of eq. (e:sys) with y from (e:y), evaluated from the kernel
    definitions (no full matrix is formed)."""
    K = kernel_rows(eta, etap, A, n, rows)
    idx = np.arange(eta.shape[0])[rows]
    B, D = K.imag, K.real
    amu = 2.0 * mu[idx] + np.sum(B * (mu[idx][:, None] - mu[None, :]), axis=1)
    y = np.sum(D * (gam[None, :] - gam[idx][:, None]), axis=1)
    L = circulant_L(n)
    k, p = np.divmod(idx, n)
    for q, (kk, pp) in enumerate(zip(k, p)):
        y[q] += L[pp] @ gam[kk * n:(kk + 1) * n]
    return amu + y, y
