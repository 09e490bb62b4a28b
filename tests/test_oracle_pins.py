"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself: exact closed
forms (unit disk, circulant spectrum), invariants that hold for the continuous
operators (eqs. (e:NM-const), (e:Nk-const)), closed-form solutions of the
Riemann-Hilbert problem (eq. (e:ex-gam)), the two routes for the right-hand
side (eq. (e:phi-kp) vs (e:y)), the two forms of the vector e ((e:ei) vs
(e:bve)), and brute force on tiny meshes. A dropped term, a wrong sign or a
transposed operand in the oracle fails at least one of them.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import nystrom as orc


def _dense_E(eta):
    N = eta.shape[0]
    d = eta[:, None] - eta[None, :]
    d[np.arange(N), np.arange(N)] = 1.0
    E = 1.0 / d
    E[np.arange(N), np.arange(N)] = 0.0
    return E


# ---------------------------------------------------------------- exact forms
@pytest.mark.parametrize("n", [8, 16, 32])
def test_disk_operators_exact(n):
    """Unit disk with A = eta: B_ij = -1/n, so 2I+diag(B1)-B = I + 11^T/n exactly,
    and D - diag(D1) + L = -K_wittich (Wittich's matrix)."""
    d = wl.disk(n)
    K = orc.kernel_matrix(d.eta, d.etap, d.A, n)
    off = ~np.eye(n, dtype=bool)
    assert np.max(np.abs(K.imag[off] + 1.0 / n)) < 1e-14
    Aop, Cop = orc.fbie_operators(d.eta, d.etap, d.A, n)
    assert np.max(np.abs(Aop - (np.eye(n) + np.ones((n, n)) / n))) < 1e-14
    assert np.max(np.abs(Cop + orc.wittich_K(n))) < 1e-13


@pytest.mark.parametrize("n", [8, 16, 64, 256])
def test_circulant_L_spectrum(n):
    """L is circulant with first column b; fft(b)_k = 2ik/n for the signed
    frequency |k| < n/2 and 0 at k = n/2 (the symbol of (2/n) d/dt)."""
    L = orc.circulant_L(n)
    b = L[:, 0]
    for j in range(n):
        assert np.max(np.abs(L[:, j] - np.roll(b, j))) < 1e-14
    k = np.fft.fftfreq(n, 1.0 / n)
    lam = 2j * k / n
    lam[n // 2] = 0.0
    assert np.max(np.abs(np.fft.fft(b) - lam)) < 1e-13
    assert np.max(np.abs(L + L.T)) == 0.0          # antisymmetric
    assert np.max(np.abs(L @ np.ones(n))) < 1e-14  # Lhat 1 = 0


@pytest.mark.parametrize("n", [8, 32])
def test_K_L_identity(n):
    """(e:K-L): -K_pq + (1/n) cot((p-q) pi/n) = L_pq for p != q."""
    p = np.arange(n)
    d = p[:, None] - p[None, :]
    cot = np.zeros((n, n))
    cot[d != 0] = (1.0 / n) / np.tan(d[d != 0] * np.pi / n)
    lhs = -orc.wittich_K(n) + cot
    assert np.max(np.abs(lhs - orc.circulant_L(n))) < 1e-14


# -------------------------------------------------------------- invariants
@pytest.mark.parametrize("n", [64, 128])
def test_rowsum_N_is_minus_one(n):
    """int_J N(s,t) dt = -1 for admissible A (eq. (e:NM-const)): the trapezoidal
    row sum B1_i + (2 pi/n) N(t_i,t_i), with N(t,t) from (e:N-tt), tends to -1."""
    d = wl.annulus(n)
    B = orc.kernel_matrix(d.eta, d.etap, d.A, n).imag
    Ntt = (0.5 * (d.etapp / d.etap).imag - (d.Ap / d.A).imag) / np.pi
    rs = B.sum(axis=1) + (2 * np.pi / n) * Ntt
    tol = 1e-6 if n == 64 else 1e-12
    assert np.max(np.abs(rs + 1.0)) < tol


@pytest.mark.parametrize("kind", ["bounded", "unbounded"])
def test_neumann_kernel_constant(kind):
    """int_J N_k(s,t) dt = c (eq. (e:Nk-const)): c = 1 bounded, -1 unbounded."""
    n = 128
    if kind == "bounded":
        d = wl.annulus(n)
    else:
        d = wl.circles_unbounded(n, [0j, 1.5 + 0.2j], [0.5, 0.4])
    Nk = orc.kernel_matrix(d.eta, d.etap, np.ones_like(d.eta), n).imag
    rs = Nk.sum(axis=1) + (1.0 / n) * (d.etapp / d.etap).imag
    assert np.max(np.abs(rs - d.c)) < 1e-12


def test_two_routes_for_y():
    """y by Wittich's matrix + M_1 (eq. (e:phi-kp)) equals y = (D - diag(D1) + Lhat) gamma (eq. (e:y))."""
    n = 64
    d, gam = wl.config0("eta-alpha")
    # coarsen the mesh of the same geometry
    d = wl.annulus(n, r_in=0.3, alpha=0.55, center_in=0.1 - 0.05j)
    gam = np.log(np.abs(d.eta - 0.5))
    _, Cop = orc.fbie_operators(d.eta, d.etap, d.A, n)
    y1 = Cop @ gam
    y2 = orc.rhs_wittich(d.eta, d.etap, d.A, gam, n)
    assert np.max(np.abs(y1 - y2)) < 1e-13 * max(1.0, np.max(np.abs(y1)))


def test_e_vector_two_forms():
    """e from (e:ei)+(e:ri) (oracle) equals the Cauchy-matrix form (e:bve)."""
    n = 48
    d = wl.annulus(n, r_in=0.35, alpha=0.6, center_in=0.05 + 0.1j)
    e1 = orc.fbiead_e(d.eta, d.etap, d.etapp, d.A, d.Ap, n, d.c)
    E = _dense_E(d.eta)
    e2 = 1 - d.c - (2.0 / n) * (E @ d.etap).imag + (2.0 / n) * (d.etapp / d.etap - d.Ap / d.A).imag
    assert np.max(np.abs(e1 - e2)) < 1e-12


# ------------------------------------------------------------ closed forms
def test_closed_form_annulus_converges():
    """gamma = Re[A f(eta)] (eq. (e:ex-gam)) => mu = Im[A f(eta)], h = 0, with
    exponential convergence in n for analytic data."""
    errs = []
    for n in (16, 32, 64, 128):
        d = wl.annulus(n)
        f = lambda z: np.sin(z) + 1.0 / (z - 2.0) + 0.3 / (z - 0.05j)
        gam, mu_ex = wl.closed_form_rhs(d, f)
        mu, h = orc.fbie(d.eta, d.etap, d.A, gam, n)
        errs.append((np.max(np.abs(mu - mu_ex)), np.max(np.abs(h))))
    e_mu = [e[0] for e in errs]
    e_h = [e[1] for e in errs]
    assert e_mu[-1] < 1e-12 and e_h[-1] < 1e-12
    assert e_mu[0] > 1e3 * e_mu[2]          # exponential decay


def test_closed_form_unbounded_circles():
    """Unbounded, A = 1, f(infinity) = 0 with poles inside the holes."""
    n = 96
    cs = [0j, 1.3 + 0.4j, -0.9 + 1.1j]
    rs = [0.5, 0.35, 0.4]
    d = wl.circles_unbounded(n, cs, rs)
    f = lambda z: 1.0 / (z - cs[1] - 0.1) + 0.5j / (z - cs[2]) ** 2 + 1.0 / (z - 0.05)
    gam, mu_ex = wl.closed_form_rhs(d, f)
    mu, h = orc.fbie(d.eta, d.etap, d.A, gam, n)
    assert np.max(np.abs(mu - mu_ex)) < 1e-11
    assert np.max(np.abs(h)) < 1e-11


def test_closed_form_theta_nonconstant():
    """Example 2 geometry, theta = (pi/2, 0, pi/2, 0, pi/2): still mu = Im[A f], h = 0."""
    n = 256
    d = wl.example2_circles(n, 0.1, theta=[np.pi / 2, 0, np.pi / 2, 0, np.pi / 2])
    f = lambda z: np.sin(z) + 1.0 / (z - 2.0)
    gam, mu_ex = wl.closed_form_rhs(d, f)
    mu, h = orc.fbie(d.eta, d.etap, d.A, gam, n)
    assert np.max(np.abs(mu - mu_ex)) < 1e-9
    assert np.max(np.abs(h)) < 1e-9


def test_disk_bandlimited_exact():
    """On the disk the discrete solution is exact for band-limited f."""
    n = 32
    d = wl.disk(n)
    f = lambda z: 1.0 + 0.5 * z ** 3 - 0.25j * z ** 5
    gam, mu_ex = wl.closed_form_rhs(d, f)
    mu, h = orc.fbie(d.eta, d.etap, d.A, gam, n)
    assert np.max(np.abs(mu - mu_ex)) < 1e-13
    assert np.max(np.abs(h)) < 1e-13


def test_fbiead_invariants():
    """(I + N* + J) phi = 1 => J phi = 1 and int gamma phi = 0 for gamma = Re[A f]
    (paper Example 1); E_n = |(2 pi/n) sum gamma phi| decays exponentially."""
    E = []
    for n in (32, 64, 128):
        d = wl.annulus(n)
        f = lambda z: np.sin(z) + 1.0 / (z - 2.0)
        gam, _ = wl.closed_form_rhs(d, f)
        phi = orc.fbiead(d.eta, d.etap, d.etapp, d.A, d.Ap, np.ones(d.N), n, d.c)
        means = orc.component_means(phi, n)
        assert np.max(np.abs(means - 1.0)) < 1e-8 or n < 64
        E.append(abs((2 * np.pi / n) * np.sum(gam * phi)))
    assert E[-1] < 1e-12 and E[0] > 1e3 * E[-1]


def test_fbiead_unbounded_invariants():
    n = 96
    cs = [0j, 1.4 + 0.3j]
    d = wl.circles_unbounded(n, cs, [0.5, 0.45])
    f = lambda z: 1.0 / (z - 0.1) + 1.0 / (z - cs[1])
    gam, _ = wl.closed_form_rhs(d, f)
    phi = orc.fbiead(d.eta, d.etap, d.etapp, d.A, d.Ap, np.ones(d.N), n, d.c)
    assert np.max(np.abs(orc.component_means(phi, n) - 1.0)) < 1e-11
    assert abs((2 * np.pi / n) * np.sum(gam * phi)) < 1e-11


# --------------------------------------------------------------- brute force
def _N_kernel(As, At, etas, etat, etapt):
    return (1 / np.pi) * ((As / At) * etapt / (etat - etas)).imag


def _M_kernel(As, At, etas, etat, etapt):
    return (1 / np.pi) * ((As / At) * etapt / (etat - etas)).real


def test_bruteforce_tiny_fbie_system():
    """Literal double loops over (e:ie-sys2) and (e:phi-kp3) on a tiny mesh."""
    n = 6
    d = wl.annulus(n, r_in=0.3, alpha=0.6)
    N = d.N
    w = 2 * np.pi / n
    Aop = np.zeros((N, N))
    for i in range(N):
        diag = 2.0
        for j in range(N):
            if j == i:
                continue
            v = w * _N_kernel(d.A[i], d.A[j], d.eta[i], d.eta[j], d.etap[j])
            diag += v
            Aop[i, j] -= v
        Aop[i, i] += diag
    Cop = np.zeros((N, N))
    for i in range(N):
        k, p = divmod(i, n)
        for j in range(N):
            l, q = divmod(j, n)
            if j != i:
                v = w * _M_kernel(d.A[i], d.A[j], d.eta[i], d.eta[j], d.etap[j])
                Cop[i, j] += v
                Cop[i, i] -= v
            if l == k and q != p:
                Lpq = (-1) ** (p - q) * (1.0 / n) / np.tan((p - q) * np.pi / n)
                Cop[i, j] += Lpq
                Cop[i, i] -= Lpq
    A2, C2 = orc.fbie_operators(d.eta, d.etap, d.A, n)
    assert np.max(np.abs(A2 - Aop)) < 1e-13
    assert np.max(np.abs(C2 - Cop)) < 1e-13


def test_bruteforce_tiny_fbiead_system():
    """Literal loops over (e:ie*-sys2) with r(t_i) from (e:ri)."""
    n = 6
    d = wl.annulus(n, r_in=0.3, alpha=0.6)
    N = d.N
    w = 2 * np.pi / n
    G = np.zeros((N, N))
    for i in range(N):
        r = w * (1 / np.pi) * (d.etapp[i] / d.etap[i] - d.Ap[i] / d.A[i]).imag
        for j in range(N):
            if j != i:
                Ng = (1 / np.pi) * ((d.A[i] * d.etap[j] - d.A[j] * d.etap[i])
                                    / (d.A[i] * (d.eta[j] - d.eta[i]))).imag
                r += w * Ng
        coef = 1 - d.c + r
        for j in range(N):
            if j == i:
                continue
            v = w * _N_kernel(d.A[j], d.A[i], d.eta[j], d.eta[i], d.etap[i])   # N(t_j, t_i)
            coef -= v
            G[i, j] += v
        G[i, i] += coef
        k = i // n
        for j in range(k * n, (k + 1) * n):
            G[i, j] += w * (1 / (2 * np.pi))
    G2 = orc.fbiead_operator(d.eta, d.etap, d.etapp, d.A, d.Ap, n, d.c)
    assert np.max(np.abs(G - G2)) < 1e-13


def test_config0_as_stated_is_nonsingular():
    """A = 1 on a bounded domain is outside (e:A); the discrete system is still
    uniquely solvable and the row sums of B tend to +1 instead of -1."""
    d, gam = wl.config0("one")
    Aop, Cop = orc.fbie_operators(d.eta, d.etap, d.A, d.n)
    K = orc.kernel_matrix(d.eta, d.etap, d.A, d.n)
    rs = K.imag.sum(axis=1) + (1.0 / d.n) * (d.etapp / d.etap).imag
    assert np.max(np.abs(rs - 1.0)) < 1e-8
    s = np.linalg.svd(Aop, compute_uv=False)
    assert s[-1] > 1e-3


def test_kernel_rows_equal_full_matrix():
    d = wl.annulus(32)
    K = orc.kernel_matrix(d.eta, d.etap, d.A, d.n)
    for sl in (slice(0, 5), slice(30, 40), slice(60, 64)):
        assert np.array_equal(orc.kernel_rows(d.eta, d.etap, d.A, d.n, sl), K[sl])


def test_residual_rows_equal_dense_residual():
    d = wl.annulus(24)
    gam = np.log(np.abs(d.eta - 0.55))
    Aop, Cop = orc.fbie_operators(d.eta, d.etap, d.A, d.n)
    mu = np.random.default_rng(2).normal(size=d.N)
    full = Aop @ mu + Cop @ gam
    rows = np.array([0, 5, 23, 24, 40, 47])
    res, y = orc.fbie_residual_rows(d.eta, d.etap, d.A, gam, mu, d.n, rows)
    assert np.max(np.abs(res - full[rows])) < 1e-13
    assert np.max(np.abs(y - (Cop @ gam)[rows])) < 1e-13
