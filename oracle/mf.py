"""Matrix-free FP64 route of the CPU oracle, for sizes where the dense FBIE
matrices do not fit in memory (the close-boundary workload, N = 133120; the
perturbed-circles workload, N = 264192; the larger domains of the batched
workload).

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call, link or
execute anything under ``oracle/``; only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.

What it computes is the same discrete system as ``oracle.nystrom``:
  * ``fbie_ops``: (2I + diag(B1) - B) x and (D - diag(D1) + Lhat) x, or their
    transposes, with every kernel entry K_ij = (2/n)(A_i/A_j) eta'_j/(eta_j - eta_i)
    evaluated from its definition (eqs. (e:N), (e:M), (e:B), matrix D of Sec. 3.3)
    in plain C loops (oracle/mf.c, OpenMP over rows), and Lhat applied as the
    dense n x n matrix L of Sec. 3.3 on each component (no FFT);
  * ``gmres``: textbook restarted GMRES (Arnoldi with modified Gram-Schmidt,
    repeated once, Givens rotations, least squares by back substitution), one
    Krylov space per column, the products of all columns taken together; a
    column stops when its true residual ||b - Ax||_2/||b||_2, recomputed at
    every restart, is at most tol (x0 = 0, b = 0 gives x = 0);
  * ``fbie``: y = Cop gamma, mu from Aop mu = -y, h = (Cop mu - Aop gamma)/2
    (Sec. 3.3-3.6, eq. (e:bh));
  * ``fbie_adjoint``: lam = Aop^{-T}(Cop^T g_h/2 + g_mu) and
    dL/dgamma = -Aop^T g_h/2 - Cop^T lam, the reverse-mode rules of
    ``oracle.gradient`` with the transposed products in place of dense LU.

It is checked against the dense LU route on the same seeded geometries at
reduced sizes (tests/test_oracle_mf.py).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .nystrom import circulant_L

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mf.c")
_lib = None


def _cpu_has_avx512():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("flags"):
                    return "avx512f" in line.split()
    except OSError:
        pass
    return False


def lib_path(level=None):
    """The shared library for this host's vector level (x86-64-v4 with AVX-512, else v3)."""
    if level is None:
        level = "v4" if _cpu_has_avx512() else "v3"
    return os.path.join(_HERE, f"libgnk_oracle_{level}.so")


def build(levels=("v3", "v4")):
    """Compile oracle/mf.c (gcc, OpenMP) for both x86-64 vector levels."""
    for lv in levels:
        out = lib_path(lv)
        subprocess.run(["gcc", "-O3", f"-march=x86-64-{lv}", "-fopenmp", "-shared", "-fPIC", "-o", out, _SRC],
                       check=True)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("GNK_ORACLE_LIB")      # another build of mf.c (the sanitizer test)
    if not path:
        path = lib_path()
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build()
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.gnk_oracle_fbie_ops.argtypes = [ctypes.c_int64, ctypes.c_int] + [dp] * 6 + \
        [ctypes.c_int, dp, ctypes.c_int, dp, dp, ctypes.c_int]
    lib.gnk_oracle_fbie_ops.restype = ctypes.c_int
    lib.gnk_oracle_fbie_rows.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int64, ctypes.c_int64] + \
        [dp] * 6 + [ctypes.c_int, dp, ctypes.c_int, dp, dp, ctypes.c_int]
    lib.gnk_oracle_fbie_rows.restype = ctypes.c_int
    lib.gnk_oracle_kernel_rows.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int64, ctypes.c_int64] + \
        [dp] * 8 + [ctypes.c_int]
    lib.gnk_oracle_kernel_rows.restype = None
    lib.gnk_oracle_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Geometry:
    """eta, eta', A of one domain, split into contiguous real and imaginary parts."""

    def __init__(self, eta, etap, A, n):
        self.N = int(np.asarray(eta).shape[0])
        self.n = int(n)
        if self.N % self.n:
            raise ValueError("N must be a multiple of n")
        self.m1 = self.N // self.n
        self.parts = [np.ascontiguousarray(f(np.asarray(v, np.complex128)))
                      for v in (eta, etap, A) for f in (np.real, np.imag)]
        self.L = circulant_L(self.n)


def max_threads():
    return int(_load().gnk_oracle_max_threads())


def fbie_ops(geo: Geometry, x, trans=False, nthreads=0):
    """(Aop x, Cop x) with Aop = 2I + diag(B1) - B (eq. (e:sys)) and
    Cop = D - diag(D1) + Lhat (eqs. (e:y), (e:bh)); trans: (Aop^T x, Cop^T x)
    with Aop^T = 2I + diag(B1) - B^T, Cop^T = D^T - diag(D1) + Lhat^T.
    x: (N,) or (N, ncols)."""
    x = np.asarray(x, np.float64)
    one = x.ndim == 1
    X = np.asfortranarray(x.reshape(geo.N, -1))
    nc = X.shape[1]
    ya = np.zeros((geo.N, nc), order="F")
    yc = np.zeros((geo.N, nc), order="F")
    st = _load().gnk_oracle_fbie_ops(geo.N, geo.n, *[_p(a) for a in geo.parts], nc, _p(X), int(bool(trans)),
                                     _p(ya), _p(yc), int(nthreads))
    if st != 0:
        raise MemoryError("oracle row buffers")
    Lb = geo.L.T if trans else geo.L
    Xk = np.asarray(X).reshape(geo.m1, geo.n, nc)                # component k, node p, column
    yc += np.matmul(Lb[None, :, :], Xk).reshape(geo.N, nc)
    if one:
        return ya[:, 0].copy(), yc[:, 0].copy()
    return np.ascontiguousarray(ya), np.ascontiguousarray(yc)


def fbie_rows(geo: Geometry, x, i0, i1, nthreads=0):
    """Rows i0..i1-1 of (2I + diag(B1) - B) x and (D - diag(D1)) x (the circulant
    part left out), for timing samples of the product; x: (N,) or (N, ncols)."""
    X = np.asfortranarray(np.asarray(x, np.float64).reshape(geo.N, -1))
    nc = X.shape[1]
    ya = np.zeros((geo.N, nc), order="F")
    yc = np.zeros((geo.N, nc), order="F")
    st = _load().gnk_oracle_fbie_rows(geo.N, geo.n, int(i0), int(i1), *[_p(a) for a in geo.parts], nc, _p(X), 0,
                                      _p(ya), _p(yc), int(nthreads))
    if st != 0:
        raise ValueError(f"oracle rows {i0}..{i1}: status {st}")
    return ya[i0:i1], yc[i0:i1]


def kernel_rows(geo: Geometry, i0, i1, nthreads=0):
    """Rows i0..i1-1 of K (complex, (i1 - i0) x N) from the C loops."""
    kr = np.zeros((i1 - i0, geo.N))
    ki = np.zeros((i1 - i0, geo.N))
    _load().gnk_oracle_kernel_rows(geo.N, geo.n, i0, i1, *[_p(a) for a in geo.parts], _p(kr), _p(ki),
                                   int(nthreads))
    return kr + 1j * ki


def gmres(apply, b, tol=1e-14, restart=100, maxit=20, log=None):
    """Restarted GMRES for the columns of b (N x ncols), each in its own Krylov
    space; apply(V) returns A V for an N x ncols block. Returns (x, info) with
    info = dict(iters, cycles, relres) per column (true residuals)."""
    b = np.asarray(b, np.float64)
    N, nc = b.shape
    x = np.zeros_like(b)
    bnorm = np.linalg.norm(b, axis=0)
    iters = np.zeros(nc, int)
    r = b.copy()
    rnorm = bnorm.copy()
    cycles = 0
    for cycles in range(1, maxit + 1):
        live = rnorm > tol * bnorm
        if not live.any():
            cycles -= 1
            break
        V = np.zeros((restart + 1, N, nc))
        H = np.zeros((restart + 1, restart, nc))
        cs = np.zeros((restart, nc))
        sn = np.zeros((restart, nc))
        g = np.zeros((restart + 1, nc))
        g[0] = np.where(live, rnorm, 0.0)
        V[0] = np.where(live, r / np.where(live, rnorm, 1.0), 0.0)
        steps = np.zeros(nc, int)
        going = live.copy()
        for j in range(restart):
            w = apply(V[j] * going)
            for _ in range(2):                              # modified Gram-Schmidt, twice
                for i in range(j + 1):
                    hij = np.sum(V[i] * w, axis=0)
                    w -= V[i] * hij
                    H[i, j] += hij
            hn = np.linalg.norm(w, axis=0)
            H[j + 1, j] = hn
            V[j + 1] = np.where(going & (hn > 0), w / np.where(hn > 0, hn, 1.0), 0.0)
            for i in range(j):                               # earlier rotations
                a, c_ = H[i, j].copy(), H[i + 1, j].copy()
                H[i, j] = cs[i] * a + sn[i] * c_
                H[i + 1, j] = -sn[i] * a + cs[i] * c_
            a, c_ = H[j, j], H[j + 1, j]
            den = np.hypot(a, c_)
            den = np.where(den > 0, den, 1.0)
            cs[j], sn[j] = a / den, c_ / den
            H[j, j] = cs[j] * a + sn[j] * c_
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            steps = np.where(going, j + 1, steps)
            going = going & (np.abs(g[j + 1]) > 0.5 * tol * bnorm) & (hn > 0)
            if log is not None and (j % 10 == 9 or not going.any()):
                est = np.max(np.abs(g[j + 1]) / np.where(bnorm > 0, bnorm, 1.0))
                log(f"  cycle {cycles} step {j + 1}: max estimated relres {est:.3e}, live {int(going.sum())}")
            if not going.any():
                break
        for c in range(nc):                                  # back substitution, update
            k = steps[c]
            if k == 0:
                continue
            y = np.zeros(k)
            for i in range(k - 1, -1, -1):
                y[i] = (g[i, c] - H[i, i + 1:k, c] @ y[i + 1:k]) / H[i, i, c]
            x[:, c] += V[:k, :, c].T @ y
            iters[c] += k
        r = b - apply(x)
        rnorm = np.linalg.norm(r, axis=0)
        if log is not None:
            log(f"  cycle {cycles}: true relres max {np.max(rnorm / np.where(bnorm > 0, bnorm, 1.0)):.3e}")
    relres = rnorm / np.where(bnorm > 0, bnorm, 1.0)
    return x, dict(iters=iters, cycles=cycles, relres=relres)


def fbie(geo: Geometry, gam, tol=1e-14, restart=100, maxit=20, nthreads=0, log=None):
    """mu, h of FBIE (Sec. 3.3-3.6) and the GMRES info; gam: (N,) or (N, ncols)."""
    g = np.asarray(gam, np.float64)
    one = g.ndim == 1
    G = g.reshape(geo.N, -1)
    ag, y = fbie_ops(geo, G, nthreads=nthreads)            # Aop gamma, y = Cop gamma (eq. (e:y))
    mu, info = gmres(lambda v: fbie_ops(geo, v, nthreads=nthreads)[0], -y, tol, restart, maxit, log)
    _, cmu = fbie_ops(geo, mu, nthreads=nthreads)
    h = (cmu - ag) / 2.0                                     # eq. (e:bh)
    if one:
        return mu[:, 0], h[:, 0], info
    return mu, h, info


def fbie_adjoint(geo: Geometry, g_mu=None, g_h=None, tol=1e-14, restart=100, maxit=20, nthreads=0, log=None):
    """lam = Aop^{-T}(Cop^T g_h/2 + g_mu) and dL/dgamma = -Aop^T g_h/2 - Cop^T lam
    for one column (the reverse-mode rules of the FBIE map)."""
    N = geo.N
    g_mu = np.zeros(N) if g_mu is None else np.asarray(g_mu, np.float64)
    g_h = np.zeros(N) if g_h is None else np.asarray(g_h, np.float64)
    atg, ctg = fbie_ops(geo, g_h, trans=True, nthreads=nthreads)
    rhs = 0.5 * ctg + g_mu
    lam, info = gmres(lambda v: fbie_ops(geo, v, trans=True, nthreads=nthreads)[0], rhs[:, None], tol, restart,
                      maxit, log)
    lam = lam[:, 0]
    _, ctl = fbie_ops(geo, lam, trans=True, nthreads=nthreads)
    g_gam = -0.5 * atg - ctl
    return lam, g_gam, info
