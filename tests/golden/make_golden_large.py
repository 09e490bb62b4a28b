"""Write the oracle's reference solutions for the workloads whose dense matrices
do not fit in memory, to tests/golden/:

  cfg2   close-boundary workload (65 boundaries, n = 2048, N = 133120):
         mu and h of FBIE, matrix-free route.
  cfg4   perturbed circles (129 x 16 Fourier coefficients, n = 2048,
         N = 264192): mu, h of FBIE, then the reverse-mode derivatives of
         L = sum_k h_k^2 (h_k the component means): dL/dgamma on every node and
         dL/dcoef for every coefficient of four seeded components.
  cfg3   batched workload (64 domains): dense LU for N <= 12288 (every column),
         matrix-free above (four columns per domain); mu and h on 64 seeded
         rows per column, the column norms and the component means of h.

Calls only the CPU oracle (``oracle/``) on the seeded inputs of ``workloads/``.
Run from the repository root, one workload per call:
    python tests/golden/make_golden_large.py cfg2|cfg4|cfg3
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as wl                 # noqa: E402
from oracle import gradient as og      # noqa: E402
from oracle import mf                  # noqa: E402
from oracle import nystrom as orc      # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))
TOL = 1e-15            # GMRES tolerance of the matrix-free route (reached or reported)
T0 = time.time()


def log(msg):
    print(f"[{time.time() - T0:8.1f}s] {msg}", flush=True)


def _checksum(dom):
    return np.array([dom.eta.real.sum(), dom.eta.imag.sum(), float(dom.N)])


def cfg2():
    dom, gam = wl.config2()
    g = gam[:, 0]
    geo = mf.Geometry(dom.eta, dom.etap, dom.A, dom.n)
    log(f"cfg2: N = {dom.N}, {mf.max_threads()} threads")
    t = time.time()
    mu, h, info = mf.fbie(geo, g, tol=TOL, restart=400, maxit=3, log=log)
    secs = time.time() - t
    log(f"cfg2 done in {secs:.0f}s: {info}")
    np.savez_compressed(os.path.join(OUT, "cfg2_oracle.npz"), mu=mu, h=h, iters=info["iters"],
                        relres=info["relres"], seconds=secs, tol=TOL, eta_checksum=_checksum(dom))


COMPONENTS4 = 4        # components of the perturbed-circles workload whose coefficients get a reference gradient


def cfg4():
    dom, gam = wl.config4()
    g = gam[:, 0]
    n, m1 = dom.n, dom.m1
    geo = mf.Geometry(dom.eta, dom.etap, dom.A, n)
    log(f"cfg4: N = {dom.N}, {mf.max_threads()} threads")
    t = time.time()
    mu, h, info = mf.fbie(geo, g, tol=TOL, restart=200, maxit=3, log=log)
    t_fwd = time.time() - t
    log(f"cfg4 forward done in {t_fwd:.0f}s: {info}")
    path = os.path.join(OUT, "cfg4_oracle.npz")
    np.savez_compressed(path, mu=mu, h=h, iters=info["iters"], relres=info["relres"], seconds_forward=t_fwd,
                        tol=TOL, eta_checksum=_checksum(dom))
    L, g_h = og.mean_square_loss(h, n)
    t = time.time()
    lam, g_gam, info_ad = mf.fbie_adjoint(geo, g_h=g_h, tol=TOL, restart=200, maxit=3, log=log)
    t_adj = time.time() - t
    log(f"cfg4 adjoint done in {t_adj:.0f}s: {info_ad}")
    coeffs, kmin = dom.meta["coeffs"], dom.meta["kmin"]
    comps = np.sort(np.random.default_rng([13085351, 4, 99]).choice(m1, COMPONENTS4, replace=False))
    terms = og.fbie_geom_terms(g_h, lam, mu, g)
    t = time.time()
    g_coef = np.zeros((COMPONENTS4, coeffs.shape[1]), np.complex128)
    for q, j in enumerate(comps):
        idx = np.arange(j * n, (j + 1) * n)
        ge, gp, _ = og.bilinear_geom_grad_rows(dom.eta, dom.etap, dom.A, n, terms, idx)
        g_coef[q] = og.fourier_coef_grad(ge, gp, None, kmin, coeffs.shape[1], n)[0]
        log(f"cfg4 geometry gradient, component {j}: max|g| {np.abs(g_coef[q]).max():.3e}")
    t_geo = time.time() - t
    np.savez_compressed(path, mu=mu, h=h, iters=info["iters"], relres=info["relres"], seconds_forward=t_fwd,
                        tol=TOL, eta_checksum=_checksum(dom), loss=L, g_gam=g_gam, lam_iters=info_ad["iters"],
                        lam_relres=info_ad["relres"], seconds_adjoint=t_adj, seconds_geometry=t_geo,
                        g_coef_components=comps, g_coef=g_coef)
    log(f"cfg4 written: L = {L:.6e}")


DENSE_MAX = 12288      # batched domains up to this size take the dense LU route
ROWS3 = 64             # sampled rows per column
MF_COLS = 4            # columns per matrix-free domain


def cfg3():
    out = {}
    for d in range(64):
        dom, gam = wl.batch_domain(d)
        N, nc = dom.N, gam.shape[1]
        rng = np.random.default_rng([13085351, 3, d, 7])
        t = time.time()
        if N <= DENSE_MAX:
            cols = np.arange(nc)
            mu, h = orc.fbie(dom.eta, dom.etap, dom.A, gam, dom.n)
            route, it, rr = "dense", np.zeros(nc, int), np.zeros(nc)
        else:
            cols = np.unique(np.concatenate([[0, nc - 1], rng.choice(nc, MF_COLS - 2, replace=False)]))
            geo = mf.Geometry(dom.eta, dom.etap, dom.A, dom.n)
            mu, h, info = mf.fbie(geo, gam[:, cols], tol=TOL, restart=120, maxit=3)
            route, it, rr = "mf", info["iters"], info["relres"]
            gam = gam[:, cols]
        rows = np.sort(rng.choice(N, ROWS3, replace=False))
        out[f"d{d}_cols"] = cols
        out[f"d{d}_rows"] = rows
        out[f"d{d}_mu"] = mu[rows]
        out[f"d{d}_h"] = h[rows]
        out[f"d{d}_mu_max"] = np.max(np.abs(mu), axis=0)
        out[f"d{d}_h_max"] = np.max(np.abs(h), axis=0)
        out[f"d{d}_gam_max"] = np.max(np.abs(gam), axis=0)
        out[f"d{d}_hk"] = orc.component_means(h, dom.n)
        out[f"d{d}_iters"] = it
        out[f"d{d}_relres"] = rr
        out[f"d{d}_route"] = np.array(route)
        out[f"d{d}_checksum"] = _checksum(dom)
        log(f"cfg3 domain {d}: N = {N}, {len(cols)} of {nc} columns, {route}, {time.time() - t:.0f}s, "
            f"iters {list(it)}, relres max {np.max(rr):.2e}")
        np.savez_compressed(os.path.join(OUT, "cfg3_oracle.npz"), tol=TOL, rows_per_column=ROWS3, **out)
    log("cfg3 written")


if __name__ == "__main__":
    {"cfg2": cfg2, "cfg4": cfg4, "cfg3": cfg3}[sys.argv[1]]()
