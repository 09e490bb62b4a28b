"""GPU parity of the conformal slit maps (gnk_circular_slit_map, gnk_slit_map)
against the oracle (oracle/maps.py): boundary values and slit levels to the
1e-10 bound of the solves on Examples 2 and 4's domains and the 17-component
domain, closed forms for one circle, the map's properties checked through the
GPU's own Cauchy integral (gnk_fcau): f(alpha) = 0 and |f| < 1 inside, and
the argument errors (alpha outside G, theta_0, the bounded flag)."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as wl
from oracle.maps import circular_slit_map as map_ref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gk():
    from paper_1308_5351_amd import gnk
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return gnk


@pytest.fixture(scope="module")
def ctx(gk):
    c = gk.Context(0)
    yield c
    c.close()


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("eps,n", [(0.1, 128), (0.01, 256)])
def test_slit_map_example2_matches_oracle(gk, ctx, eps, n):
    d = wl.example2_circles(n, eps)
    print(f"[map] example2 eps={eps} n={n}", flush=True)
    f, R, info, st = ctx.circular_slit_map(_cuda(d.eta), _cuda(d.etap), d.m1, d.n, 0.0, tol=1e-13, restart=40)
    assert st == gk.OK, info
    f_r, R_r, _, _ = map_ref(d.eta, d.etap, 0.0, n)
    assert np.max(np.abs(f.cpu().numpy() - f_r)) < 1e-10
    assert np.max(np.abs(R - R_r)) < 1e-10
    z = np.array([0.0, 0.05 + 0.02j, -0.3j, 0.6])
    fz = ctx.fcau(_cuda(d.eta), _cuda(d.etap), f, _cuda(z), d.m1, d.n).cpu().numpy()
    assert abs(fz[0]) < 1e-9 and np.all(np.abs(fz[1:]) < 1.0)


def test_slit_map_config1_properties(gk, ctx):
    # 17 components, N = 17408, alpha = 0 (in G): |f| = 1 on the unit circle, radii in (0, 1),
    # f(alpha) = 0 through the Cauchy integral of the boundary values; the direct and
    # treecode solves agree
    d, _ = wl.config1()
    f, R, info, st = ctx.circular_slit_map(_cuda(d.eta), _cuda(d.etap), d.m1, d.n, 0.0)
    assert st == gk.OK, info
    fh = f.cpu().numpy()
    assert np.max(np.abs(np.abs(fh[:d.n]) - 1.0)) < 1e-12
    assert R[0] == 1.0 and np.all((R[1:] > 0) & (R[1:] < 1))
    for k in range(1, d.m1):
        seg = np.abs(fh[k * d.n:(k + 1) * d.n])
        assert np.max(np.abs(seg - R[k])) < 1e-12
    f0 = ctx.fcau(_cuda(d.eta), _cuda(d.etap), f, _cuda(np.array([0.0 + 0.0j])), d.m1, d.n).cpu().numpy()
    assert abs(f0[0]) < 1e-9
    ft, Rt, _, st = ctx.circular_slit_map(_cuda(d.eta), _cuda(d.etap), d.m1, d.n, 0.0, far_tol=1e-13)
    assert st == gk.OK
    assert np.max(np.abs(ft.cpu().numpy() - fh)) < 1e-10 and np.max(np.abs(Rt - R)) < 1e-10


# ------------------------------------------------- circular and radial slits (gnk_slit_map)
from oracle.maps import slit_map as slit_ref  # noqa: E402

THETA_EX3 = np.array([np.pi / 2, 0.0, np.pi / 2, 0.0, np.pi / 2])


@pytest.mark.parametrize("eps,n", [(0.1, 128), (0.01, 512)])
def test_radial_slit_map_example2_matches_oracle(gk, ctx, eps, n):
    d = wl.example2_circles(n, eps)
    print(f"[map] radial+circular example2 eps={eps} n={n}", flush=True)
    f, lev, info, st = ctx.slit_map(_cuda(d.eta), _cuda(d.etap), d.m1, d.n, 0.0, THETA_EX3, tol=1e-13, restart=40)
    assert st == gk.OK, info
    f_r, lev_r, _, _ = slit_ref(d.eta, d.etap, 0.0, THETA_EX3, n)
    assert np.max(np.abs(f.cpu().numpy() - f_r)) < 1e-10
    assert np.max(np.abs(lev - lev_r)) < 1e-10
    # the angles the domain's symmetry fixes (a property of the exact map: with non-constant
    # theta, FBIE at eps = 0.01 misses them by 1e-4 at n = 256, 1e-7 at n = 512 and 1e-13 at
    # n = 1024, Example 2's finding), and f(alpha) = 0 through the GPU's Cauchy integral
    tol = 1e-10 if eps >= 0.1 else 1e-6
    assert abs(np.angle(np.exp(-1j * lev[1]) * np.exp(-1j * np.pi / 4))) < tol
    assert abs(np.angle(np.exp(-1j * lev[3]) * np.exp(3j * np.pi / 4))) < tol
    z = np.array([0.0, 0.05 + 0.02j, 0.6])       # points of G for both separations
    fz = ctx.fcau(_cuda(d.eta), _cuda(d.etap), f, _cuda(z), d.m1, d.n).cpu().numpy()
    assert abs(fz[0]) < 1e3 * tol and np.all(np.abs(fz[1:]) < 1.0)


def test_slit_map_mixed_theta_config1(gk, ctx):
    # the 17-component domain at n = 256 (N = 4352): radial slits on the odd components,
    # circular on the even ones, one spiral (theta = 0.4); the oracle on the same nodes,
    # and the treecode solve
    d, _ = wl.config1(n=256)
    theta = np.where(np.arange(d.m1) % 2 == 1, 0.0, np.pi / 2)
    theta[4] = 0.4
    print(f"[map] config1 mixed theta N={d.eta.shape[0]}", flush=True)
    f, lev, info, st = ctx.slit_map(_cuda(d.eta), _cuda(d.etap), d.m1, d.n, 0.0, theta, tol=1e-13, restart=40)
    assert st == gk.OK, info
    f_r, lev_r, _, _ = slit_ref(d.eta, d.etap, 0.0, theta, d.n)
    assert np.max(np.abs(f.cpu().numpy() - f_r)) < 1e-10
    assert np.max(np.abs(lev - lev_r)) < 1e-10
    ft, lt, _, st = ctx.slit_map(_cuda(d.eta), _cuda(d.etap), d.m1, d.n, 0.0, theta, tol=1e-13, restart=40,
                                 far_tol=1e-13)
    assert st == gk.OK
    assert np.max(np.abs(ft.cpu().numpy() - f_r)) < 1e-10 and np.max(np.abs(lt - lev_r)) < 1e-10


def test_slit_map_pi_over_2_equals_circular_map(gk, ctx):
    d = wl.example2_circles(64, 0.05)
    f, lev, _, st = ctx.slit_map(_cuda(d.eta), _cuda(d.etap), d.m1, d.n, 0.0, np.full(5, np.pi / 2))
    fc, R, _, st2 = ctx.circular_slit_map(_cuda(d.eta), _cuda(d.etap), d.m1, d.n, 0.0)
    assert st == gk.OK and st2 == gk.OK
    assert torch.equal(f, fc) and np.array_equal(np.exp(lev), R)


def test_slit_map_argument_errors(gk, ctx):
    d = wl.example2_circles(32, 0.1)
    e, p = _cuda(d.eta), _cuda(d.etap)
    bad = [dict(alpha=0.0, theta=np.array([0.0, 0, 0, 0, 0])),          # theta_0 != pi/2
           dict(alpha=0.0, theta=np.array([np.pi / 2, np.nan, 0, 0, 0])),  # non-finite theta
           dict(alpha=0.3 + 0.3j, theta=THETA_EX3),                       # alpha inside a hole
           dict(alpha=2.0, theta=THETA_EX3)]                              # alpha outside the unit circle
    for kw in bad:
        with pytest.raises(gk.GnkError) as ex:
            ctx.slit_map(e, p, d.m1, d.n, kw["alpha"], kw["theta"])
        assert ex.value.status == gk.ERR_ARG, kw
    with pytest.raises(gk.GnkError) as ex:
        ctx.circular_slit_map(e, p, d.m1, d.n, 0.3 + 0.3j)
    assert ex.value.status == gk.ERR_ARG
    f, lev, info, st = ctx.slit_map(e, p, d.m1, d.n, 0.0, THETA_EX3)
    assert st == gk.OK


# ------------------------------------------------------------- unbounded domains (Example 4)
def _circle_nodes(n, ccw):
    t = 2 * np.pi * np.arange(n) / n
    e = np.exp(1j * t) if ccw else np.exp(-1j * t)
    return e, (1j if ccw else -1j) * e


@pytest.mark.parametrize("alpha", [2.0, 1.5 - 0.7j])
def test_slit_maps_exterior_of_circle_closed_forms(gk, ctx, alpha):
    # |z| > 1: circular slit F = z (z - alpha)/(z - 1/conj(alpha)), radial slit
    # F = z + e^{2i phi}/z - e^{i phi}(|alpha| + 1/|alpha|); and the disc's Moebius map
    n = 256
    eta, etap = _circle_nodes(n, False)
    print(f"[map] exterior of the unit circle alpha={alpha}", flush=True)
    F, lev, info, st = ctx.slit_map(_cuda(eta), _cuda(etap), 1, n, alpha, [np.pi / 2], bounded=False, tol=1e-13)
    assert st == gk.OK, info
    assert np.max(np.abs(F.cpu().numpy() - eta * (eta - alpha) / (eta - 1 / np.conj(alpha)))) < 1e-10
    assert abs(lev[0] - np.log(abs(alpha))) < 1e-10
    F, lev, info, st = ctx.slit_map(_cuda(eta), _cuda(etap), 1, n, alpha, [0.0], bounded=False, tol=1e-13)
    assert st == gk.OK, info
    ph = np.angle(alpha)
    ex = eta + np.exp(2j * ph) / eta - np.exp(1j * ph) * (abs(alpha) + 1 / abs(alpha))
    assert np.max(np.abs(F.cpu().numpy() - ex)) < 1e-10
    eta, etap = _circle_nodes(n, True)
    a = 0.3 + 0.4j
    f, lev, info, st = ctx.slit_map(_cuda(eta), _cuda(etap), 1, n, a, [np.pi / 2], tol=1e-13)
    assert st == gk.OK, info
    assert np.max(np.abs(f.cpu().numpy() - (eta - a) / (1 - np.conj(a) * eta))) < 1e-10


@pytest.mark.parametrize("eps,n", [(0.1, 128), (0.01, 256)])
def test_slit_map_example4_matches_oracle(gk, ctx, eps, n):
    d = wl.example4_circles(n, eps)
    print(f"[map] example4 eps={eps} n={n}", flush=True)
    for theta in (THETA_EX3, np.full(5, np.pi / 2)):
        F, lev, info, st = ctx.slit_map(_cuda(d.eta), _cuda(d.etap), d.m1, d.n, 2.0 + 2.0j, theta, bounded=False,
                                        tol=1e-13, restart=40)
        assert st == gk.OK, info
        F_r, lev_r, _, _ = slit_ref(d.eta, d.etap, 2.0 + 2.0j, theta, n, bounded=False)
        s = np.max(np.abs(F_r))
        assert np.max(np.abs(F.cpu().numpy() - F_r)) / s < 1e-10
        assert np.max(np.abs(lev - lev_r)) < 1e-10


def test_slit_map_unbounded_argument_errors(gk, ctx):
    d = wl.example4_circles(32, 0.1)
    e, p = _cuda(d.eta), _cuda(d.etap)
    for alpha in (0.0, 1.0 + 1.0j):      # inside the centre circle, inside a corner circle
        with pytest.raises(gk.GnkError) as ex:
            ctx.slit_map(e, p, d.m1, d.n, alpha, THETA_EX3, bounded=False)
        assert ex.value.status == gk.ERR_ARG
    lib = gk.load_library()
    f = torch.empty_like(e)
    al = (ctypes.c_double * 2)(2.0, 2.0)
    assert lib.gnk_slit_map(ctx.h, d.m1, d.n, e.data_ptr(), p.data_ptr(), 2, al, None, None, f.data_ptr(),
                            None, None) == gk.ERR_ARG
    # theta_0 is free for an unbounded domain
    F, lev, info, st = ctx.slit_map(e, p, d.m1, d.n, 2.0 + 2.0j, [0.0, 0.0, np.pi / 2, 0.0, np.pi / 2],
                                    bounded=False)
    assert st == gk.OK


def test_slit_map_unbounded_treecode(gk, ctx):
    # Example 4's domain at n = 1024 (N = 5120): the treecode solve gives the direct one's map
    d = wl.example4_circles(1024, 0.1)
    e, p = _cuda(d.eta), _cuda(d.etap)
    print(f"[map] example4 treecode N={d.eta.shape[0]}", flush=True)
    F, lev, info, st = ctx.slit_map(e, p, d.m1, d.n, 2.0 + 2.0j, THETA_EX3, bounded=False, tol=1e-13, restart=40)
    Ft, levt, infot, stt = ctx.slit_map(e, p, d.m1, d.n, 2.0 + 2.0j, THETA_EX3, bounded=False, tol=1e-13,
                                       restart=40, far_tol=1e-13)
    assert st == gk.OK and stt == gk.OK
    Fh = F.cpu().numpy()
    assert np.max(np.abs(Ft.cpu().numpy() - Fh)) / np.max(np.abs(Fh)) < 1e-10
    assert np.max(np.abs(levt - lev)) < 1e-10
