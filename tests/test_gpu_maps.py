"""GPU parity of the circular-slit conformal map (gnk_circular_slit_map)
against the oracle (oracle/maps.py): boundary values and slit radii to the
1e-10 bound of the solves, plus the map's properties checked through the
GPU's own Cauchy integral (gnk_fcau): f(alpha) = 0 and |f| < 1 inside."""
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
