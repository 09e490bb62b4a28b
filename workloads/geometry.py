"""Boundary curves for the synthetic workloads (seeded, host-side, NumPy).

This module only builds *inputs*: boundary nodes eta(t_i), eta'(t_i), eta''(t_i)
on the trapezoidal mesh, the coefficient A (and A'), and right-hand sides.
It contains none of the solver's arithmetic (no kernel, no Nystrom matrix,
no Krylov step), so both the CPU oracle and the GPU path may consume it.

Conventions (paper Sec. 2.1 and Sec. 2.4):
  * m+1 boundary components, each parametrised on [0, 2*pi] and sampled at the
    n equidistant nodes s_p = (p-1) 2 pi / n, p = 1..n  (n even);
  * node i = k*n + p (0-based here: i = k*n + q, q = 0..n-1) is component k,
    i.e. component-major storage (the ordering of eq. (e:ti-skp));
  * the domain G lies on the left of every boundary: for a bounded domain the
    outer curve is counter-clockwise and the inner curves clockwise, for an
    unbounded domain all curves are clockwise (Sec. 2.1, Fig. 1).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

TWO_PI = 2.0 * np.pi


def nodes(n: int) -> np.ndarray:
    """Equidistant trapezoidal nodes s_p = (p-1) 2 pi / n (Sec. 2.4)."""
    return TWO_PI * np.arange(n, dtype=np.float64) / n


# ----------------------------------------------------------------------------
# Elementary curves. Each returns (eta, eta', eta'') evaluated at parameter t.
# ----------------------------------------------------------------------------
def circle(t, center=0j, radius=1.0, ccw=True):
    s = 1.0 if ccw else -1.0
    e = np.exp(1j * s * t)
    return center + radius * e, radius * 1j * s * e, -radius * e


def ellipse(t, center=0j, a=1.0, b=0.5, phi=0.0, ccw=False):
    """z0 + e^{i phi} (a cos t + i s b sin t), s = +1 (ccw) or -1 (cw)."""
    s = 1.0 if ccw else -1.0
    rot = np.exp(1j * phi)
    ct, st = np.cos(t), np.sin(t)
    eta = center + rot * (a * ct + 1j * s * b * st)
    d1 = rot * (-a * st + 1j * s * b * ct)
    d2 = rot * (-a * ct - 1j * s * b * st)
    return eta, d1, d2


def fourier_curve(t, coeffs: np.ndarray, kmin: int, ccw=False):
    """eta(t) = sum_k c_k e^{i s k t} for k = kmin .. kmin+len(c)-1, s=+1 ccw / -1 cw."""
    s = 1.0 if ccw else -1.0
    ks = np.arange(kmin, kmin + len(coeffs), dtype=np.float64)
    ph = np.exp(1j * s * np.outer(t, ks))
    eta = ph @ coeffs
    d1 = ph @ (coeffs * (1j * s * ks))
    d2 = ph @ (coeffs * (-(ks ** 2)))
    return eta, d1, d2


# ----------------------------------------------------------------------------
# Kress graded mesh (paper Sec. 6, eqs. (e:omega), (e:omega-v), (e:delta_j)).
# ----------------------------------------------------------------------------
def _kress_v(t, p):
    a = 1.0 / p - 0.5
    x = (np.pi - t) / np.pi
    v = a * x ** 3 + (t - np.pi) / (p * np.pi) + 0.5
    dv = -3.0 * a * x ** 2 / np.pi + 1.0 / (p * np.pi)
    ddv = 6.0 * a * x / (np.pi ** 2)
    return v, dv, ddv


def kress_omega(t, p: int):
    """omega(t) of eq. (e:omega) and its first two derivatives, t in [0, 2 pi]."""
    t = np.asarray(t, dtype=np.float64)
    v1, dv1, ddv1 = _kress_v(t, p)
    v2, dv2, ddv2 = _kress_v(TWO_PI - t, p)
    u = v1 ** p
    w = v2 ** p
    du = p * v1 ** (p - 1) * dv1
    dw = -p * v2 ** (p - 1) * dv2
    ddu = p * (p - 1) * v1 ** (p - 2) * dv1 ** 2 + p * v1 ** (p - 1) * ddv1
    ddw = p * (p - 1) * v2 ** (p - 2) * dv2 ** 2 + p * v2 ** (p - 1) * ddv2
    s = u + w
    om = TWO_PI * u / s
    num1 = du * w - u * dw
    dom = TWO_PI * num1 / s ** 2
    ddom = TWO_PI * ((ddu * w - u * ddw) * s - 2.0 * num1 * (du + dw)) / s ** 3
    return om, dom, ddom


def kress_delta(t, pj: int, p: int):
    """delta_j(t) of eq. (e:delta_j): corners at c_k = (k-1) 2 pi / pj.

    Returns delta, delta', delta''."""
    t = np.asarray(t, dtype=np.float64)
    h = TWO_PI / pj
    k = np.minimum(np.floor(t / h), pj - 1)
    ck = k * h
    om, dom, ddom = kress_omega(pj * (t - ck), p)
    return om / pj + ck, dom, pj * ddom


# ----------------------------------------------------------------------------
# Rounded-corner polygon zeta(tau), tau in [0, 2 pi]: p equal parameter
# intervals, interval k centred on the midpoint of the arc that rounds corner
# k. Inside an interval the parameter is proportional to arclength.
# ----------------------------------------------------------------------------
@dataclass
class RoundedPolygon:
    verts: np.ndarray          # p vertices, counter-clockwise
    rad: float                 # arc radius
    ccw: bool = False
    _segs: list = field(default_factory=list, repr=False)

    def __post_init__(self):
        V = np.asarray(self.verts, dtype=np.complex128)
        p = len(V)
        segs = []   # per corner k: list of pieces covering [arc-mid_k -> arc-mid_{k+1}]
        # tangent points and arc centres
        info = []
        for k in range(p):
            v, vp, vn = V[k], V[k - 1], V[(k + 1) % p]
            u1 = (vp - v) / abs(vp - v)
            u2 = (vn - v) / abs(vn - v)
            ang = np.arccos(np.clip((u1.conjugate() * u2).real, -1, 1))  # interior angle
            d = self.rad / np.tan(ang / 2)       # distance vertex -> tangent point
            bis = (u1 + u2) / abs(u1 + u2)
            cen = v + bis * self.rad / np.sin(ang / 2)
            t_in = v + u1 * d                    # tangent point on incoming edge
            t_out = v + u2 * d                   # tangent point on outgoing edge
            a_in = np.angle(t_in - cen)
            a_out = np.angle(t_out - cen)
            # ccw polygon: arc runs ccw from a_in to a_out
            da = (a_out - a_in) % TWO_PI
            info.append((cen, a_in, da, t_in, t_out))
        for k in range(p):
            cen, a_in, da, t_in, t_out = info[k]
            cen2, a_in2, da2, t_in2, _ = info[(k + 1) % p]
            # half arc k (mid -> out), straight edge (out_k -> in_{k+1}), half arc k+1 (in -> mid)
            pieces = [
                ("arc", cen, a_in + da / 2, da / 2),
                ("line", t_out, t_in2),
                ("arc", cen2, a_in2, da2 / 2),
            ]
            lens = [self.rad * da / 2, abs(t_in2 - t_out), self.rad * da2 / 2]
            segs.append((pieces, np.array(lens)))
        self._segs = segs

    @property
    def p(self):
        return len(self.verts)

    def __call__(self, tau):
        """zeta, zeta', zeta'' at tau (tau in [0, 2 pi])."""
        tau = np.asarray(tau, dtype=np.float64) % TWO_PI
        p = self.p
        h = TWO_PI / p
        z = np.empty(tau.shape, np.complex128)
        dz = np.empty_like(z)
        ddz = np.empty_like(z)
        # orientation: the polygon is stored ccw; cw traversal uses tau -> -tau
        tt = tau if self.ccw else (TWO_PI - tau) % TWO_PI
        sgn = 1.0 if self.ccw else -1.0
        k = np.minimum(np.floor(tt / h).astype(int), p - 1)
        for kk in range(p):
            msk = k == kk
            if not np.any(msk):
                continue
            pieces, lens = self._segs[kk]
            Ltot = lens.sum()
            speed = Ltot / h                      # d(arclength)/d tau
            sl = (tt[msk] - kk * h) * speed       # arclength within interval
            zz = np.empty(sl.shape, np.complex128)
            d1 = np.empty_like(zz)
            d2 = np.empty_like(zz)
            starts = np.concatenate([[0.0], np.cumsum(lens)[:-1]])
            for piece, L0, Lp in zip(pieces, starts, lens):
                m = (sl >= L0) & (sl <= L0 + Lp + 1e-300)
                s = sl[m] - L0
                if piece[0] == "arc":
                    _, cen, a0, _ = piece
                    ang = a0 + s / self.rad
                    e = np.exp(1j * ang)
                    zz[m] = cen + self.rad * e
                    d1[m] = 1j * e * speed
                    d2[m] = -e / self.rad * speed ** 2
                else:
                    _, za, zb = piece
                    u = (zb - za) / abs(zb - za)
                    zz[m] = za + u * s
                    d1[m] = u * speed
                    d2[m] = 0.0
            z[msk] = zz
            dz[msk] = d1 * sgn
            ddz[msk] = d2
        return z, dz, ddz


def graded_polygon(t, poly: RoundedPolygon, grade: int):
    """eta = zeta o delta (eq. (e:zet-et)) with the Kress map for p_j = poly.p corners.

    eta' = zeta'(delta) delta',  eta'' = zeta''(delta) delta'^2 + zeta'(delta) delta''."""
    d, dd, ddd = kress_delta(t, poly.p, grade)
    z, dz, ddz = poly(d)
    return z, dz * dd, ddz * dd ** 2 + dz * ddd
