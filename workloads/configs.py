"""Seeded synthetic workloads for the generalized-Neumann-kernel solver.

Every workload is a list of boundary components sampled on the trapezoidal
mesh, plus the coefficient A (and A') and one or more right-hand sides.
Seeds: ``numpy.random.default_rng([13085351, cfg])`` and, for the batched
workload, ``[13085351, 3, d]`` for domain d.

Shapes and value distributions follow the paper's workloads (Sec. 7):
multiply connected domains of circles / ellipses / piecewise smooth curves on
Kress-graded meshes, with boundaries close to each other. The concrete layouts
below are seeded stand-ins; the paper's own layouts only exist in figures.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import geometry as geo

SEED = 13085351


@dataclass
class Domain:
    """Discretised boundary of an (m+1)-connected domain (paper Sec. 2.1, 2.4).

    All arrays are complex128 of length N = m1 * n in component-major order."""
    m1: int
    n: int
    eta: np.ndarray
    etap: np.ndarray
    etapp: np.ndarray
    A: np.ndarray
    Ap: np.ndarray
    bounded: bool
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.m1 * self.n

    @property
    def c(self) -> int:
        """+1 for bounded, -1 for unbounded (eq. (e:c))."""
        return 1 if self.bounded else -1

    def comp(self, k):
        return slice(k * self.n, (k + 1) * self.n)


def _assemble(curves, n, bounded, A_kind, alpha=0j, theta=None, name="", meta=None):
    """curves: list of callables t -> (eta, eta', eta''). A_kind: 'one' | 'eta-alpha'."""
    t = geo.nodes(n)
    parts = [c(t) for c in curves]
    eta = np.concatenate([p[0] for p in parts])
    etap = np.concatenate([p[1] for p in parts])
    etapp = np.concatenate([p[2] for p in parts])
    m1 = len(curves)
    if theta is None:
        rot = np.ones(eta.shape, np.complex128)
    else:
        th = np.repeat(np.asarray(theta, np.float64), n)
        rot = np.exp(1j * (np.pi / 2 - th))
    if A_kind == "one":
        A = np.ones_like(eta) if theta is None else rot.copy()
        Ap = np.zeros_like(eta)
    elif A_kind == "eta-alpha":
        # eq. (e:A), bounded case: A = e^{i(pi/2-theta)} (eta - alpha)
        A = rot * (eta - alpha)
        Ap = rot * etap
    else:
        raise ValueError(A_kind)
    return Domain(m1, n, eta, etap, etapp, A, Ap, bounded, name, meta or {})


# ----------------------------------------------------------------------------
# Small closed-form domains used as pins (disk, annulus, circles).
# ----------------------------------------------------------------------------
def disk(n: int, A_kind="eta-alpha"):
    """Unit disk, alpha = 0, theta = pi/2 -> A = eta (eq. (e:A))."""
    return _assemble([lambda t: geo.circle(t, 0j, 1.0, True)], n, True, A_kind, 0j, name="disk")


def annulus(n: int, r_in=0.4, alpha=0.7j * 0 + 0.7, center_in=0j):
    """Bounded annulus: outer unit circle ccw, inner circle cw; A = eta - alpha."""
    curves = [lambda t: geo.circle(t, 0j, 1.0, True),
              lambda t: geo.circle(t, center_in, r_in, False)]
    return _assemble(curves, n, True, "eta-alpha", alpha, name="annulus")


def circles_unbounded(n: int, centers, radii, theta=None):
    """Exterior of several circles (all cw), A = e^{i(pi/2 - theta)} (eq. (e:A))."""
    curves = [(lambda t, c=c, r=r: geo.circle(t, c, r, False)) for c, r in zip(centers, radii)]
    return _assemble(curves, n, False, "one", theta=theta, name="circles")


def example2_circles(n: int, eps: float, theta=None):
    """Paper Example 2: unit circle and four inner circles at separation eps."""
    s = 2.0 + 2.0 * np.sqrt(2.0)
    r = (2.0 - eps * s) / s
    off = (2.0 - eps) / s
    cs = [off + 1j * off, -off + 1j * off, -off - 1j * off, off - 1j * off]
    curves = [lambda t: geo.circle(t, 0j, 1.0, True)] + \
             [(lambda t, c=c: geo.circle(t, c, r, False)) for c in cs]
    return _assemble(curves, n, True, "eta-alpha", 0j, theta=theta, name=f"ex2-eps{eps:g}")


def example4_circles(n: int, eps: float, theta=None):
    """Paper Example 4: unbounded, five circles at mutual distance eps."""
    cs = [0j, 1 + 1j, -1 + 1j, -1 - 1j, 1 - 1j]
    rs = [np.sqrt(2.0) - 1.0 - eps / 2] + [1.0 - eps / 2] * 4
    return circles_unbounded(n, cs, rs, theta)


# ----------------------------------------------------------------------------
# Benchmark workloads.
# ----------------------------------------------------------------------------
def _point_outside_ellipse(z, c, a, b, phi, margin):
    w = (z - c) * np.exp(-1j * phi)
    return (w.real / (a + margin)) ** 2 + (w.imag / (b + margin)) ** 2 > 1.0


def config0(A_kind="one"):
    """Doubly connected, bounded: unit circle + cw ellipse; n = 256; alpha = 0.5.

    A_kind='one' is the workload as stated (A = 1 on a bounded domain);
    A_kind='eta-alpha' is the admissible companion A = eta - 0.5."""
    rng = np.random.default_rng([SEED, 0])
    alpha = 0.5 + 0j
    while True:
        r0 = 0.2 * np.sqrt(rng.uniform())
        c = r0 * np.exp(1j * rng.uniform(0, 2 * np.pi))
        a = rng.uniform(0.2, 0.35)
        b = rng.uniform(0.1, 0.2)
        phi = rng.uniform(0, np.pi)
        if _point_outside_ellipse(alpha, c, a, b, phi, 0.05 * a):
            break
    n = 256
    curves = [lambda t: geo.circle(t, 0j, 1.0, True),
              lambda t: geo.ellipse(t, c, a, b, phi, ccw=False)]
    dom = _assemble(curves, n, True, A_kind, alpha, name="cfg0" + ("" if A_kind == "one" else "b"),
                    meta=dict(alpha=alpha, ellipse=(c, a, b, phi)))
    gam = np.log(np.abs(dom.eta - alpha))
    return dom, gam[:, None]


def config1(n: int = 1024, m_inner: int = 16):
    """Bounded, unit circle + 16 seeded cw ellipses; A = eta (alpha = 0); gamma = -log|eta|."""
    rng = np.random.default_rng([SEED, 1])
    placed = []   # (center, a, b, phi)
    gap = 0.04
    while len(placed) < m_inner:
        a = rng.uniform(0.03, 0.08)
        b = rng.uniform(0.03, 0.08)
        phi = rng.uniform(0, np.pi)
        R = max(a, b)
        rho = (1.0 - R - gap) * np.sqrt(rng.uniform())
        c = rho * np.exp(1j * rng.uniform(0, 2 * np.pi))
        if abs(c) < R + gap:          # keep alpha = 0 in G
            continue
        ok = all(abs(c - c2) >= R + max(a2, b2) + gap for c2, a2, b2, _ in placed)
        if ok:
            placed.append((c, a, b, phi))
    curves = [lambda t: geo.circle(t, 0j, 1.0, True)] + \
             [(lambda t, p=p: geo.ellipse(t, p[0], p[1], p[2], p[3], ccw=False)) for p in placed]
    dom = _assemble(curves, n, True, "eta-alpha", 0j, name="cfg1", meta=dict(ellipses=placed))
    gam = -np.log(np.abs(dom.eta))
    return dom, gam[:, None]


def fourier_perturbed_circles(m1: int, n: int, seed, side=13.0, dmin=1.0,
                              rrange=(0.25, 0.35), nterms=16, amp=0.1):
    """Unbounded domain exterior to m1 perturbed circles, each a 16-term Fourier
    series eta_j(t) = sum_{k=-7..8} c_{j,k} e^{-ikt} (clockwise)."""
    rng = np.random.default_rng(seed)
    centers = []
    while len(centers) < m1:
        c = complex(*rng.uniform(-side / 2, side / 2, 2))
        if all(abs(c - c2) >= dmin for c2 in centers):
            centers.append(c)
    kmin = -7
    coeffs = np.zeros((m1, nterms), np.complex128)
    for j, c in enumerate(centers):
        r = rng.uniform(*rrange)
        cj = (rng.uniform(-1, 1, nterms) + 1j * rng.uniform(-1, 1, nterms)) * amp * r / np.sqrt(2)
        ks = np.arange(kmin, kmin + nterms)
        cj[ks == 0] = c
        cj[ks == 1] = r
        pert = (ks != 0) & (ks != 1)
        s = np.sum(np.abs(ks[pert]) * np.abs(cj[pert]))
        if s > 0.5 * r:
            cj[pert] *= 0.5 * r / s
        coeffs[j] = cj
    return coeffs, kmin


def config4(n: int = 2048, m1: int = 129):
    """Unbounded, 129 perturbed circles (16 Fourier coefficients each); A = 1; gamma = Re(eta^2)."""
    coeffs, kmin = fourier_perturbed_circles(m1, n, [SEED, 4])
    dom = domain_from_fourier(coeffs, kmin, n)
    gam = (dom.eta ** 2).real
    return dom, gam[:, None]


def domain_from_fourier(coeffs, kmin, n, name="fourier"):
    curves = [(lambda t, cj=cj: geo.fourier_curve(t, cj, kmin, ccw=False)) for cj in coeffs]
    d = _assemble(curves, n, False, "one", name=name)
    d.meta.update(coeffs=np.array(coeffs), kmin=kmin)
    return d


def closed_form_rhs(dom: Domain, f):
    """gamma = Re[A f(eta)], exact mu = Im[A f(eta)], h = 0 (paper eq. (e:ex-gam))."""
    v = dom.A * f(dom.eta)
    return v.real.copy(), v.imag.copy()


# ----------------------------------------------------------------------------
# Close-boundary workload: sequential adjacency growth of ellipses and
# Kress-graded rounded polygons (unbounded domain, all boundaries clockwise).
# ----------------------------------------------------------------------------
class _Shape:
    """A convex boundary template placed at `center`.

    `pts(m)` gives m boundary samples relative to the centre (counter-clockwise)."""

    def __init__(self, kind, size, params):
        self.kind = kind
        self.size = size
        self.params = params
        self.center = 0j
        self._cache = {}

    def rel_curve(self, t):
        if self.kind == "ellipse":
            a, b, phi = self.params
            return geo.ellipse(t, 0j, a, b, phi, ccw=True)
        return self.params["poly_ccw"](t)

    def pts(self, m):
        if m not in self._cache:
            t = 2 * np.pi * np.arange(m) / m
            self._cache[m] = self.rel_curve(t)[0]
        return self._cache[m]

    @property
    def R(self):
        return float(np.max(np.abs(self.pts(512))))


def _inside_convex(poly_ccw, p):
    """Points p (complex) strictly inside the convex polygon with ccw vertices poly_ccw."""
    e = np.roll(poly_ccw, -1) - poly_ccw
    rel = p[:, None] - poly_ccw[None, :]
    cross = (np.conj(e)[None, :] * rel).imag
    return np.all(cross > 0, axis=1)


def _gap(sa, sb, m_in=256, m_dist=2048):
    """Distance between the boundaries of two placed convex shapes, -1 if they overlap."""
    from scipy.spatial import cKDTree
    A = sa.pts(m_in) + sa.center
    B = sb.pts(m_in) + sb.center
    if np.any(_inside_convex(A, B)) or np.any(_inside_convex(B, A)):
        return -1.0
    Ad = sa.pts(m_dist) + sa.center
    Bd = sb.pts(m_dist) + sb.center
    tree = cKDTree(np.c_[Ad.real, Ad.imag])
    d, _ = tree.query(np.c_[Bd.real, Bd.imag])
    return float(d.min())


def _make_shape(rng, kind):
    a = rng.uniform(0.8, 1.0)
    if kind == "ellipse":
        b = a * rng.uniform(0.5, 0.8)
        return _Shape("ellipse", b, (a, b, rng.uniform(0, np.pi)))
    p = int(rng.integers(4, 7))
    ang = 2 * np.pi * np.arange(p) / p + rng.uniform(-0.2, 0.2, p) * 2 * np.pi / p + rng.uniform(0, 2 * np.pi)
    verts = a * np.exp(1j * np.sort(ang % (2 * np.pi)))
    side = np.min(np.abs(np.roll(verts, -1) - verts))
    rad = 0.1 * side
    poly_ccw = geo.RoundedPolygon(verts, rad, ccw=True)
    poly_cw = geo.RoundedPolygon(verts, rad, ccw=False)
    inr = a * np.cos(np.pi / p) * 0.8
    return _Shape("poly", inr, {"verts": verts, "rad": rad, "p": p, "poly_ccw": poly_ccw, "poly_cw": poly_cw})


_SHAPES_CACHE = {}


def close_shapes(m1, seed, gap_range=(1e-3, 1e-2), poly_every=4):
    key = (m1, tuple(np.atleast_1d(seed)), gap_range, poly_every)
    if key not in _SHAPES_CACHE:
        _SHAPES_CACHE[key] = _close_shapes(m1, seed, gap_range, poly_every)
    return _SHAPES_CACHE[key]


def _close_shapes(m1, seed, gap_range, poly_every):
    """Place m1 convex shapes by adjacency growth with boundary gaps g * size,
    g log-uniform in gap_range, by bisection on the centre distance."""
    rng = np.random.default_rng(seed)
    shapes = []
    for k in range(m1):
        kind = "poly" if (poly_every and k % poly_every == 0) else "ellipse"
        s = _make_shape(rng, kind)
        if not shapes:
            shapes.append(s)
            continue
        for _attempt in range(500):
            anchor = shapes[int(rng.integers(len(shapes)))]
            d = np.exp(1j * rng.uniform(0, 2 * np.pi))
            g = 10 ** rng.uniform(np.log10(gap_range[0]), np.log10(gap_range[1]))
            target = g * min(s.size, anchor.size)
            lo, hi = 0.0, anchor.R + s.R + 4 * target
            for _ in range(60):
                mid = 0.5 * (lo + hi)
                s.center = anchor.center + mid * d
                gm = _gap(anchor, s)
                if gm < 0 or gm < target:
                    lo = mid
                else:
                    hi = mid
                if gm > 0 and abs(gm - target) < 0.02 * target:
                    break
            s.center = anchor.center + hi * d
            ok = True
            for o in shapes:
                if o is anchor:
                    continue
                if abs(o.center - s.center) > o.R + s.R + 1e-2:
                    continue
                go = _gap(o, s)
                if go < 1e-3 * min(o.size, s.size):
                    ok = False
                    break
            if ok:
                shapes.append(s)
                break
        else:
            raise RuntimeError("could not place shape %d" % k)
    return shapes


def config2(n: int = 2048, m1: int = 65, grade: int = 3):
    """Unbounded domain exterior to m1 close boundaries (every 4th a rounded
    polygon on a Kress-graded mesh); A = 1; gamma = Re(eta^2)."""
    shapes = close_shapes(m1, [SEED, 2])
    curves = []
    for s in shapes:
        if s.kind == "ellipse":
            a, b, phi = s.params
            curves.append(lambda t, c=s.center, a=a, b=b, phi=phi: geo.ellipse(t, c, a, b, phi, ccw=False))
        else:
            poly = s.params["poly_cw"]

            def cv(t, poly=poly, c=s.center):
                z, dz, ddz = geo.graded_polygon(t, poly, grade)
                return z + c, dz, ddz
            curves.append(cv)
    dom = _assemble(curves, n, False, "one", name=f"cfg2-m{m1}-n{n}",
                    meta=dict(kinds=[s.kind for s in shapes], centers=[s.center for s in shapes]))
    gam = (dom.eta ** 2).real
    return dom, gam[:, None]


# ----------------------------------------------------------------------------
# Batched workload: many unbounded domains of uneven size, each with m+1
# right-hand sides gamma_k = log|eta - alpha_k|, alpha_k inside hole k.
# ----------------------------------------------------------------------------
def batch_domain(d: int, m1_range=(2, 40), ns=(256, 512, 1024, 2048), rrange=(0.05, 0.1)):
    """Domain d of the batched workload (seed [SEED, 3, d])."""
    rng = np.random.default_rng([SEED, 3, d])
    m1 = int(rng.integers(m1_range[0], m1_range[1] + 1))
    n = int(rng.choice(ns))
    side = 0.5 * np.sqrt(m1)
    holes = []        # (center, a, b, phi)
    while len(holes) < m1:
        r = rng.uniform(*rrange)
        if rng.uniform() < 0.5:
            a = b = r
            phi = 0.0
        else:
            a = r
            b = r * rng.uniform(0.5, 1.0)
            phi = rng.uniform(0, np.pi)
        cen = complex(*rng.uniform(-side / 2, side / 2, 2))
        ok = all(abs(cen - c2) >= a + a2 + 0.5 * max(a, a2) for c2, a2, _, _ in holes)
        if ok:
            holes.append((cen, a, b, phi))
    curves = [(lambda t, h=h: geo.ellipse(t, h[0], h[1], h[2], h[3], ccw=False)) for h in holes]
    dom = _assemble(curves, n, False, "one", name=f"batch{d}", meta=dict(holes=holes))
    alphas = [h[0] + 0.3 * h[1] * np.sqrt(rng.uniform()) * np.exp(1j * rng.uniform(0, 2 * np.pi)) for h in holes]
    gam = np.stack([np.log(np.abs(dom.eta - al)) for al in alphas], axis=1)
    return dom, gam


def config3(ndom: int = 64, **kw):
    """The batched workload: `ndom` domains (see batch_domain)."""
    return [batch_domain(d, **kw) for d in range(ndom)]


# ----------------------------------------------------------------------------
# Points of G for the Cauchy integral formula at interior points.
def _near_factor(rng, k):
    return np.exp(rng.uniform(np.log(1e-4), np.log(1e-2), k))


def interior_points_config1(dom: Domain, nz: int, seed, near: float = 0.25):
    """nz seeded points of a config-1 domain (inside the unit circle, outside
    every ellipse): uniform in the disk by rejection, and a fraction `near` of
    them next to a random node, 1e-4..1e-2 of its curve's size inside G."""
    rng = np.random.default_rng(seed)
    ell = dom.meta["ellipses"]

    def inside_G(z):
        ok = np.abs(z) < 1.0
        for c, a, b, phi in ell:
            w = (z - c) * np.exp(-1j * phi)
            ok &= (w.real / a) ** 2 + (w.imag / b) ** 2 > 1.0
        return ok

    out = []
    n_near = int(round(near * nz))
    while len(out) < n_near:
        j = rng.integers(0, dom.eta.shape[0], 64)
        k = j // dom.n
        d = _near_factor(rng, j.shape[0])
        z = np.where(k == 0, dom.eta[j] * (1.0 - d), 0j)
        for e, (c, _, _, _) in enumerate(ell):
            m = k == e + 1
            z[m] = c + (dom.eta[j[m]] - c) * (1.0 + d[m])
        out.extend(z[inside_G(z)].tolist())
    out = out[:n_near]
    while len(out) < nz:
        z = np.sqrt(rng.uniform(0, 1, 256)) * np.exp(2j * np.pi * rng.uniform(0, 1, 256))
        out.extend(z[inside_G(z)].tolist())
    z = np.array(out[:nz], np.complex128)
    return z[rng.permutation(nz)]


def exterior_points_fourier(dom: Domain, nz: int, seed, near: float = 0.25, margin: float = 1.0):
    """nz seeded points outside every perturbed circle of a Fourier domain
    (config 4): uniform in the bounding square grown by `margin` by rejection
    (at least 1.5 r_j from centre j), and a fraction `near` next to a random
    node, its radius from its curve's centre grown by 1e-4..1e-2."""
    rng = np.random.default_rng(seed)
    coeffs, kmin = dom.meta["coeffs"], dom.meta["kmin"]
    cen = coeffs[:, -kmin]
    rad = np.abs(coeffs[:, 1 - kmin])

    def outside_all(z, skip=None):
        ok = np.ones(z.shape, bool)
        for q in range(cen.shape[0]):
            far = np.abs(z - cen[q]) > 1.5 * rad[q]
            ok &= far if skip is None else (far | (skip == q))
        return ok

    out = []
    n_near = int(round(near * nz))
    while len(out) < n_near:
        j = rng.integers(0, dom.eta.shape[0], 64)
        k = j // dom.n
        z = cen[k] + (dom.eta[j] - cen[k]) * (1.0 + _near_factor(rng, j.shape[0]))
        out.extend(z[outside_all(z, skip=k)].tolist())
    out = out[:n_near]
    lo = min(cen.real.min(), cen.imag.min()) - margin
    hi = max(cen.real.max(), cen.imag.max()) + margin
    while len(out) < nz:
        z = rng.uniform(lo, hi, 512) + 1j * rng.uniform(lo, hi, 512)
        out.extend(z[outside_all(z)].tolist())
    z = np.array(out[:nz], np.complex128)
    return z[rng.permutation(nz)]
