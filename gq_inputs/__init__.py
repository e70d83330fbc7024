"""Seeded synthetic inputs for 2-D Laplace layer-potential evaluation by QBX.

This module holds none of the method's arithmetic. It produces only the *inputs* that the
paper's algorithm assumes (Sec. 2.1 discretisation, Sec. 2.2.2 center placement, Sec. 4.2 inputs
(a)-(d)): panel-discretised closed curves with Gauss-Legendre nodes, quadrature weights that
include the arclength element, unit outward normals, QBX centers placed at y -/+ r n, the
target-to-center association for on-surface targets, densities, and harmonic test fields.

Both the CPU oracle's callers and the GPU library's callers take their inputs from here; neither
the oracle nor the library's compute path imports this module (the offline trainer of the
order-prediction network draws its training geometries from here).

Random numbers come from numpy's PCG64 generator (``numpy.random.default_rng(seed)``), so every
workload is reproducible from its seed.

Conventions
-----------
* Curves are parametrised counter-clockwise by an angle theta in [0, 2 pi); panels are uniform in
  theta. The outward unit normal of a counter-clockwise curve is the unit tangent rotated by -90
  degrees.
* Centers are stored two per source node: index 2i is the interior center y_i - r_i n_i (side -),
  index 2i+1 the exterior center y_i + r_i n_i (side +). The on-surface target i lists both, so
  the evaluated value is the average of the two one-sided limits.
* The center radius is ``radius_factor`` times the arclength L_k of the node's panel. The paper
  places centers at half of its "panel length" h_k, which it defines as half the arclength
  (Sec. 2.2.2); ``radius_factor=0.25`` reproduces that literal placement, the default 0.5 places them
  at half the arclength.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import copy
import math

import numpy as np

__all__ = [
    "StarCurve", "Geometry", "gauss_legendre", "discretize", "fourier_density",
    "unit_circle", "starfish_c1", "paper_starfish", "random_stars", "ragged_star_batch",
    "wavy_lattice", "green_test_field", "point_charge_field", "config_geometry",
]


def gauss_legendre(n: int):
    """Gauss-Legendre nodes and weights on [-1, 1] (numpy's Golub-Welsch based routine)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return x.astype(np.float64), w.astype(np.float64)


@dataclass(frozen=True)
class StarCurve:
    """r(theta) = R (1 + amp cos(arms theta + phase)), centred at (cx, cy)."""

    cx: float = 0.0
    cy: float = 0.0
    R: float = 1.0
    amp: float = 0.0
    arms: int = 0
    phase: float = 0.0

    def radius(self, th):
        return self.R * (1.0 + self.amp * np.cos(self.arms * th + self.phase))

    def dradius(self, th):
        return -self.R * self.amp * self.arms * np.sin(self.arms * th + self.phase)

    def point(self, th):
        r = self.radius(th)
        return np.stack([self.cx + r * np.cos(th), self.cy + r * np.sin(th)], axis=-1)

    def tangent(self, th):
        """Derivative of the parametrisation with respect to theta."""
        r, dr = self.radius(th), self.dradius(th)
        c, s = np.cos(th), np.sin(th)
        return np.stack([dr * c - r * s, dr * s + r * c], axis=-1)

    def max_radius(self):
        return self.R * (1.0 + abs(self.amp))


@dataclass
class Geometry:
    """Discretised source curves plus QBX centers and on-surface targets (host numpy arrays)."""

    src_xy: np.ndarray          # (N, 2) quadrature nodes
    src_nrm: np.ndarray         # (N, 2) unit outward normals
    src_w: np.ndarray           # (N,)  Gauss weight x |gamma'| x panel Jacobian
    theta: np.ndarray           # (N,)  curve parameter of each node
    curve_id: np.ndarray        # (N,)  which curve a node lies on
    panel_id: np.ndarray        # (N,)  global panel index
    panel_len: np.ndarray       # (N,)  arclength L_k of the node's panel
    ctr_xy: np.ndarray          # (2N, 2) centers, interior then exterior per node
    ctr_r: np.ndarray           # (2N,) expansion radii
    tgt_xy: np.ndarray          # (N, 2) on-surface targets (= nodes)
    tgt_ctr: np.ndarray         # (N, 2) int32 centers associated with each target
    curves: list = field(default_factory=list)
    geom_offsets: np.ndarray | None = None   # (n_geom+1,) source offsets for ragged batches

    @property
    def n_src(self):
        return self.src_xy.shape[0]

    @property
    def n_ctr(self):
        return self.ctr_xy.shape[0]

    @property
    def n_tgt(self):
        return self.tgt_xy.shape[0]

    def one_sided(self, side: int) -> "Geometry":
        """Copy whose targets use only the interior (side=-1) or exterior (side=+1) center."""
        col = 0 if side < 0 else 1
        tc = np.full_like(self.tgt_ctr, -1)
        tc[:, 0] = self.tgt_ctr[:, col]
        g = Geometry(**{k: getattr(self, k) for k in self.__dataclass_fields__})
        g.tgt_ctr = tc
        return g


def _discretize_curve(curve: StarCurve, n_panels: int, order: int, radius_factor: float):
    t, wgl = gauss_legendre(order)
    edges = np.linspace(0.0, 2.0 * np.pi, n_panels + 1)
    dth = edges[1:] - edges[:-1]
    th = (edges[:-1, None] + 0.5 * (t[None, :] + 1.0) * dth[:, None]).reshape(-1)
    xy = curve.point(th)
    tan = curve.tangent(th)
    speed = np.hypot(tan[:, 0], tan[:, 1])
    w = (wgl[None, :] * 0.5 * dth[:, None]).reshape(-1) * speed
    nrm = np.stack([tan[:, 1], -tan[:, 0]], axis=-1) / speed[:, None]
    plen = w.reshape(n_panels, order).sum(axis=1)
    plen_node = np.repeat(plen, order)
    return th, xy, nrm, w, plen_node


def discretize(curves, n_panels, order: int = 16, radius_factor: float = 0.5,
               src_order: int | None = None) -> Geometry:
    """Discretise curves into ``n_panels`` (int or per-curve list) Gauss panels of ``order`` nodes.

    With ``src_order`` the source quadrature is upsampled (Sec. 2: geometry and density are
    taken to p_quad nodes per panel for QBX): sources are the ``src_order``-node Gauss rule on
    the same panels, while centers and targets stay at the ``order`` nodes."""
    if np.isscalar(n_panels):
        n_panels = [int(n_panels)] * len(curves)
    if src_order is not None and src_order != order:
        g = discretize(curves, n_panels, order, radius_factor)
        f = discretize(curves, n_panels, src_order, radius_factor)
        g.src_xy, g.src_nrm, g.src_w = f.src_xy, f.src_nrm, f.src_w
        g.theta, g.curve_id, g.panel_id = f.theta, f.curve_id, f.panel_id
        g.panel_len = f.panel_len
        g.geom_offsets = f.geom_offsets
        return g
    parts = [_discretize_curve(c, p, order, radius_factor) for c, p in zip(curves, n_panels)]
    th = np.concatenate([p[0] for p in parts])
    xy = np.concatenate([p[1] for p in parts])
    nrm = np.concatenate([p[2] for p in parts])
    w = np.concatenate([p[3] for p in parts])
    plen = np.concatenate([p[4] for p in parts])
    cid = np.concatenate([np.full(p[0].shape[0], i, dtype=np.int32) for i, p in enumerate(parts)])
    pid = np.repeat(np.arange(sum(n_panels), dtype=np.int32), order)
    n = xy.shape[0]
    r = radius_factor * plen
    ctr = np.empty((2 * n, 2))
    ctr[0::2] = xy - r[:, None] * nrm
    ctr[1::2] = xy + r[:, None] * nrm
    ctr_r = np.repeat(r, 2)
    tgt_ctr = np.stack([np.arange(0, 2 * n, 2), np.arange(1, 2 * n, 2)], axis=1).astype(np.int32)
    offs = np.concatenate([[0], np.cumsum([p[0].shape[0] for p in parts])]).astype(np.int64)
    return Geometry(src_xy=np.ascontiguousarray(xy), src_nrm=np.ascontiguousarray(nrm),
                    src_w=np.ascontiguousarray(w), theta=th, curve_id=cid, panel_id=pid,
                    panel_len=plen, ctr_xy=ctr, ctr_r=ctr_r, tgt_xy=xy.copy(),
                    tgt_ctr=tgt_ctr, curves=list(curves), geom_offsets=offs)


def fourier_density(geom: Geometry, seed: int, kmax: int = 10, with_mean: bool = False):
    """mu(theta) = sum_{k=1..kmax} a_k cos k theta + b_k sin k theta, a_k, b_k ~ N(0, 1/k^2).

    Each curve draws its own coefficients from one generator seeded with ``seed``.
    """
    rng = np.random.default_rng(seed)
    mu = np.zeros(geom.n_src)
    ks = np.arange(1, kmax + 1)
    for c in range(len(geom.curves)):
        sel = geom.curve_id == c
        a = rng.normal(0.0, 1.0 / ks)
        b = rng.normal(0.0, 1.0 / ks)
        a0 = rng.normal() if with_mean else 0.0
        th = geom.theta[sel]
        mu[sel] = a0 + (np.cos(np.outer(th, ks)) @ a) + (np.sin(np.outer(th, ks)) @ b)
    return mu


def unit_circle(n_panels=64, order=16, radius_factor=0.5) -> Geometry:
    return discretize([StarCurve()], n_panels, order, radius_factor)


def starfish_c1(order=16, radius_factor=0.5) -> Geometry:
    """r(theta) = 1 + 0.25 cos 5 theta, 64 panels x 16 nodes = 1024 sources."""
    return discretize([StarCurve(amp=0.25, arms=5)], 64, order, radius_factor)


def paper_starfish(n_arms: int, n_panels: int, order=16, radius_factor=0.5) -> Geometry:
    """The paper's starfish family (Sec. 5): (1 + 0.8 sin(2 pi n t)) (cos 2 pi t, sin 2 pi t)."""
    return discretize([StarCurve(amp=0.8, arms=n_arms, phase=-0.5 * np.pi)], n_panels, order,
                      radius_factor)


def random_stars(n_curves=16, panels_per_curve=512, seed=1, box=40.0, order=16,
                 radius_factor=0.5, arms=(3, 9), amp=(0.1, 0.3), min_gap=0.5) -> Geometry:
    """Non-overlapping random stars r = 1 + a cos(k theta + phi) with centres in [0, box]^2.

    k ~ U{arms}, a ~ U(amp), phi ~ U(0, 2 pi); centres are rejection sampled in
    [1.5, box - 1.5]^2 so that outer circles (radius 1 + a_max) are at least ``min_gap`` apart.
    """
    rng = np.random.default_rng(seed)
    curves = []
    lo, hi = 1.5, box - 1.5
    rmax = 1.0 + amp[1]
    while len(curves) < n_curves:
        c = rng.uniform(lo, hi, size=2)
        if all(math.hypot(c[0] - o.cx, c[1] - o.cy) > 2 * rmax + min_gap for o in curves):
            curves.append(StarCurve(cx=float(c[0]), cy=float(c[1]), R=1.0,
                                    amp=float(rng.uniform(*amp)),
                                    arms=int(rng.integers(arms[0], arms[1] + 1)),
                                    phase=float(rng.uniform(0.0, 2.0 * np.pi))))
    return discretize(curves, panels_per_curve, order, radius_factor)


def ragged_star_batch(n_geoms=32, seed=200, min_nodes=1024, max_nodes=65536, order=16,
                      radius_factor=0.5):
    """Separate single-star geometries with log-uniform node counts (multiples of ``order``)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_geoms):
        nodes = int(order * round(math.exp(rng.uniform(math.log(min_nodes),
                                                       math.log(max_nodes))) / order))
        curve = StarCurve(R=1.0, amp=float(rng.uniform(0.1, 0.3)),
                          arms=int(rng.integers(3, 10)), phase=float(rng.uniform(0, 2 * np.pi)))
        out.append(discretize([curve], nodes // order, order, radius_factor))
    return out


def wavy_lattice(nx=8, ny=8, panels_per_curve=1024, seed=300, order=16, radius_factor=0.5,
                 gap_in_radii=4.0, src_order=None):
    """Wavy closed curves on an nx x ny lattice, spaced so neighbours nearly touch.

    r = 1 + a cos(k theta + phi), k ~ U{8..16}, a ~ U(0.05, 0.15); the lattice pitch leaves a
    gap of ``gap_in_radii`` times the largest expansion radius between neighbouring outer circles.
    """
    rng = np.random.default_rng(seed)
    specs = [(float(rng.uniform(0.05, 0.15)), int(rng.integers(8, 17)),
              float(rng.uniform(0, 2 * np.pi))) for _ in range(nx * ny)]
    # expansion radius is ~ radius_factor * perimeter / panels; bound the perimeter generously
    rmax_ctr = radius_factor * 2 * np.pi * 1.15 * 2.0 / panels_per_curve
    pitch = 2 * 1.15 + gap_in_radii * rmax_ctr
    curves = []
    for j in range(ny):
        for i in range(nx):
            a, k, ph = specs[j * nx + i]
            curves.append(StarCurve(cx=1.2 + i * pitch, cy=1.2 + j * pitch, R=1.0, amp=a,
                                    arms=k, phase=ph))
    return discretize(curves, panels_per_curve, order, radius_factor, src_order)


def per_center_targets(geom: Geometry) -> Geometry:
    """Copy of ``geom`` (as made by ``discretize``: target i is the node of centers 2i, 2i+1)
    with one target per center: center c evaluates at its own node alone."""
    g = copy.copy(geom)
    n = geom.tgt_xy.shape[0]
    g.tgt_xy = np.repeat(geom.tgt_xy, 2, axis=0)
    g.tgt_ctr = np.stack([np.arange(2 * n, dtype=np.int32), np.full(2 * n, -1, np.int32)], axis=1)
    return g


def order_training_geometry(seed: int, order: int = 16, radius_factor: float = 0.5,
                            src_order: int = 64):
    """A 2 x 2 lattice of random stars and a charge point x0 between them.

    Per geometry: panels per curve ~ U{64..512}; per curve k ~ U{3..16} arms with amplitude
    a ~ U(0.05, min(0.3, 2.4 / k)); the gap between neighbouring outer circles is drawn
    log-uniformly from 2.5 to 40 expansion radii, so some pairs of curves nearly touch. The
    charge point x0 (harmonic field for Green's formula) lies outside the lattice, 0.3 to 2 away
    from its bounding box, so that the density is smooth on the scale of the panels and the QBX
    error is governed by the geometry. Sources are upsampled to ``src_order`` nodes per panel.
    """
    rng = np.random.default_rng(seed)
    panels = int(rng.integers(64, 513))
    specs = []
    for _ in range(4):
        k = int(rng.integers(3, 17))
        specs.append((float(rng.uniform(0.05, min(0.3, 2.4 / k))), k,
                      float(rng.uniform(0, 2 * np.pi))))
    amax = max(a for a, _, _ in specs)
    perim = 2 * np.pi * max(math.hypot(1 + a, a * k) for a, k, _ in specs)
    rmax_ctr = radius_factor * perim / panels
    gap = float(np.exp(rng.uniform(np.log(2.5), np.log(40.0)))) * rmax_ctr
    pitch = 2 * (1 + amax) + gap
    curves = [StarCurve(cx=i * pitch, cy=j * pitch, R=1.0, amp=a, arms=k, phase=ph)
              for (a, k, ph), (i, j) in zip(specs, [(0, 0), (1, 0), (0, 1), (1, 1)])]
    geom = discretize(curves, panels, order, radius_factor, src_order)
    lo = geom.src_xy.min(axis=0)
    hi = geom.src_xy.max(axis=0)
    side = int(rng.integers(0, 4))
    dist = float(rng.uniform(0.3, 2.0))
    t = float(rng.uniform(0.0, 1.0))
    if side < 2:   # left / right of the box
        x0 = np.array([lo[0] - dist if side == 0 else hi[0] + dist, lo[1] + t * (hi[1] - lo[1])])
    else:          # below / above
        x0 = np.array([lo[0] + t * (hi[0] - lo[0]), lo[1] - dist if side == 2 else hi[1] + dist])
    return geom, x0


def point_charge_field(points: np.ndarray, normals: np.ndarray, x0):
    """u = log|x - x0| and its normal derivative n . grad u at the given points."""
    d = points - np.asarray(x0, dtype=np.float64)[None, :]
    r2 = np.einsum("ij,ij->i", d, d)
    u = 0.5 * np.log(r2)
    dudn = np.einsum("ij,ij->i", normals, d) / r2
    return u, dudn


def green_test_field(geom: Geometry, x0):
    """Densities for Green's formula S(du/dn) - D(u) with u = log|x - x0|: returns
    (sigma = du/dn at the sources, tau = u at the sources, u at the targets)."""
    u, dudn = point_charge_field(geom.src_xy, geom.src_nrm, x0)
    d = geom.tgt_xy - np.asarray(x0, dtype=np.float64)[None, :]
    return dudn, u, 0.5 * np.log(np.einsum("ij,ij->i", d, d))


def neumann_test_problem(geom: Geometry, n_charges: int = 25, seed: int = 5,
                         inner: float = 0.5, outer: float = 1.5):
    """A manufactured exterior Neumann problem in the manner of Table 5: for every curve of the
    geometry, n_charges point charges ~ N(0, 1) (seeded) at radius inner x R about its center at
    angles pi/2 + 2 pi i / n_charges, and as many check points at radius outer x R on the
    opposite rays. With u(x) = -1/(2 pi) sum_j q_j log|x - z_j|, returns (g, x_check, u_check):
    g = n . grad u at the nodes (the Neumann data), the check points and u there."""
    rng = np.random.default_rng(seed)
    zs, qs, xs = [], [], []
    al = np.pi / 2 + 2 * np.pi * np.arange(n_charges) / n_charges
    for c in geom.curves:
        zs.append(np.stack([c.cx + inner * c.R * np.cos(al), c.cy + inner * c.R * np.sin(al)], 1))
        qs.append(rng.standard_normal(n_charges))
        xs.append(np.stack([c.cx + outer * c.R * np.cos(np.pi + al),
                            c.cy + outer * c.R * np.sin(np.pi + al)], 1))
    z, q, xc = np.concatenate(zs), np.concatenate(qs), np.concatenate(xs)

    def field(x, nrm=None):
        d = x[:, None, :] - z[None, :, :]
        r2 = d[..., 0] ** 2 + d[..., 1] ** 2
        if nrm is None:
            return -(0.5 / np.pi) * (q[None, :] * 0.5 * np.log(r2)).sum(1)
        dn = (nrm[:, None, 0] * d[..., 0] + nrm[:, None, 1] * d[..., 1]) / r2
        return -(0.5 / np.pi) * (q[None, :] * dn).sum(1)

    return field(geom.src_xy, geom.src_nrm), xc, field(xc)


def config_geometry(name: str) -> Geometry:
    """Named workloads: 'c1' starfish (1024 sources), 'c2' 16 random stars (131072 sources)."""
    if name == "c1":
        return starfish_c1()
    if name == "c2":
        return random_stars(n_curves=16, panels_per_curve=512, seed=1)
    raise ValueError(name)
