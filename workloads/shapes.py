"""Boundary point samples of the synthetic solids used as workloads.

Every solid is represented the way the affinity integral (eq. 13) consumes
it: a finite set of boundary points q_j with outward unit normals n_j and
quadrature weights w_j (area elements in 3D, arc lengths in 2D), so that
sum_j w_j g(q_j) approximates the surface integral of g over the boundary.

Shapes:
  * 2D peg-in-hole pair: polygons sampled at arc-length midpoints with a
    seeded tangential jitter (the validation section's planar examples use
    piecewise-linear boundaries integrated by Riemann sums).
  * 3D mechanical pair: a box with a cylindrical hole and a plate with a
    cylindrical peg, sampled by stratified jittered cells at a given density.
  * protein-like pairs: unions of spheres on a self-avoiding random-walk
    chain, sampled with Fibonacci points per sphere, points buried inside a
    neighbouring sphere dropped.

All randomness comes from ``numpy.random.default_rng(seed)``.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class PointSamples:
    """Oriented boundary samples of one solid.

    q: (n, 3) float64 positions; n: (n, 3) float64 outward unit normals;
    w: (n,) float64 quadrature weights.  2D solids use z = 0 and in-plane
    normals.
    """

    q: np.ndarray
    n: np.ndarray
    w: np.ndarray

    def __post_init__(self):
        self.q = np.ascontiguousarray(self.q, dtype=np.float64).reshape(-1, 3)
        self.n = np.ascontiguousarray(self.n, dtype=np.float64).reshape(-1, 3)
        self.w = np.ascontiguousarray(self.w, dtype=np.float64).reshape(-1)
        if not (len(self.q) == len(self.n) == len(self.w)):
            raise ValueError("q, n, w must have the same number of samples")

    @property
    def count(self) -> int:
        return len(self.w)

    def translated(self, d) -> "PointSamples":
        return PointSamples(self.q + np.asarray(d, dtype=np.float64), self.n.copy(), self.w.copy())

    @staticmethod
    def concat(parts) -> "PointSamples":
        parts = list(parts)
        return PointSamples(np.concatenate([p.q for p in parts]),
                            np.concatenate([p.n for p in parts]),
                            np.concatenate([p.w for p in parts]))


# ---------------------------------------------------------------------------
# 2D polygons
# ---------------------------------------------------------------------------

def polygon_signed_area(verts) -> float:
    v = np.asarray(verts, dtype=np.float64)
    x, y = v[:, 0], v[:, 1]
    return 0.5 * float(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))


def sample_polygon(verts, count: int, rng: np.random.Generator | None, jitter: float = 0.05) -> PointSamples:
    """Sample a closed counter-clockwise polygon at ``count`` arc-length points.

    Point i sits at arc length (i + 1/2) L / count plus a uniform tangential
    jitter in [-jitter, jitter] (wrapped around the loop); its weight is
    L / count and its normal is the outward normal of the edge it lands on.
    """
    v = np.asarray(verts, dtype=np.float64)
    if polygon_signed_area(v) <= 0:
        raise ValueError("polygon must be counter-clockwise")
    nxt = np.roll(v, -1, axis=0)
    edge = nxt - v
    elen = np.hypot(edge[:, 0], edge[:, 1])
    cum = np.concatenate([[0.0], np.cumsum(elen)])
    total = cum[-1]
    s = (np.arange(count) + 0.5) * (total / count)
    if rng is not None and jitter > 0:
        s = s + rng.uniform(-jitter, jitter, size=count)
    s = np.mod(s, total)
    e = np.clip(np.searchsorted(cum, s, side="right") - 1, 0, len(v) - 1)
    t = (s - cum[e]) / elen[e]
    pts = v[e] + t[:, None] * edge[e]
    d = edge[e] / elen[e][:, None]
    nrm = np.stack([d[:, 1], -d[:, 0]], axis=1)  # outward for a CCW loop
    q = np.zeros((count, 3))
    q[:, :2] = pts
    n3 = np.zeros((count, 3))
    n3[:, :2] = nrm
    w = np.full(count, total / count)
    return PointSamples(q, n3, w)


HOLE_PART_2D = [(-40.0, -40.0), (40.0, -40.0), (40.0, 40.0), (10.0, 40.0), (10.0, 0.0),
                (-10.0, 0.0), (-10.0, 40.0), (-40.0, 40.0)]
"""80 x 80 square with a 20 x 40 slot cut from its top edge (CCW)."""

PEG_2D = [(-10.0, -20.0), (10.0, -20.0), (10.0, 20.0), (-10.0, 20.0)]
"""20 x 40 rectangle centred at the origin (CCW)."""


# ---------------------------------------------------------------------------
# 3D analytic patches, stratified jittered sampling
# ---------------------------------------------------------------------------

def _jittered_cells(nu: int, nv: int, rng: np.random.Generator):
    iu, iv = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    u = (iu.ravel() + rng.uniform(0.0, 1.0, iu.size)) / nu
    v = (iv.ravel() + rng.uniform(0.0, 1.0, iv.size)) / nv
    return u, v


def sample_rect(origin, eu, ev, normal, density: float, rng, hole=None) -> PointSamples:
    """Planar parallelogram origin + u*eu + v*ev, u, v in [0, 1].

    ``hole`` = (centre(3), radius): points inside the disk are dropped and the
    weight becomes (area - hole area) / kept count.
    """
    origin, eu, ev = (np.asarray(a, dtype=np.float64) for a in (origin, eu, ev))
    lu, lv = np.linalg.norm(eu), np.linalg.norm(ev)
    nu = max(1, int(round(lu * math.sqrt(density))))
    nv = max(1, int(round(lv * math.sqrt(density))))
    u, v = _jittered_cells(nu, nv, rng)
    pts = origin + u[:, None] * eu + v[:, None] * ev
    area = lu * lv
    if hole is not None:
        c, r = np.asarray(hole[0], dtype=np.float64), float(hole[1])
        keep = np.linalg.norm(pts - c, axis=1) >= r
        pts = pts[keep]
        area -= math.pi * r * r
    nrm = np.broadcast_to(np.asarray(normal, dtype=np.float64), pts.shape).copy()
    return PointSamples(pts, nrm, np.full(len(pts), area / len(pts)))


def sample_disk(centre, radius: float, normal_z: float, density: float, rng) -> PointSamples:
    """Horizontal disk; jittered cells of the bounding square, outside dropped."""
    c = np.asarray(centre, dtype=np.float64)
    side = 2.0 * radius
    n1 = max(1, int(round(side * math.sqrt(density))))
    u, v = _jittered_cells(n1, n1, rng)
    x = c[0] - radius + side * u
    y = c[1] - radius + side * v
    keep = (x - c[0]) ** 2 + (y - c[1]) ** 2 < radius * radius
    pts = np.stack([x[keep], y[keep], np.full(keep.sum(), c[2])], axis=1)
    nrm = np.zeros_like(pts)
    nrm[:, 2] = normal_z
    return PointSamples(pts, nrm, np.full(len(pts), math.pi * radius * radius / len(pts)))


def sample_cylinder_wall(centre_xy, radius: float, z0: float, z1: float, outward: bool,
                         density: float, rng) -> PointSamples:
    """Vertical cylinder wall; ``outward`` False makes normals point to the axis."""
    circ = 2.0 * math.pi * radius
    h = z1 - z0
    nphi = max(3, int(round(circ * math.sqrt(density))))
    nz = max(1, int(round(h * math.sqrt(density))))
    u, v = _jittered_cells(nphi, nz, rng)
    phi = 2.0 * math.pi * u
    cx, cy = centre_xy
    pts = np.stack([cx + radius * np.cos(phi), cy + radius * np.sin(phi), z0 + h * v], axis=1)
    sgn = 1.0 if outward else -1.0
    nrm = np.stack([sgn * np.cos(phi), sgn * np.sin(phi), np.zeros_like(phi)], axis=1)
    return PointSamples(pts, nrm, np.full(len(pts), circ * h / len(pts)))


def sample_box_faces(lo, hi, density: float, rng, skip_top=False) -> list:
    """Five or six faces of an axis-aligned box with outward normals."""
    (x0, y0, z0), (x1, y1, z1) = lo, hi
    dx, dy, dz = x1 - x0, y1 - y0, z1 - z0
    faces = [
        sample_rect((x0, y0, z0), (0, dy, 0), (dx, 0, 0), (0, 0, -1), density, rng),  # bottom
        sample_rect((x0, y0, z0), (0, 0, dz), (0, dy, 0), (-1, 0, 0), density, rng),  # x-
        sample_rect((x1, y0, z0), (0, dy, 0), (0, 0, dz), (1, 0, 0), density, rng),  # x+
        sample_rect((x0, y0, z0), (dx, 0, 0), (0, 0, dz), (0, -1, 0), density, rng),  # y-
        sample_rect((x0, y1, z0), (0, 0, dz), (dx, 0, 0), (0, 1, 0), density, rng),  # y+
    ]
    if not skip_top:
        faces.append(sample_rect((x0, y0, z1), (dx, 0, 0), (0, dy, 0), (0, 0, 1), density, rng))
    return faces


def box_with_hole(density: float, rng) -> PointSamples:
    """Part A: [-30,30]^2 x [-15,15] minus the cylinder r = 10, z in [-5, 15]."""
    faces = sample_box_faces((-30.0, -30.0, -15.0), (30.0, 30.0, 15.0), density, rng, skip_top=True)
    faces.append(sample_rect((-30.0, -30.0, 15.0), (60.0, 0, 0), (0, 60.0, 0), (0, 0, 1), density, rng,
                             hole=((0.0, 0.0, 15.0), 10.0)))
    faces.append(sample_cylinder_wall((0.0, 0.0), 10.0, -5.0, 15.0, False, density, rng))
    faces.append(sample_disk((0.0, 0.0, -5.0), 10.0, +1.0, density, rng))
    return PointSamples.concat(faces)


def plate_with_peg(density: float, rng) -> PointSamples:
    """Part B: [-15,15]^2 x [-5,5] plus the cylinder r = 9.5, z in [5, 23]."""
    faces = sample_box_faces((-15.0, -15.0, -5.0), (15.0, 15.0, 5.0), density, rng, skip_top=True)
    faces.append(sample_rect((-15.0, -15.0, 5.0), (30.0, 0, 0), (0, 30.0, 0), (0, 0, 1), density, rng,
                             hole=((0.0, 0.0, 5.0), 9.5)))
    faces.append(sample_cylinder_wall((0.0, 0.0), 9.5, 5.0, 23.0, True, density, rng))
    faces.append(sample_disk((0.0, 0.0, 23.0), 9.5, +1.0, density, rng))
    return PointSamples.concat(faces)


def sphere_samples(centre, radius: float, density: float) -> PointSamples:
    """Fibonacci points on one sphere, weight = area / count."""
    n = max(8, int(round(density * 4.0 * math.pi * radius * radius)))
    i = np.arange(n) + 0.5
    z = 1.0 - 2.0 * i / n
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    d = np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)
    return PointSamples(np.asarray(centre) + radius * d, d, np.full(n, 4.0 * math.pi * radius * radius / n))


# ---------------------------------------------------------------------------
# union-of-spheres chains (protein-like)
# ---------------------------------------------------------------------------

def random_walk_chain(count: int, box: float, rng, step: float = 3.8, min_sep: float = 3.0,
                      rmin: float = 1.5, rmax: float = 2.0, tries: int = 64):
    """Self-avoiding random walk of sphere centres inside the cube [0, box]^3.

    Each new centre is one ``step`` away from the previous one in a uniformly
    random direction, keeps its sphere fully inside the box and keeps
    ``min_sep`` from every earlier centre.  When ``tries`` directions all fail,
    the in-box candidate farthest from the chain is taken.
    Returns (centres (count, 3), radii (count,)).
    """
    radii = rng.uniform(rmin, rmax, size=count)
    cen = np.zeros((count, 3))
    cen[0] = box / 2.0
    # Earlier centres are kept in cubic cells of side step + min_sep.  Every
    # candidate lies within `step` of the previous centre, so the centres
    # that can be within min_sep of a candidate lie in the 27 cells around
    # the previous centre's; the distances are computed exactly as over all
    # centres, so every decision (and the fallback's argmax, taken only when
    # every in-box candidate has a centre closer than min_sep) is the same.
    cell = step + min_sep
    cells = {}

    def key(p):
        return (int(p[0] // cell), int(p[1] // cell), int(p[2] // cell))

    cells.setdefault(key(cen[0]), []).append(0)
    for i in range(1, count):
        r = radii[i]
        d = rng.normal(size=(tries, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        cand = cen[i - 1] + step * d
        inside = np.all((cand >= r) & (cand <= box - r), axis=1)
        kx, ky, kz = key(cen[i - 1])
        near = [j for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)
                for j in cells.get((kx + a, ky + b, kz + c), ())]
        if near:
            prev = cen[sorted(near)]
            dmin = np.sqrt(((cand[:, None, :] - prev[None, :, :]) ** 2).sum(-1)).min(axis=1)
        else:
            dmin = np.full(tries, np.inf)
        ok = inside & (dmin >= min_sep)
        if ok.any():
            cen[i] = cand[np.argmax(ok)]
        elif inside.any():
            score = np.where(inside, dmin, -np.inf)
            cen[i] = cand[np.argmax(score)]
        else:
            cen[i] = np.clip(cand[0], r, box - r)
        cells.setdefault(key(cen[i]), []).append(i)
    return cen, radii


def union_of_spheres_samples(centres, radii, density: float) -> PointSamples:
    """Boundary samples of a union of spheres: per-sphere Fibonacci points,
    points strictly inside another sphere dropped; weights keep area/count of
    their own sphere."""
    from scipy.spatial import cKDTree

    centres = np.asarray(centres, dtype=np.float64)
    radii = np.asarray(radii, dtype=np.float64)
    tree = cKDTree(centres)
    rmax = float(radii.max())
    out = []
    for i, (c, r) in enumerate(zip(centres, radii)):
        s = sphere_samples(c, r, density)
        near = tree.query_ball_point(c, r + rmax)
        keep = np.ones(s.count, dtype=bool)
        for j in near:
            if j == i:
                continue
            keep &= np.linalg.norm(s.q - centres[j], axis=1) >= radii[j]
        if keep.any():
            out.append(PointSamples(s.q[keep], s.n[keep], s.w[keep]))
    return PointSamples.concat(out)


def bounding_radius(samples: PointSamples, origin) -> float:
    return float(np.linalg.norm(samples.q - np.asarray(origin), axis=1).max())
