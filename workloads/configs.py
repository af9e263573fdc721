"""The synthetic workloads: grids, parameters and part pairs.

Conventions shared by every consumer:
  * a grid has n = (nx, ny, nz) nodes (nz = 1 for planar work), spacing h and
    origin o; node p = (i, j, k) sits at o + h * p.  Flat index
    (k * ny + j) * nx + i (x fastest).
  * the fixed part S1 lives on an N^3 (or N^2 x 1) grid; the moving part S2 on
    its own body box of N_M^3 nodes whose node k sits at body position
    x_k = h (k - N_M / 2) relative to the body origin.
  * a pose (R, t) maps the body point x to R x + o_F + h t (t in grid units).

Parameters default to the values of the planar validation runs:
lambda1 = 1, lambda2 = 3, sigma = 0.5, eps = 3 sigma = 1.5.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import rotations as rot
from . import shapes


@dataclass(frozen=True)
class GridSpec:
    n: tuple  # (nx, ny, nz)
    origin: tuple  # world position of node (0, 0, 0)
    h: float = 1.0

    @property
    def size(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def planar(self) -> bool:
        return self.n[2] == 1

    def node_positions(self) -> np.ndarray:
        """(size, 3) world positions in flat (x fastest) order."""
        nx, ny, nz = self.n
        k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        p = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64)
        return np.asarray(self.origin, dtype=np.float64) + self.h * p


@dataclass(frozen=True)
class SDFParams:
    lambda1: float = 1.0
    lambda2: float = 3.0
    sigma: float = 0.5
    eps: float = 1.5
    xi_floor: float = 0.5


@dataclass
class PartSpec:
    samples: shapes.PointSamples
    grid: GridSpec
    body_origin: tuple = (0.0, 0.0, 0.0)


@dataclass
class PairSpec:
    name: str
    fixed: PartSpec
    moving: PartSpec
    params: SDFParams
    quats: np.ndarray
    dtype: str = "f32"
    notes: dict = field(default_factory=dict)

    @property
    def n_fixed(self) -> int:
        return self.fixed.grid.n[0]

    @property
    def n_moving(self) -> int:
        return self.moving.grid.n[0]


def body_grid(n_m: int, body_origin, h: float = 1.0, planar: bool = False) -> GridSpec:
    """Body box whose node k is at body_origin + h (k - n_m/2)."""
    o = np.asarray(body_origin, dtype=np.float64) - h * (n_m / 2.0)
    if planar:
        return GridSpec((n_m, n_m, 1), (float(o[0]), float(o[1]), float(body_origin[2])), h)
    return GridSpec((n_m, n_m, n_m), tuple(float(v) for v in o), h)


def fits_on_torus(n: int, n_m: int, planar: bool = False) -> bool:
    """A rotated body box plus its 4-wide spreading stencil never overlaps
    itself on the N-periodic grid."""
    diag = math.sqrt(2.0 if planar else 3.0) * n_m
    return math.ceil(diag) + 4 <= n


# ---------------------------------------------------------------------------
# config 1: planar peg in hole
# ---------------------------------------------------------------------------

def peg_in_hole_2d(seed: int = 0, n: int = 128, n_m: int = 64, samples: int = 512,
                   n_rot: int = 36) -> PairSpec:
    rng = np.random.default_rng(seed)
    hole = shapes.sample_polygon(shapes.HOLE_PART_2D, samples, rng, 0.05)
    peg = shapes.sample_polygon(shapes.PEG_2D, samples, rng, 0.05)
    half = (n - 1) / 2.0
    fixed = PartSpec(hole, GridSpec((n, n, 1), (-half, -half, 0.0), 1.0))
    body_origin = (0.5, 0.5, 0.0)  # peg centroid + half a voxel
    moving = PartSpec(peg, body_grid(n_m, body_origin, 1.0, planar=True), body_origin)
    return PairSpec("peg_in_hole_2d", fixed, moving, SDFParams(), rot.planar_rotations(10.0, n_rot), "f64",
                    notes={"seated_t": (64, 84), "seated_theta_deg": (0.0, 180.0)})


# ---------------------------------------------------------------------------
# config 2: 3D mechanical pair
# ---------------------------------------------------------------------------

def mechanical_3d(seed: int = 0, n: int = 128, n_m: int = 64, density: float = 1.0, hopf_level: int = 1) -> PairSpec:
    rng = np.random.default_rng(seed)
    a = shapes.box_with_hole(density, rng)
    b = shapes.plate_with_peg(density, rng)
    half = (n - 1) / 2.0
    fixed = PartSpec(a, GridSpec((n, n, n), (-half, -half, -half), 1.0))
    body_origin = (0.5, 0.5, 9.5)  # bounding-box centre of B + half a voxel
    moving = PartSpec(b, body_grid(n_m, body_origin, 1.0), body_origin)
    return PairSpec("mechanical_3d", fixed, moving, SDFParams(), rot.hopf_grid(hopf_level), "f32")


# ---------------------------------------------------------------------------
# config 3/4: protein-like union-of-spheres pairs
# ---------------------------------------------------------------------------

def sphere_part(count: int, box: float, seed: int, density: float = 4.0):
    rng = np.random.default_rng(seed)
    cen, rad = shapes.random_walk_chain(count, box, rng)
    return shapes.union_of_spheres_samples(cen, rad, density), cen, rad


def protein_like(seed: int = 0, n: int = 128, n_m: int = 64, receptor_spheres: int = 2000,
                 ligand_spheres: int = 500, n_rot: int = 3600, density: float = 4.0) -> PairSpec:
    box_r = 45.0 * (receptor_spheres / 2000.0) ** (1.0 / 3.0)
    box_l = 45.0 * (ligand_spheres / 2000.0) ** (1.0 / 3.0)
    rec, _, _ = sphere_part(receptor_spheres, box_r, seed * 2 + 1, density)
    lig, _, _ = sphere_part(ligand_spheres, box_l, seed * 2 + 2, density)
    half = (n - 1) / 2.0
    c = box_r / 2.0
    fixed = PartSpec(rec, GridSpec((n, n, n), (c - half, c - half, c - half), 1.0))
    body_origin = (box_l / 2.0,) * 3
    moving = PartSpec(lig, body_grid(n_m, body_origin, 1.0), body_origin)
    return PairSpec("protein_like", fixed, moving, SDFParams(), rot.uniform_quaternions(n_rot, 1000 + seed),
                    "f32", notes={"receptor_box": box_r, "ligand_box": box_l})


def uneven_pair(index: int, base_seed: int = 4000, n_rot: int = 512, density: float = 4.0) -> PairSpec:
    """Pair ``index`` of the uneven batch: log-uniform sphere counts, grid and
    body-box sizes chosen from the extents."""
    rng = np.random.default_rng(base_seed + index)
    nr = int(round(math.exp(rng.uniform(math.log(200), math.log(3000)))))
    nl = int(round(math.exp(rng.uniform(math.log(100), math.log(800)))))
    box_r = 45.0 * (nr / 2000.0) ** (1.0 / 3.0)
    box_l = 45.0 * (nl / 2000.0) ** (1.0 / 3.0)
    rec, _, _ = sphere_part(nr, box_r, base_seed * 7 + 2 * index + 1, density)
    lig, _, _ = sphere_part(nl, box_l, base_seed * 7 + 2 * index + 2, density)
    body_origin = (box_l / 2.0,) * 3
    diam = 2.0 * shapes.bounding_radius(lig, body_origin)
    n_m = next((m for m in (32, 48, 64) if m >= diam + 8), 64)
    need = max(box_r + diam + 8, math.ceil(math.sqrt(3.0) * n_m) + 4)
    n = next((m for m in (64, 96, 128) if m >= need), 128)
    half = (n - 1) / 2.0
    c = box_r / 2.0
    fixed = PartSpec(rec, GridSpec((n, n, n), (c - half, c - half, c - half), 1.0))
    moving = PartSpec(lig, body_grid(n_m, body_origin, 1.0), body_origin)
    return PairSpec(f"uneven_{index}", fixed, moving, SDFParams(),
                    rot.uniform_quaternions(n_rot, base_seed * 13 + index), "f32",
                    notes={"receptor_spheres": nr, "ligand_spheres": nl, "ligand_diameter": diam})


def _uneven_one(args):
    index, n_rot = args
    return uneven_pair(index, n_rot=n_rot)


def uneven_batch(n_pairs: int = 256, n_rot: int = 512, workers: int = 1) -> list:
    """Pairs 0 .. n_pairs - 1 of the uneven batch, generated by ``workers``
    processes (started fresh, so a parent that already uses a GPU is not
    forked)."""
    jobs = [(i, n_rot) for i in range(n_pairs)]
    if workers <= 1:
        return [_uneven_one(j) for j in jobs]
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(workers) as pool:
        return pool.map(_uneven_one, jobs, chunksize=1)


# ---------------------------------------------------------------------------
# small cases that the oracle finishes in seconds
# ---------------------------------------------------------------------------

def small_3d(seed: int = 0, n: int = 16, n_m: int = 6, n_rot: int = 5) -> PairSpec:
    """A miniature mechanical pair (scaled down so the oracle is instant)."""
    rng = np.random.default_rng(seed)
    s = n / 128.0 * 2.0
    a = shapes.PointSamples.concat(shapes.sample_box_faces((-6 * s, -6 * s, -3 * s), (6 * s, 6 * s, 3 * s), 4.0, rng))
    b = shapes.PointSamples.concat(shapes.sample_box_faces((-1.5 * s, -1.0 * s, -1.0 * s), (1.5 * s, 1.0 * s, 1.0 * s),
                                                           16.0, rng))
    half = (n - 1) / 2.0
    fixed = PartSpec(a, GridSpec((n, n, n), (-half, -half, -half), 1.0))
    body_origin = (0.25, 0.25, 0.25)
    moving = PartSpec(b, body_grid(n_m, body_origin, 1.0), body_origin)
    return PairSpec(f"small_3d_{n}", fixed, moving, SDFParams(xi_floor=0.25), rot.uniform_quaternions(n_rot, 77 + seed),
                    "f32")
