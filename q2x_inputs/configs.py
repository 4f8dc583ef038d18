"""The synthetic workloads (seeded; shapes follow the paper's tests).

Each builder returns plain numpy arrays: vertices, connectivity, densities,
element->box map and box centres/radii.  Seeds: numpy default_rng(seed) with
the workload's own seed; the draw order is fixed in each function.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import meshes, octree

TRI_SINGLE, TRI_DOUBLE, SEGMENT, TET = 0, 1, 2, 3
VERTS_PER_KIND = {TRI_SINGLE: 3, TRI_DOUBLE: 3, SEGMENT: 2, TET: 4}
KIND_NAMES = {TRI_SINGLE: "tri_single", TRI_DOUBLE: "tri_double", SEGMENT: "segment", TET: "tet"}


@dataclass
class Job:
    """One Q2X problem: a mesh of one element kind with densities and boxes."""
    name: str
    kind: int
    p: int
    verts: np.ndarray          # [V,3] float64
    elems: np.ndarray          # [N,k] int32
    density: np.ndarray        # [N] float64
    boxes: octree.Boxes
    meta: dict = field(default_factory=dict)

    @property
    def n_elems(self) -> int:
        return int(self.elems.shape[0])

    @property
    def n_boxes(self) -> int:
        return self.boxes.n_boxes

    @property
    def elem_box(self):
        return self.boxes.elem_box

    @property
    def box_center(self):
        return self.boxes.center

    @property
    def box_radius(self):
        return self.boxes.radius


def _job(name, kind, p, verts, elems, density, level, half=None, **meta):
    bx = octree.assign(verts, elems, level, half=half)
    return Job(name=name, kind=kind, p=p, verts=np.ascontiguousarray(verts, dtype=np.float64),
               elems=np.ascontiguousarray(elems, dtype=np.int32),
               density=np.ascontiguousarray(density, dtype=np.float64), boxes=bx, meta=dict(meta))


def sphere_small(seed: int = 1, p: int = 8, k: int = 3, level: int = 3, kind: int = TRI_SINGLE) -> Job:
    """Unit icosphere (20*4^k triangles), sigma ~ U[-1,1], [-1,1]^3 octree."""
    rng = np.random.default_rng(seed)
    v, f = meshes.icosphere(k)
    sigma = rng.uniform(-1.0, 1.0, f.shape[0])
    return _job(f"icosphere{k}_L{level}_p{p}", kind, p, v, f, sigma, level, half=1.0)


def perturbed_sphere_pair(seed: int = 2, p: int = 16, k: int = 6, level: int = 5):
    """Perturbed icosphere (radii 1+0.1 N(0,1), one smoothing pass), separate
    single- and double-layer densities U[-1,1].  Returns (single_job, double_job)."""
    rng = np.random.default_rng(seed)
    v, f = meshes.icosphere(k)
    v = meshes.perturb_radii(v, f, rng)
    s1 = rng.uniform(-1.0, 1.0, f.shape[0])
    s2 = rng.uniform(-1.0, 1.0, f.shape[0])
    a = _job(f"perturbed_icosphere{k}_L{level}_p{p}_single", TRI_SINGLE, p, v, f, s1, level)
    b = Job(name=f"perturbed_icosphere{k}_L{level}_p{p}_double", kind=TRI_DOUBLE, p=p, verts=a.verts,
            elems=a.elems, density=np.ascontiguousarray(s2), boxes=a.boxes)
    return a, b


def kuhn_tet_volume(seed: int = 3, p: int = 12, cells: int = 44, level: int = 6) -> Job:
    """6*cells^3 Kuhn tetrahedra of a 0.2h-jittered grid in [-1,1]^3, charge U[-1,1]."""
    rng = np.random.default_rng(seed)
    v, t = meshes.kuhn_tets(cells, rng)
    f = rng.uniform(-1.0, 1.0, t.shape[0])
    return _job(f"kuhn{cells}_tets_L{level}_p{p}", TET, p, v, t, f, level, half=1.0)


def random_filaments(seed: int = 3, p: int = 12, n_lines: int = 1000, n_steps: int = 1000,
                     level: int = 6) -> Job:
    """Random-walk polylines (step 0.002) in [-1,1]^3, line density U[-1,1]."""
    rng = np.random.default_rng(seed + 100)
    v, s = meshes.random_walks(n_lines, n_steps, rng)
    lam = rng.uniform(-1.0, 1.0, s.shape[0])
    return _job(f"walks{n_lines}x{n_steps}_L{level}_p{p}", SEGMENT, p, v, s, lam, level, half=1.0)


def large_sphere(seed: int = 7, p: int = 16, k: int = 8, level: int = 7, kind: int = TRI_SINGLE) -> Job:
    """Icosphere k=8 (1,310,720 triangles) at level 7: the >=1M-element p=16 workload."""
    rng = np.random.default_rng(seed)
    v, f = meshes.icosphere(k)
    sigma = rng.uniform(-1.0, 1.0, f.shape[0])
    return _job(f"icosphere{k}_L{level}_p{p}", kind, p, v, f, sigma, level, half=1.0)


def nu_for(n_target: float) -> int:
    return max(1, int(round(math.sqrt(n_target / 20.0))))


def perturbed_or_ellipsoid(rng, n_target: float, ellipsoid: bool):
    """A geodesic sphere with ~n_target triangles, either radially perturbed
    (as above) or scaled to an ellipsoid with axes U[0.5,1.5]."""
    v, f = meshes.geodesic_sphere(nu_for(n_target))
    if ellipsoid:
        axes = rng.uniform(0.5, 1.5, 3)
        v = v * axes[None, :]
    else:
        v = meshes.perturb_radii(v, f, rng)
    return v, f


def batch_meshes(seed: int = 4, n_meshes: int = 256, nmin: float = 1e3, nmax: float = 2e5,
                 orders=(4, 8, 12, 16, 20), scale: float = 1.0):
    """Uneven batch: n_meshes perturbed spheres or ellipsoids, N log-uniform in
    [nmin, nmax] (rounded to 20 nu^2), p from `orders`, single/double 50/50,
    octree level ceil(log8(N/32)).  `scale` shrinks N for quick tests."""
    rng = np.random.default_rng(seed)
    jobs = []
    for j in range(n_meshes):
        n = math.exp(rng.uniform(math.log(nmin), math.log(nmax))) * scale
        ell = bool(rng.integers(0, 2))
        p = int(rng.choice(orders))
        kind = TRI_SINGLE if rng.integers(0, 2) == 0 else TRI_DOUBLE
        v, f = perturbed_or_ellipsoid(rng, n, ell)
        level = max(1, int(math.ceil(math.log(max(f.shape[0], 33) / 32.0, 8))))
        sigma = rng.uniform(-1.0, 1.0, f.shape[0])
        jobs.append(_job(f"batch{j}", kind, p, v, f, sigma, level))
    return jobs


def serving_job(rng, nmin: float = 1e4, nmax: float = 2e6, pmin: int = 8, pmax: int = 24, scale: float = 1.0):
    """One serving request: perturbed geodesic sphere, N log-uniform in
    [nmin, nmax], p uniform in [pmin, pmax], single/double 50/50,
    level clamp(ceil(log4(N/32)), 2, 8)."""
    n = math.exp(rng.uniform(math.log(nmin), math.log(nmax))) * scale
    p = int(rng.integers(pmin, pmax + 1))
    kind = TRI_SINGLE if rng.integers(0, 2) == 0 else TRI_DOUBLE
    v, f = perturbed_or_ellipsoid(rng, n, False)
    level = int(min(8, max(2, math.ceil(math.log(max(f.shape[0], 33) / 32.0, 4)))))
    sigma = rng.uniform(-1.0, 1.0, f.shape[0])
    return _job(f"serve_N{f.shape[0]}_p{p}", kind, p, v, f, sigma, level)
