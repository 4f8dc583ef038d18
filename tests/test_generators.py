"""The seeded synthetic workloads: element and box counts, reproducibility,
orientation, octree assignment and Morton numbering (no part of the method
is computed by the generators; these tests pin the inputs every parity test
and the benchmark rely on)."""
import numpy as np
import pytest

from q2x_inputs import configs, meshes, octree


def _normals(job):
    x = job.verts[job.elems]
    return np.cross(x[:, 1] - x[:, 0], x[:, 2] - x[:, 0]), x.mean(axis=1)


def _check_boxes(job):
    """Only occupied boxes, numbered in increasing Morton order; each element's
    centroid lies in its box (half-open boxes, the last one closed); centres
    and radii follow the level's box size."""
    bx = job.boxes
    assert np.all(np.diff(bx.morton) > 0)
    assert np.array_equal(np.bincount(bx.elem_box, minlength=bx.n_boxes), bx.counts)
    assert np.all(bx.counts > 0)
    cen = job.verts[job.elems].mean(axis=1)
    d = cen - bx.center[bx.elem_box]
    assert np.all(np.abs(d) <= bx.h / 2 * (1 + 1e-12))
    np.testing.assert_allclose(octree.box_centers(bx.morton, bx.level, bx.lo, bx.half), bx.center, rtol=0,
                               atol=1e-15)
    np.testing.assert_allclose(bx.radius, np.sqrt(3) * bx.h / 2, rtol=1e-15)


def test_icosphere_k3_counts_orientation_and_boxes():
    job = configs.sphere_small()
    assert job.n_elems == 1_280 and job.verts.shape == (642, 3)
    assert job.boxes.level == 3 and job.boxes.half == 1.0 and job.n_boxes == 248
    assert job.p == 8
    nrm, cen = _normals(job)
    assert np.all(np.einsum("ij,ij->i", nrm, cen) > 0)  # outward (counter-clockwise seen from outside)
    np.testing.assert_allclose(np.linalg.norm(job.verts, axis=1), 1.0, rtol=1e-15)
    assert np.all((job.density >= -1) & (job.density <= 1))
    _check_boxes(job)


def test_perturbed_sphere_counts_orientation_and_reproducibility():
    a, b = configs.perturbed_sphere_pair()
    assert a.n_elems == 81_920 and a.verts.shape == (40_962, 3)
    assert a.p == 16 and a.boxes.level == 5 and a.n_boxes == 6_617
    assert int(a.boxes.counts.max()) == 39
    nrm, cen = _normals(a)
    assert np.all(np.einsum("ij,ij->i", nrm, cen) > 0)
    r = np.linalg.norm(a.verts, axis=1)
    assert 0.6 < r.min() and r.max() < 1.4
    # the single- and double-layer densities are separate draws
    assert not np.array_equal(a.density, b.density)
    a2, b2 = configs.perturbed_sphere_pair()
    assert np.array_equal(a.verts, a2.verts) and np.array_equal(a.density, a2.density)
    assert np.array_equal(b.density, b2.density) and np.array_equal(a.elem_box, a2.elem_box)
    a3, _ = configs.perturbed_sphere_pair(seed=3)
    assert not np.array_equal(a.verts, a3.verts)
    _check_boxes(a)


def test_kuhn_tets_tile_the_cube():
    job = configs.kuhn_tet_volume()
    assert job.n_elems == 511_104 == 6 * 44 ** 3
    assert job.verts.shape == (45 ** 3, 3)
    x = job.verts[job.elems]
    vol = np.abs(np.einsum("ij,ij->i", np.cross(x[:, 1] - x[:, 0], x[:, 2] - x[:, 0]), x[:, 3] - x[:, 0])) / 6
    # jitter moves interior vertices only, so the tets still tile [-1, 1]^3
    assert abs(vol.sum() - 8.0) < 1e-9
    h = 2.0 / 44
    assert vol.min() > 0.1 * h ** 3 / 6
    assert np.all(np.abs(job.verts) <= 1.0)
    assert job.p == 12 and job.boxes.level == 6
    _check_boxes(job)


def test_random_walk_segments():
    job = configs.random_filaments()
    assert job.n_elems == 1_000_000
    x = job.verts[job.elems]
    length = np.linalg.norm(x[:, 1] - x[:, 0], axis=1)
    assert np.all(length <= 0.002 * (1 + 1e-12))
    assert np.mean(np.abs(length - 0.002) < 1e-12) > 0.99  # reflections at the walls shorten a few
    assert np.all(np.abs(job.verts) <= 1.0)
    # polylines: consecutive segments share a vertex
    e = job.elems.reshape(1000, 1000, 2)
    assert np.array_equal(e[:, 1:, 0], e[:, :-1, 1])
    assert job.p == 12 and job.boxes.level == 6
    _check_boxes(job)


@pytest.mark.parametrize("nu", [1, 3, 7])
def test_geodesic_sphere_counts_and_orientation(nu):
    v, f = meshes.geodesic_sphere(nu)
    assert f.shape == (20 * nu * nu, 3) and v.shape == (10 * nu * nu + 2, 3)
    x = v[f]
    nrm = np.cross(x[:, 1] - x[:, 0], x[:, 2] - x[:, 0])
    assert np.all(np.einsum("ij,ij->i", nrm, x.mean(axis=1)) > 0)
    # a closed surface: every edge is shared by exactly two faces, in opposite directions
    edges = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])
    fwd = {tuple(e) for e in edges}
    assert len(fwd) == edges.shape[0]
    assert all((b, a) in fwd for a, b in fwd)


def test_batch_meshes_shape():
    """The uneven batch (a scaled-down draw): sizes 20 nu^2, orders from the
    set, octree level ceil(log8(N/32))."""
    jobs = configs.batch_meshes(n_meshes=12, scale=0.05)
    import math
    for j in jobs:
        nu = int(round(math.sqrt(j.n_elems / 20)))
        assert j.n_elems == 20 * nu * nu
        assert j.p in (4, 8, 12, 16, 20) and j.kind in (0, 1)
        assert j.boxes.level == max(1, int(math.ceil(math.log(max(j.n_elems, 33) / 32.0, 8))))
        _check_boxes(j)
    again = configs.batch_meshes(n_meshes=12, scale=0.05)
    assert all(np.array_equal(a.verts, b.verts) and a.p == b.p for a, b in zip(jobs, again))
