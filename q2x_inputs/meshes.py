"""Seeded synthetic meshes shaped like the paper's test workloads.

Nothing here computes any part of the Q2X method: these are plain geometry
generators (vertex arrays, connectivity, densities) shared by the tests, the
benchmark and the smoke check.  Every random draw comes from the generator
object passed in, in a fixed order.
"""
from __future__ import annotations

import numpy as np

_PHI = (1.0 + 5.0 ** 0.5) / 2.0


def icosahedron():
    """Unit icosahedron, 12 vertices, 20 faces, counter-clockwise seen from outside."""
    v = np.array([
        [-1, _PHI, 0], [1, _PHI, 0], [-1, -_PHI, 0], [1, -_PHI, 0],
        [0, -1, _PHI], [0, 1, _PHI], [0, -1, -_PHI], [0, 1, -_PHI],
        [_PHI, 0, -1], [_PHI, 0, 1], [-_PHI, 0, -1], [-_PHI, 0, 1],
    ], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int64)
    return v, f


def _subdivide(v, f):
    """One 4-way midpoint subdivision with midpoints projected to the unit sphere."""
    nv = v.shape[0]
    a, b, c = f[:, 0], f[:, 1], f[:, 2]
    e = np.stack([np.stack([a, b], 1), np.stack([b, c], 1), np.stack([c, a], 1)], 0)  # 3 x F x 2
    lo = np.minimum(e[..., 0], e[..., 1])
    hi = np.maximum(e[..., 0], e[..., 1])
    key = lo * nv + hi
    uk, inv = np.unique(key.reshape(-1), return_inverse=True)
    inv = inv.reshape(3, -1)
    ea, eb = uk // nv, uk % nv
    mid = v[ea] + v[eb]
    mid /= np.linalg.norm(mid, axis=1, keepdims=True)
    vn = np.concatenate([v, mid], 0)
    ab, bc, ca = inv[0] + nv, inv[1] + nv, inv[2] + nv
    fn = np.concatenate([
        np.stack([a, ab, ca], 1), np.stack([b, bc, ab], 1),
        np.stack([c, ca, bc], 1), np.stack([ab, bc, ca], 1)], 0)
    # keep children of one parent together (spatially coherent element order)
    order = np.arange(fn.shape[0]).reshape(4, -1).T.reshape(-1)
    return vn, fn[order]


def icosphere(k: int):
    """Unit sphere: icosahedron subdivided k times (20*4^k triangles, outward CCW)."""
    v, f = icosahedron()
    for _ in range(k):
        v, f = _subdivide(v, f)
    return v, f.astype(np.int32)


def geodesic_sphere(nu: int):
    """Class-I geodesic sphere of frequency nu: each icosahedron face cut into
    nu^2 triangles on a barycentric grid, vertices projected to the unit sphere.
    20*nu^2 triangles, 10*nu^2+2 vertices, outward CCW."""
    v0, f0 = icosahedron()
    nu = int(nu)
    if nu < 1:
        raise ValueError("nu >= 1")
    ii, jj = np.meshgrid(np.arange(nu + 1), np.arange(nu + 1), indexing="ij")
    m = (ii + jj) <= nu
    ii, jj = ii[m], jj[m]
    kk = nu - ii - jj
    npt = ii.shape[0]
    loc = -np.ones((nu + 1, nu + 1), dtype=np.int64)
    loc[ii, jj] = np.arange(npt)
    # canonical key of every grid point: sorted (vertex id, weight) over the face corners
    fa = np.repeat(f0, npt, axis=0).reshape(20, npt, 3)
    w = np.stack([np.broadcast_to(ii, (20, npt)), np.broadcast_to(jj, (20, npt)),
                  np.broadcast_to(kk, (20, npt))], -1)
    vid = np.where(w > 0, fa, 10 ** 6)
    order = np.argsort(vid, axis=-1, kind="stable")
    vs = np.take_along_axis(vid, order, -1)
    ws = np.take_along_axis(w, order, -1)
    key = np.concatenate([vs, ws], -1).reshape(-1, 6)
    uk, inv = np.unique(key, axis=0, return_inverse=True)
    inv = inv.reshape(20, npt)
    pos = np.zeros((uk.shape[0], 3))
    for t in range(3):
        valid = uk[:, t] < 10 ** 6
        pos[valid] += uk[valid, 3 + t, None] * v0[uk[valid, t]]
    pos /= np.linalg.norm(pos, axis=1, keepdims=True)
    # small triangles of one face: up (i,j),(i+1,j),(i,j+1) and down (i+1,j),(i+1,j+1),(i,j+1)
    tri_local = []
    for i in range(nu):
        for j in range(nu - i):
            tri_local.append((loc[i, j], loc[i + 1, j], loc[i, j + 1]))
            if i + j + 1 < nu:
                tri_local.append((loc[i + 1, j], loc[i + 1, j + 1], loc[i, j + 1]))
    tri_local = np.array(tri_local, dtype=np.int64)
    faces = inv[:, tri_local].reshape(-1, 3)
    # orientation: the face corners are (A,B,C) with weights (i,j,k); the local
    # triangle above has the same handedness as (A,B,C) when viewed via (i,j).
    # Verify against the outward normal and flip where needed.
    p0, p1, p2 = pos[faces[:, 0]], pos[faces[:, 1]], pos[faces[:, 2]]
    nrm = np.cross(p1 - p0, p2 - p0)
    flip = np.einsum("ij,ij->i", nrm, p0 + p1 + p2) < 0
    faces[flip] = faces[flip][:, [0, 2, 1]]
    return pos, faces.astype(np.int32)


def vertex_neighbours_mean(values, faces, nv):
    """Mean of `values` over each vertex's edge neighbours (edges from faces)."""
    f = faces.astype(np.int64)
    e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]], 0)
    lo = np.minimum(e[:, 0], e[:, 1])
    hi = np.maximum(e[:, 0], e[:, 1])
    uk = np.unique(lo * nv + hi)
    a, b = uk // nv, uk % nv
    s = np.bincount(a, weights=values[b], minlength=nv) + np.bincount(b, weights=values[a], minlength=nv)
    cnt = np.bincount(a, minlength=nv) + np.bincount(b, minlength=nv)
    return s / np.maximum(cnt, 1)


def perturb_radii(verts, faces, rng, sigma=0.1, smooth=0.5):
    """Vertex radii 1 + sigma*N(0,1), then one umbrella (Laplacian) pass with
    weight `smooth` on the radii: r <- r + smooth*(mean_nbr(r) - r)."""
    nv = verts.shape[0]
    r = 1.0 + sigma * rng.standard_normal(nv)
    r = r + smooth * (vertex_neighbours_mean(r, faces, nv) - r)
    d = verts / np.linalg.norm(verts, axis=1, keepdims=True)
    return d * r[:, None]


def kuhn_tets(cells: int, rng, jitter=0.2, lo=-1.0, hi=1.0):
    """Kuhn 6-tet split of a jittered cells^3 grid in [lo,hi]^3.
    Interior vertices are jittered by U[-jitter*h, jitter*h]^3.
    Returns (verts [(cells+1)^3,3], tets [6*cells^3,4] int32)."""
    n = cells + 1
    h = (hi - lo) / cells
    g = np.arange(n) * h + lo
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    verts = np.stack([X, Y, Z], -1).reshape(-1, 3)
    idx = np.arange(n)
    I, J, K = np.meshgrid(idx, idx, idx, indexing="ij")
    interior = ((I > 0) & (I < cells) & (J > 0) & (J < cells) & (K > 0) & (K < cells)).reshape(-1)
    jit = rng.uniform(-jitter * h, jitter * h, size=(verts.shape[0], 3))
    verts = verts + jit * interior[:, None]

    def vid(i, j, k):
        return (i * n + j) * n + k

    ci, cj, ck = np.meshgrid(np.arange(cells), np.arange(cells), np.arange(cells), indexing="ij")
    ci, cj, ck = ci.reshape(-1), cj.reshape(-1), ck.reshape(-1)
    unit = np.eye(3, dtype=np.int64)
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    tets = np.zeros((ci.shape[0], 6, 4), dtype=np.int64)
    for t, (a, b, c) in enumerate(perms):
        p0 = np.stack([ci, cj, ck], 1)
        p1 = p0 + unit[a]
        p2 = p1 + unit[b]
        p3 = p2 + unit[c]
        for q, pp in enumerate((p0, p1, p2, p3)):
            tets[:, t, q] = vid(pp[:, 0], pp[:, 1], pp[:, 2])
    return verts, tets.reshape(-1, 4).astype(np.int32)


def random_walks(n_lines: int, n_steps: int, rng, step=0.002, start_box=0.9, wall=1.0):
    """n_lines random-walk polylines of n_steps segments each.  Starts are
    U[-start_box, start_box]^3, step directions uniform on the sphere, and a
    step that leaves [-wall, wall]^3 is reflected at the face.
    Returns (verts [n_lines*(n_steps+1),3], segs [n_lines*n_steps,2] int32)."""
    pts = np.zeros((n_lines, n_steps + 1, 3))
    pts[:, 0] = rng.uniform(-start_box, start_box, size=(n_lines, 3))
    d = rng.standard_normal((n_steps, n_lines, 3))
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    cur = pts[:, 0].copy()
    for s in range(n_steps):
        nxt = cur + step * d[s]
        nxt = np.where(nxt > wall, 2 * wall - nxt, nxt)
        nxt = np.where(nxt < -wall, -2 * wall - nxt, nxt)
        pts[:, s + 1] = nxt
        cur = nxt
    verts = pts.reshape(-1, 3)
    base = (np.arange(n_lines) * (n_steps + 1))[:, None] + np.arange(n_steps)[None, :]
    segs = np.stack([base.reshape(-1), base.reshape(-1) + 1], 1)
    return verts, segs.astype(np.int32)
