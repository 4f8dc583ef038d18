"""GPU parity of the near-field potentials (q2x_near: closed form of
Sec. 4.1, Eq. (63), double layer with the sign of the height) against the
oracle's polar quadrature, per pair and summed per target."""
import math

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

EPS = 2.2e-16


def _targets_for(xv, rng, n=24):
    """Targets above/below the interior and outside, near edges and vertices,
    heights from 1e-9 to ~3 element sizes, both sides, plus one on the element."""
    nrm = np.cross(xv[1] - xv[0], xv[2] - xv[0])
    nrm /= np.linalg.norm(nrm)
    out = []
    for _ in range(n):
        if rng.random() < 0.6:
            w = rng.dirichlet([1, 1, 1])
        else:
            w12 = rng.uniform(-0.5, 1.2, 2)
            w = np.array([w12[0], w12[1], 1.0 - w12.sum()])
        h = 10.0 ** rng.uniform(-9, 0.5) * (1 if rng.random() < 0.5 else -1)
        out.append(w @ xv + h * nrm)
    for q in range(3):
        out.append(xv[q] + 1e-7 * nrm)
        out.append(0.5 * (xv[q] + xv[(q + 1) % 3]) - 1e-6 * nrm)
    out.append(xv.mean(axis=0))  # collocation on the element itself
    return out


def _dist_to_boundary(r, xv):
    d = np.inf
    for q in range(3):
        a, b = xv[q], xv[(q + 1) % 3]
        t = np.clip(np.dot(r - a, b - a) / np.dot(b - a, b - a), 0.0, 1.0)
        d = min(d, np.linalg.norm(r - (a + t * (b - a))))
    return d


def _t(a, dt):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt).cuda()


def _run(verts, tris, targets, ps, pt, ds=None, dd=None, **kw):
    import torch
    from paper_2107_10942_amd import q2x
    ws = q2x.alloc_near_workspace()
    ent, pot = q2x.near(_t(verts, torch.float64), _t(tris, torch.int32), _t(targets, torch.float64),
                        _t(ps, torch.int64), _t(pt, torch.int32),
                        None if ds is None else _t(ds, torch.float64), None if dd is None else _t(dd, torch.float64),
                        workspace=ws, **kw)
    st = q2x.status(ws)
    torch.cuda.synchronize()
    ent = None if ent is None else (ent[0].cpu().numpy(), ent[1].cpu().numpy())
    return ent, (None if pot is None else pot.cpu().numpy()), st


def _problem(seed):
    rng = np.random.default_rng(seed)
    tris_v = [rng.normal(size=(3, 3)) * rng.uniform(0.05, 1.0) + rng.normal(size=3) for _ in range(6)]
    a = 0.7
    eq = np.array([[0, 0, 0], [a, 0, 0], [a / 2, a * math.sqrt(3) / 2, 0]])
    tris_v.append(eq)  # exactly in z = 0
    verts = np.concatenate(tris_v)
    tris = np.arange(verts.shape[0], dtype=np.int32).reshape(-1, 3)
    targets, rows = [], []
    for j, xv in enumerate(tris_v):
        for r in _targets_for(xv, rng):
            targets.append(r)
            # each target: its own triangle plus a random subset of the others, random order
            others = [k for k in range(len(tris_v)) if k != j and rng.random() < 0.5]
            row = [j] + others
            rng.shuffle(row)
            rows.append(row)
    rows[3] = []  # an empty row
    targets.append(np.array([0.3, 0.3, 0.0]))  # on the plane of the z = 0 triangle
    rows.append([len(tris_v) - 1])
    ps = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    pt = np.concatenate([np.asarray(r, np.int32) for r in rows]).astype(np.int32)
    return verts, tris, np.array(targets), ps, pt, rng


def _check_entries(verts, tris, targets, ps, pt, L, M):
    """Per-pair parity; returns the oracle's values and the per-pair bars."""
    Lr, Mr = oracle.near(verts, tris, targets, ps, pt)
    TL = np.zeros_like(Lr)
    TM = np.zeros_like(Mr)
    worstL = worstM = 0.0
    for t in range(len(targets)):
        for p in range(ps[t], ps[t + 1]):
            xv = verts[tris[pt[p]]]
            S = float(np.abs(xv).max() + np.abs(targets[t]).max())
            dL = abs(L[p] - Lr[p])
            dM = abs(M[p] - Mr[p])
            # the contour sum cancels terms of size ~ d ln d against a result of
            # size ~ area / d: relative rounding ~ eps (d / a)^2 (a the longest
            # edge, d the distance to the centroid); M is an angle: absolute
            # rounding, conditioned by 1 / (distance to the boundary)
            a = max(np.linalg.norm(xv[1] - xv[0]), np.linalg.norm(xv[2] - xv[1]), np.linalg.norm(xv[0] - xv[2]))
            d = np.linalg.norm(targets[t] - xv.mean(axis=0))
            tolL = (1e-13 + 64 * EPS * (d / a) ** 2) * abs(Lr[p])
            tolM = 1e-13 + 8 * EPS * S / max(_dist_to_boundary(targets[t], xv), 1e-300)
            assert dL <= tolL + 1e-300, (t, p, L[p], Lr[p], tolL)
            assert dM <= tolM, (t, p, M[p], Mr[p], tolM)
            TL[p], TM[p] = tolL, tolM
            worstL = max(worstL, dL / abs(Lr[p]))
            worstM = max(worstM, dM)
    print(f"near entries: worst rel L {worstL:.2e}, worst abs M {worstM:.2e}", flush=True)
    return Lr, Mr, TL, TM


def _pot_bar(ds, dd, Lr, Mr, TL, TM):
    """Bar of a target's potential: the density-weighted per-pair bars plus
    the rounding of the sum."""
    b = np.sum(np.abs(ds) * TL)
    s = np.sum(np.abs(ds * Lr))
    if dd is not None:
        b += np.sum(np.abs(dd) * TM)
        s += np.sum(np.abs(dd * Mr))
    return b + 1e-14 * s + 1e-300


def test_near_entries_and_potentials():
    verts, tris, targets, ps, pt, rng = _problem(5)
    ds = rng.uniform(-1, 1, tris.shape[0])
    dd = rng.uniform(-1, 1, tris.shape[0])
    (L, M), pot, st = _run(verts, tris, targets, ps, pt, ds, dd)
    assert st == (0, 0, 0)
    Lr, Mr, TL, TM = _check_entries(verts, tris, targets, ps, pt, L, M)
    for t in range(len(targets)):
        sl = slice(ps[t], ps[t + 1])
        ref = np.sum(ds[pt[sl]] * Lr[sl] + dd[pt[sl]] * Mr[sl])
        bar = _pot_bar(ds[pt[sl]], dd[pt[sl]], Lr[sl], Mr[sl], TL[sl], TM[sl])
        assert abs(pot[t] - ref) <= bar, (t, pot[t], ref, bar)
    assert pot[3] == 0.0  # empty row
    # on the element (centroid rows) and on the plane: principal value M = 0
    assert M[ps[-2]] == 0.0
    # entries only / potential only / single-layer density only give the same numbers
    (L2, M2), pot2, _ = _run(verts, tris, targets, ps, pt, ds, dd, potential=False)
    assert pot2 is None and np.array_equal(L2, L) and np.array_equal(M2, M)
    ent3, pot3, _ = _run(verts, tris, targets, ps, pt, ds, dd, entries=False)
    assert ent3 is None and np.array_equal(pot3, pot)
    _, pot4, _ = _run(verts, tris, targets, ps, pt, ds, None, entries=False)
    for t in range(len(targets)):
        sl = slice(ps[t], ps[t + 1])
        bar = _pot_bar(ds[pt[sl]], None, Lr[sl], Mr[sl], TL[sl], TM[sl])
        assert abs(pot4[t] - np.sum(ds[pt[sl]] * Lr[sl])) <= bar


def test_near_accumulate_and_bad_inputs():
    import torch
    from paper_2107_10942_amd import q2x
    verts, tris, targets, ps, pt, rng = _problem(6)
    ds = rng.uniform(-1, 1, tris.shape[0])
    _, pot, _ = _run(verts, tris, targets, ps, pt, ds, None, entries=False)
    base = rng.normal(size=len(targets))
    out = torch.as_tensor(base).cuda()
    _, pota, _ = _run(verts, tris, targets, ps, pt, ds, None, entries=False, accumulate=True, out_potential=out)
    assert np.max(np.abs(pota - (base + pot))) <= 1e-14 * (1 + np.abs(pota).max())
    # bad triangle id, bad vertex index, non-finite vertex, degenerate triangle
    v2, t2, pt2 = verts.copy(), tris.copy(), pt.copy()
    pt2[0] = tris.shape[0] + 3
    t2[1, 2] = verts.shape[0] + 1
    v2[t2[2, 0]] = np.nan
    t2[3, 2] = t2[3, 1]  # zero area
    (L, M), _, (flags, ndeg, nskip) = _run(v2, t2, targets, ps, pt2, ds, None)
    assert flags & q2x.FLAG_BAD_BOX and flags & q2x.FLAG_BAD_VERTEX and flags & q2x.FLAG_NONFINITE
    bad = (pt2 >= tris.shape[0]) | np.isin(pt2, [1, 2])
    assert nskip == int(bad.sum()) and ndeg == int(np.sum(pt2 == 3))
    assert np.all(L[bad] == 0) and np.all(L[pt2 == 3] == 0) and np.all(M[pt2 == 3] == 0)
    # a malformed row (decreasing pair_start) reads no pairs and is flagged
    ps3 = ps.copy()
    ps3[5] = ps3[6] + 1
    _, pot5, (f5, _, _) = _run(verts, tris, targets, ps3, pt, ds, None, entries=False)
    assert f5 & q2x.FLAG_BAD_BOX and pot5[5] == 0.0


@pytest.mark.parametrize("sample", [997])
def test_near_sphere_collocation_sampled(sample):
    """The 81,920-triangle perturbed sphere, targets at the triangle centroids
    (collocation), pairs with every triangle of the 27 boxes around the
    target's box (25.2M pairs, the benchmark's launch); every 997th target's
    row checked against the oracle, entries and potentials (single + double)."""
    import torch
    from paper_2107_10942_amd import q2x
    from q2x_inputs import configs, octree
    single, double = configs.perturbed_sphere_pair()
    cen = single.verts[single.elems].mean(axis=1)
    ps, pe = octree.near_pairs(single.boxes, single.elem_box, single.elem_box)
    (L, M), pot, st = _run(single.verts, single.elems, cen, ps, pe, single.density, double.density)
    assert st == (0, 0, 0)
    pick = np.arange(0, len(cen), sample)
    rows = [np.arange(ps[t], ps[t + 1]) for t in pick]
    sps = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    idx = np.concatenate(rows)
    Ls, Ms = L[idx], M[idx]
    Lr, Mr, TL, TM = _check_entries(single.verts, single.elems, cen[pick], sps, pe[idx], Ls, Ms)
    for k, t in enumerate(pick):
        sl = slice(sps[k], sps[k + 1])
        tri = pe[idx][sl]
        ref = np.sum(single.density[tri] * Lr[sl] + double.density[tri] * Mr[sl])
        bar = _pot_bar(single.density[tri], double.density[tri], Lr[sl], Mr[sl], TL[sl], TM[sl])
        assert abs(pot[t] - ref) <= bar
        # the target's own triangle: principal value
        own = np.nonzero(tri == t)[0]
        assert len(own) == 1 and Ms[sps[k] + own[0]] == 0.0
    del torch
