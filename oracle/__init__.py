"""CPU FP64 oracle for the Q2X hot path -- TEST INFRASTRUCTURE ONLY.

Plain Gauss-Legendre quadrature on collapsed (Duffy) coordinates of the
regular solid harmonics R_n^m (Sec. 3.2, Eqs. (10)-(11)), summed per box
(Sec. 2, Eq. (5); Sec. 3.2, Eq. (14)).  See ``q2x_oracle.c`` for the method.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg may import this package.  It shares no code with the GPU library.
"""
import ctypes
import os

import numpy as np

from . import build as _build

KIND_TRI_SINGLE = 0
KIND_TRI_DOUBLE = 1
KIND_SEGMENT = 2
KIND_TET = 3
NORM_FMM = 0
NORM_MOMENT = 1
VERTS_PER_KIND = {KIND_TRI_SINGLE: 3, KIND_TRI_DOUBLE: 3, KIND_SEGMENT: 2, KIND_TET: 4}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        lp = ctypes.POINTER(ctypes.c_int64)
        i64 = ctypes.c_int64
        ci = ctypes.c_int
        L.orc_solid_harmonics.argtypes = [ci, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp]
        L.orc_gauss_legendre01.argtypes = [ci, dp, dp]
        L.orc_default_nodes.argtypes = [ci]
        L.orc_element_integral.argtypes = [ci, ci, dp, dp, ci, dp, dp]
        L.orc_bucket.argtypes = [ip, i64, i64, ip, lp, lp]
        L.orc_q2x_boxes.argtypes = [ci, ci, ci, dp, i64, ip, i64, dp, ip, dp, i64, lp, i64, ci, ci, dp]
        L.orc_q2x.argtypes = [ci, ci, ci, dp, i64, ip, i64, dp, ip, dp, i64, ci, ci, dp]
        L.orc_element_norms.argtypes = [ci, ci, dp, i64, ip, i64, ip, dp, i64, ci, ci, dp]
        L.orc_eval.argtypes = [ci, ci, dp, i64, ip, i64, ip, dp, i64, dp, ci, ci, dp, dp]
        L.orc_m2m.argtypes = [ci, ci, dp, dp, ip, i64, dp, i64, dp, dp]
        L.orc_near_one.argtypes = [dp, dp, dp, dp, ci, dp, dp]
        L.orc_near.argtypes = [dp, i64, ip, i64, dp, i64, lp, ip, ci, ci, dp, dp]
        L.orc_max_threads.argtypes = []
        _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _l(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _cplx(buf):
    return buf[..., 0] + 1j * buf[..., 1]


def max_threads() -> int:
    return int(lib().orc_max_threads())


def default_nodes(p: int) -> int:
    return int(lib().orc_default_nodes(p))


def solid_harmonics(p, x, y, z, grad=False):
    """R_n^m(x,y,z) for n<=p, m=-n..n, complex array indexed n*n+n+m.
    With grad=True also returns the (3, (p+1)^2) complex gradient."""
    nc = (p + 1) ** 2
    out = np.zeros((nc, 2))
    g = np.zeros((3, nc, 2)) if grad else None
    _, po = _d(out)
    out_p = out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    g_p = g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if grad else None
    rc = lib().orc_solid_harmonics(p, float(x), float(y), float(z), out_p, g_p)
    assert rc == 0
    if grad:
        return _cplx(out), _cplx(g)
    return _cplx(out)


def gauss_legendre01(k):
    x = np.zeros(k)
    w = np.zeros(k)
    rc = lib().orc_gauss_legendre01(k, x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    w.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert rc == 0
    return x, w


def element_integral(kind, p, xv, c, nodes=0):
    """Unit-density integral of R_n^m (double layer: n.grad R_n^m) over one
    element with vertices xv about centre c.  Returns (complex[(p+1)^2], J)."""
    nc = (p + 1) ** 2
    out = np.zeros((nc, 2))
    xv, pxv = _d(np.asarray(xv, dtype=np.float64).reshape(-1))
    c, pc = _d(np.asarray(c, dtype=np.float64).reshape(3))
    jac = ctypes.c_double(0.0)
    rc = lib().orc_element_integral(kind, p, pxv, pc, nodes, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    ctypes.byref(jac))
    assert rc == 0, rc
    return _cplx(out), jac.value


def bucket(elem_box, n_boxes):
    """Stable bucketing: (perm[valid], box_start[n_boxes+1], n_invalid)."""
    eb, peb = _i(elem_box)
    n = eb.shape[0]
    perm = np.zeros(max(n, 1), dtype=np.int32)
    bs = np.zeros(n_boxes + 1, dtype=np.int64)
    bad = ctypes.c_int64(0)
    lib().orc_bucket(peb, n, n_boxes, perm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                     bs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.byref(bad))
    return perm[: bs[-1]].copy(), bs, int(bad.value)


def q2x(kind, p, verts, elems, density, elem_box, box_center, norm=NORM_FMM, boxes=None, nodes=0,
        threads=0):
    """Per-box coefficients, complex array [n_boxes or len(boxes)][(p+1)^2]."""
    verts, pv = _d(verts)
    elems, pe = _i(elems)
    density, pd = _d(density)
    elem_box, peb = _i(elem_box)
    box_center, pbc = _d(box_center)
    nv = verts.reshape(-1, 3).shape[0]
    ne = elem_box.shape[0]
    nb = box_center.reshape(-1, 3).shape[0]
    assert elems.size == ne * VERTS_PER_KIND[kind]
    assert density.shape[0] == ne
    nc = (p + 1) ** 2
    if boxes is None:
        out = np.zeros((nb, nc, 2))
        rc = lib().orc_q2x(kind, p, norm, pv, nv, pe, ne, pd, peb, pbc, nb, nodes, threads,
                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    else:
        bl, pbl = _l(boxes)
        out = np.zeros((bl.shape[0], nc, 2))
        rc = lib().orc_q2x_boxes(kind, p, norm, pv, nv, pe, ne, pd, peb, pbc, nb, pbl, bl.shape[0], nodes,
                                 threads, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert rc == 0, rc
    return _cplx(out)


def evaluate(kind, p, verts, elems, elem_box, box_center, local, nodes=0, threads=0):
    """Receiving side: per element, sum_{n,m} L_b[n,m] int_e R_n^m(y - c_b) (double layer: n.grad R).
    `local` is complex [n_boxes][(p+1)^2].  Returns (values complex [N], scale [N])."""
    verts, pv = _d(verts)
    elems, pe = _i(elems)
    elem_box, peb = _i(elem_box)
    box_center, pbc = _d(box_center)
    nv = verts.reshape(-1, 3).shape[0]
    ne = elem_box.shape[0]
    nb = box_center.reshape(-1, 3).shape[0]
    assert elems.size == ne * VERTS_PER_KIND[kind]
    loc = np.ascontiguousarray(np.stack([np.real(local), np.imag(local)], axis=-1), dtype=np.float64)
    assert loc.shape == (nb, (p + 1) ** 2, 2)
    out = np.zeros((ne, 2))
    sc = np.zeros(ne)
    dp = ctypes.POINTER(ctypes.c_double)
    rc = lib().orc_eval(kind, p, pv, nv, pe, ne, peb, pbc, nb, loc.ctypes.data_as(dp), nodes, threads,
                        out.ctypes.data_as(dp), sc.ctypes.data_as(dp))
    assert rc == 0, rc
    return out[:, 0] + 1j * out[:, 1], sc


def m2m(p, child, child_center, child_parent, parent_center, norm=NORM_FMM):
    """Translate child expansions (complex [n_child][(p+1)^2]) to their parents'
    centres and sum per parent (addition theorem of R).  Returns
    (parent coefficients complex [n_parent][(p+1)^2], scale [n_parent][(p+1)^2], skipped)."""
    cc, pcc = _d(child_center)
    cp, pcp = _i(child_parent)
    pc, ppc = _d(parent_center)
    nchild = cp.shape[0]
    npar = pc.reshape(-1, 3).shape[0]
    ch = np.ascontiguousarray(np.stack([np.real(child), np.imag(child)], axis=-1), dtype=np.float64)
    assert ch.shape == (nchild, (p + 1) ** 2, 2)
    out = np.zeros((npar, (p + 1) ** 2, 2))
    sc = np.zeros((npar, (p + 1) ** 2))
    dp = ctypes.POINTER(ctypes.c_double)
    rc = lib().orc_m2m(p, norm, ch.ctypes.data_as(dp), pcc, pcp, nchild, ppc, npar, out.ctypes.data_as(dp),
                       sc.ctypes.data_as(dp))
    assert rc >= 0, rc
    return out[..., 0] + 1j * out[..., 1], sc, rc


def near_one(r, xv, k=24):
    """Single- and double-layer potentials (L, M) of the unit-density triangle
    xv [3][3] at the point r (polar quadrature about the projection of r)."""
    r, pr = _d(r)
    xv = np.ascontiguousarray(xv, dtype=np.float64)
    dp = ctypes.POINTER(ctypes.c_double)
    L = ctypes.c_double(0.0)
    M = ctypes.c_double(0.0)
    rc = lib().orc_near_one(pr, xv[0].ctypes.data_as(dp), xv[1].ctypes.data_as(dp), xv[2].ctypes.data_as(dp), k,
                            ctypes.byref(L), ctypes.byref(M))
    assert rc == 0, rc
    return L.value, M.value


def near(verts, tris, targets, pair_start, pair_tri, k=24, threads=0):
    """Per (target, triangle) pair in CSR order: (L [P], M [P]) of unit density."""
    verts, pv = _d(verts)
    tris, pt = _i(tris)
    targets, ptg = _d(targets)
    pair_start, pps = _l(pair_start)
    pair_tri, ppt = _i(pair_tri)
    npair = pair_tri.shape[0]
    L = np.zeros(npair)
    M = np.zeros(npair)
    dp = ctypes.POINTER(ctypes.c_double)
    rc = lib().orc_near(pv, verts.reshape(-1, 3).shape[0], pt, tris.reshape(-1, 3).shape[0], ptg,
                        targets.reshape(-1, 3).shape[0], pps, ppt, k, threads, L.ctypes.data_as(dp),
                        M.ctypes.data_as(dp))
    assert rc == 0, rc
    return L, M


def element_norms(kind, p, verts, elems, elem_box, box_center, nodes=0, threads=0):
    """out[e][n] = ||unit-density FMM coefficients of element e at degree n||_2."""
    verts, pv = _d(verts)
    elems, pe = _i(elems)
    elem_box, peb = _i(elem_box)
    box_center, pbc = _d(box_center)
    nv = verts.reshape(-1, 3).shape[0]
    ne = elem_box.shape[0]
    nb = box_center.reshape(-1, 3).shape[0]
    out = np.zeros((ne, p + 1))
    rc = lib().orc_element_norms(kind, p, pv, nv, pe, ne, peb, pbc, nb, nodes, threads,
                                 out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert rc == 0, rc
    return out
