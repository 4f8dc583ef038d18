"""Pins of the oracle's error denominators.

Every parity gate divides the GPU/oracle difference by a scale computed by the
oracle: the per-element, per-degree norms A_{b,n} (element_norms), the
receiving side's sum of |L||I| (evaluate) and the upward pass's sum of
|coefficient||R| (m2m).  A wrong constant there (a dropped 1/4pi, a degree
slice shifted by one, |sum| in place of sum of |.|) would loosen or tighten
every gate without any parity test noticing, so each of them is checked here
against closed forms of the coefficient definition (Sec. 3.2, Eqs. (14),(20):
F_n^m = sigma (1/4pi)(-1)^n int R_n^{-m}; degree 0 is the measure, degree 1
the centroid / normal) and against R_n^m from scipy's associated Legendre
functions (Sec. 3.2, Eq. (10)), which share nothing with the oracle.
"""
import math

import numpy as np
import pytest

import oracle
import refmath

RNG = np.random.default_rng(2024)
KINDS = {"single": oracle.KIND_TRI_SINGLE, "double": oracle.KIND_TRI_DOUBLE,
         "segment": oracle.KIND_SEGMENT, "tet": oracle.KIND_TET}
NV = {"single": 3, "double": 3, "segment": 2, "tet": 4}


def idx(n, m):
    return n * n + n + m


def measure(kind, xv):
    if kind == "segment":
        return float(np.linalg.norm(xv[1] - xv[0]))
    if kind in ("single", "double"):
        return 0.5 * float(np.linalg.norm(np.cross(xv[1] - xv[0], xv[2] - xv[0])))
    return abs(float(np.dot(np.cross(xv[1] - xv[0], xv[2] - xv[0]), xv[3] - xv[0]))) / 6


def unit_normal(xv):
    cr = np.cross(xv[1] - xv[0], xv[2] - xv[0])
    return cr / np.linalg.norm(cr)


def _elements(kind, n, rng, scale=0.3):
    """n random simplices around three box centres (element e in box e % 3)."""
    nv = NV[kind]
    centres = np.array([[0.1, -0.2, 0.05], [-0.3, 0.25, 0.4], [0.5, 0.1, -0.35]])
    eb = (np.arange(n) % 3).astype(np.int32)
    xv = centres[eb][:, None, :] + scale * rng.standard_normal((n, nv, 3))
    verts = xv.reshape(-1, 3)
    elems = np.arange(n * nv, dtype=np.int32).reshape(n, nv)
    return verts, elems, eb, centres, xv


# ------------------------------------------------------------ element norms
@pytest.mark.parametrize("kind", list(KINDS))
def test_element_norms_degree0_and_degree1_closed_forms(kind):
    """||F_0|| = mu/4pi (0 for the double layer); ||F_1||^2 = (mu/4pi)^2
    (z_c^2 + (x_c^2 + y_c^2)/2) with the centroid relative to c (double layer:
    the unit normal in place of the centroid)."""
    verts, elems, eb, centres, xv = _elements(kind, 9, RNG)
    A = oracle.element_norms(KINDS[kind], 6, verts, elems, eb, centres)
    assert A.shape == (9, 7)
    for e in range(9):
        mu = measure(kind, xv[e])
        if kind == "double":
            assert A[e, 0] == 0.0
            u = unit_normal(xv[e])
        else:
            assert abs(A[e, 0] - mu / (4 * math.pi)) <= 1e-15 * mu
            u = xv[e].mean(axis=0) - centres[eb[e]]
        d1 = mu / (4 * math.pi) * math.sqrt(u[2] ** 2 + 0.5 * (u[0] ** 2 + u[1] ** 2))
        assert abs(A[e, 1] - d1) <= 1e-14 * d1, (kind, e, A[e, 1], d1)


@pytest.mark.parametrize("kind", ["single", "segment", "tet"])
def test_element_norms_point_limit_against_scipy(kind):
    """An element shrunk to a point y0 with measure mu has ||F_n|| ->
    mu/4pi ||R_n^(.)(y0 - c)|| (the monopole limit), with R from scipy; the
    relative deviation is O(n * size / |y0 - c|)."""
    p = 12
    rng = np.random.default_rng(7)
    y0 = np.array([0.21, -0.13, 0.34])
    c = np.array([-0.05, 0.02, 0.01])
    xv = y0 + 1e-7 * rng.standard_normal((NV[kind], 3))
    A = oracle.element_norms(KINDS[kind], p, xv, np.arange(NV[kind], dtype=np.int32)[None],
                             np.zeros(1, np.int32), c[None])[0]
    R = refmath.solid_R_scipy(p, *(y0 - c))
    mu = measure(kind, xv)
    for n in range(p + 1):
        ref = mu / (4 * math.pi) * np.linalg.norm(R[n * n:(n + 1) * (n + 1)])
        assert abs(A[n] - ref) <= 1e-5 * ref, (kind, n, A[n], ref)


@pytest.mark.parametrize("kind", list(KINDS))
def test_element_norms_are_the_norms_of_one_element_expansions(kind):
    """Row e equals the per-degree 2-norms of the unit-density coefficients of
    element e alone in its box (oracle.q2x, itself pinned by the closed forms
    and exact rationals of test_oracle_pins); bad box ids give a zero row."""
    p = 9
    verts, elems, eb, centres, xv = _elements(kind, 8, RNG)
    eb_bad = eb.copy()
    eb_bad[3] = -1
    eb_bad[5] = 3
    A = oracle.element_norms(KINDS[kind], p, verts, elems, eb_bad, centres)
    for e in range(8):
        if e in (3, 5):
            assert np.all(A[e] == 0.0)
            continue
        F = oracle.q2x(KINDS[kind], p, verts, elems[e:e + 1], np.ones(1), eb[e:e + 1], centres)[eb[e]]
        for n in range(p + 1):
            ref = np.linalg.norm(F[n * n:(n + 1) * (n + 1)])
            assert abs(A[e, n] - ref) <= 1e-14 * ref + 1e-300, (kind, e, n)


def test_gate_denominator_of_a_box():
    """A[b, n] = sum over the box's elements of |sigma_e| ||F^(e)_n||: the
    degree-0 entry of a box of triangles is sum |sigma_e| area_e / 4pi."""
    import metrics
    verts, elems, eb, centres, xv = _elements("single", 12, RNG)
    dens = RNG.uniform(-1, 1, 12)
    A = metrics.scale_denominator(oracle.element_norms(0, 4, verts, elems, eb, centres), dens, eb, 3)
    for b in range(3):
        ref = sum(abs(dens[e]) * measure("single", xv[e]) for e in range(12) if eb[e] == b) / (4 * math.pi)
        assert abs(A[b, 0] - ref) <= 1e-14 * ref


# ----------------------------------------------------------- receiving side
def _eval(kind, xv, c, L, p):
    vals, sc = oracle.evaluate(KINDS[kind], p, xv, np.arange(len(xv), dtype=np.int32)[None], np.zeros(1, np.int32),
                               np.asarray(c, float)[None], L[None])
    return vals[0], sc[0]


@pytest.mark.parametrize("kind", list(KINDS))
def test_eval_scale_closed_forms(kind):
    """scale = sum |L_n^m| |int R_n^m|: with L on (0,0), (1,0) and (1,-1) the
    integrals are mu, -mu z_c and mu (y_c + i x_c)/2 (double layer: 0,
    -mu n_z, mu (n_y + i n_x)/2); the phases are chosen so |value| < scale,
    so a |sum| in place of the sum of magnitudes fails."""
    p = 3
    xv = np.asarray([0.1, -0.05, 0.2]) + 0.3 * RNG.standard_normal((NV[kind], 3))
    c = np.array([0.02, 0.01, -0.04])
    mu = measure(kind, xv)
    u = unit_normal(xv) if kind == "double" else xv.mean(axis=0) - c
    i00 = 0.0 if kind == "double" else mu
    i10 = -mu * u[2]
    i1m = mu * (u[1] + 1j * u[0]) / 2
    a00, a10, a1m = 0.7 - 0.2j, -1.3 + 0.4j, 0.5 + 0.9j
    L = np.zeros((p + 1) ** 2, complex)
    L[idx(0, 0)], L[idx(1, 0)], L[idx(1, -1)] = a00, a10, a1m
    v, sc = _eval(kind, xv, c, L, p)
    ref_v = a00 * i00 + a10 * i10 + a1m * i1m
    ref_sc = abs(a00) * abs(i00) + abs(a10) * abs(i10) + abs(a1m) * abs(i1m)
    assert abs(v - ref_v) <= 1e-14 * ref_sc
    assert abs(sc - ref_sc) <= 1e-14 * ref_sc, (kind, sc, ref_sc)
    assert abs(v) < 0.999 * sc


# ----------------------------------------------------------------------- M2M
@pytest.mark.parametrize("norm", [oracle.NORM_FMM, oracle.NORM_MOMENT])
def test_m2m_scale_closed_form(norm):
    """One child with coefficients a on (0,0) and b on (1,0): the translated
    degree-n coefficients are sums of two terms a R_n and b R_{n-1} of the shift
    (Sec. 3.2, Eq. (15) by Taylor expansion), and scale[n, m] is the sum of
    their magnitudes, |a||R_n^{(.)}| + |b||R_{n-1}^{(.)}|, with R from scipy."""
    p = 10
    cc = np.array([0.12, -0.31, 0.22])
    cp = np.array([-0.2, 0.15, -0.05])
    a, b = 0.8 - 0.3j, -0.4 + 1.1j
    F = np.zeros((1, (p + 1) ** 2), complex)
    F[0, idx(0, 0)] = a
    F[0, idx(1, 0)] = b
    par, sc, skipped = oracle.m2m(p, F, cc[None], np.zeros(1, np.int32), cp[None], norm=norm)
    assert skipped == 0
    R = refmath.solid_R_scipy(p, *(cc - cp))

    def r(n, q):  # the shift's harmonic that multiplies the (k, l) = (n - j, 0) coefficient
        if abs(q) > n:
            return 0.0
        if norm == oracle.NORM_MOMENT:
            return R[idx(n, q)]
        return (-1) ** n * R[idx(n, -q)]
    for n in range(p + 1):
        for m in range(-n, n + 1):
            ta = a * r(n, m)
            tb = b * r(n - 1, m) if n >= 1 else 0.0
            ref_sc = abs(ta) + abs(tb)
            assert abs(sc[0, idx(n, m)] - ref_sc) <= 1e-14 * ref_sc + 1e-300, (norm, n, m)
            assert abs(par[0, idx(n, m)] - (ta + tb)) <= 1e-14 * ref_sc + 1e-300, (norm, n, m)
