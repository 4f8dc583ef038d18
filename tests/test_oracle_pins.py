"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms, exact rational brute force, library routines, invariants, the
paper's printed starting values and its analytic far-field potentials.
A plausible slip in the oracle (a dropped (-1)^n, the wrong sign of m, a
missing Condon-Shortley phase, a wrong Duffy Jacobian, a transposed normal)
fails at least one of them.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import refmath
from q2x_inputs import configs, meshes, octree

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.default_rng(12345)
KINDS = {"single": oracle.KIND_TRI_SINGLE, "double": oracle.KIND_TRI_DOUBLE,
         "segment": oracle.KIND_SEGMENT, "tet": oracle.KIND_TET}


def idx(n, m):
    return n * n + n + m


def _rand_simplex(nv, scale=0.3, centre=(0.2, -0.1, 0.15), rng=RNG):
    return np.asarray(centre) + scale * rng.standard_normal((nv, 3))


# ----------------------------------------------------------------- quadrature
@pytest.mark.parametrize("k", [1, 2, 5, 9, 14, 20])
def test_gauss_legendre_exact_on_monomials(k):
    x, w = oracle.gauss_legendre01(k)
    for j in range(2 * k):
        assert abs(np.sum(w * x ** j) - 1.0 / (j + 1)) < 1e-15
    xr, wr = np.polynomial.legendre.leggauss(k)
    np.testing.assert_allclose(np.sort(x), np.sort(0.5 * (xr + 1)), atol=1e-15)


# ----------------------------------------------------------- solid harmonics
@pytest.mark.parametrize("pt", [(0.3, -0.2, 0.5), (-0.7, 0.1, -0.2), (0.05, 0.9, 0.01), (0.0, 0.0, -0.8)])
def test_R_matches_scipy_lpmv(pt):
    p = 12
    R = oracle.solid_harmonics(p, *pt)
    ref = refmath.solid_R_scipy(p, *pt)
    np.testing.assert_allclose(R, ref, rtol=0, atol=1e-15 * np.max(np.abs(ref)) + 1e-300)


def test_R_at_origin_is_delta():
    R = oracle.solid_harmonics(6, 0.0, 0.0, 0.0)
    assert R[0] == 1.0 and np.all(R[1:] == 0.0)


@pytest.mark.parametrize("n,m", [(n, m) for n in range(5) for m in range(-n, n + 1)])
def test_R_exact_polynomial(n, m):
    """Exact Rodrigues-formula polynomial (sympy) at a rational point."""
    import sympy as sp
    expr, (x, y, z) = refmath.R_poly(n, m)
    pt = (sp.Rational(3, 7), sp.Rational(-2, 5), sp.Rational(5, 11))
    val = complex(expr.subs({x: pt[0], y: pt[1], z: pt[2]}))
    R = oracle.solid_harmonics(n, float(pt[0]), float(pt[1]), float(pt[2]))
    assert abs(R[idx(n, m)] - val) <= 1e-16 + 1e-15 * abs(val)


def test_symmetry_negative_m():
    """R_n^{-m} = (-1)^m conj(R_n^m)  (Sec. 3.2, Eq. (12))."""
    p = 10
    R = oracle.solid_harmonics(p, 0.4, -0.3, 0.6)
    for n in range(p + 1):
        for m in range(1, n + 1):
            assert abs(R[idx(n, -m)] - (-1) ** m * np.conj(R[idx(n, m)])) < 1e-17


def test_addition_theorem():
    """G = (1/4pi) sum (-1)^n R_n^{-m}(r') S_n^m(r), |r| > |r'| (Sec. 3.2, Eq. (13)).
    Pins the R normalisation against an independently built S."""
    p = 40
    rp = np.array([0.2, -0.15, 0.1])
    r = np.array([0.9, 0.7, -0.6])
    R = oracle.solid_harmonics(p, *rp)
    S = refmath.solid_S_scipy(p, *r)
    tot = 0.0
    for n in range(p + 1):
        for m in range(-n, n + 1):
            tot += (-1) ** n * R[idx(n, -m)] * S[idx(n, m)]
    exact = 1.0 / np.linalg.norm(r - rp)
    assert abs(tot - exact) / exact < 1e-13


def test_gradient_matches_finite_differences():
    p = 10
    x0 = np.array([0.31, -0.27, 0.44])
    R, G = oracle.solid_harmonics(p, *x0, grad=True)
    h = 1e-5
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        fd = (oracle.solid_harmonics(p, *(x0 + e)) - oracle.solid_harmonics(p, *(x0 - e))) / (2 * h)
        np.testing.assert_allclose(G[d], fd, atol=1e-9)


@pytest.mark.parametrize("n,m", [(n, m) for n in range(1, 5) for m in range(-n, n + 1)])
def test_gradient_exact_polynomial(n, m):
    import sympy as sp
    expr, (x, y, z) = refmath.R_poly(n, m)
    pt = {x: sp.Rational(2, 9), y: sp.Rational(-4, 7), z: sp.Rational(1, 3)}
    _, G = oracle.solid_harmonics(n, 2 / 9, -4 / 7, 1 / 3, grad=True)
    for d, s in enumerate((x, y, z)):
        val = complex(sp.diff(expr, s).subs(pt))
        assert abs(G[d][idx(n, m)] - val) <= 1e-15 * (1 + abs(val))


def test_ladder_relations_hold():
    """The derivative relations of Sec. 3.2, Eq. (15) hold for the oracle's
    R and gradient (a cross-check of both; the oracle does not use them)."""
    p = 8
    R, G = oracle.solid_harmonics(p, 0.35, -0.2, 0.5, grad=True)
    dx, dy, dz = G
    for n in range(1, p + 1):
        for m in range(-n, n + 1):
            lo = lambda mm: R[idx(n - 1, mm)] if abs(mm) <= n - 1 else 0.0  # noqa: E731
            assert abs(dz[idx(n, m)] + lo(m)) < 1e-15
            # d/deta = d/dx + i d/dy -> i R_{n-1}^{m+1};  d/dxi = d/dx - i d/dy -> i R_{n-1}^{m-1}
            assert abs(dx[idx(n, m)] + 1j * dy[idx(n, m)] - 1j * lo(m + 1)) < 1e-15
            assert abs(dx[idx(n, m)] - 1j * dy[idx(n, m)] - 1j * lo(m - 1)) < 1e-15


# ------------------------------------------------------------- start values
def test_start_values_golden():
    """Measures of the unit simplices = the recursion start values (Sec. 3.4, Eq. (42))."""
    vals = {}
    with open(os.path.join(GOLDEN, "start_values.txt")) as f:
        for ln in f:
            if ln.startswith("#") or not ln.strip():
                continue
            k, v = ln.split()
            vals[k] = float(Fraction(v))
    c = np.zeros(3)
    unit = {"segment": [[0, 0, 0], [1, 0, 0]],
            "single": [[0, 0, 0], [1, 0, 0], [0, 1, 0]],
            "tet": [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]]}
    I, J = oracle.element_integral(oracle.KIND_SEGMENT, 0, unit["segment"], c)
    assert J == 1.0 and abs(I[0] / J - vals["p0"]) < 1e-15 and vals["p0"] == vals["j0"]
    I, J = oracle.element_integral(oracle.KIND_TRI_SINGLE, 0, unit["single"], c)
    assert abs(I[0] / J - vals["i0"]) < 1e-15 and vals["i0"] == vals["b0"]
    I, J = oracle.element_integral(oracle.KIND_TET, 0, unit["tet"], c)
    assert abs(I[0] / J - vals["a0"]) < 1e-15
    R = oracle.solid_harmonics(0, 0.3, 0.2, 0.1)
    assert R[0] == vals["q0"]


# ----------------------------------------------- exact rational brute force
def _exact_case(kind):
    x1 = [Fraction(1, 5), Fraction(-1, 3), Fraction(2, 7)]
    edges = {"segment": [[Fraction(1, 2), Fraction(1, 4), Fraction(-1, 3)]],
             "single": [[Fraction(1, 2), Fraction(1, 4), Fraction(-1, 3)], [Fraction(-1, 5), Fraction(3, 5), Fraction(1, 6)]],
             "double": [[Fraction(1, 2), Fraction(1, 4), Fraction(-1, 3)], [Fraction(-1, 5), Fraction(3, 5), Fraction(1, 6)]],
             "tet": [[Fraction(1, 2), Fraction(1, 4), Fraction(-1, 3)], [Fraction(-1, 5), Fraction(3, 5), Fraction(1, 6)],
                     [Fraction(1, 7), Fraction(-1, 8), Fraction(2, 3)]]}[kind]
    return x1, edges


@pytest.mark.parametrize("kind", ["segment", "single", "tet", "double"])
def test_element_integral_exact_rational(kind):
    """n <= 4: exact integrals of the Rodrigues-formula polynomials over the
    element by the Dirichlet monomial rule (Sec. 3.1, Eqs. (6)-(9))."""
    import sympy as sp
    x1, edges = _exact_case(kind)
    pmax = 4
    xv = [[float(c) for c in x1]] + [[float(x1[k] + e[k]) for k in range(3)] for e in edges]
    I, J = oracle.element_integral(KINDS[kind], pmax, xv, [0.0, 0.0, 0.0])
    E = np.array([[float(c) for c in e] for e in edges])
    if kind == "segment":
        Jx = np.linalg.norm(E[0])
    elif kind in ("single", "double"):
        cr = np.cross(E[0], E[1])
        Jx = np.linalg.norm(cr)
    else:
        Jx = abs(np.dot(np.cross(E[0], E[1]), E[2]))
    assert abs(J - Jx) < 1e-15
    for n in range(pmax + 1):
        for m in range(-n, n + 1):
            expr, syms = refmath.R_poly(n, m)
            if kind == "double":
                # J * n . int grad R = (Ru x Rv) . int grad R  (rational)
                crq = [edges[0][1] * edges[1][2] - edges[0][2] * edges[1][1],
                       edges[0][2] * edges[1][0] - edges[0][0] * edges[1][2],
                       edges[0][0] * edges[1][1] - edges[0][1] * edges[1][0]]
                expr = sum(sp.Rational(crq[d].numerator, crq[d].denominator) * sp.diff(expr, syms[d]) for d in range(3))
                re, im = refmath.exact_simplex_integral(expr, syms, x1, edges)
                ex = float(re) + 1j * float(im)
            else:
                re, im = refmath.exact_simplex_integral(expr, syms, x1, edges)
                ex = (float(re) + 1j * float(im)) * Jx
            assert abs(I[idx(n, m)] - ex) <= 2e-16 * (1 + abs(ex)) * 8, (n, m, I[idx(n, m)], ex)


# ----------------------------------------------------------- closed forms
def _one_element_q2x(kind, xv, sigma, c, p, norm=oracle.NORM_FMM):
    nv = len(xv)
    return oracle.q2x(kind, p, np.asarray(xv, dtype=float), np.arange(nv, dtype=np.int32)[None],
                      np.array([sigma]), np.array([0], dtype=np.int32), np.asarray(c, dtype=float)[None],
                      norm=norm)[0]


@pytest.mark.parametrize("kind", ["single", "segment", "tet"])
def test_monopole_dipole_closed_form(kind):
    """F_0^0 = sigma mu/4pi, F_1^0 = sigma mu z_c/4pi,
    F_1^{+-1} = -+ sigma mu (y_c +- i x_c)/8pi (centroid relative to c)."""
    nv = {"single": 3, "segment": 2, "tet": 4}[kind]
    xv = _rand_simplex(nv)
    c = np.array([0.05, 0.02, -0.03])
    sigma = -0.73
    F = _one_element_q2x(KINDS[kind], xv, sigma, c, 2)
    if kind == "segment":
        mu = np.linalg.norm(xv[1] - xv[0])
    elif kind == "single":
        mu = 0.5 * np.linalg.norm(np.cross(xv[1] - xv[0], xv[2] - xv[0]))
    else:
        mu = abs(np.dot(np.cross(xv[1] - xv[0], xv[2] - xv[0]), xv[3] - xv[0])) / 6
    xc, yc, zc = xv.mean(axis=0) - c
    s = sigma * mu
    assert abs(F[idx(0, 0)] - s / (4 * math.pi)) < 1e-15
    assert abs(F[idx(1, 0)] - s * zc / (4 * math.pi)) < 1e-15
    assert abs(F[idx(1, 1)] - (-s * (yc + 1j * xc) / (8 * math.pi))) < 1e-15
    assert abs(F[idx(1, -1)] - (s * (yc - 1j * xc) / (8 * math.pi))) < 1e-15


def test_double_layer_closed_form():
    """F_0^0 = 0, F_1^0 = sigma A n_z/4pi, F_1^{+-1} = -+ sigma A (n_y +- i n_x)/8pi."""
    xv = _rand_simplex(3)
    c = np.array([0.1, -0.2, 0.3])
    sigma = 1.37
    F = _one_element_q2x(oracle.KIND_TRI_DOUBLE, xv, sigma, c, 3)
    cr = np.cross(xv[1] - xv[0], xv[2] - xv[0])
    A = 0.5 * np.linalg.norm(cr)
    nx, ny, nz = cr / np.linalg.norm(cr)
    s = sigma * A
    assert F[idx(0, 0)] == 0.0
    assert abs(F[idx(1, 0)] - s * nz / (4 * math.pi)) < 1e-15
    assert abs(F[idx(1, 1)] - (-s * (ny + 1j * nx) / (8 * math.pi))) < 1e-15
    assert abs(F[idx(1, -1)] - (s * (ny - 1j * nx) / (8 * math.pi))) < 1e-15


# --------------------------------------------------------------- invariants
def _subdivide(kind, xv):
    x = [np.asarray(v, dtype=float) for v in xv]
    if kind == "segment":
        mid = 0.5 * (x[0] + x[1])
        return [[x[0], mid], [mid, x[1]]]
    if kind in ("single", "double"):
        a, b, c = x
        ab, bc, ca = 0.5 * (a + b), 0.5 * (b + c), 0.5 * (c + a)
        return [[a, ab, ca], [ab, b, bc], [ca, bc, c], [ab, bc, ca]]
    a, b, c, d = x
    m = lambda p, q: 0.5 * (p + q)  # noqa: E731
    ab, ac, ad, bc, bd, cd = m(a, b), m(a, c), m(a, d), m(b, c), m(b, d), m(c, d)
    return [[a, ab, ac, ad], [ab, b, bc, bd], [ac, bc, c, cd], [ad, bd, cd, d],
            [ab, ac, ad, bd], [ab, ac, bc, bd], [ac, ad, bd, cd], [ac, bc, bd, cd]]


@pytest.mark.parametrize("kind", ["segment", "single", "double", "tet"])
def test_subdivision_additivity(kind):
    nv = {"segment": 2, "single": 3, "double": 3, "tet": 4}[kind]
    xv = _rand_simplex(nv)
    c = np.array([0.0, 0.05, 0.0])
    p = 10
    whole, _ = oracle.element_integral(KINDS[kind], p, xv, c)
    parts = sum(oracle.element_integral(KINDS[kind], p, s, c)[0] for s in _subdivide(kind, xv))
    scale = np.max(np.abs(whole))
    np.testing.assert_allclose(parts, whole, atol=1e-14 * scale)


def test_closed_surface_double_layer_vanishes():
    """Constant-density double layer over a closed surface: every moment is
    zero (the flux of grad R_n^m through a closed surface is int Laplacian = 0)."""
    v, f = meshes.icosphere(1)
    v = v * np.array([1.0, 0.8, 1.3]) + np.array([0.1, -0.2, 0.05])
    p = 8
    n = f.shape[0]
    F = oracle.q2x(oracle.KIND_TRI_DOUBLE, p, v, f, np.ones(n), np.zeros(n, dtype=np.int32),
                   np.array([[0.02, 0.03, -0.01]]))[0]
    el = oracle.q2x(oracle.KIND_TRI_DOUBLE, p, v, f, np.ones(n), np.arange(n, dtype=np.int32),
                    np.tile([[0.02, 0.03, -0.01]], (n, 1)))
    assert np.max(np.abs(F)) < 1e-14 * np.max(np.abs(el))


def test_tet_equals_face_sum():
    """int_V R_n dV = 1/(n+3) sum_f h_f int_f R_n dS, h_f the signed outward
    distance of face f from the centre (Euler homogeneity + divergence theorem;
    cf. Sec. 3.3 Lemma 4 and Sec. 4.1, Eq. (66))."""
    xv = _rand_simplex(4)
    c = np.array([0.03, -0.02, 0.01])
    p = 9
    V, _ = oracle.element_integral(oracle.KIND_TET, p, xv, c)
    cen = xv.mean(axis=0)
    tot = np.zeros_like(V)
    for f in ((1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)):
        tri = xv[list(f)]
        nrm = np.cross(tri[1] - tri[0], tri[2] - tri[0])
        nrm /= np.linalg.norm(nrm)
        if np.dot(tri.mean(axis=0) - cen, nrm) < 0:
            nrm = -nrm
        h = np.dot(tri[0] - c, nrm)
        Sf, _ = oracle.element_integral(oracle.KIND_TRI_SINGLE, p, tri, c)
        tot += h * Sf
    for n in range(p + 1):
        sl = slice(n * n, (n + 1) * (n + 1))
        np.testing.assert_allclose(V[sl], tot[sl] / (n + 3), atol=1e-15 * np.max(np.abs(V[sl])) + 1e-300)


@pytest.mark.parametrize("kind", ["single", "double", "segment", "tet"])
def test_coefficient_symmetry(kind):
    """F_n^{-m} = (-1)^m conj(F_n^m) for real densities (Sec. 3.2, Eq. (12))."""
    nv = {"segment": 2, "single": 3, "double": 3, "tet": 4}[kind]
    F = _one_element_q2x(KINDS[kind], _rand_simplex(nv), 0.6, np.zeros(3), 9)
    for n in range(10):
        for m in range(1, n + 1):
            assert abs(F[idx(n, -m)] - (-1) ** m * np.conj(F[idx(n, m)])) <= 1e-16 + 1e-15 * abs(F[idx(n, m)])
        assert abs(F[idx(n, 0)].imag) <= 1e-15 * abs(F[idx(n, 0)]) + 1e-300


@pytest.mark.parametrize("kind", ["single", "double", "segment", "tet"])
def test_rotation_and_mirror(kind):
    """Rotating sources about z by alpha multiplies F_n^m by e^{-i m alpha};
    z -> -z multiplies by (-1)^{n+m}, and by -(-1)^{n+m} for the double layer
    (the right-hand normal of the mirrored vertex order flips)."""
    nv = {"segment": 2, "single": 3, "double": 3, "tet": 4}[kind]
    xv = _rand_simplex(nv)
    p = 8
    F = _one_element_q2x(KINDS[kind], xv, 1.0, np.zeros(3), p)
    a = 0.7
    Rz = np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1]])
    Fr = _one_element_q2x(KINDS[kind], xv @ Rz.T, 1.0, np.zeros(3), p)
    Fm = _one_element_q2x(KINDS[kind], xv * np.array([1, 1, -1]), 1.0, np.zeros(3), p)
    sc = np.max(np.abs(F))
    for n in range(p + 1):
        for m in range(-n, n + 1):
            assert abs(Fr[idx(n, m)] - np.exp(-1j * m * a) * F[idx(n, m)]) < 1e-14 * sc
            sgn = (-1) ** (n + m) * (-1 if kind == "double" else 1)
            assert abs(Fm[idx(n, m)] - sgn * F[idx(n, m)]) < 1e-14 * sc


@pytest.mark.parametrize("kind", ["single", "segment", "tet"])
def test_point_limit(kind):
    """A shrinking element of measure mu at y0 tends to the point source
    sigma mu (-1)^n R_n^{-m}(y0 - c)/4pi."""
    nv = {"single": 3, "segment": 2, "tet": 4}[kind]
    y0 = np.array([0.3, -0.4, 0.25])
    shape = RNG.standard_normal((nv, 3))
    shape -= shape.mean(axis=0)
    eps = 1e-6
    xv = y0 + eps * shape
    p = 6
    F = _one_element_q2x(KINDS[kind], xv, 1.0, np.zeros(3), p)
    mu = F[0].real * 4 * math.pi
    R = refmath.solid_R_scipy(p, *y0)
    for n in range(p + 1):
        for m in range(-n, n + 1):
            pt = mu * (-1) ** n * R[idx(n, -m)] / (4 * math.pi)
            assert abs(F[idx(n, m)] - pt) <= 1e-9 * mu


def test_moment_norm_relation():
    """MOMENT output = int sigma R_n^m = (-1)^{n+m} 4pi conj(F_n^m)."""
    xv = _rand_simplex(3)
    c = np.array([0.1, 0.0, -0.1])
    for kind in (oracle.KIND_TRI_SINGLE, oracle.KIND_TRI_DOUBLE):
        F = _one_element_q2x(kind, xv, 0.8, c, 7)
        M = _one_element_q2x(kind, xv, 0.8, c, 7, norm=oracle.NORM_MOMENT)
        for n in range(8):
            for m in range(-n, n + 1):
                assert abs(M[idx(n, m)] - (-1) ** (n + m) * 4 * math.pi * np.conj(F[idx(n, m)])) < 1e-15
    # and the MOMENT monopole is sigma * area
    area = 0.5 * np.linalg.norm(np.cross(xv[1] - xv[0], xv[2] - xv[0]))
    M = _one_element_q2x(oracle.KIND_TRI_SINGLE, xv, 0.8, c, 1, norm=oracle.NORM_MOMENT)
    assert abs(M[0] - 0.8 * area) < 1e-15


@pytest.mark.parametrize("kind", ["single", "double", "segment", "tet"])
def test_quadrature_converged(kind):
    """The default node count is exact: k+2 nodes agree to round-off."""
    nv = {"segment": 2, "single": 3, "double": 3, "tet": 4}[kind]
    xv = _rand_simplex(nv)
    for p in (4, 11, 16, 24):
        k = oracle.default_nodes(p)
        a, _ = oracle.element_integral(KINDS[kind], p, xv, np.zeros(3), nodes=k)
        b, _ = oracle.element_integral(KINDS[kind], p, xv, np.zeros(3), nodes=k + 2)
        for n in range(p + 1):
            sl = slice(n * n, (n + 1) * (n + 1))
            assert np.linalg.norm(a[sl] - b[sl]) <= 5e-14 * np.linalg.norm(b[sl]) + 1e-300
        # and one node fewer is NOT exact at the top degree for the tet
        if kind == "tet" and p % 2 == 1:
            c, _ = oracle.element_integral(KINDS[kind], p, xv, np.zeros(3), nodes=k - 1)
            assert np.linalg.norm(c[p * p:] - b[p * p:]) > 1e-13 * np.linalg.norm(b[p * p:])


# ------------------------------------------------- far field (E1 geometry)
def _e1_vertices(kind, rt=0.1):
    rows = []
    with open(os.path.join(GOLDEN, "e1_geometry.txt")) as f:
        for ln in f:
            if ln.startswith("#") or not ln.strip():
                continue
            k, _, *xyz = ln.split()
            if k == kind:
                rows.append([float(eval(t, {"sqrt": math.sqrt})) for t in xyz])
    rc = np.array([math.sqrt(3) / 2, 0.0, 0.0])
    return rc + rt * np.array(rows)


@pytest.mark.parametrize("kind", ["segment", "single", "double", "tet"])
@pytest.mark.parametrize("d", [1.5, 3.0, 6.0])
def test_far_field_within_truncation_bound(kind, d):
    """The order-p expansion about the origin reproduces the potential of the
    E1 element at r = d (sqrt3/2, 0, 1/2) (Sec. 4.1, Eqs. (57)-(58)) within the
    rigorous truncation bound.  The reference is direct 40-point-per-direction
    quadrature of G (numpy's Gauss-Legendre); at d = 1.5 the paper's closed
    forms (segment Eq. (59), triangle L of Eq. (63), tetrahedron by faces
    Eq. (66)) are checked against it too."""
    geo = {"segment": "segment", "single": "triangle", "double": "triangle", "tet": "tet"}[kind]
    xv = _e1_vertices(geo)
    r = d * np.array([math.sqrt(3) / 2, 0.0, 0.5])
    exact = refmath.direct_potential(kind, r, xv)
    if kind == "segment":
        closed = refmath.segment_potential(r, xv[0], xv[1])
        mu = np.linalg.norm(xv[1] - xv[0])
    elif kind == "single":
        closed = refmath.triangle_potential_L(r, xv)
        mu = 0.5 * np.linalg.norm(np.cross(xv[1] - xv[0], xv[2] - xv[0]))
    elif kind == "double":
        closed = exact
        mu = 0.5 * np.linalg.norm(np.cross(xv[1] - xv[0], xv[2] - xv[0]))
    else:
        closed = refmath.tet_potential_faces(r, xv)
        mu = abs(np.dot(np.cross(xv[1] - xv[0], xv[2] - xv[0]), xv[3] - xv[0])) / 6
    if d == 1.5:
        assert abs(closed - exact) <= 1e-12 * abs(exact)
    a = np.max(np.linalg.norm(xv, axis=1))
    for p in (4, 8, 12, 16, 20):
        F = _one_element_q2x(KINDS[kind], xv, 1.0, np.zeros(3), p)
        val = refmath.expansion_value(F, p, r)
        assert abs(val.imag) < 1e-14 * abs(exact) + 1e-18
        err = abs(val.real - exact)
        bound = refmath.truncation_bound("double" if kind == "double" else "single", p, mu, a, d)
        assert err <= bound + 1e-14 * abs(exact), (p, err, bound)
    # convergence: at d=6 and p=20 the expansion is at round-off level
    if d == 6.0:
        assert err <= 1e-13 * abs(exact)


# ----------------------------------------------------------------- bucketing
def test_bucket_matches_stable_argsort():
    rng = np.random.default_rng(5)
    nb = 37
    eb = rng.integers(-2, nb + 3, size=1000).astype(np.int32)
    perm, bs, bad = oracle.bucket(eb, nb)
    valid = (eb >= 0) & (eb < nb)
    ref = np.argsort(np.where(valid, eb, nb + 10), kind="stable")[: valid.sum()]
    assert np.array_equal(perm, ref)
    assert bad == int((~valid).sum())
    assert np.array_equal(np.diff(bs), np.bincount(eb[valid], minlength=nb))


def test_box_sum_is_sum_of_elements():
    """Per-box output = sum of its elements' single-element outputs (Sec. 2, Eq. (5))."""
    job = configs.sphere_small(p=5)
    F = oracle.q2x(job.kind, job.p, job.verts, job.elems, job.density, job.elem_box, job.box_center)
    b = int(np.argmax(job.boxes.counts))
    members = np.nonzero(job.elem_box == b)[0]
    tot = 0
    for e in members:
        tot = tot + _one_element_q2x(job.kind, job.verts[job.elems[e]], job.density[e], job.box_center[b], job.p)
    np.testing.assert_allclose(F[b], tot, atol=1e-16)


# ------------------------------------------------- receiving side (evaluation)
def _eval_one(kind, xv, c, local, p):
    nv = xv.shape[0]
    vals, sc = oracle.evaluate(kind, p, xv, np.arange(nv, dtype=np.int32)[None], np.zeros(1, np.int32),
                               np.asarray(c, dtype=float)[None], local[None])
    return vals[0], sc[0]


@pytest.mark.parametrize("kind", ["single", "double", "segment", "tet"])
def test_eval_low_order_closed_forms(kind):
    """A field 1 (L_0^0 = 1) integrates to the element's measure (0 for the
    double layer: grad 1 = 0); R_1^0 = -z and R_1^{-1} = (y + i x)/2 (the
    normalisation of Sec. 3.2, Eq. (10)) give -measure * (centroid height) and
    measure * (y_c + i x_c)/2 (double layer: the normal's components times the
    area)."""
    nv = {"single": 3, "double": 3, "segment": 2, "tet": 4}[kind]
    code = {"single": 0, "double": 1, "segment": 2, "tet": 3}[kind]
    xv = _rand_simplex(nv)
    c = np.array([0.05, 0.02, -0.03])
    p = 3
    if kind == "segment":
        mu = np.linalg.norm(xv[1] - xv[0])
    elif kind in ("single", "double"):
        mu = 0.5 * np.linalg.norm(np.cross(xv[1] - xv[0], xv[2] - xv[0]))
    else:
        mu = abs(np.dot(np.cross(xv[1] - xv[0], xv[2] - xv[0]), xv[3] - xv[0])) / 6
    xc, yc, zc = xv.mean(axis=0) - c
    L = np.zeros((p + 1) ** 2, complex)
    L[idx(0, 0)] = 1.0
    v, _ = _eval_one(code, xv, c, L, p)
    assert abs(v - (0.0 if kind == "double" else mu)) < 1e-15 * max(mu, 1)
    L[:] = 0
    L[idx(1, 0)] = 2.5
    v, _ = _eval_one(code, xv, c, L, p)
    if kind == "double":
        cr = np.cross(xv[1] - xv[0], xv[2] - xv[0])
        nz = cr[2] / np.linalg.norm(cr)
        assert abs(v + 2.5 * mu * nz) < 1e-15
    else:
        assert abs(v + 2.5 * mu * zc) < 1e-15
    L[:] = 0
    L[idx(1, -1)] = 1.0 - 0.5j
    v, _ = _eval_one(code, xv, c, L, p)
    if kind == "double":
        cr = np.cross(xv[1] - xv[0], xv[2] - xv[0])
        nx, ny, _ = cr / np.linalg.norm(cr)
        assert abs(v - (1.0 - 0.5j) * mu * (ny + 1j * nx) / 2) < 1e-15
    else:
        assert abs(v - (1.0 - 0.5j) * mu * (yc + 1j * xc) / 2) < 1e-15


@pytest.mark.parametrize("kind", ["single", "double", "segment", "tet"])
def test_eval_point_source_local_expansion(kind):
    """The local expansion about c of G(s, y) = 1/(4 pi |y - s|), built from an
    independent S_n^m (scipy) by the addition theorem of Sec. 3.2, Eq. (13):
    L_n^m = (1/4pi)(-1)^n S_n^{-m}(s - c).  Its integral over an element near c
    must match direct quadrature of G (of dG/dn for the double layer) within
    the rigorous truncation bound."""
    nv = {"single": 3, "double": 3, "segment": 2, "tet": 4}[kind]
    code = {"single": 0, "double": 1, "segment": 2, "tet": 3}[kind]
    xv = _rand_simplex(nv, scale=0.25, centre=(0.05, 0.0, 0.02))
    c = np.array([0.02, -0.01, 0.03])
    s_pt = np.array([1.1, -0.7, 0.9])
    a = float(np.max(np.linalg.norm(xv - c, axis=1)))
    d = float(np.linalg.norm(s_pt - c))
    if kind == "segment":
        mu = np.linalg.norm(xv[1] - xv[0])
    elif kind in ("single", "double"):
        mu = 0.5 * np.linalg.norm(np.cross(xv[1] - xv[0], xv[2] - xv[0]))
    else:
        mu = abs(np.dot(np.cross(xv[1] - xv[0], xv[2] - xv[0]), xv[3] - xv[0])) / 6
    ref = refmath.direct_potential({"single": "single", "double": "double", "segment": "segment",
                                    "tet": "tet"}[kind], s_pt, list(xv), k=40)
    # (for the double layer direct_potential gives n.(s - y)/(4 pi |s - y|^3) = dG/dn_y)
    for p in (6, 12, 20):
        S = refmath.solid_S_scipy(p, *(s_pt - c))
        L = np.zeros((p + 1) ** 2, complex)
        for n in range(p + 1):
            for m in range(-n, n + 1):
                L[idx(n, m)] = (-1) ** n * S[idx(n, -m)] / (4 * math.pi)
        v, sc = _eval_one(code, xv, c, L, p)
        bound = refmath.truncation_bound("double" if kind == "double" else "single", p, mu, a, d)
        assert abs(v.imag) < 1e-14 * sc
        assert abs(v.real - ref) <= bound + 1e-14 * abs(ref) + 1e-15, (kind, p, v, ref, bound)


# ----------------------------------------------------------------- M2M (upward pass)
def _child_parent_setup(kind, n_child=7, n_parent=3, n_el=40, seed=0):
    """Random elements in child boxes; children assigned to random parents
    (translation of truncated multipoles is a finite identity: any centres)."""
    rng = np.random.default_rng(seed)
    nv = oracle.VERTS_PER_KIND[kind]
    cc = rng.uniform(-1, 1, (n_child, 3))
    pc = rng.uniform(-1, 1, (n_parent, 3))
    cp = np.arange(n_child, dtype=np.int32) % n_parent
    eb = rng.integers(0, n_child, n_el).astype(np.int32)
    verts = (cc[eb][:, None, :] + 0.2 * rng.standard_normal((n_el, nv, 3))).reshape(-1, 3)
    elems = np.arange(n_el * nv, dtype=np.int32).reshape(n_el, nv)
    dens = rng.uniform(-1, 1, n_el)
    return verts, elems, dens, eb, cc, cp, pc


@pytest.mark.parametrize("norm", [oracle.NORM_FMM, oracle.NORM_MOMENT])
@pytest.mark.parametrize("kind", ["single", "double", "segment", "tet"])
def test_m2m_equals_expansion_about_the_parent(kind, norm):
    """Translating the children's coefficients (addition theorem) gives the
    coefficients computed directly about the parent's centre by quadrature of
    R_n^m(y - c_parent): a wrong sign, index or dropped term fails."""
    code = KINDS[kind]
    p = 9
    verts, elems, dens, eb, cc, cp, pc = _child_parent_setup(code, seed=3 + code)
    child = oracle.q2x(code, p, verts, elems, dens, eb, cc, norm=norm)
    par, sc, skipped = oracle.m2m(p, child, cc, cp, pc, norm=norm)
    assert skipped == 0
    direct = oracle.q2x(code, p, verts, elems, dens, cp[eb], pc, norm=norm)
    err = np.abs(par - direct) / (sc + np.abs(direct) + 1e-300)
    assert err.max() < 1e-13, err.max()
    assert np.abs(direct).max() > 1e-3


@pytest.mark.parametrize("norm", [oracle.NORM_FMM, oracle.NORM_MOMENT])
def test_m2m_point_source_closed_form(norm):
    """A unit point charge at y has coefficients (1/4pi)(-1)^n R_n^{-m}(y - c)
    (FMM; MOMENT: R_n^m(y - c)), here from scipy's associated Legendre
    functions; translated from c_c they must equal the same formula at c_p."""
    p = 12
    y = np.array([0.31, -0.12, 0.27])
    c1 = np.array([0.1, 0.05, -0.2])
    c2 = np.array([-0.4, 0.3, 0.25])

    def point(c):
        R = refmath.solid_R_scipy(p, *(y - c))
        if norm == oracle.NORM_MOMENT:
            return R
        F = np.zeros_like(R)
        for n in range(p + 1):
            for m in range(-n, n + 1):
                F[idx(n, m)] = (-1) ** n * R[idx(n, -m)] / (4 * math.pi)
        return F
    par, sc, _ = oracle.m2m(p, point(c1)[None], c1[None], np.zeros(1, np.int32), c2[None], norm=norm)
    ref = point(c2)
    assert np.max(np.abs(par[0] - ref) / (sc[0] + 1e-300)) < 1e-14


def test_m2m_identity_composition_and_skips():
    """Zero shift is the identity (exactly); c1 -> c2 -> c3 equals c1 -> c3;
    several children of one parent add; bad parent ids are skipped and counted."""
    p = 8
    rng = np.random.default_rng(9)
    F = rng.uniform(-1, 1, (1, (p + 1) ** 2)) + 1j * rng.uniform(-1, 1, (1, (p + 1) ** 2))
    c1, c2, c3 = rng.uniform(-1, 1, (3, 3))
    z = np.zeros(1, np.int32)
    same, _, _ = oracle.m2m(p, F, c1[None], z, c1[None])
    assert np.array_equal(same, F)
    a, _, _ = oracle.m2m(p, F, c1[None], z, c2[None])
    b, sb, _ = oracle.m2m(p, a, c2[None], z, c3[None])
    d, sd, _ = oracle.m2m(p, F, c1[None], z, c3[None])
    assert np.max(np.abs(b - d) / (sd + 1e-300)) < 1e-13
    two, _, _ = oracle.m2m(p, np.concatenate([F, a]), np.stack([c1, c2]), np.zeros(2, np.int32), c3[None])
    assert np.max(np.abs(two - 2 * d) / (sd + 1e-300)) < 1e-13
    bad, _, skipped = oracle.m2m(p, np.concatenate([F, F]), np.stack([c1, c1]), np.array([0, 5], np.int32), c3[None])
    assert skipped == 1 and np.array_equal(bad, d)


# ----------------------------------------------------------------- near field (analytic integrals)
_NEAR_TRI = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.05], [0.3, 0.9, -0.1]])


def _mp_vec(v):
    import mpmath as mp
    return [mp.mpf(float(c)) for c in v]


def _solid_angle_mp(r, xv):
    """Signed solid angle of the triangle seen from r, closed form of Van
    Oosterom & Strackee (IEEE Trans. Biomed. Eng. 30 (1983)), R_i = x_i - r,
    evaluated with 50 digits on the given (double) inputs."""
    import mpmath as mp
    mp.mp.dps = 50
    rr = _mp_vec(r)
    R = [[c - d for c, d in zip(_mp_vec(x), rr)] for x in xv]
    dot = lambda a, b: sum(a[i] * b[i] for i in range(3))  # noqa: E731
    cross = lambda a, b: [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]  # noqa: E731
    nr = [mp.sqrt(dot(x, x)) for x in R]
    num = dot(R[0], cross(R[1], R[2]))
    den = nr[0] * nr[1] * nr[2] + dot(R[0], R[1]) * nr[2] + dot(R[0], R[2]) * nr[1] + dot(R[1], R[2]) * nr[0]
    return 2 * mp.atan2(num, den)


def _contour_L_mp(r, xv):
    """The contour formula of Sec. 4.1, Eq. (63) for L (no sign choice
    needed), evaluated with 50 digits on the given (double) inputs."""
    import mpmath as mp
    mp.mp.dps = 50
    X = [_mp_vec(x) for x in xv]
    rr = _mp_vec(r)
    sub = lambda a, b: [a[i] - b[i] for i in range(3)]  # noqa: E731
    dot = lambda a, b: sum(a[i] * b[i] for i in range(3))  # noqa: E731
    cross = lambda a, b: [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]  # noqa: E731
    nv = cross(sub(X[1], X[0]), sub(X[2], X[0]))
    nn = mp.sqrt(dot(nv, nv))
    nv = [c / nn for c in nv]
    h = abs(dot(sub(rr, X[0]), nv))

    def MP(x, y, z):
        R = mp.sqrt(x * x + y * y + z * z)
        den = R * z * z + y * x * x
        return mp.mpf(0) if den == 0 else -mp.atan(x * z * (R - y) / den)

    def LP(x, y, z):
        R = mp.sqrt(x * x + y * y + z * z)
        return -y * MP(x, y, z) - (z * mp.log(abs(R + x)) if z != 0 else 0)

    tot = mp.mpf(0)
    for q in range(3):
        e = sub(X[(q + 1) % 3], X[q])
        lq = mp.sqrt(dot(e, e))
        iq = [c / lq for c in e]
        nq = cross(iq, nv)
        xx = dot(sub(rr, X[q]), iq)
        zq = dot(sub(rr, X[q]), nq)
        tot += LP(lq - xx, h, zq) - LP(-xx, h, zq)
    return tot / (4 * mp.pi)


def _dist_to_boundary(r, xv):
    d = np.inf
    for q in range(3):
        a, b = xv[q], xv[(q + 1) % 3]
        t = np.clip(np.dot(r - a, b - a) / np.dot(b - a, b - a), 0.0, 1.0)
        d = min(d, np.linalg.norm(r - (a + t * (b - a))))
    return d


def _near_targets(xv, rng, n=40):
    """Targets above/below the interior, near edges and vertices, at heights
    from 1e-9 to 3 element sizes (both sides)."""
    nrm = np.cross(xv[1] - xv[0], xv[2] - xv[0])
    nrm /= np.linalg.norm(nrm)
    out = []
    for _ in range(n):
        if rng.random() < 0.6:
            w = rng.dirichlet([1, 1, 1])
        else:
            w12 = rng.uniform(-0.5, 1.2, 2)
            w = np.array([w12[0], w12[1], 1.0 - w12.sum()])
        base = w @ xv
        h = 10.0 ** rng.uniform(-9, 0.5) * (1 if rng.random() < 0.5 else -1)
        out.append(base + h * nrm)
    for q in range(3):  # just above a vertex and an edge midpoint
        out.append(xv[q] + 1e-7 * nrm)
        out.append(0.5 * (xv[q] + xv[(q + 1) % 3]) - 1e-6 * nrm)
    return out


def test_near_far_matches_direct_quadrature():
    """Away from the triangle plain Gauss quadrature of G and dG/dn converges:
    the near-field oracle must agree with it (single and double layer)."""
    rng = np.random.default_rng(21)
    for _ in range(12):
        xv = _rand_simplex(3, scale=0.4, rng=rng)
        r = xv.mean(axis=0) + rng.normal(size=3) * 1.5
        L, M = oracle.near_one(r, xv)
        dl = refmath.direct_potential("single", r, list(xv), k=60)
        dm = refmath.direct_potential("double", r, list(xv), k=60)
        assert abs(L - dl) <= 1e-13 * abs(dl)
        assert abs(M - dm) <= 1e-13 * abs(L)  # M is bounded by the single layer's scale here


def test_near_double_layer_is_the_solid_angle():
    """M(r) = -Omega(r)/(4 pi) for a flat triangle (Omega: the closed form of
    Van Oosterom & Strackee at 50 digits), at heights down to 1e-9 over the
    interior, the edges and the vertices, on both sides; M = 0 on the plane.
    Near the boundary M varies like 1/delta with the distance delta to it, so
    the bar is 1e-14 + 4 eps S / delta (S the coordinate scale): the rounding of
    the inputs' projections alone moves M by that much."""
    rng = np.random.default_rng(22)
    for xv in (_NEAR_TRI, _rand_simplex(3, scale=0.5, rng=rng)):
        S = float(np.abs(xv).max()) + 1.0
        for r in _near_targets(xv, rng):
            _, M = oracle.near_one(r, xv)
            ref = float(-_solid_angle_mp(r, xv) / (4 * math.pi))
            tol = 1e-14 + 4 * 2.2e-16 * S / _dist_to_boundary(r, xv)
            assert abs(M - ref) <= tol, (r, M, ref)
    # exactly on the plane (a triangle in z = 0, targets with z = 0): M = 0
    eq = np.array([[0.1, 0.0, 0.0], [0.9, 0.2, 0.0], [0.3, 0.8, 0.0]])
    for r in (np.array([0.4, 0.3, 0.0]), np.array([2.0, -1.0, 0.0])):
        assert oracle.near_one(r, eq)[1] == 0.0


def test_near_single_layer_closed_forms():
    """(i) the contour formula of Sec. 4.1, Eq. (63) (its L part) at 50 digits,
    at near targets on both sides; (ii) the centroid of an equilateral
    triangle of side a, on its plane: sqrt(3) a ln(2 + sqrt(3)) / (4 pi);
    (iii) continuity through the plane with the jump -1/2 of the normal
    derivative: L(h) = L(0) - h/2 + O(h^2 log h) over an interior point, and
    M -> +-1/2 there."""
    rng = np.random.default_rng(23)
    for xv in (_NEAR_TRI, _rand_simplex(3, scale=0.5, rng=rng)):
        for r in _near_targets(xv, rng):
            L, _ = oracle.near_one(r, xv)
            ref = float(_contour_L_mp(r, xv))
            assert abs(L - ref) <= 5e-14 * abs(ref), (r, L, ref)
    a = 0.7
    eq = np.array([[0, 0, 0], [a, 0, 0], [a / 2, a * math.sqrt(3) / 2, 0]])
    L, M = oracle.near_one(eq.mean(axis=0), eq)
    assert abs(L - math.sqrt(3) * a * math.log(2 + math.sqrt(3)) / (4 * math.pi)) <= 1e-15 and M == 0.0
    x0 = 0.25 * _NEAR_TRI[0] + 0.35 * _NEAR_TRI[1] + 0.4 * _NEAR_TRI[2]
    nrm = np.cross(_NEAR_TRI[1] - _NEAR_TRI[0], _NEAR_TRI[2] - _NEAR_TRI[0])
    nrm /= np.linalg.norm(nrm)
    L0, _ = oracle.near_one(x0, _NEAR_TRI)
    for h in (1e-4, 1e-6):
        for sgn in (1, -1):
            Lh, Mh = oracle.near_one(x0 + sgn * h * nrm, _NEAR_TRI)
            assert abs(Lh - (L0 - h / 2)) <= 20 * h * h * abs(math.log(h)) + 1e-15
            assert abs(Mh - sgn * 0.5) <= 10 * h  # the solid angle tends to 2 pi from either side


def test_near_on_element_is_the_principal_value():
    """Collocation at a point of the element itself (its centroid, whose
    computed height is rounding noise): M = 0 and L = its value on the plane;
    a height of 1e-9 (above the 1e-12 on-plane band) gives the one-sided limits
    M = +-1/2."""
    a = 0.7
    eq = np.array([[0, 0, 0], [a, 0, 0], [a / 2, a * math.sqrt(3) / 2, 0]])
    Rz = np.array([[0.6, -0.8, 0.0], [0.48, 0.36, -0.8], [0.64, 0.48, 0.6]])  # a rotation
    xv = eq @ Rz.T + np.array([0.3, -0.2, 0.1])
    c = xv.mean(axis=0)
    L, M = oracle.near_one(c, xv)
    assert M == 0.0
    assert abs(L - math.sqrt(3) * a * math.log(2 + math.sqrt(3)) / (4 * math.pi)) <= 1e-14
    nrm = np.cross(xv[1] - xv[0], xv[2] - xv[0])
    nrm /= np.linalg.norm(nrm)
    for sgn in (1, -1):
        _, M1 = oracle.near_one(c + sgn * 1e-9 * nrm, xv)
        assert abs(M1 - sgn * 0.5) <= 1e-8


def test_near_pairs_csr_and_bad_ids():
    """The CSR entry point reproduces near_one per pair; bad triangle ids are
    reported and their entries left 0."""
    rng = np.random.default_rng(24)
    verts = rng.normal(size=(12, 3))
    tris = np.array([[0, 1, 2], [3, 4, 5], [6, 7, 8], [9, 10, 11]], np.int32)
    targets = rng.normal(size=(3, 3))
    ps = np.array([0, 2, 2, 5], np.int64)
    pt = np.array([1, 3, 0, 2, 3], np.int32)
    L, M = oracle.near(verts, tris, targets, ps, pt)
    for t in range(3):
        for p in range(ps[t], ps[t + 1]):
            l1, m1 = oracle.near_one(targets[t], verts[tris[pt[p]]])
            assert L[p] == l1 and M[p] == m1
    with pytest.raises(AssertionError):
        oracle.near(verts, tris, targets, ps, np.array([1, 3, 0, 9, 3], np.int32))
