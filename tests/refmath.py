"""Independent reference mathematics for pinning the oracle (tests only).

Nothing here imports the oracle or the GPU library.  These are textbook or
library routes to the same quantities:
  * R_n^m, S_n^m from scipy's associated Legendre function (Sec. 3.2, Eq. (10));
  * exact rational R_n^m polynomials from the Rodrigues formula (Eq. (11)) with
    sympy, integrated exactly over simplices by the Dirichlet monomial rule;
  * closed-form potentials of a segment, triangle and tetrahedron
    (Sec. 4.1, Eqs. (59)-(66)) and direct high-order quadrature of G.
"""
from __future__ import annotations

import math
from fractions import Fraction
from functools import lru_cache

import numpy as np
from scipy.special import lpmv


# ----------------------------------------------------------------- harmonics
def solid_R_scipy(p, x, y, z):
    """R_n^m via scipy.special.lpmv (Condon-Shortley phase included), Eq. (10)."""
    r = math.sqrt(x * x + y * y + z * z)
    out = np.zeros((p + 1) ** 2, dtype=complex)
    if r == 0.0:
        out[0] = 1.0
        return out
    ct = z / r
    phi = math.atan2(y, x)
    for n in range(p + 1):
        for m in range(-n, n + 1):
            am = abs(m)
            val = ((-1) ** n) * (1j ** am) / math.factorial(n + am) * r ** n * lpmv(am, n, ct) * np.exp(1j * m * phi)
            out[n * n + n + m] = val
    return out


def solid_S_scipy(p, x, y, z):
    """S_n^m via scipy.special.lpmv, Eq. (10)."""
    r = math.sqrt(x * x + y * y + z * z)
    ct = z / r
    phi = math.atan2(y, x)
    out = np.zeros((p + 1) ** 2, dtype=complex)
    for n in range(p + 1):
        for m in range(-n, n + 1):
            am = abs(m)
            out[n * n + n + m] = (1j ** (-am)) * math.factorial(n - am) * r ** (-n - 1) * lpmv(am, n, ct) * np.exp(1j * m * phi)
    return out


def expansion_value(F, p, r_minus_c):
    """sum_{n<=p} sum_m F_n^m S_n^m(r - c)."""
    S = solid_S_scipy(p, *r_minus_c)
    nc = (p + 1) ** 2
    return complex(np.sum(F[:nc] * S))


# ------------------------------------------------- exact polynomials (sympy)
@lru_cache(maxsize=None)
def R_poly(n, m):
    """Exact R_n^m(x,y,z) as a sympy expression from the Rodrigues formula."""
    import sympy as sp
    x, y, z, mu = sp.symbols("x y z mu", real=True)
    am = abs(m)
    # P_n^{|m|}(mu) = (-1)^m (1-mu^2)^{m/2} / (2^n n!) d^{n+m}/dmu^{n+m} (mu^2-1)^n
    Q = sp.diff((mu ** 2 - 1) ** n, mu, n + am) / (2 ** n * sp.factorial(n))
    Q = sp.Poly(sp.expand(Q), mu)
    r2 = x ** 2 + y ** 2 + z ** 2
    # r^{n-|m|} Q(z/r): Q has the parity of n-|m|, so this is polynomial
    body = 0
    for (k,), c in Q.terms():
        e = n - am - k  # even
        body += c * z ** k * r2 ** (e // 2)
    w = x + sp.I * y if m >= 0 else x - sp.I * y
    W = (-1) ** am * w ** am * body  # r^n P_n^{|m|} e^{i m phi}
    R = (-1) ** n * sp.I ** am / sp.factorial(n + am) * W
    return sp.expand(R), (x, y, z)


def _dirichlet(exps):
    """int over the unit simplex of prod u_i^{a_i} = prod a_i! / (sum a + d)!."""
    d = len(exps)
    num = 1
    for a in exps:
        num *= math.factorial(a)
    return Fraction(num, math.factorial(sum(exps) + d))


def exact_simplex_integral(expr, syms, x1, edges):
    """Exact int over the unit simplex of expr(x1 + sum_i t_i edges_i) dt,
    with rational vertex data; returns a complex of Fractions (re, im)."""
    import sympy as sp
    d = len(edges)
    ts = sp.symbols(f"t0:{d}", real=True)
    sub = {}
    for k, s in enumerate(syms):
        sub[s] = sp.Rational(x1[k]) + sum(sp.Rational(edges[i][k]) * ts[i] for i in range(d))
    e = sp.expand(expr.subs(sub, simultaneous=True))
    if e == 0:
        return Fraction(0), Fraction(0)
    P = sp.Poly(e, *ts)
    re = Fraction(0)
    im = Fraction(0)
    for exps, c in P.terms():
        w = _dirichlet(exps)
        cr, ci = sp.re(c), sp.im(c)
        re += Fraction(int(sp.numer(cr)), int(sp.denom(cr))) * w
        im += Fraction(int(sp.numer(ci)), int(sp.denom(ci))) * w
    return re, im


# ------------------------------------------------ potentials (E1 reference)
def segment_potential(r, x1, x2):
    """(1/4pi) int_segment dl/|r - r'| = (1/4pi) ln((R1+R2+L)/(R1+R2-L))."""
    R1 = np.linalg.norm(r - x1)
    R2 = np.linalg.norm(r - x2)
    L = np.linalg.norm(x2 - x1)
    return math.log((R1 + R2 + L) / (R1 + R2 - L)) / (4 * math.pi)


def triangle_potential_L(r, xs):
    """Single-layer potential of a flat triangle, unit density: the contour
    formula of Sec. 4.1, Eq. (63) (its L part, which needs no sign choice)."""
    xs = [np.asarray(x, dtype=float) for x in xs]
    nrm = np.cross(xs[1] - xs[0], xs[2] - xs[0])
    nrm /= np.linalg.norm(nrm)
    h = abs(np.dot(r - xs[0], nrm))

    def MP(x, y, z):
        rr = math.sqrt(x * x + y * y + z * z)
        den = rr * z * z + y * x * x
        if den == 0.0:
            return 0.0
        return -math.atan(x * z * (rr - y) / den)

    def LP(x, y, z):
        rr = math.sqrt(x * x + y * y + z * z)
        return -y * MP(x, y, z) - z * math.log(abs(rr + x))

    tot = 0.0
    for q in range(3):
        xq = xs[q]
        xn = xs[(q + 1) % 3]
        lq = np.linalg.norm(xn - xq)
        iq = (xn - xq) / lq
        nq = np.cross(iq, nrm)
        xx = np.dot(r - xq, iq)
        zq = np.dot(r - xq, nq)
        tot += LP(lq - xx, h, zq) - LP(-xx, h, zq)
    return tot / (4 * math.pi)


def _gauss01(k):
    x, w = np.polynomial.legendre.leggauss(k)
    return 0.5 * (x + 1), 0.5 * w


def direct_potential(kind, r, xs, k=40):
    """Direct quadrature (numpy Gauss-Legendre on collapsed coordinates) of
    int G(r, r') dmu(r') (kind 'single', 'segment', 'tet') or
    int dG/dn(r') dS(r') (kind 'double') with unit density; r far away."""
    xs = [np.asarray(x, dtype=float) for x in xs]
    g, w = _gauss01(k)
    if kind == "segment":
        L = np.linalg.norm(xs[1] - xs[0])
        pts = xs[0][None] + g[:, None] * (xs[1] - xs[0])[None]
        d = np.linalg.norm(r[None] - pts, axis=1)
        return float(np.sum(w / d) * L / (4 * math.pi))
    if kind in ("single", "double"):
        Ru, Rv = xs[1] - xs[0], xs[2] - xs[0]
        cr = np.cross(Ru, Rv)
        J = np.linalg.norm(cr)
        n = cr / J
        S, T = np.meshgrid(g, g, indexing="ij")
        W = np.outer(w, w) * (1 - S)
        u, v = S, (1 - S) * T
        pts = xs[0] + u[..., None] * Ru + v[..., None] * Rv
        diff = r - pts
        d = np.linalg.norm(diff, axis=-1)
        if kind == "single":
            return float(np.sum(W / d) * J / (4 * math.pi))
        # dG/dn' = n . (r - r') / (4 pi |r - r'|^3)
        return float(np.sum(W * (diff @ n) / d ** 3) * J / (4 * math.pi))
    if kind == "tet":
        Ru, Rv, Rw = xs[1] - xs[0], xs[2] - xs[0], xs[3] - xs[0]
        J = abs(np.dot(np.cross(Ru, Rv), Rw))
        S, T, U = np.meshgrid(g, g, g, indexing="ij")
        W = w[:, None, None] * w[None, :, None] * w[None, None, :] * (1 - S) ** 2 * (1 - T)
        u, v, ww = S, (1 - S) * T, (1 - S) * (1 - T) * U
        pts = xs[0] + u[..., None] * Ru + v[..., None] * Rv + ww[..., None] * Rw
        d = np.linalg.norm(r - pts, axis=-1)
        return float(np.sum(W / d) * J / (4 * math.pi))
    raise ValueError(kind)


def tet_potential_faces(r, xs):
    """Volume potential of a tetrahedron, unit density, from its faces by the
    divergence theorem, Sec. 4.1, Eq. (66): N = -1/2 sum_f n_f.(r - r_cf) L_f."""
    xs = [np.asarray(x, dtype=float) for x in xs]
    cen = sum(xs) / 4
    tot = 0.0
    for f in ((1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)):
        a, b, c = (xs[i] for i in f)
        n = np.cross(b - a, c - a)
        n /= np.linalg.norm(n)
        rc = (a + b + c) / 3
        if np.dot(rc - cen, n) < 0:
            n = -n
        tot += -0.5 * np.dot(n, r - rc) * triangle_potential_L(r, [a, b, c])
    return tot


def truncation_bound(kind, p, sigma_mu, a, d):
    """Rigorous bound on the far-field error of the order-p expansion of a
    source of total |sigma|*measure = sigma_mu inside the ball |r'-c| <= a,
    evaluated at |r-c| = d > a.  Single layer / segment / volume: the
    Legendre tail of 1/|r-r'| with |P_n| <= 1.  Double layer: the tail of the
    source-point gradient, |grad (r'^n P_n)| <= (n+1) a^(n-1)."""
    q = a / d
    if kind == "double":
        s = sum((n + 1) * q ** (n - 1) for n in range(p + 1, p + 400))
        return sigma_mu * s / (4 * math.pi * d * d)
    return sigma_mu * q ** (p + 1) / (d - a) / (4 * math.pi)
