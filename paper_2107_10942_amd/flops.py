"""Algorithmic work model of the Q2X tile kernel (per element, order p).

FLOPs are counted operation by operation as the recursion of Sec. 3.4,
Eqs. (50)-(56), is evaluated in the m >= 0 form with zero padding pruned
(entries with m > n are never touched), one FMA = 2 FLOPs:

  ladder step to degree n (one array): order 0: 1 multiply + 2 FMAs;
  orders m >= 1: the -xi F^{m-1} + eta F^{m+1} pair costs 10 FLOPs when
  F^{m+1} exists, 6 when it does not (2 at m = 1, where F^0 is real), the
  -z F^m term 4 FLOPs when F^m exists, and the source term (j, i, b, a, p
  recursions) 2 FLOPs (1 at m = 0).
  Per degree:  triangle single = q + j(+q) + i(+j);  segment = q + p(+q);
  tetrahedron = q + j + b + a;  double layer = one D_nu step on i_{n-1}
  (no source) plus the q, j, i steps to degree n-1; single + double of one
  mesh (one recursion) = the D_nu step plus the q, j, i steps to degree n.
  The recursion runs on G_n = (n+k)! t_n, so it has no per-step constants;
  the FP64 factor s_e a_e^n/(n+k)! costs 2 multiplies per degree, and the
  reduction one FP64 FMA per real component of every element-coefficient
  (4 FLOPs per complex coefficient).  Geometry (~60 FLOPs) is counted once.

Bytes (algorithmic, per launch): inputs read once (per element: k vertex
indices, density, box id, and k vertices of 24 B counted per element) plus the
box coefficients written, B_occ (p+1)^2 16 B.
"""
from __future__ import annotations

TRI_SINGLE, TRI_DOUBLE, SEGMENT, TET, TRI_BOTH, SEGMENT_VEC = 0, 1, 2, 3, 4, 5
NV = {TRI_SINGLE: 3, TRI_DOUBLE: 3, SEGMENT: 2, TET: 4, TRI_BOTH: 3, SEGMENT_VEC: 2}
NOUT = {TRI_SINGLE: 1, TRI_DOUBLE: 1, SEGMENT: 1, TET: 1, TRI_BOTH: 2, SEGMENT_VEC: 3}
GEOMETRY_FLOPS = 60


def ladder_flops(n: int, add: bool, prescale: bool = False) -> int:
    """FLOPs of one ladder step to degree n of one array (see the module doc)."""
    f = 1  # order 0: -z F^0
    if n - 1 >= 1:
        f += 4  # 2 xi_r F^1_r + 2 xi_i F^1_i (doubled xi precomputed per element)
    if add:
        f += 1
    for m in range(1, n + 1):
        if m + 1 <= n - 1:
            f += 10
        elif m == 1:
            f += 2
        else:
            f += 6
        if m <= n - 1:
            f += 4
        if add:
            f += 2
    return f


def recursion_flops(kind: int, p: int) -> int:
    f = 0
    if kind == TRI_SINGLE:
        for n in range(1, p + 1):
            f += ladder_flops(n, False) + 2 * ladder_flops(n, True)
    elif kind in (SEGMENT, SEGMENT_VEC):
        for n in range(1, p + 1):
            f += ladder_flops(n, False) + ladder_flops(n, True)
    elif kind == TET:
        for n in range(1, p + 1):
            f += ladder_flops(n, False) + 3 * ladder_flops(n, True)
    elif kind == TRI_DOUBLE:
        for n in range(1, p + 1):
            f += ladder_flops(n, False)  # l_n = D_nu i_{n-1}
            if n < p:
                f += ladder_flops(n, False) + 2 * ladder_flops(n, True)
    elif kind == TRI_BOTH:
        for n in range(1, p + 1):
            f += ladder_flops(n, False)  # l_n = D_nu i_{n-1}
            f += ladder_flops(n, False) + 2 * ladder_flops(n, True)
    else:
        raise ValueError(kind)
    return f


def element_flops(kind: int, p: int) -> int:
    """Total FLOPs per element: geometry + recursion + factors + reduction."""
    nct = (p + 1) * (p + 2) // 2
    return GEOMETRY_FLOPS + recursion_flops(kind, p) + NOUT[kind] * (2 * (p + 1) + 4 * nct)


def launch_flops(kind: int, p: int, n_elems: int) -> int:
    return element_flops(kind, p) * n_elems


def launch_bytes(kind: int, p: int, n_elems: int, n_boxes_occupied: int) -> int:
    per_elem = 4 * NV[kind] + 8 * NOUT[kind] + 4 + 4 + 24 * NV[kind]  # indices, densities, box id, perm, vertices
    return per_elem * n_elems + NOUT[kind] * 16 * (p + 1) ** 2 * n_boxes_occupied


def eval_element_flops(kind: int, p: int) -> int:
    """Receiving side (q2x_eval), per element: geometry + the same recursion +
    per degree the FP64 weight (2) and per order m >= 0 the weighted value (2),
    L^m t (6), L^{-m} conj(t) for m > 0 (8) and the (-i)^m accumulation (2),
    + the final J factor (2).  The double layer has no degree 0."""
    f = GEOMETRY_FLOPS + recursion_flops(kind, p) + 2
    for n in range(1 if kind == TRI_DOUBLE else 0, p + 1):
        f += 2 + 10 + 18 * n
    return f


def eval_launch_bytes(kind: int, p: int, n_elems: int, n_boxes_occupied: int) -> int:
    """Algorithmic bytes of one q2x_eval launch: per element its vertex indices,
    vertices, box id, permutation entry and complex result; each occupied box's
    local coefficients read once."""
    per_elem = 4 * NV[kind] + 24 * NV[kind] + 4 + 4 + 16
    return per_elem * n_elems + 16 * (p + 1) ** 2 * n_boxes_occupied


def m2m_child_flops(p: int) -> int:
    """One child-to-parent translation (q2x_m2m): every output (n, m >= 0) sums
    A_k^l R_{n-k}^{l-m} over k <= n and |l| <= k, |l - m| <= n - k, one complex
    multiply-add (4 FMAs = 8 FLOPs) each; plus the ladder for R of the shift
    (~10 FLOPs per (j, q)).  Expansions are read once per child."""
    macs = 0
    for n in range(p + 1):
        for m in range(n + 1):
            for k in range(n + 1):
                j = n - k
                lo, hi = max(-k, m - j), min(k, m + j)
                macs += max(0, hi - lo + 1)
    return 8 * macs + 10 * (p + 1) * (p + 2) // 2


# A second, coarser count: the recursion of Eqs. (50)-(56) evaluated as
# written, every complex product with xi or eta a full complex multiply-add
# (8 FLOPs), zero padding pruned, FMA = 2.  Per element and order p it is a
# quadratic in p (exact at p = 8, 12, 16, 20, 24):
#   triangle single 32p^2 - 5p + 12, triangle double 41p^2 - 10p + 20,
#   segment 21p^2 - 4p + 8, tetrahedron 43p^2 - 6p + 16
# (2,020 / 4,560 / 8,124 / 12,712 / 18,324 for the single layer), plus
# 4 (p+1)(p+2)/2 FLOPs per output for the FP64 weight and box sum.  The
# single + double pass of one mesh shares the single layer's recursion to
# degree p-1: single(p) + double(p) - single(p-1).  This is the count the
# roofline's `achieved` uses; the leaner operation-by-operation model above
# (which uses the conjugate pair xi, eta) is reported beside it.
_SCOPE_QUAD = {TRI_SINGLE: (32, -5, 12), TRI_DOUBLE: (41, -10, 20), SEGMENT: (21, -4, 8), TET: (43, -6, 16)}


def scope_recursion_flops(kind: int, p: int) -> int:
    if kind == TRI_BOTH:
        return scope_recursion_flops(TRI_SINGLE, p) + scope_recursion_flops(TRI_DOUBLE, p) - \
            scope_recursion_flops(TRI_SINGLE, p - 1)
    if kind == SEGMENT_VEC:
        return scope_recursion_flops(SEGMENT, p)
    a, b, c = _SCOPE_QUAD[kind]
    return a * p * p + b * p + c if p > 0 else 0


def scope_element_flops(kind: int, p: int) -> int:
    nct = (p + 1) * (p + 2) // 2
    return scope_recursion_flops(kind, p) + NOUT[kind] * 4 * nct


def scope_launch_flops(kind: int, p: int, n_elems: int) -> int:
    return scope_element_flops(kind, p) * n_elems


# MI355X vector-ALU peaks.  256 CUs x 4 SIMDs x 16 lanes = 4096 FMA lanes per
# clock at 2.4 GHz: FP64 FMA 4096 x 2 x 2.4e9 = 78.6 TFLOP/s.  FP32 FMA
# issues at twice that rate even as plain (non-packed) v_fma_f32: a loop of
# independent non-packed FP32 FMAs (q2x_peak_measure) reaches about 140
# TFLOP/s, so FP32 work is priced against the published 157.3 TFLOP/s.
CUS, LANES_PER_CU, CLOCK_HZ = 256, 64, 2.4e9
PEAK_FP64_TFLOPS = CUS * LANES_PER_CU * 2 * CLOCK_HZ / 1e12  # 78.64
PEAK_FP32_TFLOPS = 2 * PEAK_FP64_TFLOPS                      # 157.3


def peak_valu_tflops(fp32: bool) -> float:
    """Vector-ALU peak of the recursion's arithmetic type."""
    return PEAK_FP32_TFLOPS if fp32 else PEAK_FP64_TFLOPS


PEAK_HBM_GBS = 8000.0


if __name__ == "__main__":
    for k, name in ((0, "tri_single"), (1, "tri_double"), (2, "segment"), (3, "tet"), (4, "tri_both"),
                    (5, "segment_vec")):
        print(name, [recursion_flops(k, p) for p in (8, 12, 16, 20, 24)], [element_flops(k, p) for p in (8, 12, 16, 20, 24)])
