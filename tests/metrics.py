"""Error metrics for comparing per-box coefficients with the oracle.

Scale-aware error per (box b, degree n):
    err[b, n] = ||F_gpu[b, n, :] - F_ref[b, n, :]||_2 / A[b, n],
    A[b, n]   = sum_{e in b} |sigma_e| * ||F^{(e)}_{n, :}||_2
where F^{(e)} are the unit-density coefficients of element e (oracle).  It is
the rounding error relative to the size of the terms that were summed, and so
stays meaningful when a box sum cancels or a high order is tiny.
"""
import numpy as np


def degree_slices(p):
    return [slice(n * n, (n + 1) * (n + 1)) for n in range(p + 1)]


def per_degree_norms(F, p):
    """||F[..., n, :]||_2 over m for every degree: [..., p+1]."""
    return np.stack([np.linalg.norm(F[..., sl], axis=-1) for sl in degree_slices(p)], axis=-1)


def scale_denominator(elem_norms, density, elem_box, n_boxes, boxes=None):
    """A[b, n] for all boxes (or the listed ones)."""
    p1 = elem_norms.shape[1]
    A = np.zeros((n_boxes, p1))
    w = np.abs(density)[:, None] * elem_norms
    valid = (elem_box >= 0) & (elem_box < n_boxes)
    np.add.at(A, elem_box[valid], w[valid])
    return A if boxes is None else A[np.asarray(boxes)]


def scale_aware_error(F_gpu, F_ref, A, p):
    d = per_degree_norms(F_gpu - F_ref, p)
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.where(A > 0, d / A, np.where(d > 0, np.inf, 0.0))
    return e


def normwise_error(F_gpu, F_ref, p):
    d = per_degree_norms(F_gpu - F_ref, p)
    r = per_degree_norms(F_ref, p)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(r > 0, d / r, np.where(d > 0, np.inf, 0.0))


def summary(F_gpu, F_ref, A, p):
    sa = scale_aware_error(F_gpu, F_ref, A, p)
    nw = normwise_error(F_gpu, F_ref, p)
    diff = np.abs(F_gpu - F_ref)
    ref = np.abs(F_ref)
    mask = ref > 1e-300
    rel = diff[mask] / ref[mask]
    return {
        "scale_aware_max": float(np.max(sa)) if sa.size else 0.0,
        "normwise_max": float(np.max(nw[np.isfinite(nw)])) if nw.size else 0.0,
        "coef_rel_median": float(np.median(rel)) if rel.size else 0.0,
        "coef_rel_p99": float(np.percentile(rel, 99)) if rel.size else 0.0,
    }
