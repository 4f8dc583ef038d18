/*
 * q2x_oracle.c -- plain, slow, CPU FP64 oracle for the Quadrature-to-Expansion
 * (Q2X) multipole coefficients of flat simplices (Gumerov, Kaneko, Duraiswami,
 * "Recursive computation of the multipole expansions of layer potential
 * integrals over simplices ...", arXiv 2107.10942).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU product path
 * never calls, links or includes anything from this directory, and this file
 * shares no code, header or table with it.
 *
 * What it computes (the plain definition, Sec. 2 Eqs. (1),(3),(4),(5) and
 * Sec. 3.2 Eq. (14)): for every box b, 0 <= n <= p, -n <= m <= n,
 *
 *   F_{b,n}^m = sum_{e in b} sigma_e (1/4pi) (-1)^n  int_e R_n^{-m}(y - c_b) dmu(y)
 *
 * (single layer, segment, tetrahedron), and for the double layer the integrand
 * is n_e . grad R_n^{-m}(y - c_b).  With norm = MOMENT the output is instead the
 * raw moment  sum_e sigma_e int_e R_n^{m}(y - c_b) dmu  (resp. n.grad R_n^m).
 *
 * How (deliberately NOT the paper's recursions of Sec. 3.3-3.4):
 *  - R_n^m is evaluated from its definition Eq. (10) with the associated
 *    Legendre functions of Eq. (11) (Condon-Shortley phase included), through
 *    the textbook three-term recurrence in the degree, written for the solid
 *    (r^n-scaled) functions so that it is a polynomial recurrence in x,y,z.
 *  - The gradient needed by the double layer is obtained by forward-mode
 *    differentiation of that same recurrence (product rule), i.e. not from the
 *    ladder relations Eqs. (15)-(18).
 *  - The element integral is Gauss-Legendre quadrature on collapsed (Duffy)
 *    coordinates of the unit simplex of Sec. 3.1 Eqs. (6)-(9).  R_n^m is a
 *    polynomial of degree n (Sec. 4.2.1), so with k nodes per direction and
 *    2k-1 >= n + (simplex dimension - 1) the rule is exact.
 *  - Box sums run over the elements of a box in increasing element index.
 *
 * Output layout: out[b][(p+1)^2][2] (re, im), coefficient (n,m) at n*n+n+m.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_TRI_SINGLE 0
#define ORC_TRI_DOUBLE 1
#define ORC_SEGMENT 2
#define ORC_TET 3

#define ORC_NORM_FMM 0
#define ORC_NORM_MOMENT 1

#define ORC_PMAX 64
#define ORC_KMAX 64

static const double ORC_PI = 3.14159265358979323846264338327950288;

/* ------------------------------------------------------------------------- */
/* Associated Legendre recurrence for the solid functions                    */
/*   W_n^m(x,y,z) = r^n P_n^m(cos theta) e^{i m phi},  m >= 0,               */
/* with P_n^m carrying the Condon-Shortley factor (-1)^m (Eq. (11)):         */
/*   W_0^0 = 1                                                               */
/*   W_m^m = -(2m-1) (x+iy) W_{m-1}^{m-1}                                    */
/*   W_{m+1}^m = (2m+1) z W_m^m                                              */
/*   (n-m) W_n^m = (2n-1) z W_{n-1}^m - (n+m-1) r^2 W_{n-2}^m                */
/* (the standard recurrences of P_n^m in n, multiplied through by r^n, using */
/*  r cos(theta) = z and r sin(theta) e^{i phi} = x + i y).                  */
/* Optional forward-mode derivatives d/dx, d/dy, d/dz are carried alongside. */
/* Arrays are indexed [n*(n+1)/2 + m], m = 0..n.                             */
/* ------------------------------------------------------------------------- */
static inline int tri_idx(int n, int m) { return n * (n + 1) / 2 + m; }

static void legendre_solid(int p, double x, double y, double z, double *wr, double *wi,
                           double *gxr, double *gxi, double *gyr, double *gyi,
                           double *gzr, double *gzi) {
  const int grad = (gxr != NULL);
  const double r2 = x * x + y * y + z * z;
  wr[0] = 1.0;
  wi[0] = 0.0;
  if (grad) {
    gxr[0] = gxi[0] = gyr[0] = gyi[0] = gzr[0] = gzi[0] = 0.0;
  }
  for (int m = 0; m <= p; ++m) {
    const int mm = tri_idx(m, m);
    if (m > 0) {
      /* W_m^m = -(2m-1) (x+iy) W_{m-1}^{m-1} */
      const int pm = tri_idx(m - 1, m - 1);
      const double a = -(2.0 * m - 1.0);
      const double ur = wr[pm], ui = wi[pm];
      wr[mm] = a * (x * ur - y * ui);
      wi[mm] = a * (x * ui + y * ur);
      if (grad) {
        /* d/dx[(x+iy) U] = U + (x+iy) dU/dx ; d/dy = i U + (x+iy) dU/dy ; d/dz = (x+iy) dU/dz */
        gxr[mm] = a * (ur + x * gxr[pm] - y * gxi[pm]);
        gxi[mm] = a * (ui + x * gxi[pm] + y * gxr[pm]);
        gyr[mm] = a * (-ui + x * gyr[pm] - y * gyi[pm]);
        gyi[mm] = a * (ur + x * gyi[pm] + y * gyr[pm]);
        gzr[mm] = a * (x * gzr[pm] - y * gzi[pm]);
        gzi[mm] = a * (x * gzi[pm] + y * gzr[pm]);
      }
    }
    if (m + 1 <= p) {
      /* W_{m+1}^m = (2m+1) z W_m^m */
      const int i1 = tri_idx(m + 1, m);
      const double a = 2.0 * m + 1.0;
      wr[i1] = a * z * wr[mm];
      wi[i1] = a * z * wi[mm];
      if (grad) {
        gxr[i1] = a * z * gxr[mm];
        gxi[i1] = a * z * gxi[mm];
        gyr[i1] = a * z * gyr[mm];
        gyi[i1] = a * z * gyi[mm];
        gzr[i1] = a * (wr[mm] + z * gzr[mm]);
        gzi[i1] = a * (wi[mm] + z * gzi[mm]);
      }
    }
    for (int n = m + 2; n <= p; ++n) {
      const int i0 = tri_idx(n, m), i1 = tri_idx(n - 1, m), i2 = tri_idx(n - 2, m);
      const double a = (2.0 * n - 1.0) / (double)(n - m);
      const double b = (double)(n + m - 1) / (double)(n - m);
      wr[i0] = a * z * wr[i1] - b * r2 * wr[i2];
      wi[i0] = a * z * wi[i1] - b * r2 * wi[i2];
      if (grad) {
        gxr[i0] = a * z * gxr[i1] - b * (2.0 * x * wr[i2] + r2 * gxr[i2]);
        gxi[i0] = a * z * gxi[i1] - b * (2.0 * x * wi[i2] + r2 * gxi[i2]);
        gyr[i0] = a * z * gyr[i1] - b * (2.0 * y * wr[i2] + r2 * gyr[i2]);
        gyi[i0] = a * z * gyi[i1] - b * (2.0 * y * wi[i2] + r2 * gyi[i2]);
        gzr[i0] = a * (wr[i1] + z * gzr[i1]) - b * (2.0 * z * wr[i2] + r2 * gzr[i2]);
        gzi[i0] = a * (wi[i1] + z * gzi[i1]) - b * (2.0 * z * wi[i2] + r2 * gzi[i2]);
      }
    }
  }
}

static double factorial(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; ++i) f *= (double)i;
  return f;
}

/* i^k for integer k >= 0, as (re, im). */
static void ipow(int k, double *re, double *im) {
  switch (k & 3) {
    case 0: *re = 1; *im = 0; break;
    case 1: *re = 0; *im = 1; break;
    case 2: *re = -1; *im = 0; break;
    default: *re = 0; *im = -1; break;
  }
}

/*
 * Regular solid harmonics R_n^m(x,y,z) of Eq. (10), n <= p, m = -n..n,
 * out[2*(n*n+n+m) + {0,1}].  R_n^m = (-1)^n i^{|m|} W_n^{|m|} / (n+|m|)! for
 * m >= 0 and with conj(W) for m < 0 (e^{i m phi} = conj(e^{i|m|phi})).
 * If grad != NULL, grad[3][...] receives d/dx, d/dy, d/dz in the same layout.
 */
int orc_solid_harmonics(int p, double x, double y, double z, double *out, double *grad) {
  if (p < 0 || p > ORC_PMAX) return -1;
  const int nt = (p + 1) * (p + 2) / 2;
  double *buf = (double *)malloc(sizeof(double) * 8 * (size_t)nt);
  if (!buf) return -2;
  double *wr = buf, *wi = buf + nt;
  double *g[6] = {NULL, NULL, NULL, NULL, NULL, NULL};
  if (grad) {
    for (int k = 0; k < 6; ++k) g[k] = (double *)malloc(sizeof(double) * (size_t)nt);
  }
  legendre_solid(p, x, y, z, wr, wi, g[0], g[1], g[2], g[3], g[4], g[5]);
  const int ncoef = (p + 1) * (p + 1);
  for (int n = 0; n <= p; ++n) {
    const double sgn = (n & 1) ? -1.0 : 1.0;
    for (int m = -n; m <= n; ++m) {
      const int am = m < 0 ? -m : m;
      const int t = tri_idx(n, am);
      double ir, ii;
      ipow(am, &ir, &ii);
      const double s = sgn / factorial(n + am);
      const double cj = (m < 0) ? -1.0 : 1.0; /* conjugate for m < 0 */
      const int o = n * n + n + m;
      /* value */
      {
        const double ur = wr[t], ui = cj * wi[t];
        out[2 * o] = s * (ir * ur - ii * ui);
        out[2 * o + 1] = s * (ir * ui + ii * ur);
      }
      if (grad) {
        for (int d = 0; d < 3; ++d) {
          const double ur = g[2 * d][t], ui = cj * g[2 * d + 1][t];
          grad[2 * (d * ncoef + o)] = s * (ir * ur - ii * ui);
          grad[2 * (d * ncoef + o) + 1] = s * (ir * ui + ii * ur);
        }
      }
    }
  }
  free(buf);
  if (grad)
    for (int k = 0; k < 6; ++k) free(g[k]);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Gauss-Legendre rule on [0,1]: Newton iteration on P_k (three-term         */
/* recurrence), weights 2/((1-x^2) P_k'(x)^2) on [-1,1], then mapped.        */
/* ------------------------------------------------------------------------- */
int orc_gauss_legendre01(int k, double *nodes, double *weights) {
  if (k < 1 || k > 4 * ORC_KMAX) return -1;
  for (int i = 0; i < k; ++i) {
    double x = cos(ORC_PI * (i + 0.75) / (k + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int j = 2; j <= k; ++j) {
        const double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      const double pk = (k == 1) ? x : p1;
      const double pkm1 = (k == 1) ? 1.0 : p0;
      dp = k * (x * pk - pkm1) / (x * x - 1.0);
      const double dx = pk / dp;
      x -= dx;
      if (fabs(dx) < 1e-17) break;
    }
    /* recompute derivative at the converged node */
    {
      double p0 = 1.0, p1 = x;
      for (int j = 2; j <= k; ++j) {
        const double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      const double pk = (k == 1) ? x : p1;
      const double pkm1 = (k == 1) ? 1.0 : p0;
      dp = k * (x * pk - pkm1) / (x * x - 1.0);
    }
    const double w = 2.0 / ((1.0 - x * x) * dp * dp);
    nodes[i] = 0.5 * (x + 1.0);
    weights[i] = 0.5 * w;
  }
  return 0;
}

/* Nodes per collapsed direction used when the caller passes 0: ceil((p+3)/2).
 * The collapsed tetrahedron integrand has degree <= p+2 in its first variable
 * (p in the harmonic, 2 in the Duffy Jacobian), so 2k-1 >= p+2 makes the rule
 * exact for every kind. */
int orc_default_nodes(int p) { return (p + 4) / 2; }

/* ------------------------------------------------------------------------- */
/* Element geometry (Sec. 3.1, Eqs. (8),(9)).                                */
/* ------------------------------------------------------------------------- */
static void sub3(const double *a, const double *b, double *o) {
  o[0] = a[0] - b[0];
  o[1] = a[1] - b[1];
  o[2] = a[2] - b[2];
}
static void cross3(const double *a, const double *b, double *o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/*
 * Integral over one element with unit density about the centre c:
 *   single/segment/tet:  out[n,m] = int_e R_n^m(y - c) dmu(y)
 *   double:              out[n,m] = int_e n_e . grad R_n^m(y - c) dS(y)
 * for all n <= p, m = -n..n (layout 2*(n*n+n+m)).  xv holds the element's
 * vertices (2, 3 or 4 points, absolute coordinates).  `nodes` Gauss points per
 * collapsed direction (0 = default).  Returns the Jacobian J via *jac.
 */
int orc_element_integral(int kind, int p, const double *xv, const double *c, int nodes,
                         double *out, double *jac) {
  if (p < 0 || p > ORC_PMAX) return -1;
  if (nodes <= 0) nodes = orc_default_nodes(p);
  if (nodes > ORC_KMAX) return -1;
  const int ncoef = (p + 1) * (p + 1);
  memset(out, 0, sizeof(double) * 2 * (size_t)ncoef);
  double gx[ORC_KMAX], gw[ORC_KMAX];
  orc_gauss_legendre01(nodes, gx, gw);

  double R0[3], Ru[3] = {0, 0, 0}, Rv[3] = {0, 0, 0}, Rw[3] = {0, 0, 0};
  sub3(&xv[0], c, R0); /* x1 - c */
  double J = 0.0, nrm[3] = {0, 0, 0};
  if (kind == ORC_SEGMENT) {
    sub3(&xv[3], &xv[0], Ru);
    J = sqrt(dot3(Ru, Ru));
  } else if (kind == ORC_TRI_SINGLE || kind == ORC_TRI_DOUBLE) {
    sub3(&xv[3], &xv[0], Ru);
    sub3(&xv[6], &xv[0], Rv);
    double cr[3];
    cross3(Ru, Rv, cr);
    J = sqrt(dot3(cr, cr));
    if (J > 0) {
      nrm[0] = cr[0] / J;
      nrm[1] = cr[1] / J;
      nrm[2] = cr[2] / J;
    }
  } else if (kind == ORC_TET) {
    sub3(&xv[3], &xv[0], Ru);
    sub3(&xv[6], &xv[0], Rv);
    sub3(&xv[9], &xv[0], Rw);
    double cr[3];
    cross3(Ru, Rv, cr);
    J = fabs(dot3(cr, Rw));
  } else {
    return -1;
  }
  if (jac) *jac = J;
  if (!(J > 0.0)) return 0; /* degenerate element: contributes exactly zero */

  double *val = (double *)malloc(sizeof(double) * 2 * (size_t)ncoef);
  double *grd = (kind == ORC_TRI_DOUBLE) ? (double *)malloc(sizeof(double) * 6 * (size_t)ncoef) : NULL;

  const int nd1 = nodes, nd2 = (kind == ORC_SEGMENT) ? 1 : nodes, nd3 = (kind == ORC_TET) ? nodes : 1;
  for (int a = 0; a < nd1; ++a) {
    for (int b = 0; b < nd2; ++b) {
      for (int g = 0; g < nd3; ++g) {
        double u = 0, v = 0, w = 0, wt = 0;
        if (kind == ORC_SEGMENT) {
          u = gx[a];
          wt = gw[a];
        } else if (kind == ORC_TET) {
          /* u = s, v = (1-s) t, w = (1-s)(1-t) r ; dV = (1-s)^2 (1-t) ds dt dr */
          const double s = gx[a], t = gx[b], r = gx[g];
          u = s;
          v = (1.0 - s) * t;
          w = (1.0 - s) * (1.0 - t) * r;
          wt = gw[a] * gw[b] * gw[g] * (1.0 - s) * (1.0 - s) * (1.0 - t);
        } else {
          /* u = s, v = (1-s) t ; dS = (1-s) ds dt */
          const double s = gx[a], t = gx[b];
          u = s;
          v = (1.0 - s) * t;
          wt = gw[a] * gw[b] * (1.0 - s);
        }
        const double px = R0[0] + u * Ru[0] + v * Rv[0] + w * Rw[0];
        const double py = R0[1] + u * Ru[1] + v * Rv[1] + w * Rw[1];
        const double pz = R0[2] + u * Ru[2] + v * Rv[2] + w * Rw[2];
        const double f = wt * J;
        if (kind == ORC_TRI_DOUBLE) {
          orc_solid_harmonics(p, px, py, pz, val, grd);
          for (int o = 0; o < ncoef; ++o) {
            const double dr = nrm[0] * grd[2 * o] + nrm[1] * grd[2 * (ncoef + o)] +
                              nrm[2] * grd[2 * (2 * ncoef + o)];
            const double di = nrm[0] * grd[2 * o + 1] + nrm[1] * grd[2 * (ncoef + o) + 1] +
                              nrm[2] * grd[2 * (2 * ncoef + o) + 1];
            out[2 * o] += f * dr;
            out[2 * o + 1] += f * di;
          }
        } else {
          orc_solid_harmonics(p, px, py, pz, val, NULL);
          for (int o = 0; o < ncoef; ++o) {
            out[2 * o] += f * val[2 * o];
            out[2 * o + 1] += f * val[2 * o + 1];
          }
        }
      }
    }
  }
  free(val);
  free(grd);
  return 0;
}

/*
 * Turn the unit-density integrals I[n,m] = int R_n^m (or n.grad R_n^m) of one
 * element into its weighted coefficients and add them to acc:
 *   norm FMM:    acc[n,m] += sigma (1/4pi) (-1)^n I[n,-m]   (Eq. (14))
 *   norm MOMENT: acc[n,m] += sigma I[n,m]
 */
static void add_coeffs(int p, int norm, double sigma, const double *I, double *acc) {
  for (int n = 0; n <= p; ++n) {
    for (int m = -n; m <= n; ++m) {
      const int o = n * n + n + m;
      if (norm == ORC_NORM_MOMENT) {
        acc[2 * o] += sigma * I[2 * o];
        acc[2 * o + 1] += sigma * I[2 * o + 1];
      } else {
        const int om = n * n + n - m;
        const double s = sigma * ((n & 1) ? -1.0 : 1.0) / (4.0 * ORC_PI);
        acc[2 * o] += s * I[2 * om];
        acc[2 * o + 1] += s * I[2 * om + 1];
      }
    }
  }
}

static int nverts_of(int kind) {
  switch (kind) {
    case ORC_SEGMENT: return 2;
    case ORC_TET: return 4;
    default: return 3;
  }
}

/*
 * Stable bucketing of elements by box: perm lists the valid elements grouped
 * by box in increasing box id, increasing element index inside a box;
 * box_start[b]..box_start[b+1] is box b's range.  Elements whose box id is
 * outside [0, nb) are left out and counted in *n_invalid.
 */
int orc_bucket(const int32_t *elem_box, int64_t ne, int64_t nb, int32_t *perm, int64_t *box_start,
               int64_t *n_invalid) {
  int64_t bad = 0;
  for (int64_t b = 0; b <= nb; ++b) box_start[b] = 0;
  for (int64_t e = 0; e < ne; ++e) {
    const int32_t b = elem_box[e];
    if (b < 0 || b >= nb) {
      ++bad;
      continue;
    }
    box_start[b + 1] += 1;
  }
  for (int64_t b = 0; b < nb; ++b) box_start[b + 1] += box_start[b];
  int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nb > 0 ? nb : 1));
  for (int64_t b = 0; b < nb; ++b) cur[b] = box_start[b];
  for (int64_t e = 0; e < ne; ++e) {
    const int32_t b = elem_box[e];
    if (b < 0 || b >= nb) continue;
    perm[cur[b]++] = (int32_t)e;
  }
  free(cur);
  if (n_invalid) *n_invalid = bad;
  return 0;
}

/*
 * Per-box coefficients for the boxes listed in box_list (or all boxes when
 * box_list == NULL, nlist = nb).  out[l][(p+1)^2][2] for list entry l.
 * Elements are summed per box in increasing element index; OpenMP over boxes.
 */
int orc_q2x_boxes(int kind, int p, int norm, const double *verts, int64_t nv, const int32_t *elems,
                  int64_t ne, const double *density, const int32_t *elem_box, const double *box_center,
                  int64_t nb, const int64_t *box_list, int64_t nlist, int nodes, int nthreads,
                  double *out) {
  if (p < 0 || p > ORC_PMAX || kind < 0 || kind > 3) return -1;
  const int nvk = nverts_of(kind);
  const int ncoef = (p + 1) * (p + 1);
  int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ne > 0 ? ne : 1));
  int64_t *bs = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nb + 1));
  orc_bucket(elem_box, ne, nb, perm, bs, NULL);
  memset(out, 0, sizeof(double) * 2 * (size_t)ncoef * (size_t)nlist);
  int err = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int64_t l = 0; l < nlist; ++l) {
    const int64_t b = box_list ? box_list[l] : l;
    if (b < 0 || b >= nb) continue;
    double *I = (double *)malloc(sizeof(double) * 2 * (size_t)ncoef);
    double xv[12];
    for (int64_t q = bs[b]; q < bs[b + 1]; ++q) {
      const int32_t e = perm[q];
      int ok = 1;
      for (int k = 0; k < nvk; ++k) {
        const int32_t vi = elems[(int64_t)e * nvk + k];
        if (vi < 0 || vi >= nv) { ok = 0; break; }
        xv[3 * k] = verts[3 * (int64_t)vi];
        xv[3 * k + 1] = verts[3 * (int64_t)vi + 1];
        xv[3 * k + 2] = verts[3 * (int64_t)vi + 2];
      }
      if (!ok) { err = -3; continue; }
      orc_element_integral(kind, p, xv, &box_center[3 * b], nodes, I, NULL);
      add_coeffs(p, norm, density[e], I, &out[2 * (size_t)ncoef * (size_t)l]);
    }
    free(I);
  }
  free(perm);
  free(bs);
  return err;
}

int orc_q2x(int kind, int p, int norm, const double *verts, int64_t nv, const int32_t *elems, int64_t ne,
            const double *density, const int32_t *elem_box, const double *box_center, int64_t nb,
            int nodes, int nthreads, double *out) {
  return orc_q2x_boxes(kind, p, norm, verts, nv, elems, ne, density, elem_box, box_center, nb, NULL, nb,
                       nodes, nthreads, out);
}

/*
 * Per-element, per-degree 2-norms of the unit-density FMM coefficients:
 * out[e][n] = || (1/4pi) int_e R_n^{-m}(y - c_{box(e)}) dmu ||_2 over m.
 * Used to build the scale-aware error denominator A_{b,n} = sum |sigma_e| out[e][n].
 */
int orc_element_norms(int kind, int p, const double *verts, int64_t nv, const int32_t *elems, int64_t ne,
                      const int32_t *elem_box, const double *box_center, int64_t nb, int nodes,
                      int nthreads, double *out) {
  const int nvk = nverts_of(kind);
  const int ncoef = (p + 1) * (p + 1);
  int err = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
  for (int64_t e = 0; e < ne; ++e) {
    double *I = (double *)malloc(sizeof(double) * 2 * (size_t)ncoef);
    double xv[12];
    const int32_t b = elem_box[e];
    for (int n = 0; n <= p; ++n) out[(size_t)e * (p + 1) + n] = 0.0;
    int ok = (b >= 0 && b < nb);
    for (int k = 0; ok && k < nvk; ++k) {
      const int32_t vi = elems[(int64_t)e * nvk + k];
      if (vi < 0 || vi >= nv) { ok = 0; break; }
      xv[3 * k] = verts[3 * (int64_t)vi];
      xv[3 * k + 1] = verts[3 * (int64_t)vi + 1];
      xv[3 * k + 2] = verts[3 * (int64_t)vi + 2];
    }
    if (ok) {
      orc_element_integral(kind, p, xv, &box_center[3 * (int64_t)b], nodes, I, NULL);
      for (int n = 0; n <= p; ++n) {
        double s = 0.0;
        for (int m = -n; m <= n; ++m) {
          const int o = n * n + n + m;
          s += I[2 * o] * I[2 * o] + I[2 * o + 1] * I[2 * o + 1];
        }
        out[(size_t)e * (p + 1) + n] = sqrt(s) / (4.0 * ORC_PI);
      }
    } else if (b >= 0 && b < nb) {
      err = -3;
    }
    free(I);
  }
  return err;
}

/*
 * Receiving side (Sec. 2 after Eq. (5): the same integrals serve the
 * evaluation stage of a Galerkin method): for every element e with box b,
 *   out[e]   = sum_{n<=p} sum_{m=-n..n} L_b[n,m] * I_e[n,m]
 *   scale[e] = sum_{n,m} |L_b[n,m]| |I_e[n,m]|
 * with I_e the unit-density integrals of orc_element_integral (int R_n^m, or
 * n.grad R_n^m for the double layer) about the box centre, L [nb][(p+1)^2][2]
 * local coefficients of a field sum L_n^m R_n^m(y - c_b).  Elements with a
 * box id outside [0, nb) get 0.  OpenMP over elements.
 */
int orc_eval(int kind, int p, const double *verts, int64_t nv, const int32_t *elems, int64_t ne,
             const int32_t *elem_box, const double *box_center, int64_t nb, const double *local, int nodes,
             int nthreads, double *out, double *scale) {
  if (p < 0 || p > ORC_PMAX || kind < 0 || kind > 3) return -1;
  const int nvk = nverts_of(kind);
  const int ncoef = (p + 1) * (p + 1);
  int err = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
  for (int64_t e = 0; e < ne; ++e) {
    out[2 * e] = out[2 * e + 1] = 0.0;
    if (scale) scale[e] = 0.0;
    const int32_t b = elem_box[e];
    if (b < 0 || b >= nb) continue;
    double xv[12];
    int ok = 1;
    for (int k = 0; ok && k < nvk; ++k) {
      const int32_t vi = elems[(int64_t)e * nvk + k];
      if (vi < 0 || vi >= nv) { ok = 0; break; }
      xv[3 * k] = verts[3 * (int64_t)vi];
      xv[3 * k + 1] = verts[3 * (int64_t)vi + 1];
      xv[3 * k + 2] = verts[3 * (int64_t)vi + 2];
    }
    if (!ok) { err = -3; continue; }
    double *I = (double *)malloc(sizeof(double) * 2 * (size_t)ncoef);
    orc_element_integral(kind, p, xv, &box_center[3 * (int64_t)b], nodes, I, NULL);
    const double *L = &local[2 * (size_t)ncoef * (size_t)b];
    double re = 0.0, im = 0.0, sc = 0.0;
    for (int o = 0; o < ncoef; ++o) {
      re += L[2 * o] * I[2 * o] - L[2 * o + 1] * I[2 * o + 1];
      im += L[2 * o] * I[2 * o + 1] + L[2 * o + 1] * I[2 * o];
      sc += hypot(L[2 * o], L[2 * o + 1]) * hypot(I[2 * o], I[2 * o + 1]);
    }
    out[2 * e] = re;
    out[2 * e + 1] = im;
    if (scale) scale[e] = sc;
    free(I);
  }
  return err;
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/*
 * Multipole-to-multipole translation (the upward pass of the FMM that
 * consumes the box coefficients; Sec. 1-2).  R_n^m is a homogeneous harmonic
 * polynomial whose derivatives are again R's (Sec. 3.2, Eq. (15)); Taylor
 * expansion of R_n^m(u + t) in t therefore gives the finite addition theorem
 *   R_n^m(u + t) = sum_{k=0}^{n} sum_{l=-k}^{k} R_k^l(u) R_{n-k}^{m-l}(t)
 * (terms with |m - l| > n - k are zero).  Applied to y - c_p = (y - c_c) +
 * (c_c - c_p) inside the definition of the coefficients:
 *   MOMENT: M_n^m(c_p) = sum_{k,l} M_k^l(c_c) R_{n-k}^{m-l}(c_c - c_p)
 *   FMM   : F_n^m(c_p) = sum_{k,l} F_k^l(c_c) (-1)^{n-k} R_{n-k}^{l-m}(c_c - c_p)
 * (FMM: F_n^m = (1/4pi)(-1)^n int R_n^{-m}, Sec. 3.2 Eq. (14)).  The
 * translation of an expansion truncated at p is exact for every n <= p.
 * For every child c with parent child_parent[c] in [0, n_parent):
 *   out[parent] += translated child coefficients
 *   scale[parent][n*n+n+m] += sum_{k,l} |coef_k^l| |R_{n-k}^{.}|
 * All (n, m) of the input are read (no symmetry is assumed).  Children with a
 * parent id outside [0, n_parent) are skipped (return value counts them).
 * Sequential over children in index order.
 */
int orc_m2m(int p, int norm, const double *child, const double *child_center, const int32_t *child_parent,
            int64_t n_child, const double *parent_center, int64_t n_parent, double *out, double *scale) {
  if (p < 0 || p > ORC_PMAX) return -1;
  const int nc = (p + 1) * (p + 1);
  memset(out, 0, sizeof(double) * 2 * (size_t)nc * (size_t)n_parent);
  memset(scale, 0, sizeof(double) * (size_t)nc * (size_t)n_parent);
  double *R = (double *)malloc(sizeof(double) * 2 * (size_t)nc);
  if (!R) return -2;
  int skipped = 0;
  for (int64_t c = 0; c < n_child; ++c) {
    const int32_t b = child_parent[c];
    if (b < 0 || b >= n_parent) {
      ++skipped;
      continue;
    }
    double t[3];
    sub3(&child_center[3 * c], &parent_center[3 * (int64_t)b], t);
    orc_solid_harmonics(p, t[0], t[1], t[2], R, NULL);
    const double *in = child + 2 * (size_t)nc * (size_t)c;
    double *o = out + 2 * (size_t)nc * (size_t)b;
    double *sc = scale + (size_t)nc * (size_t)b;
    for (int n = 0; n <= p; ++n) {
      for (int m = -n; m <= n; ++m) {
        double sr = 0.0, si = 0.0, sa = 0.0;
        for (int k = 0; k <= n; ++k) {
          const int j = n - k;
          for (int l = -k; l <= k; ++l) {
            const int q = (norm == ORC_NORM_MOMENT) ? (m - l) : (l - m);
            if (q < -j || q > j) continue;
            const double ar = in[2 * (k * k + k + l)], ai = in[2 * (k * k + k + l) + 1];
            double rr = R[2 * (j * j + j + q)], ri = R[2 * (j * j + j + q) + 1];
            if (norm != ORC_NORM_MOMENT && (j & 1)) {
              rr = -rr;
              ri = -ri;
            }
            sr += ar * rr - ai * ri;
            si += ar * ri + ai * rr;
            sa += sqrt(ar * ar + ai * ai) * sqrt(rr * rr + ri * ri);
          }
        }
        const int oi = n * n + n + m;
        o[2 * oi] += sr;
        o[2 * oi + 1] += si;
        sc[oi] += sa;
      }
    }
  }
  free(R);
  return skipped;
}

/*
 * Near field: the single- and double-layer potentials of one flat triangle
 * with unit density at a point r (the integrals L and M of Sec. 4.1,
 * Eq. (63), which the paper evaluates in closed form; computed here WITHOUT
 * that formula):
 *   L(r) = int_T G(r, y) dS_y,   M(r) = int_T dG/dn_y dS_y = int_T hs / (4 pi |r - y|^3) dS_y,
 * G = 1/(4 pi |r - y|), n the unit normal (x2 - x1) x (x3 - x1) / |.|, hs =
 * (r - x1) . n the signed height, h = |hs|.  The triangle is split at the
 * projection r0 = r - hs n into the three triangles (r0, x_q, x_q+1), signed
 * by orientation, and each is integrated in polar coordinates about r0.  The
 * radial integrals are elementary:
 *   int_0^rho s ds / sqrt(s^2 + h^2)          = rho^2 / (R + h),        R = sqrt(rho^2 + h^2)
 *   int_0^rho hs s ds / (s^2 + h^2)^(3/2)     = sign(hs) rho^2 / (R (R + h))
 * and along an edge y(t) = a + t (b - a) the angle element is
 * dphi = A2 / rho(t)^2 dt, A2 = ((a - r0) x (b - a)) . n, so
 *   L = (1/4pi) sum_edges A2 int_0^1 dt / (R(t) + h)
 *   M = (1/4pi) sign(hs) sum_edges A2 int_0^1 dt / (R(t) (R(t) + h)).
 * The t-integrals use Gauss-Legendre (k nodes) on panels graded
 * geometrically towards the foot t* of the perpendicular from r0 to the edge
 * line (widths sqrt(d^2 + h^2)/|b - a| times powers of 2), where the integrand
 * varies fastest.  On the plane M = 0 (the principal value); a target within
 * 1e-12 times the longest edge of the plane counts as on it, so that
 * collocation at a point of the element itself (whose computed height is
 * rounding noise) gets the principal value rather than a one-sided +-1/2.
 */
static void near_edge(const double *a, const double *b, const double *r0, const double *n, double h,
                      const double *gx, const double *gw, int k, double *iL, double *iM) {
  double e[3], ar[3], c[3];
  sub3(b, a, e);
  sub3(a, r0, ar);
  cross3(ar, e, c);
  const double A2 = dot3(c, n);
  *iL = 0.0;
  *iM = 0.0;
  const double L2 = dot3(e, e);
  if (A2 == 0.0 || L2 == 0.0) return;
  const double ts = -dot3(ar, e) / L2;
  /* distance of r0 from the edge line: |A2| = d |b - a| (r0, a, b lie in the
     plane), consistent with A2 and free of the cancellation of |ar|^2 - (ar.e)^2/L2 */
  const double d2 = A2 * A2 / L2;
  const double w0 = sqrt((d2 + h * h) / L2);
  /* breakpoints: 0, 1 and t* +- w0 2^j inside (0, 1) */
  double bp[256];
  int nb = 0;
  bp[nb++] = 0.0;
  bp[nb++] = 1.0;
  if (ts > 0.0 && ts < 1.0) bp[nb++] = ts;
  for (int j = 0; j < 60 && nb < 250; ++j) {
    const double w = w0 * ldexp(1.0, j);
    if (w > 2.0) break;
    if (ts - w > 0.0 && ts - w < 1.0) bp[nb++] = ts - w;
    if (ts + w > 0.0 && ts + w < 1.0) bp[nb++] = ts + w;
  }
  /* sort (insertion; nb is small) */
  for (int i = 1; i < nb; ++i) {
    const double v = bp[i];
    int j = i - 1;
    while (j >= 0 && bp[j] > v) {
      bp[j + 1] = bp[j];
      --j;
    }
    bp[j + 1] = v;
  }
  double sL = 0.0, sM = 0.0;
  for (int i = 0; i + 1 < nb; ++i) {
    const double t0 = bp[i], t1 = bp[i + 1], dt = t1 - t0;
    if (!(dt > 0.0)) continue;
    for (int g = 0; g < k; ++g) {
      const double t = t0 + dt * gx[g];
      const double rho2 = d2 + L2 * (t - ts) * (t - ts);
      const double R = sqrt(rho2 + h * h);
      sL += dt * gw[g] / (R + h);
      sM += dt * gw[g] / (R * (R + h));
    }
  }
  *iL = A2 * sL;
  *iM = A2 * sM;
}

int orc_near_one(const double *r, const double *x1, const double *x2, const double *x3, int k, double *L,
                 double *M) {
  if (k < 1 || k > 4 * ORC_KMAX) return -1;
  double gx[4 * ORC_KMAX], gw[4 * ORC_KMAX];
  orc_gauss_legendre01(k, gx, gw);
  double u[3], v[3], n[3], rx[3];
  sub3(x2, x1, u);
  sub3(x3, x1, v);
  cross3(u, v, n);
  const double J = sqrt(dot3(n, n));
  *L = 0.0;
  *M = 0.0;
  if (!(J > 0.0)) return 0; /* degenerate: zero area */
  for (int i = 0; i < 3; ++i) n[i] /= J;
  sub3(r, x1, rx);
  double hs = dot3(rx, n);
  double r0[3];
  for (int i = 0; i < 3; ++i) r0[i] = r[i] - hs * n[i];
  /* a target within 1e-12 (longest edge) of the plane is on it: principal
     value M = 0 and h = 0 (collocation on the element itself) */
  {
    double e1[3], e2[3], e3[3];
    sub3(x2, x1, e1);
    sub3(x3, x2, e2);
    sub3(x1, x3, e3);
    const double lmax = sqrt(fmax(dot3(e1, e1), fmax(dot3(e2, e2), dot3(e3, e3))));
    if (fabs(hs) <= 1e-12 * lmax) hs = 0.0;
  }
  const double h = fabs(hs);
  const double *xs[4] = {x1, x2, x3, x1};
  double sL = 0.0, sM = 0.0;
  for (int q = 0; q < 3; ++q) {
    double iL, iM;
    near_edge(xs[q], xs[q + 1], r0, n, h, gx, gw, k, &iL, &iM);
    sL += iL;
    sM += iM;
  }
  *L = sL / (4.0 * ORC_PI);
  *M = (hs > 0.0 ? 1.0 : (hs < 0.0 ? -1.0 : 0.0)) * sM / (4.0 * ORC_PI);
  return 0;
}

/*
 * Per pair p in [pair_start[t], pair_start[t+1]) of target t: L and M of
 * triangle pair_tri[p] at targets[t] (unit density).  Bad triangle or vertex
 * indices give -1 and leave the pair's outputs 0.  OpenMP over targets.
 */
int orc_near(const double *verts, int64_t nv, const int32_t *tris, int64_t ntri, const double *targets, int64_t nt,
             const int64_t *pair_start, const int32_t *pair_tri, int k, int nthreads, double *out_L, double *out_M) {
  int err = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 16) reduction(min : err)
  for (int64_t t = 0; t < nt; ++t) {
    for (int64_t p = pair_start[t]; p < pair_start[t + 1]; ++p) {
      out_L[p] = 0.0;
      out_M[p] = 0.0;
      const int32_t j = pair_tri[p];
      if (j < 0 || j >= ntri) {
        err = -1;
        continue;
      }
      const int32_t *tv = &tris[3 * (int64_t)j];
      if (tv[0] < 0 || tv[0] >= nv || tv[1] < 0 || tv[1] >= nv || tv[2] < 0 || tv[2] >= nv) {
        err = -1;
        continue;
      }
      orc_near_one(&targets[3 * t], &verts[3 * (int64_t)tv[0]], &verts[3 * (int64_t)tv[1]],
                   &verts[3 * (int64_t)tv[2]], k, &out_L[p], &out_M[p]);
    }
  }
  return err;
}
