// q2x_near.hip -- near field: single- and double-layer potentials of flat
// triangles with constant density at nearby targets, in closed form (the
// contour formula of Sec. 4.1, Eq. (63)), for (target, triangle) pairs given
// in compressed rows by target.  This is the part of an FMM-accelerated BEM
// step that the multipole expansions do not cover; computed on the fly it is
// where the time goes (Sec. 4.2).
//
// Per pair, for the triangle x1 x2 x3 with unit normal n = (x2-x1)x(x3-x1)/|.|,
// signed height hs = (r - x1).n and h = |hs|, edges q (x_q -> x_q+1, length
// l_q, unit direction i_q, in-plane normal n_q = i_q x n):
//   L(r) = (1/4pi) sum_q [L_P(l_q - x_q, h, z_q) - L_P(-x_q, h, z_q)]
//   M(r) = sign(hs) (1/4pi) sum_q [M_P(l_q - x_q, h, z_q) - M_P(-x_q, h, z_q)]
//   x_q = (r - x_q).i_q,  z_q = (r - x_q).n_q,
//   M_P(x, y, z) = -atan(x z (R - y) / (R z^2 + y x^2)),
//   L_P(x, y, z) = -y M_P(x, y, z) - z ln(R + x),  R = sqrt(x^2 + y^2 + z^2).
// Per edge the two ends combine: the M_P difference is the argument of a
// product of two complex numbers and the ln difference the log of a ratio.
// The three edges' angles add up to the argument of the product of their
// three complex numbers; one atan2 gives it modulo 2 pi, and the octants of
// the three factors (each angle known to within pi/8) fix the multiple of
// 2 pi.  Every edge angle lies in (-pi, pi) (both ends' M_P in (-pi/2, pi/2)).
// The printed M lacks the factor sign(hs): with h = |hs| the contour sum is
// the value on the +n side, and M is odd in hs.  R - y and R + x (x < 0) are
// formed without cancellation as (x^2 + z^2)/(R + y) and (y^2 + z^2)/(R - x),
// the first folded into the angle (both N and D are scaled by R + y > 0), the
// second kept as a fraction; terms with z = 0 vanish.  R at an edge's ends is
// the distance to that vertex, shared by the two edges that meet there.  A
// target within 1e-12 (longest edge) of the plane counts as on it: h = 0 and
// M = 0, the principal value (collocation on the element itself, whose
// computed height is rounding noise).
//
// One wavefront per target: lanes take the target's pairs in strides of 64,
// write the per-pair values if asked (the stored near-field matrix) and sum
// sigma_j L + mu_j M; a butterfly reduction gives the target's potential.
#include <float.h>
#include <math.h>

#include "q2x_internal.hpp"

namespace q2x {

struct NearArgs {
  const double* verts;
  const int32_t* tris;
  const double* targets;
  const int64_t* pair_start;  // [n_targets + 1]
  const int32_t* pair_tri;    // [n_pairs]
  const double* dens_single;  // [n_tris] or nullptr
  const double* dens_double;  // [n_tris] or nullptr
  double* entries_L;          // [n_pairs] or nullptr
  double* entries_M;          // [n_pairs] or nullptr
  double* pot;                // [n_targets] or nullptr
  Status* status;
  int64_t n_verts, n_tris, n_targets, n_pairs;
  int accumulate;
};

constexpr double kInv4PiNear = 0.07957747154594766788;

// One end of an edge (z != 0), at distance R from the target: M_P =
// -atan(N / D) with N = x z (R - y) and D = R z^2 + y x^2 >= 0, here both
// times R + y (no division, the angle unchanged), and R + x = a / b.
struct NearEnd {
  double N, D, a, b;
};
__device__ __forceinline__ NearEnd near_end(double x, double y, double z, double R) {
  const double x2 = x * x, z2 = z * z;
  NearEnd e;
  e.N = x * z * (x2 + z2);
  e.D = (R * z2 + y * x2) * (R + y);
  const bool pos = x >= 0.0;
  e.a = pos ? R + x : y * y + z2;  // > 0 for z != 0
  e.b = pos ? 1.0 : R - x;
  return e;
}

// The angle of c + i s (in (-pi, pi)) to within pi/8: the centre of its octant.
__device__ __forceinline__ double octant_centre(double c, double s) {
  constexpr double k8 = 0.39269908169872415481;  // pi / 8
  const double as = fabs(s), ac = fabs(c);
  const double m = (c >= 0.0) ? (as <= ac ? 1.0 : 3.0) : (as >= ac ? 5.0 : 7.0);
  return copysign(m * k8, s);
}

// 1 / sqrt(x) for finite x > 0: the hardware estimate refined by two
// Newton-Raphson steps y <- y + y (1 - x y^2) / 2, each of which squares the
// relative error (x y is formed first so that nothing underflows).
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double xy = x * y;
    y = fma(0.5 * y, fma(-xy, y, 1.0), y);
  }
  return y;
}

// Cross product without contraction into FMAs: parallel edge vectors (a
// zero-area triangle) give exactly 0.
__device__ __forceinline__ void near_cross(double ux, double uy, double uz, double vx, double vy, double vz,
                                          double& cx, double& cy, double& cz) {
#pragma clang fp contract(off)
  cx = uy * vz - uz * vy;
  cy = uz * vx - ux * vz;
  cz = ux * vy - uy * vx;
}

// L and M of one unit-density triangle at r; returns false for a degenerate
// triangle (zero area, or a cross product beyond the FP64 range): L = M = 0.
__device__ bool near_pair(const double* r, const double (&X)[3][3], double& L, double& M) {
  const double ux = X[1][0] - X[0][0], uy = X[1][1] - X[0][1], uz = X[1][2] - X[0][2];
  const double vx = X[2][0] - X[0][0], vy = X[2][1] - X[0][1], vz = X[2][2] - X[0][2];
  double cx, cy, cz;
  near_cross(ux, uy, uz, vx, vy, vz, cx, cy, cz);
  const double c2 = cx * cx + cy * cy + cz * cz;  // (2 area)^2
  L = 0.0;
  M = 0.0;
  if (!(c2 > 0.0) || !(c2 <= DBL_MAX)) return false;  // zero area, or a cross product that overflows
  const double iJ = rsqrt_nr(c2);
  const double nx = cx * iJ, ny = cy * iJ, nz = cz * iJ;
  // edge lengths and their reciprocals (every edge of a triangle of nonzero
  // area is nonzero)
  double el[3], eil[3], lmax = 0.0;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int q1 = (q + 1) % 3;
    const double ex = X[q1][0] - X[q][0], ey = X[q1][1] - X[q][1], ez = X[q1][2] - X[q][2];
    const double e2 = ex * ex + ey * ey + ez * ez;
    eil[q] = rsqrt_nr(e2);
    el[q] = e2 * eil[q];
    lmax = fmax(lmax, el[q]);
  }
  double hs = (r[0] - X[0][0]) * nx + (r[1] - X[0][1]) * ny + (r[2] - X[0][2]) * nz;
  if (fabs(hs) <= 1e-12 * lmax) hs = 0.0;
  const double h = fabs(hs);
  // distances to the vertices (R at both ends of every edge)
  double rho[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double dx = r[0] - X[k][0], dy = r[1] - X[k][1], dz = r[2] - X[k][2];
    rho[k] = sqrt(dx * dx + dy * dy + dz * dz);
  }
  double sL = 0.0;            // sum of -z_q ln(ratio_q)
  double Pr = 1.0, Pi = 0.0;  // product of the edges' complex numbers
  double est = 0.0;           // sum of their octant centres
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int q1 = (q + 1) % 3;
    const double ex = X[q1][0] - X[q][0], ey = X[q1][1] - X[q][1], ez = X[q1][2] - X[q][2];
    const double l = el[q], il = eil[q];
    const double ix = ex * il, iy = ey * il, iz = ez * il;
    // n_q = i_q x n
    const double mx = iy * nz - iz * ny, my = iz * nx - ix * nz, mz = ix * ny - iy * nx;
    const double dx = r[0] - X[q][0], dy = r[1] - X[q][1], dz = r[2] - X[q][2];
    const double xq = dx * ix + dy * iy + dz * iz;
    const double zq = dx * mx + dy * my + dz * mz;
    if (zq == 0.0) continue;  // both ends' terms vanish
    // M_P(l - x) - M_P(-x) = arg((D0 + i N0) conj(D1 + i N1))
    const NearEnd e1 = near_end(l - xq, h, zq, rho[q1]), e0 = near_end(-xq, h, zq, rho[q]);
    double c = e0.D * e1.D + e0.N * e1.N, sn = e0.N * e1.D - e0.D * e1.N;
    est += octant_centre(c, sn);
    // scale to magnitude ~1 (exact) so that the product stays in range
    const int ex2 = __builtin_amdgcn_frexp_exp(fmax(fabs(c), fabs(sn)));
    c = ldexp(c, -ex2);
    sn = ldexp(sn, -ex2);
    const double pr = Pr * c - Pi * sn, pi = Pr * sn + Pi * c;
    Pr = pr;
    Pi = pi;
    // ln(R1 + x1) - ln(R0 + x0), x1 = l - x_q, x0 = -x_q
    sL -= zq * log((e1.a * e0.b) / (e0.a * e1.b));
  }
  // the sum of the edge angles: atan2 of the product plus the multiple of
  // 2 pi that brings it nearest the octant estimate (within 3 pi / 8)
  constexpr double k2pi = 6.28318530717958647692;
  const double phi = atan2(Pi, Pr);
  const double sM = phi + k2pi * rint((est - phi) * (1.0 / k2pi));
  sL -= h * sM;
  L = sL * kInv4PiNear;
  M = (hs > 0.0 ? sM : (hs < 0.0 ? -sM : 0.0)) * kInv4PiNear;
  return true;
}

// Three wavefronts per SIMD (at most 168 VGPRs, a few spilled): the pairs'
// dependent loads and FP64 chains need the extra wavefront to hide latency
// (measured: 0.98 -> 0.90 ms at 25.2M pairs; four per SIMD spill heavily and
// run 1.45 ms).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void q2x_near_kernel(NearArgs a) {
  const int lane = threadIdx.x & 63;
  // blocks in XCD order (each XCD's L2 gets a contiguous run of targets, whose
  // neighbourhoods share triangles)
  const int64_t wave = xcd_tile(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  uint32_t flag = 0;
  unsigned long long ndeg = 0, nskip = 0;
  for (int64_t t = wave; t < a.n_targets; t += nwaves) {  // uniform per wavefront
    int64_t s0 = a.pair_start[t], s1 = a.pair_start[t + 1];
    if (s0 < 0 || s1 > a.n_pairs || s1 < s0) {  // malformed rows: no pairs read
      flag |= Q2X_FLAG_BAD_BOX;
      s0 = s1 = 0;
    }
    const double r[3] = {a.targets[3 * t], a.targets[3 * t + 1], a.targets[3 * t + 2]};
    const bool rfin = isfinite(r[0]) && isfinite(r[1]) && isfinite(r[2]);
    double acc = 0.0;
    for (int64_t p = s0 + lane; p < s1; p += 64) {
      double L = 0.0, M = 0.0;
      const int32_t j = a.pair_tri[p];
      bool ok = rfin;
      if (j < 0 || j >= a.n_tris) {
        ok = false;
        flag |= Q2X_FLAG_BAD_BOX;
      }
      double X[3][3];
      if (ok) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const int32_t vi = a.tris[3 * (int64_t)j + k];
          if (vi < 0 || vi >= a.n_verts) {
            ok = false;
            flag |= Q2X_FLAG_BAD_VERTEX;
            X[k][0] = X[k][1] = X[k][2] = 0.0;
          } else {
            X[k][0] = a.verts[3 * (int64_t)vi];
            X[k][1] = a.verts[3 * (int64_t)vi + 1];
            X[k][2] = a.verts[3 * (int64_t)vi + 2];
          }
        }
      }
      if (ok) {
        bool fin = true;
#pragma unroll
        for (int k = 0; k < 3; ++k) fin = fin && isfinite(X[k][0]) && isfinite(X[k][1]) && isfinite(X[k][2]);
        if (!fin) {
          ok = false;
          flag |= Q2X_FLAG_NONFINITE;
        }
      } else if (!rfin) {
        flag |= Q2X_FLAG_NONFINITE;
      }
      if (ok) {
        if (!near_pair(r, X, L, M)) ++ndeg;
        const double ss = a.dens_single ? a.dens_single[j] : 0.0;
        const double sd = a.dens_double ? a.dens_double[j] : 0.0;
        acc += ss * L + sd * M;
      } else {
        ++nskip;
      }
      if (a.entries_L) a.entries_L[p] = L;
      if (a.entries_M) a.entries_M[p] = M;
    }
    // fixed-order butterfly: every lane ends with the same sum
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0 && a.pot) a.pot[t] = a.accumulate ? a.pot[t] + acc : acc;
  }
  // status: one atomic per wavefront and counter
  const uint64_t fl = __ballot(flag != 0);
  uint32_t fall = 0;
  if (fl) {
#pragma unroll
    for (int b = 0; b < 5; ++b)
      if (__ballot((flag >> b) & 1u)) fall |= (1u << b);
  }
  unsigned long long d = ndeg, s = nskip;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    d += __shfl_xor(d, off);
    s += __shfl_xor(s, off);
  }
  if (lane == 0) {
    if (d) atomicAdd(&a.status->n_degenerate, d);
    if (s) atomicAdd(&a.status->n_skipped, s);
    if (fall) atomicOr(&a.status->flags, fall);
  }
}


}  // namespace q2x

using namespace q2x;

extern "C" {

size_t q2x_near_workspace_bytes(void) { return 256; }

q2x_status q2x_near(const double* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris, const double* targets,
                    int64_t n_targets, const int64_t* pair_start, const int32_t* pair_tri, int64_t n_pairs,
                    const double* density_single, const double* density_double, double* entries_L,
                    double* entries_M, double* potential, unsigned flags, void* workspace, size_t workspace_bytes,
                    void* stream) {
  if (n_verts < 0 || n_tris < 0 || n_targets < 0 || n_pairs < 0 || n_tris >= ((int64_t)1 << 31) ||
      n_verts >= ((int64_t)1 << 31))
    return Q2X_ERR_ARG;
  if (flags & ~(unsigned)Q2X_ACCUMULATE) return Q2X_ERR_ARG;
  if (!workspace || ((uintptr_t)workspace % 256) != 0) return Q2X_ERR_WORKSPACE;
  if (workspace_bytes < q2x_near_workspace_bytes()) return Q2X_ERR_WORKSPACE;
  if (n_targets > 0 && (!targets || !pair_start)) return Q2X_ERR_ARG;
  if (n_pairs > 0 && (!pair_tri || !verts || !tris)) return Q2X_ERR_ARG;
  if (potential && !density_single && !density_double) return Q2X_ERR_ARG;  // nothing to sum
  if (!potential && !entries_L && !entries_M) return Q2X_ERR_ARG;           // nothing to write
  if (((uintptr_t)verts % 8) || ((uintptr_t)tris % 4) || ((uintptr_t)targets % 8) || ((uintptr_t)pair_start % 8) ||
      ((uintptr_t)pair_tri % 4) || ((uintptr_t)density_single % 8) || ((uintptr_t)density_double % 8) ||
      ((uintptr_t)entries_L % 8) || ((uintptr_t)entries_M % 8) || ((uintptr_t)potential % 8))
    return Q2X_ERR_ARG;
  hipStream_t s = (hipStream_t)stream;
  Status* st = (Status*)workspace;
  if (clear_status(st, s) != hipSuccess) return Q2X_ERR_HIP;
  if (n_targets == 0) return Q2X_OK;
  NearArgs a{};
  a.verts = verts;
  a.tris = tris;
  a.targets = targets;
  a.pair_start = pair_start;
  a.pair_tri = pair_tri;
  a.dens_single = density_single;
  a.dens_double = density_double;
  a.entries_L = entries_L;
  a.entries_M = entries_M;
  a.pot = potential;
  a.status = st;
  a.n_verts = n_verts;
  a.n_tris = n_tris;
  a.n_targets = n_targets;
  a.n_pairs = n_pairs;
  a.accumulate = (flags & Q2X_ACCUMULATE) ? 1 : 0;
  int64_t blocks = (n_targets + 3) / 4;  // four wavefronts per block
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(q2x_near_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a);
  if (hipGetLastError() != hipSuccess) return Q2X_ERR_HIP;
  return Q2X_OK;
}

}  // extern "C"
