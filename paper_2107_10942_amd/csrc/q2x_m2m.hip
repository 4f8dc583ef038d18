// q2x_m2m.hip -- multipole-to-multipole translation: the step of the FMM
// upward pass that consumes the box coefficients (Sec. 1-2).
//
// R_n^m is a homogeneous harmonic polynomial whose derivatives are again
// R's (Sec. 3.2, Eq. (15)), so Taylor expansion gives the finite addition
// theorem R_n^m(u + t) = sum_{k<=n, l} R_k^l(u) R_{n-k}^{m-l}(t).  Inside the
// definition of the coefficients (Sec. 3.2, Eq. (14)) this translates a
// child's expansion about c_c to its parent's centre c_p exactly (n <= p):
//   MOMENT: M_n^m(c_p) = sum_{k,l} M_k^l(c_c) R_{n-k}^{m-l}(c_c - c_p)
//   FMM   : F_n^m(c_p) = sum_{k,l} F_k^l(c_c) R_{n-k}^{l-m}(c_p - c_c)
// (FMM: (-1)^(n-k) R_{n-k}(c_c - c_p) = R_{n-k}(c_p - c_c), R being
// homogeneous of degree n - k).
//
// Expansions of real densities satisfy A_n^{-m} = (-1)^m conj(A_n^m) (the
// symmetry Eq. (12) carried through Eq. (14)), and so does their
// translation: the kernel reads orders m >= 0 only, computes outputs m >= 0
// and writes m < 0 from the symmetry.
//
// One workgroup of 256 threads per parent.  For each child (the children of
// a parent are a contiguous run of the box-sorted order): the child's m >= 0
// coefficients go to LDS, and R_j^q(d) (q >= 0) of the shift d is built in LDS
// degree by degree with the ladder recursion of the vertex harmonic (Sec. 3.4,
// Eq. (50): G_j = D G_{j-1}, G_0 = 1, R_j^q = (-i)^q G_j^q / j!).  Thread t
// then owns outputs (n, m) with tri index t, t + 256, t + 512 and adds
// sum_{k<=n} sum_l A_k^l R_{n-k}^{+-(l-m)} in FP64 registers.
#include <math.h>

#include "q2x_internal.hpp"

namespace q2x {

constexpr int kM2MThreads = 256;
constexpr int kM2MMaxTri = tri(Q2X_P_MAX + 1);              // 561 coefficients with m >= 0
constexpr int kM2MPerThread = (kM2MMaxTri + kM2MThreads - 1) / kM2MThreads;  // 3

__device__ __forceinline__ int tri_degree(int o) {
  int n = (int)((sqrt(8.0 * o + 1.0) - 1.0) * 0.5);
  while (tri(n + 1) <= o) ++n;
  while (tri(n) > o) --n;
  return n;
}

__global__ __launch_bounds__(kM2MThreads) void q2x_m2m_kernel(M2MArgs a) {
  __shared__ double sAr[kM2MMaxTri], sAi[kM2MMaxTri];  // child coefficients, m >= 0
  __shared__ double sRr[kM2MMaxTri], sRi[kM2MMaxTri];  // G_j^q of the shift, then R_j^q
  __shared__ int s_skip;
  const int t = threadIdx.x;
  const int p = a.p;
  const int ntri = tri(p + 1);
  const int64_t ncoef = (int64_t)(p + 1) * (p + 1);
  const bool moment = (a.norm == Q2X_NORM_MOMENT);

  if (blockIdx.x == 0 && t == 0 && a.presorted_bad) {
    // presorted input: ids below 0 sort first, ids >= n_parent last
    const int64_t bad = (int64_t)a.box_start[0] + (a.n_child - (int64_t)a.box_start[a.n_parent]);
    if (bad > 0) {
      atomicAdd(&a.status->n_skipped, (unsigned long long)bad);
      atomicOr(&a.status->flags, (uint32_t)Q2X_FLAG_BAD_BOX);
    }
  }

  for (int64_t b = blockIdx.x; b < a.n_parent; b += gridDim.x) {
    int no[kM2MPerThread], mo[kM2MPerThread];
    double accr[kM2MPerThread], acci[kM2MPerThread];
#pragma unroll
    for (int r = 0; r < kM2MPerThread; ++r) {
      const int o = t + r * kM2MThreads;
      no[r] = (o < ntri) ? tri_degree(o) : -1;
      mo[r] = (o < ntri) ? o - tri(no[r]) : 0;
      accr[r] = 0.0;
      acci[r] = 0.0;
    }
    const double pcx = a.parent_center[3 * b], pcy = a.parent_center[3 * b + 1], pcz = a.parent_center[3 * b + 2];
    const bool pfin = isfinite(pcx) && isfinite(pcy) && isfinite(pcz);
    const int64_t s0 = a.box_start[b], s1 = a.box_start[b + 1];
    if (t == 0) s_skip = 0;
    for (int64_t s = s0; s < s1; ++s) {
      const int64_t c = a.perm ? (int64_t)a.perm[s] : s;
      const double ccx = a.child_center[3 * c], ccy = a.child_center[3 * c + 1], ccz = a.child_center[3 * c + 2];
      const bool ok = pfin && isfinite(ccx) && isfinite(ccy) && isfinite(ccz);  // uniform
      if (!ok) {
        if (t == 0) ++s_skip;
        continue;
      }
      // shift d: FMM c_p - c_c, MOMENT c_c - c_p
      const double sg = moment ? 1.0 : -1.0;
      const double dx = sg * (ccx - pcx), dy = sg * (ccy - pcy), dz = sg * (ccz - pcz);
      const double* in = a.child + (size_t)c * ncoef * 2;
      __syncthreads();  // previous child's LDS reads are done
      for (int o = t; o < ntri; o += kM2MThreads) {
        const int n = tri_degree(o), m = o - tri(n);
        const int64_t g = (int64_t)n * n + n + m;
        sAr[o] = in[2 * g];
        sAi[o] = in[2 * g + 1];
      }
      // ladder: degree j from degree j - 1 (thread q computes order q)
      const double xr = 0.5 * dx, xi = 0.5 * dy;  // xi = (d_x + i d_y)/2, eta = conj(xi)
      if (t == 0) {
        sRr[0] = 1.0;
        sRi[0] = 0.0;
      }
      for (int j = 1; j <= p; ++j) {
        __syncthreads();
        double vr = 0.0, vi = 0.0;
        const int q = t;
        if (q <= j) {
          const int b0 = tri(j - 1);
          auto F = [&](int k, double& fr, double& fi) {
            if (k < 0 || k > j - 1) {
              fr = fi = 0.0;
            } else {
              fr = sRr[b0 + k];
              fi = sRi[b0 + k];
            }
          };
          double ar, ai, br, bi, cr, ci;
          if (q == 0) {
            // 2 Re(eta F^1) - z F^0
            F(1, br, bi);
            F(0, cr, ci);
            vr = 2.0 * (xr * br + xi * bi) - dz * cr;
            vi = 0.0;
          } else {
            F(q - 1, ar, ai);
            F(q + 1, br, bi);
            F(q, cr, ci);
            // -xi F^{q-1} + eta F^{q+1} - z F^q
            vr = -(xr * ar - xi * ai) + (xr * br + xi * bi) - dz * cr;
            vi = -(xr * ai + xi * ar) + (xr * bi - xi * br) - dz * ci;
          }
        }
        __syncthreads();
        if (q <= j) {
          sRr[tri(j) + q] = vr;
          sRi[tri(j) + q] = vi;
        }
      }
      __syncthreads();
      // R_j^q = (-i)^q G_j^q / j!
      for (int o = t; o < ntri; o += kM2MThreads) {
        const int j = tri_degree(o), q = o - tri(j);
        double f = 1.0;
        for (int i = 2; i <= j; ++i) f *= (double)i;
        const double gr = sRr[o] / f, gi = sRi[o] / f;
        double rr, ri;
        switch (q & 3) {  // (-i)^q
          case 0: rr = gr; ri = gi; break;
          case 1: rr = gi; ri = -gr; break;
          case 2: rr = -gr; ri = -gi; break;
          default: rr = -gi; ri = gr; break;
        }
        sRr[o] = rr;
        sRi[o] = ri;
      }
      __syncthreads();
      // out_n^m += sum_{k<=n} sum_l A_k^l R_{n-k}^{qq}, qq = l - m (FMM) or m - l (MOMENT)
#pragma unroll
      for (int r = 0; r < kM2MPerThread; ++r) {
        const int n = no[r], m = mo[r];
        if (n < 0) continue;
        double sr = 0.0, si = 0.0;
        for (int k = 0; k <= n; ++k) {
          const int j = n - k;
          const int lo = max(-k, m - j), hi = min(k, m + j);
          const int tk = tri(k), tj = tri(j);
          for (int l = lo; l <= hi; ++l) {
            const int al = l < 0 ? -l : l;
            double ar = sAr[tk + al], ai = sAi[tk + al];
            if (l < 0) {  // A^{-|l|} = (-1)^l conj(A^{|l|})
              ai = -ai;
              if (al & 1) {
                ar = -ar;
                ai = -ai;
              }
            }
            const int qq = moment ? (m - l) : (l - m);
            const int aq = qq < 0 ? -qq : qq;
            double rr = sRr[tj + aq], ri = sRi[tj + aq];
            if (qq < 0) {
              ri = -ri;
              if (aq & 1) {
                rr = -rr;
                ri = -ri;
              }
            }
            sr = fma(ar, rr, sr);
            sr = fma(-ai, ri, sr);
            si = fma(ar, ri, si);
            si = fma(ai, rr, si);
          }
        }
        accr[r] += sr;
        acci[r] += si;
      }
    }
    // write +m and -m = (-1)^m conj(+m); m = 0 is real
    double* out = a.out + (size_t)b * ncoef * 2;
#pragma unroll
    for (int r = 0; r < kM2MPerThread; ++r) {
      const int n = no[r], m = mo[r];
      if (n < 0) continue;
      double vr = accr[r], vi = (m == 0) ? 0.0 : acci[r];
      const int64_t gp = (int64_t)n * n + n + m, gm = (int64_t)n * n + n - m;
      const double sgn = (m & 1) ? -1.0 : 1.0;
      double wr = sgn * vr, wi = -sgn * vi;
      if (a.accumulate) {
        vr += out[2 * gp];
        vi += out[2 * gp + 1];
        if (m > 0) {
          wr += out[2 * gm];
          wi += out[2 * gm + 1];
        }
      }
      out[2 * gp] = vr;
      out[2 * gp + 1] = vi;
      if (m > 0) {
        out[2 * gm] = wr;
        out[2 * gm + 1] = wi;
      }
    }
    __syncthreads();
    if (t == 0 && s_skip > 0) {
      atomicAdd(&a.status->n_skipped, (unsigned long long)s_skip);
      atomicOr(&a.status->flags, (uint32_t)Q2X_FLAG_NONFINITE);
    }
  }
}

hipError_t launch_m2m(const M2MArgs& a, hipStream_t s) {
  int64_t blocks = a.n_parent;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(q2x_m2m_kernel, dim3((unsigned)blocks), dim3(kM2MThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace q2x
