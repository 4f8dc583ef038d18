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
// One workgroup per parent, NW wavefronts; wavefront w takes the parent's
// children w, w + NW, ... (the children of a parent are a contiguous run of
// the parent-sorted order).  Per child the wavefront builds, in its own LDS
// region, the child's expansion for all orders (m < 0 from the symmetry) and
// R_j^q(d) of the shift for all orders: the m >= 0 part by the ladder
// recursion of the vertex harmonic (Sec. 3.4, Eq. (50): G_j = D G_{j-1},
// G_0 = 1, R_j^q = (-i)^q G_j^q / j!), then q < 0 from Eq. (12).  Lane l owns
// the outputs (n, m >= 0) with triangular index T - 1 - l, T - 65 - l, ...
// (T = (p + 1)(p + 2) / 2: degrees descending, so that the lanes of a round
// have loops of similar length) and adds
// sum_{k<=n} sum_l A_k^l R_{n-k}^{+-(l-m)}: two contiguous LDS streams per
// degree k.  The wavefronts' partial sums meet in LDS in a fixed order.
#include <math.h>

#include "q2x_internal.hpp"

namespace q2x {

__device__ __forceinline__ int tri_degree(int o) {
  int n = (int)((sqrt(8.0 * o + 1.0) - 1.0) * 0.5);
  while (tri(n + 1) <= o) ++n;
  while (tri(n) > o) --n;
  return n;
}

__device__ __forceinline__ int sq_degree(int idx) {  // n with n^2 <= idx < (n+1)^2
  int n = (int)sqrt((double)idx);
  while ((n + 1) * (n + 1) <= idx) ++n;
  while (n * n > idx) --n;
  return n;
}

template <bool B>
struct BoolC {
  static constexpr bool value = B;
};

// wave-scope ordering of this wavefront's LDS writes before its later reads
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <int P, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NW >= 4 ? 4 : 1))) void q2x_m2m_kernel(M2MArgs a) {
  constexpr int NC = (P + 1) * (P + 1);
  constexpr int NT = tri(P + 1);
  constexpr int PER = (NT + 63) / 64;  // outputs per lane
  __shared__ double2 sbuf[NW][2][NC];  // per wavefront: A (all orders), R (all orders)
  __shared__ unsigned s_skip[NW];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  double2* const A = sbuf[w][0];
  double2* const R = sbuf[w][1];
  const int p = a.p;
  const int ncoef = (p + 1) * (p + 1);
  const int ntri = tri(p + 1);
  const bool moment = (a.norm == Q2X_NORM_MOMENT);

  if (blockIdx.x == 0 && threadIdx.x == 0 && a.presorted_bad) {
    // presorted input: ids below 0 sort first, ids >= n_parent last
    const int64_t bad = (int64_t)a.box_start[0] + (a.n_child - (int64_t)a.box_start[a.n_parent]);
    if (bad > 0) {
      atomicAdd(&a.status->n_skipped, (unsigned long long)bad);
      atomicOr(&a.status->flags, (uint32_t)Q2X_FLAG_BAD_BOX);
    }
  }

  // outputs in descending triangular order, 64 per round: the lanes of a
  // round run their loops in lockstep, and outputs of nearby degrees have
  // similar loop lengths (the longest output of a round sets its time)
  auto out_index = [&](int r) { return ntri - 1 - (64 * r + lane); };
  int no[PER], mo[PER];
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    const int o = out_index(r);
    no[r] = (o >= 0) ? tri_degree(o) : -1;
    mo[r] = (o >= 0) ? o - tri(no[r]) : 0;
  }

  // per-lane index tables, the same for every child: entry idx = lane + 64 i
  // of the full-order expansion and its source (order |m|, sign pattern of the
  // symmetry), and the R entries (j, q >= 0) with triangular index
  // lane + 64 i and their 1 / j!
  constexpr int NA = (NC + 63) / 64;
  constexpr int NR = (NT + 63) / 64;
  constexpr int kNeg = 1 << 16, kOdd = 1 << 17;
  int acode[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    const int idx = lane + 64 * i;
    acode[i] = -1;
    if (idx < ncoef) {
      const int n = sq_degree(idx), m = idx - n * n - n;
      const int am = m < 0 ? -m : m;
      acode[i] = (n * n + n + am) | (m < 0 ? kNeg : 0) | ((am & 1) ? kOdd : 0);
    }
  }
  int rjq[NR];  // j << 8 | q, or -1
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    const int o = lane + 64 * i;
    rjq[i] = -1;
    if (o < ntri) {
      const int j = tri_degree(o);
      rjq[i] = (j << 8) | (o - tri(j));
    }
  }
  // 1 / j! for j <= P (one table per workgroup)
  __shared__ double s_invf[P + 1];
  if (threadIdx.x <= P) {
    double f = 1.0;
    for (int k = 2; k <= (int)threadIdx.x; ++k) f *= (double)k;
    s_invf[threadIdx.x] = 1.0 / f;
  }
  __syncthreads();

  for (int64_t b = blockIdx.x; b < a.n_parent; b += gridDim.x) {
    double accr[PER], acci[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) accr[r] = acci[r] = 0.0;
    const double pcx = a.parent_center[3 * b], pcy = a.parent_center[3 * b + 1], pcz = a.parent_center[3 * b + 2];
    const bool pfin = isfinite(pcx) && isfinite(pcy) && isfinite(pcz);
    const int64_t s0 = a.box_start[b], s1 = a.box_start[b + 1];
    unsigned skipped = 0;
    for (int64_t s = s0 + w; s < s1; s += NW) {  // uniform per wavefront
      const int64_t c = a.perm ? (int64_t)a.perm[s] : s;
      const double ccx = a.child_center[3 * c], ccy = a.child_center[3 * c + 1], ccz = a.child_center[3 * c + 2];
      if (!(pfin && isfinite(ccx) && isfinite(ccy) && isfinite(ccz))) {
        ++skipped;
        continue;
      }
      // shift d: FMM c_p - c_c, MOMENT c_c - c_p
      const double sg = moment ? 1.0 : -1.0;
      const double dx = sg * (ccx - pcx), dy = sg * (ccy - pcy), dz = sg * (ccz - pcz);
      const double* in = a.child + (size_t)c * (size_t)ncoef * 2;
      wave_sync();  // this wavefront's reads of the previous child are done
      // the child's expansion, all orders: A^{-m} = (-1)^m conj(A^m)
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        const int code = acode[i];
        if (code >= 0) {
          const int g = code & (kNeg - 1);
          double re = in[2 * g], im = in[2 * g + 1];
          if (code & kNeg) {
            im = -im;
            if (code & kOdd) {
              re = -re;
              im = -im;
            }
          }
          A[lane + 64 * i] = make_double2(re, im);
        }
      }
      // G_j^q (q >= 0) of the shift at R[j^2 + j + q], degree by degree
      const double xr = 0.5 * dx, xi = 0.5 * dy;  // xi = (d_x + i d_y)/2, eta = conj(xi)
      if (lane == 0) R[0] = make_double2(1.0, 0.0);
      for (int j = 1; j <= p; ++j) {
        wave_sync();
        const int q = lane;
        const int b0 = (j - 1) * (j - 1) + (j - 1);
        double vr = 0.0, vi = 0.0;
        if (q <= j) {
          auto F = [&](int k) -> double2 { return (k >= 0 && k <= j - 1) ? R[b0 + k] : make_double2(0.0, 0.0); };
          const double2 f1 = F(q + 1), f0 = F(q);
          if (q == 0) {  // 2 Re(eta F^1) - z F^0
            vr = 2.0 * (xr * f1.x + xi * f1.y) - dz * f0.x;
          } else {  // -xi F^{q-1} + eta F^{q+1} - z F^q
            const double2 fm = F(q - 1);
            vr = -(xr * fm.x - xi * fm.y) + (xr * f1.x + xi * f1.y) - dz * f0.x;
            vi = -(xr * fm.y + xi * fm.x) + (xr * f1.y - xi * f1.x) - dz * f0.y;
          }
        }
        wave_sync();
        if (q <= j) R[j * j + j + q] = make_double2(vr, vi);
      }
      wave_sync();
      // R_j^q = (-i)^q G_j^q / j!  (q >= 0, in place; one lane per entry)
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        if (rjq[i] < 0) continue;
        const int j = rjq[i] >> 8, q = rjq[i] & 255;
        const double2 g = R[j * j + j + q];
        const double invf = s_invf[j];
        const double gr = g.x * invf, gi = g.y * invf;
        double rr, ri;
        switch (q & 3) {
          case 0: rr = gr; ri = gi; break;
          case 1: rr = gi; ri = -gr; break;
          case 2: rr = -gr; ri = -gi; break;
          default: rr = -gi; ri = gr; break;
        }
        R[j * j + j + q] = make_double2(rr, ri);
      }
      wave_sync();
      // q < 0: R^{-q} = (-1)^q conj(R^q)
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        if (rjq[i] < 0) continue;
        const int j = rjq[i] >> 8, q = rjq[i] & 255;
        if (q == 0) continue;
        const double2 v = R[j * j + j + q];
        const double sgn = (q & 1) ? -1.0 : 1.0;
        R[j * j + j - q] = make_double2(sgn * v.x, -sgn * v.y);
      }
      wave_sync();
      // out_n^m += sum_{k<=n} sum_l A_k^l R_{n-k}^{qq}, qq = l - m (FMM) or m - l
      // (MOMENT); instantiated per normalisation so that the step of qq is a
      // constant (immediate LDS offsets)
      auto macs = [&](auto MOMc) {
        constexpr bool MOM = decltype(MOMc)::value;
        constexpr int step = MOM ? -1 : 1;
#pragma unroll
        for (int r = 0; r < PER; ++r) {
          const int n = no[r], m = mo[r];
          if (n < 0 || n > p) continue;
          double sr[4] = {0.0, 0.0, 0.0, 0.0}, si[4] = {0.0, 0.0, 0.0, 0.0};
          auto mac = [&](int u, const double2 av, const double2 rv) {
            sr[u] = fma(av.x, rv.x, sr[u]);
            sr[u] = fma(-av.y, rv.y, sr[u]);
            si[u] = fma(av.x, rv.y, si[u]);
            si[u] = fma(av.y, rv.x, si[u]);
          };
          for (int k = 0; k <= n; ++k) {
            const int j = n - k;
            const int lo = max(-k, m - j), hi = min(k, m + j);
            const double2* pa = A + k * k + k + lo;
            const double2* pr = R + j * j + j + (MOM ? (m - lo) : (lo - m));
            int cnt = hi - lo + 1;
            if (cnt >= 4) {  // four independent chains; the next block's reads issued before this block's FMAs
              double2 a0 = pa[0], a1 = pa[1], a2 = pa[2], a3 = pa[3];
              double2 r0 = pr[0], r1 = pr[step], r2 = pr[2 * step], r3 = pr[3 * step];
              for (; cnt >= 8; cnt -= 4) {
                pa += 4;
                pr += 4 * step;
                const double2 b0 = pa[0], b1 = pa[1], b2 = pa[2], b3 = pa[3];
                const double2 t0 = pr[0], t1 = pr[step], t2 = pr[2 * step], t3 = pr[3 * step];
                mac(0, a0, r0);
                mac(1, a1, r1);
                mac(2, a2, r2);
                mac(3, a3, r3);
                a0 = b0; a1 = b1; a2 = b2; a3 = b3;
                r0 = t0; r1 = t1; r2 = t2; r3 = t3;
              }
              mac(0, a0, r0);
              mac(1, a1, r1);
              mac(2, a2, r2);
              mac(3, a3, r3);
              pa += 4;
              pr += 4 * step;
              cnt -= 4;
            }
            for (; cnt > 0; --cnt, ++pa, pr += step) mac(0, pa[0], pr[0]);
          }
          accr[r] += (sr[0] + sr[1]) + (sr[2] + sr[3]);
          acci[r] += (si[0] + si[1]) + (si[2] + si[3]);
        }
      };
      if (moment)
        macs(BoolC<true>{});
      else
        macs(BoolC<false>{});
    }
    if (lane == 0) s_skip[w] = skipped;
    __syncthreads();  // every wavefront is done with its A and R
    // partial sums of the wavefronts -> LDS (A region of wavefront w)
#pragma unroll
    for (int r = 0; r < PER; ++r) {
      const int o = out_index(r);
      if (o >= 0) sbuf[w][0][o] = make_double2(accr[r], acci[r]);
    }
    __syncthreads();
    // fixed-order sum over the wavefronts, write +m and -m = (-1)^m conj(+m)
    double* out = a.out + (size_t)b * (size_t)ncoef * 2;
    for (int o = threadIdx.x; o < ntri; o += 64 * NW) {
      const int n = tri_degree(o), m = o - tri(n);
      double vr = 0.0, vi = 0.0;
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) {
        vr += sbuf[ww][0][o].x;
        vi += sbuf[ww][0][o].y;
      }
      if (m == 0) vi = 0.0;
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
    if (threadIdx.x == 0) {
      unsigned sk = 0;
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) sk += s_skip[ww];
      if (sk) {
        atomicAdd(&a.status->n_skipped, (unsigned long long)sk);
        atomicOr(&a.status->flags, (uint32_t)Q2X_FLAG_NONFINITE);
      }
    }
    __syncthreads();  // before the next parent reuses the LDS
  }
}

template <int PP, int NWV>
hipError_t launch_m2m_nw(const M2MArgs& a, int64_t blocks, hipStream_t s) {
  hipLaunchKernelGGL((q2x_m2m_kernel<PP, NWV>), dim3((unsigned)blocks), dim3(64 * NWV), 0, s, a);
  return hipGetLastError();
}

// Wavefronts per parent: 4 up to P = 20 (2 above, for the LDS), and 8 up to
// P = 16 when the level has at most 512 parents -- there a parent's ~5-8
// children then run at once instead of two after another (measured at p = 16:
// 285 parents 55 -> 45 us, 61 parents 48 -> 32 us; with 1,373 parents the
// four-wavefront launch stays ahead, 109.5 against 112 us).
hipError_t launch_m2m(const M2MArgs& a, hipStream_t s) {
  int64_t blocks = a.n_parent;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  const bool few = a.n_parent <= 512;
  switch (bucket_order(a.p)) {
    case 4: return few ? launch_m2m_nw<4, 8>(a, blocks, s) : launch_m2m_nw<4, 4>(a, blocks, s);
    case 8: return few ? launch_m2m_nw<8, 8>(a, blocks, s) : launch_m2m_nw<8, 4>(a, blocks, s);
    case 12: return few ? launch_m2m_nw<12, 8>(a, blocks, s) : launch_m2m_nw<12, 4>(a, blocks, s);
    case 16: return few ? launch_m2m_nw<16, 8>(a, blocks, s) : launch_m2m_nw<16, 4>(a, blocks, s);
    case 20: return launch_m2m_nw<20, 4>(a, blocks, s);
    case 24: return launch_m2m_nw<24, 2>(a, blocks, s);
    case 28: return launch_m2m_nw<28, 2>(a, blocks, s);
    case 32: return launch_m2m_nw<32, 2>(a, blocks, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace q2x
