// q2x_eval.hpp -- the receiving side: integrals of a local expansion over
// elements (the evaluation stage of a Galerkin method, which uses the same
// integrals: Sec. 2 after Eq. (5), and the Conclusions, where the far field
// of a Galerkin FMM is a series in R_n^m to be integrated over the receiving
// triangles).
//
// For element e of box b with local coefficients L_b (a field
// sum_{n<=p, |m|<=n} L_{b,n}^m R_n^m(y - c_b)):
//   out_e = sum_{n,m} L_{b,n}^m int_e R_n^m(y - c_b) dmu(y)
// (double layer: int_e n . grad R_n^m dS).  The element integrals are the
// recursion of the tile kernel (lane = element, state in VGPRs, Sec. 3.4,
// Eqs. (50)-(56)): with t_n^m = a_e^(n - shift) G_n^m / (n + depth)!,
//   int_e R_n^m = J (-1)^m i^m t_n^m,  int_e R_n^{-m} = J (-1)^m i^m conj(t_n^m)
// (Sec. 3.4, Eqs. (47),(49); symmetry Eq. (12)), so that each degree adds
//   J sum_{m>=0} (-i)^m (L_n^m t_n^m + [m > 0] L_n^{-m} conj(t_n^m))
// to the element's FP64 sum as soon as the recursion produces it.  No box
// reduction: every lane writes its own element.  The elements are visited in
// box order (when sorted) so that the lanes of a wavefront read few rows of L.
#pragma once

#include "q2x_tile.hpp"

namespace q2x {

// Both parts of every order of one recursion array (one lane per element).
template <typename T, int P1>
struct CArr {
  T r[P1];
  T i[P1];
};

// One application of the ladder operator of Sec. 3.4, Eqs. (50)-(51) (tilde
// form), degree N from degree N-1, both parts in one lane (the recursion
// kernel's split form, ladder(), has the full statement):
//   out^0 = 2 Re(eta F^1) - z F^0 + add^0
//   out^m = -xi F^{m-1} + eta F^{m+1} - z F^m + add^m,   m >= 1,
// xi = xr + i xi, eta = conj(xi), z; (xr2, xi2) = 2 (xr, xi).
template <int N, bool ADD, typename T, int P1>
__device__ __forceinline__ void ladder(CArr<T, P1>& out, const CArr<T, P1>& F, const CArr<T, P1>& add, T xr, T xi,
                                       T z, T xr2, T xi2) {
  static_assert(N >= 1 && N < P1, "degree out of range");
  {
    T v = ADD ? fmaT(-z, F.r[0], add.r[0]) : -z * F.r[0];
    if constexpr (N - 1 >= 1) {
      v = fmaT(xr2, F.r[1], v);
      v = fmaT(xi2, F.i[1], v);
    }
    out.r[0] = v;
    out.i[0] = T(0);
  }
  static_for<1, N + 1>([&](auto MM) Q2X_INLINE {
    constexpr int m = decltype(MM)::value;
    const T amr = F.r[m - 1];
    // -xi F^{m-1}:  re -= xr Ar - xi Ai ;  im -= xr Ai + xi Ar
    T re = ADD ? fmaT(-xr, amr, add.r[m]) : -xr * amr;
    T im = ADD ? fmaT(-xi, amr, add.i[m]) : -xi * amr;
    if constexpr (m - 1 > 0) {
      const T ami = F.i[m - 1];
      re = fmaT(xi, ami, re);
      im = fmaT(-xr, ami, im);
    }
    // eta F^{m+1}:  re += xr Br + xi Bi ;  im += xr Bi - xi Br
    if constexpr (m + 1 <= N - 1) {
      const T apr = F.r[m + 1], api = F.i[m + 1];
      re = fmaT(xr, apr, re);
      re = fmaT(xi, api, re);
      im = fmaT(xr, api, im);
      im = fmaT(-xi, apr, im);
    }
    // -z F^m
    if constexpr (m <= N - 1) {
      re = fmaT(-z, F.r[m], re);
      im = fmaT(-z, F.i[m], im);
    }
    out.r[m] = re;
    out.i[m] = im;
  });
}

template <int P, int KIND, typename T>
__global__ __launch_bounds__(kTile) void q2x_eval_kernel(EvalArgs a, int64_t n_tiles) {
  using KI = KindInfo<KIND>;
  static_assert(KI::nout == 1, "one output per element kind");
  constexpr int P1 = P + 1;
  constexpr int NV = KI::nv;
  constexpr int NCH = KI::nch;
  constexpr bool SCALED = PrecInfo<T>::scaled;
  constexpr int SHIFT = KI::shift(0), DEPTH = KI::depth(0);

  const int64_t tile = xcd_tile(blockIdx.x, n_tiles);
  const int lane = threadIdx.x;
  const int64_t q0 = tile * kTile;
  if (q0 >= a.n_pos) return;  // uniform (never taken with the host's grid)
  const int64_t q = q0 + lane;
  const bool in_range = q < a.n_pos;
  const int key = in_range ? a.keys[q] : INT32_MIN;
  const bool box_ok = in_range && key >= 0 && key < a.n_boxes;
  const int64_t e = in_range ? (a.perm ? (int64_t)a.perm[q] : q) : 0;
  const ElemGeom<NV, T> gm =
      element_geometry<NV, T, SCALED>(a.verts, a.n_verts, a.elems, e, a.box_center, key, box_ok, nullptr, 0);
  const bool ok = gm.ok;
  {
    const uint64_t deg_mask = __ballot(ok && !(gm.J > 0.0));
    const uint64_t skip_mask = __ballot(box_ok && !ok);
    const uint64_t bad_mask = a.count_bad_ids ? __ballot(in_range && !box_ok) : 0ull;
    uint32_t fall = bad_mask ? (uint32_t)Q2X_FLAG_BAD_BOX : 0u;
#pragma unroll
    for (int b = 0; b < 5; ++b)
      if (__ballot((gm.flag >> b) & 1u)) fall |= (1u << b);
    if (lane == 0) {
      if (deg_mask) atomicAdd(&a.status->n_degenerate, (unsigned long long)__popcll(deg_mask));
      if (skip_mask | bad_mask)
        atomicAdd(&a.status->n_skipped, (unsigned long long)__popcll(skip_mask | bad_mask));
      if (fall) atomicOr(&a.status->flags, fall);
    }
  }
  const int p = a.p;
  const int64_t ncoef = (int64_t)(p + 1) * (p + 1);
  const double* Lrow = a.local + (ok ? (int64_t)key : 0) * ncoef * 2;
  // FP64 weight of degree n: a_e^max(0, n - shift) / (n + depth)! (a_e = 1
  // unscaled; the double layer's degree 0, the only one with n < shift, is zero)
  double wpow = inv_factorial(DEPTH);
  double accr = 0.0, acci = 0.0;

  // degree N of the output: add its terms (exec-masked loads: lanes without
  // a valid element read nothing)
  auto consume = [&](auto NNc, const CArr<T, P1>& V) Q2X_INLINE {
    constexpr int N = decltype(NNc)::value;
    if (ok) {
      static_for<0, N + 1>([&](auto MM) Q2X_INLINE {
        constexpr int m = decltype(MM)::value;
        const double tr = wpow * (double)V.r[m], ti = wpow * (double)V.i[m];
        const double* lp = Lrow + 2 * (N * N + N + m);
        double cr = lp[0] * tr - lp[1] * ti;
        double ci = lp[0] * ti + lp[1] * tr;
        if constexpr (m > 0) {
          const double* lm = Lrow + 2 * (N * N + N - m);
          cr += lm[0] * tr + lm[1] * ti;
          ci += lm[1] * tr - lm[0] * ti;
        }
        // (-i)^m
        if constexpr ((m & 3) == 0) {
          accr += cr;
          acci += ci;
        } else if constexpr ((m & 3) == 1) {
          accr += ci;
          acci -= cr;
        } else if constexpr ((m & 3) == 2) {
          accr -= cr;
          acci -= ci;
        } else {
          accr -= ci;
          acci += cr;
        }
      });
    }
    if constexpr (SCALED) {
      if constexpr (N + 1 - SHIFT > 0) wpow *= gm.scl;
    }
    constexpr double inv_next = 1.0 / (double)(N + 1 + DEPTH);
    wpow *= inv_next;
  };

  auto advance = [&](auto NNc, CArr<T, P1>(&nS)[NCH], const CArr<T, P1>(&S)[NCH]) Q2X_INLINE {
    constexpr int N = decltype(NNc)::value;
    static_for<0, NCH>([&](auto KK) Q2X_INLINE {
      constexpr int k = decltype(KK)::value;
      constexpr int v = KI::vert(k);
      if constexpr (k == 0)
        ladder<N, false>(nS[0], S[0], S[0], gm.vxr[v], gm.vxi[v], gm.vz[v], gm.vxr2[v], gm.vxi2[v]);
      else
        ladder<N, true>(nS[k], S[k], nS[k - 1], gm.vxr[v], gm.vxi[v], gm.vz[v], gm.vxr2[v], gm.vxi2[v]);
    });
  };

  CArr<T, P1> S0[NCH];
#pragma unroll
  for (int k = 0; k < NCH; ++k) {
    S0[k].r[0] = T(1);
    S0[k].i[0] = T(0);
  }
  if constexpr (!KI::dbl(0)) {
    // S holds degree N
    auto rec = [&](auto self, auto NNc, const CArr<T, P1>(&S)[NCH]) Q2X_INLINE -> void {
      constexpr int N = decltype(NNc)::value;
      consume(IC<N>{}, S[NCH - 1]);
      if constexpr (N < P) {
        if (N < p) {
          CArr<T, P1> nS[NCH];
          advance(IC<N + 1>{}, nS, S);
          self(self, IC<N + 1>{}, nS);
        }
      }
    };
    rec(rec, IC<0>{}, S0);
  } else {
    // double layer: l~_N = D_nu i~_{N-1} (Sec. 3.4, Eq. (56)); degree 0 is zero.  S holds degree N-1.
    const T hnx = (T)(0.5 * gm.nx), hny = (T)(0.5 * gm.ny), tnz = (T)gm.nz, nx2 = (T)gm.nx, ny2 = (T)gm.ny;
    auto rec = [&](auto self, auto NNc, const CArr<T, P1>(&S)[NCH]) Q2X_INLINE -> void {
      constexpr int N = decltype(NNc)::value;
      {
        CArr<T, P1> Lv;
        ladder<N, false>(Lv, S[NCH - 1], S[NCH - 1], hnx, hny, tnz, nx2, ny2);
        consume(IC<N>{}, Lv);
      }
      if constexpr (N < P) {
        if (N < p) {
          CArr<T, P1> nS[NCH];
          advance(IC<N>{}, nS, S);
          self(self, IC<N + 1>{}, nS);
        }
      }
    };
    // degree 0 contributes nothing; advance the weight past it
    wpow *= (SCALED && 1 - SHIFT > 0 ? gm.scl : 1.0) / (double)(1 + DEPTH);
    if (0 < p) rec(rec, IC<1>{}, S0);
  }

  if (in_range) {
    double* o = a.out + 2 * e;
    double vr = box_ok ? gm.J * accr : 0.0, vi = box_ok ? gm.J * acci : 0.0;
    if (a.accumulate) {
      vr += o[0];
      vi += o[1];
    }
    o[0] = vr;
    o[1] = vi;
  }
}

}  // namespace q2x
