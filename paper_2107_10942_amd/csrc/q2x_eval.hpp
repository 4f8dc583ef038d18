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
// recursion of the tile kernel (two adjacent lanes per element, the real and
// the imaginary parts, state in VGPRs, Sec. 3.4, Eqs. (50)-(56)): with t_n^m = a_e^(n - shift) G_n^m / (n + depth)!,
//   int_e R_n^m = J (-1)^m i^m t_n^m,  int_e R_n^{-m} = J (-1)^m i^m conj(t_n^m)
// (Sec. 3.4, Eqs. (47),(49); symmetry Eq. (12)), so that each degree adds
//   J sum_{m>=0} (-i)^m (L_n^m t_n^m + [m > 0] L_n^{-m} conj(t_n^m))
// to the element's FP64 sum as soon as the recursion produces it.  No box
// reduction: every lane pair writes its own element.  The elements are visited in
// box order (when sorted) so that the lanes of a wavefront read few rows of L.
#pragma once

#include "q2x_tile.hpp"

namespace q2x {

// Lane pair (2e, 2e + 1) holds element e: the real lane's part f of t_n^m is
// Re t, the imaginary lane's Im t.  The product of one order,
//   c = L_n^m t + L_n^{-m} conj(t)   (m > 0;  m = 0: L_n^0 t, t real),
// is split between the pair: the real lane takes L_n^m (x + i y) with
// (x, y) = (Re t, Im t), the imaginary lane L_n^{-m} (x + i y) with
// (x, y) = (Re t, -Im t).  Each lane reads one complex entry of L per order,
// takes the other part of t from its neighbour (one lane swap), and the
// pair's two sums add up to the element's value.
typedef double GD2 __attribute__((ext_vector_type(2)));  // one complex entry of L (16-byte load)

template <int P, int KIND, typename T>
__global__ __launch_bounds__(kTile) void q2x_eval_kernel(EvalArgs a, int64_t n_tiles) {
  using KI = KindInfo<KIND>;
  static_assert(KI::nout == 1, "one output per element kind");
  constexpr int P1 = P + 1;
  constexpr int NV = KI::nv;
  constexpr int NCH = KI::nch;
  constexpr bool SCALED = PrecInfo<T>::scaled;
  constexpr int SHIFT = KI::shift(0), DEPTH = KI::depth(0);
  constexpr int TE = kTileElems;
  static_assert(2 * TE == kTile, "two lanes per element");

  const int64_t tile = xcd_tile(blockIdx.x, n_tiles);
  const int lane = threadIdx.x;
  const int el = lane >> 1;    // the lane's element in the tile
  const bool imag = lane & 1;  // the lane holds imaginary parts
  const bool lead = !imag;     // the lane that counts and writes the element
  const int64_t q0 = tile * TE;
  if (q0 >= a.n_pos) return;  // uniform (never taken with the host's grid)
  const int64_t q = q0 + el;
  const bool in_range = q < a.n_pos;
  const int key = in_range ? as_global(a.keys)[q] : INT32_MIN;
  const bool box_ok = in_range && key >= 0 && key < a.n_boxes;
  const int64_t e = in_range ? (a.perm ? (int64_t)as_global(a.perm)[q] : q) : 0;
  const ElemGeom<NV, T> gm =
      element_geometry<NV, T, SCALED>(a.verts, a.n_verts, a.elems, e, a.box_center, key, box_ok, nullptr, 0);
  const bool ok = gm.ok;
  {
    const uint64_t deg_mask = __ballot(lead && ok && !(gm.J > 0.0));
    const uint64_t skip_mask = __ballot(lead && box_ok && !ok);
    const uint64_t bad_mask = a.count_bad_ids ? __ballot(lead && in_range && !box_ok) : 0ull;
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
  LCoef<T> cv[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) cv[k] = ladder_coef(imag, gm.vxr[k], gm.vxi[k], gm.vz[k], gm.vxr2[k], gm.vxi2[k]);
  const int p = a.p;
  const int64_t ncoef = (int64_t)(p + 1) * (p + 1);
  // the lane's entries of the box's row of L: L_n^m (real lane) or L_n^{-m}
  // (imaginary lane) sits at centre_n + dm m, centre_n = 2 (n^2 + n)
  cgdouble* const Lrow = as_global(a.local) + (ok ? (int64_t)key : 0) * ncoef * 2;
  const int dm = imag ? -2 : 2;
  // FP64 weight of degree n: a_e^max(0, n - shift) / (n + depth)! (a_e = 1
  // unscaled; the double layer's degree 0, the only one with n < shift, is zero)
  double wpow = inv_factorial(DEPTH);
  double accr = 0.0, acci = 0.0;

  // degree N of the output (the lane's part V, its neighbour's parts G from
  // spread): its orders summed in FP64, then weighted once.  The loads are
  // exec-masked (pairs without a valid element read nothing).
  auto consume = [&](auto NNc, const CVec<T, P1>& V, const T(&G)[P1]) Q2X_INLINE {
    constexpr int N = decltype(NNc)::value;
    T X[P1], Y[P1];
    X[0] = V.v[0];  // Re t on the real lane, 0 (= Im t_n^0) on the imaginary one
    static_for<1, N + 1>([&](auto MM) Q2X_INLINE {
      constexpr int m = decltype(MM)::value;
      const T f = V.v[m], g = G[m];
      X[m] = imag ? g : f;
      Y[m] = imag ? -f : g;
    });
    if (ok) {
      double dr = 0.0, di = 0.0;
      static_for<0, N + 1>([&](auto MM) Q2X_INLINE {
        constexpr int m = decltype(MM)::value;
        const GD2 lv = *(const GD2 __attribute__((address_space(1)))*)(Lrow + 2 * (N * N + N) + dm * m);
        struct {
          double x, y;
        } l{lv.x, lv.y};
        const double x = (double)X[m];
        // (-i)^m (Re + i Im)(x + i y)
        if constexpr (m == 0) {
          dr = l.x * x;
          di = l.y * x;
        } else {
          const double y = (double)Y[m];
          if constexpr ((m & 3) == 0) {  // += (Re x - Im y) + i (Im x + Re y)
            dr = fmaT(l.x, x, fmaT(-l.y, y, dr));
            di = fmaT(l.y, x, fmaT(l.x, y, di));
          } else if constexpr ((m & 3) == 1) {  // += (Im x + Re y) - i (Re x - Im y)
            dr = fmaT(l.y, x, fmaT(l.x, y, dr));
            di = fmaT(-l.x, x, fmaT(l.y, y, di));
          } else if constexpr ((m & 3) == 2) {  // -= (Re x - Im y) + i (Im x + Re y)
            dr = fmaT(-l.x, x, fmaT(l.y, y, dr));
            di = fmaT(-l.y, x, fmaT(-l.x, y, di));
          } else {  // -= (Im x + Re y) - i (Re x - Im y)
            dr = fmaT(-l.y, x, fmaT(-l.x, y, dr));
            di = fmaT(l.x, x, fmaT(-l.y, y, di));
          }
        }
      });
      accr = fmaT(wpow, dr, accr);
      acci = fmaT(wpow, di, acci);
    }
    if constexpr (SCALED) {
      if constexpr (N + 1 - SHIFT > 0) wpow *= gm.scl;
    }
    constexpr double inv_next = 1.0 / (double)(N + 1 + DEPTH);
    wpow *= inv_next;
  };

  // one degree of every array of the chain: nS (degree N) from S (degree N-1).
  // LASTG: the neighbour's parts of the last array, already spread (USE_LAST).
  auto advance = [&](auto NNc, auto USE_LAST, CVec<T, P1>(&nS)[NCH], const CVec<T, P1>(&S)[NCH],
                     const T(&LASTG)[P1]) Q2X_INLINE {
    constexpr int N = decltype(NNc)::value;
    static_for<0, NCH>([&](auto KK) Q2X_INLINE {
      constexpr int k = decltype(KK)::value;
      constexpr int v = KI::vert(k);
      auto step = [&](const T(&G)[P1]) Q2X_INLINE {
        if constexpr (k == 0)
          ladder<N, false>(nS[0], S[0], G, S[0], cv[v]);
        else
          ladder<N, true>(nS[k], S[k], G, nS[k - 1], cv[v]);
      };
      if constexpr (decltype(USE_LAST)::value && k == NCH - 1) {
        step(LASTG);
      } else {
        T G[P1];
        spread<N>(S[k], G);
        step(G);
      }
    });
  };

  CVec<T, P1> S0[NCH];
#pragma unroll
  for (int k = 0; k < NCH; ++k) S0[k].v[0] = imag ? T(0) : T(1);
  if constexpr (!KI::dbl(0)) {
    // S holds degree N
    auto rec = [&](auto self, auto NNc, const CVec<T, P1>(&S)[NCH]) Q2X_INLINE -> void {
      constexpr int N = decltype(NNc)::value;
      T G[P1];  // the neighbour's parts of the last array (consumed, then the next ladder's)
      spread<N + 1>(S[NCH - 1], G);
      consume(IC<N>{}, S[NCH - 1], G);
      if constexpr (N < P) {
        if (N < p) {
          CVec<T, P1> nS[NCH];
          advance(IC<N + 1>{}, IC<1>{}, nS, S, G);
          self(self, IC<N + 1>{}, nS);
        }
      }
    };
    rec(rec, IC<0>{}, S0);
  } else {
    // double layer: l~_N = D_nu i~_{N-1} (Sec. 3.4, Eq. (56)); degree 0 is zero.  S holds degree N-1.
    const LCoef<T> cn = ladder_coef(imag, (T)(0.5 * gm.nx), (T)(0.5 * gm.ny), (T)gm.nz, (T)gm.nx, (T)gm.ny);
    auto rec = [&](auto self, auto NNc, const CVec<T, P1>(&S)[NCH]) Q2X_INLINE -> void {
      constexpr int N = decltype(NNc)::value;
      T G[P1];  // the neighbour's parts of the last array (degree N-1)
      spread<N>(S[NCH - 1], G);
      {
        CVec<T, P1> Lv;
        T GL[P1];
        ladder<N, false>(Lv, S[NCH - 1], G, S[NCH - 1], cn);
        spread<N + 1>(Lv, GL);
        consume(IC<N>{}, Lv, GL);
      }
      if constexpr (N < P) {
        if (N < p) {
          CVec<T, P1> nS[NCH];
          advance(IC<N>{}, IC<1>{}, nS, S, G);
          self(self, IC<N + 1>{}, nS);
        }
      }
    };
    // degree 0 contributes nothing; advance the weight past it
    wpow *= (SCALED && 1 - SHIFT > 0 ? gm.scl : 1.0) / (double)(1 + DEPTH);
    if (0 < p) rec(rec, IC<1>{}, S0);
  }

  // the element's value: the sum of the pair's parts (every lane takes part
  // in the exchange)
  accr += neighbour(accr);
  acci += neighbour(acci);
  if (in_range && lead) {
    double* o = a.out + 2 * e;  // 8-byte aligned
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
