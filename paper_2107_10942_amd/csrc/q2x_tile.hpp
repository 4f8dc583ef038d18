// q2x_tile.hpp -- the Q2X recursion + box reduction kernel (one wavefront per
// tile of 64 box-sorted elements, one lane per element).
//
// Per lane: FP64 geometry of its element relative to its box centre, then the
// m >= 0 ("tilde") recursions of Sec. 3.4, Eqs. (50)-(55), degree by degree,
// with the whole recursion state in VGPRs (template order P, fully unrolled).
// Every degree's weighted outputs s_e t~_n^m go to an LDS stage; when a group
// of degrees ("chunk", <= CMAX coefficients) is complete the wavefront
// transposes through LDS -- lane = coefficient -- and walks the 64 elements in
// order, summing in FP64 and flushing at every box boundary (boxes are
// contiguous because elements are sorted by box).  Boxes wholly inside the tile
// are finalised and stored directly; a box cut by a tile edge leaves a raw
// partial sum for the fix-up kernel.  The order of every sum is fixed by the
// element order, so results are bitwise reproducible.
#pragma once

#include "q2x_internal.hpp"

namespace q2x {

template <int N>
struct IC {
  static constexpr int value = N;
};

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(IC<B>{});
    static_for<B + 1, E>(f);
  }
}

template <typename T>
struct Cx2;
template <>
struct Cx2<float> {
  using type = float2;
};
template <>
struct Cx2<double> {
  using type = double2;
};

template <typename T, int P1>
struct CArr {
  T r[P1];
  T i[P1];
};

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// One application of the ladder operator of Sec. 3.4, Eqs. (50)-(51) (tilde
// form), producing degree N (orders 0..N) from degree N-1 (orders 0..N-1):
//   out^0 = [2 Re(eta F^1) - z F^0 + add^0] * inv
//   out^m = [-xi F^{m-1} + eta F^{m+1} - z F^m + add^m] * inv,   m >= 1,
// with xi = (Y_x + i Y_y)/2, eta = conj(xi), z = Y_z and F^k = 0 for k > N-1.
// The caller passes sxr = Re(xi)*inv, sxi = Im(xi)*inv, sz = z*inv.
template <int N, bool ADD, typename T, int P1>
__device__ __forceinline__ void ladder(CArr<T, P1>& out, const CArr<T, P1>& F, const CArr<T, P1>& add, T sxr,
                                       T sxi, T sz, T inv) {
  static_assert(N >= 1 && N < P1, "degree out of range");
  // m = 0
  {
    T v = -sz * F.r[0];
    if constexpr (N - 1 >= 1) {
      v = fmaT(sxr + sxr, F.r[1], v);
      v = fmaT(sxi + sxi, F.i[1], v);
    }
    if constexpr (ADD) v = fmaT(inv, add.r[0], v);
    out.r[0] = v;
    out.i[0] = T(0);
  }
  static_for<1, N + 1>([&](auto MM) {
    constexpr int m = decltype(MM)::value;
    // Am = F^{m-1}; Ap = F^{m+1} (if m+1 <= N-1); C = F^m (if m <= N-1)
    const T amr = F.r[m - 1];
    const T ami = (m - 1 == 0) ? T(0) : F.i[m - 1];
    T re, im;
    if constexpr (m + 1 <= N - 1) {
      const T apr = F.r[m + 1], api = F.i[m + 1];
      re = sxr * (apr - amr);
      re = fmaT(sxi, ami + api, re);
      im = sxr * (api - ami);
      im = fmaT(-sxi, amr + apr, im);
    } else {
      re = fmaT(-sxr, amr, sxi * ami);
      im = fmaT(-sxr, ami, -sxi * amr);
    }
    if constexpr (m <= N - 1) {
      re = fmaT(-sz, F.r[m], re);
      im = fmaT(-sz, F.i[m], im);
    }
    if constexpr (ADD) {
      re = fmaT(inv, add.r[m], re);
      im = fmaT(inv, add.i[m], im);
    }
    out.r[m] = re;
    out.i[m] = im;
  });
}

// Greedy grouping of degrees 0..P into chunks of at most CMAX tilde
// coefficients (degree n has n+1 of them).
template <int P, int CMAX>
struct ChunkPlan {
  static constexpr int first_level(int n) {
    int s = 0;
    for (int l = 0; l <= n; ++l)
      if (tri(l + 1) - tri(s) > CMAX) s = l;
    return s;
  }
  static constexpr bool is_end(int n) { return n == P || first_level(n + 1) == n + 1; }
  static constexpr int end_of(int n) {
    int e = n;
    while (!is_end(e)) ++e;
    return e;
  }
};

__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int KIND>
struct KindInfo;
template <>
struct KindInfo<Q2X_TRI_SINGLE> {
  static constexpr int nv = 3;
  static constexpr int rho_shift = 0;
};
template <>
struct KindInfo<Q2X_TRI_DOUBLE> {
  static constexpr int nv = 3;
  static constexpr int rho_shift = 1;
};
template <>
struct KindInfo<Q2X_SEGMENT> {
  static constexpr int nv = 2;
  static constexpr int rho_shift = 0;
};
template <>
struct KindInfo<Q2X_TET> {
  static constexpr int nv = 4;
  static constexpr int rho_shift = 0;
};

template <typename T>
struct PrecInfo;
template <>
struct PrecInfo<float> {
  static constexpr bool scaled = true;  // FP32 recursion on (y - c)/rho
  static constexpr int cmax = 64;
};
template <>
struct PrecInfo<double> {
  static constexpr bool scaled = false;  // plain FP64 recursion on y - c
  static constexpr int cmax = 32;
};

template <int P, int KIND, typename T>
__global__ __launch_bounds__(kTile) void q2x_tile_kernel(TileArgs a, int64_t n_tiles) {
  using C2 = typename Cx2<T>::type;
  constexpr int P1 = P + 1;
  constexpr int NV = KindInfo<KIND>::nv;
  constexpr int CMAX = (PrecInfo<T>::cmax > P + 1) ? PrecInfo<T>::cmax : P + 1;
  constexpr int SSTR = kTile + 1;  // padded stride of one coefficient row in the stage
  constexpr int NCT = tri(P + 1);
  constexpr bool SCALED = PrecInfo<T>::scaled;
  using Plan = ChunkPlan<P, CMAX>;

  __shared__ C2 stage[CMAX * SSTR];

  const int64_t tile = xcd_tile(blockIdx.x, n_tiles);
  const int lane = threadIdx.x;
  const int64_t q0 = tile * kTile;
  const int64_t pos_end = a.box_start[a.n_boxes];
  if (q0 >= pos_end) return;  // uniform
  const int ne = (int)min<int64_t>(kTile, pos_end - q0);
  const int64_t q = q0 + lane;
  const bool in_range = lane < ne;

  // ---- element, box and FP64 geometry (Sec. 3.1, Eqs. (8)-(9); Sec. 3.3, Eq. (21))
  int key = in_range ? a.keys[q] : INT32_MIN;
  const bool box_ok = in_range && key >= 0 && key < a.n_boxes;
  int64_t e = in_range ? (a.perm ? (int64_t)a.perm[q] : q) : 0;
  uint32_t flag = 0;
  bool ok = box_ok;
  double xv[NV][3];
  for (int k = 0; k < NV; ++k) xv[k][0] = xv[k][1] = xv[k][2] = 0.0;
  double sigma = 0.0, cx = 0.0, cy = 0.0, cz = 0.0, rho = 1.0;
  // (ids outside [0, B) were counted by the bucketing step)
  if (ok) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int32_t vi = a.elems[e * NV + k];
      if (vi < 0 || vi >= a.n_verts) {
        ok = false;
        flag |= Q2X_FLAG_BAD_VERTEX;
      } else {
        xv[k][0] = a.verts[3 * (int64_t)vi];
        xv[k][1] = a.verts[3 * (int64_t)vi + 1];
        xv[k][2] = a.verts[3 * (int64_t)vi + 2];
      }
    }
    sigma = a.density[e];
    cx = a.box_center[3 * (int64_t)key];
    cy = a.box_center[3 * (int64_t)key + 1];
    cz = a.box_center[3 * (int64_t)key + 2];
    if constexpr (SCALED) {
      rho = a.box_radius[key];
      if (!(rho > 0.0) || !isfinite(rho)) {
        ok = false;
        flag |= Q2X_FLAG_BAD_RADIUS;
      }
    }
  }
  // edge vectors from the absolute vertices; Jacobian (Eq. (9)) and normal
  double J = 0.0, nx = 0.0, ny = 0.0, nz = 0.0;
  if (ok) {
    bool fin = isfinite(sigma) && isfinite(cx) && isfinite(cy) && isfinite(cz);
#pragma unroll
    for (int k = 0; k < NV; ++k) fin = fin && isfinite(xv[k][0]) && isfinite(xv[k][1]) && isfinite(xv[k][2]);
    if (!fin) {
      ok = false;
      flag |= Q2X_FLAG_NONFINITE;
    }
  }
  bool degenerate = false;
  if (ok) {
    const double ux = xv[1][0] - xv[0][0], uy = xv[1][1] - xv[0][1], uz = xv[1][2] - xv[0][2];
    if constexpr (KIND == Q2X_SEGMENT) {
      J = sqrt(ux * ux + uy * uy + uz * uz);
    } else {
      const double vx = xv[2][0] - xv[0][0], vy = xv[2][1] - xv[0][1], vz = xv[2][2] - xv[0][2];
      const double crx = uy * vz - uz * vy, cry = uz * vx - ux * vz, crz = ux * vy - uy * vx;
      if constexpr (KIND == Q2X_TET) {
        const double wx = xv[3][0] - xv[0][0], wy = xv[3][1] - xv[0][1], wz = xv[3][2] - xv[0][2];
        J = fabs(crx * wx + cry * wy + crz * wz);
      } else {
        J = sqrt(crx * crx + cry * cry + crz * crz);
        if (J > 0.0) {
          nx = crx / J;
          ny = cry / J;
          nz = crz / J;
        }
      }
    }
    degenerate = !(J > 0.0);
  }
  if (!ok) {
    // skipped element: zero weight and zero (finite) geometry
    J = 0.0;
    nx = ny = nz = 0.0;
  }
  // weight s_e = sigma J / (4 pi) (Sec. 3.2, Eq. (20))
  const double w64 = ok ? sigma * J * kInv4Pi : 0.0;
  const T w = (T)w64;
  const double inv_rho = SCALED ? 1.0 / rho : 1.0;

  // scaled vertex coordinates Y_k = (x_k - c)/rho  ->  xi_k = (Y_x + i Y_y)/2, z_k = Y_z
  T vxr[NV], vxi[NV], vz[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const double X = ok ? (xv[k][0] - cx) * inv_rho : 0.0;
    const double Y = ok ? (xv[k][1] - cy) * inv_rho : 0.0;
    const double Z = ok ? (xv[k][2] - cz) * inv_rho : 0.0;
    vxr[k] = (T)(0.5 * X);
    vxi[k] = (T)(0.5 * Y);
    vz[k] = (T)Z;
  }

  // ---- status (one atomic per wavefront)
  {
    const uint64_t deg_mask = __ballot(degenerate);
    const uint64_t skip_mask = __ballot(box_ok && !ok);
    uint32_t f = flag;
    // OR-reduce the flags over the wave (few distinct bits: ballot each)
    uint32_t fall = 0;
#pragma unroll
    for (int b = 0; b < 5; ++b)
      if (__ballot((f >> b) & 1u)) fall |= (1u << b);
    if (lane == 0) {
      if (deg_mask) atomicAdd(&a.status->n_degenerate, (unsigned long long)__popcll(deg_mask));
      if (skip_mask) atomicAdd(&a.status->n_skipped, (unsigned long long)__popcll(skip_mask));
      if (fall) atomicOr(&a.status->flags, fall);
    }
  }

  // ---- box boundaries inside the tile (uniform bit mask), open tile edges
  const int key_prev = (in_range && lane > 0) ? a.keys[q - 1] : INT32_MIN;
  const uint64_t bnd = __ballot(in_range && (lane == 0 || key != key_prev));
  bool head_open = false, tail_open = false;
  if (q0 > 0) head_open = (a.keys[q0 - 1] == a.keys[q0]);
  if (ne == kTile && q0 + kTile < pos_end) tail_open = (a.keys[q0 + kTile] == a.keys[q0 + kTile - 1]);
  const int p = a.p;
  const int ncoef_out = (p + 1) * (p + 1);

  // ---- reduction of one chunk of degrees [L0, L1] (lane = coefficient)
  auto reduce_chunk = [&](auto L0c, auto L1c) {
    constexpr int L0 = decltype(L0c)::value;
    constexpr int L1 = decltype(L1c)::value;
    constexpr int CB = tri(L0);
    constexpr int C = tri(L1 + 1) - tri(L0);
    static_assert(C <= CMAX, "chunk too large");
    __syncthreads();
    const int c = lane;
    const bool act = c < C;
    int n = 0, m = 0;
    tri_nm(CB + c, n, m);
    const bool wr = act && n <= p;
    const int kpow = n - KindInfo<KIND>::rho_shift;
    double accr = 0.0, acci = 0.0;
    int seg_a = 0;
    auto flush = [&](int sa, int sb) {
      const int box = __builtin_amdgcn_readlane(key, sa);
      const double rb = SCALED ? readlane_d(rho, sa) : 1.0;
      if (box < 0 || box >= a.n_boxes) return;  // skipped (invalid) elements
      const bool open = (sa == 0 && head_open) || (sb == kTile && tail_open);
      if (!wr) return;
      if (open) {
        const int slot = (sa == 0) ? 0 : 1;
        double* pp = a.partials + ((tile * 2 + slot) * (int64_t)NCT + CB + c) * 2;
        pp[0] = accr;
        pp[1] = acci;
      } else {
        const double rk = SCALED ? ipow_d(rb, kpow) : 1.0;
        finalize_store(a.coeffs + (int64_t)box * ncoef_out * 2, n, m, accr, acci, rk, a.norm, a.accumulate);
      }
    };
    for (int el = 0; el < ne; ++el) {
      if (el > 0 && ((bnd >> el) & 1ull)) {
        flush(seg_a, el);
        accr = 0.0;
        acci = 0.0;
        seg_a = el;
      }
      if (act) {
        const C2 v = stage[c * SSTR + el];
        accr += (double)v.x;
        acci += (double)v.y;
      }
    }
    flush(seg_a, ne);
    __syncthreads();
  };

  auto put = [&](int idx, T re, T im) {
    C2 v;
    v.x = w * re;
    v.y = w * im;
    stage[idx * SSTR + lane] = v;
  };

  // ---- recursion over degrees (Sec. 3.4): outputs staged degree by degree
  if constexpr (KIND == Q2X_TRI_SINGLE || KIND == Q2X_TRI_DOUBLE) {
    CArr<T, P1> Q, Jj, I;
    Q.r[0] = T(1);
    Q.i[0] = T(0);
    Jj.r[0] = T(1);
    Jj.i[0] = T(0);
    I.r[0] = T(0.5);
    I.i[0] = T(0);
    const T hnx = (T)(0.5 * nx), hny = (T)(0.5 * ny), tnz = (T)nz;
    bool done = false;
    static_for<0, P + 1>([&](auto NN) {
      constexpr int N = decltype(NN)::value;
      constexpr int L0 = Plan::first_level(N);
      if (!done) {
        if (N > p) {
          done = true;
        } else {
          if constexpr (KIND == Q2X_TRI_SINGLE) {
            if constexpr (N >= 1) {
              CArr<T, P1> nQ, nJ, nI;
              constexpr T i1 = T(1) / T(N), i2 = T(1) / T(N + 1), i3 = T(1) / T(N + 2);
              ladder<N, false>(nQ, Q, Q, vxr[1] * i1, vxi[1] * i1, vz[1] * i1, i1);  // q at x2, Eq. (50)
              ladder<N, true>(nJ, Jj, nQ, vxr[2] * i2, vxi[2] * i2, vz[2] * i2, i2);  // j along x3->x2, Eq. (52)
              ladder<N, true>(nI, I, nJ, vxr[0] * i3, vxi[0] * i3, vz[0] * i3, i3);  // i from x1, Eq. (52)
              Q = nQ;
              Jj = nJ;
              I = nI;
            }
            static_for<0, N + 1>([&](auto MM) {
              constexpr int m = decltype(MM)::value;
              put(tri(N) - tri(L0) + m, I.r[m], I.i[m]);
            });
          } else {
            // double layer: l~_N = D_nu i~_{N-1}, nu = (n_x + i n_y)/2 (Sec. 3.4, Eq. (56))
            if constexpr (N == 0) {
              put(0, T(0), T(0));
            } else {
              CArr<T, P1> L;
              ladder<N, false>(L, I, I, hnx, hny, tnz, T(1));
              static_for<0, N + 1>([&](auto MM) {
                constexpr int m = decltype(MM)::value;
                put(tri(N) - tri(L0) + m, L.r[m], L.i[m]);
              });
              if constexpr (N < P) {
                if (N < p) {
                  CArr<T, P1> nQ, nJ, nI;
                  constexpr T i1 = T(1) / T(N), i2 = T(1) / T(N + 1), i3 = T(1) / T(N + 2);
                  ladder<N, false>(nQ, Q, Q, vxr[1] * i1, vxi[1] * i1, vz[1] * i1, i1);
                  ladder<N, true>(nJ, Jj, nQ, vxr[2] * i2, vxi[2] * i2, vz[2] * i2, i2);
                  ladder<N, true>(nI, I, nJ, vxr[0] * i3, vxi[0] * i3, vz[0] * i3, i3);
                  Q = nQ;
                  Jj = nJ;
                  I = nI;
                }
              }
            }
          }
          if constexpr (Plan::is_end(N)) {
            reduce_chunk(IC<L0>{}, IC<N>{});
          } else if (N == p) {
            reduce_chunk(IC<L0>{}, IC<Plan::end_of(N)>{});
          }
        }
      }
    });
  } else if constexpr (KIND == Q2X_SEGMENT) {
    CArr<T, P1> Q, Pp;
    Q.r[0] = T(1);
    Q.i[0] = T(0);
    Pp.r[0] = T(1);
    Pp.i[0] = T(0);
    bool done = false;
    static_for<0, P + 1>([&](auto NN) {
      constexpr int N = decltype(NN)::value;
      constexpr int L0 = Plan::first_level(N);
      if (!done) {
        if (N > p) {
          done = true;
        } else {
          if constexpr (N >= 1) {
            CArr<T, P1> nQ, nP;
            constexpr T i1 = T(1) / T(N), i2 = T(1) / T(N + 1);
            ladder<N, false>(nQ, Q, Q, vxr[1] * i1, vxi[1] * i1, vz[1] * i1, i1);  // q at x2, Eq. (50)
            ladder<N, true>(nP, Pp, nQ, vxr[0] * i2, vxi[0] * i2, vz[0] * i2, i2);  // p from x1, Eq. (50)
            Q = nQ;
            Pp = nP;
          }
          static_for<0, N + 1>([&](auto MM) {
            constexpr int m = decltype(MM)::value;
            put(tri(N) - tri(L0) + m, Pp.r[m], Pp.i[m]);
          });
          if constexpr (Plan::is_end(N)) {
            reduce_chunk(IC<L0>{}, IC<N>{});
          } else if (N == p) {
            reduce_chunk(IC<L0>{}, IC<Plan::end_of(N)>{});
          }
        }
      }
    });
  } else {  // Q2X_TET
    CArr<T, P1> Q, Jj, B, A;
    Q.r[0] = T(1);
    Q.i[0] = T(0);
    Jj.r[0] = T(1);
    Jj.i[0] = T(0);
    B.r[0] = T(0.5);
    B.i[0] = T(0);
    A.r[0] = T(1) / T(6);
    A.i[0] = T(0);
    bool done = false;
    static_for<0, P + 1>([&](auto NN) {
      constexpr int N = decltype(NN)::value;
      constexpr int L0 = Plan::first_level(N);
      if (!done) {
        if (N > p) {
          done = true;
        } else {
          if constexpr (N >= 1) {
            CArr<T, P1> nQ, nJ, nB, nA;
            constexpr T i1 = T(1) / T(N), i2 = T(1) / T(N + 1), i3 = T(1) / T(N + 2), i4 = T(1) / T(N + 3);
            ladder<N, false>(nQ, Q, Q, vxr[1] * i1, vxi[1] * i1, vz[1] * i1, i1);   // q at x2
            ladder<N, true>(nJ, Jj, nQ, vxr[2] * i2, vxi[2] * i2, vz[2] * i2, i2);  // j along x3->x2
            ladder<N, true>(nB, B, nJ, vxr[3] * i3, vxi[3] * i3, vz[3] * i3, i3);   // b from x4, Eq. (54)
            ladder<N, true>(nA, A, nB, vxr[0] * i4, vxi[0] * i4, vz[0] * i4, i4);   // a from x1, Eq. (54)
            Q = nQ;
            Jj = nJ;
            B = nB;
            A = nA;
          }
          static_for<0, N + 1>([&](auto MM) {
            constexpr int m = decltype(MM)::value;
            put(tri(N) - tri(L0) + m, A.r[m], A.i[m]);
          });
          if constexpr (Plan::is_end(N)) {
            reduce_chunk(IC<L0>{}, IC<N>{});
          } else if (N == p) {
            reduce_chunk(IC<L0>{}, IC<Plan::end_of(N)>{});
          }
        }
      }
    });
  }
}

}  // namespace q2x
