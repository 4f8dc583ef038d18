// q2x_tile.hpp -- the Q2X recursion + box reduction kernel (one wavefront per
// tile of 64 box-sorted elements, one lane per element).
//
// Per lane: FP64 geometry of its element relative to its box centre, then the
// m >= 0 ("tilde") recursions of Sec. 3.4, Eqs. (50)-(56), degree by degree,
// with the whole recursion state in VGPRs (template order P, fully unrolled).
// The recursion carries G_n = (n+k)! t~_n (k = nesting depth), which removes
// every division from Eqs. (50)-(55) and keeps the values O(1) at any order.
// The FP32 path runs it on Y = (x - c)/a_e, a_e the element's largest vertex
// distance from c, so nothing underflows whatever the element's size and
// position (degree n of the result scales as a_e^n); the FP64 path runs on
// x - c unscaled.
// An element kind has one output (single layer, double layer, segment, tet)
// or two (single and double layer of one triangle mesh from one recursion).
// Every degree's outputs go to an LDS stage (real and imaginary parts in
// separate rows), and the FP64 factors s_e a_e^n / (n+k)!
// (s_e = sigma_e J_e / 4pi) to a small table beside it.  When a group of
// outputs ("chunk", <= CMAX coefficients) is complete the wavefront transposes
// through LDS -- lane = coefficient -- and walks the 64 elements in order, one
// box segment at a time, summing factor * value in FP64.  Boxes wholly inside
// the tile are finalised and stored directly; a box cut by a tile edge leaves
// a raw partial sum for the fix-up kernel.  The order of every sum is fixed by
// the element order, so results are bitwise reproducible.
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

template <typename T, int P1>
struct CArr {
  T r[P1];
  T i[P1];
};

// Cross product with every product rounded on its own (no FMA contraction),
// so that u x u is exactly zero and a repeated vertex gives J = 0.
__device__ __forceinline__ void cross_nofma(double ux, double uy, double uz, double vx, double vy, double vz,
                                            double& cx, double& cy, double& cz) {
#pragma clang fp contract(off)
  cx = uy * vz - uz * vy;
  cy = uz * vx - ux * vz;
  cz = ux * vy - uy * vx;
}

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// One application of the ladder operator of Sec. 3.4, Eqs. (50)-(51) (tilde
// form), producing degree N (orders 0..N) from degree N-1 (orders 0..N-1):
//   out^0 = 2 Re(eta F^1) - z F^0 + add^0
//   out^m = -xi F^{m-1} + eta F^{m+1} - z F^m + add^m,   m >= 1,
// with xi = (Y_x + i Y_y)/2 = xr + i xi, eta = conj(xi), z = Y_z and F^k = 0
// for k > N-1.  The recursions of Eqs. (50)-(55) divide this by (n+k) at the
// k-th nesting level; the kernel carries G_n = (n+k)! F_n instead, for which
// the division disappears (G_n = D G_{n-1} + G^{(k-1)}_n, every start value 1),
// and folds 1/(n+k)! into the FP64 per-degree factor.  Every real output is a
// chain of FMAs (5 for an interior order with a source term).
// (xr2, xi2) = 2 (xr, xi).
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
  static_for<1, N + 1>([&](auto MM) {
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

// Greedy grouping of the staged outputs into chunks of at most CMAX
// coefficients.  The unit of grouping is one output of one degree (n + 1
// coefficients): unit u = NOUT n + s holds degree n, slot s, in the order the
// recursion produces them, so a chunk may end between the outputs of a degree.
template <int P, int CMAX, int NOUT>
struct ChunkPlan {
  static constexpr int U = NOUT * (P + 1);  // number of units
  static constexpr int level(int u) { return u / NOUT; }
  static constexpr int size(int u) { return u / NOUT + 1; }
  static constexpr int off(int u) { return NOUT * tri(u / NOUT) + (u % NOUT) * (u / NOUT + 1); }
  static constexpr int first_unit(int u) {
    int s = 0;
    for (int l = 0; l <= u; ++l)
      if (off(l + 1) - off(s) > CMAX) s = l;
    return s;
  }
  static constexpr bool is_end(int u) { return u == U - 1 || first_unit(u + 1) == u + 1; }
  static constexpr int end_of(int u) {
    int e = u;
    while (!is_end(e)) ++e;
    return e;
  }
  static constexpr int max_units() {
    int mx = 0;
    for (int u = 0; u < U; ++u) {
      const int d = u - first_unit(u) + 1;
      if (d > mx) mx = d;
    }
    return mx;
  }
};

// The recursion chain of each element kind (Sec. 3.4): array k of the chain is
// laddered about vertex vert(k) and fed by array k-1.  Output o of degree n is
// the chain's last array (double layer: D_nu of it one degree lower, Eq. (56));
// it scales as a^(n - shift(o)), carries G / (n + depth(o))! and is staged in
// slot slot(o) of its degree (the order the recursion produces the outputs).
template <int KIND>
struct KindInfo;
template <>
struct KindInfo<Q2X_TRI_SINGLE> {  // q at x2, j along x3->x2, i from x1 (Eqs. (50)-(53))
  static constexpr int nv = 3, nch = 3, nout = 1;
  static constexpr int vert(int k) { return k == 0 ? 1 : (k == 1 ? 2 : 0); }
  static constexpr bool dbl(int) { return false; }
  static constexpr int shift(int) { return 0; }
  static constexpr int depth(int) { return 2; }
  static constexpr int slot(int) { return 0; }
};
template <>
struct KindInfo<Q2X_TRI_DOUBLE> {  // the same chain; output Eq. (56)
  static constexpr int nv = 3, nch = 3, nout = 1;
  static constexpr int vert(int k) { return k == 0 ? 1 : (k == 1 ? 2 : 0); }
  static constexpr bool dbl(int) { return true; }
  static constexpr int shift(int) { return 1; }
  static constexpr int depth(int) { return 1; }
  static constexpr int slot(int) { return 0; }
};
template <>
struct KindInfo<Q2X_SEGMENT> {  // q at x2, p from x1 (Eqs. (50)-(51))
  static constexpr int nv = 2, nch = 2, nout = 1;
  static constexpr int vert(int k) { return k == 0 ? 1 : 0; }
  static constexpr bool dbl(int) { return false; }
  static constexpr int shift(int) { return 0; }
  static constexpr int depth(int) { return 1; }
  static constexpr int slot(int) { return 0; }
};
template <>
struct KindInfo<Q2X_TET> {  // q at x2, j along x3->x2, b from x4, a from x1 (Eqs. (54)-(55))
  static constexpr int nv = 4, nch = 4, nout = 1;
  static constexpr int vert(int k) { return k == 0 ? 1 : (k == 1 ? 2 : (k == 2 ? 3 : 0)); }
  static constexpr bool dbl(int) { return false; }
  static constexpr int shift(int) { return 0; }
  static constexpr int depth(int) { return 3; }
  static constexpr int slot(int) { return 0; }
};
template <>
struct KindInfo<Q2X_TRI_BOTH> {  // output 0 single layer, output 1 double layer, one chain
  static constexpr int nv = 3, nch = 3, nout = 2;
  static constexpr int vert(int k) { return k == 0 ? 1 : (k == 1 ? 2 : 0); }
  static constexpr bool dbl(int o) { return o == 1; }
  static constexpr int shift(int o) { return o == 1 ? 1 : 0; }
  static constexpr int depth(int o) { return o == 1 ? 1 : 2; }
  static constexpr int slot(int o) { return o == 1 ? 0 : 1; }  // l~_n (from degree n-1) before i~_n
};

template <typename T>
struct PrecInfo;
template <>
struct PrecInfo<float> {
  static constexpr bool scaled = true;  // FP32 recursion on (y - c)/a_e
  // 31 coefficients per chunk keep the stage + factor table within 20 KB, so
  // two wavefronts fit per SIMD (160 KB LDS per CU)
  static constexpr int cmax = 31;
};
template <>
struct PrecInfo<double> {
  static constexpr bool scaled = false;  // plain FP64 recursion on y - c
  static constexpr int cmax = 32;
};

constexpr double inv_fact(int k) { return k <= 1 ? 1.0 : (k == 2 ? 0.5 : (k == 3 ? 1.0 / 6.0 : 1.0 / 24.0)); }

template <int P, int KIND, typename T>
__global__ __launch_bounds__(kTile) void q2x_tile_kernel(TileArgs a, int64_t n_tiles) {
  using KI = KindInfo<KIND>;
  constexpr int P1 = P + 1;
  constexpr int NV = KI::nv;
  constexpr int NCH = KI::nch;
  constexpr int NOUT = KI::nout;
  constexpr int CMAX = (PrecInfo<T>::cmax > P + 1) ? PrecInfo<T>::cmax : P + 1;
  constexpr int SSTR = kTile + 1;  // padded row stride (elements) of the stage and factor tables
  constexpr int NCT = tri(P + 1);
  constexpr bool SCALED = PrecInfo<T>::scaled;
  using Plan = ChunkPlan<P, CMAX, NOUT>;
  constexpr int DMAX = Plan::max_units();

  // stage: real part of chunk coefficient c in row c, imaginary part in row CMAX + c
  __shared__ T stage[2 * CMAX * SSTR];
  __shared__ double fac[DMAX * SSTR];         // row u - U0 (unit u of a chunk starting at unit U0)
  __shared__ int tkey[kTile];                 // box id of every element of the tile

  const int64_t tile = xcd_tile(blockIdx.x, n_tiles);
  const int lane = threadIdx.x;
  const int64_t q0 = tile * kTile;
  const int64_t pos_end = a.n_pos;
  if (q0 >= pos_end) return;  // uniform (never taken with the host's grid)
  const int ne = (int)min<int64_t>(kTile, pos_end - q0);
  const int64_t q = q0 + lane;
  const bool in_range = lane < ne;

  // ---- element, box and FP64 geometry (Sec. 3.1, Eqs. (8)-(9); Sec. 3.3, Eq. (21))
  const int key = in_range ? a.keys[q] : INT32_MIN;
  const bool box_ok = in_range && key >= 0 && key < a.n_boxes;  // (bad ids were counted by the bucketing)
  const int64_t e = in_range ? (a.perm ? (int64_t)a.perm[q] : q) : 0;
  uint32_t flag = 0;
  bool ok = box_ok;
  double xv[NV][3];
#pragma unroll
  for (int k = 0; k < NV; ++k) xv[k][0] = xv[k][1] = xv[k][2] = 0.0;
  double sigma[NOUT];
#pragma unroll
  for (int o = 0; o < NOUT; ++o) sigma[o] = 0.0;
  double cx = 0.0, cy = 0.0, cz = 0.0;
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
    sigma[0] = a.density[e];
    if constexpr (NOUT == 2) sigma[1] = a.density2[e];
    cx = a.box_center[3 * (int64_t)key];
    cy = a.box_center[3 * (int64_t)key + 1];
    cz = a.box_center[3 * (int64_t)key + 2];
  }
  if (ok) {
    bool fin = isfinite(cx) && isfinite(cy) && isfinite(cz);
#pragma unroll
    for (int o = 0; o < NOUT; ++o) fin = fin && isfinite(sigma[o]);
#pragma unroll
    for (int k = 0; k < NV; ++k) fin = fin && isfinite(xv[k][0]) && isfinite(xv[k][1]) && isfinite(xv[k][2]);
    if (!fin) {
      ok = false;
      flag |= Q2X_FLAG_NONFINITE;
    }
  }
  // Jacobian (Eq. (9)) and unit normal from the absolute vertices
  double J = 0.0, nx = 0.0, ny = 0.0, nz = 0.0;
  if (ok) {
    const double ux = xv[1][0] - xv[0][0], uy = xv[1][1] - xv[0][1], uz = xv[1][2] - xv[0][2];
    if constexpr (KIND == Q2X_SEGMENT) {
      J = sqrt(ux * ux + uy * uy + uz * uz);
    } else {
      const double vx = xv[2][0] - xv[0][0], vy = xv[2][1] - xv[0][1], vz = xv[2][2] - xv[0][2];
      double crx, cry, crz;
      cross_nofma(ux, uy, uz, vx, vy, vz, crx, cry, crz);
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
  }
  const bool degenerate = ok && !(J > 0.0);

  // element scale a_e (FP32 path) and the recursion's vertex data
  double X[NV][3];
  double amax2 = 0.0;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    X[k][0] = ok ? xv[k][0] - cx : 0.0;
    X[k][1] = ok ? xv[k][1] - cy : 0.0;
    X[k][2] = ok ? xv[k][2] - cz : 0.0;
    amax2 = fmax(amax2, X[k][0] * X[k][0] + X[k][1] * X[k][1] + X[k][2] * X[k][2]);
  }
  double scl = 1.0;
  if constexpr (SCALED) {
    scl = sqrt(amax2);
    if (!(scl > 0.0)) scl = 1.0;
  }
  const double inv_scl = 1.0 / scl;
  T vxr[NV], vxi[NV], vz[NV], vxr2[NV], vxi2[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    vxr[k] = (T)(0.5 * X[k][0] * inv_scl);
    vxi[k] = (T)(0.5 * X[k][1] * inv_scl);
    vz[k] = (T)(X[k][2] * inv_scl);
    vxr2[k] = (T)(X[k][0] * inv_scl);
    vxi2[k] = (T)(X[k][1] * inv_scl);
  }
  // running FP64 factors s_e a_e^(n - shift) / (n + depth)! of the degree being
  // produced; s_e = sigma_e J / (4 pi) (Sec. 3.2, Eq. (20)), 0 for skipped elements
  double fpow[NOUT];
  static_for<0, NOUT>([&](auto OO) {
    constexpr int o = decltype(OO)::value;
    const double w64 = ok ? sigma[o] * J * kInv4Pi : 0.0;
    fpow[o] = ((KI::shift(o) == 1) ? w64 * inv_scl : w64) * inv_fact(KI::depth(o));
  });

  // ---- box start table: box_start[b] = first position whose key >= b, keys
  // outside [0, B) counting as -1 / B (the fix-up kernel reads it)
  const int key_prev = (in_range && q > 0) ? a.keys[q - 1] : INT32_MIN;
  if (in_range) {
    const int64_t nb = a.n_boxes;
    const int64_t kc = key < 0 ? -1 : (key >= nb ? nb : key);
    const int64_t kp = (q == 0 || key_prev < 0) ? -1 : (key_prev >= nb ? nb : key_prev);
    if (kp > kc) flag |= Q2X_FLAG_NOT_SORTED;
    for (int64_t b = kp + 1; b <= kc; ++b) a.box_start[b] = (int32_t)q;
    if (q == pos_end - 1)
      for (int64_t b = kc + 1; b <= nb; ++b) a.box_start[b] = (int32_t)pos_end;
  }

  // ---- status (one atomic per wavefront and counter)
  {
    const uint64_t deg_mask = __ballot(degenerate);
    const uint64_t skip_mask = __ballot(box_ok && !ok);
    uint32_t fall = 0;
#pragma unroll
    for (int b = 0; b < 5; ++b)
      if (__ballot((flag >> b) & 1u)) fall |= (1u << b);
    if (lane == 0) {
      if (deg_mask) atomicAdd(&a.status->n_degenerate, (unsigned long long)__popcll(deg_mask));
      if (skip_mask) atomicAdd(&a.status->n_skipped, (unsigned long long)__popcll(skip_mask));
      if (fall) atomicOr(&a.status->flags, fall);
    }
  }

  // ---- box boundaries inside the tile (uniform bit mask), open tile edges
  const uint64_t bnd = __ballot(in_range && (lane == 0 || key != key_prev));
  tkey[lane] = key;  // read after the barrier that opens every chunk reduction
  bool head_open = false, tail_open = false;
  if (q0 > 0) head_open = (a.keys[q0 - 1] == a.keys[q0]);
  if (ne == kTile && q0 + kTile < pos_end) tail_open = (a.keys[q0 + kTile] == a.keys[q0 + kTile - 1]);
  const int p = a.p;
  const int ncoef_out = (p + 1) * (p + 1);

  // ---- reduction of one chunk of units [U0, U1]
  // lane = (group g, coefficient c): with CMAX <= 32 the two half-waves walk
  // elements [0,32) and [32,64) of the same coefficient (G = 2), otherwise one
  // lane walks all 64 (G = 1).  Within a group every box segment is summed in
  // element order and flushed where it ends; the one segment that may straddle
  // the halves is summed by both and joined (tail of half 0 + head of half 1).
  auto flush = [&](int sa, int sb, double accr, double acci, bool wr, int n, int m, double* out, int g_coef) {
    const int box = tkey[sa];  // (an LDS table: flushes run in lane-divergent code)
    if (!(wr && box >= 0 && box < a.n_boxes)) return;
    const bool open = (sa == 0 && head_open) || (sb == kTile && tail_open);
    if (open) {
      const int slot = (sa == 0) ? 0 : 1;
      double* pp = a.partials + ((tile * 2 + slot) * (int64_t)(NOUT * NCT) + g_coef) * 2;
      pp[0] = accr;
      pp[1] = acci;
    } else {
      finalize_store(out + (int64_t)box * ncoef_out * 2, n, m, accr, acci, a.norm, a.accumulate);
    }
  };
  auto reduce_chunk = [&](auto U0c, auto U1c) {
    constexpr int U0 = decltype(U0c)::value;
    constexpr int U1 = decltype(U1c)::value;
    constexpr int C = Plan::off(U1 + 1) - Plan::off(U0);
    static_assert(C <= CMAX && U1 - U0 + 1 <= DMAX, "chunk too large");
    constexpr int G = (CMAX <= 32) ? 2 : 1;
    constexpr int E = kTile / G;
    __syncthreads();
    const int g = (G == 2) ? (lane >> 5) : 0;
    const int c = (G == 2) ? (lane & 31) : lane;
    const bool act = c < C;
    const int cc = act ? c : 0;
    // decode chunk coefficient cc -> unit u (degree n, output o), order m
    int u = U0, r = cc;
    static_for<U0, U1>([&](auto UU) {
      constexpr int l = decltype(UU)::value;
      if (u == l && r >= Plan::size(l)) {
        r -= Plan::size(l);
        u = l + 1;
      }
    });
    const int n = u / NOUT;
    const int o = (NOUT == 1) ? 0 : ((u % NOUT) == KI::slot(0) ? 0 : 1);
    const int m = r;
    const bool wr = act && n <= p;
    double* out = (o == 0) ? a.coeffs : a.coeffs2;
    const int g_coef = o * NCT + tri(n) + m;
    const T* rre = stage + cc * SSTR;
    const T* rim = stage + (CMAX + cc) * SSTR;
    const double* frow = fac + (u - U0) * SSTR;
    const int gs = g * E;
    const int ge = min(gs + E, ne);
    const bool cont_in = (g > 0) && (gs < ne) && !((bnd >> gs) & 1ull);
    double accr = 0.0, acci = 0.0, hr = 0.0, hi = 0.0;
    int seg = gs, head_end = ge;
    bool in_head = cont_in;
    // Walk i = 0..E-1 (element gs + i) in pieces cut at every boundary of
    // either half, so that each piece is a tight loop with uniform control;
    // at a cut only the half whose box changes there closes its segment.
    // Elements past ne carry weight 0 and add exact zeros.
    const uint64_t mybits = (G == 2) ? (bnd >> gs) : bnd;  // this half's boundaries at i
    const uint64_t cuts = ((G == 2) ? ((bnd | (bnd >> 32)) & 0xffffffffull) : bnd) & ~1ull;
    const T* pre = rre + gs;
    const T* pim = rim + gs;
    const double* pf = frow + gs;
    int i0 = 0;
    while (i0 < E) {  // uniform
      const uint64_t nxt = (i0 + 1 < 64) ? (cuts >> (i0 + 1)) : 0ull;
      const int i1 = nxt ? i0 + 1 + __builtin_ctzll(nxt) : E;
#pragma unroll 4
      for (int i = i0; i < i1; ++i) {
        const double f = pf[i];
        accr = __builtin_fma((double)pre[i], f, accr);
        acci = __builtin_fma((double)pim[i], f, acci);
      }
      if (i1 < E && ((mybits >> i1) & 1ull)) {  // this half's segment ends at gs + i1
        const int el = gs + i1;
        if (in_head) {  // the continued segment ends inside this half: keep it for the join
          hr = accr;
          hi = acci;
          head_end = el;
          in_head = false;
        } else {
          flush(seg, el, accr, acci, wr, n, m, out, g_coef);
        }
        accr = 0.0;
        acci = 0.0;
        seg = el;
      }
      i0 = i1;
    }
    // last segment of the half: flushed here unless it is joined with the other half
    const bool cont_out = (G == 2) && (g == 0) && (ge == E) && (E < ne) && !((bnd >> E) & 1ull);
    if (gs < ne) {
      if (in_head) {  // continued segment covers the rest of half 1
        hr = accr;
        hi = acci;
        head_end = ge;
      } else if (!cont_out) {
        flush(seg, ge, accr, acci, wr, n, m, out, g_coef);
      }
    }
    if constexpr (G == 2) {
      // join: half 0's open tail + half 1's head (lane c+32 -> lane c)
      const double jr = __shfl(hr, lane + 32);
      const double ji = __shfl(hi, lane + 32);
      const int jend = __shfl(head_end, lane + 32);
      if (cont_out) flush(seg, jend, accr + jr, acci + ji, wr, n, m, out, g_coef);
    }
    __syncthreads();
  };

  // output o of degree N: stage it and its FP64 factors; reduce at chunk ends
  // (and after the last output of the requested order when that falls inside
  // a chunk)
  auto emit = [&](auto NNc, auto OO, const CArr<T, P1>& V) {
    constexpr int N = decltype(NNc)::value;
    constexpr int o = decltype(OO)::value;
    constexpr int u = NOUT * N + KI::slot(o);
    constexpr int U0 = Plan::first_unit(u);
    constexpr int row0 = Plan::off(u) - Plan::off(U0);
    static_for<0, N + 1>([&](auto MM) {
      constexpr int m = decltype(MM)::value;
      stage[(row0 + m) * SSTR + lane] = V.r[m];
      stage[(CMAX + row0 + m) * SSTR + lane] = V.i[m];
    });
    fac[(u - U0) * SSTR + lane] = fpow[o];
    constexpr double inv_next = 1.0 / (double)(N + 1 + KI::depth(o));
    fpow[o] = fpow[o] * scl * inv_next;
    if constexpr (Plan::is_end(u)) {
      reduce_chunk(IC<U0>{}, IC<u>{});
    } else if (KI::slot(o) == NOUT - 1 && N == p) {
      reduce_chunk(IC<U0>{}, IC<Plan::end_of(u)>{});
    }
  };

  // one degree of every array of the chain: nS (degree N) from S (degree N-1)
  auto advance = [&](auto NNc, CArr<T, P1>(&nS)[NCH], const CArr<T, P1>(&S)[NCH]) {
    constexpr int N = decltype(NNc)::value;
    static_for<0, NCH>([&](auto KK) {
      constexpr int k = decltype(KK)::value;
      constexpr int v = KI::vert(k);
      if constexpr (k == 0)
        ladder<N, false>(nS[0], S[0], S[0], vxr[v], vxi[v], vz[v], vxr2[v], vxi2[v]);
      else
        ladder<N, true>(nS[k], S[k], nS[k - 1], vxr[v], vxi[v], vz[v], vxr2[v], vxi2[v]);
    });
  };

  // ---- recursion over degrees (Sec. 3.4).  Nested rather than sequential, so
  // that skipping the degrees above p merges no register state.
  CArr<T, P1> S0[NCH];
#pragma unroll
  for (int k = 0; k < NCH; ++k) {
    S0[k].r[0] = T(1);
    S0[k].i[0] = T(0);
  }
  constexpr bool HAS_DBL = KI::dbl(NOUT - 1);
  if constexpr (!HAS_DBL) {
    // S holds degree N; emit the chain's last array
    auto rec = [&](auto self, auto NNc, const CArr<T, P1>(&S)[NCH]) -> void {
      constexpr int N = decltype(NNc)::value;
      emit(IC<N>{}, IC<0>{}, S[NCH - 1]);
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
    // double layer (output NOUT-1): l~_N = D_nu i~_{N-1}, nu = (n_x + i n_y)/2
    // (Sec. 3.4, Eq. (56)); with two outputs the single layer (output 0) is i~_N.
    // S holds degree max(N-1, 0).
    constexpr int OD = NOUT - 1;
    const T hnx = (T)(0.5 * nx), hny = (T)(0.5 * ny), tnz = (T)nz, nx2 = (T)nx, ny2 = (T)ny;
    auto rec = [&](auto self, auto NNc, const CArr<T, P1>(&S)[NCH]) -> void {
      constexpr int N = decltype(NNc)::value;
      if constexpr (N == 0) {
        CArr<T, P1> Z;
        Z.r[0] = T(0);
        Z.i[0] = T(0);
        emit(IC<0>{}, IC<OD>{}, Z);
        if constexpr (NOUT == 2) emit(IC<0>{}, IC<0>{}, S[NCH - 1]);
        if (0 < p) self(self, IC<1>{}, S);
      } else {
        {
          CArr<T, P1> L;
          ladder<N, false>(L, S[NCH - 1], S[NCH - 1], hnx, hny, tnz, nx2, ny2);
          emit(IC<N>{}, IC<OD>{}, L);
        }
        if constexpr (NOUT == 2) {
          CArr<T, P1> nS[NCH];
          advance(IC<N>{}, nS, S);
          emit(IC<N>{}, IC<0>{}, nS[NCH - 1]);
          if constexpr (N < P) {
            if (N < p) self(self, IC<N + 1>{}, nS);
          }
        } else if constexpr (N < P) {
          if (N < p) {
            CArr<T, P1> nS[NCH];
            advance(IC<N>{}, nS, S);
            self(self, IC<N + 1>{}, nS);
          }
        }
      }
    };
    rec(rec, IC<0>{}, S0);
  }
}

}  // namespace q2x
