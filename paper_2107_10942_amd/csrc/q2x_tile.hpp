// q2x_tile.hpp -- the Q2X recursion + box reduction kernel (one wavefront per
// tile of up to 32 box-sorted elements, two adjacent lanes per element).
//
// Per element: FP64 geometry relative to its box centre, then the m >= 0
// ("tilde") recursions of Sec. 3.4, Eqs. (50)-(56), degree by degree, with
// the whole recursion state in VGPRs (template order P, fully unrolled).
// Lane 2e holds the real parts of element e's orders, lane 2e + 1 the
// imaginary parts.  Each lane forms its own part of every new order from its
// own parts of the previous degree and its neighbour's (one DPP lane swap per
// order, read into a fresh register): six instructions per order instead of
// ten in one lane, so a wave's instruction stream is about 40% shorter than
// with one lane per element, for half as many elements.
// The recursion carries G_n = (n+k)! t~_n (k = nesting depth), which removes
// every division from Eqs. (50)-(55) and keeps the values O(1) at any order.
// The FP32 path runs it on Y = (x - c)/a_e, a_e the element's largest vertex
// distance from c, so nothing underflows whatever the element's size and
// position (degree n of the result scales as a_e^n); the FP64 path runs on
// x - c unscaled.
// An element kind has one output (single layer, double layer, segment, tet)
// or two (single and double layer of one triangle mesh from one recursion) or
// three (segments with a vector density).
// Every degree's outputs go to an LDS stage (real and imaginary parts in
// separate rows, each written by the lane that holds it), and the FP64
// factors s_e a_e^n / (n+k)! (s_e = sigma_e J_e / 4pi) to a small table
// beside it.  When a group of outputs ("chunk", <= CMAX coefficients) is
// complete the wavefront transposes through LDS -- lane = coefficient -- and
// walks the tile's elements in order, one box segment at a time, summing
// factor * value in FP64.  Boxes wholly inside the tile are finalised and
// stored directly; a box cut by a tile edge leaves a raw partial sum for the
// fix-up kernel.  The order of every sum is fixed by the element order, so
// results are bitwise reproducible.
#pragma once

#include "q2x_internal.hpp"

namespace q2x {

// Every lambda of the kernel body is inlined: an outlined one would become a
// real call with its captures on the scratch stack.
#define Q2X_INLINE __attribute__((always_inline))

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

// One part (real or imaginary) of every order of one recursion array.
template <typename T, int P1>
struct CVec {
  T v[P1];
};

// Per-lane coefficients of one application of the ladder operator of Sec.
// 3.4, Eqs. (50)-(51) (tilde form), which makes degree N (orders 0..N) from
// degree N-1 (orders 0..N-1):
//   out^0 = 2 Re(eta F^1) - z F^0 + add^0
//   out^m = -xi F^{m-1} + eta F^{m+1} - z F^m + add^m,   m >= 1,
// with xi = x + i y (the vertex or normal, halved), eta = conj(xi) and F^k = 0
// for k > N-1.  The recursions of Eqs. (50)-(55) divide this by (n+k) at the
// k-th nesting level; the kernel carries G_n = (n+k)! F_n instead, for which
// the division disappears (G_n = D G_{n-1} + G^{(k-1)}_n, every start value
// 1), and folds 1/(n+k)! into the FP64 per-degree factor.
// Split into parts, with f the lane's own part and g its neighbour's (the
// real lane's g is the imaginary part and the other way round):
//   out^m = -x (f^{m-1} - f^{m+1}) + s y (g^{m-1} + g^{m+1}) - z f^m + add^m
// with s = +1 on the real lane and -1 on the imaginary lane, and
//   out^0 = 2x f^1 + 2y g^1 - z f^0 + add^0   (real lane),
//   out^0 = -z f^0 + add^0 = 0               (imaginary lane: f^0 = 0).
template <typename T>
struct LCoef {
  T x, ys, mz, c0f, c0g;  // x, s y, -z, and the order-0 factors of f^1, g^1
};

template <typename T>
__device__ __forceinline__ LCoef<T> ladder_coef(bool imag, T x, T y, T z, T x2, T y2) {
  LCoef<T> c;
  c.x = x;
  c.ys = imag ? -y : y;
  c.mz = -z;
  c.c0f = imag ? T(0) : x2;
  c.c0g = imag ? T(0) : y2;
  return c;
}

// The neighbouring lane's value (lanes 2e and 2e + 1 exchange: DPP
// quad_perm [1,0,3,2]).
__device__ __forceinline__ float neighbour(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ double neighbour(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0xB1, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// The neighbour's parts of orders 0..N-1 of an array.
template <int N, typename T, int P1>
__device__ __forceinline__ void spread(const CVec<T, P1>& F, T (&G)[P1]) {
  static_for<0, N>([&](auto MM) Q2X_INLINE {
    constexpr int m = decltype(MM)::value;
    G[m] = neighbour(F.v[m]);
  });
}

// The lane's part of degree N from degree N-1: F (own parts), G (the
// neighbour's parts of orders 0..N-1, from spread), add (own parts of the
// source term).  Every output is a chain of FMAs (5 for an interior order
// with a source).
template <int N, bool ADD, typename T, int P1>
__device__ __forceinline__ void ladder(CVec<T, P1>& out, const CVec<T, P1>& F, const T (&G)[P1],
                                       const CVec<T, P1>& add, const LCoef<T>& c) {
  static_assert(N >= 1 && N < P1, "degree out of range");
  {
    T v = ADD ? fmaT(c.mz, F.v[0], add.v[0]) : c.mz * F.v[0];
    if constexpr (N - 1 >= 1) {
      v = fmaT(c.c0g, G[1], v);
      v = fmaT(c.c0f, F.v[1], v);
    }
    out.v[0] = v;
  }
  static_for<1, N + 1>([&](auto MM) Q2X_INLINE {
    constexpr int m = decltype(MM)::value;
    T v = ADD ? fmaT(c.ys, G[m - 1], add.v[m]) : c.ys * G[m - 1];
    if constexpr (m + 1 <= N - 1) {
      v = fmaT(c.ys, G[m + 1], v);
      v = fmaT(c.x, F.v[m + 1], v);
    }
    if constexpr (m <= N - 1) v = fmaT(c.mz, F.v[m], v);
    v = fmaT(-c.x, F.v[m - 1], v);
    out.v[m] = v;
  });
}

// Staged coefficients of one element, in the order the recursion produces
// them: unit u = NOUT n + s is output slot s of degree n (n + 1 coefficients,
// m = 0..n) and starts at slot off(u).  Chunk j is slots [j CMAX, (j+1) CMAX);
// a chunk may end inside a unit, whose remaining coefficients open the next.
template <int P, int CMAX, int NOUT>
struct ChunkPlan {
  static constexpr int U = NOUT * (P + 1);      // units
  static constexpr int K = NOUT * tri(P + 1);   // staged coefficients per element
  static constexpr int NCHUNK = (K + CMAX - 1) / CMAX;
  static constexpr int off(int u) { return NOUT * tri(u / NOUT) + (u % NOUT) * (u / NOUT + 1); }
  static constexpr int unit_of(int k) {
    int u = 0;
    while (off(u + 1) <= k) ++u;
    return u;
  }
  static constexpr int first_unit(int j) { return unit_of(j * CMAX); }
  static constexpr int last_unit(int j) { return unit_of((j * CMAX + CMAX < K ? j * CMAX + CMAX : K) - 1); }
  static constexpr int max_units() {
    int mx = 0;
    for (int j = 0; j < NCHUNK; ++j) {
      const int d = last_unit(j) - first_unit(j) + 1;
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
template <>
struct KindInfo<Q2X_SEGMENT_VEC> {  // the segment chain; three outputs, one per density component
  static constexpr int nv = 2, nch = 2, nout = 3;
  static constexpr int vert(int k) { return k == 0 ? 1 : 0; }
  static constexpr bool dbl(int) { return false; }
  static constexpr int shift(int) { return 0; }
  static constexpr int depth(int) { return 1; }
  static constexpr int slot(int o) { return o; }
};

// output staged in slot s of a degree (inverse of KindInfo::slot)
template <typename KI>
__host__ __device__ constexpr int out_of_slot(int s) {
  for (int o = 0; o < KI::nout; ++o)
    if (KI::slot(o) == s) return o;
  return 0;
}

template <typename T>
struct PrecInfo;
template <>
struct PrecInfo<float> {
  static constexpr bool scaled = true;  // FP32 recursion on (y - c)/a_e
  static constexpr int cmax = 32;       // 16.6 KB stage
};
template <>
struct PrecInfo<double> {
  static constexpr bool scaled = false;  // plain FP64 recursion on y - c
  static constexpr int cmax = 32;
};

// 1/k!, the same sequence of roundings at compile time and at run time
__host__ __device__ constexpr double inv_factorial(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; ++i) f *= (double)i;
  return 1.0 / f;
}
constexpr int kNoExp = -4000;  // exponent of a box segment with no nonzero weight

// Per-element data of the recursion: validity and status bits, Jacobian J
// (Sec. 3.1, Eq. (9)), unit normal (triangles), the element scale a_e
// (largest vertex distance from the box centre; 1 when unscaled) and the
// vertex coordinates relative to the box centre divided by a_e, in the forms
// the ladder takes ((x, y)/2, z, (x, y)).
template <int NV, typename T>
struct ElemGeom {
  bool ok;
  uint32_t flag;
  double J, nx, ny, nz, scl;
  T vxr[NV], vxi[NV], vz[NV], vxr2[NV], vxi2[NV];
};

// Element e of box `key` (box_ok: key names a box); sigma[0..nsig) are its
// densities, checked for finiteness with the coordinates.  A bad vertex index
// or a non-finite input clears ok and sets the matching status bit; the
// element then has J = 0 and zero coordinates.
template <int NV, typename T, bool SCALED>
__device__ __forceinline__ ElemGeom<NV, T> element_geometry(const double* verts, int64_t n_verts,
                                                            const int32_t* elems, int64_t e,
                                                            const double* box_center, int key, bool box_ok,
                                                            const double* sigma, int nsig) {
  ElemGeom<NV, T> g;
  g.flag = 0;
  bool ok = box_ok;
  double xv[NV][3];
#pragma unroll
  for (int k = 0; k < NV; ++k) xv[k][0] = xv[k][1] = xv[k][2] = 0.0;
  double cx = 0.0, cy = 0.0, cz = 0.0;
  if (ok) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int32_t vi = as_global(elems)[e * NV + k];
      if (vi < 0 || vi >= n_verts) {
        ok = false;
        g.flag |= Q2X_FLAG_BAD_VERTEX;
      } else {
        cgdouble* const vp = as_global(verts) + 3 * (int64_t)vi;
        xv[k][0] = vp[0];
        xv[k][1] = vp[1];
        xv[k][2] = vp[2];
      }
    }
    cgdouble* const cp = as_global(box_center) + 3 * (int64_t)key;
    cx = cp[0];
    cy = cp[1];
    cz = cp[2];
  }
  if (ok) {
    bool fin = isfinite(cx) && isfinite(cy) && isfinite(cz);
    for (int o = 0; o < nsig; ++o) fin = fin && isfinite(sigma[o]);
#pragma unroll
    for (int k = 0; k < NV; ++k) fin = fin && isfinite(xv[k][0]) && isfinite(xv[k][1]) && isfinite(xv[k][2]);
    if (!fin) {
      ok = false;
      g.flag |= Q2X_FLAG_NONFINITE;
    }
  }
  // Jacobian (Eq. (9)) and unit normal from the absolute vertices
  double J = 0.0, nx = 0.0, ny = 0.0, nz = 0.0;
  if (ok) {
    const double ux = xv[1][0] - xv[0][0], uy = xv[1][1] - xv[0][1], uz = xv[1][2] - xv[0][2];
    static_assert(NV >= 2 && NV <= 4, "segments, triangles or tetrahedra");
    if constexpr (NV == 2) {  // segment: length
      J = sqrt(ux * ux + uy * uy + uz * uz);
    } else {
      const double vx = xv[2][0] - xv[0][0], vy = xv[2][1] - xv[0][1], vz = xv[2][2] - xv[0][2];
      double crx, cry, crz;
      cross_nofma(ux, uy, uz, vx, vy, vz, crx, cry, crz);
      if constexpr (NV == 4) {  // tetrahedron: |det|
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
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    g.vxr[k] = (T)(0.5 * X[k][0] * inv_scl);
    g.vxi[k] = (T)(0.5 * X[k][1] * inv_scl);
    g.vz[k] = (T)(X[k][2] * inv_scl);
    g.vxr2[k] = (T)(X[k][0] * inv_scl);
    g.vxi2[k] = (T)(X[k][1] * inv_scl);
  }
  g.ok = ok;
  g.J = J;
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  g.scl = scl;
  return g;
}

// Bit e of the result = bit 2e of x (element e's lead lane in a ballot).
__device__ __forceinline__ uint64_t even_bits(uint64_t x) {
  x &= 0x5555555555555555ull;
  x = (x | (x >> 1)) & 0x3333333333333333ull;
  x = (x | (x >> 2)) & 0x0F0F0F0F0F0F0F0Full;
  x = (x | (x >> 4)) & 0x00FF00FF00FF00FFull;
  x = (x | (x >> 8)) & 0x0000FFFF0000FFFFull;
  x = (x | (x >> 16)) & 0x00000000FFFFFFFFull;
  return x;
}

__device__ __forceinline__ int64_t readlane64(int64_t v, int i) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, i);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), i);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

template <int P, int KIND, typename T>
__global__ __launch_bounds__(kTile) void q2x_tile_kernel(TileArgs args, int64_t n_tiles) {
  using KI = KindInfo<KIND>;
  constexpr int P1 = P + 1;
  constexpr int NV = KI::nv;
  constexpr int NCH = KI::nch;
  constexpr int NOUT = KI::nout;
  constexpr int CMAX = PrecInfo<T>::cmax;  // coefficients per chunk (<= 32: lanes c and c + 32)
  static_assert(CMAX <= 32, "one lane pair per chunk coefficient");
  // padded row stride (elements) of the stage: SSTR sizeof(T) = 16 (mod 128),
  // so rows start 16-byte aligned and the 16-byte reads of eight lanes (eight
  // rows) cover the 32 banks once
  constexpr int TE = kTileElems;  // elements per tile (lanes e and e + TE)
  static_assert(2 * TE == kTile, "two lanes per element");
  constexpr int SSTR = (sizeof(T) == 4) ? TE + 4 : TE + 2;
  constexpr bool SCALED = PrecInfo<T>::scaled;
  using Plan = ChunkPlan<P, CMAX, NOUT>;

  // stage: weighted value of chunk coefficient c of every element, real part
  // in row c, imaginary part in row CMAX + c
  __shared__ __align__(16) T stage[2 * CMAX * SSTR];
  // FP32 path: scale exponents of every box segment of the tile (row 0: the
  // element scales a_e, row 1 + o: the weights s_e of output o)
  __shared__ int sexp[SCALED ? (NOUT + 1) * TE : 1];

  // a split tile has two workgroups (consecutive virtual ids, so the same
  // XCD): both run the recursion, workgroup wpart stages and reduces the chunks
  // J with J % 2 == wpart -- shorter waves where the grid is too small to fill
  // the chip, bitwise the same sums.  Split tiles are spread evenly: tile t's
  // first virtual id is t + floor(t S / n_tiles) (S = n_split), and t is split
  // iff the next one is two further on.
  const int64_t S = args.n_split;
  const int64_t vb = xcd_tile(blockIdx.x, n_tiles + S);
  int64_t tile = vb;
  int wpart = 0, ns = 1;
  if (S > 0) {  // uniform
    uint32_t t;
    split_tile((uint32_t)vb, (uint32_t)n_tiles, (uint32_t)S, t, wpart, ns);
    tile = t;
  }
  const int lane = threadIdx.x;
  const int el = lane >> 1;        // the lane's element in the tile
  const bool imag = lane & 1;      // the lane holds imaginary parts
  const bool lead = !imag;         // the lane that counts and records the element
  TileArgs a = args;
  int te = a.te;               // elements per tile (uniform, 1..TE; a batch job's own)
  int64_t q0 = tile * te;      // first sorted position of the tile
  int64_t pos_end = a.n_pos;   // end of the sorted range the tile belongs to
  int64_t key_off = 0;         // sorted keys are key_off + box id
  int64_t elem_off = 0;        // the permutation holds elem_off + element index
  int64_t ltile = tile;        // the tile's index within its job's partial sums
  const bool batch = (a.bjobs != nullptr);
  if (batch) {
    // this tile's job: tiles [bgroup_tiles[j], bgroup_tiles[j + 1]) belong to job bgroup_jobs[j]
    int lo = 0, hi = a.bng;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (a.bgroup_tiles[mid] <= tile) lo = mid;
      else hi = mid;
    }
    const int jid = a.bgroup_jobs[lo];
    const BatchJob& J = a.bjobs[jid];
    a.verts = J.verts;
    a.elems = J.elems;
    a.dens[0] = J.dens[0];
    a.dens[1] = J.dens[1];
    a.dens[2] = J.dens[2];
    a.dstride = J.dstride;
    a.box_center = J.box_center;
    a.outs[0] = J.outs[0];
    a.outs[1] = J.outs[1];
    a.outs[2] = J.outs[2];
    a.status = a.bstatus + jid;
    a.n_verts = J.n_verts;
    a.n_boxes = J.n_boxes;
    a.p = J.p;
    a.norm = J.norm;
    a.accumulate = J.accumulate;
    key_off = J.box_base;
    const int64_t s0 = a.bbox_start[J.box_base];
    pos_end = a.bbox_start[J.box_base + J.n_boxes];
    te = J.te;
    ltile = tile - a.bgroup_tiles[lo];
    q0 = s0 + ltile * te;
    elem_off = J.elem_base;  // positions in the concatenation of all jobs
    a.partials += J.part_off;
  }
  if (q0 >= pos_end) return;  // uniform (past the job's valid elements)
  const int ne = (int)min<int64_t>(te, pos_end - q0);
  const int64_t q = q0 + el;
  const bool in_range = el < ne;

  // ---- element, box and FP64 geometry (Sec. 3.1, Eqs. (8)-(9); Sec. 3.3, Eq. (21))
  const int key = in_range ? (int)(a.keys[q] - key_off) : INT32_MIN;
  // ids outside [0, B) were counted by the bucketing, or are counted below
  // when the caller presorted the input
  const bool box_ok = in_range && key >= 0 && key < a.n_boxes;
  const int64_t e = in_range ? (a.perm ? (int64_t)a.perm[q] - elem_off : q) : 0;
  double sigma[NOUT];
#pragma unroll
  for (int o = 0; o < NOUT; ++o) sigma[o] = box_ok ? as_global(a.dens[o])[e * a.dstride] : 0.0;
  const ElemGeom<NV, T> gm = element_geometry<NV, T, SCALED>(a.verts, a.n_verts, a.elems, e, a.box_center, key,
                                                             box_ok, sigma, NOUT);
  const bool ok = gm.ok;
  uint32_t flag = gm.flag;
  const double J = gm.J, nx = gm.nx, ny = gm.ny, nz = gm.nz, scl = gm.scl;
  const bool degenerate = ok && !(J > 0.0);
  // the lane's ladder coefficients about every vertex
  LCoef<T> cv[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) cv[k] = ladder_coef(imag, gm.vxr[k], gm.vxi[k], gm.vz[k], gm.vxr2[k], gm.vxi2[k]);
  // s_e = sigma_e J / (4 pi) (Sec. 3.2, Eq. (20)); 0 for skipped elements
  double sw[NOUT];
  static_for<0, NOUT>([&](auto OO) Q2X_INLINE {
    constexpr int o = decltype(OO)::value;
    sw[o] = ok ? sigma[o] * J * kInv4Pi : 0.0;
  });

  // ---- box start table: box_start[b] = first position whose key >= b, keys
  // outside [0, B) counting as -1 / B (the fix-up kernel reads it)
  const int key_prev = (in_range && q > 0) ? (int)(a.keys[q - 1] - key_off) : INT32_MIN;
  const int ncoef_out = (a.p + 1) * (a.p + 1);
  if (in_range && lead && !batch && wpart == 0) {
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
    const uint64_t deg_mask = __ballot(lead && degenerate);
    const uint64_t skip_mask = __ballot(lead && ((box_ok && !ok) || (a.count_bad_ids && in_range && !box_ok)));
    uint32_t fall = 0;
#pragma unroll
    for (int b = 0; b < 5; ++b)
      if (__ballot((flag >> b) & 1u)) fall |= (1u << b);
    if (a.count_bad_ids && __ballot(in_range && !box_ok)) fall |= Q2X_FLAG_BAD_BOX;
    if (lane == 0 && wpart == 0) {
      if (deg_mask) atomicAdd(&a.status->n_degenerate, (unsigned long long)__popcll(deg_mask));
      if (skip_mask) atomicAdd(&a.status->n_skipped, (unsigned long long)__popcll(skip_mask));
      if (fall) atomicOr(&a.status->flags, fall);
    }
  }

  // ---- box boundaries inside the tile (uniform bit mask), open tile edges
  // (bit i: element i, from its lead lane 2i)
  const bool seg_start = lead && in_range && (el == 0 || key != key_prev);
  const uint64_t bnd = even_bits(__ballot(seg_start));
  const uint64_t vseg = even_bits(__ballot(seg_start && box_ok));  // segments whose box is valid (flushed)
  bool head_open = false, tail_open = false;
  if (q0 > 0) head_open = (a.keys[q0 - 1] == a.keys[q0]);
  if (ne == te && q0 + te < pos_end) tail_open = (a.keys[q0 + te] == a.keys[q0 + te - 1]);
  // segments finished here (valid box, not continued from the previous tile
  // or into the next) and segments whose raw sums go to the partials (the
  // first, continued from the previous tile: slot 0; the last, continued into
  // the next: slot 1)
  uint64_t cont = head_open ? 1ull : 0ull;
  if (tail_open) cont |= 1ull << (63 - __clzll(bnd));  // (bit 0 of bnd is always set here)
  const uint64_t fin_mask = vseg & ~cont;
  const uint64_t part_mask = vseg & cont;
  const int p = a.p;
  // offset (doubles) of the element's box row in an output, read by the
  // reduction with readlane at segment starts
  const int64_t row_off = box_ok ? (int64_t)key * ncoef_out * 2 : 0;

  // ---- weights of the staged values.  Output o of degree n of an element is
  // s_e a_e^(n - shift) G_n / (n + depth)!, G_n the recursion value (on Y =
  // (y - c)/a_e in FP32, on y - c with a_e = 1 in FP64).
  //   FP64: the stage holds G_n s_e / (n + depth)!.
  //   FP32: the stage holds G_n (s_e / 2^Es) (a_e / 2^Eb)^(n - shift), with
  //   2^Eb >= every a_e and 2^Es >= every |s_e| of the element's box segment in
  //   the tile, so the weight lies in [-1, 1] and cannot overflow; a weight that
  //   underflows belongs to an element below 2^-126 of its box's largest.  The
  //   flush restores 2^((n - shift) Eb + Es) / (n + depth)! in FP64.
  double wgt[NOUT];
  double rr = 1.0;     // FP32: a_e / 2^Eb
  int seg_eb = 0;      // FP32: Eb and Es of this element's box segment (read by
  int seg_es[NOUT];    // the reduction with readlane at segment starts)
#pragma unroll
  for (int o = 0; o < NOUT; ++o) seg_es[o] = 0;
  if constexpr (SCALED) {
    const int si = __popcll(bnd & ((2ull << el) - 1)) - 1;  // box segment of this element
    if (lead) {
#pragma unroll
      for (int t = 0; t <= NOUT; ++t) sexp[t * TE + el] = kNoExp;
    }
    __syncthreads();
    if (ok && lead) {
      int ea;
      (void)frexp(scl, &ea);
      atomicMax(&sexp[si], ea);
#pragma unroll
      for (int o = 0; o < NOUT; ++o) {
        if (sw[o] != 0.0) {
          int es;
          (void)frexp(sw[o], &es);
          atomicMax(&sexp[(1 + o) * TE + si], es);
        }
      }
    }
    __syncthreads();
    seg_eb = sexp[si];
#pragma unroll
    for (int o = 0; o < NOUT; ++o) seg_es[o] = sexp[(1 + o) * TE + si];
#pragma unroll
    for (int o = 0; o < NOUT; ++o) wgt[o] = 0.0;
    if (ok) {
      rr = ldexp(scl, -seg_eb);
#pragma unroll
      for (int o = 0; o < NOUT; ++o) wgt[o] = ldexp(sw[o], -seg_es[o]);
    }
  } else {
    static_for<0, NOUT>([&](auto OO) Q2X_INLINE {
      constexpr int o = decltype(OO)::value;
      wgt[o] = sw[o] * inv_factorial(KI::depth(o));
    });
  }

  // ---- reduction of chunk J (staged slots [J CMAX, J CMAX + CMAX))
  // Lane c + 32 h holds coefficient c of the chunk, real part (h = 0) or
  // imaginary part (h = 1), and walks the tile's elements in order,
  // summing the staged values in FP64 (elements at even and odd positions in
  // two partial sums, added where a box segment ends).  Box changes are
  // therefore the same for every lane; at each one the wave pairs the real and
  // imaginary sums across the halves (v_permlane32_swap) and lane c stores
  // coefficient +m, lane c + 32 the coefficient -m.  The walk reads each half
  // of the next 8 elements as soon as the same half of the current 8 is
  // summed; the box id and scale exponents of a new segment come from the
  // lane of its first element (readlane), so a segment end touches no LDS.
  // Elements past ne carry weight 0 and add exact zeros.
  const uint64_t cuts = bnd & ~1ull;  // bit i: a box segment ends before element i
  // Reduction of the chunk with first slot K0 (CJ slots); the lane's slot
  // K0 + c decodes to degree n, output o and order m; shift and invf =
  // 1/(n + depth)! are output o's.
  auto reduce_body = [&](int K0, int CJ, int n, int o, int m, int shift, double invf) Q2X_INLINE {
    constexpr int BATCH = 8;
    const int h = lane >> 5;
    const int c = lane & 31;
    const bool act = c < CJ;
    const bool live = act && n <= p;             // a requested coefficient
    const bool wr = live && (h == 0 || m != 0);  // lane h = 1 writes -m for m > 0
    const int nct_p = tri(p + 1);  // partial sums are laid out for the requested order
    const int g_coef = o * nct_p + tri(n) + m;
    // Finalisation of a raw tilde sum T = tr + i ti into the +m and -m
    // coefficients (Sec. 3.4, Eqs. (47),(49); symmetry Eq. (12)):
    //   FMM    : F^{+m} = base i^{-m} conj(T), F^{-m} = base i^{-m} T, base = (-1)^n
    //   MOMENT : M^{+m} = base i^{m} T,       M^{-m} = base i^{m} conj(T), base = (-1)^m 4pi
    // With i^{-m} = fc + i fs (one of fc, fs is 0), cp = base fc, sp = base fs
    // and eta = +1 (FMM) or -1 (MOMENT):
    //   +m: (cp tr + sp ti, eta (sp tr - cp ti));  -m: (cp tr - sp ti, eta (sp tr + cp ti)).
    // F_n^0 is real: its imaginary part (round-off) is written as 0.
    const int r4 = m & 3;
    const double fc = (r4 == 0) ? 1.0 : ((r4 == 2) ? -1.0 : 0.0);
    const double fs = (r4 == 1) ? -1.0 : ((r4 == 3) ? 1.0 : 0.0);
    const bool fmm = (a.norm == Q2X_NORM_FMM);
    const double base = fmm ? ((n & 1) ? -1.0 : 1.0) : ((m & 1) ? -k4Pi : k4Pi);
    const double cp = base * fc, sp = base * fs;
    const double cq = fmm ? cp : -cp, sq = fmm ? sp : -sp;
    const bool im0 = (h == 0 && m == 0);
    const double A1 = cp, A2 = h ? -sp : sp;
    const double B1 = im0 ? 0.0 : sq, B2 = im0 ? 0.0 : (h ? cq : -cq);
    const int idx = h ? (n * n + n - m) : (n * n + n + m);
    double* const obase = ((NOUT == 1 || o == 0) ? a.outs[0] : (o == 1 ? a.outs[1] : a.outs[2])) + 2 * idx;
    double* const pbase = a.partials + (ltile * 2 * (int64_t)(NOUT * nct_p) + g_coef) * 2;
    const int nsh = (n > shift) ? n - shift : 0;
    // segment state (uniform): first element, box row offset, scale exponents
    // segment state, taken when the segment opens so that its flush does not
    // wait for it: first element, the lane's output address in the segment's
    // box row and (FP32) its FP64 factor 2^((n - shift) Eb + Es) / (n + depth)!
    int seg = 0;
    gdouble* dst = nullptr;
    double seg_scale = 1.0;
    auto open_segment = [&](int i) Q2X_INLINE {
      seg = i;
      dst = as_global(obase + readlane64(row_off, 2 * i));
      if constexpr (SCALED) {
        const int eb = __builtin_amdgcn_readlane(seg_eb, 2 * i);
        int es = __builtin_amdgcn_readlane(seg_es[0], 2 * i);
        if constexpr (NOUT >= 2) {
          const int es1 = __builtin_amdgcn_readlane(seg_es[1], 2 * i);
          if (o == 1) es = es1;
        }
        if constexpr (NOUT >= 3) {
          const int es2 = __builtin_amdgcn_readlane(seg_es[2], 2 * i);
          if (o == 2) es = es2;
        }
        seg_scale = ldexp(invf, nsh * eb + es);
      }
    };
    open_segment(0);
    auto flush = [&](double t) Q2X_INLINE {
      const bool fin = (fin_mask >> seg) & 1ull;  // (uniform)
      const bool prt = (part_mask >> seg) & 1ull;
      if (!fin && !prt) return;  // uniform: the segment's box id is outside [0, B)
      if constexpr (SCALED) t *= seg_scale;
      // pair the halves: tr from lane c, ti from lane c + 32, on every lane
      const uint32_t lo = (uint32_t)__double2loint(t), hi = (uint32_t)__double2hiint(t);
      const auto slo = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
      const auto shi = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
      const double tr = __hiloint2double((int)shi[0], (int)slo[0]);
      const double ti = __hiloint2double((int)shi[1], (int)slo[1]);
      // uniform: the box continues in another tile.  Its raw sum goes to slot
      // 0 (the tile's first segment, continued from the previous tile) or
      // slot 1 (the last segment, continued in the next tile)
      if (prt) {
        if (h == 0 && live) {
          const bool head = (seg == 0) && head_open;
          gdouble* pp = as_global(pbase + (head ? 0 : (int64_t)(NOUT * nct_p) * 2));
          pp[0] = tr;
          pp[1] = ti;
        }
        return;
      }
      if (!wr) return;
      double x = A1 * tr + A2 * ti, y = B1 * tr + B2 * ti;
      if (a.accumulate) {
        x += dst[0];
        y += dst[1];
      }
      dst[0] = x;
      dst[1] = y;
    };
    const T* pv = stage + ((h ? CMAX : 0) + (act ? c : 0)) * SSTR;
    // Half H (BATCH / 2 consecutive staged values from position off + H BATCH / 2)
    // of the lane's row, in 16-byte reads, into dst[H BATCH / 2 ...]
    auto load_half = [&](auto HH, int off, T (&dst)[BATCH]) Q2X_INLINE {
      constexpr int H = decltype(HH)::value;
      constexpr int B2 = BATCH / 2;
      if constexpr (sizeof(T) == 4) {
        const float4* q = reinterpret_cast<const float4*>(pv + off + H * B2);
        static_for<0, B2 / 4>([&](auto II) Q2X_INLINE {
          constexpr int i = decltype(II)::value;
          const float4 v = q[i];
          dst[H * B2 + 4 * i] = v.x;
          dst[H * B2 + 4 * i + 1] = v.y;
          dst[H * B2 + 4 * i + 2] = v.z;
          dst[H * B2 + 4 * i + 3] = v.w;
        });
      } else {
        const double2* q = reinterpret_cast<const double2*>(pv + off + H * B2);
        static_for<0, B2 / 2>([&](auto II) Q2X_INLINE {
          constexpr int i = decltype(II)::value;
          const double2 v = q[i];
          dst[H * B2 + 2 * i] = v.x;
          dst[H * B2 + 2 * i + 1] = v.y;
        });
      }
    };
    double a0 = 0.0, a1 = 0.0;  // sums over even / odd positions of the open segment
    // cur holds the batch being summed; each half is refilled from the next
    // batch as soon as it has been summed (no second buffer, no copies)
    T cur[BATCH];
    load_half(IC<0>{}, 0, cur);
    load_half(IC<1>{}, 0, cur);
    const int nwalk = (ne + BATCH - 1) & ~(BATCH - 1);  // the tile's elements (the rest of the batch adds zeros)
#pragma unroll 1
    for (int b0 = 0; b0 < nwalk; b0 += BATCH) {  // uniform
      const int bn = (b0 + BATCH < nwalk) ? b0 + BATCH : b0;  // (last batch: a harmless reload)
      const uint32_t uc = (uint32_t)(cuts >> b0) & 0xffu;
      static_for<0, BATCH>([&](auto JB) Q2X_INLINE {
        constexpr int j = decltype(JB)::value;
        if ((uc >> j) & 1u) {  // uniform: a segment ends before element b0 + j
          flush(a0 + a1);
          a0 = 0.0;
          a1 = 0.0;
          open_segment(b0 + j);
        }
        if constexpr (j & 1)
          a1 += (double)cur[j];
        else
          a0 += (double)cur[j];
        if constexpr (j == BATCH / 2 - 1) load_half(IC<0>{}, bn, cur);
        if constexpr (j == BATCH - 1) load_half(IC<1>{}, bn, cur);
      });
    }
    flush(a0 + a1);  // the tile's last segment
    __syncthreads();
  };
  // chunk J, decoded at compile time (natural chunk ends inside the recursion)
  auto reduce_chunk = [&](auto JJc) Q2X_INLINE {
    constexpr int J = decltype(JJc)::value;
    if (J % ns != wpart) return;  // uniform: the other workgroup's chunk
    constexpr int K0 = J * CMAX;
    constexpr int CJ = (Plan::K - K0 < CMAX) ? Plan::K - K0 : CMAX;
    constexpr int UF = Plan::first_unit(J), UL = Plan::last_unit(J);
    __syncthreads();
    const int c = lane & 31;
    const int k = K0 + ((c < CJ) ? c : 0);
    constexpr int OF = out_of_slot<KI>(UF % NOUT);
    int u = UF, ku = Plan::off(UF), sh = KI::shift(OF);
    double invf = inv_factorial(UF / NOUT + KI::depth(OF));
    static_for<UF, UL>([&](auto LL) Q2X_INLINE {
      constexpr int l = decltype(LL)::value;
      constexpr int ol = out_of_slot<KI>((l + 1) % NOUT);
      if (k >= Plan::off(l + 1)) {
        u = l + 1;
        ku = Plan::off(l + 1);
        sh = KI::shift(ol);
        invf = inv_factorial((l + 1) / NOUT + KI::depth(ol));
      }
    });
    const int o = out_of_slot<KI>(u % NOUT);
    reduce_body(K0, CJ, u / NOUT, o, k - ku, sh, invf);
  };
  // unit and order of slot k (run-time decode; units are degree-major)
  auto decode = [&](int k, int& u, int& ku) Q2X_INLINE {
    int n, mm;
    tri_nm(k / NOUT, n, mm);  // NOUT tri(n) <= k < NOUT tri(n + 1)
    const int r = k - NOUT * tri(n);
    const int sl = r / (n + 1);
    u = NOUT * n + sl;
    ku = NOUT * tri(n) + sl * (n + 1);
  };

  // output o of degree N: stage it, weighted, and reduce each chunk as soon
  // as it is full
  // (a split tile's workgroups both stage every chunk and reduce their own)
  T* const slane = stage + (imag ? CMAX * SSTR : 0) + el;
  auto emit = [&](auto NNc, auto OO, const CVec<T, P1>& V) Q2X_INLINE {
    constexpr int N = decltype(NNc)::value;
    constexpr int o = decltype(OO)::value;
    constexpr int u = NOUT * N + KI::slot(o);
    constexpr int k0 = Plan::off(u), k1 = Plan::off(u + 1);
    constexpr int j1 = (k1 - 1) / CMAX;
    const T w = (T)wgt[o];
    static_for<0, N + 1>([&](auto MM) Q2X_INLINE {
      constexpr int m = decltype(MM)::value;
      constexpr int kk = k0 + m;
      constexpr int row = kk % CMAX;
      slane[row * SSTR] = V.v[m] * w;
      if constexpr (row == CMAX - 1) reduce_chunk(IC<kk / CMAX>{});  // chunk kk / CMAX is full
    });
    if constexpr (SCALED) {
      if constexpr (N + 1 - KI::shift(o) > 0) wgt[o] *= rr;
    } else {
      constexpr double inv_next = 1.0 / (double)(N + 1 + KI::depth(o));
      wgt[o] *= inv_next;
    }
    if constexpr (k1 % CMAX != 0 && k1 == Plan::K) reduce_chunk(IC<j1>{});  // last, partly filled chunk
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

  // ---- recursion over degrees (Sec. 3.4).  Nested rather than sequential, so
  // that skipping the degrees above p merges no register state.
  CVec<T, P1> S0[NCH];
#pragma unroll
  for (int k = 0; k < NCH; ++k) S0[k].v[0] = imag ? T(0) : T(1);
  constexpr bool HAS_DBL = KI::dbl(NOUT - 1);
  if constexpr (!HAS_DBL) {
    // S holds degree N; emit the chain's last array for every output (one
    // weight per output)
    auto rec = [&](auto self, auto NNc, const CVec<T, P1>(&S)[NCH]) Q2X_INLINE -> void {
      constexpr int N = decltype(NNc)::value;
      static_for<0, NOUT>([&](auto OO) Q2X_INLINE { emit(IC<N>{}, OO, S[NCH - 1]); });
      if constexpr (N < P) {
        if (N < p) {
          CVec<T, P1> nS[NCH];
          T none[P1];
          advance(IC<N + 1>{}, IC<0>{}, nS, S, none);
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
    const LCoef<T> cn = ladder_coef(imag, (T)(0.5 * nx), (T)(0.5 * ny), (T)nz, (T)nx, (T)ny);
    auto rec = [&](auto self, auto NNc, const CVec<T, P1>(&S)[NCH]) Q2X_INLINE -> void {
      constexpr int N = decltype(NNc)::value;
      if constexpr (N == 0) {
        CVec<T, P1> Z;
        Z.v[0] = T(0);
        emit(IC<0>{}, IC<OD>{}, Z);
        if constexpr (NOUT == 2) emit(IC<0>{}, IC<0>{}, S[NCH - 1]);
        if (0 < p) self(self, IC<1>{}, S);
      } else {
        T G[P1];  // the neighbour's parts of the last array (degree N-1)
        spread<N>(S[NCH - 1], G);
        {
          CVec<T, P1> L;
          ladder<N, false>(L, S[NCH - 1], G, S[NCH - 1], cn);
          emit(IC<N>{}, IC<OD>{}, L);
        }
        if constexpr (NOUT == 2) {
          CVec<T, P1> nS[NCH];
          advance(IC<N>{}, IC<1>{}, nS, S, G);
          emit(IC<N>{}, IC<0>{}, nS[NCH - 1]);
          if constexpr (N < P) {
            if (N < p) self(self, IC<N + 1>{}, nS);
          }
        } else if constexpr (N < P) {
          if (N < p) {
            CVec<T, P1> nS[NCH];
            advance(IC<N>{}, IC<1>{}, nS, S, G);
            self(self, IC<N + 1>{}, nS);
          }
        }
      }
    };
    rec(rec, IC<0>{}, S0);
  }
  // a run stopped at p < P: reduce the chunk that holds the last coefficients
  // of degree p unless it ended exactly there
  if (p < P) {
    const int kend = NOUT * tri(p + 1);
    if (kend % CMAX != 0 && ((kend - 1) / CMAX) % ns == wpart) {
      const int J = (kend - 1) / CMAX;
      const int K0 = J * CMAX;
      const int CJ = min(CMAX, Plan::K - K0);
      int u, ku;
      const int k = K0 + (((lane & 31) < CJ) ? (lane & 31) : 0);
      decode(k, u, ku);
      const int o = out_of_slot<KI>(u % NOUT);
      __syncthreads();
      reduce_body(K0, CJ, u / NOUT, o, k - ku, KI::shift(o), inv_factorial(u / NOUT + KI::depth(o)));
    }
  }

}

}  // namespace q2x
