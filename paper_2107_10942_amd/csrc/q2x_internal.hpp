// q2x_internal.hpp -- shared device-side definitions of the Q2X library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/q2x.h"

namespace q2x {

constexpr int kTile = 64;            // lanes of a tile workgroup (one wavefront)
constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kTileElems = 32;       // elements per recursion tile (two lanes per element)
constexpr double kInv4Pi = 0.07957747154594766788;  // 1/(4 pi)
constexpr double k4Pi = 12.566370614359172954;

// Status block at the head of every workspace.
struct Status {
  uint32_t flags;
  uint32_t pad;
  unsigned long long n_degenerate;
  unsigned long long n_skipped;
  unsigned long long reserved[5];
};
static_assert(sizeof(Status) == 64, "status block is 64 bytes");

// Global-memory view of a device pointer.  A pointer picked at run time from
// an argument struct or a job table is generic to the compiler, which then
// emits FLAT accesses; a FLAT store also counts against the LDS wait counter,
// so the next wait for LDS reads would wait for the store to reach memory.
// Accesses through this view are GLOBAL (vector-memory counter only).
typedef __attribute__((address_space(1))) double gdouble;
typedef const __attribute__((address_space(1))) double cgdouble;
typedef const __attribute__((address_space(1))) int32_t cgint;
__device__ __forceinline__ gdouble* as_global(double* p) { return (gdouble*)p; }
__device__ __forceinline__ cgdouble* as_global(const double* p) { return (cgdouble*)p; }
__device__ __forceinline__ cgint* as_global(const int32_t* p) { return (cgint*)p; }

// Number of m >= 0 ("tilde") coefficients of degrees 0..n-1.
__host__ __device__ constexpr int tri(int n) { return n * (n + 1) / 2; }

struct BatchJob;

// Arguments of the recursion + reduction kernel.  A single call fills the
// per-mesh fields; a batch launch (one group of jobs of the same kind,
// precision and order bucket) sets `bjobs`, and every workgroup then takes its
// job's fields from the job table.
struct TileArgs {
  const double* verts;
  const int32_t* elems;
  const double* dens[3];     // density of output o (unused entries nullptr); element e at dens[o][e * dstride]
  int32_t dstride;
  const int32_t* keys;       // box id of each sorted position (elem_box itself when presorted)
  const int32_t* perm;       // sorted position -> element index (nullptr: identity)
  const double* box_center;
  int32_t* box_start;        // [n_boxes + 1] out: start position of each box
  double* outs[3];           // coefficients of output o: [n_boxes][(p+1)^2][2]
  double* partials;          // [n_tiles][2][nout][tri(p+1)][2] raw sums of boxes cut by tile edges (a batch
                             // job's own region, tiles numbered from the job's first)
  Status* status;
  int64_t n_verts;
  int64_t n_pos;             // number of positions covered by tiles (= n_elems)
  int64_t n_boxes;
  int p;                     // requested order (<= template P)
  int norm;
  int accumulate;
  int count_bad_ids;         // presorted input (no bucketing pass): count ids outside [0, n_boxes) here
  int32_t te;                // elements per tile (1..32; tile t covers sorted positions [t te, (t + 1) te))
  int64_t n_split;           // tiles that get two workgroups (0 <= n_split <= n_tiles <= 2048 when > 0; spread evenly:
                             // tile t is split iff floor((t+1) n_split / n_tiles) > floor(t n_split / n_tiles));
                             // workgroup w of a split tile stages and reduces the chunks J with J % 2 == w.
                             // The grid holds n_tiles + n_split workgroups
  // batch launch (nullptr otherwise)
  const BatchJob* bjobs;       // job table
  const int32_t* bgroup_jobs;  // [bng] jobs of this launch
  const int64_t* bgroup_tiles; // [bng + 1] tile prefix of those jobs
  int32_t bng;
  Status* bstatus;             // [n_jobs] status blocks
  const int32_t* bbox_start;   // [total boxes + 1] start of every global box in the sorted order
};

// One job of a batch as the kernels see it (device table built by the plan).
struct BatchJob {
  const double* verts;
  const int32_t* elems;
  const double* dens[3];
  const int32_t* elem_box;
  const double* box_center;
  double* outs[3];
  int64_t n_verts, n_elems, n_boxes;
  int64_t elem_base;   // first element in the concatenation of all jobs
  int64_t box_base;    // first global box id
  int64_t tile_base;   // first tile of the job within its group's launch
  int64_t part_off;    // offset (doubles) of the job's partials ([tiles][2][nout][tri(p+1)][2]) in the workspace
  int32_t kind, prec, P, p, norm, accumulate, nout, group, dstride;
  int32_t te;          // elements per tile: the single call's (tile_width), so the sums are bitwise the same
};

// Elements per tile of a call: 32, two lanes per element (the recursion
// kernel's layout).
inline int tile_width(int64_t, int) { return kTileElems; }

// Arguments of the receiving-side kernel (integrals of local expansions over
// elements; one lane per element, no reduction).
struct EvalArgs {
  const double* verts;
  const int32_t* elems;
  const int32_t* keys;   // box id per position (sorted, or elem_box itself)
  const int32_t* perm;   // position -> element (nullptr: identity)
  const double* box_center;
  const double* local;   // [n_boxes][(p+1)^2][2]
  double* out;           // [n_elems][2]
  Status* status;
  int64_t n_verts;
  int64_t n_pos;
  int64_t n_boxes;
  int p;
  int accumulate;
  int count_bad_ids;     // presorted input (no bucketing pass): count ids outside [0, n_boxes) here
};

// Arguments of the multipole-to-multipole kernel (one workgroup per parent).
struct M2MArgs {
  const double* child;         // [n_child][(p+1)^2][2] child expansions (orders m >= 0 read)
  const double* child_center;  // [n_child][3]
  const int32_t* perm;         // sorted position -> child (nullptr: identity)
  const int32_t* box_start;    // [n_parent + 1] first sorted position of each parent's children
  const double* parent_center; // [n_parent][3]
  double* out;                 // [n_parent][(p+1)^2][2]
  Status* status;
  int64_t n_child;
  int64_t n_parent;
  int p;
  int norm;
  int accumulate;
  int presorted_bad;           // presorted input: count the ids outside [0, n_parent) from box_start
};

// Arguments of the fix-up kernel (boxes cut by tile edges, empty boxes).
struct FixupArgs {
  const int32_t* box_start;  // written by the tile kernel (unused when n_pos == 0)
  const double* partials;
  double* outs[3];
  int64_t n_pos;
  int64_t n_boxes;
  int p;
  int nout;                  // outputs per element kind (1; 2 for Q2X_TRI_BOTH; 3 for Q2X_SEGMENT_VEC)
  int norm;
  int accumulate;
  int te;                    // elements per tile of the recursion launch
};

// Logical tile of a workgroup: the hardware deals workgroups round-robin to
// the 8 XCDs (each with its own L2); give every XCD one contiguous range of
// tiles so that neighbouring tiles, which share vertices and box data, hit
// the same L2.
__host__ __device__ inline int64_t xcd_tile(int64_t bid, int64_t nblk) {
  const int64_t q = nblk / 8, r = nblk % 8;
  const int64_t x = bid % 8, k = bid / 8;
  return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Split tiles (two workgroups each) in a launch of n tiles: s of them, spread
// evenly -- tile t is split iff floor((t+1) s / n) > floor(t s / n) -- so the
// launch has n + s workgroups and tile t's first virtual id is t + floor(t s / n).
// The tile, workgroup part (0 or 1) and part count of virtual id v < n + s,
// in 32-bit arithmetic (the host splits tiles only in launches of at most
// 2,048 tiles, so (n + s) n fits).  The same function serves the kernel and
// the host-side check of the mapping.
__host__ __device__ inline void split_tile(uint32_t v, uint32_t n, uint32_t s, uint32_t& tile, int& part, int& parts) {
  uint32_t t = v * n / (n + s);  // within one of the answer
  while (t + 1 < n && (t + 1) + (t + 1) * s / n <= v) ++t;
  while (t > 0 && t + t * s / n > v) --t;
  tile = t;
  part = (int)(v - (t + t * s / n));
  parts = ((t + 1) * s / n > t * s / n) ? 2 : 1;
}

// How many tiles of a single call's launch get two workgroups.  Small grids
// leave the chip latency-bound, and there two workgroups share a tile's chunks
// (each runs the recursion): FP64 splits every tile of launches of up to
// 2,048 tiles; FP32 every tile up to 512, and between 1,024 and 2,048 tiles
// just enough for 2,048 workgroups, two per SIMD.
inline int64_t split_count(int64_t n_tiles, int prec) {
  if (prec == Q2X_FP64) return (n_tiles <= 2048) ? n_tiles : 0;
  if (n_tiles <= 512) return n_tiles;
  if (n_tiles > 1024 && n_tiles < 2048) return 2048 - n_tiles;
  return 0;
}

// Turn the raw tilde box sum T_n^m (sum_e s_e t~_{e,n}^m, m >= 0) into the two
// output coefficients and store (or add) them.  With i^{-m} = c + i s:
//   FMM   : F_n^{m}  = (-1)^n i^{-m} conj(T),  F_n^{-m} = (-1)^n i^{-m} T
//   MOMENT: M_n^{m}  = (-1)^m 4pi i^{m} T,     M_n^{-m} = (-1)^m 4pi i^{m} conj(T)
// (tilde <-> plain: Sec. 3.4, Eqs. (47),(49); symmetry Eq. (12); weights Eq. (20)).
// Branch-free in m (lanes of a wavefront hold different orders).
__device__ __forceinline__ void finalize_store(double* row_generic, int n, int m, double tr, double ti, int norm,
                                               int accumulate) {
  const int r = m & 3;
  const double c = (r == 0) ? 1.0 : ((r == 2) ? -1.0 : 0.0);
  const double s = (r == 1) ? -1.0 : ((r == 3) ? 1.0 : 0.0);
  double a, b, cc, d;  // (a, b) for +m, (cc, d) for -m
  if (norm == Q2X_NORM_FMM) {
    const double base = (n & 1) ? -1.0 : 1.0;
    const double xr = base * tr, xi = base * ti;
    a = c * xr + s * xi;   // (c + i s)(xr - i xi)
    b = s * xr - c * xi;
    cc = c * xr - s * xi;  // (c + i s)(xr + i xi)
    d = c * xi + s * xr;
  } else {
    const double base = (m & 1) ? -k4Pi : k4Pi;
    const double xr = base * tr, xi = base * ti;
    a = c * xr + s * xi;   // (c - i s)(xr + i xi)
    b = c * xi - s * xr;
    cc = c * xr - s * xi;  // (c - i s)(xr - i xi)
    d = -c * xi - s * xr;
  }
  if (m == 0) b = 0.0;  // F_n^0 is real; its imaginary part is round-off
  const int ip = n * n + n + m;
  const int im = n * n + n - m;
  // one 16-byte access per coefficient (rows are 16-byte aligned; the
  // callers use no LDS, so the generic access costs nothing here)
  double2* const row2 = reinterpret_cast<double2*>(row_generic);
  if (accumulate) {
    const double2 o = row2[ip];
    a += o.x;
    b += o.y;
  }
  row2[ip] = make_double2(a, b);
  if (m != 0) {
    if (accumulate) {
      const double2 o = row2[im];
      cc += o.x;
      d += o.y;
    }
    row2[im] = make_double2(cc, d);
  }
}

// Degree and order of the g-th tilde coefficient (g = tri(n) + m).
__device__ __forceinline__ void tri_nm(int g, int& n, int& m) {
  int nn = (int)((__fsqrt_rn(8.0f * (float)g + 1.0f) - 1.0f) * 0.5f);
  while (tri(nn + 1) <= g) ++nn;
  while (tri(nn) > g) --nn;
  n = nn;
  m = g - tri(nn);
}

// Box b spans tiles t0 < t1: sum its per-tile partial sums in tile order,
// finalise and store.  Tile t0 left the raw sum of its last segment in slot 1,
// every later tile that of its first segment in slot 0; a partial block is
// [tile][slot][nout][tri(p+1)][2] doubles.  One wavefront.
__device__ __forceinline__ void finish_cut_box(int lane, int64_t t0, int64_t t1, const double* partials,
                                               double* out0, double* out1, double* out2, int64_t b, int nout, int p,
                                               int norm, int accumulate) {
  const int ncoef = (p + 1) * (p + 1);
  const int nct_out = tri(p + 1);
  const int64_t pstride = (int64_t)nout * nct_out;  // partial sums per (tile, slot)
  const int total = nout * nct_out;
  // four coefficients per lane at a time, the first two tiles' partials of
  // all four loaded before any is used (a box spans two tiles but for boxes
  // longer than a tile), then the rest in tile order; sums in tile order.
  // (Eight at a time measured slower: 44 -> 72 VGPRs, 11.1 -> 13.4 us.)
  constexpr int U = 4;
  auto part = [&](int64_t tt, int gg) -> const double2* {
    const int o = gg / nct_out;
    const int g = gg - o * nct_out;
    const int slot = (tt == t0) ? 1 : 0;
    return reinterpret_cast<const double2*>(partials + ((tt * 2 + slot) * pstride + o * nct_out + g) * 2);
  };
  for (int g0 = lane; g0 < total; g0 += 64 * U) {
    double2 va[U], vb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int gg = g0 + 64 * u;
      const bool on = gg < total;
      va[u] = make_double2(0.0, 0.0);
      vb[u] = make_double2(0.0, 0.0);
      if (on) {
        va[u] = *part(t0, gg);
        vb[u] = *part(t0 + 1, gg);
      }
    }
    double ar[U], ai[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ar[u] = va[u].x + vb[u].x;
      ai[u] = va[u].y + vb[u].y;
    }
    for (int64_t tt = t0 + 2; tt <= t1; ++tt) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int gg = g0 + 64 * u;
        if (gg < total) {
          const double2 v = *part(tt, gg);
          ar[u] += v.x;
          ai[u] += v.y;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int gg = g0 + 64 * u;
      if (gg < total) {
        const int o = gg / nct_out;
        const int g = gg - o * nct_out;
        int n, m;
        tri_nm(g, n, m);
        double* const out = (o == 0) ? out0 : ((o == 1) ? out1 : out2);  // (selects: no indexed register array)
        finalize_store(out + b * (int64_t)ncoef * 2, n, m, ar[u], ai[u], norm, accumulate);
      }
    }
  }
}

// Box b of a sorted range [s, t) whose tiles of te elements start at
// position base (tile 0 of `partials`): finish it if tile edges cut it; empty
// boxes get zeros unless accumulating.  One wavefront.
__device__ __forceinline__ void fixup_box(int lane, int64_t s, int64_t t, int64_t base, int te,
                                          const double* partials, double* const* outs, int64_t b, int nout, int p,
                                          int norm, int accumulate) {
  const int ncoef = (p + 1) * (p + 1);
  if (t <= s) {
    if (!accumulate)
      for (int o = 0; o < nout; ++o) {
        double* row = outs[o] + b * (int64_t)ncoef * 2;
        for (int i = lane; i < 2 * ncoef; i += 64) row[i] = 0.0;
      }
    return;
  }
  const int64_t t0 = (s - base) / te, t1 = (t - 1 - base) / te;
  if (t0 == t1) return;  // finished by the tile kernel
  finish_cut_box(lane, t0, t1, partials, outs[0], nout > 1 ? outs[1] : nullptr, nout > 2 ? outs[2] : nullptr, b,
                 nout, p, norm, accumulate);
}

}  // namespace q2x

// Host-side launchers implemented in the per-kind translation units.
namespace q2x {
// bucketing (q2x_bucket.hip): sort elem_box -> (keys, perm); the first kernel
// also clears the status block
hipError_t bucket_elements(const int32_t* elem_box, int64_t n, int64_t nb, int32_t* scratch, Status* status,
                           hipStream_t s, const int32_t** keys_out, const int32_t** perm_out);
hipError_t launch_box_bounds(const int32_t* keys, int64_t n, int64_t nb, int32_t* box_start, hipStream_t s,
                             Status* order_check);
hipError_t clear_status(Status* st, hipStream_t s);
hipError_t copy_words(int32_t* dst, const int32_t* src, int64_t n, hipStream_t s);
size_t bucket_scratch_bytes(int64_t n, int64_t nb);
hipError_t launch_tiles(int kind, int prec, int P, const TileArgs& a, int64_t n_tiles, hipStream_t s);
int bucket_order(int p);  // smallest compiled bucket >= p (or -1)
hipError_t launch_eval(int kind, int prec, int P, const EvalArgs& a, int64_t n_tiles, hipStream_t s);
hipError_t launch_m2m(const M2MArgs& a, hipStream_t s);
}  // namespace q2x
