// q2x_api.hip -- C ABI entry points: argument checks, workspace layout, the
// launch sequence of one call (status clear -> bucketing -> recursion tiles ->
// fix-up of boxes cut by tile edges), status readback and kernel timing.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "q2x_internal.hpp"

namespace q2x {


// Boxes whose elements span more than one tile: sum the per-tile partials in
// tile order, finalise and store.  Empty boxes: zeros (unless accumulating).
// One wavefront per box; grid-stride over boxes.
__global__ __launch_bounds__(256) void q2x_fixup_kernel(FixupArgs f) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t b = wave; b < f.n_boxes; b += nwaves) {
    int64_t s = 0, t = 0;
    if (f.n_pos) {  // (uniform) both starts loaded before either is used
      const int32_t s0 = f.box_start[b], s1 = f.box_start[b + 1];
      s = s0;
      t = s1;
    }
    fixup_box(lane, s, t, 0, f.te, f.partials, f.outs, b, f.nout, f.p, f.norm, f.accumulate);
  }
}

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct Layout {
  size_t status, box_start, sort, partials, total;
  int te;
  int64_t n_tiles;
};

// Partial sums are laid out for the requested order p: [n_tiles][2][nout][tri(p+1)][2].
Layout layout(int64_t n, int64_t nb, int p, int nout, int prec) {
  Layout L;
  L.te = tile_width(n, prec);
  L.n_tiles = (n + L.te - 1) / L.te;
  size_t off = 0;
  L.status = off;
  off += align_up(sizeof(Status));
  L.box_start = off;
  off += align_up((size_t)(nb + 1) * sizeof(int32_t));
  L.sort = off;
  off += align_up(bucket_scratch_bytes(n, nb));
  L.partials = off;
  off += align_up((size_t)L.n_tiles * 2 * (size_t)nout * (size_t)tri(p + 1) * 2 * sizeof(double));
  L.total = off;
  return L;
}

constexpr int kKinds = 6;
int outputs_per_kind(int kind) { return kind == Q2X_TRI_BOTH ? 2 : (kind == Q2X_SEGMENT_VEC ? 3 : 1); }

// ---- kernel timing (measurement aid)
struct Prof {
  std::mutex mu;
  bool on = false;
  struct Ev {
    hipEvent_t a, b, c, d;  // call start, recursion start, recursion end, call end
    int kind;
  };
  std::vector<Ev> evs;
  std::vector<Ev> pool;
};
Prof& prof() {
  static Prof p;
  return p;
}

// A set of four timing events (from the pool, else new); false if HIP could
// not create them (the call then runs untimed).
bool get_ev(Prof::Ev& e) {
  Prof& P = prof();
  if (!P.pool.empty()) {
    e = P.pool.back();
    P.pool.pop_back();
    return true;
  }
  if (hipEventCreate(&e.a) != hipSuccess || hipEventCreate(&e.b) != hipSuccess ||
      hipEventCreate(&e.c) != hipSuccess || hipEventCreate(&e.d) != hipSuccess)
    return false;
  return true;
}

// One call.  Output o (o < outputs of the kind) takes its density from
// dens[o][e * dstride] and writes outs[o].
// ext_status: the status block lives there instead of at the head of the
// workspace (whose first slot is then unused); allow_timing: the call may
// take part in kernel timing (which can create HIP events).
q2x_status run(int kind, const double* verts, int64_t n_verts, const int32_t* elems, int64_t n_elems,
               const double* const* dens, int dstride, const int32_t* elem_box, const double* box_center,
               const double* box_radius, int64_t n_boxes, int p, int prec, int norm, unsigned flags,
               double* const* outs, void* workspace, size_t workspace_bytes, void* stream,
               Status* ext_status = nullptr, bool allow_timing = true) {
  const int nout = outputs_per_kind(kind);
  if (p < 0 || p > Q2X_P_MAX) return Q2X_ERR_P_RANGE;
  if (n_verts < 0 || n_elems < 0 || n_boxes < 0 || n_elems >= ((int64_t)1 << 31) - 64 ||
      n_boxes >= ((int64_t)1 << 31) - 1 || n_verts >= ((int64_t)1 << 31))
    return Q2X_ERR_ARG;
  if (prec != Q2X_FP64 && prec != Q2X_FP32_MIXED) return Q2X_ERR_ARG;
  if (norm != Q2X_NORM_FMM && norm != Q2X_NORM_MOMENT) return Q2X_ERR_ARG;
  if (flags & ~(unsigned)(Q2X_ACCUMULATE | Q2X_PRESORTED)) return Q2X_ERR_ARG;
  if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return Q2X_ERR_WORKSPACE;
  (void)box_radius;  // accepted for interface compatibility; not read (see q2x.h)
  if (n_boxes > 0 && !box_center) return Q2X_ERR_ARG;
  if (n_elems > 0 && (!verts || !elems || !elem_box)) return Q2X_ERR_ARG;
  if (((uintptr_t)verts % 8) || ((uintptr_t)box_center % 8) || ((uintptr_t)elems % 4) || ((uintptr_t)elem_box % 4))
    return Q2X_ERR_ARG;
  const size_t out_bytes = (size_t)n_boxes * (size_t)(p + 1) * (size_t)(p + 1) * 2 * sizeof(double);
  for (int o = 0; o < nout; ++o) {
    if (n_boxes > 0 && !outs[o]) return Q2X_ERR_ARG;
    if (n_elems > 0 && !dens[o]) return Q2X_ERR_ARG;
    if (((uintptr_t)outs[o] % 8) || ((uintptr_t)dens[o] % 8)) return Q2X_ERR_ARG;
    for (int q = 0; q < o; ++q) {  // outputs must not overlap
      const uintptr_t c1 = (uintptr_t)outs[q], c2 = (uintptr_t)outs[o];
      if (n_boxes > 0 && c1 < c2 + out_bytes && c2 < c1 + out_bytes) return Q2X_ERR_ARG;
    }
  }
  const int P = bucket_order(p);
  if (P < 0) return Q2X_ERR_UNSUPPORTED;
  const Layout L = layout(n_elems, n_boxes, p, nout, prec);
  if (workspace_bytes < L.total) return Q2X_ERR_WORKSPACE;

  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)workspace;
  Status* st = ext_status ? ext_status : (Status*)(ws + L.status);
  int32_t* box_start = (int32_t*)(ws + L.box_start);
  int32_t* sort_scratch = (int32_t*)(ws + L.sort);
  double* partials = (double*)(ws + L.partials);

  Prof& PR = prof();
  Prof::Ev ev{};
  bool timing = false;
  if (allow_timing) {
    std::lock_guard<std::mutex> g(PR.mu);
    timing = PR.on && get_ev(ev);
  }
  if (timing && hipEventRecord(ev.a, s) != hipSuccess) return Q2X_ERR_HIP;

  // status clear + bucketing (the first sort kernel clears the status block);
  // the tile kernel writes the box start table
  const int32_t* keys = elem_box;
  const int32_t* perm = nullptr;
  hipError_t err;
  if ((flags & Q2X_PRESORTED) || n_elems == 0) {
    err = clear_status(st, s);
  } else {
    err = bucket_elements(elem_box, n_elems, n_boxes, sort_scratch, st, s, &keys, &perm);
  }
  if (err != hipSuccess) return Q2X_ERR_HIP;

  TileArgs a{};
  a.verts = verts;
  a.elems = elems;
  for (int o = 0; o < nout; ++o) a.dens[o] = dens[o];
  a.dstride = dstride;
  a.keys = keys;
  a.perm = perm;
  a.box_center = box_center;
  a.box_start = box_start;
  for (int o = 0; o < nout; ++o) a.outs[o] = outs[o];
  a.partials = partials;
  a.status = st;
  a.n_verts = n_verts;
  a.n_pos = n_elems;
  a.n_boxes = n_boxes;
  a.p = p;
  a.norm = norm;
  a.accumulate = (flags & Q2X_ACCUMULATE) ? 1 : 0;
  a.count_bad_ids = (flags & Q2X_PRESORTED) ? 1 : 0;
  a.te = L.te;
  const int64_t n_tiles = L.n_tiles;
  a.n_split = split_count(n_tiles, prec);
  if (timing && hipEventRecord(ev.b, s) != hipSuccess) return Q2X_ERR_HIP;
  if (n_tiles > 0) {
    err = launch_tiles(kind, prec, P, a, n_tiles, s);
    if (err != hipSuccess) return Q2X_ERR_HIP;
  }
  if (timing && hipEventRecord(ev.c, s) != hipSuccess) return Q2X_ERR_HIP;
  if (n_boxes > 0) {
    FixupArgs f{};
    f.box_start = box_start;
    f.partials = partials;
    f.n_pos = n_elems;
    f.te = L.te;
    for (int o = 0; o < nout; ++o) f.outs[o] = outs[o];
    f.n_boxes = n_boxes;
    f.p = p;
    f.nout = nout;
    f.norm = norm;
    f.accumulate = a.accumulate;
    const int64_t waves = n_boxes;
    int64_t blocks = (waves + 3) / 4;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(q2x_fixup_kernel, dim3((unsigned)blocks), dim3(256), 0, s, f);
    if (hipGetLastError() != hipSuccess) return Q2X_ERR_HIP;
  }
  if (timing) {
    if (hipEventRecord(ev.d, s) != hipSuccess) return Q2X_ERR_HIP;
    ev.kind = kind;
    std::lock_guard<std::mutex> g(PR.mu);
    PR.evs.push_back(ev);
  }
  return Q2X_OK;
}

// ---- scratch of the entry point that allocates nothing (q2x_tri_both_noalloc)
// One array per GPU, loaded with the code object and held until the process
// ends.  In host code `scratch` only names the symbol: its device address
// comes from hipGetSymbolAddress, once per device, with that device current.
constexpr size_t kNoAllocBytes = (size_t)Q2X_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (nullptr on failure).
void* scratch_of_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

}  // namespace
}  // namespace q2x

using namespace q2x;

extern "C" {

size_t q2x_workspace_bytes(int kind, int64_t n_elems, int64_t n_boxes, int p, int precision) {
  if (kind < 0 || kind >= kKinds || n_elems < 0 || n_boxes < 0 || p < 0 || p > Q2X_P_MAX) return 0;
  if (precision != Q2X_FP64 && precision != Q2X_FP32_MIXED) return 0;
  const int P = bucket_order(p);
  if (P < 0) return 0;
  return layout(n_elems, n_boxes, p, outputs_per_kind(kind), precision).total;
}

#define Q2X_ENTRY(name, KIND)                                                                                      \
  q2x_status name(const double* verts, int64_t n_verts, const int32_t* el, int64_t n_el, const double* density,   \
                  const int32_t* elem_box, const double* box_center, const double* box_radius, int64_t n_boxes,  \
                  int p, int precision, int norm, unsigned flags, double* coeffs, void* workspace,                \
                  size_t workspace_bytes, void* stream) {                                                         \
    const double* dens[1] = {density};                                                                           \
    double* outs[1] = {coeffs};                                                                                    \
    return run(KIND, verts, n_verts, el, n_el, dens, 1, elem_box, box_center, box_radius, n_boxes, p, precision,  \
               norm, flags, outs, workspace, workspace_bytes, stream);                                            \
  }

Q2X_ENTRY(q2x_tri_single, Q2X_TRI_SINGLE)
Q2X_ENTRY(q2x_tri_double, Q2X_TRI_DOUBLE)
Q2X_ENTRY(q2x_segment, Q2X_SEGMENT)
Q2X_ENTRY(q2x_tet, Q2X_TET)

q2x_status q2x_tri_both(const double* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                        const double* density_single, const double* density_double, const int32_t* elem_box,
                        const double* box_center, const double* box_radius, int64_t n_boxes, int p,
                        int precision, int norm, unsigned flags, double* coeffs_single, double* coeffs_double,
                        void* workspace, size_t workspace_bytes, void* stream) {
  const double* dens[2] = {density_single, density_double};
  double* outs[2] = {coeffs_single, coeffs_double};
  return run(Q2X_TRI_BOTH, verts, n_verts, tris, n_tris, dens, 1, elem_box, box_center, box_radius, n_boxes, p,
             precision, norm, flags, outs, workspace, workspace_bytes, stream);
}

q2x_status q2x_tri_both_noalloc(const double* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                                const double* density_single, const double* density_double, const int32_t* elem_box,
                                const double* box_center, const double* box_radius, int64_t n_boxes, int p,
                                int precision, int norm, unsigned flags, double* coeffs_single,
                                double* coeffs_double, void* status, void* stream) {
  if (!status || ((uintptr_t)status % 8) != 0) return Q2X_ERR_ARG;
  if (p < 0 || p > Q2X_P_MAX) return Q2X_ERR_P_RANGE;
  if (n_tris < 0 || n_boxes < 0) return Q2X_ERR_ARG;
  if (precision != Q2X_FP64 && precision != Q2X_FP32_MIXED) return Q2X_ERR_ARG;
  const int P = bucket_order(p);
  if (P < 0) return Q2X_ERR_UNSUPPORTED;
  if (n_tris >= ((int64_t)1 << 31) - 64 || n_boxes >= ((int64_t)1 << 31) - 1) return Q2X_ERR_ARG;
  // the scratch holds the workspace of q2x_tri_both (its status slot unused)
  if (layout(n_tris, n_boxes, p, 2, precision).total > kNoAllocBytes) return Q2X_ERR_TOO_LARGE;
  void* ws = scratch_of_current_device();
  if (!ws) return Q2X_ERR_HIP;
  const double* dens[2] = {density_single, density_double};
  double* outs[2] = {coeffs_single, coeffs_double};
  return run(Q2X_TRI_BOTH, verts, n_verts, tris, n_tris, dens, 1, elem_box, box_center, box_radius, n_boxes, p,
             precision, norm, flags, outs, ws, kNoAllocBytes, stream, (Status*)status, false);
}

q2x_status q2x_segment_vec(const double* verts, int64_t n_verts, const int32_t* segs, int64_t n_segs,
                           const double* density3, const int32_t* elem_box, const double* box_center,
                           const double* box_radius, int64_t n_boxes, int p, int precision, int norm, unsigned flags,
                           double* coeffs3, void* workspace, size_t workspace_bytes, void* stream) {
  if (p < 0 || p > Q2X_P_MAX) return Q2X_ERR_P_RANGE;
  if (n_boxes < 0) return Q2X_ERR_ARG;
  const int64_t plane = n_boxes * (int64_t)(p + 1) * (p + 1) * 2;  // doubles per component
  const double* dens[3] = {density3, density3 ? density3 + 1 : nullptr, density3 ? density3 + 2 : nullptr};
  double* outs[3] = {coeffs3, coeffs3 ? coeffs3 + plane : nullptr, coeffs3 ? coeffs3 + 2 * plane : nullptr};
  return run(Q2X_SEGMENT_VEC, verts, n_verts, segs, n_segs, dens, 3, elem_box, box_center, box_radius, n_boxes, p,
             precision, norm, flags, outs, workspace, workspace_bytes, stream);
}

size_t q2x_eval_workspace_bytes(int64_t n_elems, int64_t n_boxes) {
  if (n_elems < 0 || n_boxes < 0) return 0;
  return align_up(sizeof(Status)) + align_up(bucket_scratch_bytes(n_elems, n_boxes));
}

q2x_status q2x_eval(int kind, const double* verts, int64_t n_verts, const int32_t* elems, int64_t n_elems,
                    const int32_t* elem_box, const double* box_center, int64_t n_boxes, const double* local, int p,
                    int precision, unsigned flags, double* out, void* workspace, size_t workspace_bytes,
                    void* stream) {
  if (kind < Q2X_TRI_SINGLE || kind > Q2X_TET) return Q2X_ERR_ARG;
  if (p < 0 || p > Q2X_P_MAX) return Q2X_ERR_P_RANGE;
  if (n_verts < 0 || n_elems < 0 || n_boxes < 0 || n_elems >= ((int64_t)1 << 31) - 64 ||
      n_boxes >= ((int64_t)1 << 31) - 1 || n_verts >= ((int64_t)1 << 31))
    return Q2X_ERR_ARG;
  if (precision != Q2X_FP64 && precision != Q2X_FP32_MIXED) return Q2X_ERR_ARG;
  if (flags & ~(unsigned)(Q2X_ACCUMULATE | Q2X_PRESORTED)) return Q2X_ERR_ARG;
  if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return Q2X_ERR_WORKSPACE;
  if (n_boxes > 0 && (!box_center || !local)) return Q2X_ERR_ARG;
  if (n_elems > 0 && (!verts || !elems || !elem_box || !out)) return Q2X_ERR_ARG;
  if (((uintptr_t)verts % 8) || ((uintptr_t)box_center % 8) || ((uintptr_t)local % 8) || ((uintptr_t)out % 8) ||
      ((uintptr_t)elems % 4) || ((uintptr_t)elem_box % 4))
    return Q2X_ERR_ARG;
  const int P = bucket_order(p);
  if (P < 0) return Q2X_ERR_UNSUPPORTED;
  if (workspace_bytes < q2x_eval_workspace_bytes(n_elems, n_boxes)) return Q2X_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  Status* st = (Status*)workspace;
  int32_t* scratch = (int32_t*)((char*)workspace + align_up(sizeof(Status)));
  const bool presorted = (flags & Q2X_PRESORTED) != 0;
  const int32_t* keys = elem_box;
  const int32_t* perm = nullptr;
  hipError_t err;
  // grouping by box only orders the work (lanes of a wavefront then share
  // rows of L); each element's result does not depend on it
  if (presorted || n_elems == 0) err = clear_status(st, s);
  else err = bucket_elements(elem_box, n_elems, n_boxes, scratch, st, s, &keys, &perm);
  if (err != hipSuccess) return Q2X_ERR_HIP;
  if (n_elems == 0) return Q2X_OK;
  EvalArgs a{};
  a.verts = verts;
  a.elems = elems;
  a.keys = keys;
  a.perm = perm;
  a.box_center = box_center;
  a.local = local;
  a.out = out;
  a.status = st;
  a.n_verts = n_verts;
  a.n_pos = n_elems;
  a.n_boxes = n_boxes;
  a.p = p;
  a.accumulate = (flags & Q2X_ACCUMULATE) ? 1 : 0;
  a.count_bad_ids = presorted ? 1 : 0;
  const int64_t n_tiles = (n_elems + kTileElems - 1) / kTileElems;  // two lanes per element
  if (launch_eval(kind, precision, P, a, n_tiles, s) != hipSuccess) return Q2X_ERR_HIP;
  return Q2X_OK;
}

size_t q2x_m2m_workspace_bytes(int64_t n_child, int64_t n_parent) {
  if (n_child < 0 || n_parent < 0) return 0;
  return align_up(sizeof(Status)) + align_up((size_t)(n_parent + 1) * sizeof(int32_t)) +
         align_up(bucket_scratch_bytes(n_child, n_parent));
}

q2x_status q2x_m2m(const double* child_coeffs, const double* child_center, const int32_t* child_parent,
                   int64_t n_child, const double* parent_center, int64_t n_parent, int p, int norm, unsigned flags,
                   double* parent_coeffs, void* workspace, size_t workspace_bytes, void* stream) {
  if (p < 0 || p > Q2X_P_MAX) return Q2X_ERR_P_RANGE;
  if (n_child < 0 || n_parent < 0 || n_child >= ((int64_t)1 << 31) - 64 || n_parent >= ((int64_t)1 << 31) - 1)
    return Q2X_ERR_ARG;
  if (norm != Q2X_NORM_FMM && norm != Q2X_NORM_MOMENT) return Q2X_ERR_ARG;
  if (flags & ~(unsigned)(Q2X_ACCUMULATE | Q2X_PRESORTED)) return Q2X_ERR_ARG;
  if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return Q2X_ERR_WORKSPACE;
  if (n_child > 0 && (!child_coeffs || !child_center || !child_parent)) return Q2X_ERR_ARG;
  if (n_parent > 0 && (!parent_center || !parent_coeffs)) return Q2X_ERR_ARG;
  if (((uintptr_t)child_coeffs % 8) || ((uintptr_t)child_center % 8) || ((uintptr_t)child_parent % 4) ||
      ((uintptr_t)parent_center % 8) || ((uintptr_t)parent_coeffs % 8))
    return Q2X_ERR_ARG;
  const size_t row = (size_t)(p + 1) * (size_t)(p + 1) * 2 * sizeof(double);
  if (n_child > 0 && n_parent > 0) {  // the parents' rows are written while the children's are read
    const uintptr_t c0 = (uintptr_t)child_coeffs, c1 = c0 + row * (size_t)n_child;
    const uintptr_t p0 = (uintptr_t)parent_coeffs, p1 = p0 + row * (size_t)n_parent;
    if (c0 < p1 && p0 < c1) return Q2X_ERR_ARG;
  }
  if (workspace_bytes < q2x_m2m_workspace_bytes(n_child, n_parent)) return Q2X_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)workspace;
  Status* st = (Status*)ws;
  int32_t* box_start = (int32_t*)(ws + align_up(sizeof(Status)));
  int32_t* scratch = (int32_t*)(ws + align_up(sizeof(Status)) + align_up((size_t)(n_parent + 1) * sizeof(int32_t)));
  const bool presorted = (flags & Q2X_PRESORTED) != 0;
  const int32_t* keys = child_parent;
  const int32_t* perm = nullptr;
  hipError_t err;
  if (presorted || n_child == 0) err = clear_status(st, s);
  else err = bucket_elements(child_parent, n_child, n_parent, scratch, st, s, &keys, &perm);
  if (err != hipSuccess) return Q2X_ERR_HIP;
  if (n_parent == 0) return Q2X_OK;
  if (launch_box_bounds(keys, n_child, n_parent, box_start, s, presorted ? st : nullptr) != hipSuccess)
    return Q2X_ERR_HIP;
  M2MArgs a{};
  a.child = child_coeffs;
  a.child_center = child_center;
  a.perm = perm;
  a.box_start = box_start;
  a.parent_center = parent_center;
  a.out = parent_coeffs;
  a.status = st;
  a.n_child = n_child;
  a.n_parent = n_parent;
  a.p = p;
  a.norm = norm;
  a.accumulate = (flags & Q2X_ACCUMULATE) ? 1 : 0;
  a.presorted_bad = (presorted && n_child > 0) ? 1 : 0;
  if (launch_m2m(a, s) != hipSuccess) return Q2X_ERR_HIP;
  return Q2X_OK;
}

size_t q2x_bucket_workspace_bytes(int64_t n_elems, int64_t n_boxes) {
  if (n_elems < 0 || n_boxes < 0) return 0;
  return align_up(sizeof(Status)) + align_up(bucket_scratch_bytes(n_elems, n_boxes));
}

q2x_status q2x_bucket(const int32_t* elem_box, int64_t n_elems, int64_t n_boxes, int32_t* perm, int32_t* box_start,
                      void* workspace, size_t workspace_bytes, void* stream) {
  if (n_elems < 0 || n_boxes < 0 || n_elems >= ((int64_t)1 << 31) - 64 || n_boxes >= ((int64_t)1 << 31) - 1)
    return Q2X_ERR_ARG;
  if (!box_start || (n_elems > 0 && (!elem_box || !perm))) return Q2X_ERR_ARG;
  if (((uintptr_t)elem_box % 4) || ((uintptr_t)perm % 4) || ((uintptr_t)box_start % 4)) return Q2X_ERR_ARG;
  if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return Q2X_ERR_WORKSPACE;
  if (workspace_bytes < q2x_bucket_workspace_bytes(n_elems, n_boxes)) return Q2X_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  Status* st = (Status*)workspace;
  int32_t* scratch = (int32_t*)((char*)workspace + align_up(sizeof(Status)));
  const int32_t* keys = elem_box;
  const int32_t* pm = nullptr;
  if (n_elems == 0) {
    if (clear_status(st, s) != hipSuccess) return Q2X_ERR_HIP;
  } else if (bucket_elements(elem_box, n_elems, n_boxes, scratch, st, s, &keys, &pm) != hipSuccess) {
    return Q2X_ERR_HIP;
  }
  if (launch_box_bounds(keys, n_elems, n_boxes, box_start, s, nullptr) != hipSuccess) return Q2X_ERR_HIP;
  if (n_elems > 0 && copy_words(perm, pm, n_elems, s) != hipSuccess) return Q2X_ERR_HIP;
  return Q2X_OK;
}

q2x_status q2x_status_get(const void* workspace, void* stream, uint32_t* device_flags, int64_t* n_degenerate,
                          int64_t* n_skipped) {
  if (!workspace) return Q2X_ERR_ARG;
  Status h;
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(&h, workspace, sizeof(Status), hipMemcpyDeviceToHost, s) != hipSuccess) return Q2X_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return Q2X_ERR_HIP;
  if (device_flags) *device_flags = h.flags;
  if (n_degenerate) *n_degenerate = (int64_t)h.n_degenerate;
  if (n_skipped) *n_skipped = (int64_t)h.n_skipped;
  return Q2X_OK;
}

const char* q2x_status_string(int status) {
  switch (status) {
    case Q2X_OK: return "Q2X_OK";
    case Q2X_ERR_ARG: return "Q2X_ERR_ARG: invalid argument";
    case Q2X_ERR_P_RANGE: return "Q2X_ERR_P_RANGE: p outside [0, Q2X_P_MAX]";
    case Q2X_ERR_WORKSPACE: return "Q2X_ERR_WORKSPACE: workspace missing, misaligned or too small";
    case Q2X_ERR_HIP: return "Q2X_ERR_HIP: HIP runtime error";
    case Q2X_ERR_UNSUPPORTED: return "Q2X_ERR_UNSUPPORTED";
    case Q2X_ERR_TOO_LARGE:
      return "Q2X_ERR_TOO_LARGE: the call needs more scratch than the no-allocation entry point holds "
             "(Q2X_NOALLOC_SCRATCH_BYTES per GPU)";
    default: return "unknown q2x_status";
  }
}

void q2x_profile_enable(int on) {
  Prof& P = prof();
  std::lock_guard<std::mutex> g(P.mu);
  P.on = (on != 0);
}

void q2x_profile_reset(void) {
  Prof& P = prof();
  std::lock_guard<std::mutex> g(P.mu);
  for (auto& e : P.evs) P.pool.push_back(e);
  P.evs.clear();
}

q2x_status q2x_profile_read(double* recursion_ms, double* call_ms, int64_t* calls) {
  Prof& P = prof();
  std::lock_guard<std::mutex> g(P.mu);
  double rec[kKinds] = {}, tot[kKinds] = {};
  int64_t cnt[kKinds] = {};
  for (auto& e : P.evs) {
    if (hipEventSynchronize(e.d) != hipSuccess) return Q2X_ERR_HIP;
    float a = 0.f, b = 0.f;
    if (hipEventElapsedTime(&a, e.b, e.c) != hipSuccess) return Q2X_ERR_HIP;
    if (hipEventElapsedTime(&b, e.a, e.d) != hipSuccess) return Q2X_ERR_HIP;
    rec[e.kind] += a;
    tot[e.kind] += b;
    cnt[e.kind] += 1;
  }
  for (int k = 0; k < kKinds; ++k) {
    if (recursion_ms) recursion_ms[k] = rec[k];
    if (call_ms) call_ms[k] = tot[k];
    if (calls) calls[k] = cnt[k];
  }
  return Q2X_OK;
}

const char* q2x_version(void) { return "q2x-mi355x 0.1 (gfx950)"; }

}  // extern "C"
