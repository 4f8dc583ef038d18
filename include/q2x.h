/*
 * q2x.h -- C ABI of the MI355X Quadrature-to-Expansion (Q2X) library.
 *
 * For flat simplices with piecewise-constant density the library computes the
 * Laplace multipole coefficients of each element about the centre of the leaf
 * box that owns it, with the O(1)-per-moment recursions of Gumerov, Kaneko &
 * Duraiswami (arXiv 2107.10942, Sec. 3.3-3.4, Eqs. (50)-(56)), and sums them
 * into one expansion per box (Sec. 2, Eq. (5)).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every array argument is a DEVICE pointer owned by the caller.  The
 *    library allocates nothing per call; scratch memory is the caller's
 *    `workspace` of at least q2x_workspace_bytes(...) bytes (256-byte aligned).
 *  - Calls are asynchronous on `stream` (a hipStream_t; NULL = default
 *    stream).  Argument errors are returned synchronously; data errors are
 *    reported through the device status word in the workspace (see
 *    q2x_status_get), after the caller synchronises the stream.
 *  - Sizes: n_elems < 2^31, n_boxes < 2^31, 0 <= p <= Q2X_P_MAX.
 *  - Output `coeffs` is [n_boxes][(p+1)^2][2] doubles (re, im); coefficient
 *    (n, m), -n <= m <= n, sits at index n*n + n + m.  Without
 *    Q2X_ACCUMULATE every box in [0, n_boxes) is overwritten (empty boxes get
 *    zeros); with it the new coefficients are added to what is there.
 *  - Normalisation (`norm`):
 *      Q2X_NORM_FMM    : F_n^m = sum_e sigma_e (1/4pi)(-1)^n int_e R_n^{-m}(y-c) dmu
 *                        (Sec. 3.2, Eqs. (14),(20)), so that
 *                        sum_{n<=p} sum_m F_n^m S_n^m(r - c) is the potential
 *                        (Sec. 2, Eq. (5); Sec. 3.2, Eq. (13)).
 *      Q2X_NORM_MOMENT : M_n^m = sum_e sigma_e int_e R_n^{m}(y-c) dmu
 *                        = (-1)^{n+m} 4pi conj(F_n^m); M_0^0 = sum sigma*measure.
 *    R_n^m, S_n^m are the solid harmonics of Sec. 3.2, Eq. (10).
 *  - Element -> box: elem_box[e] in [0, n_boxes) names the leaf box whose
 *    centre c = box_center[b] is the expansion centre (Sec. 2, after Eq. (5)).
 *    Elements are grouped by box internally (stable counting sort, increasing
 *    element index inside a box) unless Q2X_PRESORTED says elem_box is
 *    already non-decreasing.  An id outside [0, n_boxes) sets
 *    Q2X_FLAG_BAD_BOX and the element is skipped.
 *  - Precision: Q2X_FP64 runs the recursion in FP64 on y - c.  Q2X_FP32_MIXED
 *    runs it in FP32 on (y - c)/a_e, a_e the element's largest vertex distance
 *    from c, so the recursion works on O(1) values for any element size and
 *    order; the geometry, the weights s_e a_e^n and the box sums stay FP64.
 *  - box_radius is accepted for interface compatibility and is not read (the
 *    scaling above is per element); it may be NULL.
 *  - Degenerate elements (zero length/area/volume) contribute exactly zero and
 *    are counted.  Elements with non-finite coordinates, density or box centre set
 *    Q2X_FLAG_NONFINITE and are skipped; vertex indices outside [0, n_verts)
 *    set Q2X_FLAG_BAD_VERTEX and are skipped.  Nothing is ever written out of
 *    bounds.
 *  - Calls are reentrant when they use distinct workspaces; two calls that
 *    share a workspace must be ordered on one stream.
 */
#ifndef Q2X_H
#define Q2X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define Q2X_P_MAX 32

typedef enum {
  Q2X_OK = 0,
  Q2X_ERR_ARG = -1,         /* null/misaligned pointer, negative size, bad enum */
  Q2X_ERR_P_RANGE = -2,     /* p < 0 or p > Q2X_P_MAX */
  Q2X_ERR_WORKSPACE = -3,   /* workspace too small or misaligned */
  Q2X_ERR_HIP = -4,         /* a HIP runtime call failed */
  Q2X_ERR_UNSUPPORTED = -5, /* valid request this build does not implement */
  Q2X_ERR_TOO_LARGE = -6    /* q2x_tri_both_noalloc: the call does not fit its static scratch */
} q2x_status;

typedef enum {
  Q2X_TRI_SINGLE = 0,
  Q2X_TRI_DOUBLE = 1,
  Q2X_SEGMENT = 2,
  Q2X_TET = 3,
  Q2X_TRI_BOTH = 4,   /* single + double layer of one triangle mesh (q2x_tri_both) */
  Q2X_SEGMENT_VEC = 5 /* segments with a vector density, three outputs (q2x_segment_vec) */
} q2x_kind;
typedef enum { Q2X_FP64 = 0, Q2X_FP32_MIXED = 1 } q2x_precision;
typedef enum { Q2X_NORM_FMM = 0, Q2X_NORM_MOMENT = 1 } q2x_norm;

enum {
  Q2X_ACCUMULATE = 1u, /* add into coeffs instead of overwriting */
  Q2X_PRESORTED = 2u   /* elem_box is non-decreasing: skip the bucketing sort */
};

/* Device status word bits (q2x_status_get). */
enum {
  Q2X_FLAG_BAD_BOX = 1u,
  Q2X_FLAG_NONFINITE = 2u,
  Q2X_FLAG_RESERVED = 4u, /* not set by this implementation */
  Q2X_FLAG_BAD_VERTEX = 8u,
  Q2X_FLAG_NOT_SORTED = 16u /* Q2X_PRESORTED given but elem_box decreases */
};

/* Bytes of workspace one call of this shape needs (0 on invalid arguments). */
size_t q2x_workspace_bytes(int kind, int64_t n_elems, int64_t n_boxes, int p, int precision);

/*
 * Single-layer potential of flat triangles with constant density per
 * triangle (Sec. 2, Eq. (1) first line; coefficients L of Sec. 3.2,
 * Eqs. (14),(20)).  Recursion: vertex values q at x2 (Eqs. (40)-(41)), edge
 * integrals j along x3->x2 (Lemma 3, Eq. (32)), surface integrals i coned from
 * x1 (Lemma 2, Eq. (26)), in the m >= 0 form of Sec. 3.4, Eqs. (50)-(53).
 *   verts   [n_verts][3] double     vertex coordinates
 *   tris    [n_tris][3] int32       vertex indices (x1, x2, x3)
 *   density [n_tris] double         sigma_e
 *   elem_box[n_tris] int32          owning leaf box of each triangle
 *   box_center [n_boxes][3] double; box_radius unused (may be NULL)
 */
q2x_status q2x_tri_single(const double* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                          const double* density, const int32_t* elem_box, const double* box_center,
                          const double* box_radius, int64_t n_boxes, int p, int precision, int norm,
                          unsigned flags, double* coeffs, void* workspace, size_t workspace_bytes,
                          void* stream);

/*
 * Double-layer potential of flat triangles (Sec. 2, Eq. (1) second line;
 * coefficients M of Sec. 3.2, Eqs. (14),(18),(20)), from the single-layer
 * surface integrals of the previous degree (Sec. 3.4, Eq. (56)).  The normal
 * is n = (x2-x1)x(x3-x1)/|.| (right-hand rule on the given vertex order).
 * Same arguments as q2x_tri_single.
 */
q2x_status q2x_tri_double(const double* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                          const double* density, const int32_t* elem_box, const double* box_center,
                          const double* box_radius, int64_t n_boxes, int p, int precision, int norm,
                          unsigned flags, double* coeffs, void* workspace, size_t workspace_bytes,
                          void* stream);

/*
 * Single AND double layer of the same triangles in one call: one bucketing
 * and one recursion, since the double layer of degree n is D_nu applied to the
 * single-layer surface integrals of degree n-1 (Sec. 3.4, Eqs. (53),(56)).
 * Results equal q2x_tri_single(density_single) -> coeffs_single and
 * q2x_tri_double(density_double) -> coeffs_double (same rounding, bitwise);
 * the workspace is q2x_workspace_bytes(Q2X_TRI_BOTH, ...).  The two output
 * arrays must not overlap.  Other arguments as for q2x_tri_single.
 */
q2x_status q2x_tri_both(const double* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                        const double* density_single, const double* density_double, const int32_t* elem_box,
                        const double* box_center, const double* box_radius, int64_t n_boxes, int p,
                        int precision, int norm, unsigned flags, double* coeffs_single, double* coeffs_double,
                        void* workspace, size_t workspace_bytes, void* stream);

/*
 * q2x_tri_both for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same computation and results (bitwise) without a workspace argument.
 *   status   caller-owned device buffer of 64 bytes (8-byte aligned) that
 *            receives the call's status block; read it with
 *            q2x_status_get(status, stream, ...)
 * The scratch memory (sort buffers, box start table, partial sums of boxes
 * cut by tile edges) is a static device array of Q2X_NOALLOC_SCRATCH_BYTES
 * bytes, one per GPU, loaded with the library's code and held until the
 * process ends.  A call that needs more, i.e. when
 * q2x_workspace_bytes(Q2X_TRI_BOTH, n_tris, n_boxes, p, precision) exceeds
 * Q2X_NOALLOC_SCRATCH_BYTES (about 200,000 triangles at p = 16, one box per 12), returns
 * Q2X_ERR_TOO_LARGE without doing anything.  The call makes no hipMalloc,
 * hipFree or other allocation and no kernel timing; the first call on a
 * device looks up the array's device address (hipGetSymbolAddress).
 * Every call on one GPU shares that GPU's array (it keeps the previous call's
 * contents; nothing in it needs to start at zero): calls that overlap in
 * time on one GPU race, so order them on one stream.  Other arguments and
 * errors as for q2x_tri_both.
 */
#define Q2X_NOALLOC_SCRATCH_BYTES (64u << 20)
q2x_status q2x_tri_both_noalloc(const double* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                                const double* density_single, const double* density_double,
                                const int32_t* elem_box, const double* box_center, const double* box_radius,
                                int64_t n_boxes, int p, int precision, int norm, unsigned flags,
                                double* coeffs_single, double* coeffs_double, void* status, void* stream);

/*
 * Line segments with constant scalar line density (the integrals K of Sec. 2,
 * Eq. (3), one density component; Sec. 3.2, Eqs. (14),(20)).  Recursion:
 * vertex values q at x2 and segment integrals p from x1 (Lemma 1, Eq. (25);
 * Sec. 3.4, Eqs. (50)-(51)).
 *   segs [n_segs][2] int32 vertex indices (x1, x2); other arguments as above.
 */
q2x_status q2x_segment(const double* verts, int64_t n_verts, const int32_t* segs, int64_t n_segs,
                       const double* density, const int32_t* elem_box, const double* box_center,
                       const double* box_radius, int64_t n_boxes, int p, int precision, int norm,
                       unsigned flags, double* coeffs, void* workspace, size_t workspace_bytes,
                       void* stream);

/*
 * Segments with a constant VECTOR line density (the integrals K of Sec. 2,
 * Eq. (3), all three components, as in Biot-Savart vortex filaments): one
 * recursion per segment (as q2x_segment) and three outputs, component c with
 * density density3[e][c].  Equal bitwise to three q2x_segment calls with the
 * component densities.
 *   segs     [n_segs][2] int32; density3 [n_segs][3] double
 *   coeffs3  [3][n_boxes][(p+1)^2][2] double (component-major)
 * Workspace: q2x_workspace_bytes(Q2X_SEGMENT_VEC, ...).  Other arguments as above.
 */
q2x_status q2x_segment_vec(const double* verts, int64_t n_verts, const int32_t* segs, int64_t n_segs,
                           const double* density3, const int32_t* elem_box, const double* box_center,
                           const double* box_radius, int64_t n_boxes, int p, int precision, int norm, unsigned flags,
                           double* coeffs3, void* workspace, size_t workspace_bytes, void* stream);

/*
 * Tetrahedra with constant charge (the volume integrals N of Sec. 2, Eq. (4);
 * Sec. 3.2, Eqs. (14),(20)).  Recursion: q at x2, j along x3->x2, face
 * integrals b coned from x4 (Lemma 5, Eq. (38)), volume integrals a coned from
 * x1 (Lemma 4, Eq. (34)); Sec. 3.4, Eqs. (54)-(55).  J = |det| (orientation free).
 *   tets [n_tets][4] int32 vertex indices (x1, x2, x3, x4); other arguments as above.
 */
q2x_status q2x_tet(const double* verts, int64_t n_verts, const int32_t* tets, int64_t n_tets,
                   const double* density, const int32_t* elem_box, const double* box_center,
                   const double* box_radius, int64_t n_boxes, int p, int precision, int norm,
                   unsigned flags, double* coeffs, void* workspace, size_t workspace_bytes, void* stream);

/*
 * The bucketing step on its own: stable grouping of elements by leaf box
 * (every element belongs to exactly one box, Sec. 2 after Eq. (5)).
 *   elem_box  [n_elems] int32   box id of each element
 *   perm      [n_elems] int32   out: element indices grouped by increasing box
 *                               id, increasing element index inside a box; the
 *                               elements with ids outside [0, n_boxes) follow
 *                               the valid ones, in element order
 *   box_start [n_boxes+1] int32 out: box b owns perm[box_start[b] .. box_start[b+1])
 * Workspace: q2x_bucket_workspace_bytes(n_elems, n_boxes) bytes.  Ids outside
 * [0, n_boxes) set Q2X_FLAG_BAD_BOX and are counted as skipped.
 */
size_t q2x_bucket_workspace_bytes(int64_t n_elems, int64_t n_boxes);
q2x_status q2x_bucket(const int32_t* elem_box, int64_t n_elems, int64_t n_boxes, int32_t* perm, int32_t* box_start,
                      void* workspace, size_t workspace_bytes, void* stream);

/*
 * Receiving side: integrals of local expansions over elements, the evaluation
 * stage of a Galerkin method, which uses the same element integrals as Q2X
 * (Sec. 2 after Eq. (5) and the Conclusions; the recursions of Sec. 3.4,
 * Eqs. (50)-(56)).
 *   kind       Q2X_TRI_SINGLE (int_e R_n^m dS), Q2X_TRI_DOUBLE
 *              (int_e n . grad_y R_n^m dS, n the unit normal (x2-x1) x (x3-x1)),
 *              Q2X_SEGMENT (int_e R_n^m ds) or Q2X_TET (int_e R_n^m dV)
 *   elems      [n_elems][2|3|4] int32 vertex indices, as for the Q2X calls
 *   elem_box   [n_elems] int32 box of each element; box_center [n_boxes][3]
 *   local      [n_boxes][(p+1)^2][2] doubles: coefficients L_n^m of the field
 *              sum_{n<=p} sum_m L_n^m R_n^m(y - c_b) in box b, (n, m) at
 *              index n*n + n + m (the layout of coeffs above)
 *   out        [n_elems][2] doubles, out: for element e of box b,
 *              out[e] = sum_{n<=p} sum_m L_b[n,m] int_e R_n^m(y - c_b)
 *              (with Q2X_ACCUMULATE the value is added to out[e])
 *   flags      Q2X_ACCUMULATE; Q2X_PRESORTED (elem_box non-decreasing: skip
 *              the grouping of elements by box, which only orders the work so
 *              that neighbouring lanes share rows of `local`; results do not
 *              depend on it)
 *   precision  Q2X_FP64, or Q2X_FP32_MIXED (recursion in FP32 on (y - c)/a_e;
 *              weights a_e^n/(n+k)!, products with L and sums in FP64)
 * Elements with a box id outside [0, n_boxes), bad vertex indices or
 * non-finite coordinates get 0 (nothing added when accumulating), set the
 * matching Q2X_FLAG_* and are counted as skipped; degenerate elements get 0
 * and are counted.  Non-finite entries of `local` reach the outputs of the
 * elements of that box.  Workspace: q2x_eval_workspace_bytes(n_elems,
 * n_boxes) bytes; status as for the other calls.
 */
size_t q2x_eval_workspace_bytes(int64_t n_elems, int64_t n_boxes);
q2x_status q2x_eval(int kind, const double* verts, int64_t n_verts, const int32_t* elems, int64_t n_elems,
                    const int32_t* elem_box, const double* box_center, int64_t n_boxes, const double* local, int p,
                    int precision, unsigned flags, double* out, void* workspace, size_t workspace_bytes,
                    void* stream);

/*
 * Multipole-to-multipole translation: the upward-pass step of the FMM that
 * consumes the box coefficients (Sec. 1-2).  Each child expansion about its
 * centre c_c is translated to its parent's centre c_p with the finite
 * addition theorem of the regular solid harmonics (a consequence of the
 * derivative relations of Sec. 3.2, Eq. (15)), exact for every n <= p, and
 * the children of a parent are summed:
 *   Q2X_NORM_FMM   : F_n^m(c_p) = sum_c sum_{k<=n,l} F_k^l(c_c) R_{n-k}^{l-m}(c_p - c_c)
 *   Q2X_NORM_MOMENT: M_n^m(c_p) = sum_c sum_{k<=n,l} M_k^l(c_c) R_{n-k}^{m-l}(c_c - c_p)
 *   child_coeffs  [n_child][(p+1)^2][2] doubles, the layout of the Q2X outputs.
 *                 Only orders m >= 0 are read: the expansions must satisfy
 *                 A_n^{-m} = (-1)^m conj(A_n^m) (Sec. 3.2, Eq. (12); every
 *                 expansion of a real density does, so do all Q2X outputs)
 *   child_center  [n_child][3];  child_parent [n_child] int32 parent of each child
 *   parent_center [n_parent][3]
 *   parent_coeffs [n_parent][(p+1)^2][2] out; every parent is overwritten
 *                 (parents without children get zeros) unless Q2X_ACCUMULATE;
 *                 m < 0 written from the symmetry, imag(A_n^0) = 0.  Must not
 *                 overlap child_coeffs (one call per tree level)
 *   flags         Q2X_ACCUMULATE; Q2X_PRESORTED (child_parent non-decreasing,
 *                 as for Morton-ordered boxes: skip the grouping sort; a
 *                 decrease sets Q2X_FLAG_NOT_SORTED and the result is undefined)
 * Children with a parent id outside [0, n_parent) set Q2X_FLAG_BAD_BOX,
 * children whose centre or parent centre is non-finite set
 * Q2X_FLAG_NONFINITE; both are skipped and counted.  FP64 throughout.
 * Workspace: q2x_m2m_workspace_bytes(n_child, n_parent) bytes.
 */
size_t q2x_m2m_workspace_bytes(int64_t n_child, int64_t n_parent);
q2x_status q2x_m2m(const double* child_coeffs, const double* child_center, const int32_t* child_parent,
                   int64_t n_child, const double* parent_center, int64_t n_parent, int p, int norm, unsigned flags,
                   double* parent_coeffs, void* workspace, size_t workspace_bytes, void* stream);

/*
 * Near field: single- and double-layer potentials of flat triangles with
 * constant density at nearby targets, in closed form (Sec. 4.1, Eq. (63);
 * the double layer multiplied by sign((r - x1).n), which the printed formula
 * omits), for (target, triangle) pairs in compressed rows by target:
 *   L_j(r) = int_Tj G(r, y) dS_y,   M_j(r) = int_Tj dG/dn_y dS_y,   G = 1/(4 pi |r - y|),
 *   n = (x2 - x1) x (x3 - x1)/|.| on the given vertex order.
 *   targets     [n_targets][3]
 *   pair_start  [n_targets + 1] int64: target t's pairs are
 *               pair_tri[pair_start[t] .. pair_start[t+1]) (triangle indices)
 *   entries_L/M [n_pairs] out, or NULL: the unit-density values (the stored
 *               near-field matrix)
 *   potential   [n_targets] out, or NULL: sum over the target's pairs of
 *               density_single[j] L_j + density_double[j] M_j (either density
 *               may be NULL: its term is omitted; at least one is needed);
 *               Q2X_ACCUMULATE adds to it
 * A target within 1e-12 times the triangle's longest edge of its plane counts
 * as on it: M = 0 (the principal value) and L its value on the plane; this
 * covers collocation on the element itself.  Bad triangle ids and malformed
 * rows set Q2X_FLAG_BAD_BOX, bad vertex indices Q2X_FLAG_BAD_VERTEX,
 * non-finite coordinates Q2X_FLAG_NONFINITE; such pairs give 0 and are
 * counted as skipped; zero-area triangles give 0 and are counted as
 * degenerate.  FP64.  Workspace: q2x_near_workspace_bytes() bytes (the status
 * block).
 */
size_t q2x_near_workspace_bytes(void);
q2x_status q2x_near(const double* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris, const double* targets,
                    int64_t n_targets, const int64_t* pair_start, const int32_t* pair_tri, int64_t n_pairs,
                    const double* density_single, const double* density_double, double* entries_L,
                    double* entries_M, double* potential, unsigned flags, void* workspace, size_t workspace_bytes,
                    void* stream);

/*
 * Batches: many meshes (jobs) in one replayed launch sequence.  A job is one
 * single call's arguments; kind may be any q2x_kind (density2/coeffs2 only for
 * Q2X_TRI_BOTH; for Q2X_SEGMENT_VEC density is [N][3] and coeffs [3][B][..]).  Q2X_PRESORTED is accepted and has no effect (the batch always
 * sorts); Q2X_ACCUMULATE adds into that job's output.  Results are bitwise the
 * results of the single calls on the same jobs.
 *   q2x_batch_plan     host only: checks every job (synchronous errors as for
 *                      the single calls), groups jobs by (kind, precision,
 *                      order bucket) and lays out the workspace.  The job
 *                      arrays must stay valid while the plan is used; their
 *                      contents may change between runs.
 *   q2x_batch_run      enqueues the batch on `stream`.  The first run on a
 *                      workspace copies the job tables to a small device
 *                      buffer owned by the plan (allocated once, freed by
 *                      q2x_batch_destroy) and captures the launch sequence in
 *                      a HIP graph; later runs on that workspace replay it.
 *                      Unless a schedule was set or is cached for this
 *                      device, library build and plan shape, and unless a job
 *                      accumulates, that first run times the candidate
 *                      schedules (q2x_schedule), keeps the fastest, caches it
 *                      and synchronises `stream`.  Calls that share a plan
 *                      must be ordered on one stream.
 *   q2x_batch_launch   enqueues the batch on `stream` directly, without a
 *                      graph and without any allocation: the job tables are
 *                      copied into the workspace on `stream` (for batches that
 *                      run once, e.g. in serving).
 *   q2x_batch_job_status  q2x_status_get for one job of the last run.
 *   q2x_batch_groups / q2x_batch_mode  number of launch groups; chosen capture
 *                      (0 serial, 1 parallel branches, -1 not run yet).
 *
 * Schedules.  How a batch is launched never changes a bit of its results:
 *   mode   0: group launches in one stream order; 1: parallel graph branches;
 *   split  1: in groups of at most 2,048 tiles every tile gets two
 *          workgroups, each staging every chunk and reducing half of them;
 *   merge  a (kind, precision) order bucket whose jobs take at most `merge`
 *          tiles runs in the next bucket up (0 never; INT_MAX: one group per
 *          kind and precision);
 *   tuned  (output only) 0 default, 1 chosen by timing or from the cache,
 *          2 set by q2x_batch_set_schedule.
 *   q2x_batch_get_schedule  the plan's current schedule.
 *   q2x_batch_set_schedule  use `s` from now on (no tuning for this plan);
 *                      Q2X_ERR_ARG for values out of range or a merge value
 *                      whose layout needs more workspace than
 *                      q2x_batch_workspace_bytes reported.
 *   q2x_tune_cache_load / q2x_tune_cache_save  read / write the tuning cache
 *                      as text, one line per entry: "device|build|shape",
 *                      a tab, "mode split merge".  Entries of other devices
 *                      or library builds are kept and never used.  When the
 *                      environment variable Q2X_TUNE_CACHE names a file, it
 *                      is read before the first lookup and every new tuning
 *                      is appended to it.  Q2X_ERR_ARG if the file cannot be
 *                      opened.
 *   q2x_build_id       hash of the library's sources (part of the cache key).
 */
typedef struct q2x_job {
  int kind, p, precision, norm;
  unsigned flags;
  const double* verts;
  int64_t n_verts;
  const int32_t* elems;
  int64_t n_elems;
  const double* density;
  const double* density2;
  const int32_t* elem_box;
  const double* box_center;
  int64_t n_boxes;
  double* coeffs;
  double* coeffs2;
} q2x_job;
typedef struct q2x_plan q2x_plan;
q2x_status q2x_batch_plan(const q2x_job* jobs, int n_jobs, q2x_plan** plan);
size_t q2x_batch_workspace_bytes(const q2x_plan* plan);
q2x_status q2x_batch_run(q2x_plan* plan, void* workspace, size_t workspace_bytes, void* stream);
q2x_status q2x_batch_launch(q2x_plan* plan, void* workspace, size_t workspace_bytes, void* stream);
q2x_status q2x_batch_job_status(const q2x_plan* plan, const void* workspace, int job, void* stream,
                                uint32_t* device_flags, int64_t* n_degenerate, int64_t* n_skipped);
int q2x_batch_groups(const q2x_plan* plan);
int q2x_batch_mode(const q2x_plan* plan);
void q2x_batch_destroy(q2x_plan* plan);
typedef struct q2x_schedule {
  int32_t mode, split, merge, tuned;
} q2x_schedule;
q2x_status q2x_batch_get_schedule(const q2x_plan* plan, q2x_schedule* out);
q2x_status q2x_batch_set_schedule(q2x_plan* plan, const q2x_schedule* s);
q2x_status q2x_tune_cache_load(const char* path);
q2x_status q2x_tune_cache_save(const char* path);
const char* q2x_build_id(void);

/*
 * Read the device status word of the last call that used `workspace`
 * (synchronises `stream`).  device_flags: OR of Q2X_FLAG_*; n_degenerate:
 * number of zero-measure elements; n_skipped: elements skipped for a bad box
 * id or vertex index or for non-finite data.  Either output may be NULL.
 */
q2x_status q2x_status_get(const void* workspace, void* stream, uint32_t* device_flags, int64_t* n_degenerate,
                          int64_t* n_skipped);

/* Human-readable name of a q2x_status value. */
const char* q2x_status_string(int status);

/*
 * Kernel timing for measurement.  When enabled, each call records HIP events
 * on its own stream around its recursion kernel and around the whole call;
 * q2x_profile_read synchronises those events and returns, per element kind
 * (arrays of 6 indexed by q2x_kind), the summed recursion-kernel time (ms),
 * the summed whole-call time (ms, bucketing and fix-up included) and the
 * number of calls since the last reset.  Any output pointer may be NULL.
 */
void q2x_profile_enable(int on);
void q2x_profile_reset(void);
q2x_status q2x_profile_read(double* recursion_ms, double* call_ms, int64_t* calls);

/*
 * Peak microbenchmarks of the running GPU (measurement aid; the measured
 * denominators beside the published peaks of the roofline fractions).
 *   which 0: FP64 FMA rate, 1: FP32 FMA rate (non-packed, as the library is
 *   built), both in TFLOP/s; 2: HBM copy bandwidth in GB/s (bytes read +
 *   written), copying the first half of `buffer` to the second.
 *   buffer  device memory (256-byte aligned) the kernels may overwrite: at
 *           least 2 MB for 0/1; for 2 the copy size is buffer_bytes / 2
 *   reps    timed launches (after one warm-up); value: the rate; ms_per_rep:
 *           the average launch time (may be NULL).  Synchronises `stream`.
 */
q2x_status q2x_peak_measure(int which, void* buffer, size_t buffer_bytes, int reps, void* stream, double* value,
                            double* ms_per_rep);

/* Library version string. */
const char* q2x_version(void);

#ifdef __cplusplus
}
#endif

#endif /* Q2X_H */
