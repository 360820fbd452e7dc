/*
 * fmm.h -- C ABI of the MI355X (gfx950) balanced-tree fast multipole library
 * for the 3D harmonic kernel.
 *
 * The library evaluates, for N source points x_i with charges q_i,
 *     phi_i = sum_{j != i} q_j / |x_i - x_j|           (Section 2, eq. (2.1))
 *     E_i   = -grad phi_i = sum_{j != i} q_j (x_i - x_j) / |x_i - x_j|^3
 * with the balanced-tree FMM of Bull & Engblom (Section 2): a tree of L
 * levels of 8-way median splits (Section 2.1.2, eta = 1), theta-criterion
 * connectivity (Section 2.1.1, eq. (2.2)), P2M/M2M upward (Algorithm 1),
 * M2L/L2L downward (Algorithm 3) and L2P/P2P evaluation (Algorithm 4).
 * Pairs of points at distance zero contribute nothing.
 *
 * Conventions shared by every entry point:
 *  - Point data are structure-of-arrays, IEEE binary64, in the caller's order.
 *  - Arrays named "device" are HIP device pointers that must stay valid until
 *    the work enqueued on `stream` has completed; the library never frees
 *    caller memory.  Arrays named "host" are ordinary host memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *  - Every function returns FMM_OK (0) or a negative fmm_status; on failure
 *    no output is defined and fmm_last_error() returns a message (per
 *    calling thread).  A failed call frees every device allocation it made
 *    (stream-ordered on its stream) and leaves no new handle behind; a tree
 *    passed to a failed evaluation stays valid and can be evaluated again or
 *    freed.  Argument checks happen before any work is enqueued.  No
 *    exception crosses the ABI.
 *  - Device memory comes from the allocator set by fmm_set_allocator, else
 *    from the device's default stream-ordered pool.
 *  - A tree handle may be used by one thread at a time.  Different handles
 *    may be used by different threads at once, each on its own stream
 *    (blocking or non-blocking).  A tree may be evaluated on any stream: an
 *    evaluation on another stream than the build's waits (on the device) for
 *    the build, and fmm_free waits (on the device) for every evaluation
 *    enqueued on the tree before its memory is released.
 *  - The first evaluation at an order p on a device makes that order's
 *    operator tables (kept until the process ends) and waits for `stream`
 *    once, so that the tables are on the device before any stream uses them;
 *    every later evaluation is fully asynchronous.
 */
#ifndef FMM_H
#define FMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fmm_tree fmm_tree;

typedef enum fmm_status {
  FMM_OK = 0,
  FMM_EINVAL = -1,       /* invalid argument (NULL pointer, range, non-finite coordinate) */
  FMM_ENOMEM = -2,       /* device or host allocation failed */
  FMM_EDEVICE = -3,      /* HIP runtime error (no device, launch failure, ...) */
  FMM_EUNSUPPORTED = -4  /* valid request that the library does not support */
} fmm_status;

#define FMM_MAX_LEVELS 8
#define FMM_MAX_ORDER 20
#define FMM_MAX_POINTS 2147483647LL

/* Result selection for fmm_evaluate_tree_parts (Algorithm 4 splits the
 * evaluation into the far field, L2P, and the near field, P2P). */
#define FMM_PART_NEAR 1
#define FMM_PART_FAR 2
#define FMM_PART_ALL 3

/*
 * Device allocator hook (the paper's solver is meant as a plug-in for other
 * applications, Section 2.2.2: a host application brings its own memory
 * manager, e.g. the caching allocator of PyTorch).
 *   alloc(bytes, stream, user)  returns device memory usable by work enqueued
 *                               on `stream` (a hipStream_t), or NULL on failure;
 *                               the library then fails the call with
 *                               FMM_ENOMEM and frees what it allocated.
 *   free(ptr, stream, user)     releases a block; work enqueued on `stream`
 *                               before the call may still read it, so a
 *                               stream-ordered allocator must not hand the
 *                               block out again before that work completes.
 * Both must be thread-safe when handles are used from several threads.
 * Passing alloc = free = NULL restores the default pool.  A tree keeps the
 * allocator it was built with and is freed through it; scratch memory of an
 * evaluation comes from the allocator set at the time of the call.  Returns
 * FMM_EINVAL when exactly one of alloc and free is NULL.
 */
typedef void* (*fmm_alloc_fn)(size_t bytes, void* stream, void* user);
typedef void (*fmm_free_fn)(void* ptr, void* stream, void* user);
fmm_status fmm_set_allocator(fmm_alloc_fn alloc, fmm_free_fn free, void* user);

/*
 * Builds the tree (Section 2.1.2 and Algorithm 2 on one process).
 *   x, y, z  device, n doubles each: point coordinates (finite, |coord| <= 1e300).
 *   n        1 <= n <= FMM_MAX_POINTS.
 *   levels   0 <= levels <= FMM_MAX_LEVELS; the tree has 8^levels leaves.
 *   theta    0 <= theta < 1, the parameter of eq. (2.2).
 *   out      host: receives a new handle that owns all device workspace.
 * The coordinates are read during the call only (the handle keeps a copy in
 * tree order).  The call synchronises `stream` once per level (interaction
 * list sizes are read back to size the lists).  Non-finite coordinates give
 * FMM_EINVAL.
 */
fmm_status fmm_build(const double* x, const double* y, const double* z, int64_t n, int levels, double theta,
              void* stream, fmm_tree** out);

/*
 * Evaluates potential and field for charges q on a built tree (Algorithm 1:
 * P2M, M2M, then Algorithm 3 and Algorithm 4).
 *   q                      device, n doubles, caller's point order.
 *   p                      0 <= p <= FMM_MAX_ORDER: expansions keep degrees 0..p.
 *   pot, ex, ey, ez        device, n doubles each, written in the caller's order.
 * Fully asynchronous on `stream`; may be called many times on one tree.
 */
fmm_status fmm_evaluate_tree(fmm_tree* tree, const double* q, int p, double* pot, double* ex, double* ey, double* ez,
                      void* stream);

/* As fmm_evaluate_tree, but writes only the near-field (P2P) part, the
 * far-field (L2P) part, or both (FMM_PART_*): used to check each half of
 * Algorithm 4 separately. */
fmm_status fmm_evaluate_tree_parts(fmm_tree* tree, const double* q, int p, int parts, double* pot, double* ex, double* ey,
                            double* ez, void* stream);

/* Arithmetic of the evaluation (fmm_evaluate_tree_ex). */
#define FMM_PREC_F64 0   /* every step in IEEE binary64 */
#define FMM_PREC_MIXED 1 /* M2L in binary32 (see below); the rest in binary64 */
#define FMM_PREC_F32 2   /* M2L and the near field (P2P) in binary32 (see below) */

/*
 * As fmm_evaluate_tree_parts, with a choice of arithmetic.  FMM_PREC_MIXED
 * evaluates the dominant M2L step (Section 2.1.3) in binary32 for orders
 * p <= 15: the multipoles are scaled by powers of their box radius, so that
 * every translation factor (r_source/rho)^n, (r_target/rho)^j is below one;
 * the rotations and the z-axis translation run on the binary32 matrix cores
 * (one pair per lane up to order 14, 16-pair tiles at order 15); the pair
 * results of a batch are summed in binary32 and the batches in binary64;
 * the local expansions are unscaled into binary64.  The tree, P2M, M2M, L2L,
 * L2P and the near field (P2P) stay in binary64, as do all final sums.  The
 * far field then differs from the binary64 one by about 1e-7 relative
 * (normwise) on the workloads tested.  Higher orders run in binary64.
 * FMM_PREC_F32 also evaluates the near field (P2P, Algorithm 4) in binary32:
 * coordinates relative to the target leaf's cell centre (formed in binary64,
 * then rounded), the binary32 reciprocal square root, binary32 sums over each
 * staged chunk of sources added into Kahan-compensated binary32 totals, which
 * are widened to binary64 before the far field is added.  Its field differs
 * from the binary64 one by up to a few 1e-5 relative on clustered clouds
 * (cancellation among near contributions): it is meant for loose tolerances.
 * Two distinct points whose relative binary32 coordinates coincide count as
 * coincident.  Returns FMM_EINVAL for an unknown precision.
 */
fmm_status fmm_evaluate_tree_ex(fmm_tree* tree, const double* q, int p, int parts, int precision, double* pot, double* ex,
                         double* ey, double* ez, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, hosts that forbid allocation): as
 * fmm_evaluate_tree_ex, but every scratch buffer of the evaluation is carved
 * from one fixed device array of 64 MiB per GPU, held from the library's
 * load until the process ends.  The call allocates nothing, records no event
 * and never waits on the host, so it may be captured into a HIP graph.
 *   - FMM_EINVAL when the evaluation needs more scratch than the array holds
 *     (fmm_tree_bytes' eval_bytes plus alignment slack, checked before any
 *     work is enqueued; about 2e5 points at 4 levels and p = 12 fit).
 *   - FMM_EUNSUPPORTED when the operator tables of order p are not on the
 *     device yet: one evaluation at order p through an allocating entry point
 *     makes them.
 *   - Every call on a GPU shares that GPU's array, and the array keeps the
 *     last call's contents: calls that overlap on one GPU (other streams,
 *     other threads, graph replays in flight) race and give wrong results.
 *     Order them on one stream or wait in between.
 *   - The tree's build must be complete on the device (or ordered before the
 *     call on `stream`), and the tree must not be freed while work enqueued
 *     by this call is pending: unlike the other entry points this one does
 *     not track the streams that use the tree.
 *   - Phase timing (fmm_set_profiling) does not cover this call.
 */
fmm_status fmm_evaluate_tree_noalloc(fmm_tree* tree, const double* q, int p, int parts, int precision, double* pot,
                                     double* ex, double* ey, double* ez, void* stream);

/*
 * fmm_build with the split parameter eta and separate evaluation targets
 * (Section 2.1.2; the convergence test of Section 3.1 evaluates at points
 * that are not sources).
 *   x, y, z, n, levels, theta   as in fmm_build.
 *   tx, ty, tz   device, m doubles each: target coordinates (finite,
 *                |coord| <= 1e300); NULL allowed when m = 0.  Read during
 *                the call only.
 *   m            0 <= m <= FMM_MAX_POINTS.
 *   eta          0 <= eta <= 1.  Every box is split by three successive
 *                bisections along the longest edge of the current cell, at
 *                the plane (1 - eta) * (cell midpoint) + eta * (median plane),
 *                where the median plane lies midway between the two middle
 *                coordinates.  eta = 1 is fmm_build's median split (the low
 *                side gets floor(n/2) points, ties by input order); for
 *                eta < 1 the points strictly below the plane form the low
 *                side, so children may hold unequal numbers of points or none.
 * The root cell is the bounding box of the sources and the targets.  Each
 * target belongs to the leaf reached from the root by taking, at every
 * level, the first child (in child order) whose closed cell holds it.
 * Synchronises `stream` as fmm_build does, plus once for the targets; for
 * eta < 1 also once per bisection round, from the second, while every
 * segment of the round before held at least 8192 points and the round has
 * at most 512 segments (the segment sizes choose the round's kernels).
 */
fmm_status fmm_build_ex(const double* x, const double* y, const double* z, int64_t n, const double* tx, const double* ty,
                 const double* tz, int64_t m, int levels, double theta, double eta, void* stream, fmm_tree** out);

/*
 * Potential and field at the tree's m separate targets, for charges q on
 * its sources: the far field from the local expansion of the target's leaf
 * (L2P), the near field from the sources of the leaves strongly connected to
 * it (P2P); a source at the target's own position contributes nothing.
 *   q                  device, n doubles, caller's source order.
 *   p, parts, precision  as in fmm_evaluate_tree_ex.
 *   pot, ex, ey, ez    device, m doubles each, written in the caller's
 *                      target order (may be NULL when m = 0).
 * Fully asynchronous on `stream`.  A tree without targets does nothing.
 */
fmm_status fmm_evaluate_targets(fmm_tree* tree, const double* q, int p, int parts, int precision, double* pot, double* ex,
                         double* ey, double* ez, void* stream);

/* Number of separate targets of a tree and, when `leaf` (host, m int32) is
 * not NULL, the leaf that holds each of them (caller's target order). */
fmm_status fmm_tree_targets(const fmm_tree* tree, int64_t* m, int32_t* leaf);

/* One-shot form: fmm_build + fmm_evaluate_tree + fmm_free.  All arrays are
 * device arrays of n doubles. */
fmm_status fmm_evaluate(const double* x, const double* y, const double* z, const double* q, int64_t n, double theta, int p,
                 int levels, double* pot, double* ex, double* ey, double* ez, void* stream);

/* Releases a handle and its device memory (stream-ordered on the stream of the
 * last call that used it).  NULL is accepted. */
fmm_status fmm_free(fmm_tree* tree);

/* Message describing the last failure on the calling thread ("" if none). */
const char* fmm_last_error(void);

/* ---- Introspection (used by parity tests; synchronous, host outputs) ---- */

/* n, levels and theta of a tree (any output pointer may be NULL). */
fmm_status fmm_tree_info(const fmm_tree* tree, int64_t* n, int* levels, double* theta);

/* host perm[n]: original index of the point at each tree position.  Points
 * of every leaf occupy a contiguous range in ascending original index. */
fmm_status fmm_tree_perm(const fmm_tree* tree, int32_t* perm);

/* host geom[8^level * 10]: per box lo[3], hi[3], centre[3], radius (cell
 * centre and half-diagonal, Section 2.1.1), and host start[8^level + 1]:
 * point range of each box in tree order (either pointer may be NULL). */
fmm_status fmm_tree_boxes(const fmm_tree* tree, int level, double* geom, int64_t* start);

/* Connectivity of one level (Section 2.2.1: per-level sparse connectivity),
 * as CSR by target box, ascending source box index within each row.
 *   kind 0 = strongly connected (incl. the box itself), 1 = weakly connected.
 *   nnz      host, receives the number of entries.
 *   offsets  host, 8^level + 1 entries, or NULL.
 *   idx      host, nnz entries (box indices of that level), or NULL. */
fmm_status fmm_tree_lists(const fmm_tree* tree, int level, int kind, int64_t* nnz, int64_t* offsets, int32_t* idx);

/* Work counts of a tree: M2L translations (weak pairs over all levels) and
 * P2P interactions (ordered point pairs in strongly connected leaves, minus
 * the n self pairs). */
fmm_status fmm_tree_stats(const fmm_tree* tree, int64_t* m2l_pairs, int64_t* p2p_pairs);

/* ---- Phase timing ------------------------------------------------------ */

/* Phases timed with HIP events on the call's stream when profiling is on. */
enum fmm_phase {
  FMM_PH_TREE = 0,  /* bounding box, median bisections, box geometry */
  FMM_PH_LISTS,     /* theta-criterion lists */
  FMM_PH_P2M,
  FMM_PH_M2M,
  FMM_PH_M2L,
  FMM_PH_L2L,
  FMM_PH_L2P,
  FMM_PH_P2P,       /* near field, combined with L2P and scattered to the caller's order */
  FMM_NUM_PHASES
};

/* Turns event timing on (1) or off (0) for subsequent calls on this thread. */
fmm_status fmm_set_profiling(int on);

/* host ms[FMM_NUM_PHASES]: durations of the phases of the most recent
 * fmm_build / fmm_evaluate_tree on this thread (0 for phases not run).
 * Waits for those events. */
fmm_status fmm_last_timings(double* ms);

/* Device memory of a built tree: *tree_bytes (may be NULL) receives the
 * bytes the handle owns (tree, lists, plans); *eval_bytes (may be NULL) the
 * peak scratch bytes one evaluation at order p and the given precision
 * allocates on top (sources, and the separate targets when the tree has
 * them).  Unlike fmm_bytes_estimate these are exact, for any point cloud. */
fmm_status fmm_tree_bytes(const fmm_tree* tree, int p, int precision, size_t* tree_bytes, size_t* eval_bytes);

/* Estimate of the device bytes a build + evaluation needs, for admission
 * control before a build.  The interaction lists are sized as for a uniform cloud, so the
 * estimate bounds roughly uniform data from above; on strongly clustered
 * clouds the lists can be more than ten times larger (2^27 Plummer points of
 * scale radius 0.02 at 7 levels: 2.2e10 weak pairs against 1.8e9 list
 * entries in the estimate).  Returns 0 for arguments that fmm_build rejects. */
size_t fmm_bytes_estimate(int64_t n, int levels, double theta, int p);

#ifdef __cplusplus
}
#endif

#endif /* FMM_H */
