/*
 * fmm.h -- C ABI of the MI355X (gfx950) Laplace fast multipole library.
 *
 * The library evaluates, for N charged particles in a cube, the 1/r potential
 *     phi_i = sum_{j != i, x_j != x_i} q_j / |x_i - x_j|
 * and the field E_i = -grad phi_i (or the force F_i = q_i E_i) with the fast
 * multipole method of Yokota & Barba, arXiv:1106.2176: the problem statement
 * of Sec. 2.1 (N sources of a 1/r potential, O(N) instead of O(N^2)), the
 * operator sequence of Fig. 1 and Fig. 3 (P2M, M2M, M2L, L2L, L2P, and the
 * near-field P2P of Sec. 3.1), expansions "truncated after p terms" (Sec. 2.1,
 * read here as spherical-harmonic degrees 0..p-1, i.e. p^2 real coefficients
 * per box), and a uniform octree whose leaves are Morton-indexed boxes at one
 * prescribed level (Sec. 2.2 and the future-directions paragraph of Sec. 5).
 *
 * Conventions shared by every entry point:
 *  - extern "C", plain pointers and sizes; no C++ types cross the ABI and no
 *    exception escapes it.
 *  - "device" pointers are HIP device memory on the current HIP device, owned
 *    by the caller, which must keep them alive until the stream work that
 *    uses them has completed.  "host" pointers are ordinary CPU memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    fmm_build_tree blocks once, until two counters (the level-selection
 *    maximum and the count of invalid positions) have reached the host; the
 *    rest of the build stays queued on `stream`.  fmm_evaluate and
 *    fmm_backward are asynchronous on `stream`.  A tree is used by one stream
 *    at a time.
 *  - Every call returns an fmm_status; after a non-OK status the outputs are
 *    unspecified.  fmm_last_error_message() gives a thread-local description
 *    of the most recent failure on the calling thread.
 *  - Results are deterministic: no floating-point atomics are used, so two
 *    calls with the same inputs and configuration give bitwise equal outputs.
 */
#ifndef FMM_H
#define FMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FMM_ABI_VERSION 1u
#define FMM_P_MAX 16
#define FMM_MAX_LEVEL 10

typedef enum {
    FMM_OK = 0,
    FMM_EINVAL = 1,       /* bad argument: n < 1, p outside [1, FMM_P_MAX], leaf_max < 1,
                             box_size <= 0, max_level outside [0, FMM_MAX_LEVEL], NULL required
                             pointer, unknown dtype/precision, ABI version mismatch */
    FMM_EDOMAIN = 2,      /* a coordinate is not finite or lies outside [lo, lo + size] */
    FMM_ENOMEM = 3,       /* the allocator returned NULL */
    FMM_EDEVICE = 4,      /* a HIP launch, copy or synchronisation failed */
    FMM_EUNSUPPORTED = 5  /* valid request this build does not implement */
} fmm_status;

typedef enum { FMM_F32 = 0, FMM_F64 = 1 } fmm_dtype;

typedef enum {
    /* plain form: every step in FP64 (P2P, P2M/L2P, M2M/L2L, M2L on FP64 MFMA) */
    FMM_PREC_FP64 = 0,
    /* mixed form: P2P in FP32 on leaf-relative coordinates with FP64 merges,
     * M2L as split-BF16 products on MFMA with FP32 accumulation merged into
     * FP64, P2M/L2P and fine-level M2M/L2L in FP32, coarse-level (<= 4096
     * boxes) M2M/L2L and the final far+near sum in FP64 */
    FMM_PREC_MIXED = 1
} fmm_precision;

/* Allocator callbacks: return device memory of `bytes` usable in stream order
 * on `stream`, or NULL on failure (reported as FMM_ENOMEM).  When `alloc` is
 * NULL the library uses hipMallocAsync/hipFreeAsync on the call's stream. */
typedef void *(*fmm_alloc_fn)(size_t bytes, void *stream, void *ctx);
typedef void (*fmm_free_fn)(void *ptr, void *stream, void *ctx);

typedef struct {
    uint32_t abi_version;      /* must equal FMM_ABI_VERSION */
    int32_t p;                 /* expansion order: harmonic degrees 0..p-1, 1 <= p <= 16 */
    int32_t leaf_max;          /* leaf cap: the leaf level is the smallest level l <= max_level
                                  whose fullest box holds <= leaf_max particles (max_level if
                                  none does) */
    int32_t max_level;         /* 0..10; keys are 3*level <= 30 bits */
    int32_t precision;         /* fmm_precision */
    int32_t bf16_splits;       /* mixed form with m2l_fp16 = 0 only: the M2L
                                  operands in 2 (hi+lo, 3 MFMA products) or 3
                                  (hi+mid+lo, 6 products) bf16 parts; 0 selects
                                  3.  Supports p <= 13 with 3 parts and p <= 10
                                  with 2 parts (FMM_EUNSUPPORTED otherwise) */
    double box_lo[3];          /* root cube corner */
    double box_size;           /* root cube edge, > 0 */
    fmm_alloc_fn alloc;        /* optional, see above */
    fmm_free_fn free;
    void *alloc_ctx;
    int32_t profile;           /* nonzero: record HIP events around each stage of
                                  fmm_evaluate (read with fmm_stage_times) */
    uint32_t profile_stages;   /* with profile: bit i selects stage i (numbering
                                  of fmm_stage_times); events are recorded only
                                  at the boundaries of selected stages.  0: all */
    int32_t overlap_near;      /* nonzero: run the near field (P2P) concurrently
                                  with the far field on a stream of the library's
                                  own, forked from and joined back into the
                                  caller's stream within each call (same results);
                                  zero (default): after the far field */
    int32_t graph;             /* nonzero: fmm_evaluate and fmm_backward replay a
                                  HIP graph of their kernel chain.  A call whose
                                  arguments (pointers, flags, stream-independent)
                                  differ from the cached graph's, or that follows
                                  a rebuild that changed the level, the particle
                                  count or the tree's memory, runs eagerly and then
                                  captures the chain on a stream of the library's
                                  own (capture executes nothing); later calls
                                  launch the graph on their stream.  Same kernels,
                                  same results.  Exclusive with `profile`
                                  (FMM_EINVAL). */
    int32_t m2l_fp16;          /* mixed form only: nonzero = the M2L operands in
                                  two IEEE binary16 parts (3 MFMA products, about
                                  22 bits per operand) instead of bf16_splits
                                  bf16 parts.  Operators and multipoles are
                                  scaled degree by degree by powers of two (the
                                  size of the regular harmonics over a box), the
                                  multipoles also per level by the power of two
                                  that puts the level's largest one just below
                                  2^14; the results are scaled back exactly.
                                  Supports every p <= 16. */
    int32_t m2l_rotation;      /* FP64 form only (FMM_EINVAL otherwise), p >= 2:
                                  nonzero = M2L by rotation: the multipole rotated
                                  so that the offset lies on the z axis,
                                  translated along z and rotated back, O(p^3)
                                  per pair instead of the dense O(p^4) product
                                  (same results to round-off).  Its tables are
                                  made on the first build that asks for them (a
                                  quadrature per offset, about a second of host
                                  time at p = 16) and kept per device and p. */
    int32_t adaptive;          /* not with m2l_rotation, nor with the bf16
                                  encodings (m2l_fp16 = 0) of the mixed form
                                  (FMM_EUNSUPPORTED):
                                  nonzero = the adaptive octree of the
                                  construction Sec. 5 names beside the uniform
                                  one.  A box is split while it holds more than
                                  leaf_max particles and its level is below
                                  max_level; empty children are dropped, so
                                  leaves sit at many levels.  The build sorts
                                  the particles by their key at max_level (a
                                  radix sort of the keys, no bin per finest
                                  box) and finds box ranges in the sorted keys
                                  through a table of 8^min(max_level, 7) + 1
                                  words (8 MiB at most), so a deeper cap costs
                                  little.  The interactions follow the
                                  U/V/W/X lists of the adaptive FMM: U(b), b a
                                  leaf: b and the leaves touching it (P2P); V(b):
                                  the children of the colleagues of b's parent
                                  not touching b (M2L, the dense FP64 product
                                  on the matrix cores); W(b), b a leaf: the
                                  descendants of b's colleagues that do not
                                  touch b but whose parent does (the multipole
                                  evaluated at b's particles, M2P); X(b): the
                                  leaves c with b in W(c) (each particle of c
                                  expanded about b's centre, P2L).  Two boxes
                                  touch when their closed cubes intersect and
                                  neither contains the other.  Every step is
                                  FP64 except, in the mixed form, the M2L (the
                                  binary16 encoding described at m2l_fp16,
                                  with one operand scale per level), the
                                  P2P pairs (FP32 on FP64 differences, FP64
                                  merges) and the P2M, L2P, P2L and M2P
                                  terms (FP32 per particle and box, summed
                                  in FP64).
                                  fmm_backward runs the transposed chain over
                                  the same lists; the build
                                  blocks once per tree level and once more at
                                  the end, until a few counts have reached the
                                  host. */
    int32_t reserved[1];       /* zero */
} fmm_config;


/* Fill `cfg` with defaults: p = 8, leaf_max = 64, max_level = 10, mixed
 * precision with the binary16 M2L encoding (m2l_fp16 = 1; bf16_splits = 3
 * when it is switched off), root cube [0,1)^3, library allocator, no
 * profiling. */
void fmm_config_default(fmm_config *cfg);

typedef struct fmm_tree fmm_tree; /* opaque, library-owned */

typedef struct {
    int32_t levels;            /* leaf level L (the tree has levels 0..L); adaptive
                                  tree: its deepest level */
    int32_t p;
    int64_t n;
    int64_t n_leaves;          /* 8^L; adaptive tree: its (non-empty) leaves */
    int64_t max_leaf_count;    /* fullest leaf */
    int64_t p2p_pairs;         /* ordered pairs (i, j), i != j, in each other's near field
                                  (27-leaf neighbourhood; adaptive tree: the U lists),
                                  i.e. P2P interactions evaluated */
    int64_t m2l_pairs;         /* (target box, source box) M2L translations over all levels
                                  (adaptive tree: the V lists) */
    size_t workspace_bytes;    /* device memory held by the tree */
    int64_t n_boxes;           /* boxes of all levels (uniform tree: sum of 8^l) */
    int64_t m2p_evals;         /* adaptive tree: (particle, box) pairs of the W
                                  lists, i.e. multipole evaluations; 0 otherwise */
    int64_t p2l_evals;         /* adaptive tree: (particle, box) pairs of the X
                                  lists, i.e. particle-to-local expansions */
} fmm_tree_info_t;

/*
 * Build the octree for `n` particles (Sec. 2.1 hierarchical subdivision;
 * Morton keys and the sorted start/offset particle layout of Sec. 5).
 *   pos    device [n][3] row-major, in `dtype`.  The build's sort kernels
 *          read it after the call has returned, in stream order on `stream`:
 *          keep it valid and unchanged until that stream work has completed.
 *          The tree keeps its own copy (sorted, leaf-relative), so later
 *          calls on the tree do not read `pos`.
 *   out    receives the tree.  If *out is a tree previously built by this
 *          library, it is rebuilt in place and its memory reused when large
 *          enough; its p, precision, M2L encoding (bf16_splits, m2l_fp16;
 *          mixed form), tree kind (adaptive), dtype and allocator callbacks
 *          (alloc, free, alloc_ctx) must equal the ones it was created with, else the call returns FMM_EINVAL before any
 *          allocation or launch and leaves the tree as it was.  Otherwise *out
 *          must be NULL and a new tree is created.  The translation tables of
 *          p (made once per device and p, held until the process ends) are
 *          ready when the call returns.
 * Steps: Morton key per particle with the leaf-occupancy histogram at the
 * predicted level, level selection (one host wait; a finer level is tried
 * when the predicted one's fullest leaf exceeds leaf_max), exclusive scan of
 * leaf counts, stable counting sort (ties keep input order) and a gather of
 * leaf-relative coordinates.  An adaptive tree (cfg.adaptive) sorts at
 * max_level, then builds its boxes level by level and its lists; it waits
 * for the host once per level and once more at the end.
 * Errors: FMM_EINVAL, FMM_EDOMAIN (detected at the synchronisation; a
 * coordinate equal to lo + size is clamped into the last box), FMM_ENOMEM
 * (the allocator callback returned NULL, or hipMallocAsync failed),
 * FMM_EDEVICE.  On error a newly created tree is destroyed and *out is set
 * to NULL; a tree passed in for reuse stays valid for fmm_tree_destroy only
 * (except after the FMM_EINVAL of a settings mismatch, which leaves it
 * untouched).
 */
fmm_status fmm_build_tree(const fmm_config *cfg, int64_t n, int32_t dtype, const void *pos,
                          void *stream, fmm_tree **out);

#define FMM_VEC_NONE 0  /* no vector output */
#define FMM_VEC_FIELD 1 /* vec = E_i = -grad phi at x_i */
#define FMM_VEC_FORCE 2 /* vec = F_i = q_i E_i */
/* optional part selection, OR-ed into flags (default: both parts) */
#define FMM_PART_NEAR_ONLY 4 /* only the P2P (near-field) part */
#define FMM_PART_FAR_ONLY 8  /* only the P2M..L2P (far-field) part */

/*
 * Evaluate potentials (and optionally fields or forces) for charges `q`
 * (device [n] in the tree's dtype) at the tree's particles, in the caller's
 * particle order: P2M, M2M (upward sweep), M2L at every level >= 2 (the
 * levels are independent and run in one launch, Sec. 5), L2L
 * (downward sweep), L2P, P2P and the far + near sum (Fig. 1, Fig. 3).
 *   phi  device [n] output (tree dtype), required.
 *   vec  device [n][3] output (tree dtype), required unless the vector
 *        kind (flags & 3) is FMM_VEC_NONE.
 *   flags  vector kind (FMM_VEC_*) OR-ed with at most one FMM_PART_* bit,
 *        which restricts the output to the near or far part (for per-part
 *        verification; the work of the other part is skipped).
 * Errors: FMM_EINVAL (NULL tree/q/phi, bad flags), FMM_ENOMEM, FMM_EDEVICE.
 */
fmm_status fmm_evaluate(fmm_tree *tree, const void *q, void *phi, void *vec, int32_t flags,
                        void *stream);

/*
 * fmm_evaluate for callers that cannot allocate device memory: code under
 * HIP graph capture, serving loops and harnesses that forbid hipMalloc.
 * Same arguments, outputs and errors as fmm_evaluate, and the same kernels in
 * the same order (bitwise equal results), but every buffer of the call (near
 * and far partial results, multipole and local coefficient grids, M2L
 * operand grids and K-split partial sums) is carved from the library's
 * static device array of FMM_NOALLOC_SCRATCH_BYTES instead of the tree's
 * workspace: the call allocates nothing, creates no stream or event and
 * captures no graph.  It runs the near field after the far field on
 * `stream` whatever cfg.overlap_near says, and records no profiling events.
 * The tree itself comes from fmm_build_tree, which does allocate (its
 * sorted particles and, for a far field, the translation tables of p).
 *   - A tree whose evaluation needs more scratch than the array holds is
 *     rejected with FMM_EINVAL before any launch (the message gives the
 *     size).  Roughly: 64 B per particle plus the coefficient and M2L grids
 *     of the levels, e.g. N <= 10^5 at p = 10, leaf_max = 64.
 *   - Every call on one device uses that device's one array, which keeps
 *     the last call's contents; nothing in it needs clearing.  Calls that
 *     overlap on one device (on different streams or host threads) race
 *     on it: the caller orders them.
 *   - Each device the library runs on holds its array from the library's
 *     load until the process ends.
 */
#define FMM_NOALLOC_SCRATCH_BYTES (64u << 20)
fmm_status fmm_evaluate_noalloc(fmm_tree *tree, const void *q, void *phi, void *vec, int32_t flags,
                                void *stream);

/*
 * Gradient of the weighted-potential loss  Loss = sum_i w_i phi_i  of the
 * FMM as computed by fmm_evaluate on the same tree and charges, with respect
 * to the charges and positions.  Hand-written adjoint: the transposed
 * operator chain L2P^T, L2L^T (upward), M2L^T, M2M^T (downward), P2M^T with
 * its position derivative, plus P2P with charges w; leaf assignments are
 * held fixed (they are piecewise constant in the positions).
 *   q          device [n] charges used in the forward evaluation.
 *   w          device [n] dLoss/dphi.
 *   field_fwd  device [n][3] the field E (FMM_VEC_FIELD) of the forward
 *              evaluation with charges q on this tree.
 *   grad_q     device [n] output dLoss/dq, or NULL.
 *   grad_pos   device [n][3] output dLoss/dx, or NULL.
 *   grad_q_i   = psi_i + phi_w,i   (adjoint far potential + P2P potential of w)
 *   grad_pos_i = -(w_i E_i + q_i E_w,i)
 * All arrays are in the tree's dtype and the caller's particle order.
 * Errors: FMM_EINVAL, FMM_ENOMEM, FMM_EDEVICE.
 */
fmm_status fmm_backward(fmm_tree *tree, const void *q, const void *w, const void *field_fwd,
                        void *grad_q, void *grad_pos, void *stream);

/* Sizes and work counts of a built tree (host struct, filled synchronously;
 * a small kernel counts the pairs, and on a uniform tree the M2L pairs are
 * counted on the host). */
fmm_status fmm_tree_info(const fmm_tree *tree, fmm_tree_info_t *info);

/* Stage timings (milliseconds) on a tree built with cfg.profile != 0: HIP
 * events are recorded around each stage on the stream of every
 * fmm_evaluate / fmm_backward, and this returns the mean over the most recent
 * min(calls, 32) calls since the tree was created or fmm_stage_times_reset
 * (rebuilding the tree does not reset it).  Waits for those calls' events.
 * Stages, in order:
 *   0 gather   1 P2M   2 M2M   3 pack (M2L operand)   4 M2L   5 L2L
 *   6 L2P      7 P2P   8 combine
 * On an adaptive tree stage 3 is P2L (the X lists, and in the mixed form
 * the M2L operand pack) and stage 6 holds L2P and M2P (the W lists).
 * A uniform tree's forward evaluation ends its last kernel with the combine
 * (P2P's, or L2P's with overlap_near), so its stage 8 is only the event
 * markers; the adaptive tree and fmm_backward run a combine kernel there.
 * `ms` receives min(n_stages, 9) values; stages outside cfg.profile_stages
 * (when it is nonzero) receive NaN.  FMM_EINVAL if profiling is off or no
 * call was recorded. */
fmm_status fmm_stage_times(const fmm_tree *tree, double *ms, int32_t n_stages);

/* Forget the recorded stage timings of `tree` (the next fmm_stage_times
 * averages only calls made after this one). */
fmm_status fmm_stage_times_reset(fmm_tree *tree);

/* Copy the tree's sorting results to host memory (any pointer may be NULL):
 * perm[n] (sorted position -> input index, uint32), leaf_start[n_leaves + 1]
 * (uint32; the uniform tree's 8^L leaves in Morton order, an adaptive tree's
 * leaves in particle order).  Synchronous. */
fmm_status fmm_tree_export(const fmm_tree *tree, uint32_t *perm, uint32_t *leaf_start);

/* The boxes and interaction lists of an adaptive tree (cfg.adaptive), copied
 * to host memory; synchronous.  FMM_EINVAL on a uniform tree.
 *   sizes   host int64[6] out: boxes, then the item counts of the U, V, W
 *           and X lists, then the deepest level.  Call with the other
 *           pointers NULL to size the arrays.
 *   boxes   host int32 [boxes][8] or NULL: level, ix, iy, iz (integer box
 *           coordinates at that level), start, end (the box's particles are
 *           sorted positions [start, end)), parent (-1 for the root), leaf
 *           (0/1).  Boxes are numbered breadth first, Morton order within a
 *           level, box 0 the root.
 *   perm    host uint32 [n] or NULL: sorted position -> input index.
 *   list_start  host int64 [4][boxes + 1] or NULL: list k (U, V, W, X) of
 *           box b is items[off_k + list_start[k][b], off_k +
 *           list_start[k][b + 1]), off_k the item counts of the lists
 *           before k (list_start[k][0] = 0).
 *   items   host int32 [sum of the four counts] or NULL: box ids; the order
 *           within a list is unspecified. */
fmm_status fmm_tree_export_adaptive(const fmm_tree *tree, int64_t *sizes, int32_t *boxes, uint32_t *perm,
                                    int64_t *list_start, int32_t *items);

/* Release all device memory of the tree (stream ordered on the build stream).
 * NULL is ignored. */
void fmm_tree_destroy(fmm_tree *tree);

/* Host-side translation operators in the library's real basis, FP64,
 * row-major [rows][cols] with rows = cols = p^2 (host, synchronous, no GPU):
 *   kind 0: M2M child -> parent, child octant `index` in 0..7 (bit 0 x, bit 1 y, bit 2 z)
 *   kind 1: L2L parent -> child, child octant `index`
 *   kind 2: M2L, offset index `index` = (ox+3) + 7 (oy+3) + 49 (oz+3), target minus source
 *           in box widths, |o|_inf in 2..3
 *   kind 3: the rotation D of the rotation-based M2L for offset `index` (any nonzero
 *           offset): rho(Q u) = D rho(u) for the rotation Q that takes the offset's
 *           direction to +z; block diagonal by degree
 *   kind 4: the M2L matrix Tz of the offset (0, 0, |o|) for offset `index`; couples
 *           only coefficients of equal order and kind, and M2L(o) = D^T Tz D
 * Basis: multipole vector mu = sum_j q_j rho(u_j) and potential
 * phi(x) = (1/w) ell . rho(u) with u = (x - c)/w, rho the real and imaginary
 * parts of the regular solid harmonics R_n^m (m >= 0) defined by
 * sum_{n,m} R_n^m(x) s^n t^m = exp(s (z + (x+iy)/(2t) - t (x-iy)/2)).
 * `out` receives p^4 doubles.  For inspection and host tests. */
fmm_status fmm_operator_host(int32_t p, int32_t kind, int32_t index, double *out);

const char *fmm_status_string(fmm_status s);
const char *fmm_last_error_message(void);

#ifdef __cplusplus
}
#endif

#endif /* FMM_H */
