/*
 * pkifmm.h -- C interface of the periodic kernel-independent FMM evaluation
 * pass for AMD Instinct MI355X (gfx950).
 *
 * The library evaluates the periodic sum of the paper's problem statement
 * (Yan & Shelley, "Flexibly imposing periodicity in kernel independent FMM:
 * a multipole-to-local operator approach", Section 2, Eq. pfmmDef):
 *
 *     q_t = sum_{p in P} sum_s K(x_t - (y_s + p L)) phi_s ,
 *
 * where P is the lattice of periodic shifts (components only along the
 * periodic axes), L the edge of the cubic box [0, L)^3, and K one of the
 * paper's example kernels (Section 2, Eq. kexamples):
 *     PKIFMM_LAPLACE     K(r) = 1 / (4 pi |r|)                          k = 1
 *     PKIFMM_STOKES      K(r) = (1/(8 pi)) (I/|r| + r r^T / |r|^3)       k = 3
 * A pair at exactly zero separation contributes nothing.  The targets are the
 * sources unless a separate target set is given (pkifmm_set_points).  Periodic sums that only converge conditionally are taken in the
 * following sense: singly (SP) and doubly (DP) periodic -- the limit of
 * symmetric image truncations, which requires zero net density (Section 2,
 * Eq. compatcondition, neutrality); each image term is taken relative to the
 * kernel's value at its lattice point, which fixes the additive constant;
 * triply periodic (TP) -- the Ewald sum with the k = 0 Fourier mode removed
 * (zero mean; Section 3, triply periodic Stokes, which allows a net force).
 *
 * The method is Algorithm 2 of the paper with its step d folded into the
 * tree: an octree covers the original box and its images with |p|_inf <= 1;
 * the far field (|p|_inf >= 2) is one precomputed periodic operator applied to
 * the root's upward equivalent density and added to the root's downward check
 * potential.  For triply periodic Laplace the zero-mean sum carries a uniform
 * neutralising background (the one-component-plasma remark of the paper's
 * Discussions): its far kernel is harmonic plus |y - c|^2 / 6 in the source
 * position, a part no equivalent density reproduces, so the constant it adds,
 * (sum_s phi_s |y_s - c|^2 - sum_j phi^{B0,u}_j |y_j - c|^2) / 6 (c the box
 * centre), is added to every target.
 *
 * Conventions for every call:
 *   * return value: 0 (PKIFMM_OK) or a negative status code below;
 *   * device pointers are HIP device memory owned by the caller, which must
 *     keep them alive until the stream work completes; the library never
 *     frees them;
 *   * `stream` is a hipStream_t passed as void* (NULL = the null stream);
 *   * a plan is used by one host thread and one stream at a time.
 */
#ifndef PKIFMM_H
#define PKIFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pkifmm_plan pkifmm_plan;

/* kernels */
#define PKIFMM_LAPLACE 1
#define PKIFMM_STOKES 2

/* periodic axes (bit mask): 0 = free space, one axis = singly periodic, two axes = doubly
 * periodic, X|Y|Z = triply periodic (every combination, both kernels) */
#define PKIFMM_PERIODIC_X 1u
#define PKIFMM_PERIODIC_Y 2u
#define PKIFMM_PERIODIC_Z 4u

/* arithmetic of the evaluation pass */
#define PKIFMM_FP64 0        /* every step in double precision */
#define PKIFMM_MIXED 1       /* near field (U lists and direct W/X leaf pairs) in float32 on
                                exact integer separations, with float64 partial-sum
                                accumulation; the V-list M2L (Section 2.2) on int8 digit slices
                                of the operators and upward densities (6 base-2^7 digits each,
                                products accumulated exactly in int32, recombined in float64:
                                about 42 significant bits); S2M, X, M2M, L2L, the solves, the
                                root far field, W and L2T in float64.  Target: 1e-6 relative L2
                                against the float64 result.  Points are resolved to 2^-29 of
                                their leaf's edge: two points closer than that in every
                                coordinate may meet as coincident points (contributing nothing
                                to each other; pkifmm_set_points detects such inputs and guards
                                every pair then).  Density magnitudes outside about
                                1e-28 ... 1e29 are outside this form's range: the near field
                                rounds densities to float32 and its terms reach 2^-31 ... 2^31
                                times them (PKIFMM_FP64 has neither limit) */

/* status codes */
#define PKIFMM_OK 0
#define PKIFMM_ERR_INVALID_ARG -1
#define PKIFMM_ERR_OUT_OF_BOX -2     /* a coordinate on a non-periodic axis outside [0, L], or not finite */
#define PKIFMM_ERR_INCOMPATIBLE -3   /* SP or DP input with a non-zero net density: |sum phi| > 1e-12 sum |phi|
                                        for some problem, right-hand side and component */
#define PKIFMM_ERR_UNSUPPORTED -4    /* kernel x periodicity without a far-field operator (none at present) */
#define PKIFMM_ERR_OOM -5
#define PKIFMM_ERR_HIP -6
#define PKIFMM_ERR_NO_POINTS -7      /* evaluate before set_points */
#define PKIFMM_ERR_NUMERICS -8       /* operator construction failed its self-check */
#define PKIFMM_ERR_CAPACITY -9       /* pkifmm_evaluate_noalloc: the workspace exceeds its static array */
#define PKIFMM_ERR_CACHE_CORRUPT -10 /* an operator cache file fails its checks (magic, version, key,
                                        sizes, checksum, or the solves' backward-error check) */

typedef struct {
    int kernel;                  /* PKIFMM_LAPLACE or PKIFMM_STOKES */
    unsigned periodic_mask;      /* 0, one axis, two axes, or X|Y|Z */
    int p;                       /* surface points per cube edge, 4..16 */
    int max_pts_per_leaf;        /* s: a box holding more points is split */
    int precision;               /* PKIFMM_FP64 or PKIFMM_MIXED */
    double box_length;           /* L > 0 */
    double svd_rel_threshold;    /* singular values <= this * s_max are dropped from the
                                    check-to-equivalent solves (Appendix B's (V S^+)(U^T q), whose
                                    cutoff the paper leaves free); 0 selects 1e-11.  Below it a
                                    solve turns the rounding of its input (sums with cancellation,
                                    tens of ulps) into equivalent-density noise and gains no
                                    accuracy: against the exact periodic sums, Stokes TP p = 8
                                    measures 5.2e-6 at 1e-11 and 1.9e-5 at Table 1's rank
                                    criterion 2^-52 dim(A) (p = 10: 9.6e-8 and 1.3e-7; p = 12:
                                    4.0e-9 and 3.1e-9), while rounding-level changes of the solve
                                    inputs move the result 85, 20 and 5 times less */
    unsigned flags;              /* an OR of the PKIFMM_* flags below; other bits are invalid */
    const char *operator_cache_dir;  /* NULL or "": no cache.  Else a writable directory holding the
                                    costly Stage-1 operators (the solve factors U^T, V S^+ and the
                                    periodic root operator, which depend on kernel, periodic axes, p
                                    and the solve cutoff only; the paper computes them once for all
                                    simulations, Section 2.2): pkifmm_plan_create loads them from
                                    there when present (and re-checks the solves) and stores them
                                    otherwise; one file per key, written under a temporary name and
                                    renamed.  Read during pkifmm_plan_create only */
    void *alloc_ctx;             /* passed to alloc and free */
    void *(*alloc)(void *ctx, size_t bytes, void *stream);   /* NULL (with free NULL): hipMalloc;
                                    else every device buffer the plan owns comes from it (operator
                                    tables, tree, work lists, workspace), 256-byte aligned, usable on
                                    any stream once returned; NULL return = out of memory.  stream is
                                    the stream of the library call that asks (NULL in plan creation) */
    void (*free)(void *ctx, void *ptr, void *stream);   /* releases what alloc returned, only once no
                                    work of the plan uses it any more */
    const char *tuning_file;     /* NULL or "": default launch choices.  Else a text file of records
                                    written by pkifmm_autotune; the records of this device's
                                    architecture, kernel, periodic axes, p and precision are used for
                                    the evaluations with their n_rhs.  Read during plan creation only */
    int near_layers;             /* 0 or 1: the tree covers the images |p|_inf <= 1 and the far-field
                                    operator the rest.  2 or 3 (singly and triply periodic sums): the
                                    near field of Algorithm 2 spans l layers of images (Section 3.6,
                                    Table 4): the root's images with 2 <= |p|_inf <= l act on it by
                                    M2L (they are the root's V list) and the far-field operator covers
                                    |p|_inf > l.  The results agree with l = 1 to the FMM's accuracy */
} pkifmm_config;

#define PKIFMM_SKIP_CHECKS 1u    /* skip the SP/DP neutrality check (no device-to-host read) */
#define PKIFMM_PHASE_TIMING 2u   /* record HIP events around the phases of every evaluate on its
                                    stream; pkifmm_get_stats waits for them and reports averages */
#define PKIFMM_GRAPH 4u          /* pkifmm_evaluate captures its launch sequence into a HIP graph
                                    (once per points/n_rhs/density/potential pointers) and replays
                                    it on `stream`; implies no neutrality check and no phase timing */
#define PKIFMM_FAR_STEP_D 8u     /* the far field (images beyond the first layer) is solved into the
                                    root's own downward equivalent density T_M2L phi^{B0,u}
                                    (Section 3.4) and evaluated at every target directly
                                    (Algorithm 2, step d: n_surf extra float64 kernel evaluations per
                                    target, in the W/L2T launch), instead of being added to the
                                    root's downward check potential and handed down the tree.  The
                                    results agree to the FMM's truncation accuracy, not to rounding.
                                    No effect when periodic_mask is 0. */

/* phases of one evaluation: up and M2L on the caller's stream; the near field on a
 * library-owned stream, starting during M2L; then down and leaf on the caller's stream.
 * The X list runs on a third stream beside the upward pass and M2L (its time counts in
 * neither phase) */
#define PKIFMM_PHASE_NEAR 0      /* U-list and direct W/X sums (leaf points to leaf points) */
#define PKIFMM_PHASE_UP 1        /* S2M, M2M, upward solves */
#define PKIFMM_PHASE_M2L 2       /* root far field, V-list M2L and its per-target sums */
#define PKIFMM_PHASE_DOWN 3      /* after M2L: waits for the near field and the X list, then L2L
                                    and the downward solves */
#define PKIFMM_PHASE_LEAF 4      /* W-list M2T, L2T, output permutation */
#define PKIFMM_NUM_PHASES 5

typedef struct {
    int64_t n_points;
    int n_problems;
    int n_boxes, n_leaves, depth;
    int64_t n_u, n_v, n_w, n_x;  /* list entries */
    int64_t u_pairs;             /* point pairs summed directly over the U lists */
    int64_t near_pairs;          /* point pairs of the near-field launch: U lists plus the W/X
                                    entries evaluated directly */
    int svd_rank_up, svd_rank_down;
    double ms_set_points;        /* host wall time of the last pkifmm_set_points (one problem:
                                    without the list build it leaves running on a host thread) */
    double ms_evaluate;          /* host wall time of the last pkifmm_evaluate call (enqueue only
                                    unless a check synchronised) */
    int n_timed;                 /* evaluations averaged in ms_phase (PKIFMM_PHASE_TIMING) */
    double ms_phase[PKIFMM_NUM_PHASES];   /* average device time per phase, HIP events */
    int close_points;            /* mixed form: 1 if pkifmm_set_points found points of different
                                    leaves or images closer than 2^-27 L in every coordinate (every
                                    near-field pair then guards zero separations), else 0 */
    int tune_near_wpc;           /* launch choices of the last evaluation (pkifmm_autotune): near-field */
    int tune_rb_near;            /* workgroups per compute unit; right-hand sides per geometry pass of */
    int tune_rb_s2m;             /* the near field and of the points-to-surface sums (0: the most) */
    double tune_ms;              /* pkifmm_autotune: the best evaluation time it measured */
    int tune_m2l_rows;           /* mixed form: operator rows per tile of the int8 M2L (64 or 128) */
} pkifmm_stats;

/* Fill `cfg` with defaults: Laplace, free space, p = 8, s = 64, FP64, L = 1, no operator cache,
 * hipMalloc. */
int pkifmm_config_default(pkifmm_config *cfg);

/*
 * Build the operators of Algorithm 2, Stage 1 (Section 2 and Section 3.1):
 * check-to-equivalent solves from the SVD of A (applied as (V S^+)(U^T q),
 * Appendix B), M2M/L2L for eight octants, M2L for the 316 offsets, and the
 * periodic root operator K^{P,F} over images |p|_inf >= 2.  Runs on the
 * current HIP device; blocking.  *out receives a plan owned by the caller
 * (release with pkifmm_plan_destroy).
 * Errors (*out is then NULL): INVALID_ARG (NULL argument, a field out of range,
 * unknown flag bits, only one of alloc and free), CACHE_CORRUPT (the operator cache file
 * for this key exists but fails its checks; it is left as it is), NUMERICS (a solve failed its backward-error self-check: on the kept
 * subspace, ||A (V S^+)(U^T A x) - A x|| must stay below 1e-13 s_max ||x||), OOM, HIP.
 */
int pkifmm_plan_create(const pkifmm_config *cfg, pkifmm_plan **out);

/*
 * Wrap, validate, Morton-sort the points and build the adaptive octree and
 * the periodic U/V/W/X lists.
 *   src_xyz: device, [n_src][3] float64, row-major, n_src >= 0: the sources;
 *   trg_xyz: NULL (with n_trg = 0): the targets are the sources; else device
 *            [n_trg][3], n_trg >= 0 target points apart from the sources (Section 2's
 *            problem statement: T targets, S sources).  The octree is then built over the
 *            union (a box holding more than s points of either kind is split), a target
 *            carries no density, and every leaf keeps its sources before its targets;
 *   both are copied and may be freed after the call returns.
 * Waits for the plan's last evaluation to finish (on whatever stream it ran) and
 * synchronises `stream` (the tree's box table is read back to the host).  For one problem
 * the U/V/W/X lists are then completed on a host thread that the call starts and leaves
 * running: pkifmm_evaluate, pkifmm_get_stats and pkifmm_get_list wait for it (and return
 * an error raised while building them, OOM), and the next set_points and
 * pkifmm_plan_destroy let it finish first.  A batch builds its lists in the call.  In the mixed form it
 * also looks for points of different leaves, or a point and another point's periodic
 * image, closer than 2^-27 L in every coordinate; if there are any, every near-field
 * segment guards zero separations (such points then meet as coincident points, at the
 * cost of one instruction per pair).
 * Errors: OUT_OF_BOX (nothing is kept), INVALID_ARG, OOM, HIP.
 */
int pkifmm_set_points(pkifmm_plan *plan, int64_t n_src, const double *src_xyz, int64_t n_trg,
                      const double *trg_xyz, void *stream);

/*
 * Several independent problems in one plan (the batched form): problem i owns
 * counts[i] points, packed one problem after another in `xyz` (device,
 * [sum counts][3] float64).  Each problem is its own periodic box [0, L)^3 with
 * its own octree and lists; pkifmm_evaluate then evaluates every problem in
 * one launch sequence, with densities and potentials packed the same way
 * ([n_rhs][sum counts][k]).  A problem's result does not depend on the other
 * problems in the batch (bitwise).  counts: host, n_problems entries >= 0.  The targets
 * are the sources.  pkifmm_set_points(plan, n, xyz, 0, NULL, s) is this call with one
 * problem.
 * Errors: as pkifmm_set_points.
 */
int pkifmm_set_points_batch(pkifmm_plan *plan, int n_problems, const int64_t *counts, const double *xyz,
                            void *stream);

/*
 * Evaluate the periodic sum for n_rhs densities on the current points.
 *   density:   device, [n_rhs][n_src][k] float64 (k = 1 Laplace, 3 Stokes), source order
 *   potential: device, [n_rhs][n_trg][k] float64 (n_trg = n_src when the targets are the
 *              sources), overwritten, target order
 * Work is enqueued on `stream` (the near field and the X list on two
 * library-owned streams that fork from and join back into `stream`, so
 * completion of `stream` covers all of it); the call returns after enqueueing
 * unless the SP/DP neutrality check runs (it reads one reduction back).  The
 * first evaluation after set_points also builds the work lists on the host,
 * stage by stage while the previous stage's kernels run.  Each call is ordered on the device
 * after the plan's previous evaluation, also when that ran on another stream; a call with a
 * different n_rhs than the previous one first waits on the host for it to finish (its work
 * lists are rebuilt).  The output is float64 in every
 * precision mode.  Densities are not checked: a non-finite density makes non-finite
 * potentials wherever its terms reach.  When the targets are the sources, density and
 * potential may be the same buffer (the first kernel reads every density into library
 * storage, the last writes the potentials); partly overlapping ranges are not supported.
 * Errors: NO_POINTS, INVALID_ARG, INCOMPATIBLE, OOM, HIP.
 */
int pkifmm_evaluate(pkifmm_plan *plan, int n_rhs, const double *density, double *potential,
                    void *stream);

/*
 * pkifmm_evaluate without any allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid it).  Same
 * arguments, layouts and result as pkifmm_evaluate; the result is bitwise that of
 * pkifmm_evaluate (same kernels in the same order).  Differences:
 *   * the work lists for (points, n_rhs) must exist already: pkifmm_evaluate with this n_rhs on
 *     the current points has been called once (else INVALID_ARG; it would have to allocate them);
 *   * the evaluation's workspace (permuted densities, potentials, per-box check potentials and
 *     densities, M2L and split-K temporaries, near-field partial slots, int8 digit slices, the
 *     work counter) is a static device array of 64 MiB per GPU, held from the library's first
 *     use on that GPU until the process ends (its address on each device is looked up when a plan
 *     is created there); a larger need returns CAPACITY (it holds, for example, a Stokes problem
 *     at p = 6 of 1.2e4 points with 3 right-hand sides, or of 2e4 points with 1);
 *   * no neutrality check and no phase timing; never captured by the library (PKIFMM_GRAPH is
 *     ignored), but the caller may capture `stream` around the call;
 *   * every call on a GPU shares that GPU's array, which keeps the previous call's contents (every
 *     region is written or cleared before it is read): calls that overlap in time on one GPU,
 *     from any plans or threads, race and give wrong results.
 * Calls no hipMalloc, hipFree or allocating library routine.
 * Errors: NO_POINTS, INVALID_ARG, CAPACITY, HIP.
 */
int pkifmm_evaluate_noalloc(pkifmm_plan *plan, int n_rhs, const double *density, double *potential,
                            void *stream);

/*
 * Copy the factors of one check-to-equivalent solve (Section 3.1, Appendix B: the solution
 * is (V S^+)(U^T q)) to host arrays, for inspection.
 *   which: 0 upward (check: outer surface, equivalent: inner), 1 downward (check: inner,
 *          equivalent: outer), both for the unit box centred at the origin, raw kernels
 *          1/|r| and I/|r| + r r^T/|r|^3 (no 1/(4 pi), 1/(8 pi)), surface points ordered
 *          lexicographically, k components per point;
 *   rank:  out, the singular values kept (r);
 *   Ut:    NULL or host [kn][r] column-major (= U^T, r x kn), VS: NULL or host [r][kn]
 *          column-major (= V S^+, kn x r), kn = k n_surf.
 * Errors: INVALID_ARG (NULL plan or rank, unknown `which`).
 */
int pkifmm_get_solve_factors(const pkifmm_plan *plan, int which, int *rank, double *Ut, double *VS);

/*
 * Choose the launch parameters of the evaluation for the current points and n_rhs by timing it
 * (coordinate descent, median of 5 timed evaluations per candidate, a change kept only if it
 * wins by more than 2 %): the near field's
 * workgroups per compute unit, the right-hand sides that share one pass over the geometry
 * in the near field and in the points-to-surface sums, and (mixed form) the operator rows per
 * tile of the int8 M2L (64 or 128; the int32 sums are exact either way).  Only choices that leave every result
 * bit unchanged are tuned (each sum is formed in the same order whichever is taken).  The plan
 * keeps the best choice for this n_rhs; with tuning_file non-NULL its record (architecture,
 * kernel, periodic axes, p, precision, n_rhs) is added to or replaced in that file, which
 * pkifmm_config::tuning_file reads at plan creation.  density/potential as pkifmm_evaluate
 * (potential is overwritten).  Synchronises `stream`.
 * Errors: NO_POINTS, INVALID_ARG (also: the tuning file could not be written), OOM, HIP.
 */
int pkifmm_autotune(pkifmm_plan *plan, int n_rhs, const double *density, double *potential, void *stream,
                    const char *tuning_file);

/* Tree and list sizes of the current points and the last call timings.  With
 * PKIFMM_PHASE_TIMING this waits for the recorded events of every evaluation since
 * the previous call, reports their per-phase averages and starts a new window.  Waits
 * for the list build that pkifmm_set_points left running (the list sizes).
 * Errors: INVALID_ARG (NULL argument), OOM (raised while building the lists), HIP
 * (waiting for the events). */
int pkifmm_get_stats(pkifmm_plan *plan, pkifmm_stats *out);

/*
 * Copy the tree to host arrays for inspection (each may be NULL):
 *   perm   [n]        int64: sorted position -> input index (with separate targets, n =
 *                     n_src + n_trg and target i has index n_src + i; each leaf lists its
 *                     sources first, then its targets, both in Morton-key order)
 *   boxes  [nbox][8]  int32: level, ix, iy, iz, begin, end, parent, first child or -1
 * Boxes are numbered level by level, in Morton order within a level (for a
 * batch: level by level, problems in order within a level, Morton order
 * within a problem; begin/end index the packed points).
 * Errors: INVALID_ARG (NULL plan), NO_POINTS, HIP (copying the permutation).
 */
int pkifmm_get_tree(const pkifmm_plan *plan, int64_t *perm, int32_t *boxes);

/*
 * Copy one interaction list to host arrays.
 *   which: 'U', 'V', 'W' or 'X'
 *   offsets [nbox + 1] int64 (CSR over boxes; boxes without such a list are empty)
 *   entries [offsets[nbox]][4] int32: source box, shift x, shift y, shift z
 * Call with entries = NULL to obtain offsets (and so the size) first.
 * Waits for the list build that pkifmm_set_points left running.
 * Errors: INVALID_ARG (NULL plan or offsets, unknown `which`), NO_POINTS, OOM (raised
 * while building the lists).
 */
int pkifmm_get_list(const pkifmm_plan *plan, char which, int64_t *offsets, int32_t *entries);

/*
 * Host-only inspection of the topology code (no GPU is touched): build the
 * octree from Morton keys already sorted by (key, input index) and return one
 * interaction list, exactly as pkifmm_set_points would.
 *   sorted_keys: host, [n] 63-bit keys (x bit above y bit above z bit per level)
 *   which:       'U', 'V', 'W' or 'X'
 *   n_boxes:     out, number of boxes
 *   boxes:       NULL or host [n_boxes][8] int32 (same rows as pkifmm_get_tree)
 *   offsets:     NULL or host [n_boxes + 1] int64
 *   entries:     NULL or host [offsets[n_boxes]][4] int32 (same rows as pkifmm_get_list)
 * Call first with the arrays NULL to size them.
 * Errors: INVALID_ARG (NULL n_boxes, n < 0, max_pts_per_leaf < 1, NULL keys with
 * n > 0, mask bits above 7, unknown `which`), OOM.
 */
int pkifmm_host_topology(const uint64_t *sorted_keys, int64_t n, int max_pts_per_leaf, unsigned periodic_mask,
                         char which, int64_t *n_boxes, int32_t *boxes, int64_t *offsets, int32_t *entries);

/*
 * Check an operator cache file (as pkifmm_plan_create reads it: magic, version, sizes,
 * checksum) on the host alone; no GPU is touched.
 * Errors: INVALID_ARG (NULL path or no such file), CACHE_CORRUPT.
 */
int pkifmm_operator_cache_check(const char *path);

/* Release the plan and every buffer it owns (waiting for its last evaluation first).
 * NULL is accepted. */
int pkifmm_plan_destroy(pkifmm_plan *plan);

/* Static text for a status code. */
const char *pkifmm_status_string(int status);

/* Text of the last error on this plan (valid until the next call on it). */
const char *pkifmm_last_error(const pkifmm_plan *plan);

#ifdef __cplusplus
}
#endif
#endif /* PKIFMM_H */
