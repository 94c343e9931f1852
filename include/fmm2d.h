/*
 * fmm2d.h -- C ABI of the MI355X (gfx950) hierarchical 2D FMM library.
 *
 * The library evaluates the complex logarithmic potential
 *
 *     Phi_j = sum_{i=1..N} u_i * log(y_j - x_i),   j = 1..M,   x, y in C
 *
 * (Luo & Duraiswami, "Alternative tilings for the fast multipole method on
 * the plane", arXiv:1204.3105, Sec. 2, eqs. 1-2) with the fast multipole
 * method on one of the paper's three tilings: the square quadtree (Sec. 4),
 * the hexagonal septree with base-7 GBT addressing (Sec. 5) or the
 * triangle-quadtree (Sec. 6).  The expansion and translation operators,
 * which the paper cites but omits, are those of Greengard & Rokhlin (1987),
 * Lemmas 2.1-2.5.  Every step of a solve runs in HIP kernels on one GPU.
 *
 * Conventions shared by every entry point
 *  - Points are complex128 arrays: 2*n doubles, interleaved (x0, y0, x1, y1,
 *    ...).  Strengths are n real doubles.  The output Phi is 2*M doubles,
 *    interleaved (Re, Im), in the caller's target order.
 *  - Branch: log z = ln|z| + i Arg z with Arg in (-pi, pi]; a -0 imaginary
 *    part counts as +0.  Far-field terms carry the branch of the expansion,
 *    Log(c_T - c_S) + Log((y - x)/(c_T - c_S)) for the unique separated cell
 *    pair (S, T), so Im Phi may differ from the principal-branch direct sum
 *    by multiples of 2 pi u_i; Re Phi is branch-free.
 *  - A source and a target with bitwise-equal coordinates do not interact.
 *  - Ownership: the caller owns every buffer it passes.  fmm_plan copies the
 *    coordinates into plan-owned device memory; the caller may free them on
 *    return.  A plan owns all of its device memory until fmm_plan_destroy.
 *  - Pointers are host pointers unless options.device_pointers is set, in
 *    which case they are device pointers on the current HIP device and the
 *    work is ordered on options.stream (hipStream_t; NULL = the null
 *    stream): inputs are read and outputs written in that stream's order,
 *    and fmm_plan_destroy returns without waiting (the plan's memory is
 *    reused only behind its last work).  With host pointers every call is
 *    synchronous.
 *  - Errors are status codes, never exceptions; fmm_last_error() returns a
 *    thread-local message for the last non-OK status.
 *  - Plans are independent; one plan must not be evaluated concurrently
 *    from two threads.
 */
#ifndef FMM2D_H
#define FMM2D_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FMM_QUADTREE = 0,     /* square quadtree, Morton Z order (Sec. 4)          */
    FMM_SEPTREE = 1,      /* hexagonal septree, base-7 GBT addresses (Sec. 5) */
    FMM_TRIQUADTREE = 2   /* triangle-quadtree (Sec. 6)                       */
} fmm_tiling;

typedef enum {
    FMM_PREC_AUTO = 0,    /* MIXED for eps >= 1e-6, FP64 below                */
    FMM_PREC_FP64 = 1,    /* every step in FP64                               */
    FMM_PREC_MIXED = 2    /* M2L as BF16x3 split products on MFMA with FP32
                             accumulation, P2P in FP32 with compensated sums;
                             monopole/log terms, P2M, M2M, L2L, L2P in FP64.
                             P2P takes FP32 offsets from leaf centres; pairs
                             closer than 1/32 of the leaf scale, and pairs
                             near the log's branch cut, are formed again
                             from the FP64 coordinates, so the error does
                             not grow for points on curves or planted next
                             to each other.  Its arithmetic floor is about
                             2e-8 in relative L2: for eps below 1e-6 a MIXED
                             request is resolved to FP64 (fmm_plan_info
                             reports the precision used)                  */
} fmm_precision;

typedef enum {
    FMM_OK = 0,
    FMM_E_INVALID = 1,    /* null pointer with n > 0, n < 0, eps not in
                             (0, 0.5), bad tiling, non-finite coordinate,
                             option out of range                             */
    FMM_E_DOMAIN = 2,     /* an explicit geometry does not cover the points  */
    FMM_E_NOMEM = 3,      /* device allocation failed or budget exceeded     */
    FMM_E_DEVICE = 4,     /* a HIP runtime call failed                        */
    FMM_E_BUSY = 5        /* serving: result not ready yet                    */
} fmm_status;

typedef struct fmm_plan_s *fmm_plan_t;

/* Leaf-level rule when neither lmax nor a geometry is given.
 * FMM_DEPTH_MEAN: the smallest level whose mean occupancy (points over the
 *   bounding box's area in leaves) is at most leaf_size (the paper's uniform
 *   per-cell population, Sec. 9).
 * FMM_DEPTH_COST: for clustered inputs; starting from the mean rule's level
 *   L0, the levels L0..L0+3 (base^level <= 2^24) are priced from the points'
 *   occupancy histogram (near-field pairs, occupied leaves, M2L pairs) and
 *   the cheapest is taken.  The tree is still the paper's uniform-depth tree;
 *   one more short readback at plan time. */
typedef enum { FMM_DEPTH_MEAN = 0, FMM_DEPTH_COST = 1 } fmm_depth_rule;

/* Plan options.  Call fmm_options_default first, then override fields. */
typedef struct {
    uint32_t struct_size;    /* sizeof(fmm_options)                           */
    int32_t leaf_size;       /* target mean points per occupied leaf (64)     */
    int32_t lmax;            /* leaf level; -1 = from leaf_size               */
    int32_t p;               /* expansion order; -1 = from eps and the
                                tiling's separation ratio (Sec. 8)            */
    int32_t precision;       /* fmm_precision                                 */
    int32_t has_geometry;    /* 1 = use geometry[] and lmax as given          */
    double geometry[3];      /* origin x, origin y, scale: quadtree = lower-
                                left corner and side of the root square;
                                septree = centre of leaf hexagon 0 and leaf
                                circumradius; triangle-quadtree = root
                                centroid and leaf circumradius                */
    void *stream;            /* hipStream_t for device-pointer calls          */
    int32_t device_pointers; /* 1 = all data pointers are device pointers     */
    int32_t depth_rule;      /* fmm_depth_rule, used when lmax < 0 and no
                                explicit geometry (FMM_DEPTH_MEAN)            */
    int32_t near_stream;     /* where fmm_eval runs the P2P near field:
                                0 = a library stream beside the far-field
                                passes (default: one solve's latency);
                                1 = the plan's own stream after them (for a
                                caller that overlaps several solves on
                                streams of its own); other values rejected   */
} fmm_options;

/* Read-only summary of a plan. */
typedef struct {
    int32_t tiling;
    int32_t lmax;            /* leaf level L (root = level 0)                 */
    int32_t p;               /* expansion order                               */
    int32_t precision;       /* resolved precision (FP64 or MIXED)            */
    double geometry[3];      /* as in fmm_options                             */
    int64_t n_src, n_tgt;
    int32_t targets_are_sources;
    int32_t e4_width;        /* slots per M2L list: 27 / 42 / 39              */
    int64_t n_cells[32];     /* occupied cells per level (sources or targets) */
    int64_t n_m2l_pairs;     /* nonempty M2L (E4) cell pairs, all levels      */
    int64_t n_near_pairs;    /* source-target point pairs in the near field   */
    int64_t device_bytes;    /* device memory held by the plan                */
    double plan_ms;          /* GPU time of the last fmm_plan                 */
    double eval_ms;          /* GPU time of the last fmm_eval                 */
    double stage_ms[8];      /* last eval: [0] upward pass, [1] M2L, [2] L2L,
                                [3] P2P near field (runs beside 0..2),
                                [4] wait for P2P + L2P; rest reserved          */
} fmm_plan_info;

/* Fill *opt with defaults: leaf_size 64, lmax -1, p -1, AUTO precision,
 * host pointers, no explicit geometry. */
fmm_status fmm_options_default(fmm_options *opt);

/* Build a plan (Secs. 4-6: CellIndex keys at the leaf level, sort, per-level
 * occupied cells, Neighbors and NeighborsE4 lists).  src: n_src complex128
 * points; tgt: n_tgt complex128 points (tgt may equal src, in which case the
 * sorted arrays are shared, and the plan also holds (near width - 1) x 2 x n
 * second-side near sums, FP32 or FP64 pairs, for the symmetric near field
 * of fmm_eval).  eps in (0, 0.5) selects p when opt->p < 0.
 * opt may be NULL (defaults).  On success *out holds the plan. */
fmm_status fmm_plan(fmm_tiling tiling, const double *src, int64_t n_src, const double *tgt,
                    int64_t n_tgt, double eps, const fmm_options *opt, fmm_plan_t *out);

/* Evaluate Phi for strengths u (n_src doubles) into phi (2*n_tgt doubles):
 * P2M, M2M, M2L, L2L, L2P and the P2P near field (GR87 Lemmas 2.1-2.5).
 * When the targets are the sources, each pair of neighbouring leaves is
 * evaluated once for both of its sides (ln|y - x| is symmetric, and the two
 * arguments differ by pi on the principal branch), so the near field's
 * rounding differs from fmm_eval_field's one-sided sums.
 * Allocates nothing.  n_src = 0 gives Phi = 0. */
fmm_status fmm_eval(fmm_plan_t plan, const double *u, double *phi);

/* As fmm_eval, and also the field Phi'(y_j) = sum_i u_i / (y_j - x_i), the
 * derivative of eq. 2 in y (branch-free): the derivative of each target
 * leaf's local expansion plus the near-field terms u_i / (y_j - x_i) over the
 * same near lists, coincident pairs skipped (same precision policy as the
 * potential).  field: 2*n_tgt doubles (complex128, caller's target order),
 * host or device like phi.  The plan takes 16 B per target more on the first
 * call.  Its potential equals fmm_eval's bitwise when the targets are not
 * the sources, and to rounding (the near sums are one-sided here) when they
 * are.  Errors as fmm_eval; FMM_E_NOMEM if the field buffers cannot be
 * allocated. */
fmm_status fmm_eval_field(fmm_plan_t plan, const double *u, double *phi, double *field);

/* Summary of a plan.  info->n_cells holds lmax+1 valid entries. */
fmm_status fmm_plan_info_get(fmm_plan_t plan, fmm_plan_info *info);

/* Export the plan's tree for parity checks (host buffers, caller-sized):
 *  src_keys[n_src], tgt_keys[n_tgt]: leaf keys (base 4 or 7) in caller order;
 *  src_perm[n_src], tgt_perm[n_tgt]: original index of each sorted position.
 * Any pointer may be NULL. */
fmm_status fmm_plan_export_points(fmm_plan_t plan, int64_t *src_keys, int64_t *tgt_keys,
                                  int64_t *src_perm, int64_t *tgt_perm);

/* Export level `level` (0..lmax), n = info.n_cells[level] cells in key
 * order: keys[n]; occupancy[n] (bit 0 = holds sources, bit 1 = targets);
 * src_range[2n] and tgt_range[2n] ([begin, end) into the sorted order);
 * e4[n * e4_width]: keys of the source-occupied NeighborsE4 cells of every
 * target-occupied cell (-1 padded, ascending); near[n * 13]: keys of the
 * source-occupied cells among {n} u Neighbors(n) at the leaf level (-1
 * padded, ascending; only filled when level == lmax).  Any pointer may be
 * NULL. */
fmm_status fmm_plan_export_level(fmm_plan_t plan, int32_t level, int64_t *keys,
                                 int32_t *occupancy, int64_t *src_range, int64_t *tgt_range,
                                 int64_t *e4, int64_t *near);

/* Release every resource of the plan.  NULL is a no-op. */
void fmm_plan_destroy(fmm_plan_t plan);

/* Thread-local message for the last non-OK status ("" if none). */
const char *fmm_last_error(void);

/* Expansion order from eps: p = ceil(ln eps / ln q) - 1 with the tiling's
 * separation ratio q = max(r/R, 1/(1 + rho/r)) (Sec. 8 error bounds; septree
 * q measured on GBT aggregates).  Returns -1 for bad arguments. */
int32_t fmm_order_for_eps(fmm_tiling tiling, double eps);

/* Direct sum (Sec. 2, eq. 2 evaluated term by term; the baseline the paper
 * compares the FMM with, Sec. 9): phi[j] = sum_i u[i] Log(tgt[j] - src[i])
 * on the principal branch, Log z = ln|z| + i Arg z with Arg in (-pi, pi]
 * and a -0 imaginary part read as +0; a source with the target's exact
 * coordinates is skipped.  FP64 with compensated sums, sources taken in
 * index order.  src: n_src complex128 points; tgt: n_tgt complex128 points
 * (may equal src); u: n_src doubles; phi: n_tgt complex128 out.  opt may be
 * NULL (host pointers); with opt->device_pointers the pointers are device
 * pointers and the work is ordered on opt->stream; other option fields are
 * ignored.  Returns FMM_E_INVALID for null arrays with nonzero sizes or
 * negative sizes, FMM_E_INVALID for a non-finite coordinate (host pointers
 * only), FMM_E_NOMEM or FMM_E_DEVICE on device failures. */
fmm_status fmm_direct(const double *src, int64_t n_src, const double *tgt, int64_t n_tgt,
                      const double *u, double *phi, const fmm_options *opt);

/* fmm_direct without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, serving loops or harnesses that
 * forbid hipMalloc).  Same sum, same kernels and the same slicing of the
 * sources as fmm_direct with device pointers, so the result is bitwise
 * fmm_direct's.  src, tgt, u, phi are device pointers on the current
 * device; work is ordered on stream (hipStream_t, NULL = null stream) and
 * the call returns without waiting.  The slices' partial sums live in a
 * fixed 16 MiB device array of the library (one per GPU, held until the
 * process ends; the slicing rule needs at most 12 MiB, and a size that
 * needed more would return FMM_E_INVALID).  Calls that overlap on one GPU
 * share that array and race: order them on one stream or wait between them.
 * Nothing needs clearing between calls (every partial sum a call reads it
 * wrote first).  Errors: FMM_E_INVALID for negative sizes or null arrays
 * with nonzero sizes; FMM_E_DEVICE if the array's address cannot be found
 * or the launch fails.  Coordinates are not checked for finiteness. */
fmm_status fmm_direct_noalloc(const double *src, int64_t n_src, const double *tgt, int64_t n_tgt,
                              const double *u, double *phi, void *stream);

/* Pair-evaluation ceiling of the FP64 near field (Sec. 2, eq. 2: the log
 * kernel's terms): runs a probe kernel in which every lane evaluates the
 * near field's FP64 pair function (ln r^2 and both arguments of the pair)
 * for `rounds` rounds of eight independent pairs held in registers -- no
 * loads, no reductions -- in one-wave blocks at the near field's occupancy,
 * on `blocks` blocks (0: 3072, three waves on each of the GPU's 1024 SIMDs),
 * and returns the measured evaluations per second in *evals_per_s.  The
 * near-field kernel's own evaluation rate divided by this one measures its
 * efficiency against what the chip sustains for this code.  Synchronous,
 * on the current device, on a stream of its own; allocates 512 B per block.
 * Errors: FMM_E_INVALID for rounds < 1, blocks < 0 or a null output;
 * FMM_E_DEVICE on device failures. */
fmm_status fmm_probe_pair_rate(int32_t rounds, int32_t blocks, double *evals_per_s);

/* ------------------------------------------------------------------ serving
 * A request loop that admits independent solves by free device memory,
 * keeps their plans resident, and runs the same phase of every admitted
 * request in one batched kernel launch per phase (continuous batching).
 * Results are bitwise identical to the same request solved alone.       */
typedef struct fmm_server_s *fmm_server_t;

typedef struct {
    uint32_t struct_size;
    int64_t hbm_budget_bytes;   /* admission budget for resident plans        */
    int32_t max_inflight;       /* maximum admitted requests at once          */
    int32_t leaf_size;          /* as fmm_options.leaf_size                   */
} fmm_server_options;

typedef struct {
    int32_t tiling;             /* fmm_tiling                                 */
    int32_t precision;          /* fmm_precision                              */
    double eps;
    int64_t n_src, n_tgt;
    const double *src;          /* host complex128 points (copied on submit)  */
    const double *tgt;          /* NULL = targets are the sources             */
    const double *u;            /* host strengths (copied on submit)          */
} fmm_request;

typedef struct {
    fmm_status status;          /* OK, or the request's error                 */
    int32_t p, lmax;
    double t_submit, t_admit, t_start, t_end;  /* seconds, steady clock       */
} fmm_result;

fmm_status fmm_server_create(const fmm_server_options *opt, fmm_server_t *out);
/* Queue a request; returns its ticket.  Inputs are copied before return. */
fmm_status fmm_submit(fmm_server_t s, const fmm_request *req, uint64_t *ticket);
/* FMM_E_BUSY until the request is done; then copies Phi (2*n_tgt doubles,
 * host) into phi (may be NULL) and fills *res.  A ticket is consumed by the
 * first non-BUSY poll. */
fmm_status fmm_poll(fmm_server_t s, uint64_t ticket, double *phi, fmm_result *res);
/* Block until every queued request is done. */
fmm_status fmm_server_drain(fmm_server_t s);
fmm_status fmm_server_destroy(fmm_server_t s);

#ifdef __cplusplus
}
#endif

#endif /* FMM2D_H */
