/*
 * skelfmm -- fast summation u = A q, A_ij = G(x_i, x_j) (i != j), A_ii = 0,
 * by the neighbor-list skeletonization FMM of Yesypenko, Chen & Martinsson
 * (arXiv 2310.16668).  Plain C boundary: no C++ type and no torch type crosses it.
 *
 * Operations and where the paper defines them:
 *   skelfmm_build          the precomputation: adaptive tree with 2:1 balance
 *                          (section 3, "Adaptive tree data structure") and strong
 *                          recursive skeletonization with proxy-surface interpolative
 *                          decompositions (section 2.1, equation (5); section 3,
 *                          "Build stage", Algorithm "Strong recursive skeletonization").
 *                          Host code, float64.
 *   skelfmm_apply          u = Atilde q, the FMM apply (section 3, "FMM apply",
 *                          equations (15)-(20) and Algorithm "FMM apply"): upward pass,
 *                          ifo / ifs / tfo translations, top-level direct sum, downward
 *                          pass.  Runs on the GPU.
 *   skelfmm_apply_adjoint  w = Atilde^H v, the transposed sweep (not in the paper):
 *                          transposed downward pass first, conjugated translations,
 *                          transposed upward pass last.  Runs on the GPU.
 *   skelfmm_apply_fwd_adj  both at once; one shared sweep for real kernels in float32.
 *
 * Conventions shared by every call:
 *   - Status codes: SKELFMM_OK on success; a negative code otherwise, with a
 *     message from skelfmm_last_error() (thread-local, valid until the next failing
 *     call on the same thread).  Argument errors return before any GPU work and leave
 *     outputs untouched.  Device errors surface as SKELFMM_EDEVICE from the failing
 *     call or the next one.  No C++ exception crosses this boundary.
 *   - Vectors q, u, v, w are caller-owned DEVICE buffers in the caller's point
 *     order, n x nrhs row-major (the nrhs values of one point contiguous); complex
 *     values are interleaved (re, im).  Outputs are overwritten, never accumulated.
 *   - An operator may run on one HIP stream at a time: its workspace lives inside it.
 *     All GPU work of apply / apply_adjoint is enqueued asynchronously on `hip_stream`
 *     (NULL = the default stream); they neither allocate nor synchronize once
 *     skelfmm_prepare has sized the workspace for that nrhs and dtype.
 */
#ifndef SKELFMM_H
#define SKELFMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct skelfmm_op skelfmm_op;        /* opaque; owned by the library */
typedef struct skelfmm_batch skelfmm_batch;  /* opaque; owned by the library */

typedef enum {
    SKELFMM_OK = 0,
    SKELFMM_EINVAL = -1,     /* invalid argument */
    SKELFMM_ENOMEM = -2,     /* host or device allocation failed */
    SKELFMM_EDEVICE = -3,    /* HIP runtime error (no device, launch failure, ...) */
    SKELFMM_ENOTSUP = -4,    /* valid request the library does not support */
    SKELFMM_EINTERNAL = -5
} skelfmm_status;

/* The *_ENUM_MAX entries are not values: they give the enum types the range of
 * int32, so an out-of-range argument from a caller is a value the library can
 * reject (EINVAL), not undefined behaviour on the C++ side. */
typedef enum { SKELFMM_LAPLACE = 0, SKELFMM_HELMHOLTZ = 1, SKELFMM_KIND_ENUM_MAX = 0x7fffffff } skelfmm_kind;

/* Arithmetic of an apply.  Laplace takes F64 or F32, Helmholtz C128 or C64. */
typedef enum {
    SKELFMM_F64 = 0, SKELFMM_F32 = 1, SKELFMM_C128 = 2, SKELFMM_C64 = 3,
    SKELFMM_DTYPE_ENUM_MAX = 0x7fffffff
} skelfmm_dtype;

/* Kernel G (section 2, equations for the Laplace and Helmholtz kernels):
 *   2D Laplace    -log(r) / (2 pi)          (dim = 2)
 *   3D Laplace    1 / (4 pi r)              (dim = 3)
 *   2D Helmholtz  (i/4) H0^(1)(kappa r)     (dim = 2, kappa >= 0; H0^(1) = J0 + i Y0,
 *                                            evaluated in float64 in every dtype)
 *   3D Helmholtz  exp(i kappa r) / (4 pi r) (dim = 3, kappa >= 0)           */
typedef struct {
    int32_t kind;            /* skelfmm_kind */
    int32_t dim;             /* 2 or 3 */
    double kappa;            /* Helmholtz wavenumber; ignored for Laplace */
} skelfmm_kernel;

/* Build and apply options; a zero-initialised struct (or NULL) means defaults. */
typedef struct {
    int32_t proxy_shape;     /* 0 default (2D circle, 3D Chebyshev box), 1 box, 2 circle (2D only) */
    int32_t proxy_points;    /* per side (box) or total (circle); 0 = default (3D 10/side, 2D 128) */
    double proxy_scale;      /* proxy box side / box side; 0 = default 2.95 (circle radius = scale/2 * side) */
    int32_t no_compression;  /* test mode: every box keeps all its points (k = n) */
    int32_t num_threads;     /* host threads for the build; 0 = all cores */
    int32_t keep_transparent;/* 1: also evaluate pairs of two uncompressed boxes, whose
                                ifo terms cancel exactly (default 0: they are skipped) */
    int32_t f64_leaf;        /* C64/F32 applies: evaluate and accumulate the near field in float64 */
    int32_t nonsymmetric;    /* 1: evaluate both orders of every colleague pair separately (default 0:
                                one evaluation of G(B_i, B_j) serves the ifo terms i <- j and j <- i,
                                since G(x, y) = G(y, x) for every kernel here (real for Laplace,
                                complex symmetric for Helmholtz); single-RHS applies only) */
    int32_t no_expansion;    /* 1: the float32 pair kernel always forms |d|^2 from coordinate
                                differences (default 0: pairs whose distance bound allows it use
                                the expanded form |t'|^2 + |s'|^2 - 2 t'.s', see skelfmm_stats) */
    int32_t compensated_leaf;/* F32 applies with one right-hand side: the symmetric pair kernel keeps
                                its float32 partial sums to at most four products per target and
                                forms its per-source column sums in float64 before everything is
                                accumulated in float64 (default 0: float32 partials over blocks of 8
                                sources and float32 column sums over the 64 x tpl targets of a pass) */
    int32_t gpu_build;       /* 1: skelfmm_build computes the interpolative decompositions (proxy
                                matrices, pivoted QR, T = R11^{-1} R12) level by level on the current
                                HIP device; the tree and neighbor lists stay on the host (default 0:
                                all on the host).  ENOTSUP when no HIP device is present */
    int32_t f32_differences; /* F32 applies with one right-hand side: symmetric pair items whose reach R
                                from the source box's first entry is at most 1024 times their
                                smallest point spacing d form |d|^2 from float32 coordinate
                                differences about that entry (one kernel value's relative error is
                                then at most about (R / |t - s| + 1) 2^-24: up to 6e-5 for the
                                closest pair an item may hold, a few float32 units for most pairs;
                                see skelfmm_stats.n_sym_f32diff).  Default 0: float64 differences
                                or the float64 expanded form */
    int32_t reserved[3];
} skelfmm_options;

/* Build-time and layout statistics (section 5 / table "Notation for reported results"). */
typedef struct {
    int64_t n_points;
    int32_t n_boxes, n_leaves, max_level, top_level, k_max, proxy_count;
    double t_tree, t_skel;           /* seconds */
    int64_t m_proj_elems;            /* sum over boxes of k (n - k): entries of all T */
    int64_t n_entries;               /* index-set entries over all levels */
    int64_t pairs_near;              /* kernel evaluations per apply (near field, all levels) */
    int64_t pairs_skel;              /* extra skeleton-pair FMAs per apply (uhat part) */
    int64_t n_tasks;                 /* near-field work items */
    int32_t tile_targets;            /* targets per near-field work item */
    int32_t n_sym_tasks;             /* symmetric colleague-pair work items (0 when not paired) */
    int64_t pairs_sym;               /* kernel evaluations of the symmetric pair items that serve both
                                        directions (each covers two of the pairs in pairs_near) */
    int64_t pairs_sym_skel;          /* skeleton pairs inside them (two uhat multiply-adds each) */
    int64_t pairs_tile;              /* one-direction evaluations in the diagonal tiles of a box
                                        paired with itself (for the current targets per lane) */
    int64_t pairs_tile_skel;         /* skeleton pairs inside them */
    int32_t n_sym_expanded;          /* pair items whose float32 evaluation expands |d|^2 about an
                                        origin (the build's distance bound allows it) */
    int32_t n_sym_f32diff;           /* pair items evaluated from float32 differences (f32_differences) */
    double t_skel_qr;                /* seconds of t_skel spent in the interpolative decompositions
                                        themselves (proxy matrices, pivoted QR, T; on the device with
                                        gpu_build, copies included) */
    double t_layout;                 /* seconds to pack the device layout (work lists, pairing) */
} skelfmm_stats;

/* Read-only host view of the skeleton operators, valid while the operator lives.
 * Boxes are numbered level by level.  Per box b:
 *   idx[idx_ptr[b] .. idx_ptr[b+1])  original point indices in natural order (a leaf:
 *                                    its points; a tree box: its children's skeleton
 *                                    points, children in order, each in skeleton order)
 *   pos[same range]                  positions within that order: the k skeleton
 *                                    positions first, then the n - k redundant ones
 *   rank[b]                          k, or -1 for boxes at or above the top level
 *   T[T_ptr[b] .. T_ptr[b+1])        interpolation matrix, column-major k x (n - k)
 *   coll / coarse / fine             CSR neighbor relations (colleagues incl. self;
 *                                    coarse = touching leaves one level up;
 *                                    fine = inverse of coarse, on leaves)            */
typedef struct {
    int32_t dim, kind;
    double kappa;
    int64_t n_points;
    const double* points;            /* n_points x dim, caller order */
    int32_t n_boxes, max_level, top_level, pad0;
    const int32_t *level, *parent, *is_leaf, *child_ptr, *child_idx, *coord;
    const int64_t *idx_ptr, *idx, *pos;
    const int32_t* rank;
    const int64_t* T_ptr;
    const double* T;
    const int32_t *coll_ptr, *coll_idx, *coarse_ptr, *coarse_idx, *fine_ptr, *fine_idx;
    double root_lo[3];
    double root_side;
} skelfmm_plan_view;

/* Build the operator for n points (host buffer, n x dim row-major, copied) with
 * interpolative-decomposition tolerance tol in (0, 1) and leaf size >= 1.
 * Synchronous; host-only unless options->gpu_build is set (then the IDs run on
 * the current HIP device and the device memory they used is freed on return).
 * On success *out owns the operator. */
skelfmm_status skelfmm_build(const double* points, int64_t n, skelfmm_kernel kernel, double tol,
                             int32_t leaf_size, const skelfmm_options* opt, skelfmm_op** out);

/* Upload the operator to the current HIP device and size its workspace for up to
 * nrhs_max right-hand sides of `dtype` (nrhs_max = 0: upload only, no workspace;
 * for skelfmm_apply_noalloc).  Synchronous; may allocate.  Calling apply with a
 * larger nrhs (or a new dtype) prepares implicitly, which then allocates. */
skelfmm_status skelfmm_prepare(skelfmm_op* op, int64_t nrhs_max, skelfmm_dtype dtype);

/* u = Atilde q on the GPU.  q, u: device buffers, n x nrhs (x2 for complex). */
skelfmm_status skelfmm_apply(skelfmm_op* op, const void* q, void* u, int64_t nrhs,
                             skelfmm_dtype dtype, void* hip_stream);

/* w = Atilde^H v on the GPU (the transposed sweep).  Same layout as skelfmm_apply. */
skelfmm_status skelfmm_apply_adjoint(skelfmm_op* op, const void* v, void* w, int64_t nrhs,
                                     skelfmm_dtype dtype, void* hip_stream);

/* u = Atilde q and w = Atilde^H v together (one right-hand side each), for callers
 * that need both (the gradient of a loss, Krylov methods such as BiCG, LSQR, QMR).
 * Same layout, stream and results as skelfmm_apply followed by skelfmm_apply_adjoint.
 * For a real kernel in float32 the two run as ONE sweep with two interleaved
 * columns: the adjoint of a real symmetric kernel's operator is the operator
 * itself (one skeleton and one T per box serve its rows and columns), so every
 * near-field kernel value and every read of T serves both vectors.  Other
 * kernels and dtypes run the two sweeps in turn.  The fused sweep sizes its own
 * workspace (two values per entry) on first use; q, v, u, w must be four distinct
 * buffers.  Errors as skelfmm_apply. */
skelfmm_status skelfmm_apply_fwd_adj(skelfmm_op* op, const void* q, const void* v, void* u, void* w,
                                     skelfmm_dtype dtype, void* hip_stream);

/* u = Atilde q (adjoint = 0) or w = Atilde^H v (adjoint = 1) without any device
 * allocation, for callers that cannot allocate while they apply (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  The same
 * sweep and kernels as skelfmm_apply / skelfmm_apply_adjoint, with the same
 * layout, stream and result; the workspace (entry and skeleton vectors, pair
 * slots) comes from one static device array of skelfmm_noalloc_scratch_bytes()
 * bytes (64 MiB) per device, held until the process ends, instead of the
 * operator.  Requires the operator uploaded for dtype on the current device
 * (skelfmm_prepare, nrhs_max = 0 is enough).  Errors (before any GPU work):
 * EINVAL if it is not uploaded, if it was prepared on another device, or if the
 * apply needs more workspace than the array holds (the message gives both sizes).
 * Every call on a device shares that device's array and leaves its contents
 * there; nothing in it needs clearing, but calls that overlap on one device
 * (two streams, two threads) race on it. */
skelfmm_status skelfmm_apply_noalloc(skelfmm_op* op, const void* q, void* u, int64_t nrhs,
                                    skelfmm_dtype dtype, int32_t adjoint, void* hip_stream);
int64_t skelfmm_noalloc_scratch_bytes(void);

skelfmm_status skelfmm_stats_get(const skelfmm_op* op, skelfmm_stats* out);

/* Near-field launch shape (an in-library autotuner).  Each near-field work item is
 * one wavefront holding 64 x tpl targets per pass (tpl targets per lane, tpl in
 * 1..SKELFMM_NTPL).  skelfmm_autotune prepares the operator for `dtype`, times the
 * near-field launches for each tpl on `hip_stream` (synchronously; it overwrites
 * the workspace), keeps the fastest and returns it in *chosen, with the timings
 * in ms[SKELFMM_NTPL] (ms[tpl - 1]; may be NULL).  skelfmm_set_targets_per_lane
 * fixes tpl without timing (for the single applies and the fused forward +
 * adjoint sweep alike). */
#define SKELFMM_NTPL 4
skelfmm_status skelfmm_autotune(skelfmm_op* op, skelfmm_dtype dtype, void* hip_stream, int32_t* chosen, float* ms);
skelfmm_status skelfmm_set_targets_per_lane(skelfmm_op* op, int32_t tpl);
/* The same for the two-column near field of the fused float32 forward + adjoint
 * sweep of a real kernel (its own setting).  ENOTSUP for complex kernels and for
 * operators built with f64_leaf. */
skelfmm_status skelfmm_autotune_fwd_adj(skelfmm_op* op, void* hip_stream, int32_t* chosen, float* ms);

/* Launch shape of the many-RHS transfers on the matrix cores (float32 Laplace
 * applies with at least 8 right-hand sides; section 3, "FMM apply", equations
 * (15)-(20): per box qhat = q_S + T q_R upward and u_R += T^* uhat downward,
 * here one GEMM per box against all right-hand sides).  Shapes 0 .. SKELFMM_NXFER-1
 * are blocks of 4 or 2 wavefronts (128 or 64 rows of the result) with 64 or 32
 * columns per wavefront: {4, 64}, {4, 32}, {2, 64}, {2, 32}.  No shape changes the
 * arithmetic of an output tile, so all give identical results.
 * skelfmm_autotune_transfers prepares the operator for nrhs float32 columns, times
 * both passes in every shape on `hip_stream` (synchronously; it overwrites the
 * workspace), keeps the fastest, returns it in *chosen and the timings in
 * ms[SKELFMM_NXFER] (may be NULL).  Errors: EINVAL for a Helmholtz operator or
 * NULL chosen, ENOTSUP when nrhs < 8 (those applies do not use the matrix cores). */
#define SKELFMM_NXFER 4
skelfmm_status skelfmm_autotune_transfers(skelfmm_op* op, int64_t nrhs, void* hip_stream, int32_t* chosen,
                                         float* ms);
skelfmm_status skelfmm_set_transfer_shape(skelfmm_op* op, int32_t shape);

/* Per-pass GPU timing.  When enabled, each apply records HIP events on its stream
 * around its passes: [0] gather, [1] upward pass, [2] near field over the segment
 * lists (ifo, ifs, tfo, top level; with symmetric pairing, what is left after
 * pairing), [3] symmetric pairs (0 when not paired), [4] reduction of the pair
 * slots into u and uhat (0 when not paired), [5] downward pass, [6] output scatter.
 * skelfmm_timing(op, 1) enables and zeroes the accumulators; (op, 0) disables.
 * skelfmm_timing_read waits for the recorded events and returns the summed
 * milliseconds per pass (ms[SKELFMM_NPASS]) and the number of timed sweeps. */
#define SKELFMM_NPASS 7
skelfmm_status skelfmm_timing(skelfmm_op* op, int32_t enable);
skelfmm_status skelfmm_timing_read(skelfmm_op* op, double* ms, int64_t* sweeps);
skelfmm_status skelfmm_export(const skelfmm_op* op, skelfmm_plan_view* out);

/* Several operators applied as one sweep: every pass of the sweep runs over the
 * union of the operators' work, so small geometries share launches with large
 * ones.  Operators must share kind and dim and outlive the batch.  q[i], u[i]:
 * device buffers of operator i.  adjoint = 1 applies the transposed sweep. */
skelfmm_status skelfmm_batch_create(skelfmm_op* const* ops, int32_t nops, skelfmm_batch** out);
skelfmm_status skelfmm_batch_apply(skelfmm_batch* b, const void* const* q, void* const* u,
                                   int64_t nrhs, skelfmm_dtype dtype, int32_t adjoint,
                                   void* hip_stream);
/* skelfmm_timing / skelfmm_timing_read for the batch's sweeps (eager applies;
 * a captured graph records no events). */
skelfmm_status skelfmm_batch_timing(skelfmm_batch* b, int32_t enable);
skelfmm_status skelfmm_batch_timing_read(skelfmm_batch* b, double* ms, int64_t* sweeps);
/* skelfmm_autotune_transfers for the batch's merged sweep. */
skelfmm_status skelfmm_batch_autotune_transfers(skelfmm_batch* b, int64_t nrhs, void* hip_stream,
                                               int32_t* chosen, float* ms);
void skelfmm_batch_destroy(skelfmm_batch* b);   /* NULL-safe */

void skelfmm_destroy(skelfmm_op* op);           /* NULL-safe; frees host and device state */
const char* skelfmm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SKELFMM_H */
