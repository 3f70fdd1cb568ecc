/*
 * fmmbem: FMM-accelerated boundary-element solves with relaxed expansion order
 * on AMD Instinct MI355X (gfx950).
 *
 * The problem (Sec. 2.1-2.3 of Wang, Layton & Barba, "Inexact Krylov
 * iterations and relaxation strategies with fast-multipole boundary element
 * method"): a closed surface made of N flat triangles, one unknown (Laplace)
 * or three (Stokes) per triangle, collocation at the triangle centroids, and
 * the first-kind single-layer system A x = b with
 *   Laplace  A_ij = int_{panel j} 1/(4 pi |x_i - y|) dA            (Eq. 3-4)
 *   Stokes   A_ij = -1/(8 pi mu) int_{panel j} G(x_i, y) dA,
 *            G_ab = delta_ab / r + r_a r_b / r^3                    (Eq. 6-7, 9)
 * integrated with 4 Gauss points on far panels (Eq. 10), a 25-point rule on
 * near-singular panels (closer than 2 sqrt(2 S_j)) and a semi-analytic rule on
 * the panel holding the target.  The mat-vec is evaluated as an N-body sum over
 * Gauss points by a fast multipole method with spherical-harmonic expansions of
 * order p (Eq. 12, 15-16), and GMRES (Sec. 2.4) lowers p as the residual falls
 * (Sec. 2.6, Eq. 17-19).
 *
 * Conventions for every entry point:
 *  - Return value: an fmmbem_status; FMMBEM_OK is 0, errors are negative.  No
 *    exception or abort crosses this interface; fmmbem_last_error() gives the
 *    message of the calling thread's last failure.
 *  - Ownership: the caller owns every buffer it passes.  fmmbem_build copies
 *    the mesh; the context owns all device state it creates and releases it in
 *    fmmbem_destroy.
 *  - Vector layout: vectors are in the caller's triangle order.  Laplace has
 *    n = N unknowns; Stokes has n = 3N, stored [N][3] (x, y, z per triangle).
 *    Arguments named *_dev are device pointers (HIP global memory); *_host are
 *    host pointers.
 *  - Streams: a hip_stream argument is a hipStream_t (NULL: the null stream).
 *    Work is enqueued on it; calls returning host data synchronise it.
 *  - Threads: a context is not thread-safe; distinct contexts may be used
 *    concurrently on distinct streams.
 */
#ifndef FMMBEM_H
#define FMMBEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fmmbem_ctx fmmbem_ctx_t;       /* one mesh: tree, lists, corrections, workspaces */
typedef struct fmmbem_server fmmbem_server_t; /* request loop */

typedef enum {
    FMMBEM_OK = 0,
    FMMBEM_EINVAL = -1,    /* invalid argument (null pointer, bad size, index, p, tol ...) */
    FMMBEM_ENOMEM = -2,    /* device or host allocation failed, or budget exceeded */
    FMMBEM_EDEVICE = -3,   /* a HIP runtime call failed */
    FMMBEM_ENOCONV = -4,   /* GMRES reached max_iter; x and the report are still filled */
    FMMBEM_EBUSY = -5,     /* server: request not finished / queue full */
    FMMBEM_EINTERNAL = -6  /* internal invariant violated */
} fmmbem_status;

/* Operators (Sec. 2.1, 2.2; unknowns per panel):
 *   LAPLACE_SL: y = V x, (V x)_i = sum_j x_j int_j G, G = 1/(4 pi r)  (first kind, 1)
 *   STOKES_SL:  y = -1/(8 pi mu) sum_j int_j G_Stokes t_j             (first kind, 3)
 *   LAPLACE_DL: y = (1/2 I - K) x, (K x)_i = sum_j x_j int_j dG/dn_y, outward
 *               normals: the second-kind operator of the exterior Neumann
 *               problem, (1/2 I - K) u = -V du/dn (Eq. 5, 11)             (second kind, 1) */
typedef enum { FMMBEM_LAPLACE_SL = 0, FMMBEM_STOKES_SL = 1, FMMBEM_LAPLACE_DL = 2 } fmmbem_kernel;

/* Arithmetic of the P2P and expansion (P2M ... L2P) kernels.  Inputs, outputs
 * and all Krylov arithmetic are FP64 in both cases; the near-singular
 * correction is summed in FP64 in both, from its values rounded to FP32 in an
 * FP32 mat-vec. */
typedef enum { FMMBEM_FP64 = 0, FMMBEM_FP32 = 1 } fmmbem_precision;

/* Expansion-order schedule for GMRES (Sec. 2.6).  With rho the relative
 * residual after the previous iteration (1 before the first) and eta the
 * solver tolerance, eps_k = min(eta / min(rho, 1), 1) (Eq. 17):
 *   FIXED        p_k = p_init
 *   RELAX_SHIFT  p_k = clamp(p_init + ceil(log2(min(rho, 1))), p_min, p_init)
 *                (Eq. 17 and 19 with the offset that maps eps = eta to p_init)
 *   RELAX_BF     p_k = clamp(ceil(-log2(eps_k)), p_min, p_init)   (Eq. 19) */
typedef enum { FMMBEM_FIXED = 0, FMMBEM_RELAX_SHIFT = 1, FMMBEM_RELAX_BF = 2 } fmmbem_rule;

#define FMMBEM_P_MAX 20        /* largest expansion order supported */
#define FMMBEM_P_MAX_FP32 14   /* largest order for the FP32 expansion kernels */

typedef struct {
    int64_t n_vertices;
    int64_t n_triangles;
    const double *xyz;   /* host, [n_vertices][3] */
    const int32_t *tri;  /* host, [n_triangles][3], counter-clockwise seen from outside */
} fmmbem_mesh;

typedef struct {
    double theta;     /* multipole acceptance criterion (Sec. 2.5), default 0.5 */
    int32_t ncrit;    /* most panels in a leaf box (Sec. 2.5), default 64, 1..1024 */
    int32_t p_max;    /* largest p the context will be asked for, 1..FMMBEM_P_MAX, default 16 */
    double mu;        /* Stokes viscosity, default 1 */
    /* 1: the regular near field (the 4-point rule between neighbouring leaves,
     * Sec. 2.3, the P2P of Sec. 2.5) is assembled once at build as a
     * block-sparse matrix, FP64 and FP32 copies, and every mat-vec multiplies
     * it (the paper's sparse near field).  Memory: 12 B per panel pair
     * (Laplace), 108 B (Stokes); see fmmbem_stats.near_entries.
     * 0 (default): evaluated on the fly by every mat-vec. */
    int32_t near_stored;
    /* 1: the FP64 M2L operator of every distinct translation (Sec. 2.5), the
     * real (2 ncoef(p_max))^2 matrix that pass 1 applies, is generated once at
     * build and stored; FP64 mat-vecs stream it through the matrix cores
     * instead of generating it from the translation's harmonics on every
     * call.  Memory: 8 D^2 bytes per translation, D = 2 ncoef(p_max) rounded
     * up to 16 rows (a sphere of 32768 panels at N_CRIT 64, p_max = 12: 2541
     * translations, 718 MB); see fmmbem_stats.n_translations and
     * m2l_op_bytes.  0 (default): generated on the fly.
     * 2: M2L by rotation at p >= 7 in both precisions: per translation
     * direction, the real forms of the rotation taking the direction to +z
     * and back (every degree <= p_max, FP64 and FP32) are built at build and
     * stored; each pair's multipole expansion is rotated, translated along
     * the axis, and its local expansion rotated back, O(p^3) per pair
     * instead of O(p^4).  Below p = 7 as with 0.  Memory: 24 T bytes per
     * direction, T = sum over n <= p_max of 64 ceil(2 (n + 1) / 16)
     * ceil(2 (n + 1) / 4) (p_max = 16: 9664 values, 232 KB). */
    int32_t m2l_stored;
    /* Quadrature of Sec. 2.3, fixed by the method as built (0 = default;
     * any other value gives FMMBEM_EINVAL):
     *   quad_far    4: the degree-3 four-point rule of Eq. 10 on every
     *               regular panel pair;
     *   quad_near   25: the 5 x 5 collapsed Gauss-Legendre rule on panels
     *               closer than near_factor sqrt(2 S_j) to the target;
     *   near_factor 2.0 (the criterion |x_i - c_j|^2 < 8 S_j). */
    int32_t quad_far;
    int32_t quad_near;
    double near_factor;
    /* Device memory.  alloc == NULL (default): hipMalloc / hipFree.
     * Otherwise every device byte the context (and, for a request, the
     * server) holds comes from alloc(bytes, alloc_user), which returns device
     * memory of the current device aligned to 256 bytes, or NULL (the call
     * then fails with FMMBEM_ENOMEM), and goes back through
     * free(ptr, alloc_user) when the context is destroyed (after the device
     * is synchronised).  Build-time temporaries use it too.  Both callbacks
     * may be called from the server's worker thread.  Pinned host memory
     * (a few KB per context) is not device memory and does not use them. */
    void *(*alloc)(size_t bytes, void *user);
    void (*free)(void *ptr, void *user);
    void *alloc_user;
} fmmbem_params;

typedef struct {
    int32_t rule;      /* fmmbem_rule */
    int32_t p_init;    /* order of the first iterations, <= p_max */
    int32_t p_min;     /* floor of the relaxed order (Sec. 3.2 recommends >= 3-5 for Stokes) */
    int32_t mixed;     /* 1: FP32 P2P/expansions when eps_k >= fp32_eps and p_k <= FMMBEM_P_MAX_FP32 */
    double fp32_eps;   /* default 1e-5 */
    int32_t restart;   /* GMRES(m) restart length, default 50 */
    int32_t max_iter;  /* total iteration cap, default 500 */
} fmmbem_schedule;

typedef struct {
    int32_t iterations, restarts, converged;
    /* restarts forced by a non-finite residual: the step's column is
     * discarded, the cycle ends with the columns before it and every later
     * mat-vec of the solve runs in FP64 */
    int32_t fallbacks;
    /* restarted cycles whose true residual exceeded twice the larger of
     * their implicit residual and tol (the relaxed products were too coarse
     * for the residual reached); each raises a floor under every later order
     * by ceil(log2(true / max(implicit, tol))) + 1 orders (the 2^-p error
     * model of Eq. 19), capped at p_init; p_floor is the floor at exit (0 if
     * no stall) */
    int32_t stalls, p_floor;
    double rel_res_implicit;   /* |g_{k+1}| / |b| at exit */
    /* |b - A x| / |b| with A at p_init in FP64; a solve is converged only
     * when this is <= tol (an implicit residual at tol with a true residual
     * above it restarts the solve) */
    double rel_res_true;
    double t_solve_s;          /* wall time of the solve (host clock, stream synchronised) */
    int64_t matvecs;
    /* device time of this solve by stage (HIP events, the stages of
     * fmmbem_set_timing), -1 for a stage that is not timed on the context:
     * near field (P2P or the stored product), M2L pass 1, the other FMM
     * stages (charges, P2M, M2M, the M2L sum, L2L, L2P, combine) and the
     * Krylov kernels (orthogonalisation, update of x, residuals) */
    double t_p2p_s, t_m2l_s, t_other_fmm_s, t_krylov_s;
    /* caller-owned histories, may be NULL; hist_cap entries each */
    int32_t hist_cap;
    int32_t *p_hist;
    uint8_t *prec_hist;
    double *res_hist;
} fmmbem_report;

typedef struct {
    int64_t n_panels, n_unknowns, n_sources;
    int32_t n_boxes, n_leaves, n_levels, max_leaf;
    int64_t n_m2l, n_p2p;        /* box pairs */
    int64_t p2p_interactions;    /* sum over P2P pairs of |targets| * |sources| */
    int64_t nnz_correction;      /* near-singular + self entries (blocks for Stokes) */
    int64_t device_bytes;        /* device memory held by the context */
    int64_t near_entries;        /* panel pairs of the stored near field (0 unless near_stored) */
    int64_t n_translations;      /* distinct M2L translations (offset and box sizes) */
    int64_t m2l_op_bytes;        /* stored M2L operators or rotations (0 unless m2l_stored) */
} fmmbem_stats;

/* Defaults described above. */
void fmmbem_params_default(fmmbem_params *prm);
void fmmbem_schedule_default(fmmbem_schedule *s, int kernel);

/* Build the context of one mesh (Sec. 2.3 and 2.5): panel geometry and Gauss
 * points, Morton octree with at most ncrit panels per leaf, M2L and P2P lists
 * from a dual traversal with acceptance theta, and the sparse near-singular and
 * self corrections.  mesh is copied; EINVAL for a null pointer, no triangle, a
 * vertex index out of range or a zero-area triangle, or params out of range. */
int fmmbem_build(const fmmbem_mesh *mesh, int kernel, const fmmbem_params *params,
                 void *hip_stream, fmmbem_ctx_t **out);

/* One FMM mat-vec y = A x at expansion order p (1..p_max) in the given
 * precision (the w <- A z of Sec. 2.4, evaluated as in Eq. 12 and Sec. 2.5).
 * x_dev and y_dev are device vectors of n doubles and must not overlap.
 * Enqueued on hip_stream; does not synchronise. */
int fmmbem_matvec(fmmbem_ctx_t *ctx, int32_t p, int32_t precision, const double *x_dev,
                  double *y_dev, void *hip_stream);

/* GMRES(m) solve of A x = b on an existing context with the order schedule s
 * (Sec. 2.4, 2.6).  b_dev, x_dev: device vectors of n doubles.  tol > 0 is the
 * relative residual target.  Returns OK or ENOCONV (x and report filled). */
int fmmbem_solve_ctx(fmmbem_ctx_t *ctx, const double *b_dev, double tol, const fmmbem_schedule *s,
                     double *x_dev, fmmbem_report *report, void *hip_stream);

/* The same solve as fmmbem_solve_ctx with nothing allocated, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the Krylov workspace
 * (basis, residual, partial sums) comes from one static device array of
 * FMMBEM_STATIC_SCRATCH_BYTES per device, held until the process ends, and
 * the Hessenberg column from pinned memory the context made at build.
 * GMRES(m) on n unknowns needs about 8 ((m + 3) n + 2 (m + 1) 256) bytes;
 * EINVAL beyond the array, for restart > FMMBEM_STATIC_MAX_RESTART, when the
 * context's device is not the current one, or while per-stage timing is on.
 * Every call on one device shares that array: calls that overlap on one
 * device (any contexts, any streams) race.  Results equal fmmbem_solve_ctx's
 * bit for bit.  Synchronises hip_stream like fmmbem_solve_ctx. */
#define FMMBEM_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
#define FMMBEM_STATIC_MAX_RESTART 64
int fmmbem_solve_ctx_static(fmmbem_ctx_t *ctx, const double *b_dev, double tol, const fmmbem_schedule *s,
                            double *x_dev, fmmbem_report *report, void *hip_stream);

/* One-shot solve: build with default params (mu from params when given),
 * copy bc (n doubles, host) to the device, solve, copy x back (host). */
int fmmbem_solve(const fmmbem_mesh *mesh, const double *bc_host, int kernel, double tol,
                 const fmmbem_schedule *s, const fmmbem_params *params, double *x_host,
                 fmmbem_report *report);

int fmmbem_get_stats(const fmmbem_ctx_t *ctx, fmmbem_stats *out);
void fmmbem_destroy(fmmbem_ctx_t *ctx);
const char *fmmbem_last_error(void);

/* Per-stage device time, accumulated with HIP events recorded on the stream
 * each kernel is launched on, while timing is enabled.  Stages: 0 P2P (one
 * kernel), 1 M2L pass 1 (the per-pair translations, one kernel), 2 P2M+M2M,
 * 3 the downward pass: the per-target sum of the M2L terms, L2L and L2P (L2P
 * also combines far field, near field and corrections, after waiting for the
 * near field; at low orders L2L and L2P run as one kernel per leaf), 4
 * charges (+ the combine when no box pair is far; inside a solve the charges
 * of a prefetched mat-vec also normalise the Arnoldi vector and are counted
 * where they are launched); entry [prec * 5 + stage] holds the launches made
 * in precision prec (FMMBEM_FP64 = 0, FMMBEM_FP32 = 1); entry 10 holds the
 * Krylov kernels of solves (FP64: Gram-Schmidt dots and update, stand-alone
 * normalisations, update of x, true residuals); FMMBEM_N_STAGES entries in
 * all.  t_ms[i] is the total time, launches[i] the number of timed launches
 * and flops[i] the algorithmic flops of those launches: P2P evaluated on the
 * fly counts 12 (Laplace single layer), 18 (double layer) or 30 (Stokes) per
 * source-target pair, the stored near field 2 per stored value (9 values
 * per panel pair for Stokes), M2L 4 (p + 1)^3 (p + 2) per box pair and
 * channel (the complex translation of Sec. 2.5 as the method states it; the
 * kernels apply it as a real (2 ncoef(p))^2 operator, 8 ncoef(p)^2 flops);
 * the other stages count 0.  Any output pointer may be NULL. */
#define FMMBEM_N_STAGES 11
int fmmbem_set_timing(fmmbem_ctx_t *ctx, int enabled);
/* Times only the stages whose bit is set in mask (bit prec * 5 + stage, or
 * 10 for the Krylov kernels: the entry layout of fmmbem_get_timing); every timed stage records two events on
 * its stream per mat-vec, so a narrow mask keeps the host work of a timed
 * solve close to that of an untimed one.  0 turns timing off; bits at or past
 * FMMBEM_N_STAGES give FMMBEM_EINVAL. */
int fmmbem_set_timing_stages(fmmbem_ctx_t *ctx, uint32_t mask);
int fmmbem_get_timing(fmmbem_ctx_t *ctx, double *t_ms, int64_t *launches, double *flops, int reset);

/* Introspection for tests: sizes, then copies of the tree and lists in the
 * same layout as the CPU reference (sorted order):
 *   sizes[4] = n_boxes, n_levels, n_m2l, n_p2p
 *   perm[N] (sorted position -> caller triangle), keys[N] (63-bit Morton),
 *   boxes[n_boxes][6] = level, begin, end, parent, first child, child count,
 *   box_real[n_boxes][5] = centre x, y, z, radius, guard,
 *   m2l[n_m2l][2], p2p[n_p2p][2] = (target box, source box) sorted,
 *   cube[4] = lower corner x, y, z, side.
 * Any output pointer may be NULL. */
int fmmbem_tree_sizes(const fmmbem_ctx_t *ctx, int64_t *sizes);
int fmmbem_tree_get(const fmmbem_ctx_t *ctx, int32_t *perm, uint64_t *keys, int32_t *boxes,
                    double *box_real, int32_t *m2l, int32_t *p2p, double *cube);

/* ---- request loop (continuous batching of solves) ---- */
typedef struct {
    int64_t hbm_budget_bytes;  /* admission limit on device memory of admitted requests */
    int32_t max_active;        /* most requests on the device at once */
    int32_t n_streams;         /* HIP streams the active requests are spread over */
} fmmbem_server_params;

typedef struct {
    double arrival_s, admit_s, finish_s;  /* server clock (seconds since create) */
    int32_t iterations, converged;
    double rel_res_true;
    int64_t device_bytes;
} fmmbem_request_info;

/* Create a server whose worker thread admits queued requests while their
 * estimated device footprint fits the budget and a slot is free, and advances
 * every admitted solve by one GMRES iteration per tick. */
int fmmbem_server_create(const fmmbem_server_params *p, fmmbem_server_t **out);
/* Queue a solve; mesh and bc are copied.  ticket identifies it. */
int fmmbem_submit(fmmbem_server_t *srv, const fmmbem_mesh *mesh, const double *bc_host, int kernel,
                  double tol, const fmmbem_schedule *s, const fmmbem_params *params, uint64_t *ticket);
/* done = 1 once the request finished (successfully or not). */
int fmmbem_poll(fmmbem_server_t *srv, uint64_t ticket, int *done);
/* Block until finished, copy x (n doubles) and the request info; releases the
 * request.  Returns the request's own status (OK, ENOCONV, ...). */
int fmmbem_wait(fmmbem_server_t *srv, uint64_t ticket, double *x_host, fmmbem_request_info *info);
void fmmbem_server_destroy(fmmbem_server_t *srv);

#ifdef __cplusplus
}
#endif
#endif
