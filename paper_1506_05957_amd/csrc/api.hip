// C-ABI entry points of libfmmbem (declared in include/fmmbem.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "common.h"

namespace fmmbem {

static thread_local std::string g_last_error;
thread_local const PinnedProvider *t_pinned = nullptr;

void set_last_error(const std::string &m) { g_last_error = m; }

// stage clocks only measure time: no system-scope fence when they complete
constexpr unsigned TIMING_EVENT_FLAGS = hipEventDefault | hipEventDisableSystemFence;

void stage_begin(fmmbem_ctx *ctx, int stage, hipStream_t st, hipEvent_t *ev)
{
    *ev = nullptr;
    if (!((ctx->timing.mask >> stage) & 1u))
        return;
    Timing &T = ctx->timing;
    if (T.pool.empty()) {
        hipEvent_t e;
        FB_HIP(hipEventCreateWithFlags(&e, TIMING_EVENT_FLAGS));
        T.pool.push_back(e);
    }
    *ev = T.pool.back();
    T.pool.pop_back();
    FB_HIP(hipEventRecord(*ev, st));
}

void timing_resolve(Timing &T)
{
    for (auto &pd : T.pending) {
        FB_HIP(hipEventSynchronize(pd.b));
        float ms = 0.f;
        FB_HIP(hipEventElapsedTime(&ms, pd.a, pd.b));
        T.t_ms[pd.stage] += ms;
        T.launches[pd.stage] += 1;
        T.pool.push_back(pd.a);
        T.pool.push_back(pd.b);
    }
    T.pending.clear();
}

void stage_end(fmmbem_ctx *ctx, int stage, hipStream_t st, hipEvent_t ev, double flops)
{
    if (!ev)  // stage not timed
        return;
    Timing &T = ctx->timing;
    if (T.pool.empty()) {
        hipEvent_t e;
        FB_HIP(hipEventCreateWithFlags(&e, TIMING_EVENT_FLAGS));
        T.pool.push_back(e);
    }
    hipEvent_t e2 = T.pool.back();
    T.pool.pop_back();
    FB_HIP(hipEventRecord(e2, st));
    T.pending.push_back({ev, e2, stage});
    T.flops[stage] += flops;
    if (T.pending.size() > 4096)
        timing_resolve(T);
}

}  // namespace fmmbem

using namespace fmmbem;

#define API_BEGIN try {
#define API_END                                                                                                      \
    }                                                                                                                \
    catch (const fmmbem::Error &e)                                                                                  \
    {                                                                                                                \
        set_last_error(e.what());                                                                                    \
        return e.code;                                                                                               \
    }                                                                                                                \
    catch (const std::bad_alloc &)                                                                                   \
    {                                                                                                                \
        set_last_error("host allocation failed");                                                                    \
        return FMMBEM_ENOMEM;                                                                                        \
    }                                                                                                                \
    catch (const std::exception &e)                                                                                  \
    {                                                                                                                \
        set_last_error(e.what());                                                                                    \
        return FMMBEM_EINTERNAL;                                                                                     \
    }                                                                                                                \
    catch (...)                                                                                                      \
    {                                                                                                                \
        set_last_error("unknown error");                                                                             \
        return FMMBEM_EINTERNAL;                                                                                     \
    }

extern "C" {

void fmmbem_params_default(fmmbem_params *prm)
{
    if (!prm)
        return;
    prm->theta = 0.5;
    prm->ncrit = 64;
    prm->p_max = 16;
    prm->mu = 1.0;
    prm->near_stored = 0;
    prm->m2l_stored = 0;
    prm->quad_far = 4;
    prm->quad_near = 25;
    prm->near_factor = 2.0;
    prm->alloc = nullptr;
    prm->free = nullptr;
    prm->alloc_user = nullptr;
}

void fmmbem_schedule_default(fmmbem_schedule *s, int kernel)
{
    if (!s)
        return;
    s->rule = FMMBEM_RELAX_BF;
    s->p_init = kernel == FMMBEM_STOKES_SL ? 16 : 12;
    s->p_min = kernel == FMMBEM_STOKES_SL ? 4 : 3;
    s->mixed = 1;
    s->fp32_eps = 1e-5;
    s->restart = 50;
    s->max_iter = 500;
}

const char *fmmbem_last_error(void) { return g_last_error.c_str(); }

static void validate_mesh(const fmmbem_mesh *mesh)
{
    FB_REQUIRE(mesh != nullptr, FMMBEM_EINVAL, "mesh is NULL");
    FB_REQUIRE(mesh->xyz != nullptr && mesh->tri != nullptr, FMMBEM_EINVAL, "mesh arrays are NULL");
    FB_REQUIRE(mesh->n_triangles >= 1, FMMBEM_EINVAL, "mesh has no triangle");
    FB_REQUIRE(mesh->n_vertices >= 3, FMMBEM_EINVAL, "mesh has fewer than 3 vertices");
    FB_REQUIRE(mesh->n_triangles < (int64_t)1 << 29, FMMBEM_EINVAL, "too many triangles (limit 2^29)");
    for (int64_t i = 0; i < 3 * mesh->n_triangles; ++i)
        FB_REQUIRE(mesh->tri[i] >= 0 && mesh->tri[i] < mesh->n_vertices, FMMBEM_EINVAL,
                   "triangle " + std::to_string(i / 3) + " has a vertex index out of range");
    for (int64_t i = 0; i < 3 * mesh->n_vertices; ++i)
        FB_REQUIRE(std::isfinite(mesh->xyz[i]), FMMBEM_EINVAL, "non-finite vertex coordinate");
}

static void validate_params(const fmmbem_params *p)
{
    FB_REQUIRE(p->theta > 0.0 && p->theta < 1.0, FMMBEM_EINVAL, "theta must be in (0, 1)");
    FB_REQUIRE(p->ncrit >= 1 && p->ncrit <= 1024, FMMBEM_EINVAL, "ncrit must be in [1, 1024]");
    FB_REQUIRE(p->p_max >= 1 && p->p_max <= FMMBEM_P_MAX, FMMBEM_EINVAL, "p_max must be in [1, 20]");
    FB_REQUIRE(p->mu > 0.0 && std::isfinite(p->mu), FMMBEM_EINVAL, "mu must be positive");
    FB_REQUIRE(p->near_stored == 0 || p->near_stored == 1, FMMBEM_EINVAL, "near_stored must be 0 or 1");
    FB_REQUIRE(p->m2l_stored >= 0 && p->m2l_stored <= 2, FMMBEM_EINVAL, "m2l_stored must be 0, 1 or 2");
    FB_REQUIRE(p->quad_far == 0 || p->quad_far == 4, FMMBEM_EINVAL, "quad_far: only the 4-point rule is built");
    FB_REQUIRE(p->quad_near == 0 || p->quad_near == 25, FMMBEM_EINVAL, "quad_near: only the 25-point rule is built");
    FB_REQUIRE(p->near_factor == 0.0 || p->near_factor == 2.0, FMMBEM_EINVAL,
               "near_factor: only 2 (|x - c_j|^2 < 8 S_j) is built");
    FB_REQUIRE((p->alloc == nullptr) == (p->free == nullptr), FMMBEM_EINVAL,
               "alloc and free must be given together");
}

int fmmbem_build(const fmmbem_mesh *mesh, int kernel, const fmmbem_params *params, void *hip_stream,
                 fmmbem_ctx_t **out)
{
    API_BEGIN
    FB_REQUIRE(out != nullptr, FMMBEM_EINVAL, "out is NULL");
    *out = nullptr;
    validate_mesh(mesh);
    FB_REQUIRE(kernel == FMMBEM_LAPLACE_SL || kernel == FMMBEM_STOKES_SL || kernel == FMMBEM_LAPLACE_DL,
               FMMBEM_EINVAL, "unknown kernel");
    fmmbem_params prm;
    fmmbem_params_default(&prm);
    if (params)
        prm = *params;
    validate_params(&prm);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    fmmbem_ctx *ctx = new fmmbem_ctx();
    try {
        ctx->kernel = kernel;
        ctx->prm = prm;
        ctx->arena.al = DevAlloc{prm.alloc, prm.free, prm.alloc_user};
        FB_HIP(hipGetDevice(&ctx->device));
        ctx->nt = mesh->n_triangles;
        ctx->nsrc = 4 * ctx->nt;
        ctx->n = kernel == FMMBEM_STOKES_SL ? 3 * ctx->nt : ctx->nt;
        ctx->nch = kernel == FMMBEM_STOKES_SL ? 4 : 1;
        FB_HIP(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
        FB_HIP(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
        FB_HIP(hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
        FB_HIP(hipEventCreateWithFlags(&ctx->ev_h_s, hipEventDisableTiming));
        ctx->hcol_s = pinned_get(sizeof(double) * hcol_len(FMMBEM_STATIC_MAX_RESTART), &ctx->hcol_s_src);
        FB_HIP(hipHostGetDevicePointer((void **)&ctx->hcol_s_dev, ctx->hcol_s, 0));
        build_geometry_and_tree(ctx, mesh, st);
        build_correction(ctx, st);
        build_translations(ctx, st);
        if (prm.near_stored)
            build_near_matrix(ctx, st);
        correction_fp32(ctx, prm.near_stored ? ctx->nearm.rest : ctx->corr, st);
        if (prm.m2l_stored == 1)
            build_m2l_operators(ctx, st);
        const int ncs = ncoef(prm.p_max);
        ctx->charges = ctx->arena.alloc<double>((size_t)(kernel == FMMBEM_LAPLACE_SL ? 4 : 8) * ctx->nsrc);
        ctx->Y = ctx->arena.alloc<double>(2 * (size_t)std::max<int64_t>(ctx->tree.n_m2l, 1) * ctx->nch * ncs);
        ctx->M = ctx->arena.alloc<double>(2 * (size_t)ctx->tree.nbox * ctx->nch * ncs);
        ctx->L = ctx->arena.alloc<double>(2 * (size_t)ctx->tree.nbox * ctx->nch * ncs);
        ctx->y_near = ctx->arena.alloc<double>(ctx->n);
        ctx->y_far = ctx->arena.alloc<double>(ctx->n);
        ctx->y_corr = ctx->arena.alloc<double>(ctx->n);
        FB_HIP(hipStreamSynchronize(st));
    } catch (...) {
        (void)hipStreamSynchronize(st);
        fmmbem_destroy(ctx);  // arena, streams, events and graphs made so far
        throw;
    }
    *out = ctx;
    return FMMBEM_OK;
    API_END
}

int fmmbem_matvec(fmmbem_ctx_t *ctx, int32_t p, int32_t precision, const double *x_dev, double *y_dev,
                  void *hip_stream)
{
    API_BEGIN
    FB_REQUIRE(ctx && x_dev && y_dev, FMMBEM_EINVAL, "null argument");
    FB_REQUIRE(p >= 1 && p <= ctx->prm.p_max, FMMBEM_EINVAL, "p outside [1, p_max]");
    FB_REQUIRE(precision == FMMBEM_FP64 || precision == FMMBEM_FP32, FMMBEM_EINVAL, "unknown precision");
    FB_REQUIRE(precision == FMMBEM_FP64 || p <= FMMBEM_P_MAX_FP32, FMMBEM_EINVAL,
               "FP32 expansions support p <= 14");
    FB_REQUIRE(x_dev + ctx->n <= y_dev || y_dev + ctx->n <= x_dev, FMMBEM_EINVAL, "x and y overlap");
    run_matvec(ctx, p, precision, x_dev, y_dev, static_cast<hipStream_t>(hip_stream));
    return FMMBEM_OK;
    API_END
}

static void validate_schedule(const fmmbem_ctx *ctx, const fmmbem_schedule *s, double tol)
{
    FB_REQUIRE(s != nullptr, FMMBEM_EINVAL, "schedule is NULL");
    FB_REQUIRE(tol > 0.0 && std::isfinite(tol), FMMBEM_EINVAL, "tol must be positive");
    FB_REQUIRE(s->rule >= FMMBEM_FIXED && s->rule <= FMMBEM_RELAX_BF, FMMBEM_EINVAL, "unknown rule");
    FB_REQUIRE(s->p_init >= 1 && s->p_init <= ctx->prm.p_max, FMMBEM_EINVAL, "p_init outside [1, p_max]");
    FB_REQUIRE(s->p_min >= 1 && s->p_min <= s->p_init, FMMBEM_EINVAL, "p_min outside [1, p_init]");
    FB_REQUIRE(s->restart >= 1 && s->restart <= 1000, FMMBEM_EINVAL, "restart outside [1, 1000]");
    FB_REQUIRE(s->max_iter >= 1, FMMBEM_EINVAL, "max_iter must be >= 1");
    FB_REQUIRE(s->fp32_eps > 0.0, FMMBEM_EINVAL, "fp32_eps must be positive");
}

int fmmbem_solve_ctx(fmmbem_ctx_t *ctx, const double *b_dev, double tol, const fmmbem_schedule *s, double *x_dev,
                     fmmbem_report *report, void *hip_stream)
{
    API_BEGIN
    FB_REQUIRE(ctx && b_dev && x_dev, FMMBEM_EINVAL, "null argument");
    validate_schedule(ctx, s, tol);
    return run_solve(ctx, b_dev, tol, s, x_dev, report, static_cast<hipStream_t>(hip_stream));
    API_END
}

int fmmbem_solve_ctx_static(fmmbem_ctx_t *ctx, const double *b_dev, double tol, const fmmbem_schedule *s,
                            double *x_dev, fmmbem_report *report, void *hip_stream)
{
    API_BEGIN
    FB_REQUIRE(ctx && b_dev && x_dev, FMMBEM_EINVAL, "null argument");
    validate_schedule(ctx, s, tol);
    FB_REQUIRE(s->restart <= FMMBEM_STATIC_MAX_RESTART, FMMBEM_EINVAL,
               "restart above FMMBEM_STATIC_MAX_RESTART for the static workspace");
    FB_REQUIRE(ctx->timing.mask == 0u, FMMBEM_EINVAL,
               "per-stage timing creates HIP events: turn it off for the allocation-free solve");
    return run_solve_static(ctx, b_dev, tol, s, x_dev, report, static_cast<hipStream_t>(hip_stream));
    API_END
}

int fmmbem_solve(const fmmbem_mesh *mesh, const double *bc_host, int kernel, double tol, const fmmbem_schedule *s,
                 const fmmbem_params *params, double *x_host, fmmbem_report *report)
{
    API_BEGIN
    FB_REQUIRE(bc_host && x_host, FMMBEM_EINVAL, "null argument");
    fmmbem_params prm;
    fmmbem_params_default(&prm);
    if (params)
        prm = *params;
    if (s && s->p_init > prm.p_max)
        prm.p_max = s->p_init;
    fmmbem_ctx_t *ctx = nullptr;
    int rc = fmmbem_build(mesh, kernel, &prm, nullptr, &ctx);
    if (rc != FMMBEM_OK)
        return rc;
    try {
        validate_schedule(ctx, s, tol);
        // the device copies of bc and x belong to the context (its allocator)
        double *b = ctx->arena.alloc<double>(ctx->n);
        double *x = ctx->arena.alloc<double>(ctx->n);
        FB_HIP(hipMemcpy(b, bc_host, sizeof(double) * ctx->n, hipMemcpyHostToDevice));
        rc = run_solve(ctx, b, tol, s, x, report, nullptr);
        FB_HIP(hipMemcpy(x_host, x, sizeof(double) * ctx->n, hipMemcpyDeviceToHost));
    } catch (...) {
        fmmbem_destroy(ctx);
        throw;
    }
    fmmbem_destroy(ctx);
    return rc;
    API_END
}

int fmmbem_get_stats(const fmmbem_ctx_t *ctx, fmmbem_stats *o)
{
    API_BEGIN
    FB_REQUIRE(ctx && o, FMMBEM_EINVAL, "null argument");
    std::memset(o, 0, sizeof(*o));
    o->n_panels = ctx->nt;
    o->n_unknowns = ctx->n;
    o->n_sources = ctx->nsrc;
    o->n_boxes = ctx->tree.nbox;
    o->n_leaves = ctx->tree.nleaf;
    o->n_levels = ctx->tree.nlevels;
    o->max_leaf = ctx->tree.max_leaf;
    o->n_m2l = ctx->tree.n_m2l;
    o->n_p2p = ctx->tree.n_p2p;
    o->p2p_interactions = ctx->tree.p2p_interactions;
    o->nnz_correction = ctx->corr.nnz;
    o->device_bytes = ctx->arena.bytes + (ctx->kw ? ctx->kw->arena.bytes : 0);
    o->near_entries = ctx->nearm.entries;
    o->n_translations = ctx->m2l.n_trans;
    o->m2l_op_bytes = ctx->m2l.ops_bytes + ctx->m2l.rot_bytes;
    return FMMBEM_OK;
    API_END
}

void fmmbem_destroy(fmmbem_ctx_t *ctx)
{
    destroy_context(ctx, true);
}

}  // extern "C"

namespace fmmbem {

void destroy_context(fmmbem_ctx *ctx, bool sync_device)
{
    if (!ctx)
        return;
    if (sync_device)
        (void)hipDeviceSynchronize();
    for (auto &pd : ctx->timing.pending) {
        (void)hipEventDestroy(pd.a);
        (void)hipEventDestroy(pd.b);
    }
    for (auto e : ctx->timing.pool)
        (void)hipEventDestroy(e);
    free_krylov(ctx);
    ctx->arena.release();
    if (ctx->ev_fork)
        (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_join)
        (void)hipEventDestroy(ctx->ev_join);
    if (ctx->ev_h_s)
        (void)hipEventDestroy(ctx->ev_h_s);
    pinned_put(ctx->hcol_s, ctx->hcol_s_src);
    if (ctx->side)
        (void)hipStreamDestroy(ctx->side);
    delete ctx;
}

}  // namespace fmmbem

extern "C" {

int fmmbem_set_timing(fmmbem_ctx_t *ctx, int enabled)
{
    API_BEGIN
    FB_REQUIRE(ctx, FMMBEM_EINVAL, "null argument");
    ctx->timing.mask = enabled ? (1u << FMMBEM_N_STAGES) - 1u : 0u;
    return FMMBEM_OK;
    API_END
}

int fmmbem_set_timing_stages(fmmbem_ctx_t *ctx, uint32_t mask)
{
    API_BEGIN
    FB_REQUIRE(ctx, FMMBEM_EINVAL, "null argument");
    FB_REQUIRE(mask < (1u << FMMBEM_N_STAGES), FMMBEM_EINVAL, "stage mask has bits past FMMBEM_N_STAGES");
    ctx->timing.mask = mask;
    return FMMBEM_OK;
    API_END
}

int fmmbem_get_timing(fmmbem_ctx_t *ctx, double *t_ms, int64_t *launches, double *flops, int reset)
{
    API_BEGIN
    FB_REQUIRE(ctx, FMMBEM_EINVAL, "null argument");
    timing_resolve(ctx->timing);
    for (int s = 0; s < FMMBEM_N_STAGES; ++s) {
        if (t_ms)
            t_ms[s] = ctx->timing.t_ms[s];
        if (launches)
            launches[s] = ctx->timing.launches[s];
        if (flops)
            flops[s] = ctx->timing.flops[s];
        if (reset) {
            ctx->timing.t_ms[s] = 0.0;
            ctx->timing.launches[s] = 0;
            ctx->timing.flops[s] = 0.0;
        }
    }
    return FMMBEM_OK;
    API_END
}

int fmmbem_tree_sizes(const fmmbem_ctx_t *ctx, int64_t *sizes)
{
    API_BEGIN
    FB_REQUIRE(ctx && sizes, FMMBEM_EINVAL, "null argument");
    sizes[0] = ctx->tree.nbox;
    sizes[1] = ctx->tree.nlevels;
    sizes[2] = ctx->tree.n_m2l;
    sizes[3] = ctx->tree.n_p2p;
    return FMMBEM_OK;
    API_END
}

int fmmbem_tree_get(const fmmbem_ctx_t *ctx, int32_t *perm, uint64_t *keys, int32_t *boxes, double *box_real,
                    int32_t *m2l, int32_t *p2p, double *cube)
{
    API_BEGIN
    FB_REQUIRE(ctx, FMMBEM_EINVAL, "null argument");
    const Tree &T = ctx->tree;
    FB_HIP(hipDeviceSynchronize());
    if (perm)
        FB_HIP(hipMemcpy(perm, T.perm, sizeof(int32_t) * T.nt, hipMemcpyDeviceToHost));
    if (keys)
        FB_HIP(hipMemcpy(keys, T.keys, sizeof(uint64_t) * T.nt, hipMemcpyDeviceToHost));
    if (boxes)
        std::memcpy(boxes, T.h_box_i.data(), sizeof(int32_t) * T.h_box_i.size());
    if (box_real)
        std::memcpy(box_real, T.h_box_r.data(), sizeof(double) * T.h_box_r.size());
    if (m2l && T.n_m2l)
        FB_HIP(hipMemcpy(m2l, T.m2l_pairs, sizeof(int32_t) * 2 * T.n_m2l, hipMemcpyDeviceToHost));
    if (p2p && T.n_p2p)
        FB_HIP(hipMemcpy(p2p, T.p2p_pairs, sizeof(int32_t) * 2 * T.n_p2p, hipMemcpyDeviceToHost));
    if (cube)
        std::memcpy(cube, T.cube, sizeof(double) * 4);
    return FMMBEM_OK;
    API_END
}

}  // extern "C"
