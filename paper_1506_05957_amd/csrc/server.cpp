// Request loop: continuous batching of BEM solves of uneven sizes.
//
// Two host threads own the device work.  Queued requests are admitted in
// arrival order while a slot is free and their device footprint fits the
// budget; an admitted request is handed to the builder thread, which builds
// its context (octree, lists, corrections, Krylov basis, all resident on the
// device) on a stream of its own, so a build never stalls the solves in
// flight.  Until its context exists a request holds an upper estimate of its
// footprint against the budget; once built it holds the context's real device
// bytes, and the difference goes back to admission at once.  The worker
// thread starts built requests on one of the server's streams and, each
// tick, advances every active solve by one GMRES iteration: all solves first
// enqueue their mat-vec and orthogonalisation on their streams, so the device
// overlaps them, and only then does the thread wait for each and apply its
// Givens update.  A finished request releases its device memory and slot at
// once.  Each solve's arithmetic is independent of the others, so a result is
// bitwise the same alone or in the mix.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "common.h"

using namespace fmmbem;

namespace {

struct Request {
    uint64_t ticket = 0;
    int kernel = 0;
    std::vector<double> xyz, bc, x;
    std::vector<int32_t> tri;
    double tol = 1e-6;
    fmmbem_schedule sched{};
    fmmbem_params prm{};
    int64_t est_bytes = 0;
    int64_t held_bytes = 0;  // charged against the budget: the estimate, then the real bytes
    // state
    int status = FMMBEM_OK;
    bool done = false;
    fmmbem_request_info info{};
    fmmbem_ctx *ctx = nullptr;
    double *d_b = nullptr, *d_x = nullptr;
    std::unique_ptr<GmresState> gm;
    int stream = 0;
};

// An upper estimate of a request's device footprint, used until its context
// is built.
int64_t estimate_bytes(int64_t nt, int kernel, const fmmbem_params &prm, const fmmbem_schedule &s)
{
    const int64_t n = kernel == FMMBEM_STOKES_SL ? 3 * nt : nt;
    const int nch = kernel == FMMBEM_STOKES_SL ? 4 : 1;
    const int64_t nbox = 2 + (nt * 8) / std::max(1, prm.ncrit);  // generous
    int64_t geo = nt * (24 + 8 + 72 + 128 + 12 + 64 + 8 + 4 + 4);
    int64_t corr = nt * 32 * (4 + (8 + 4) * (kernel == FMMBEM_STOKES_SL ? 9 : 1));  // FP64 and FP32 values
    int64_t exp = 3 * nbox * nch * ncoef(prm.p_max) * 16;
    const int64_t dop = 2 * ncoef(prm.p_max);
    int64_t ops = 8 * dop * dop * (8 + 8 + 4 + 4);  // M2M and L2L octant operators, FP64 and FP32
    int64_t lists = nbox * 400 * 4;
    int64_t work = 4 * nt * nch * 8 + 2 * n * 8;
    int64_t kry = ((int64_t)s.restart + 4) * n * 8;
    int64_t io = 2 * n * 8;
    // stored near field: about ncrit / 2 panels in each of ~20 neighbouring
    // leaves per target, FP64 + FP32 values (x 9 for Stokes)
    int64_t near = prm.near_stored ? nt * 10 * prm.ncrit * 12 * (kernel == FMMBEM_STOKES_SL ? 9 : 1) : 0;
    // stored M2L operators: at most 316 offsets per level pair class
    const int64_t ntrans = std::min<int64_t>(nbox * 27, 20000);
    int64_t m2l = prm.m2l_stored ? ntrans * ((dop + 15) / 16) * 16 * ((dop + 3) / 4) * 4 * 8 : 0;
    return geo + corr + exp + ops + lists + work + kry + io + near + m2l + (16 << 20);
}

int64_t context_bytes(const fmmbem_ctx *ctx)
{
    return ctx->arena.bytes + (ctx->kw ? ctx->kw->arena.bytes : 0);
}

// Memory of the requests' contexts.  hipFree and hipHostFree wait for the
// whole device, which would drain every other request's work each time one
// ends; so blocks that a finished request gives back are kept, by size class,
// and handed to later requests, and go back to HIP only when the server is
// destroyed (or, for device memory, when an allocation fails: then every
// cached block is freed and the allocation tried once more).
struct BlockPool {
    bool pinned = false;
    std::mutex mu;
    std::multimap<size_t, void *> cached;
    std::map<void *, size_t> cls;  // every block made, with its size class

    static size_t size_class(size_t b)
    {
        if (b <= ((size_t)64 << 10)) {
            size_t c = 256;
            while (c < b)
                c <<= 1;
            return c;
        }
        const size_t g = (size_t)1 << 20;
        return (b + g - 1) / g * g;
    }
    void *make(size_t c)
    {
        void *p = nullptr;
        if (pinned)
            return hipHostMalloc(&p, c, hipHostMallocMapped) == hipSuccess ? p : nullptr;
        return hipMalloc(&p, c) == hipSuccess ? p : nullptr;
    }
    void drop(void *p)
    {
        if (pinned)
            (void)hipHostFree(p);
        else
            (void)hipFree(p);
    }
    void *get(size_t b)
    {
        const size_t c = size_class(b);
        {
            std::lock_guard<std::mutex> lk(mu);
            auto it = cached.find(c);
            if (it != cached.end()) {
                void *p = it->second;
                cached.erase(it);
                return p;
            }
        }
        void *p = make(c);
        if (!p && !pinned) {
            trim();
            p = make(c);
        }
        if (p) {
            std::lock_guard<std::mutex> lk(mu);
            cls[p] = c;
        }
        return p;
    }
    void put(void *p)
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cls.find(p);
        if (it != cls.end())
            cached.emplace(it->second, p);
    }
    void trim()
    {
        std::lock_guard<std::mutex> lk(mu);
        for (auto &kv : cached) {
            drop(kv.second);
            cls.erase(kv.second);
        }
        cached.clear();
    }
    ~BlockPool()
    {
        for (auto &kv : cls)
            drop(kv.first);
    }
    static void *get_cb(size_t b, void *u) { return static_cast<BlockPool *>(u)->get(b); }
    static void put_cb(void *p, void *u) { static_cast<BlockPool *>(u)->put(p); }
};

}  // namespace

struct fmmbem_server {
    fmmbem_server_params prm{};
    int device = 0;
    BlockPool dev_pool, host_pool;  // declared first: released after every context
    PinnedProvider pinned{BlockPool::get_cb, BlockPool::put_cb, nullptr};
    std::vector<hipStream_t> streams;
    hipStream_t build_stream = nullptr;
    std::mutex mu;
    std::condition_variable cv_work, cv_build, cv_done;
    std::deque<Request *> queue;     // waiting for admission
    std::deque<Request *> to_build;  // admitted, waiting for the builder
    std::deque<Request *> ready;     // built, waiting for the worker
    std::map<uint64_t, std::unique_ptr<Request>> all;
    std::vector<Request *> active;   // worker thread only
    int n_admitted = 0;              // admitted and not finished (building, ready or active)
    int64_t used_bytes = 0;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker, builder;
    std::chrono::steady_clock::time_point t_origin;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t_origin).count();
    }

    // admit queued requests in arrival order while a slot is free and the
    // footprint fits; a request alone is always admitted (called with mu held)
    void admit_locked()
    {
        bool any = false;
        while (!queue.empty() && n_admitted < prm.max_active) {
            Request *r = queue.front();
            if (used_bytes + r->est_bytes > prm.hbm_budget_bytes && n_admitted > 0)
                break;  // wait for memory
            queue.pop_front();
            r->held_bytes = r->est_bytes;
            used_bytes += r->held_bytes;
            ++n_admitted;
            r->info.admit_s = now();
            to_build.push_back(r);
            any = true;
        }
        if (any)
            cv_build.notify_all();
    }

    void finish(Request *r, int status)
    {
        r->status = status;
        try {
            if (r->d_x && status != FMMBEM_EINVAL) {
                r->x.resize(r->ctx ? r->ctx->n : 0);
                if (!r->x.empty())
                    FB_HIP(hipMemcpy(r->x.data(), r->d_x, sizeof(double) * r->x.size(), hipMemcpyDeviceToHost));
            }
        } catch (const Error &e) {
            r->status = e.code;
        }
        if (r->gm) {
            r->info.iterations = r->gm->it;
            r->info.converged = r->gm->converged;
            r->info.rel_res_true = r->gm->true_rel;
        }
        r->gm.reset();
        if (r->ctx) {
            r->info.device_bytes = context_bytes(r->ctx);
            // only this request's streams are waited for, not the device
            (void)hipStreamSynchronize(streams[r->stream]);
            if (r->ctx->side)
                (void)hipStreamSynchronize(r->ctx->side);
            destroy_context(r->ctx, false);
            r->ctx = nullptr;
        }
        r->d_b = r->d_x = nullptr;  // held by the context's arena
        r->info.finish_s = now();
        std::lock_guard<std::mutex> lk(mu);
        used_bytes -= r->held_bytes;
        r->held_bytes = 0;
        --n_admitted;
        r->done = true;
        admit_locked();
        cv_done.notify_all();
    }

    // builder thread: context, device copies of b and x, Krylov workspace
    void build_loop()
    {
        (void)hipSetDevice(device);
        t_pinned = &pinned;
        while (true) {
            Request *r;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_build.wait(lk, [&] { return stop || !to_build.empty(); });
                if (stop)
                    break;
                r = to_build.front();
                to_build.pop_front();
            }
            try {
                fmmbem_mesh mesh{(int64_t)(r->xyz.size() / 3), (int64_t)(r->tri.size() / 3), r->xyz.data(),
                                 r->tri.data()};
                int rc = fmmbem_build(&mesh, r->kernel, &r->prm, build_stream, &r->ctx);
                if (rc != FMMBEM_OK) {
                    finish(r, rc);
                    continue;
                }
                r->d_b = r->ctx->arena.alloc<double>(r->ctx->n);
                r->d_x = r->ctx->arena.alloc<double>(r->ctx->n);
                FB_HIP(hipMemcpyAsync(r->d_b, r->bc.data(), sizeof(double) * r->ctx->n, hipMemcpyHostToDevice,
                                      build_stream));
                reserve_krylov(r->ctx, r->sched.restart);
                FB_HIP(hipStreamSynchronize(build_stream));
            } catch (const Error &e) {
                set_last_error(e.what());
                (void)hipStreamSynchronize(build_stream);
                finish(r, e.code);
                continue;
            } catch (...) {
                (void)hipStreamSynchronize(build_stream);
                finish(r, FMMBEM_EINTERNAL);
                continue;
            }
            std::lock_guard<std::mutex> lk(mu);
            const int64_t real = context_bytes(r->ctx);
            used_bytes += real - r->held_bytes;
            r->held_bytes = real;
            ready.push_back(r);
            admit_locked();
            cv_work.notify_all();
        }
    }

    // start the solve of a built request; false if it finished already
    bool start(Request *r)
    {
        try {
            hipStream_t st = streams[r->stream];
            r->gm.reset(new GmresState(r->ctx, r->d_b, r->tol, &r->sched, r->d_x, st));
            r->gm->start();
            if (r->gm->done) {
                finish(r, r->gm->converged ? FMMBEM_OK : FMMBEM_ENOCONV);
                return false;
            }
        } catch (const Error &e) {
            set_last_error(e.what());
            (void)hipStreamSynchronize(streams[r->stream]);
            finish(r, e.code);
            return false;
        } catch (...) {
            (void)hipStreamSynchronize(streams[r->stream]);
            finish(r, FMMBEM_EINTERNAL);
            return false;
        }
        return true;
    }

    void loop()
    {
        (void)hipSetDevice(device);
        t_pinned = &pinned;
        int rr = 0;
        while (true) {
            std::vector<Request *> fresh;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] { return stop || !ready.empty() || !active.empty(); });
                if (stop)
                    break;
                fresh.assign(ready.begin(), ready.end());
                ready.clear();
            }
            for (Request *r : fresh) {
                r->stream = rr++ % (int)streams.size();
                if (start(r))
                    active.push_back(r);
            }
            if (active.empty())
                continue;
            // one GMRES iteration for every active solve: enqueue all, then complete
            std::vector<Request *> still;
            for (Request *r : active) {
                try {
                    r->gm->enqueue_step();
                } catch (const Error &e) {
                    set_last_error(e.what());
                    (void)hipStreamSynchronize(streams[r->stream]);
                    r->gm->done = true;
                    r->status = e.code;
                }
            }
            for (Request *r : active) {
                if (r->gm->done && r->status != FMMBEM_OK) {
                    finish(r, r->status);
                    continue;
                }
                try {
                    r->gm->complete_step();
                } catch (const Error &e) {
                    set_last_error(e.what());
                    (void)hipStreamSynchronize(streams[r->stream]);
                    finish(r, e.code);
                    continue;
                }
                if (r->gm->done)
                    finish(r, r->gm->converged ? FMMBEM_OK : FMMBEM_ENOCONV);
                else
                    still.push_back(r);
            }
            active.swap(still);
        }
        // drain: release whatever is still active
        for (Request *r : active) {
            (void)hipStreamSynchronize(streams[r->stream]);
            finish(r, FMMBEM_EBUSY);
        }
        active.clear();
    }
};

extern "C" {

int fmmbem_server_create(const fmmbem_server_params *p, fmmbem_server_t **out)
{
    try {
        FB_REQUIRE(out != nullptr, FMMBEM_EINVAL, "out is NULL");
        *out = nullptr;
        auto *s = new fmmbem_server();
        s->prm.hbm_budget_bytes = (int64_t)8 << 30;
        s->prm.max_active = 16;
        s->prm.n_streams = 4;
        if (p)
            s->prm = *p;
        if (s->prm.max_active < 1 || s->prm.n_streams < 1 || s->prm.hbm_budget_bytes <= 0 || s->prm.n_streams > 64) {
            delete s;
            throw Error(FMMBEM_EINVAL, "server params out of range");
        }
        FB_HIP(hipGetDevice(&s->device));
        s->host_pool.pinned = true;
        s->pinned.user = &s->host_pool;
        for (int i = 0; i < s->prm.n_streams; ++i) {
            hipStream_t st;
            FB_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
            s->streams.push_back(st);
        }
        FB_HIP(hipStreamCreateWithFlags(&s->build_stream, hipStreamNonBlocking));
        s->t_origin = std::chrono::steady_clock::now();
        s->worker = std::thread([s] { s->loop(); });
        s->builder = std::thread([s] { s->build_loop(); });
        *out = s;
        return FMMBEM_OK;
    } catch (const Error &e) {
        set_last_error(e.what());
        return e.code;
    } catch (...) {
        set_last_error("server create failed");
        return FMMBEM_EINTERNAL;
    }
}

int fmmbem_submit(fmmbem_server_t *srv, const fmmbem_mesh *mesh, const double *bc_host, int kernel, double tol,
                  const fmmbem_schedule *s, const fmmbem_params *params, uint64_t *ticket)
{
    try {
        FB_REQUIRE(srv && mesh && bc_host && s && ticket, FMMBEM_EINVAL, "null argument");
        FB_REQUIRE(mesh->xyz && mesh->tri && mesh->n_triangles >= 1 && mesh->n_vertices >= 3, FMMBEM_EINVAL,
                   "empty mesh");
        FB_REQUIRE(kernel == FMMBEM_LAPLACE_SL || kernel == FMMBEM_STOKES_SL || kernel == FMMBEM_LAPLACE_DL,
                   FMMBEM_EINVAL, "unknown kernel");
        FB_REQUIRE(tol > 0.0, FMMBEM_EINVAL, "tol must be positive");
        auto r = std::make_unique<Request>();
        r->kernel = kernel;
        r->xyz.assign(mesh->xyz, mesh->xyz + 3 * mesh->n_vertices);
        r->tri.assign(mesh->tri, mesh->tri + 3 * mesh->n_triangles);
        const int64_t n = kernel == FMMBEM_STOKES_SL ? 3 * mesh->n_triangles : mesh->n_triangles;
        r->bc.assign(bc_host, bc_host + n);
        r->tol = tol;
        r->sched = *s;
        fmmbem_params_default(&r->prm);
        if (params)
            r->prm = *params;
        if (!r->prm.alloc) {  // the server's own cache of device blocks
            r->prm.alloc = BlockPool::get_cb;
            r->prm.free = BlockPool::put_cb;
            r->prm.alloc_user = &srv->dev_pool;
        }
        if (r->sched.p_init > r->prm.p_max)
            r->prm.p_max = std::min(r->sched.p_init, FMMBEM_P_MAX);
        r->est_bytes = estimate_bytes(mesh->n_triangles, kernel, r->prm, r->sched);
        std::lock_guard<std::mutex> lk(srv->mu);
        r->ticket = srv->next_ticket++;
        r->info.arrival_s = srv->now();
        *ticket = r->ticket;
        srv->queue.push_back(r.get());
        srv->all[r->ticket] = std::move(r);
        srv->admit_locked();
        return FMMBEM_OK;
    } catch (const Error &e) {
        set_last_error(e.what());
        return e.code;
    } catch (...) {
        set_last_error("submit failed");
        return FMMBEM_EINTERNAL;
    }
}

int fmmbem_poll(fmmbem_server_t *srv, uint64_t ticket, int *done)
{
    if (!srv || !done) {
        set_last_error("null argument");
        return FMMBEM_EINVAL;
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->all.find(ticket);
    if (it == srv->all.end()) {
        set_last_error("unknown ticket");
        return FMMBEM_EINVAL;
    }
    *done = it->second->done ? 1 : 0;
    return FMMBEM_OK;
}

int fmmbem_wait(fmmbem_server_t *srv, uint64_t ticket, double *x_host, fmmbem_request_info *info)
{
    if (!srv) {
        set_last_error("null argument");
        return FMMBEM_EINVAL;
    }
    std::unique_ptr<Request> r;
    {
        std::unique_lock<std::mutex> lk(srv->mu);
        auto it = srv->all.find(ticket);
        if (it == srv->all.end()) {
            set_last_error("unknown ticket");
            return FMMBEM_EINVAL;
        }
        Request *rp = it->second.get();
        srv->cv_done.wait(lk, [&] { return rp->done; });
        r = std::move(it->second);
        srv->all.erase(it);
    }
    if (x_host && !r->x.empty())
        std::memcpy(x_host, r->x.data(), sizeof(double) * r->x.size());
    if (info)
        *info = r->info;
    return r->status;
}

void fmmbem_server_destroy(fmmbem_server_t *srv)
{
    if (!srv)
        return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        srv->cv_work.notify_all();
        srv->cv_build.notify_all();
    }
    if (srv->builder.joinable())
        srv->builder.join();
    if (srv->worker.joinable())
        srv->worker.join();
    // built but never started: release their contexts
    std::vector<Request *> left;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        left.assign(srv->ready.begin(), srv->ready.end());
        srv->ready.clear();
    }
    for (Request *r : left)
        srv->finish(r, FMMBEM_EBUSY);
    for (auto st : srv->streams)
        (void)hipStreamDestroy(st);
    if (srv->build_stream)
        (void)hipStreamDestroy(srv->build_stream);
    delete srv;
}

}  // extern "C"
