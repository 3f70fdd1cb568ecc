// Request loop: continuous batching of BEM solves of uneven sizes.
//
// A worker thread owns the device work.  Queued requests are admitted in
// arrival order while a slot is free and their estimated device footprint
// fits the budget; each admitted request gets its own context (octree, lists,
// corrections, Krylov basis, all resident on the device) and one of the
// server's streams.  A tick advances every active solve by one GMRES
// iteration: all solves first enqueue their mat-vec and orthogonalisation on
// their streams, so the device overlaps them, and only then does the thread
// wait for each and apply its Givens update.  A finished request releases its
// device memory and slot at once, and the next queued request is admitted in
// the same tick.  Each solve's arithmetic is independent of the others, so a
// result is bitwise the same alone or in the mix.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

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
    // state
    int status = FMMBEM_OK;
    bool done = false;
    fmmbem_request_info info{};
    fmmbem_ctx *ctx = nullptr;
    double *d_b = nullptr, *d_x = nullptr;
    std::unique_ptr<GmresState> gm;
    int stream = 0;
};

int64_t estimate_bytes(int64_t nt, int kernel, const fmmbem_params &prm, const fmmbem_schedule &s)
{
    const int64_t n = kernel == FMMBEM_STOKES_SL ? 3 * nt : nt;
    const int nch = kernel == FMMBEM_STOKES_SL ? 4 : 1;
    const int64_t nbox = 2 + (nt * 8) / std::max(1, prm.ncrit);  // generous
    int64_t geo = nt * (24 + 8 + 72 + 128 + 12 + 64 + 8 + 4 + 4);
    int64_t corr = nt * 32 * (4 + 8 * (kernel == FMMBEM_STOKES_SL ? 9 : 1));
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

}  // namespace

struct fmmbem_server {
    fmmbem_server_params prm{};
    int device = 0;
    std::vector<hipStream_t> streams;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::map<uint64_t, std::unique_ptr<Request>> all;
    std::vector<Request *> active;
    int64_t used_bytes = 0;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;
    std::chrono::steady_clock::time_point t_origin;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t_origin).count();
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
            r->info.device_bytes = r->ctx->arena.bytes;
            fmmbem_destroy(r->ctx);
            r->ctx = nullptr;
        }
        r->d_b = r->d_x = nullptr;  // held by the context's arena
        r->info.finish_s = now();
        std::lock_guard<std::mutex> lk(mu);
        used_bytes -= r->est_bytes;
        r->done = true;
        cv_done.notify_all();
    }

    // build the context and start the solve; false if it failed (request finished)
    bool activate(Request *r)
    {
        r->info.admit_s = now();
        try {
            fmmbem_mesh mesh{(int64_t)(r->xyz.size() / 3), (int64_t)(r->tri.size() / 3), r->xyz.data(), r->tri.data()};
            hipStream_t st = streams[r->stream];
            int rc = fmmbem_build(&mesh, r->kernel, &r->prm, st, &r->ctx);
            if (rc != FMMBEM_OK) {
                finish(r, rc);
                return false;
            }
            r->d_b = r->ctx->arena.alloc<double>(r->ctx->n);
            r->d_x = r->ctx->arena.alloc<double>(r->ctx->n);
            FB_HIP(hipMemcpyAsync(r->d_b, r->bc.data(), sizeof(double) * r->ctx->n, hipMemcpyHostToDevice, st));
            r->gm.reset(new GmresState(r->ctx, r->d_b, r->tol, &r->sched, r->d_x, st));
            r->gm->start();
            if (r->gm->done) {
                finish(r, r->gm->converged ? FMMBEM_OK : FMMBEM_ENOCONV);
                return false;
            }
        } catch (const Error &e) {
            set_last_error(e.what());
            finish(r, e.code);
            return false;
        } catch (...) {
            finish(r, FMMBEM_EINTERNAL);
            return false;
        }
        return true;
    }

    void loop()
    {
        (void)hipSetDevice(device);
        int rr = 0;
        while (true) {
            std::vector<Request *> admit;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] { return stop || !queue.empty() || !active.empty(); });
                if (stop)
                    break;
                while (!queue.empty() && (int)(active.size() + admit.size()) < prm.max_active) {
                    Request *r = queue.front();
                    if (used_bytes + r->est_bytes > prm.hbm_budget_bytes && !(active.empty() && admit.empty()))
                        break;  // wait for memory; a lone request is always admitted
                    queue.pop_front();
                    used_bytes += r->est_bytes;
                    admit.push_back(r);
                }
            }
            for (Request *r : admit) {
                r->stream = rr++ % (int)streams.size();
                if (activate(r))
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
        for (int i = 0; i < s->prm.n_streams; ++i) {
            hipStream_t st;
            FB_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
            s->streams.push_back(st);
        }
        s->t_origin = std::chrono::steady_clock::now();
        s->worker = std::thread([s] { s->loop(); });
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
        if (r->sched.p_init > r->prm.p_max)
            r->prm.p_max = std::min(r->sched.p_init, FMMBEM_P_MAX);
        r->est_bytes = estimate_bytes(mesh->n_triangles, kernel, r->prm, r->sched);
        std::lock_guard<std::mutex> lk(srv->mu);
        r->ticket = srv->next_ticket++;
        r->info.arrival_s = srv->now();
        *ticket = r->ticket;
        srv->queue.push_back(r.get());
        srv->all[r->ticket] = std::move(r);
        srv->cv_work.notify_all();
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
    }
    if (srv->worker.joinable())
        srv->worker.join();
    for (auto st : srv->streams)
        (void)hipStreamDestroy(st);
    delete srv;
}

}  // extern "C"
