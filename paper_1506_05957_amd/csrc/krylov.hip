// GMRES(m) with a relaxed expansion order (Sec. 2.4, 2.6).
//
// Arnoldi runs on the device in FP64 with classical Gram-Schmidt applied twice
// (CGS2: as stable as modified Gram-Schmidt, and two passes of block-parallel
// dot products instead of k dependent ones); the (k+2)-entry Hessenberg column
// is copied to the host, where the Givens rotations and the least-squares
// update (a few hundred flops) run in FP64.  The rotated residual
// rho_k = |g_{k+1}| / |b| picks the order and precision of the next mat-vec
// (Eq. 17, 19).  A restart and the final check form the true residual with the
// accurate operator (p_init, FP64).  All reductions use a fixed order, so a
// solve is bitwise reproducible.
#include <chrono>
#include <cmath>
#include <vector>

#include "common.h"

namespace fmmbem {

namespace {

constexpr int DOT_BLOCK = 256;
constexpr int DOT_PER_THREAD = 2;

// Classical Gram-Schmidt dots: block (b, g) takes the rows of block b and the
// vectors j = g CGS_JG .. + CGS_JG - 1 and writes part[j][b] = V_j . w' over its
// rows, where w' = w - sum_{j < nv} hprev[j] V_j when hprev is given (the
// first pass's update, recomputed per block and not stored) and w' = w
// otherwise.  The last block to arrive (atomic ticket) sums part[j][0..nb) in
// block order into out[j] for every j and re-arms the ticket.
constexpr int CGS_JG = 8;
__global__ __launch_bounds__(DOT_BLOCK) void k_cgs_dots(int64_t n, const double *__restrict__ V, int64_t ldv, int nv,
                                                         const double *__restrict__ hprev, const double *__restrict__ w,
                                                         double *__restrict__ part, int nb, double *__restrict__ out,
                                                         unsigned int *__restrict__ ticket)
{
    constexpr int NWV = DOT_BLOCK / 64;
    __shared__ double sh[CGS_JG][NWV];
    __shared__ bool last;
    const int b = blockIdx.x, j0 = blockIdx.y * CGS_JG;
    const int nj = min(CGS_JG, nv - j0);
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t base = (int64_t)b * DOT_BLOCK * DOT_PER_THREAD;
    double wl[DOT_PER_THREAD];
#pragma unroll
    for (int k = 0; k < DOT_PER_THREAD; ++k) {
        const int64_t i = base + (int64_t)k * DOT_BLOCK + threadIdx.x;
        double x = 0.0;
        if (i < n) {
            x = w[i];
            if (hprev)
                for (int j = 0; j < nv; ++j)
                    x -= hprev[j] * V[(int64_t)j * ldv + i];
        }
        wl[k] = x;
    }
    for (int jj = 0; jj < nj; ++jj) {
        const double *v = V + (int64_t)(j0 + jj) * ldv;
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < DOT_PER_THREAD; ++k) {
            const int64_t i = base + (int64_t)k * DOT_BLOCK + threadIdx.x;
            if (i < n)
                s += v[i] * wl[k];
        }
        for (int off = 32; off > 0; off >>= 1)
            s += __shfl_down(s, off, 64);
        if (lane == 0)
            sh[jj][wv] = s;
    }
    __syncthreads();
    if ((int)threadIdx.x < nj) {
        double t = 0.0;
        for (int k = 0; k < NWV; ++k)
            t += sh[threadIdx.x][k];
        part[(int64_t)(j0 + threadIdx.x) * nb + b] = t;
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0)
        last = atomicAdd(ticket, 1u) == (unsigned)(nb * gridDim.y - 1);
    __syncthreads();
    if (!last)
        return;
    __threadfence();
    for (int j = threadIdx.x; j < nv; j += DOT_BLOCK) {
        double t = 0.0;
        for (int k = 0; k < nb; ++k)
            t += __builtin_nontemporal_load(&part[(int64_t)j * nb + k]);
        out[j] = t;
    }
    if (threadIdx.x == 0)
        *ticket = 0u;
}

// w -= sum_{j<nv} (h1[j] + h2[j]) V_j (both Gram-Schmidt passes), and |w|^2
// into *nrm2 (same last-block scheme)
__global__ __launch_bounds__(DOT_BLOCK) void k_update_norm(int64_t n, const double *__restrict__ V, int64_t ldv,
                                                            int nv, const double *__restrict__ h1,
                                                            const double *__restrict__ h2, double *__restrict__ w,
                                                            double *__restrict__ part, int nb,
                                                            double *__restrict__ nrm2, unsigned int *__restrict__ ticket)
{
    __shared__ double sh[DOT_BLOCK / 64];
    __shared__ bool last;
    const int b = blockIdx.x;
    double s = 0.0;
    const int64_t base = (int64_t)b * DOT_BLOCK * DOT_PER_THREAD;
    for (int k = 0; k < DOT_PER_THREAD; ++k) {
        int64_t i = base + (int64_t)k * DOT_BLOCK + threadIdx.x;
        if (i < n) {
            double x = w[i];
            for (int j = 0; j < nv; ++j)
                x -= (h1[j] + h2[j]) * V[(int64_t)j * ldv + i];
            w[i] = x;
            s += x * x;
        }
    }
    for (int off = 32; off > 0; off >>= 1)
        s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0)
        sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < DOT_BLOCK / 64; ++k)
            t += sh[k];
        part[b] = t;
        __threadfence();
        last = atomicAdd(ticket, 1u) == (unsigned)(nb - 1);
    }
    __syncthreads();
    if (!last)
        return;
    __threadfence();
    double t = 0.0;
    for (int k = threadIdx.x; k < nb; k += DOT_BLOCK)
        t += __builtin_nontemporal_load(&part[k]);
    for (int off = 32; off > 0; off >>= 1)
        t += __shfl_down(t, off, 64);
    if ((threadIdx.x & 63) == 0)
        sh[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (int k = 0; k < DOT_BLOCK / 64; ++k)
            r += sh[k];
        *nrm2 = r;
        *ticket = 0u;
    }
}

// v = w / sqrt(nrm2[0])
__global__ void k_normalize(int64_t n, const double *__restrict__ w, const double *__restrict__ nrm2,
                            double *__restrict__ v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    v[i] = w[i] / sqrt(nrm2[0]);
}

// x += sum_{j<nv} y[j] V_j
__global__ void k_xupdate(int64_t n, const double *__restrict__ V, int64_t ldv, int nv, const double *__restrict__ y,
                          double *__restrict__ x)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    double s = x[i];
    for (int j = 0; j < nv; ++j)
        s += y[j] * V[(int64_t)j * ldv + i];
    x[i] = s;
}

__global__ void k_sub(int64_t n, const double *__restrict__ b, const double *__restrict__ a, double *__restrict__ r)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        r[i] = b[i] - a[i];
}

KrylovWork *get_work(fmmbem_ctx *ctx, int m)
{
    KrylovWork *kw = ctx->kw;
    if (kw && kw->m >= m)
        return kw;
    if (kw) {
        kw->arena.release();
        delete kw;
        ctx->kw = nullptr;
    }
    kw = new KrylovWork();
    try {
        kw->m = m;
        kw->n = ctx->n;
        kw->nb = (int)((ctx->n + DOT_BLOCK * DOT_PER_THREAD - 1) / (DOT_BLOCK * DOT_PER_THREAD));
        kw->V = kw->arena.alloc<double>((size_t)(m + 1) * ctx->n);
        kw->w = kw->arena.alloc<double>(ctx->n);
        kw->r = kw->arena.alloc<double>(ctx->n);
        kw->part = kw->arena.alloc<double>((size_t)(m + 2) * kw->nb);
        kw->h = kw->arena.alloc<double>(2 * (size_t)(m + 2));
        kw->y = kw->arena.alloc<double>(m + 1);
        kw->ticket = kw->arena.alloc<unsigned int>(m + 2);
        FB_HIP(hipMemset(kw->ticket, 0, sizeof(unsigned int) * (m + 2)));
    } catch (...) {
        kw->arena.release();
        delete kw;
        throw;
    }
    ctx->kw = kw;
    return kw;
}

// out[0..nv) = V_j . w  (device); with hprev, w -= sum_j hprev[j] V_j first
void multidot(KrylovWork *kw, const double *V, int nv, const double *w, double *out, hipStream_t st,
              const double *hprev = nullptr)
{
    dim3 grid(kw->nb, (nv + CGS_JG - 1) / CGS_JG);
    k_cgs_dots<<<grid, DOT_BLOCK, 0, st>>>(kw->n, V, kw->n, nv, hprev, w, kw->part, kw->nb, out, kw->ticket);
    FB_HIP(hipGetLastError());
}

Sched choose(const fmmbem_schedule *s, double rho, double eta)
{
    double rm = std::min(rho, 1.0);
    double eps = std::min(eta / rm, 1.0);
    int p = s->p_init;
    if (s->rule == FMMBEM_RELAX_SHIFT) {
        p = s->p_init + (int)std::ceil(std::log2(rm));
    } else if (s->rule == FMMBEM_RELAX_BF) {
        p = (int)std::ceil(-std::log2(eps));
    }
    p = std::max(s->p_min, std::min(s->p_init, p));
    int prec = FMMBEM_FP64;
    if (s->mixed && s->rule != FMMBEM_FIXED && eps >= s->fp32_eps && p <= P_MAX_FP32)
        prec = FMMBEM_FP32;
    return {p, prec};
}

}  // namespace

void free_krylov(fmmbem_ctx *ctx)
{
    if (ctx->kw) {
        ctx->kw->arena.release();
        delete ctx->kw;
        ctx->kw = nullptr;
    }
}

GmresState::GmresState(fmmbem_ctx *c, const double *b_, double tol_, const fmmbem_schedule *s_, double *x_,
                       hipStream_t st_)
    : ctx(c), b(b_), x(x_), s(*s_), tol(tol_), st(st_)
{
    const int m = s.restart;
    kw = get_work(ctx, m);
    H.assign((size_t)(m + 1) * m, 0.0);
    cs.assign(m, 0.0);
    sn.assign(m, 0.0);
    g.assign(m + 1, 0.0);
    yv.assign(m, 0.0);
    FB_HIP(hipHostMalloc((void **)&hbuf, sizeof(double) * 2 * (m + 2), hipHostMallocDefault));
    FB_HIP(hipEventCreateWithFlags(&ev_h, hipEventDisableTiming));
}

GmresState::~GmresState()
{
    if (ev_h)
        (void)hipEventDestroy(ev_h);
    if (hbuf)
        (void)hipHostFree(hbuf);
}

void GmresState::record(int p, int prec, double r)
{
    if (it < (int)p_hist.size())
        return;
    p_hist.push_back(p);
    prec_hist.push_back((uint8_t)prec);
    res_hist.push_back(r);
}

void GmresState::begin_cycle()
{
    // v0 = r / beta
    const int64_t n = ctx->n;
    multidot(kw, kw->r, 1, kw->r, kw->h, st);
    k_normalize<<<grid_for(n, 256), 256, 0, st>>>(n, kw->r, kw->h, kw->V);
    FB_HIP(hipGetLastError());
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    k = 0;
}

void GmresState::start()
{
    t0 = std::chrono::steady_clock::now();
    const int64_t n = ctx->n;
    FB_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, st));
    FB_HIP(hipMemcpyAsync(kw->r, b, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    multidot(kw, kw->r, 1, kw->r, kw->h, st);
    FB_HIP(hipMemcpyAsync(hbuf, kw->h, sizeof(double), hipMemcpyDeviceToHost, st));
    FB_HIP(hipStreamSynchronize(st));
    bnorm = std::sqrt(hbuf[0]);
    beta = bnorm;
    if (bnorm == 0.0) {
        converged = 1;
        rel = 0.0;
        true_rel = 0.0;
        done = true;
        return;
    }
    if (s.max_iter <= 0) {
        done = true;
        return;
    }
    begin_cycle();
}

void GmresState::enqueue_step()
{
    const int m = s.restart;
    const int64_t n = ctx->n;
    cur = choose(&s, rho_prev, tol);
    double *vk = kw->V + (int64_t)k * n, *vn = kw->V + (int64_t)(k + 1) * n;
    run_matvec(ctx, cur.p, cur.prec, vk, kw->w, st);
    ++matvecs;
    multidot(kw, kw->V, k + 1, kw->w, kw->h, st);
    multidot(kw, kw->V, k + 1, kw->w, kw->h + (m + 2), st, kw->h);
    k_update_norm<<<kw->nb, DOT_BLOCK, 0, st>>>(n, kw->V, n, k + 1, kw->h, kw->h + (m + 2), kw->w, kw->part,
                                                kw->nb, kw->h + (k + 1), kw->ticket + (m + 1));
    FB_HIP(hipGetLastError());
    k_normalize<<<grid_for(n, 256), 256, 0, st>>>(n, kw->w, kw->h + (k + 1), vn);
    FB_HIP(hipGetLastError());
    // h1[0..k], |w|^2 at k + 1, and h2[0..k] at m + 2: one copy
    FB_HIP(hipMemcpyAsync(hbuf, kw->h, sizeof(double) * (m + 2 + k + 1), hipMemcpyDeviceToHost, st));
    FB_HIP(hipEventRecord(ev_h, st));
    // While the host waits for the column, start the near field of the next
    // mat-vec (its input is v_{k+1}).  Its precision follows the schedule at
    // a residual extrapolated from the last two (a hundredth of the last one when
    // there is no ratio yet); nothing is started where the extrapolated
    // residual already meets the tolerance or the cycle ends.
    if (k + 1 < m && it + 1 < s.max_iter) {
        const double ratio = rho_prev2 > 0.0 ? std::min(1.0, rho_prev / rho_prev2) : 0.01;
        const double rho_next = rho_prev * ratio;
        if (rho_next > tol)
            prefetch_near(ctx, choose(&s, rho_next, tol).prec, vn, st);
    }
}

void GmresState::end_cycle()
{
    const int m = s.restart;
    (void)m;
    const int64_t n = ctx->n;
    for (int i = k - 1; i >= 0; --i) {
        double sum = g[i];
        for (int j = i + 1; j < k; ++j)
            sum -= H[(size_t)i * s.restart + j] * yv[j];
        yv[i] = sum / H[(size_t)i * s.restart + i];
    }
    if (k > 0) {
        FB_HIP(hipMemcpyAsync(kw->y, yv.data(), sizeof(double) * k, hipMemcpyHostToDevice, st));
        k_xupdate<<<grid_for(n, 256), 256, 0, st>>>(n, kw->V, n, k, kw->y, x);
        FB_HIP(hipGetLastError());
    }
    // true residual with the accurate operator
    run_matvec(ctx, s.p_init, FMMBEM_FP64, x, kw->w, st);
    ++matvecs;
    k_sub<<<grid_for(n, 256), 256, 0, st>>>(n, b, kw->w, kw->r);
    FB_HIP(hipGetLastError());
    multidot(kw, kw->r, 1, kw->r, kw->h, st);
    FB_HIP(hipMemcpyAsync(hbuf, kw->h, sizeof(double), hipMemcpyDeviceToHost, st));
    FB_HIP(hipStreamSynchronize(st));
    beta = std::sqrt(hbuf[0]);
    true_rel = beta / bnorm;
    if (rel <= tol || true_rel <= tol) {
        converged = 1;
        done = true;
    } else if (it >= s.max_iter) {
        done = true;
    } else {
        ++restarts;
        rho_prev = true_rel;  // the schedule continues from the true residual
        rho_prev2 = -1.0;
        begin_cycle();
    }
}

void GmresState::complete_step()
{
    const int m = s.restart;
    FB_HIP(hipEventSynchronize(ev_h));
    for (int j = 0; j <= k; ++j)
        H[(size_t)j * m + k] = hbuf[j] + hbuf[m + 2 + j];
    double hn = std::sqrt(hbuf[k + 1]);
    H[(size_t)(k + 1) * m + k] = hn;
    for (int j = 0; j < k; ++j) {
        double a = H[(size_t)j * m + k], c2 = H[(size_t)(j + 1) * m + k];
        H[(size_t)j * m + k] = cs[j] * a + sn[j] * c2;
        H[(size_t)(j + 1) * m + k] = -sn[j] * a + cs[j] * c2;
    }
    double a = H[(size_t)k * m + k], c2 = H[(size_t)(k + 1) * m + k];
    double den = std::sqrt(a * a + c2 * c2);
    cs[k] = den == 0.0 ? 1.0 : a / den;
    sn[k] = den == 0.0 ? 0.0 : c2 / den;
    H[(size_t)k * m + k] = den;
    H[(size_t)(k + 1) * m + k] = 0.0;
    g[k + 1] = -sn[k] * g[k];
    g[k] = cs[k] * g[k];
    rel = std::fabs(g[k + 1]) / bnorm;
    FB_REQUIRE(std::isfinite(rel), FMMBEM_EINTERNAL, "non-finite residual in GMRES");
    record(cur.p, cur.prec, rel);
    rho_prev2 = rho_prev;
    rho_prev = rel;
    ++it;
    ++k;
    if (rel <= tol || hn == 0.0 || k == m || it >= s.max_iter)
        end_cycle();
}

void GmresState::fill_report(fmmbem_report *rep) const
{
    if (!rep)
        return;
    rep->iterations = it;
    rep->restarts = restarts;
    rep->converged = converged;
    rep->rel_res_implicit = rel;
    rep->rel_res_true = true_rel;
    rep->matvecs = matvecs;
    rep->t_solve_s = std::chrono::duration<double>(t1 - t0).count();
    for (int i = 0; i < rep->hist_cap && i < (int)p_hist.size(); ++i) {
        if (rep->p_hist)
            rep->p_hist[i] = p_hist[i];
        if (rep->prec_hist)
            rep->prec_hist[i] = prec_hist[i];
        if (rep->res_hist)
            rep->res_hist[i] = res_hist[i];
    }
}

int run_solve(fmmbem_ctx *ctx, const double *b, double tol, const fmmbem_schedule *s, double *x, fmmbem_report *rep,
              hipStream_t st)
{
    GmresState G(ctx, b, tol, s, x, st);
    G.start();
    while (!G.done) {
        G.enqueue_step();
        G.complete_step();
    }
    G.t1 = std::chrono::steady_clock::now();
    G.fill_report(rep);
    return G.converged ? FMMBEM_OK : FMMBEM_ENOCONV;
}

}  // namespace fmmbem
