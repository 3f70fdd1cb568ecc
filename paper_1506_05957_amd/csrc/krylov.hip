// GMRES(m) with a relaxed expansion order (Sec. 2.4, 2.6).
//
// Arnoldi runs on the device in FP64 with classical Gram-Schmidt applied twice
// (CGS2: as stable as modified Gram-Schmidt, and two passes of block-parallel
// dot products instead of k dependent ones); the (k+2)-entry Hessenberg column
// is copied to the host, where the Givens rotations and the least-squares
// update (a few hundred flops) run in FP64.  The rotated residual
// rho_k = |g_{k+1}| / |b| picks the order and precision of the next mat-vec
// (Eq. 17, 19).  A restart and the final check form the true residual with the
// accurate operator (p_init, FP64); the solve stops only when that residual
// meets the tolerance.  All reductions use a fixed order, so a solve is
// bitwise reproducible.
#include <chrono>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

namespace fmmbem {

namespace {

constexpr int DOT_MAX_BLOCKS = 256;  // row blocks; rows per thread grow beyond that
constexpr int AXPY_UNROLL = 8;

// The reductions of the Arnoldi step carry no atomics or fences: each kernel
// writes one partial per row block, and the next kernel of the step (ordered
// after it on the stream) sums those partials again in every block, in one
// fixed order, so that all blocks see bit-identical coefficients and a solve
// is reproducible.  Row block b holds rows b R + k DOT_BLOCK + t, k < rpt,
// R = rpt DOT_BLOCK.

// Sum over the block of one value per thread (shuffle tree per wave, then
// the waves in order); the result is valid in thread 0.
__device__ double block_total(double s, double *__restrict__ sh)
{
    for (int off = 32; off > 0; off >>= 1)
        s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0)
        sh[threadIdx.x >> 6] = s;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < DOT_NWV; ++k)
            t += sh[k];
    return t;
}

// x - sum_{j < nv} c[j] V_j[i] in the order j = 0, 1, ...; the loads of
// AXPY_UNROLL vectors are issued together so that their latencies overlap.
__device__ inline double sub_combination(double x, const double *__restrict__ V, int64_t ldv, int nv, int64_t i,
                                         const double *__restrict__ c)
{
    int j = 0;
    for (; j + AXPY_UNROLL <= nv; j += AXPY_UNROLL) {
        double v[AXPY_UNROLL];
#pragma unroll
        for (int u = 0; u < AXPY_UNROLL; ++u)
            v[u] = V[(int64_t)(j + u) * ldv + i];
#pragma unroll
        for (int u = 0; u < AXPY_UNROLL; ++u)
            x -= c[j + u] * v[u];
    }
    for (; j < nv; ++j)
        x -= c[j] * V[(int64_t)j * ldv + i];
    return x;
}

// sub_combination of two rows at once (row i1 only where has1; its reads
// then repeat row i0's), their loads issued together: twice the reads in
// flight per thread, each row's arithmetic in the same order as alone
__device__ inline void sub_combination2(double &x0, double &x1, const double *__restrict__ V, int64_t ldv, int nv,
                                        int64_t i0, int64_t i1, bool has1, const double *__restrict__ c)
{
    const int64_t j1 = has1 ? i1 : i0;
    int j = 0;
    for (; j + AXPY_UNROLL <= nv; j += AXPY_UNROLL) {
        double v0[AXPY_UNROLL], v1[AXPY_UNROLL];
#pragma unroll
        for (int u = 0; u < AXPY_UNROLL; ++u) {
            v0[u] = V[(int64_t)(j + u) * ldv + i0];
            v1[u] = V[(int64_t)(j + u) * ldv + j1];
        }
#pragma unroll
        for (int u = 0; u < AXPY_UNROLL; ++u) {
            x0 -= c[j + u] * v0[u];
            x1 -= c[j + u] * v1[u];
        }
    }
    for (; j < nv; ++j) {
        x0 -= c[j] * V[(int64_t)j * ldv + i0];
        x1 -= c[j] * V[(int64_t)j * ldv + j1];
    }
}

// Classical Gram-Schmidt dots: block (b, g) takes row block b and the vectors
// j = g CGS_JG .. + CGS_JG - 1 and writes part[j][b] = V_j . w over its rows.
constexpr int CGS_JG = 8;
__global__ __launch_bounds__(DOT_BLOCK) void k_cgs_dots(int64_t n, int rpt, const double *__restrict__ V, int64_t ldv,
                                                         int nv, const double *__restrict__ w,
                                                         double *__restrict__ part, int nb)
{
    __shared__ double sh[CGS_JG][DOT_NWV];
    const int b = blockIdx.x, j0 = blockIdx.y * CGS_JG;
    const int nj = min(CGS_JG, nv - j0);
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double s[CGS_JG];
#pragma unroll
    for (int jj = 0; jj < CGS_JG; ++jj)
        s[jj] = 0.0;
    const int64_t base = (int64_t)b * rpt * DOT_BLOCK + threadIdx.x;
    for (int k = 0; k < rpt; ++k) {
        const int64_t i = base + (int64_t)k * DOT_BLOCK;
        if (i >= n)
            break;
        const double x = w[i];
        double v[CGS_JG];
#pragma unroll
        for (int jj = 0; jj < CGS_JG; ++jj)
            v[jj] = jj < nj ? V[(int64_t)(j0 + jj) * ldv + i] : 0.0;
#pragma unroll
        for (int jj = 0; jj < CGS_JG; ++jj)
            s[jj] += v[jj] * x;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int jj = 0; jj < CGS_JG; ++jj)
            s[jj] += __shfl_down(s[jj], off, 64);
    if (lane == 0)
#pragma unroll
        for (int jj = 0; jj < CGS_JG; ++jj)
            sh[jj][wv] = s[jj];
    __syncthreads();
    if ((int)threadIdx.x < nj) {
        double t = 0.0;
        for (int k = 0; k < DOT_NWV; ++k)
            t += sh[threadIdx.x][k];
        part[(int64_t)(j0 + threadIdx.x) * nb + b] = t;
    }
}

// w -= sum_{j<nv} h1[j] V_j, h1 summed from the first pass's partials (every
// block sums them in the same order).  Dynamic LDS: nv doubles.
__global__ __launch_bounds__(DOT_BLOCK) void k_sub_first(int64_t n, int rpt, const double *__restrict__ V, int64_t ldv,
                                                          int nv, const double *__restrict__ part1, int nb,
                                                          double *__restrict__ w)
{
    extern __shared__ double hs[];  // [nv]
    block_sums(part1, nb, nv, hs);
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * rpt * DOT_BLOCK + threadIdx.x;
    for (int k = 0; k < rpt; ++k) {
        const int64_t i = base + (int64_t)k * DOT_BLOCK;
        if (i >= n)
            break;
        w[i] = sub_combination(w[i], V, ldv, nv, i, hs);
    }
}

// The first update and the second pass of CGS2 in one: w -= sum_{j<nv} h1[j]
// V_j (h1 summed from the first pass's partials, as in k_sub_first), then
// part2[j][b] = V_j . w over row block b, j < nv <= 8 NVC.  A row's vectors
// are read for the update and right after for the dots (the second read
// comes from L2); a thread keeps the partial dots of every vector over its
// rows, and the block adds them up (shuffle tree per wave, then the waves in
// order).  Dynamic LDS: nv doubles.
template <int NVC>
__global__ __launch_bounds__(DOT_BLOCK) void k_sub_dots(int64_t n, int rpt, const double *__restrict__ V, int64_t ldv,
                                                         int nv, const double *__restrict__ part1, int nb,
                                                         double *__restrict__ w, double *__restrict__ part2)
{
    extern __shared__ double hs[];  // [nv]
    __shared__ double sh[CGS_JG][DOT_NWV];
    block_sums(part1, nb, nv, hs);
    __syncthreads();
    double s[CGS_JG * NVC];
#pragma unroll
    for (int q = 0; q < CGS_JG * NVC; ++q)
        s[q] = 0.0;
    const int64_t base = (int64_t)blockIdx.x * rpt * DOT_BLOCK + threadIdx.x;
    for (int k = 0; k < rpt; k += 2) {  // rows k and k + 1 together
        const int64_t i0 = base + (int64_t)k * DOT_BLOCK, i1 = i0 + DOT_BLOCK;
        if (i0 >= n)
            break;
        const bool has1 = k + 1 < rpt && i1 < n;
        double x0 = w[i0], x1 = has1 ? w[i1] : 0.0;
        sub_combination2(x0, x1, V, ldv, nv, i0, i1, has1, hs);
        w[i0] = x0;
        if (has1)
            w[i1] = x1;
        else
            x1 = 0.0;
        const int64_t j1 = has1 ? i1 : i0;
#pragma unroll
        for (int c = 0; c < NVC; ++c) {
            double v0[CGS_JG], v1[CGS_JG];
#pragma unroll
            for (int u = 0; u < CGS_JG; ++u) {  // clamped, unguarded reads; the extra ones zeroed
                v0[u] = V[(int64_t)min(CGS_JG * c + u, nv - 1) * ldv + i0];
                v1[u] = V[(int64_t)min(CGS_JG * c + u, nv - 1) * ldv + j1];
            }
#pragma unroll
            for (int u = 0; u < CGS_JG; ++u) {
                s[CGS_JG * c + u] += (CGS_JG * c + u < nv ? v0[u] : 0.0) * x0;
                s[CGS_JG * c + u] += (CGS_JG * c + u < nv ? v1[u] : 0.0) * x1;
            }
        }
    }
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int c = 0; c < NVC; ++c) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
#pragma unroll
            for (int u = 0; u < CGS_JG; ++u)
                s[CGS_JG * c + u] += __shfl_down(s[CGS_JG * c + u], off, 64);
        if (lane == 0)
#pragma unroll
            for (int u = 0; u < CGS_JG; ++u)
                sh[u][wv] = s[CGS_JG * c + u];
        __syncthreads();
        const int j = CGS_JG * c + (int)threadIdx.x;
        if ((int)threadIdx.x < CGS_JG && j < nv) {
            double t = 0.0;
            for (int q = 0; q < DOT_NWV; ++q)
                t += sh[threadIdx.x][q];
            part2[(int64_t)j * nb + blockIdx.x] = t;
        }
        __syncthreads();
    }
}

// h1, h2 summed from the two passes' partials; w -= sum_{j<nv} h2[j] V_j (h1
// was taken off by k_sub_first before the second pass), and the partial of
// |w|^2 of this row block into partn[b].  Block 0 also writes h1 to
// hout[0..nv) and h2 to hout[off2..off2 + nv) for the host.  Dynamic LDS:
// 2 nv doubles.
__global__ __launch_bounds__(DOT_BLOCK) void k_update_norm(int64_t n, int rpt, const double *__restrict__ V,
                                                            int64_t ldv, int nv, const double *__restrict__ part1,
                                                            const double *__restrict__ part2, int nb,
                                                            double *__restrict__ w, double *__restrict__ partn,
                                                            double *__restrict__ hout, int off2)
{
    extern __shared__ double hs[];  // [2][nv]
    __shared__ double sh[DOT_NWV];
    const int b = blockIdx.x;
    block_sums(part1, nb, nv, hs);
    block_sums(part2, nb, nv, hs + nv);
    __syncthreads();
    if (b == 0)
        for (int j = threadIdx.x; j < nv; j += DOT_BLOCK) {
            hout[j] = hs[j];
            hout[off2 + j] = hs[nv + j];
        }
    double s = 0.0;
    const int64_t base = (int64_t)b * rpt * DOT_BLOCK + threadIdx.x;
    for (int k = 0; k < rpt; k += 2) {  // rows k and k + 1 together
        const int64_t i0 = base + (int64_t)k * DOT_BLOCK, i1 = i0 + DOT_BLOCK;
        if (i0 >= n)
            break;
        const bool has1 = k + 1 < rpt && i1 < n;
        double x0 = w[i0], x1 = has1 ? w[i1] : 0.0;
        sub_combination2(x0, x1, V, ldv, nv, i0, i1, has1, hs + nv);
        w[i0] = x0;
        s += x0 * x0;
        if (has1) {
            w[i1] = x1;
            s += x1 * x1;
        }
    }
    const double t = block_total(s, sh);
    if (threadIdx.x == 0)
        partn[b] = t;
}

// v = w / sqrt(nrm2) with nrm2 summed from the partials partn[0..nb); block 0
// also writes nrm2 to *nrm2_out when given.
__global__ __launch_bounds__(DOT_BLOCK) void k_normalize(int64_t n, int rpt, const double *__restrict__ w,
                                                          const double *__restrict__ partn, int nb,
                                                          double *__restrict__ v, double *__restrict__ nrm2_out)
{
    __shared__ double tot;
    block_sums(partn, nb, 1, &tot);
    __syncthreads();
    const double nrm2 = tot;
    if (blockIdx.x == 0 && threadIdx.x == 0 && nrm2_out)
        *nrm2_out = nrm2;
    const double inv = 1.0 / sqrt(nrm2);
    const int64_t base = (int64_t)blockIdx.x * rpt * DOT_BLOCK + threadIdx.x;
    for (int k = 0; k < rpt; ++k) {
        const int64_t i = base + (int64_t)k * DOT_BLOCK;
        if (i >= n)
            break;
        v[i] = w[i] * inv;
    }
}

// out[j] = sum_b part[j nb + b], j < nv (one block)
__global__ __launch_bounds__(DOT_BLOCK) void k_sum_parts(const double *__restrict__ part, int nb, int nv,
                                                          double *__restrict__ out)
{
    extern __shared__ double hs[];
    block_sums(part, nb, nv, hs);
    __syncthreads();
    for (int j = threadIdx.x; j < nv; j += DOT_BLOCK)
        out[j] = hs[j];
}

// x += sum_{j<nv} y[j] V_j
__global__ void k_xupdate(int64_t n, const double *__restrict__ V, int64_t ldv, int nv, const double *__restrict__ y,
                          double *__restrict__ x)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    double s = x[i];
    int j = 0;
    for (; j + AXPY_UNROLL <= nv; j += AXPY_UNROLL) {
        double v[AXPY_UNROLL];
#pragma unroll
        for (int u = 0; u < AXPY_UNROLL; ++u)
            v[u] = V[(int64_t)(j + u) * ldv + i];
#pragma unroll
        for (int u = 0; u < AXPY_UNROLL; ++u)
            s += y[j + u] * v[u];
    }
    for (; j < nv; ++j)
        s += y[j] * V[(int64_t)j * ldv + i];
    x[i] = s;
}

__global__ void k_sub(int64_t n, const double *__restrict__ b, const double *__restrict__ a, double *__restrict__ r)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        r[i] = b[i] - a[i];
}

__global__ void k_zero(int64_t n, double *__restrict__ x)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        x[i] = 0.0;
}

void release_work(KrylovWork *kw)
{
    if (kw->owned) {
        kw->arena.release();
        pinned_put(kw->hcol, kw->hcol_src);
        if (kw->ev_h)
            (void)hipEventDestroy(kw->ev_h);
    }
    delete kw;
}

KrylovWork *get_work(fmmbem_ctx *ctx, int m)
{
    KrylovWork *kw = ctx->kw;
    if (kw && kw->m >= m)
        return kw;
    if (kw) {
        FB_HIP(hipDeviceSynchronize());  // nothing may still use the old workspace
        release_work(kw);
        ctx->kw = nullptr;
    }
    kw = new KrylovWork();
    kw->arena.al = ctx->arena.al;
    try {
        kw->m = m;
        kw->n = ctx->n;
        krylov_blocks(ctx->n, &kw->nb, &kw->rpt);
        kw->V = kw->arena.alloc<double>((size_t)(m + 1) * ctx->n);
        kw->w = kw->arena.alloc<double>(ctx->n);
        kw->r = kw->arena.alloc<double>(ctx->n);
        kw->part1 = kw->arena.alloc<double>((size_t)(m + 1) * kw->nb);
        kw->part2 = kw->arena.alloc<double>((size_t)(m + 1) * kw->nb);
        kw->partn = kw->arena.alloc<double>(kw->nb);
        kw->y = kw->arena.alloc<double>(m + 1);
        kw->hcol = pinned_get(sizeof(double) * hcol_len(m), &kw->hcol_src);
        std::fill(kw->hcol, kw->hcol + hcol_len(m), 0.0);
        FB_HIP(hipHostGetDevicePointer((void **)&kw->hcol_dev, kw->hcol, 0));
        FB_HIP(hipEventCreateWithFlags(&kw->ev_h, hipEventDisableTiming));
    } catch (...) {
        release_work(kw);
        throw;
    }
    ctx->kw = kw;
    return kw;
}

// part[j][b] = V_j . w over row block b, j < nv
void cgs_dots(KrylovWork *kw, const double *V, int nv, const double *w, double *part, hipStream_t st)
{
    dim3 grid(kw->nb, (nv + CGS_JG - 1) / CGS_JG);
    k_cgs_dots<<<grid, DOT_BLOCK, 0, st>>>(kw->n, kw->rpt, V, kw->n, nv, w, part, kw->nb);
    FB_HIP(hipGetLastError());
}

// w -= V h1 and part2 = V^T w (h1 from part1), for the nv vectors of V
void sub_dots(KrylovWork *kw, int nv, hipStream_t st)
{
    const size_t shm = sizeof(double) * nv;
    const int64_t n = kw->n;
    switch ((nv + CGS_JG - 1) / CGS_JG) {
    case 1: k_sub_dots<1><<<kw->nb, DOT_BLOCK, shm, st>>>(n, kw->rpt, kw->V, n, nv, kw->part1, kw->nb, kw->w, kw->part2); break;
    case 2: k_sub_dots<2><<<kw->nb, DOT_BLOCK, shm, st>>>(n, kw->rpt, kw->V, n, nv, kw->part1, kw->nb, kw->w, kw->part2); break;
    case 3: k_sub_dots<3><<<kw->nb, DOT_BLOCK, shm, st>>>(n, kw->rpt, kw->V, n, nv, kw->part1, kw->nb, kw->w, kw->part2); break;
    case 4: k_sub_dots<4><<<kw->nb, DOT_BLOCK, shm, st>>>(n, kw->rpt, kw->V, n, nv, kw->part1, kw->nb, kw->w, kw->part2); break;
    case 5: k_sub_dots<5><<<kw->nb, DOT_BLOCK, shm, st>>>(n, kw->rpt, kw->V, n, nv, kw->part1, kw->nb, kw->w, kw->part2); break;
    case 6: k_sub_dots<6><<<kw->nb, DOT_BLOCK, shm, st>>>(n, kw->rpt, kw->V, n, nv, kw->part1, kw->nb, kw->w, kw->part2); break;
    case 7: k_sub_dots<7><<<kw->nb, DOT_BLOCK, shm, st>>>(n, kw->rpt, kw->V, n, nv, kw->part1, kw->nb, kw->w, kw->part2); break;
    default:  // more vectors than the fused kernel keeps: the update, then the dots
        k_sub_first<<<kw->nb, DOT_BLOCK, shm, st>>>(n, kw->rpt, kw->V, n, nv, kw->part1, kw->nb, kw->w);
        FB_HIP(hipGetLastError());
        cgs_dots(kw, kw->V, nv, kw->w, kw->part2, st);
        return;
    }
    FB_HIP(hipGetLastError());
}

// |r|^2 into entry slot of the host column (read after the stream is synchronised)
void norm2(KrylovWork *kw, const double *r, hipStream_t st, int slot = 0)
{
    cgs_dots(kw, r, 1, r, kw->part1, st);
    k_sum_parts<<<1, DOT_BLOCK, sizeof(double), st>>>(kw->part1, kw->nb, 1, kw->hcol_dev + slot);
    FB_HIP(hipGetLastError());
}

Sched choose(const fmmbem_schedule *s, double rho, double eta, bool fp64_only = false, int p_floor = 0)
{
    double rm = std::min(rho, 1.0);
    double eps = std::min(eta / rm, 1.0);
    int p = s->p_init;
    if (s->rule == FMMBEM_RELAX_SHIFT) {
        p = s->p_init + (int)std::ceil(std::log2(rm));
    } else if (s->rule == FMMBEM_RELAX_BF) {
        p = (int)std::ceil(-std::log2(eps));
    }
    p = std::max(std::max(s->p_min, p_floor), std::min(s->p_init, p));
    int prec = FMMBEM_FP64;
    if (s->mixed && !fp64_only && s->rule != FMMBEM_FIXED && eps >= s->fp32_eps && p <= P_MAX_FP32)
        prec = FMMBEM_FP32;
    return {p, prec};
}

}  // namespace

void krylov_blocks(int64_t n, int *nb, int *rpt)
{
    *rpt = (int)std::max<int64_t>(1, (n + (int64_t)DOT_BLOCK * DOT_MAX_BLOCKS - 1) /
                                         ((int64_t)DOT_BLOCK * DOT_MAX_BLOCKS));
    *nb = (int)((n + (int64_t)DOT_BLOCK * *rpt - 1) / ((int64_t)DOT_BLOCK * *rpt));
}

void fill_zero(double *x, int64_t n, hipStream_t st)
{
    if (n <= 0)
        return;
    k_zero<<<grid_for(n, 256), 256, 0, st>>>(n, x);
    FB_HIP(hipGetLastError());
}

void reserve_krylov(fmmbem_ctx *ctx, int m)
{
    (void)get_work(ctx, m);
}

void free_krylov(fmmbem_ctx *ctx)
{
    if (ctx->kw) {
        release_work(ctx->kw);
        ctx->kw = nullptr;
    }
}

GmresState::GmresState(fmmbem_ctx *c, const double *b_, double tol_, const fmmbem_schedule *s_, double *x_,
                       hipStream_t st_, fmmbem_report *rep_, KrylovWork *kw_given, double *hostw)
    : ctx(c), b(b_), x(x_), s(*s_), tol(tol_), st(st_), rep(rep_)
{
    const int m = s.restart;
    kw = kw_given ? kw_given : get_work(ctx, m);
    FB_REQUIRE(kw->m >= m && kw->n == ctx->n, FMMBEM_EINTERNAL, "Krylov workspace too small");
    if (!hostw) {
        host_own.assign(host_doubles(m), 0.0);
        hostw = host_own.data();
    } else {
        std::fill(hostw, hostw + host_doubles(m), 0.0);
    }
    cs = hostw;
    sn = cs + m;
    g = sn + m;
    yv = g + (m + 1);
    H = yv + (m + 1);  // [(m + 1) m]
    hbuf = kw->hcol;
    ev_h = kw->ev_h;
    if (ctx->timing.mask) {
        timing_resolve(ctx->timing);
        std::copy(ctx->timing.t_ms, ctx->timing.t_ms + FMMBEM_N_STAGES, t_stage0);
    }
}

GmresState::~GmresState()
{
    // a solve left early (an error, or b = 0) may still have a prefetched
    // mat-vec in flight: let it end before the context is used again
    if (ctx->spec_x || ctx->side_pending) {
        if (ctx->side_pending)
            (void)hipStreamWaitEvent(st, ctx->ev_join, 0);
        (void)hipStreamSynchronize(st);
        ctx->spec_x = nullptr;
        ctx->spec_prec = ctx->spec_up_p = -1;
        ctx->spec_near = false;
        ctx->spec_swap = false;
        ctx->side_pending = false;
    }
}

// wait for the prefetched charges, upward pass and near field, and drop them
void GmresState::drain_prefetch()
{
    if (ctx->side_pending)
        FB_HIP(hipStreamWaitEvent(st, ctx->ev_join, 0));
    FB_HIP(hipStreamSynchronize(st));
    ctx->spec_x = nullptr;
    ctx->spec_prec = ctx->spec_up_p = -1;
    ctx->spec_near = false;
    ctx->spec_swap = false;
    ctx->side_pending = false;
}

void GmresState::record(int p, int prec, double r)
{
    if (!rep || it >= rep->hist_cap)
        return;
    if (rep->p_hist)
        rep->p_hist[it] = p;
    if (rep->prec_hist)
        rep->prec_hist[it] = (uint8_t)prec;
    if (rep->res_hist)
        rep->res_hist[it] = r;
}

void GmresState::begin_cycle()
{
    // v0 = r / beta
    const int64_t n = ctx->n;
    hipEvent_t ev;
    stage_begin(ctx, 10, st, &ev);
    cgs_dots(kw, kw->r, 1, kw->r, kw->part1, st);
    k_normalize<<<kw->nb, DOT_BLOCK, 0, st>>>(n, kw->rpt, kw->r, kw->part1, kw->nb, kw->V, nullptr);
    FB_HIP(hipGetLastError());
    stage_end(ctx, 10, st, ev);
    std::fill(g, g + s.restart + 1, 0.0);
    g[0] = beta;
    k = 0;
}

void GmresState::start()
{
    t0 = std::chrono::steady_clock::now();
    const int64_t n = ctx->n;
    fill_zero(x, n, st);
    FB_HIP(hipMemcpyAsync(kw->r, b, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    // |b| is read with the first Hessenberg column, so the first mat-vec
    // starts without a round trip to the host (b = 0 is caught there: v_0 is
    // then not finite, x stays zero)
    norm2(kw, kw->r, st, 2 * (s.restart + 2));
    bnorm_known = false;
    begin_cycle();
}

void GmresState::enqueue_step()
{
    const int m = s.restart;
    const int64_t n = ctx->n;
    cur = choose(&s, rho_prev, tol, fp64_only, p_floor);
    double *vk = kw->V + (int64_t)k * n, *vn = kw->V + (int64_t)(k + 1) * n;
    run_matvec(ctx, cur.p, cur.prec, vk, kw->w, st);
    ++matvecs;
    hipEvent_t ev;
    stage_begin(ctx, 10, st, &ev);
    // CGS2: h1 = V^T w, w -= V h1, h2 = V^T w, w -= V h2 (below, with |w|^2)
    cgs_dots(kw, kw->V, k + 1, kw->w, kw->part1, st);
    sub_dots(kw, k + 1, st);
    // h1[0..k], |w|^2 at k + 1 and h2[0..k] at m + 2 go straight to the host column
    k_update_norm<<<kw->nb, DOT_BLOCK, 2 * sizeof(double) * (k + 1), st>>>(
        n, kw->rpt, kw->V, n, k + 1, kw->part1, kw->part2, kw->nb, kw->w, kw->partn, kw->hcol_dev, m + 2);
    FB_HIP(hipGetLastError());
    // Ahead of the next mat-vec (its input is v_{k+1}): its charges before the
    // host's event, then its upward pass and its near field, run while the
    // host waits for the column.  The precision follows the schedule at a residual extrapolated
    // from the last two (a hundredth of the last one when there is no ratio
    // yet); nothing is started where the extrapolated residual already meets
    // the tolerance or the cycle ends, nor before |b| is known (b = 0 would
    // leave it running).  The upward pass takes at most this
    // mat-vec's order (the GMRES residual never grows within a cycle and the
    // order never falls as the residual grows, so the next order is at most
    // this one) and at most two above the order at the extrapolated residual;
    // a mat-vec of a higher order than the prefetched pass runs its own.
    int pre_prec = -1, p_up = 0;
    bool pre_swap = false;
    if (bnorm_known && k + 1 < m && it + 1 < s.max_iter) {
        const double ratio = rho_prev2 > 0.0 ? std::min(1.0, rho_prev / rho_prev2) : 0.01;
        const double rho_next = rho_prev * ratio;
        if (rho_next > tol) {
            const Sched nx = choose(&s, rho_next, tol, fp64_only, p_floor);
            pre_prec = nx.prec;
            p_up = std::min(cur.p, nx.p + 2);
            if (pre_prec == FMMBEM_FP32)
                p_up = std::min(p_up, P_MAX_FP32);
            pre_swap = near_on_main(ctx, nx.p, pre_prec);
        }
    }
    if (pre_prec < 0) {
        k_normalize<<<kw->nb, DOT_BLOCK, 0, st>>>(n, kw->rpt, kw->w, kw->partn, kw->nb, vn, kw->hcol_dev + (k + 1));
        FB_HIP(hipGetLastError());
    }
    stage_end(ctx, 10, st, ev);
    if (pre_prec >= 0) {
        // v_{k+1} = w / |w| (and |w|^2 into the host column) is written
        // by these charges
        prefetch_charges(ctx, pre_prec, vn, st, NormIn{kw->w, kw->partn, kw->nb, kw->hcol_dev + (k + 1)},
                         pre_swap);
    }
    FB_HIP(hipEventRecord(ev_h, st));
    if (pre_prec >= 0 && pre_swap) {
        // the near field right behind the charges on this stream, the
        // upward pass on the side stream
        prefetch_near(ctx, st);
        prefetch_up(ctx, pre_prec, p_up, st);
    } else if (pre_prec >= 0) {
        prefetch_up(ctx, pre_prec, p_up, st);
        // the near field after the launches the GPU needs first: its fork
        // waits on the pending charges (several launches' worth of host
        // time, which the host would spend waiting anyway), and the product
        // is done sooner than when forked after the host's wait
        prefetch_near(ctx, st);
    }
}

void GmresState::end_cycle()
{
    const int m = s.restart;
    const int64_t n = ctx->n;
    for (int i = k - 1; i >= 0; --i) {
        double sum = g[i];
        for (int j = i + 1; j < k; ++j)
            sum -= H[(size_t)i * m + j] * yv[j];
        yv[i] = sum / H[(size_t)i * m + i];
    }
    hipEvent_t ev;
    stage_begin(ctx, 10, st, &ev);
    if (k > 0) {
        // y through the pinned column buffer: an asynchronous copy from
        // pageable memory would stage it and block the host
        double *yh = hbuf + 2 * (m + 2) + 1;
        std::copy(yv, yv + k, yh);
        FB_HIP(hipMemcpyAsync(kw->y, yh, sizeof(double) * k, hipMemcpyHostToDevice, st));
        k_xupdate<<<grid_for(n, 256), 256, 0, st>>>(n, kw->V, n, k, kw->y, x);
        FB_HIP(hipGetLastError());
    }
    stage_end(ctx, 10, st, ev);
    // true residual with the accurate operator
    run_matvec(ctx, s.p_init, FMMBEM_FP64, x, kw->w, st);
    ++matvecs;
    stage_begin(ctx, 10, st, &ev);
    k_sub<<<grid_for(n, 256), 256, 0, st>>>(n, b, kw->w, kw->r);
    FB_HIP(hipGetLastError());
    norm2(kw, kw->r, st);
    stage_end(ctx, 10, st, ev);
    FB_HIP(hipStreamSynchronize(st));
    beta = std::sqrt(hbuf[0]);
    true_rel = beta / bnorm;
    FB_REQUIRE(std::isfinite(true_rel), FMMBEM_EINTERNAL, "non-finite true residual (FP64, p_init)");
    // converged only by the true residual: with relaxed products the implicit
    // residual can reach tol while the true one has not; then the solve
    // restarts from the true residual
    if (true_rel <= tol) {
        converged = 1;
        done = true;
    } else if (it >= s.max_iter) {
        done = true;
    } else {
        ++restarts;
        const double gap = true_rel / std::max(rel, tol);
        if (gap > 2.0) {
            // a stall: the true residual is well above what the cycle's
            // implicit residual (or tol) promised, so the relaxed products
            // were less accurate than the residual needs.  The gap follows
            // the mat-vec error, which Eq. 19 takes to fall as 2^-p: every
            // later order is at least the floor raised by the orders that
            // close the gap, plus one
            ++stalls;
            const int dp = (int)std::ceil(std::log2(gap)) + 1;
            p_floor = std::min(s.p_init, std::max(p_floor, s.p_min) + dp);
        }
        rho_prev = true_rel;  // the schedule continues from the true residual
        rho_prev2 = -1.0;
        begin_cycle();
    }
}

void GmresState::complete_step()
{
    const int m = s.restart;
    FB_HIP(hipEventSynchronize(ev_h));
    if (!bnorm_known) {
        bnorm_known = true;
        bnorm = beta = std::sqrt(hbuf[2 * (m + 2)]);
        FB_REQUIRE(std::isfinite(bnorm), FMMBEM_EINVAL, "right-hand side is not finite");
        g[0] = beta;
        if (bnorm == 0.0) {
            converged = 1;
            rel = true_rel = 0.0;
            done = true;
            drain_prefetch();
            return;
        }
    }
    for (int j = 0; j <= k; ++j)
        H[(size_t)j * m + k] = hbuf[j] + hbuf[m + 2 + j];
    double hn = std::sqrt(hbuf[k + 1]);
    H[(size_t)(k + 1) * m + k] = hn;
    bool finite = std::isfinite(hn);
    for (int j = 0; j <= k; ++j)
        finite = finite && std::isfinite(H[(size_t)j * m + k]);
    if (!finite) {
        // a non-finite column (an FP32 range overflow in the mat-vec): it is
        // discarded, the cycle ends with the k columns before it (x, the true
        // residual) and the solve restarts with every later mat-vec in FP64;
        // the same in FP64 cannot be recovered
        FB_REQUIRE(cur.prec == FMMBEM_FP32 && !fp64_only, FMMBEM_EINTERNAL,
                   "non-finite Hessenberg column in an FP64 step");
        record(cur.p, cur.prec, std::nan(""));
        ++it;
        ++fallbacks;
        fp64_only = true;
        end_cycle();
        return;
    }
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

void GmresState::fill_report(fmmbem_report *r) const
{
    if (!r)
        return;
    r->iterations = it;
    r->restarts = restarts;
    r->converged = converged;
    r->fallbacks = fallbacks;
    r->stalls = stalls;
    r->p_floor = p_floor;
    r->rel_res_implicit = rel;
    r->rel_res_true = true_rel;
    r->matvecs = matvecs;
    r->t_solve_s = std::chrono::duration<double>(t1 - t0).count();
    // per-stage device time of this solve (timed stages only)
    double t[4] = {0, 0, 0, 0};
    bool timed[4] = {false, false, false, false};
    const Timing &T = ctx->timing;
    for (int i = 0; i < FMMBEM_N_STAGES; ++i) {
        const int grp = i == 10 ? 3 : (i % 5 == 0 ? 0 : i % 5 == 1 ? 1 : 2);
        if ((T.mask >> i) & 1u) {
            timed[grp] = true;
            t[grp] += (T.t_ms[i] - t_stage0[i]) * 1e-3;
        }
    }
    r->t_p2p_s = timed[0] ? t[0] : -1.0;
    r->t_m2l_s = timed[1] ? t[1] : -1.0;
    r->t_other_fmm_s = timed[2] ? t[2] : -1.0;
    r->t_krylov_s = timed[3] ? t[3] : -1.0;
}

namespace {

// Workspace of the allocation-free solve: the Krylov basis, w, r, the
// per-block partial sums and y of GMRES(m), carved from one static device
// array of FMMBEM_STATIC_SCRATCH_BYTES.  Each device holds its own copy at
// its own address, which hipGetSymbolAddress gives once per device; host
// code uses only that address.  Every such solve on a device shares its copy
// (calls that overlap on one device race; nothing in it needs clearing: each
// buffer is written before it is read).
static __device__ __align__(256) double scratch[FMMBEM_STATIC_SCRATCH_BYTES / sizeof(double)];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch[MAX_DEVICES] = {};

double *scratch_ptr(int device)
{
    FB_REQUIRE(device >= 0 && device < MAX_DEVICES, FMMBEM_EDEVICE, "device index beyond the library's table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[device]) {
        void *ptr = nullptr;
        FB_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_scratch[device] = static_cast<double *>(ptr);
    }
    return g_scratch[device];
}

// host arrays of the Givens update for restarts up to FMMBEM_STATIC_MAX_RESTART
thread_local double g_host_static[4 * FMMBEM_STATIC_MAX_RESTART + 2 +
                                  (FMMBEM_STATIC_MAX_RESTART + 1) * FMMBEM_STATIC_MAX_RESTART];

}  // namespace

int run_solve_static(fmmbem_ctx *ctx, const double *b, double tol, const fmmbem_schedule *s, double *x,
                     fmmbem_report *rep, hipStream_t st)
{
    int dev = -1;
    FB_HIP(hipGetDevice(&dev));
    FB_REQUIRE(dev == ctx->device, FMMBEM_EINVAL, "the context's device is not the current device");
    const int m = s->restart;
    const int64_t n = ctx->n;
    KrylovWork kw;
    kw.owned = false;
    kw.m = m;
    kw.n = n;
    krylov_blocks(n, &kw.nb, &kw.rpt);
    // sub-buffers at 256-byte boundaries (32 doubles)
    auto up = [](int64_t v) { return (v + 31) / 32 * 32; };
    const int64_t sizes[7] = {(int64_t)(m + 1) * n, n, n, (int64_t)(m + 1) * kw.nb, (int64_t)(m + 1) * kw.nb,
                              kw.nb, m + 1};
    int64_t need = 0;
    for (int64_t v : sizes)
        need += up(v);
    const int64_t cap = (int64_t)(FMMBEM_STATIC_SCRATCH_BYTES / sizeof(double));
    FB_REQUIRE(need <= cap, FMMBEM_EINVAL,
               "GMRES(" + std::to_string(m) + ") on " + std::to_string(n) + " unknowns needs " +
                   std::to_string(need * 8) + " bytes of workspace; the static workspace holds " +
                   std::to_string(cap * 8));
    double *base = scratch_ptr(dev);
    double *bufs[7];
    int64_t off = 0;
    for (int i = 0; i < 7; ++i) {
        bufs[i] = base + off;
        off += up(sizes[i]);
    }
    kw.V = bufs[0];
    kw.w = bufs[1];
    kw.r = bufs[2];
    kw.part1 = bufs[3];
    kw.part2 = bufs[4];
    kw.partn = bufs[5];
    kw.y = bufs[6];
    kw.hcol = ctx->hcol_s;
    kw.hcol_dev = ctx->hcol_s_dev;
    kw.ev_h = ctx->ev_h_s;
    std::fill(kw.hcol, kw.hcol + hcol_len(m), 0.0);
    GmresState G(ctx, b, tol, s, x, st, rep, &kw, g_host_static);
    G.start();
    while (!G.done) {
        G.enqueue_step();
        G.complete_step();
    }
    G.t1 = std::chrono::steady_clock::now();
    G.fill_report(rep);
    return G.converged ? FMMBEM_OK : FMMBEM_ENOCONV;
}

int run_solve(fmmbem_ctx *ctx, const double *b, double tol, const fmmbem_schedule *s, double *x, fmmbem_report *rep,
              hipStream_t st)
{
    GmresState G(ctx, b, tol, s, x, st, rep);
    G.start();
    while (!G.done) {
        G.enqueue_step();
        G.complete_step();
    }
    G.t1 = std::chrono::steady_clock::now();
    if (ctx->timing.mask)
        timing_resolve(ctx->timing);
    G.fill_report(rep);
    return G.converged ? FMMBEM_OK : FMMBEM_ENOCONV;
}

}  // namespace fmmbem
