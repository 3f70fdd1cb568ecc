// The regular near field stored as a block-sparse matrix (Sec. 2.3, 2.5): the
// 4-point rule between every target panel and the panels of the leaves in its
// P2P list, assembled once and multiplied by every mat-vec, as the paper holds
// its near field.  The near-singular and self corrections (25-point rule minus
// 4-point rule, and the analytic self integral on a block that leaves the
// target's own panel at zero) are then added into the entries of their pairs,
// so that a stored entry is the accurate integral and the mat-vec no longer
// visits them; the few pairs without a stored block keep a separate list.
#include <algorithm>
#include <vector>

#include "common.h"

namespace fmmbem {

namespace {

constexpr int NEAR_WAVES = 8;

// Layout of one stored block (n targets, ns sources padded to ns4 groups of
// four): value (target i, source j, component ab) sits at
//   off + ((j / 4) PER + ab) n 4 + 4 i + j % 4,
// so that the four sources of a group are adjacent for every target and a
// lane reads them with one 16-byte (FP32) or 32-byte (FP64) load; padding
// sources hold zeros.
__host__ __device__ inline int64_t near_index(int64_t off, int n, int per, int j, int ab, int i)
{
    return off + (((int64_t)(j >> 2) * per + ab) * n + i) * 4 + (j & 3);
}

// Entries of one stored block per HIP block, in FP64: entry (j, i) is
// sum_k w_jk G(t_i - y_jk) over the 4 Gauss points of source panel j, Laplace
// G = 1/r, Stokes G_ab = delta_ab / r + d_a d_b / r^3 (d = t - y), double layer
// G = n_j . d / r^3, without the kernel prefactor (applied when the mat-vec
// is combined).
template <int KIND>
__global__ void k_near_build(const int4 *__restrict__ units, const int32_t *__restrict__ blk_unit,
                             const NearBlock *__restrict__ blk, int64_t nt, const double *__restrict__ tc,
                             const double *__restrict__ sp, const double *__restrict__ nrm,
                             double *__restrict__ v64, float *__restrict__ v32)
{
    constexpr bool STOKES = KIND == FMMBEM_STOKES_SL;
    constexpr int PER = STOKES ? 9 : 1;
    const int64_t b = blockIdx.x;
    const NearBlock B = blk[b];
    const int4 u = units[blk_unit[b]];
    const int tb = u.x, n = u.y - u.x;
    const int64_t ns = 4 * nt;
    const int ns4 = (B.ns + 3) / 4;
    const int64_t cnt = (int64_t)n * ns4 * 4 * PER;  // in storage order
    for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) {
        const int jl = (int)(e & 3);
        const int i = (int)((e >> 2) % n);
        const int64_t r = (e >> 2) / n;
        const int ab = (int)(r % PER), j = 4 * (int)(r / PER) + jl;
        const int ti = tb + i, sj = B.j0 + j;
        double v = 0.0;
        if (j < B.ns && ti != sj) {
            const double t[3] = {tc[ti], tc[nt + ti], tc[2 * nt + ti]};
            for (int k = 0; k < 4; ++k) {
                const int64_t s = 4 * (int64_t)sj + k;
                const double d[3] = {t[0] - sp[s], t[1] - sp[ns + s], t[2] - sp[2 * ns + s]};
                const double w = sp[3 * ns + s];
                const double ri = 1.0 / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                if constexpr (KIND == FMMBEM_LAPLACE_SL) {
                    v += w * ri;
                } else if constexpr (KIND == FMMBEM_LAPLACE_DL) {
                    const double nd = nrm[sj] * d[0] + nrm[nt + sj] * d[1] + nrm[2 * nt + sj] * d[2];
                    v += w * nd * (ri * ri * ri);
                } else {
                    const int a = ab / 3, c = ab % 3;
                    v += w * ((a == c ? ri : 0.0) + d[a] * d[c] * (ri * ri * ri));
                }
            }
        }
        v64[B.off + e] = v;
        v32[B.off + e] = (float)v;
    }
}

// v64[dst[f] + 4 ab step[f]] += val[PER src[f] + ab] for every folded
// correction f and component ab; each destination is one pair's entry, so no
// two threads meet.  The FP32 copy is rounded again from the sum.
template <int PER>
__global__ void k_fold_corrections(int64_t nfold, const int64_t *__restrict__ dst, const int32_t *__restrict__ step,
                                   const int64_t *__restrict__ srcidx, const double *__restrict__ val,
                                   double *__restrict__ v64, float *__restrict__ v32)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nfold * PER)
        return;
    const int64_t f = t / PER;
    const int ab = (int)(t % PER);
    const int64_t d = dst[f] + (int64_t)ab * 4 * step[f];
    const double v = v64[d] + val[PER * srcidx[f] + ab];
    v64[d] = v;
    v32[d] = (float)v;
}

// y_near = stored near field times x: one HIP block per P2P unit, lane =
// target, the waves take the unit's blocks in turn.  Source values are
// wave-uniform and come through the scalar cache; matrix reads are coalesced
// over the targets, unrolled so that many are in flight.  Partial sums of the
// waves are added in wave order, in FP64.
template <typename R> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };

template <typename R, bool STOKES>
__global__ __launch_bounds__(64 * NEAR_WAVES) void k_near_spmv(int nunit, int per_xcd, const int4 *__restrict__ units,
                                                               const int32_t *__restrict__ blk_ptr,
                                                               const NearBlock *__restrict__ blk,
                                                               const R *__restrict__ vals,
                                                               const double *__restrict__ xs,
                                                               double *__restrict__ ynear)
{
    constexpr int NQ = STOKES ? 3 : 1;
    __shared__ double red[NEAR_WAVES][NQ][64];
    const int g = (int)(blockIdx.x % 8) * per_xcd + (int)(blockIdx.x / 8);
    if (g >= nunit)
        return;
    const int4 u = units[g];
    const int tb = u.x, n = u.y - u.x;  // 1 <= n <= 64
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const bool active = lane < n;
    R acc[NQ];
#pragma unroll
    for (int a = 0; a < NQ; ++a)
        acc[a] = 0;
    using V4 = typename Vec4<R>::type;
    if (active) {
        for (int b = blk_ptr[g] + w; b < blk_ptr[g + 1]; b += NEAR_WAVES) {
            const NearBlock B = blk[b];
            const int ns4 = (B.ns + 3) / 4;
            const V4 *v = reinterpret_cast<const V4 *>(vals + B.off) + lane;
            const double *xj = xs + (int64_t)NQ * B.j0;
            if constexpr (!STOKES) {
#pragma unroll 4
                for (int q = 0; q < ns4; ++q) {
                    const V4 a = v[(int64_t)q * n];
                    const double *xq = xj + 4 * q;
                    acc[0] += ((a.x * (R)xq[0] + a.y * (R)xq[1]) + a.z * (R)xq[2]) + a.w * (R)xq[3];
                }
            } else {
                for (int q = 0; q < ns4; ++q) {
                    const V4 *vq = v + (int64_t)q * 9 * n;
                    const double *xq = xj + 12 * q;
                    R xv[12];
#pragma unroll
                    for (int k = 0; k < 12; ++k)
                        xv[k] = (R)xq[k];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const V4 c0 = vq[(3 * a) * n], c1 = vq[(3 * a + 1) * n], c2 = vq[(3 * a + 2) * n];
                        acc[a] += ((c0.x * xv[0] + c1.x * xv[1]) + c2.x * xv[2]) +
                                  ((c0.y * xv[3] + c1.y * xv[4]) + c2.y * xv[5]) +
                                  ((c0.z * xv[6] + c1.z * xv[7]) + c2.z * xv[8]) +
                                  ((c0.w * xv[9] + c1.w * xv[10]) + c2.w * xv[11]);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int a = 0; a < NQ; ++a)
        red[w][a][lane] = (double)acc[a];
    __syncthreads();
    if (w == 0 && active) {
#pragma unroll
        for (int a = 0; a < NQ; ++a) {
            double s = 0.0;
            for (int k = 0; k < NEAR_WAVES; ++k)
                s += red[k][a][lane];
            ynear[(int64_t)NQ * (tb + lane) + a] = s;
        }
    }
}

// Adds every correction whose pair (target i, source panel j) lies in a
// stored block into that entry and collects the others, in target order, into
// the rest list that the combine step still applies.
void fold_corrections(fmmbem_ctx *ctx, const std::vector<int4> &units, const std::vector<int32_t> &bptr,
                      const std::vector<NearBlock> &blks, hipStream_t st)
{
    Tree &T = ctx->tree;
    NearMatrix &N = ctx->nearm;
    const Correction &C = ctx->corr;
    const int per = ctx->kernel == FMMBEM_STOKES_SL ? 9 : 1;
    const int64_t nt = T.nt;
    std::vector<int32_t> cptr(nt + 1), ccol(std::max<int64_t>(C.nnz, 1)), corig(std::max<int64_t>(C.nnz, 1));
    std::vector<double> cval(std::max<int64_t>(C.nnz, 1) * per);
    FB_HIP(hipMemcpyAsync(cptr.data(), C.ptr, sizeof(int32_t) * (nt + 1), hipMemcpyDeviceToHost, st));
    if (C.nnz > 0) {
        FB_HIP(hipMemcpyAsync(ccol.data(), C.col, sizeof(int32_t) * C.nnz, hipMemcpyDeviceToHost, st));
        FB_HIP(hipMemcpyAsync(corig.data(), C.col_orig, sizeof(int32_t) * C.nnz, hipMemcpyDeviceToHost, st));
        FB_HIP(hipMemcpyAsync(cval.data(), C.val, sizeof(double) * C.nnz * per, hipMemcpyDeviceToHost, st));
    }
    FB_HIP(hipStreamSynchronize(st));
    // unit of every sorted target; per unit, its blocks ordered by first panel
    std::vector<int32_t> unit_of(nt, -1);
    for (int g = 0; g < (int)units.size() && g < T.n_unit; ++g)
        for (int i = units[g].x; i < units[g].y; ++i)
            unit_of[i] = g;
    std::vector<int32_t> order(blks.size());
    for (int g = 0; g + 1 < (int)bptr.size(); ++g) {
        for (int b = bptr[g]; b < bptr[g + 1]; ++b)
            order[b] = b;
        std::sort(order.begin() + bptr[g], order.begin() + bptr[g + 1],
                  [&](int a, int b) { return blks[a].j0 < blks[b].j0; });
    }
    std::vector<int64_t> dst, srcidx;
    std::vector<int32_t> step;
    std::vector<int32_t> rptr(nt + 1, 0), rcol, rorig;
    std::vector<double> rval;
    for (int64_t i = 0; i < nt; ++i) {
        const int g = unit_of[i];
        for (int e = cptr[i]; e < cptr[i + 1]; ++e) {
            const int j = ccol[e];
            int hit = -1;
            if (g >= 0) {
                // last block (by first panel) starting at or before j
                int lo = bptr[g], hi = bptr[g + 1];
                while (hi - lo > 1) {
                    const int mid = (lo + hi) / 2;
                    if (blks[order[mid]].j0 <= j)
                        lo = mid;
                    else
                        hi = mid;
                }
                if (lo < bptr[g + 1]) {
                    const NearBlock &B = blks[order[lo]];
                    if (B.j0 <= j && j < B.j0 + B.ns)
                        hit = order[lo];
                }
            }
            if (hit >= 0) {
                const NearBlock &B = blks[hit];
                const int n = units[g].y - units[g].x;
                dst.push_back(near_index(B.off, n, per, j - B.j0, 0, (int)(i - units[g].x)));
                step.push_back(n);
                srcidx.push_back(e);
            } else {
                rcol.push_back(j);
                rorig.push_back(corig[e]);
                for (int a = 0; a < per; ++a)
                    rval.push_back(cval[(int64_t)per * e + a]);
            }
        }
        rptr[i + 1] = (int32_t)rcol.size();
    }
    N.folded = (int64_t)dst.size();
    DevArena &A = ctx->arena;
    Correction &Rr = N.rest;
    Rr.nnz = (int64_t)rcol.size();
    Rr.ptr = A.alloc<int32_t>(nt + 1);
    Rr.col = A.alloc<int32_t>(std::max<size_t>(rcol.size(), 1));
    Rr.col_orig = A.alloc<int32_t>(std::max<size_t>(rorig.size(), 1));
    Rr.val = A.alloc<double>(std::max<size_t>(rval.size(), 1));
    FB_HIP(hipMemcpyAsync(Rr.ptr, rptr.data(), sizeof(int32_t) * (nt + 1), hipMemcpyHostToDevice, st));
    if (!rcol.empty()) {
        FB_HIP(hipMemcpyAsync(Rr.col, rcol.data(), sizeof(int32_t) * rcol.size(), hipMemcpyHostToDevice, st));
        FB_HIP(hipMemcpyAsync(Rr.col_orig, rorig.data(), sizeof(int32_t) * rorig.size(), hipMemcpyHostToDevice, st));
        FB_HIP(hipMemcpyAsync(Rr.val, rval.data(), sizeof(double) * rval.size(), hipMemcpyHostToDevice, st));
    }
    if (!dst.empty()) {
        DevArena tmp(ctx->arena.al);
        try {
            int64_t *d_dst = tmp.alloc<int64_t>(dst.size());
            int32_t *d_step = tmp.alloc<int32_t>(step.size());
            int64_t *d_src = tmp.alloc<int64_t>(srcidx.size());
            FB_HIP(hipMemcpyAsync(d_dst, dst.data(), sizeof(int64_t) * dst.size(), hipMemcpyHostToDevice, st));
            FB_HIP(hipMemcpyAsync(d_step, step.data(), sizeof(int32_t) * step.size(), hipMemcpyHostToDevice, st));
            FB_HIP(hipMemcpyAsync(d_src, srcidx.data(), sizeof(int64_t) * srcidx.size(), hipMemcpyHostToDevice, st));
            const int64_t work = (int64_t)dst.size() * per;
            if (per == 9)
                k_fold_corrections<9><<<grid_for(work, 256), 256, 0, st>>>((int64_t)dst.size(), d_dst, d_step, d_src,
                                                                          C.val, N.v64, N.v32);
            else
                k_fold_corrections<1><<<grid_for(work, 256), 256, 0, st>>>((int64_t)dst.size(), d_dst, d_step, d_src,
                                                                          C.val, N.v64, N.v32);
            FB_HIP(hipGetLastError());
            FB_HIP(hipStreamSynchronize(st));
        } catch (...) {
            tmp.release();
            throw;
        }
        tmp.release();
    }
}

}  // namespace

// input values per panel (3 for Stokes)
inline int per_q(const fmmbem_ctx *ctx) { return ctx->kernel == FMMBEM_STOKES_SL ? 3 : 1; }

void build_near_matrix(fmmbem_ctx *ctx, hipStream_t st)
{
    Tree &T = ctx->tree;
    NearMatrix &N = ctx->nearm;
    const bool stokes = ctx->kernel == FMMBEM_STOKES_SL;
    const int per = stokes ? 9 : 1;
    const std::vector<int32_t> &hb = T.h_box_i;
    std::vector<int4> units(std::max(T.n_unit, 1));
    std::vector<int32_t> ptr(T.nbox + 1), src(std::max<int64_t>(T.n_p2p, 1));
    if (T.n_unit > 0)
        FB_HIP(hipMemcpyAsync(units.data(), T.p2p_unit, sizeof(int4) * T.n_unit, hipMemcpyDeviceToHost, st));
    FB_HIP(hipMemcpyAsync(ptr.data(), T.p2p_ptr, sizeof(int32_t) * (T.nbox + 1), hipMemcpyDeviceToHost, st));
    if (T.n_p2p > 0)
        FB_HIP(hipMemcpyAsync(src.data(), T.p2p_src, sizeof(int32_t) * T.n_p2p, hipMemcpyDeviceToHost, st));
    FB_HIP(hipStreamSynchronize(st));
    // leaf of every sorted panel
    std::vector<int32_t> leaf_of(T.nt, -1);
    for (int b : T.h_leaves)
        for (int i = hb[6 * b + 1]; i < hb[6 * b + 2]; ++i)
            leaf_of[i] = b;
    std::vector<int32_t> bptr(1, 0), bunit;
    std::vector<NearBlock> blks;
    int64_t off = 0, entries = 0;
    for (int g = 0; g < T.n_unit; ++g) {
        const int n = units[g].y - units[g].x;
        const int t = leaf_of[units[g].x];
        FB_REQUIRE(t >= 0, FMMBEM_EINTERNAL, "P2P unit outside every leaf");
        for (int e = ptr[t]; e < ptr[t + 1]; ++e) {
            const int s = src[e];
            const int ns = hb[6 * s + 2] - hb[6 * s + 1];
            blks.push_back(NearBlock{hb[6 * s + 1], ns, off});
            bunit.push_back(g);
            off += (int64_t)n * ((ns + 3) / 4) * 4 * per;  // padded to groups of four sources
            entries += (int64_t)n * ns;
        }
        bptr.push_back((int32_t)blks.size());
        FB_REQUIRE(blks.size() < ((size_t)1 << 31), FMMBEM_ENOMEM, "stored near field exceeds 2^31 blocks");
    }
    N.entries = entries;
    N.nblk = (int64_t)blks.size();
    DevArena &A = ctx->arena;
    N.blk_ptr = A.alloc<int32_t>(bptr.size());
    N.blk = A.alloc<NearBlock>(std::max<size_t>(blks.size(), 1));
    int32_t *blk_unit = A.alloc<int32_t>(std::max<size_t>(bunit.size(), 1));
    N.v64 = A.alloc<double>(std::max<int64_t>(off, 1));
    N.v32 = A.alloc<float>(std::max<int64_t>(off, 1));
    // the last group of a block may read up to three panels past the end
    N.xs = A.alloc<double>(ctx->n + 3 * per_q(ctx));
    FB_HIP(hipMemsetAsync(N.xs, 0, sizeof(double) * (ctx->n + 3 * per_q(ctx)), st));
    FB_HIP(hipMemcpyAsync(N.blk_ptr, bptr.data(), sizeof(int32_t) * bptr.size(), hipMemcpyHostToDevice, st));
    if (!blks.empty()) {
        FB_HIP(hipMemcpyAsync(N.blk, blks.data(), sizeof(NearBlock) * blks.size(), hipMemcpyHostToDevice, st));
        FB_HIP(hipMemcpyAsync(blk_unit, bunit.data(), sizeof(int32_t) * bunit.size(), hipMemcpyHostToDevice, st));
#define FB_NEAR_BUILD(KIND)                                                                                     \
    k_near_build<KIND><<<(unsigned)N.nblk, 256, 0, st>>>(T.p2p_unit, blk_unit, N.blk, T.nt, ctx->geo.tc, ctx->geo.sp, \
                                                         ctx->geo.nrm, N.v64, N.v32)
        if (stokes)
            FB_NEAR_BUILD(FMMBEM_STOKES_SL);
        else if (ctx->kernel == FMMBEM_LAPLACE_DL)
            FB_NEAR_BUILD(FMMBEM_LAPLACE_DL);
        else
            FB_NEAR_BUILD(FMMBEM_LAPLACE_SL);
#undef FB_NEAR_BUILD
        FB_HIP(hipGetLastError());
    }
    fold_corrections(ctx, units, bptr, blks, st);
    FB_HIP(hipStreamSynchronize(st));  // host vectors go out of scope
}

void launch_near_stored(fmmbem_ctx *ctx, int prec, hipStream_t st)
{
    Tree &T = ctx->tree;
    NearMatrix &N = ctx->nearm;
    const bool stokes = ctx->kernel == FMMBEM_STOKES_SL;
    if (T.n_unit == 0)
        return;
    const int per_xcd = (T.n_unit + 7) / 8;
    const dim3 grid(8 * per_xcd), block(64 * NEAR_WAVES);
    if (prec == FMMBEM_FP64) {
        if (stokes)
            k_near_spmv<double, true><<<grid, block, 0, st>>>(T.n_unit, per_xcd, T.p2p_unit, N.blk_ptr, N.blk, N.v64,
                                                             N.xs, ctx->y_near);
        else
            k_near_spmv<double, false><<<grid, block, 0, st>>>(T.n_unit, per_xcd, T.p2p_unit, N.blk_ptr, N.blk,
                                                              N.v64, N.xs, ctx->y_near);
    } else {
        if (stokes)
            k_near_spmv<float, true><<<grid, block, 0, st>>>(T.n_unit, per_xcd, T.p2p_unit, N.blk_ptr, N.blk, N.v32,
                                                            N.xs, ctx->y_near);
        else
            k_near_spmv<float, false><<<grid, block, 0, st>>>(T.n_unit, per_xcd, T.p2p_unit, N.blk_ptr, N.blk,
                                                             N.v32, N.xs, ctx->y_near);
    }
    FB_HIP(hipGetLastError());
}

}  // namespace fmmbem
