// The regular near field stored as a block-sparse matrix (Sec. 2.3, 2.5): the
// 4-point rule between every target panel and the panels of the leaves in its
// P2P list, assembled once and multiplied by every mat-vec, as the paper holds
// its near field.  The near-singular and self corrections stay as they are:
// the stored block leaves each target's own panel at zero, exactly as the
// on-the-fly P2P skips it.
#include <algorithm>
#include <vector>

#include "common.h"

namespace fmmbem {

namespace {

constexpr int NEAR_WAVES = 8;

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
    const int64_t cnt = (int64_t)n * B.ns * PER;
    for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) {
        const int i = (int)(e % n);
        const int64_t r = e / n;
        const int ab = (int)(r % PER), j = (int)(r / PER);
        const int ti = tb + i, sj = B.j0 + j;
        double v = 0.0;
        if (ti != sj) {
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

// xs = x in sorted panel order
template <int NQ>
__global__ void k_sort_input(int64_t nt, const int32_t *__restrict__ perm, const double *__restrict__ x,
                             double *__restrict__ xs)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nt)
        return;
    const int64_t o = perm[i];
#pragma unroll
    for (int a = 0; a < NQ; ++a)
        xs[NQ * i + a] = x[NQ * o + a];
}

// y_near = stored near field times x: one HIP block per P2P unit, lane =
// target, the waves take the unit's blocks in turn.  Source values are
// wave-uniform and come through the scalar cache; matrix reads are coalesced
// over the targets, unrolled so that many are in flight.  Partial sums of the
// waves are added in wave order, in FP64.
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
    if (active) {
        for (int b = blk_ptr[g] + w; b < blk_ptr[g + 1]; b += NEAR_WAVES) {
            const NearBlock B = blk[b];
            const R *v = vals + B.off + lane;
            const double *xj = xs + (int64_t)NQ * B.j0;
            if constexpr (!STOKES) {
#pragma unroll 16
                for (int j = 0; j < B.ns; ++j)
                    acc[0] += v[(int64_t)j * n] * (R)xj[j];
            } else {
#pragma unroll 4
                for (int j = 0; j < B.ns; ++j) {
                    const R x0 = (R)xj[3 * j], x1 = (R)xj[3 * j + 1], x2 = (R)xj[3 * j + 2];
                    const R *vj = v + (int64_t)j * 9 * n;
                    acc[0] += vj[0] * x0 + vj[n] * x1 + vj[2 * n] * x2;
                    acc[1] += vj[3 * n] * x0 + vj[4 * n] * x1 + vj[5 * n] * x2;
                    acc[2] += vj[6 * n] * x0 + vj[7 * n] * x1 + vj[8 * n] * x2;
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

}  // namespace

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
            off += (int64_t)n * ns * per;
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
    N.xs = A.alloc<double>(ctx->n);
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
    FB_HIP(hipStreamSynchronize(st));  // host vectors go out of scope
}

void sort_near_input(fmmbem_ctx *ctx, const double *x, hipStream_t st)
{
    Tree &T = ctx->tree;
    if (ctx->kernel == FMMBEM_STOKES_SL)
        k_sort_input<3><<<grid_for(T.nt, 256), 256, 0, st>>>(T.nt, T.perm, x, ctx->nearm.xs);
    else
        k_sort_input<1><<<grid_for(T.nt, 256), 256, 0, st>>>(T.nt, T.perm, x, ctx->nearm.xs);
    FB_HIP(hipGetLastError());
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
