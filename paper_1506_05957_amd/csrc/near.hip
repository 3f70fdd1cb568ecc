// Near-singular and self corrections of the BEM operator (Sec. 2.3), built
// once per mesh as a sparse matrix over sorted panels.
//
// The mat-vec evaluates every (target i, source panel j != i) pair with the
// 4-point rule, through P2P or the expansions.  The exact operator differs
// from that on two kinds of entries, which this matrix supplies:
//   near-singular (|c_i - c_j|^2 < 8 S_j, i.e. closer than 2 sqrt(2 S_j)):
//       S_ij = int_j K (25-point rule) - int_j K (4-point rule)
//   the panel holding the target (i = j):
//       S_ii = int_i K, with the polar split about the centroid of Hess and
//       Smith: radial integral exact, angular integral by 32-point
//       Gauss-Legendre quadrature on each edge.
// K is 1/r (Laplace), the Stokeslet delta/r + r r^T / r^3 (Eq. 7) or the
// double-layer kernel n_j . (x - y) / |x - y|^3 (Eq. 11, zero on the target's
// own flat panel), without the 1/(4 pi) or -1/(8 pi mu) factor.  Every near-singular pair lies inside a
// P2P box pair (the acceptance test guarantees it), so candidates come from the
// P2P lists.  Compiled with -ffp-contract=off: the near/far decision uses the
// same rounded distance as the classification of Sec. 2.3 anywhere else.
#include <hipcub/hipcub.hpp>

#include <cmath>
#include <vector>

#include "common.h"

namespace fmmbem {

namespace {

constexpr int NEAR_PTS = 25;
constexpr int NQ_ANG = 32;

struct RuleTables {
    double nb[3 * NEAR_PTS];
    double nw[NEAR_PTS];
    double gx[NQ_ANG];
    double gw[NQ_ANG];
};

__device__ inline bool is_near(const double *__restrict__ tc, const double *__restrict__ S, int64_t nt, int i, int j)
{
    double dx = tc[i] - tc[j], dy = tc[nt + i] - tc[nt + j], dz = tc[2 * nt + i] - tc[2 * nt + j];
    double d2 = (dx * dx + dy * dy) + dz * dz;
    return d2 < 8.0 * S[j];
}

__global__ void k_corr_count(int64_t nt, const int32_t *__restrict__ panel_leaf, const int32_t *__restrict__ p2p_ptr,
                             const int32_t *__restrict__ p2p_src, const int32_t *__restrict__ box_i,
                             const double *__restrict__ tc, const double *__restrict__ S, int32_t *__restrict__ cnt)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nt)
        return;
    int leaf = panel_leaf[i];
    int c = 0;
    for (int e = p2p_ptr[leaf]; e < p2p_ptr[leaf + 1]; ++e) {
        int sb = p2p_src[e];
        for (int j = box_i[6 * sb + 1]; j < box_i[6 * sb + 2]; ++j)
            if (j == (int)i || is_near(tc, S, nt, (int)i, j))
                ++c;
    }
    cnt[i] = c;
}

// angular quadrature of the polar split about x (x in the panel's plane):
// I = sum_edges int h / cos(theta) dtheta,  J = sum_edges int e e^T h / cos(theta) dtheta
__device__ void self_integral(const double *__restrict__ v, const double *x, const RuleTables &R, double &I,
                              double *J, bool want_J)
{
    I = 0.0;
    if (want_J)
        for (int k = 0; k < 9; ++k)
            J[k] = 0.0;
    for (int e = 0; e < 3; ++e) {
        const double *a = v + 3 * e, *b = v + 3 * ((e + 1) % 3);
        double ev[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        double len = sqrt(ev[0] * ev[0] + ev[1] * ev[1] + ev[2] * ev[2]);
        double t[3] = {ev[0] / len, ev[1] / len, ev[2] / len};
        double ax[3] = {a[0] - x[0], a[1] - x[1], a[2] - x[2]};
        double sa = ax[0] * t[0] + ax[1] * t[1] + ax[2] * t[2];
        double u[3] = {ax[0] - sa * t[0], ax[1] - sa * t[1], ax[2] - sa * t[2]};
        double h = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        u[0] /= h;
        u[1] /= h;
        u[2] /= h;
        double th_a = atan2(sa, h), th_b = atan2(sa + len, h);
        double mid = 0.5 * (th_a + th_b), half = 0.5 * (th_b - th_a);
        for (int q = 0; q < NQ_ANG; ++q) {
            double th = mid + half * R.gx[q];
            double cs = cos(th), sn = sin(th);
            double f = R.gw[q] * half * h / cs;
            I += f;
            if (want_J) {
                double e_[3] = {cs * u[0] + sn * t[0], cs * u[1] + sn * t[1], cs * u[2] + sn * t[2]};
                for (int p = 0; p < 3; ++p)
                    for (int r = 0; r < 3; ++r)
                        J[3 * p + r] += f * e_[p] * e_[r];
            }
        }
    }
}

template <int KIND>
__global__ void k_corr_fill(int64_t nt, const int32_t *__restrict__ panel_leaf, const int32_t *__restrict__ p2p_ptr,
                            const int32_t *__restrict__ p2p_src, const int32_t *__restrict__ box_i,
                            const double *__restrict__ tc, const double *__restrict__ S,
                            const double *__restrict__ vtx, const double *__restrict__ sp,
                            const int32_t *__restrict__ rowptr, int32_t *__restrict__ col, double *__restrict__ val,
                            const RuleTables *__restrict__ Rg, const int32_t *__restrict__ perm,
                            int32_t *__restrict__ col_orig, const double *__restrict__ nrm)
{
    constexpr bool STOKES = KIND == FMMBEM_STOKES_SL;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nt)
        return;
    const RuleTables &R = *Rg;
    const int64_t ns = 4 * nt;
    double x[3] = {tc[i], tc[nt + i], tc[2 * nt + i]};
    int leaf = panel_leaf[i];
    int64_t o = rowptr[i];
    for (int e = p2p_ptr[leaf]; e < p2p_ptr[leaf + 1]; ++e) {
        int sb = p2p_src[e];
        for (int j = box_i[6 * sb + 1]; j < box_i[6 * sb + 2]; ++j) {
            bool self = j == (int)i;
            if (!self && !is_near(tc, S, nt, (int)i, j))
                continue;
            col[o] = j;
            col_orig[o] = perm[j];
            const double *v = vtx + 9 * (int64_t)j;
            if (KIND == FMMBEM_LAPLACE_DL) {
                // n_j . (x - y) / |x - y|^3; zero on the target's own flat panel
                double acc = 0.0;
                if (!self) {
                    const double nj[3] = {nrm[j], nrm[nt + j], nrm[2 * nt + j]};
                    double a25 = 0.0, a4 = 0.0;
                    for (int k = 0; k < NEAR_PTS; ++k) {
                        const double *l = R.nb + 3 * k;
                        double y0 = (l[0] * v[0] + l[1] * v[3]) + l[2] * v[6];
                        double y1 = (l[0] * v[1] + l[1] * v[4]) + l[2] * v[7];
                        double y2 = (l[0] * v[2] + l[1] * v[5]) + l[2] * v[8];
                        double d[3] = {x[0] - y0, x[1] - y1, x[2] - y2};
                        double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
                        double r = sqrt(r2);
                        a25 += R.nw[k] * S[j] * ((nj[0] * d[0] + nj[1] * d[1]) + nj[2] * d[2]) / (r2 * r);
                    }
                    for (int k = 0; k < 4; ++k) {
                        int64_t s = 4 * (int64_t)j + k;
                        double d[3] = {x[0] - sp[s], x[1] - sp[ns + s], x[2] - sp[2 * ns + s]};
                        double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
                        double r = sqrt(r2);
                        a4 += sp[3 * ns + s] * ((nj[0] * d[0] + nj[1] * d[1]) + nj[2] * d[2]) / (r2 * r);
                    }
                    acc = a25 - a4;
                }
                val[o] = acc;
            } else if (!STOKES) {
                double acc;
                if (self) {
                    self_integral(v, x, R, acc, nullptr, false);
                } else {
                    double a25 = 0.0, a4 = 0.0;
                    for (int k = 0; k < NEAR_PTS; ++k) {
                        const double *l = R.nb + 3 * k;
                        double y0 = (l[0] * v[0] + l[1] * v[3]) + l[2] * v[6];
                        double y1 = (l[0] * v[1] + l[1] * v[4]) + l[2] * v[7];
                        double y2 = (l[0] * v[2] + l[1] * v[5]) + l[2] * v[8];
                        double dx = x[0] - y0, dy = x[1] - y1, dz = x[2] - y2;
                        a25 += R.nw[k] * S[j] / sqrt((dx * dx + dy * dy) + dz * dz);
                    }
                    for (int k = 0; k < 4; ++k) {
                        int64_t s = 4 * (int64_t)j + k;
                        double dx = x[0] - sp[s], dy = x[1] - sp[ns + s], dz = x[2] - sp[2 * ns + s];
                        a4 += sp[3 * ns + s] / sqrt((dx * dx + dy * dy) + dz * dz);
                    }
                    acc = a25 - a4;
                }
                val[o] = acc;
            } else {
                double blk[9];
                if (self) {
                    double I;
                    self_integral(v, x, R, I, blk, true);
                    blk[0] += I;
                    blk[4] += I;
                    blk[8] += I;
                } else {
                    for (int k = 0; k < 9; ++k)
                        blk[k] = 0.0;
                    for (int k = 0; k < NEAR_PTS; ++k) {
                        const double *l = R.nb + 3 * k;
                        double d[3];
                        for (int c = 0; c < 3; ++c)
                            d[c] = x[c] - ((l[0] * v[c] + l[1] * v[3 + c]) + l[2] * v[6 + c]);
                        double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
                        double r = sqrt(r2);
                        double wr = R.nw[k] * S[j] / r;
                        for (int p = 0; p < 3; ++p)
                            for (int q = 0; q < 3; ++q)
                                blk[3 * p + q] += wr * ((p == q ? 1.0 : 0.0) + d[p] * d[q] / r2);
                    }
                    for (int k = 0; k < 4; ++k) {
                        int64_t s = 4 * (int64_t)j + k;
                        double d[3] = {x[0] - sp[s], x[1] - sp[ns + s], x[2] - sp[2 * ns + s]};
                        double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
                        double r = sqrt(r2);
                        double wr = sp[3 * ns + s] / r;
                        for (int p = 0; p < 3; ++p)
                            for (int q = 0; q < 3; ++q)
                                blk[3 * p + q] -= wr * ((p == q ? 1.0 : 0.0) + d[p] * d[q] / r2);
                    }
                }
                for (int k = 0; k < 9; ++k)
                    val[9 * o + k] = blk[k];
            }
            ++o;
        }
    }
}

__global__ void k_round_f32(int64_t n, const double *__restrict__ a, float *__restrict__ b)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        b[i] = (float)a[i];
}

}  // namespace

// The FP32 mat-vecs read the correction in FP32: its rounding (2^-24
// relative per value, the products still summed in FP64) is far below the
// error those mat-vecs are allowed (the schedule takes FP32 only where
// Eq. 19 allows at least fp32_eps, 1e-5 by default), and
// the correction product, which reads the values once per mat-vec and is
// bound by that read, moves half the bytes
void correction_fp32(fmmbem_ctx *ctx, Correction &C, hipStream_t st)
{
    const int64_t n = std::max<int64_t>(C.nnz, 1) * (ctx->kernel == FMMBEM_STOKES_SL ? 9 : 1);
    C.val32 = ctx->arena.alloc<float>(n);
    k_round_f32<<<grid_for(n, 256), 256, 0, st>>>(n, C.val, C.val32);
    FB_HIP(hipGetLastError());
}

void build_correction(fmmbem_ctx *ctx, hipStream_t st)
{
    const int64_t nt = ctx->nt;
    Tree &T = ctx->tree;
    Geometry &G = ctx->geo;
    Correction &C = ctx->corr;
    DevArena tmp(ctx->arena.al);
    try {
        RuleTables R;
        near_rule_table(5, R.nb, R.nw);
        gauss_legendre_gw(NQ_ANG, R.gx, R.gw);
        RuleTables *dR = tmp.alloc<RuleTables>(1);
        FB_HIP(hipMemcpyAsync(dR, &R, sizeof(R), hipMemcpyHostToDevice, st));
        int32_t *cnt = tmp.alloc<int32_t>(nt + 1);
        FB_HIP(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (nt + 1), st));
        k_corr_count<<<grid_for(nt, 128), 128, 0, st>>>(nt, T.panel_leaf, T.p2p_ptr, T.p2p_src, T.box_i, G.tc, G.S,
                                                          cnt);
        FB_HIP(hipGetLastError());
        C.ptr = ctx->arena.alloc<int32_t>(nt + 1);
        size_t bytes = 0;
        FB_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, cnt, C.ptr, (int)(nt + 1), st));
        void *t = tmp.alloc<char>(bytes);
        FB_HIP(hipcub::DeviceScan::ExclusiveSum(t, bytes, cnt, C.ptr, (int)(nt + 1), st));
        int32_t nnz = 0;
        FB_HIP(hipMemcpyAsync(&nnz, C.ptr + nt, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        FB_HIP(hipStreamSynchronize(st));
        C.nnz = nnz;
        const bool stokes = ctx->kernel == FMMBEM_STOKES_SL;
        C.col = ctx->arena.alloc<int32_t>(std::max<int64_t>(nnz, 1));
        C.col_orig = ctx->arena.alloc<int32_t>(std::max<int64_t>(nnz, 1));
        C.val = ctx->arena.alloc<double>(std::max<int64_t>(nnz, 1) * (stokes ? 9 : 1));
#define FB_CORR_FILL(KIND)                                                                                    \
    k_corr_fill<KIND><<<grid_for(nt, 64), 64, 0, st>>>(nt, T.panel_leaf, T.p2p_ptr, T.p2p_src, T.box_i, G.tc, G.S, \
                                                       G.vtx, G.sp, C.ptr, C.col, C.val, dR, T.perm, C.col_orig, G.nrm)
        if (ctx->kernel == FMMBEM_STOKES_SL)
            FB_CORR_FILL(FMMBEM_STOKES_SL);
        else if (ctx->kernel == FMMBEM_LAPLACE_DL)
            FB_CORR_FILL(FMMBEM_LAPLACE_DL);
        else
            FB_CORR_FILL(FMMBEM_LAPLACE_SL);
#undef FB_CORR_FILL
        FB_HIP(hipGetLastError());
        FB_HIP(hipStreamSynchronize(st));
        tmp.release();
    } catch (...) {
        (void)hipStreamSynchronize(st);
        tmp.release();
        throw;
    }
}

}  // namespace fmmbem
