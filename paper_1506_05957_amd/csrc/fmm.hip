// The FMM-accelerated BEM mat-vec (Sec. 2.4-2.5, Eq. 12): charges, P2M, M2M,
// M2L, L2L, L2P, P2P and the near-field correction, for the Laplace and the
// Stokes single layer, in FP64 or FP32, with the expansion order p chosen per
// call (Sec. 2.6).
//
// Sources are the 4 Gauss points of every panel, with charge q_k S_j x_j
// (Eq. 10, 12); targets are the centroids.  Stokes uses the decomposition of
// the Stokeslet into four Laplace potentials (Sec. 3.2): with f = w t,
//   Phi_a = sum f_a / r (a = 1..3),  Phi_4 = sum f.(y - c) / r,
//   u_i(x) = Phi_i - (x - c)_j d_i Phi_j + d_i Phi_4,
// valid for any fixed c; each expansion keeps c at its own box centre and the
// translations add the change of centre (M4 += (c_old - c_new) . M).
//
// Expansions are stored scaled by the box half-size s: M~ = M / s^n and
// L~ = L s^(n+1), so that FP32 stays in range; all owner-computes, no atomics.
#include <cmath>

#include "common.h"
#include "harmonics.h"

namespace fmmbem {

__constant__ InvTable<double> c_inv_d = make_inv_table<double>();
__constant__ InvTable<float> c_inv_f = make_inv_table<float>();

template <typename R> __device__ inline R inv_int(int k);
template <> __device__ inline double inv_int<double>(int k) { return c_inv_d.v[k]; }
template <> __device__ inline float inv_int<float>(int k) { return c_inv_f.v[k]; }

namespace {

constexpr int FULL_MAX = (P_MAX + 1) * (P_MAX + 1);

__device__ inline int full_idx(int n, int m) { return n * n + n + m; }

// Column m (n = m..p) of the regular harmonics at (x, y, z), written to the
// full table (m and -m).  Called by the thread that owns column m.
template <typename R>
__device__ void regular_column_full(R x, R y, R z, int m, int p, cplx<R> *__restrict__ T)
{
    R r2 = x * x + y * y + z * z;
    R dre = 1, dim = 0;
    for (int k = 1; k <= m; ++k) {
        R f = -inv_int<R>(2 * k);
        R a = f * (x * dre - y * dim), b = f * (x * dim + y * dre);
        dre = a;
        dim = b;
    }
    R cr = dre, ci = dim, pr = 0, pi = 0;
    const R sg = (m & 1) ? R(-1) : R(1);
    for (int n = m; n <= p; ++n) {
        if (n > m) {
            R f = inv_int<R>((n - m) * (n + m));
            R a = R(2 * n - 1) * z;
            R nr = (a * cr - r2 * pr) * f, ni = (a * ci - r2 * pi) * f;
            pr = cr;
            pi = ci;
            cr = nr;
            ci = ni;
        }
        T[full_idx(n, m)] = cplx<R>{cr, ci};
        if (m > 0)
            T[full_idx(n, -m)] = cplx<R>{sg * cr, -sg * ci};
    }
}

// Column m (n = m..q) of the irregular harmonics, full table.
template <typename R>
__device__ void irregular_column_full(R x, R y, R z, int m, int q, cplx<R> *__restrict__ T)
{
    R r2 = x * x + y * y + z * z;
    R ir2 = R(1) / r2;
    R dre = R(1) / sqrt(r2), dim = 0;
    for (int k = 1; k <= m; ++k) {
        R f = -R(2 * k - 1) * ir2;
        R a = f * (x * dre - y * dim), b = f * (x * dim + y * dre);
        dre = a;
        dim = b;
    }
    R cr = dre, ci = dim, pr = 0, pi = 0;
    const R sg = (m & 1) ? R(-1) : R(1);
    for (int n = m; n <= q; ++n) {
        if (n > m) {
            R a = R(2 * n - 1) * z;
            R b = R((n - 1) * (n - 1) - m * m);
            R nr = (a * cr - b * pr) * ir2, ni = (a * ci - b * pi) * ir2;
            pr = cr;
            pi = ci;
            cr = nr;
            ci = ni;
        }
        T[full_idx(n, m)] = cplx<R>{cr, ci};
        if (m > 0)
            T[full_idx(n, -m)] = cplx<R>{sg * cr, -sg * ci};
    }
}

__device__ inline void idx_to_nm(int idx, int &n, int &m)
{
    n = (int)((sqrtf(8.0f * idx + 1.0f) - 1.0f) * 0.5f);
    while ((n + 1) * (n + 2) / 2 <= idx)
        ++n;
    while (n * (n + 1) / 2 > idx)
        --n;
    m = idx - n * (n + 1) / 2;
}

template <typename R> __device__ inline cplx<R> load_full(const cplx<R> *__restrict__ E, int n, int m)
{
    // coefficient (n, m) of a real-function expansion stored for m >= 0
    if (m >= 0)
        return E[cidx(n, m)];
    cplx<R> v = E[cidx(n, -m)];
    R sg = (m & 1) ? R(-1) : R(1);
    return cplx<R>{sg * v.re, -sg * v.im};
}

// ---------------------------------------------------------------------------
// charges (a4)
template <typename R, bool STOKES>
__global__ void k_charges(int64_t nt, const int32_t *__restrict__ perm, const int32_t *__restrict__ panel_leaf,
                          const double *__restrict__ box_r, const double *__restrict__ sp,
                          const double *__restrict__ x, R *__restrict__ q)
{
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ns = 4 * nt;
    if (s >= ns)
        return;
    int64_t j = s >> 2;
    int64_t o = perm[j];
    double w = sp[3 * ns + s];
    if (!STOKES) {
        q[s] = (R)(w * x[o]);
    } else {
        double t0 = x[3 * o], t1 = x[3 * o + 1], t2 = x[3 * o + 2];
        const double *c = box_r + 5 * (int64_t)panel_leaf[j];
        double dy0 = sp[s] - c[0], dy1 = sp[ns + s] - c[1], dy2 = sp[2 * ns + s] - c[2];
        q[s] = (R)(w * t0);
        q[ns + s] = (R)(w * t1);
        q[2 * ns + s] = (R)(w * t2);
        q[3 * ns + s] = (R)(w * ((t0 * dy0 + t1 * dy1) + t2 * dy2));
    }
}

// ---------------------------------------------------------------------------
// P2M (a5): one block per leaf; thread = (order m, source slice).
template <typename R, int NCH>
__global__ __launch_bounds__(256) void k_p2m(int p, int ncs, const int32_t *__restrict__ leaves,
                                             const int32_t *__restrict__ box_i, const double *__restrict__ box_r,
                                             double side, int64_t nt, const double *__restrict__ sp,
                                             const float *__restrict__ sp32, const R *__restrict__ q,
                                             cplx<R> *__restrict__ M)
{
    constexpr int SL = 8;
    __shared__ cplx<R> red[SL][NC_MAX];
    const int b = leaves[blockIdx.x];
    const int lv = box_i[6 * b], pb = box_i[6 * b + 1], pe = box_i[6 * b + 2];
    const double s = ldexp(side, -(lv + 1));
    const double *c = box_r + 5 * (int64_t)b;
    const int m = threadIdx.x & 31, sl = threadIdx.x >> 5;
    const int64_t ns = 4 * nt;
    const int nc = ncoef(p);
    for (int ch = 0; ch < NCH; ++ch) {
        R are[P_MAX + 1], aim[P_MAX + 1];
#pragma unroll
        for (int n = 0; n <= P_MAX; ++n)
            are[n] = aim[n] = 0;
        if (m <= p) {
            for (int64_t src = 4 * (int64_t)pb + sl; src < 4 * (int64_t)pe; src += SL) {
                R x, y, z;
                if constexpr (sizeof(R) == 8) {
                    double is = 1.0 / s;
                    x = (R)((sp[src] - c[0]) * is);
                    y = (R)((sp[ns + src] - c[1]) * is);
                    z = (R)((sp[2 * ns + src] - c[2]) * is);
                } else {
                    float is = (float)(1.0 / s);
                    x = sp32[src] * is;
                    y = sp32[ns + src] * is;
                    z = sp32[2 * ns + src] * is;
                }
                const R qq = q[ch * ns + src];
                const R r2 = x * x + y * y + z * z;
                R dre = 1, dim = 0;
                for (int k = 1; k <= m; ++k) {
                    R f = -inv_int<R>(2 * k);
                    R a = f * (x * dre - y * dim), bb = f * (x * dim + y * dre);
                    dre = a;
                    dim = bb;
                }
                R cr = 0, ci = 0, pr = 0, pi = 0;
#pragma unroll
                for (int n = 0; n <= P_MAX; ++n) {
                    if (n <= p) {
                        if (n == m) {
                            cr = dre;
                            ci = dim;
                        } else if (n > m) {
                            R f = inv_int<R>((n - m) * (n + m));
                            R a = R(2 * n - 1) * z;
                            R nr = (a * cr - r2 * pr) * f, ni = (a * ci - r2 * pi) * f;
                            pr = cr;
                            pi = ci;
                            cr = nr;
                            ci = ni;
                        }
                        if (n >= m) {
                            are[n] += qq * cr;
                            aim[n] -= qq * ci;
                        }
                    }
                }
            }
        }
        if (m <= p) {
#pragma unroll
            for (int n = 0; n <= P_MAX; ++n)
                if (n <= p && n >= m)
                    red[sl][cidx(n, m)] = cplx<R>{are[n], aim[n]};
        }
        __syncthreads();
        for (int t = threadIdx.x; t < nc; t += blockDim.x) {
            R sr = 0, si = 0;
            for (int k = 0; k < SL; ++k) {
                sr += red[k][t].re;
                si += red[k][t].im;
            }
            M[((int64_t)b * NCH + ch) * ncs + t] = cplx<R>{sr, si};
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// M2M (a6): one block per box of a level; sums its children (written before).
template <typename R, int NCH>
__global__ __launch_bounds__(64) void k_m2m(int p, int ncs, int box0, const int32_t *__restrict__ box_i,
                                            const double *__restrict__ box_r, double side, cplx<R> *__restrict__ M)
{
    __shared__ cplx<R> Rt[FULL_MAX];
    __shared__ cplx<R> Mc[NCH][FULL_MAX];
    const int P = box0 + blockIdx.x;
    const int nchild = box_i[6 * P + 5];
    if (nchild == 0)
        return;
    const int c0 = box_i[6 * P + 4], lvP = box_i[6 * P];
    const double sP = ldexp(side, -(lvP + 1));
    const double *cP = box_r + 5 * (int64_t)P;
    const int nc = ncoef(p);
    constexpr int NO = (NC_MAX + 63) / 64;
    R acc_re[NO][NCH], acc_im[NO][NCH];
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
            acc_re[o][ch] = acc_im[o][ch] = 0;
    for (int C = c0; C < c0 + nchild; ++C) {
        const double *cC = box_r + 5 * (int64_t)C;
        const double dphys[3] = {cC[0] - cP[0], cC[1] - cP[1], cC[2] - cP[2]};
        __syncthreads();
        if ((int)threadIdx.x <= p)
            regular_column_full<R>((R)(dphys[0] / sP), (R)(dphys[1] / sP), (R)(dphys[2] / sP), threadIdx.x, p, Rt);
        for (int t = threadIdx.x; t < (p + 1) * (p + 1); t += blockDim.x) {
            int n = 0;
            while ((n + 1) * (n + 1) <= t)
                ++n;
            int m = t - n * n - n;
            R sc = (R)ldexp(1.0, -n);
            for (int ch = 0; ch < NCH; ++ch) {
                cplx<R> v = load_full(M + ((int64_t)C * NCH + ch) * ncs, n, m);
                Mc[ch][t] = cplx<R>{v.re * sc, v.im * sc};
            }
        }
        __syncthreads();
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            int idx = threadIdx.x + 64 * o;
            if (idx >= nc)
                continue;
            int n, m;
            idx_to_nm(idx, n, m);
            R sre[NCH], sim[NCH];
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
                sre[ch] = sim[ch] = 0;
            for (int k = 0; k <= n; ++k) {
                int j = n - k;
                int l0 = max(-k, m - j), l1 = min(k, m + j);
                for (int l = l0; l <= l1; ++l) {
                    cplx<R> rv = Rt[full_idx(k, l)];  // conj applied below
                    int mi = full_idx(j, m - l);
#pragma unroll
                    for (int ch = 0; ch < NCH; ++ch) {
                        cplx<R> mv = Mc[ch][mi];
                        sre[ch] += rv.re * mv.re + rv.im * mv.im;
                        sim[ch] += rv.re * mv.im - rv.im * mv.re;
                    }
                }
            }
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                acc_re[o][ch] += sre[ch];
                acc_im[o][ch] += sim[ch];
            }
            if constexpr (NCH == 4) {
                acc_re[o][3] += (R)dphys[0] * sre[0] + (R)dphys[1] * sre[1] + (R)dphys[2] * sre[2];
                acc_im[o][3] += (R)dphys[0] * sim[0] + (R)dphys[1] * sim[1] + (R)dphys[2] * sim[2];
            }
        }
    }
#pragma unroll
    for (int o = 0; o < NO; ++o) {
        int idx = threadIdx.x + 64 * o;
        if (idx >= nc)
            continue;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
            M[((int64_t)P * NCH + ch) * ncs + idx] = cplx<R>{acc_re[o][ch], acc_im[o][ch]};
    }
}

// ---------------------------------------------------------------------------
// M2L (a7): one block per target box, owner-computes over its M2L list.
// L_k^l = (-1)^k sum_{n,m} M_n^m I_{n+k}^{m+l}(c_T - c_S), in scaled form with
// sigma = the larger half-size of the pair.
template <typename R, int NCH>
__global__ __launch_bounds__(64) void k_m2l(int p, int ncs, const int32_t *__restrict__ ptr,
                                            const int32_t *__restrict__ srcs, const int32_t *__restrict__ box_i,
                                            const double *__restrict__ box_r, double side,
                                            const cplx<R> *__restrict__ M, cplx<R> *__restrict__ L)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cplx<R> *It = reinterpret_cast<cplx<R> *>(smem_raw);  // (2p+1)^2
    const int q = 2 * p;
    cplx<R> *Ms = It + (q + 1) * (q + 1);                  // NCH * (p+1)^2
    const int fp = (p + 1) * (p + 1);
    const int T = blockIdx.x;
    const int lvT = box_i[6 * T];
    const double *cT = box_r + 5 * (int64_t)T;
    const int nc = ncoef(p);
    constexpr int NO = (NC_MAX + 63) / 64;
    R acc_re[NO][NCH], acc_im[NO][NCH];
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
            acc_re[o][ch] = acc_im[o][ch] = 0;
    for (int e = ptr[T]; e < ptr[T + 1]; ++e) {
        const int S = srcs[e];
        const int lvS = box_i[6 * S];
        const int lmin = min(lvS, lvT);
        const int eS = lvS - lmin, eT = lvT - lmin;
        const double sigma = ldexp(side, -(lmin + 1));
        const double *cS = box_r + 5 * (int64_t)S;
        const double d[3] = {cT[0] - cS[0], cT[1] - cS[1], cT[2] - cS[2]};
        __syncthreads();
        if ((int)threadIdx.x <= q)
            irregular_column_full<R>((R)(d[0] / sigma), (R)(d[1] / sigma), (R)(d[2] / sigma), threadIdx.x, q, It);
        for (int t = threadIdx.x; t < fp; t += blockDim.x) {
            int n = 0;
            while ((n + 1) * (n + 1) <= t)
                ++n;
            int m = t - n * n - n;
            R sc = (R)ldexp(1.0, -eS * n);
            for (int ch = 0; ch < NCH; ++ch) {
                cplx<R> v = load_full(M + ((int64_t)S * NCH + ch) * ncs, n, m);
                Ms[ch * fp + t] = cplx<R>{v.re * sc, v.im * sc};
            }
        }
        __syncthreads();
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            int idx = threadIdx.x + 64 * o;
            if (idx >= nc)
                continue;
            int k, l;
            idx_to_nm(idx, k, l);
            R sre[NCH], sim[NCH];
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
                sre[ch] = sim[ch] = 0;
            for (int n = 0; n <= p; ++n) {
                const cplx<R> *Irow = It + full_idx(n + k, l);  // + m below
                const int mb = n * n + n;
                for (int m = -n; m <= n; ++m) {
                    cplx<R> iv = Irow[m];
#pragma unroll
                    for (int ch = 0; ch < NCH; ++ch) {
                        cplx<R> mv = Ms[ch * fp + mb + m];
                        sre[ch] += mv.re * iv.re - mv.im * iv.im;
                        sim[ch] += mv.re * iv.im + mv.im * iv.re;
                    }
                }
            }
            R f = (R)ldexp((k & 1) ? -1.0 : 1.0, -eT * (k + 1));
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                acc_re[o][ch] += f * sre[ch];
                acc_im[o][ch] += f * sim[ch];
            }
            if constexpr (NCH == 4) {
                // change of centre of Phi_4 from c_S to c_T
                const R g0 = (R)(cS[0] - cT[0]), g1 = (R)(cS[1] - cT[1]), g2 = (R)(cS[2] - cT[2]);
                acc_re[o][3] += f * (g0 * sre[0] + g1 * sre[1] + g2 * sre[2]);
                acc_im[o][3] += f * (g0 * sim[0] + g1 * sim[1] + g2 * sim[2]);
            }
        }
    }
#pragma unroll
    for (int o = 0; o < NO; ++o) {
        int idx = threadIdx.x + 64 * o;
        if (idx >= nc)
            continue;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
            L[((int64_t)T * NCH + ch) * ncs + idx] = cplx<R>{acc_re[o][ch], acc_im[o][ch]};
    }
}

// ---------------------------------------------------------------------------
// L2L (a8): one block per box of a level >= 1, adds its parent's local expansion.
template <typename R, int NCH>
__global__ __launch_bounds__(64) void k_l2l(int p, int ncs, int box0, const int32_t *__restrict__ box_i,
                                            const double *__restrict__ box_r, double side, cplx<R> *__restrict__ L)
{
    __shared__ cplx<R> Rt[FULL_MAX];
    __shared__ cplx<R> Lp[NCH][FULL_MAX];
    const int C = box0 + blockIdx.x;
    const int P = box_i[6 * C + 3];
    const int lvP = box_i[6 * P];
    const double sP = ldexp(side, -(lvP + 1));
    const double *cP = box_r + 5 * (int64_t)P, *cC = box_r + 5 * (int64_t)C;
    const double dphys[3] = {cC[0] - cP[0], cC[1] - cP[1], cC[2] - cP[2]};
    if ((int)threadIdx.x <= p)
        regular_column_full<R>((R)(dphys[0] / sP), (R)(dphys[1] / sP), (R)(dphys[2] / sP), threadIdx.x, p, Rt);
    for (int t = threadIdx.x; t < (p + 1) * (p + 1); t += blockDim.x) {
        int n = 0;
        while ((n + 1) * (n + 1) <= t)
            ++n;
        int m = t - n * n - n;
        for (int ch = 0; ch < NCH; ++ch)
            Lp[ch][t] = load_full(L + ((int64_t)P * NCH + ch) * ncs, n, m);
    }
    __syncthreads();
    const int nc = ncoef(p);
    for (int idx = threadIdx.x; idx < nc; idx += blockDim.x) {
        int j, kk;
        idx_to_nm(idx, j, kk);
        R sre[NCH], sim[NCH];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
            sre[ch] = sim[ch] = 0;
        for (int n = j; n <= p; ++n) {
            int a = n - j;
            int m0 = max(-n, kk - a), m1 = min(n, kk + a);
            for (int m = m0; m <= m1; ++m) {
                cplx<R> rv = Rt[full_idx(a, m - kk)];  // conj below
                int li = full_idx(n, m);
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) {
                    cplx<R> lv = Lp[ch][li];
                    sre[ch] += lv.re * rv.re + lv.im * rv.im;
                    sim[ch] += lv.im * rv.re - lv.re * rv.im;
                }
            }
        }
        R f = (R)ldexp(1.0, -(j + 1));
        if constexpr (NCH == 4) {
            sre[3] -= (R)dphys[0] * sre[0] + (R)dphys[1] * sre[1] + (R)dphys[2] * sre[2];
            sim[3] -= (R)dphys[0] * sim[0] + (R)dphys[1] * sim[1] + (R)dphys[2] * sim[2];
        }
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            cplx<R> &dst = L[((int64_t)C * NCH + ch) * ncs + idx];
            dst.re += f * sre[ch];
            dst.im += f * sim[ch];
        }
    }
}

// ---------------------------------------------------------------------------
// L2P (a9): one block per leaf, one thread per target.
template <typename R, bool STOKES>
__global__ __launch_bounds__(64) void k_l2p(int p, int ncs, const int32_t *__restrict__ leaves,
                                            const int32_t *__restrict__ box_i, const double *__restrict__ box_r,
                                            double side, int64_t nt, const double *__restrict__ tc,
                                            const float *__restrict__ tc32, const cplx<R> *__restrict__ L,
                                            double *__restrict__ yfar)
{
    constexpr int NCH = STOKES ? 4 : 1;
    constexpr int NV = STOKES ? 3 : 1;        // potentials evaluated
    constexpr int NG = STOKES ? 12 : 0;       // gradients evaluated (channel x direction)
    __shared__ cplx<R> V[NV][NC_MAX];
    __shared__ cplx<R> G[NG > 0 ? NG : 1][STOKES ? NC_MAX : 1];
    const int b = leaves[blockIdx.x];
    const int lv = box_i[6 * b], tb = box_i[6 * b + 1], te = box_i[6 * b + 2];
    const double s = ldexp(side, -(lv + 1));
    const double *c = box_r + 5 * (int64_t)b;
    const int nc = ncoef(p);
    const cplx<R> *Lb = L + (int64_t)b * NCH * ncs;
    for (int t = threadIdx.x; t < nc; t += blockDim.x)
        for (int a = 0; a < NV; ++a)
            V[a][t] = Lb[a * ncs + t];
    if constexpr (STOKES) {
        // gradient expansions (order p-1): dz: L_{j+1}^k; dx: (L_{j+1}^{k-1} - L_{j+1}^{k+1}) / 2;
        // dy: (i/2) (L_{j+1}^{k-1} + L_{j+1}^{k+1})
        const int ncg = ncoef(p - 1);
        for (int t = threadIdx.x; t < ncg; t += blockDim.x) {
            int j, k;
            idx_to_nm(t, j, k);
            for (int ch = 0; ch < 4; ++ch) {
                const cplx<R> *E = Lb + ch * ncs;
                cplx<R> a = load_full(E, j + 1, k - 1), bb = load_full(E, j + 1, k + 1 <= j + 1 ? k + 1 : j + 1);
                if (k + 1 > j + 1)
                    bb = cplx<R>{0, 0};
                cplx<R> cz = load_full(E, j + 1, k);
                G[3 * ch + 0][t] = cplx<R>{R(0.5) * (a.re - bb.re), R(0.5) * (a.im - bb.im)};
                G[3 * ch + 1][t] = cplx<R>{-R(0.5) * (a.im + bb.im), R(0.5) * (a.re + bb.re)};
                G[3 * ch + 2][t] = cz;
            }
        }
    }
    __syncthreads();
    const int64_t ntl = nt;
    for (int i = tb + threadIdx.x; i < te; i += blockDim.x) {
        R x, y, z;
        if constexpr (sizeof(R) == 8) {
            double is = 1.0 / s;
            x = (tc[i] - c[0]) * is;
            y = (tc[ntl + i] - c[1]) * is;
            z = (tc[2 * ntl + i] - c[2]) * is;
        } else {
            float is = (float)(1.0 / s);
            x = tc32[i] * is;
            y = tc32[ntl + i] * is;
            z = tc32[2 * ntl + i] * is;
        }
        const R r2 = x * x + y * y + z * z;
        R pot[NV], grd[NG > 0 ? NG : 1];
#pragma unroll
        for (int a = 0; a < NV; ++a)
            pot[a] = 0;
#pragma unroll
        for (int a = 0; a < (NG > 0 ? NG : 1); ++a)
            grd[a] = 0;
        R dre = 1, dim = 0;  // R_m^m
        for (int m = 0; m <= p; ++m) {
            if (m > 0) {
                R f = -inv_int<R>(2 * m);
                R a = f * (x * dre - y * dim), bb = f * (x * dim + y * dre);
                dre = a;
                dim = bb;
            }
            const R wgt = m == 0 ? R(1) : R(2);
            R cr = dre, ci = dim, pr = 0, pi = 0;
            for (int n = m; n <= p; ++n) {
                if (n > m) {
                    R f = inv_int<R>((n - m) * (n + m));
                    R a = R(2 * n - 1) * z;
                    R nr = (a * cr - r2 * pr) * f, ni = (a * ci - r2 * pi) * f;
                    pr = cr;
                    pi = ci;
                    cr = nr;
                    ci = ni;
                }
                const int id = cidx(n, m);
                const R wr = wgt * cr, wi = wgt * ci;
#pragma unroll
                for (int a = 0; a < NV; ++a)
                    pot[a] += V[a][id].re * wr + V[a][id].im * wi;
                if constexpr (STOKES) {
                    if (n < p) {
#pragma unroll
                        for (int g = 0; g < NG; ++g)
                            grd[g] += G[g][id].re * wr + G[g][id].im * wi;
                    }
                }
            }
        }
        if constexpr (!STOKES) {
            yfar[i] = (double)pot[0] / s;
        } else {
            const double is = 1.0 / s, is2 = is * is;
            const double xr[3] = {(double)x * s, (double)y * s, (double)z * s};  // x - c
            for (int dir = 0; dir < 3; ++dir) {
                double u = (double)pot[dir] * is;
                for (int a = 0; a < 3; ++a)
                    u -= xr[a] * (double)grd[3 * a + dir] * is2;
                u += (double)grd[9 + dir] * is2;
                yfar[3 * (int64_t)i + dir] = u;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// P2P (a10): one block per target leaf, 4 waves splitting the source leaves,
// sources staged in LDS, fixed-order reduction of the 4 partial sums.
template <typename R, bool STOKES>
__global__ __launch_bounds__(256) void k_p2p(const int32_t *__restrict__ leaves, const int32_t *__restrict__ box_i,
                                             const int32_t *__restrict__ ptr, const int32_t *__restrict__ srcs,
                                             const double *__restrict__ box_r, int64_t nt,
                                             const double *__restrict__ tc, const float *__restrict__ tc32,
                                             const double *__restrict__ sp, const float *__restrict__ sp32,
                                             const R *__restrict__ q, double *__restrict__ ynear)
{
    constexpr int NQ = STOKES ? 3 : 1;
    constexpr int TILE = 256;
    __shared__ R sx[4][TILE], sy[4][TILE], sz[4][TILE], sq[4][NQ][TILE];
    __shared__ R red[4][NQ][64];
    const int b = leaves[blockIdx.x];
    const int tb = box_i[6 * b + 1], te = box_i[6 * b + 2];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t ns = 4 * nt;
    const double *cT = box_r + 5 * (int64_t)b;
    for (int t0 = tb; t0 < te; t0 += 64) {
        const int i = t0 + lane;
        const bool active = i < te;
        R tx = 0, ty = 0, tz = 0;
        if (active) {
            if constexpr (sizeof(R) == 8) {
                tx = tc[i];
                ty = tc[nt + i];
                tz = tc[2 * nt + i];
            } else {
                tx = tc32[i];
                ty = tc32[nt + i];
                tz = tc32[2 * nt + i];
            }
        }
        R acc[NQ];
#pragma unroll
        for (int a = 0; a < NQ; ++a)
            acc[a] = 0;
        for (int e = ptr[b] + w; e < ptr[b + 1]; e += 4) {
            const int sb = srcs[e];
            const int s0 = 4 * box_i[6 * sb + 1], s1 = 4 * box_i[6 * sb + 2];
            R ox = 0, oy = 0, oz = 0;  // target offset into the source frame (FP32)
            if constexpr (sizeof(R) == 4) {
                const double *cS = box_r + 5 * (int64_t)sb;
                ox = (float)(cT[0] - cS[0]);
                oy = (float)(cT[1] - cS[1]);
                oz = (float)(cT[2] - cS[2]);
            }
            const R px = tx + ox, py = ty + oy, pz = tz + oz;
            for (int c0 = s0; c0 < s1; c0 += TILE) {
                const int cn = min(TILE, s1 - c0);
                __builtin_amdgcn_wave_barrier();
                for (int k = lane; k < cn; k += 64) {
                    const int64_t sidx = c0 + k;
                    if constexpr (sizeof(R) == 8) {
                        sx[w][k] = sp[sidx];
                        sy[w][k] = sp[ns + sidx];
                        sz[w][k] = sp[2 * ns + sidx];
                    } else {
                        sx[w][k] = sp32[sidx];
                        sy[w][k] = sp32[ns + sidx];
                        sz[w][k] = sp32[2 * ns + sidx];
                    }
#pragma unroll
                    for (int a = 0; a < NQ; ++a)
                        sq[w][a][k] = q[a * ns + sidx];
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (active) {
                    const bool self = sb == b;
                    for (int k = 0; k < cn; ++k) {
                        if (self && ((c0 + k) >> 2) == i)
                            continue;
                        const R dx = px - sx[w][k], dy = py - sy[w][k], dz = pz - sz[w][k];
                        const R r2 = dx * dx + dy * dy + dz * dz;
                        R rinv;
                        if constexpr (sizeof(R) == 8)
                            rinv = rsqrt(r2);
                        else
                            rinv = __builtin_amdgcn_rsqf(r2);
                        if constexpr (!STOKES) {
                            acc[0] += sq[w][0][k] * rinv;
                        } else {
                            const R f0 = sq[w][0][k], f1 = sq[w][1][k], f2 = sq[w][2][k];
                            const R dot = (dx * f0 + dy * f1 + dz * f2) * (rinv * rinv * rinv);
                            acc[0] += f0 * rinv + dx * dot;
                            acc[1] += f1 * rinv + dy * dot;
                            acc[2] += f2 * rinv + dz * dot;
                        }
                    }
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
#pragma unroll
        for (int a = 0; a < NQ; ++a)
            red[w][a][lane] = acc[a];
        __syncthreads();
        if (w == 0 && active) {
#pragma unroll
            for (int a = 0; a < NQ; ++a) {
                double sum = ((double)red[0][a][lane] + (double)red[1][a][lane]) +
                             ((double)red[2][a][lane] + (double)red[3][a][lane]);
                ynear[(int64_t)NQ * i + a] = sum;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// a11 + a12: y[perm i] = pref * (far + near + sum_j S_ij x_j)
template <bool STOKES>
__global__ void k_combine(int64_t nt, const int32_t *__restrict__ perm, const int32_t *__restrict__ cptr,
                          const int32_t *__restrict__ ccol, const double *__restrict__ cval,
                          const double *__restrict__ x, const double *__restrict__ ynear,
                          const double *__restrict__ yfar, double pref, double *__restrict__ y)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nt)
        return;
    const int64_t o = perm[i];
    if (!STOKES) {
        double acc = ynear[i] + yfar[i];
        for (int e = cptr[i]; e < cptr[i + 1]; ++e)
            acc += cval[e] * x[perm[ccol[e]]];
        y[o] = pref * acc;
    } else {
        double a0 = ynear[3 * i] + yfar[3 * i], a1 = ynear[3 * i + 1] + yfar[3 * i + 1],
               a2 = ynear[3 * i + 2] + yfar[3 * i + 2];
        for (int e = cptr[i]; e < cptr[i + 1]; ++e) {
            const int64_t jo = perm[ccol[e]];
            const double *v = cval + 9 * (int64_t)e;
            const double t0 = x[3 * jo], t1 = x[3 * jo + 1], t2 = x[3 * jo + 2];
            a0 += (v[0] * t0 + v[1] * t1) + v[2] * t2;
            a1 += (v[3] * t0 + v[4] * t1) + v[5] * t2;
            a2 += (v[6] * t0 + v[7] * t1) + v[8] * t2;
        }
        y[3 * o] = pref * a0;
        y[3 * o + 1] = pref * a1;
        y[3 * o + 2] = pref * a2;
    }
}

template <typename R, int NCH>
void launch_fmm(fmmbem_ctx *ctx, int p, const double *x, hipStream_t st)
{
    constexpr bool STOKES = NCH == 4;
    Tree &T = ctx->tree;
    Geometry &G = ctx->geo;
    const int64_t nt = ctx->nt, ns = ctx->nsrc;
    const int ncs = ncoef(ctx->prm.p_max);
    const double side = T.cube[3];
    R *q = static_cast<R *>(ctx->charges);
    cplx<R> *M = static_cast<cplx<R> *>(ctx->M);
    cplx<R> *L = static_cast<cplx<R> *>(ctx->L);
    hipEvent_t ev;

    stage_begin(ctx, 4, st, &ev);
    k_charges<R, STOKES><<<grid_for(ns, 256), 256, 0, st>>>(nt, T.perm, T.panel_leaf, T.box_r, G.sp, x, q);
    FB_HIP(hipGetLastError());
    stage_end(ctx, 4, st, ev);

    if (T.n_m2l > 0) {
        stage_begin(ctx, 2, st, &ev);
        k_p2m<R, NCH><<<T.nleaf, 256, 0, st>>>(p, ncs, T.leaves, T.box_i, T.box_r, side, nt, G.sp, G.sp32, q, M);
        FB_HIP(hipGetLastError());
        for (int l = T.nlevels - 2; l >= 0; --l) {
            int b0 = T.level_begin[l], nb = T.level_begin[l + 1] - b0;
            k_m2m<R, NCH><<<nb, 64, 0, st>>>(p, ncs, b0, T.box_i, T.box_r, side, M);
            FB_HIP(hipGetLastError());
        }
        stage_end(ctx, 2, st, ev);

        stage_begin(ctx, 1, st, &ev);
        size_t shm = sizeof(cplx<R>) * ((size_t)(2 * p + 1) * (2 * p + 1) + (size_t)NCH * (p + 1) * (p + 1));
        k_m2l<R, NCH><<<T.nbox, 64, shm, st>>>(p, ncs, T.m2l_ptr, T.m2l_src, T.box_i, T.box_r, side, M, L);
        FB_HIP(hipGetLastError());
        stage_end(ctx, 1, st, ev, 4.0 * (p + 1) * (p + 1) * (p + 1) * (p + 2) * NCH * (double)T.n_m2l);

        stage_begin(ctx, 3, st, &ev);
        for (int l = 1; l < T.nlevels; ++l) {
            int b0 = T.level_begin[l], nb = T.level_begin[l + 1] - b0;
            k_l2l<R, NCH><<<nb, 64, 0, st>>>(p, ncs, b0, T.box_i, T.box_r, side, L);
            FB_HIP(hipGetLastError());
        }
        k_l2p<R, STOKES><<<T.nleaf, 64, 0, st>>>(p, ncs, T.leaves, T.box_i, T.box_r, side, nt, G.tc, G.tc32, L,
                                                 ctx->y_far);
        FB_HIP(hipGetLastError());
        stage_end(ctx, 3, st, ev);
    } else {
        FB_HIP(hipMemsetAsync(ctx->y_far, 0, sizeof(double) * ctx->n, st));
    }

    stage_begin(ctx, 0, st, &ev);
    k_p2p<R, STOKES><<<T.nleaf, 256, 0, st>>>(T.leaves, T.box_i, T.p2p_ptr, T.p2p_src, T.box_r, nt, G.tc, G.tc32,
                                              G.sp, G.sp32, q, ctx->y_near);
    FB_HIP(hipGetLastError());
    // source-target pairs actually evaluated: all P2P pairs minus the 4 self points of each target
    stage_end(ctx, 0, st, ev, (STOKES ? 30.0 : 12.0) * (double)(T.p2p_interactions - 4 * nt));
}

}  // namespace

void run_matvec(fmmbem_ctx *ctx, int p, int prec, const double *x, double *y, hipStream_t st)
{
    const bool stokes = ctx->kernel == FMMBEM_STOKES_SL;
    if (prec == FMMBEM_FP64) {
        if (stokes)
            launch_fmm<double, 4>(ctx, p, x, st);
        else
            launch_fmm<double, 1>(ctx, p, x, st);
    } else {
        if (stokes)
            launch_fmm<float, 4>(ctx, p, x, st);
        else
            launch_fmm<float, 1>(ctx, p, x, st);
    }
    hipEvent_t ev;
    stage_begin(ctx, 4, st, &ev);
    const double pref = stokes ? -1.0 / (8.0 * M_PI * ctx->prm.mu) : 1.0 / (4.0 * M_PI);
    if (stokes)
        k_combine<true><<<grid_for(ctx->nt, 256), 256, 0, st>>>(ctx->nt, ctx->tree.perm, ctx->corr.ptr, ctx->corr.col,
                                                                ctx->corr.val, x, ctx->y_near, ctx->y_far, pref, y);
    else
        k_combine<false><<<grid_for(ctx->nt, 256), 256, 0, st>>>(ctx->nt, ctx->tree.perm, ctx->corr.ptr, ctx->corr.col,
                                                                 ctx->corr.val, x, ctx->y_near, ctx->y_far, pref, y);
    FB_HIP(hipGetLastError());
    stage_end(ctx, 4, st, ev);
}

}  // namespace fmmbem
