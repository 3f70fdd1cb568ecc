// Translation tables for M2L (Sec. 2.5), built once per mesh.
//
// Box centres lie on a grid: a box of level l with integer cell i has centre
// lo + (i + 1/2) side 2^-l.  For an M2L pair (T, S), let l0 be the coarser of
// the two levels, sigma = side 2^-(l0+1) its half-size, eT = lT - l0 and
// eS = lS - l0.  Then (c_T - c_S) / sigma = D 2^-e, e = max(eT, eS), with the
// integer vector D = (2 iT + 1) 2^(e - eT) - (2 iS + 1) 2^(e - eS).  Pairs with
// equal (D, eT, eS) share one scaled M2L operator, so the irregular harmonics
// I_n^m(D 2^-e), n <= 2 p_max, are tabulated once per distinct key (FP64 and
// FP32), and the M2L kernel processes the pairs of one key together.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>
#include <vector>

#include "common.h"
#include "harmonics.h"

namespace fmmbem {

namespace {

__device__ __host__ inline uint32_t gather3(uint64_t x)
{
    x &= 0x1249249249249249ull;
    x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
    x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
    x = (x ^ (x >> 8)) & 0x1f0000ff0000ffull;
    x = (x ^ (x >> 16)) & 0x1f00000000ffffull;
    x = (x ^ (x >> 32)) & 0x1fffffull;
    return (uint32_t)x;
}

constexpr int KEY_BIAS = 1 << 15;

// key = (Dx + 2^15) | (Dy + 2^15) << 16 | (Dz + 2^15) << 32 | eT << 48 | eS << 54
__global__ void k_translation_keys(int64_t n, const int32_t *__restrict__ pairs, const int32_t *__restrict__ box_i,
                                   const uint64_t *__restrict__ keys, uint64_t *__restrict__ tkey,
                                   int32_t *__restrict__ idx, int *__restrict__ overflow)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int T = pairs[2 * i], S = pairs[2 * i + 1];
    const int lT = box_i[6 * T], lS = box_i[6 * S];
    const uint64_t pT = keys[box_i[6 * T + 1]] >> (3 * (21 - lT));
    const uint64_t pS = keys[box_i[6 * S + 1]] >> (3 * (21 - lS));
    const int l0 = min(lT, lS), eT = lT - l0, eS = lS - l0, e = max(eT, eS);
    const int64_t cT[3] = {gather3(pT >> 2), gather3(pT >> 1), gather3(pT)};
    const int64_t cS[3] = {gather3(pS >> 2), gather3(pS >> 1), gather3(pS)};
    uint64_t key = ((uint64_t)eT << 48) | ((uint64_t)eS << 54);
    bool bad = eT > 63 || eS > 63;
    for (int d = 0; d < 3; ++d) {
        int64_t D = (2 * cT[d] + 1) * ((int64_t)1 << (e - eT)) - (2 * cS[d] + 1) * ((int64_t)1 << (e - eS));
        if (D <= -KEY_BIAS || D >= KEY_BIAS)
            bad = true;
        key |= (uint64_t)((D + KEY_BIAS) & 0xffff) << (16 * d);
    }
    if (bad)
        atomicAdd(overflow, 1);
    tkey[i] = key;
    idx[i] = (int32_t)i;
}

__device__ inline int full_index(int n, int m) { return n * n + n + m; }

// One block per distinct translation: thread m computes column m of the
// irregular table (n = m..q) in FP64 and stores FP64 and FP32 copies.
__global__ void k_translation_tables(int nu, const uint64_t *__restrict__ ukey, int q, cplx<double> *__restrict__ t64,
                                     cplx<float> *__restrict__ t32)
{
    const int u = blockIdx.x;
    if (u >= nu)
        return;
    const uint64_t key = ukey[u];
    const int eT = (int)((key >> 48) & 63), eS = (int)((key >> 54) & 63), e = max(eT, eS);
    double v[3];
    for (int d = 0; d < 3; ++d)
        v[d] = ldexp((double)((int64_t)((key >> (16 * d)) & 0xffff) - KEY_BIAS), -e);
    const int fq = (q + 1) * (q + 1);
    cplx<double> *T64 = t64 + (int64_t)u * fq;
    cplx<float> *T32 = t32 + (int64_t)u * fq;
    for (int m = threadIdx.x; m <= q; m += blockDim.x) {
        const double x = v[0], y = v[1], z = v[2];
        const double r2 = x * x + y * y + z * z, ir2 = 1.0 / r2;
        double dre = 1.0 / sqrt(r2), dim = 0.0;
        for (int k = 1; k <= m; ++k) {
            double f = -(2.0 * k - 1.0) * ir2;
            double a = f * (x * dre - y * dim), b = f * (x * dim + y * dre);
            dre = a;
            dim = b;
        }
        double cr = dre, ci = dim, pr = 0.0, pi = 0.0;
        const double sg = (m & 1) ? -1.0 : 1.0;
        for (int n = m; n <= q; ++n) {
            if (n > m) {
                double a = (2.0 * n - 1.0) * z, b = (double)((n - 1) * (n - 1) - m * m);
                double nr = (a * cr - b * pr) * ir2, ni = (a * ci - b * pi) * ir2;
                pr = cr;
                pi = ci;
                cr = nr;
                ci = ni;
            }
            T64[full_index(n, m)] = cplx<double>{cr, ci};
            T32[full_index(n, m)] = cplx<float>{(float)cr, (float)ci};
            if (m > 0) {
                T64[full_index(n, -m)] = cplx<double>{sg * cr, -sg * ci};
                T32[full_index(n, -m)] = cplx<float>{(float)(sg * cr), (float)(-sg * ci)};
            }
        }
    }
}

// per position s of the rotation order (chunk order[s]) and column: the
// column's source box x channels + channel and pair x channels + channel
// ({-1, -1} past the chunk); for Stokes per pair c_S - c_T
__global__ void k_rot_columns(int nchk, int nch, const int32_t *__restrict__ order,
                              const int32_t *__restrict__ chunk_begin, const int32_t *__restrict__ pair_sorted,
                              const int32_t *__restrict__ pairs, const double *__restrict__ box_r,
                              int2 *__restrict__ cols, double *__restrict__ gc)
{
    const int s = blockIdx.x, col = threadIdx.x;
    if (s >= nchk || col >= M2L_CHUNK)
        return;
    const int c = order[s], pb = chunk_begin[c], np = chunk_begin[c + 1] - pb;
    const int pl = col / nch, ch = col - pl * nch;
    int2 v = int2{-1, -1};
    if (pl < np) {
        const int pr = pair_sorted[pb + pl];
        v = int2{pairs[2 * pr + 1] * nch + ch, pr * nch + ch};
        if (gc && ch == 0)
            for (int d = 0; d < 3; ++d)
                gc[((int64_t)s * (M2L_CHUNK / 4) + pl) * 3 + d] =
                    box_r[5 * (int64_t)pairs[2 * pr + 1] + d] - box_r[5 * (int64_t)pairs[2 * pr] + d];
    }
    cols[(int64_t)s * M2L_CHUNK + col] = v;
}

// octant digit of every box (root: 0)
__global__ void k_box_octant(int nbox, const int32_t *__restrict__ box_i, const uint64_t *__restrict__ keys,
                             int8_t *__restrict__ oct)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbox)
        return;
    const int lv = box_i[6 * b];
    oct[b] = lv == 0 ? 0 : (int8_t)((keys[box_i[6 * b + 1]] >> (3 * (21 - lv))) & 7u);
}

// regular tables R_n^m at (+-1/2, +-1/2, +-1/2), one block per octant
__global__ void k_octant_tables(int p, cplx<double> *__restrict__ t64, cplx<float> *__restrict__ t32)
{
    const int o = blockIdx.x;
    const double x = (o & 4) ? 0.5 : -0.5, y = (o & 2) ? 0.5 : -0.5, z = (o & 1) ? 0.5 : -0.5;
    const int fp = (p + 1) * (p + 1);
    for (int m = threadIdx.x; m <= p; m += blockDim.x) {
        const double r2 = x * x + y * y + z * z;
        double dre = 1.0, dim = 0.0;
        for (int k = 1; k <= m; ++k) {
            double f = -1.0 / (2.0 * k);
            double a = f * (x * dre - y * dim), b = f * (x * dim + y * dre);
            dre = a;
            dim = b;
        }
        double cr = dre, ci = dim, pr = 0.0, pi = 0.0;
        const double sg = (m & 1) ? -1.0 : 1.0;
        for (int n = m; n <= p; ++n) {
            if (n > m) {
                double f = 1.0 / (double)((n - m) * (n + m));
                double a = (2.0 * n - 1.0) * z;
                double nr = (a * cr - r2 * pr) * f, ni = (a * ci - r2 * pi) * f;
                pr = cr;
                pi = ci;
                cr = nr;
                ci = ni;
            }
            const int i1 = o * fp + full_index(n, m), i2 = o * fp + full_index(n, -m);
            t64[i1] = cplx<double>{cr, ci};
            t32[i1] = cplx<float>{(float)cr, (float)ci};
            if (m > 0) {
                t64[i2] = cplx<double>{sg * cr, -sg * ci};
                t32[i2] = cplx<float>{(float)(sg * cr), (float)(-sg * ci)};
            }
        }
    }
}

__device__ inline void index_nm(int c, int &n, int &m)
{
    n = (int)((sqrt(8.0 * c + 1.0) - 1.0) * 0.5);
    while ((n + 1) * (n + 2) / 2 <= c)
        ++n;
    while (n * (n + 1) / 2 > c)
        --n;
    m = c - n * (n + 1) / 2;
}

// (a + ib) u with u = 1 (part 0) or i (part 1); conj_u takes conj(u) instead
__device__ inline void add_unit(double a, double b, int part, bool conj_u, double &re, double &im)
{
    if (part == 0) {
        re += a;
        im += b;
    } else if (!conj_u) {
        re -= b;
        im += a;
    } else {
        re += b;
        im -= a;
    }
}

// Entry (output r, input k) of the octant operators, from the same sums as
// the translation theorems: the unit input X = 1 or i in coefficient (j, mu)
// also stands for X_j^-mu = (-1)^mu conj(X), so each entry collects at most
// two terms.
//   M2M: M_n^m(P) = sum_{j <= n} 2^-j sum_mm conj(R_{n-j}^{m-mm}(delta)) M_j^mm(C)
//   L2L: L_j^k(C) = 2^-(j+1) sum_{n >= j} sum_m L_n^m(P) conj(R_{n-j}^{m-k}(delta))
__global__ void k_octant_operators(int pm, int D, const cplx<double> *__restrict__ oct, double *__restrict__ m2m64,
                                   float *__restrict__ m2m32, double *__restrict__ l2l64, float *__restrict__ l2l32)
{
    const int o = blockIdx.y;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)D * D)
        return;
    const int k = (int)(e / D), r = (int)(e - (int64_t)(e / D) * D);
    const int pin = k & 1, pout = r & 1;
    int j, mu, n, m;
    index_nm(k >> 1, j, mu);
    index_nm(r >> 1, n, m);
    const cplx<double> *Rt = oct + (int64_t)o * (pm + 1) * (pm + 1);
    const double smu = (mu & 1) ? -1.0 : 1.0;
    double re = 0.0, im = 0.0;
    if (j <= n) {  // M2M, output (n, m), input (j, mu)
        const int a = n - j;
        const double sc = ldexp(1.0, -j);
        if (abs(m - mu) <= a) {
            const cplx<double> c = Rt[full_index(a, m - mu)];
            add_unit(sc * c.re, -sc * c.im, pin, false, re, im);
        }
        if (mu > 0 && abs(m + mu) <= a) {
            const cplx<double> c = Rt[full_index(a, m + mu)];
            add_unit(smu * sc * c.re, -smu * sc * c.im, pin, true, re, im);
        }
    }
    const int64_t at = (int64_t)o * D * D + e;
    m2m64[at] = pout ? im : re;
    m2m32[at] = (float)(pout ? im : re);
    re = im = 0.0;
    if (j >= n) {  // L2L, output (n, m), input (j, mu)
        const int a = j - n;
        const double f = ldexp(1.0, -(n + 1));
        if (abs(mu - m) <= a) {
            const cplx<double> c = Rt[full_index(a, mu - m)];
            add_unit(f * c.re, -f * c.im, pin, false, re, im);
        }
        if (mu > 0 && abs(mu + m) <= a) {
            const cplx<double> c = Rt[full_index(a, -mu - m)];
            add_unit(smu * f * c.re, -smu * f * c.im, pin, true, re, im);
        }
    }
    l2l64[at] = pout ? im : re;
    l2l32[at] = (float)(pout ? im : re);
}

// Octant operators, per-level tiles and the levels the far field uses.
void build_level_plan(fmmbem_ctx *ctx, hipStream_t st)
{
    Tree &T = ctx->tree;
    M2LPlan &P = ctx->m2l;
    const int pm = ctx->prm.p_max;
    const int D = 2 * ncoef(pm);
    P.op_dim = D;
    const size_t nop = (size_t)8 * D * D;
    P.m2m64 = ctx->arena.alloc<double>(nop);
    P.l2l64 = ctx->arena.alloc<double>(nop);
    P.m2m32 = ctx->arena.alloc<float>(nop);
    P.l2l32 = ctx->arena.alloc<float>(nop);
    {
        dim3 grid((unsigned)(((int64_t)D * D + 255) / 256), 8);
        k_octant_operators<<<grid, 256, 0, st>>>(pm, D, P.oct64, P.m2m64, P.m2m32, P.l2l64, P.l2l32);
        FB_HIP(hipGetLastError());
    }
    P.Z = ctx->arena.alloc<cplx<double>>((size_t)T.nbox * ctx->nch * ncoef(pm));
    std::vector<int8_t> oct(T.nbox);
    FB_HIP(hipMemcpyAsync(oct.data(), P.box_oct, T.nbox, hipMemcpyDeviceToHost, st));
    // coarsest M2L source and target levels
    std::vector<int32_t> ptr(T.nbox + 1), srcs(std::max<int64_t>(T.n_m2l, 1));
    FB_HIP(hipMemcpyAsync(ptr.data(), T.m2l_ptr, sizeof(int32_t) * (T.nbox + 1), hipMemcpyDeviceToHost, st));
    if (T.n_m2l > 0)
        FB_HIP(hipMemcpyAsync(srcs.data(), T.m2l_src, sizeof(int32_t) * T.n_m2l, hipMemcpyDeviceToHost, st));
    FB_HIP(hipStreamSynchronize(st));
    const std::vector<int32_t> &hb = T.h_box_i;
    P.lmin_src = P.lmin_tgt = T.nlevels;
    for (int b = 0; b < T.nbox; ++b)
        if (ptr[b + 1] > ptr[b])
            P.lmin_tgt = std::min(P.lmin_tgt, hb[6 * b]);
    for (int64_t i = 0; i < T.n_m2l; ++i)
        P.lmin_src = std::min(P.lmin_src, hb[6 * srcs[i]]);
    // the M2L sum's order of target boxes: most pairs first, so that the
    // longest blocks do not end the pass (stable: box order among equals)
    {
        std::vector<int32_t> order(T.nbox);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t a, int32_t b) { return ptr[a + 1] - ptr[a] > ptr[b + 1] - ptr[b]; });
        P.reduce_order = ctx->arena.alloc<int32_t>(std::max<size_t>(order.size(), 1));
        if (!order.empty())
            FB_HIP(hipMemcpyAsync(P.reduce_order, order.data(), sizeof(int32_t) * order.size(), hipMemcpyHostToDevice,
                                  st));
        FB_HIP(hipStreamSynchronize(st));  // order is a host vector
    }
    // per leaf, for the fused downward pass: target range, level, the chain of
    // the leaf and its ancestors down to the coarsest M2L target level, and
    // the octant of each chain box in its parent (3 bits each)
    {
        const int lmin = std::max(P.lmin_tgt, 0);
        std::vector<int32_t> rec((size_t)T.nleaf * LEAF_REC, -1);
        for (int li = 0; li < T.nleaf; ++li) {
            int32_t *r = rec.data() + (size_t)li * LEAF_REC;
            int x = T.h_leaves[li], n = 0, octs = 0;
            r[0] = hb[6 * x + 1];
            r[1] = hb[6 * x + 2];
            r[2] = hb[6 * x];
            for (;;) {
                r[4 + n] = x;
                octs |= (int)oct[x] << (3 * n);
                ++n;
                if (n == DOWN_LEAF_MAXC || hb[6 * x] <= lmin)
                    break;
                x = hb[6 * x + 3];
            }
            r[3] = n;
            r[4 + DOWN_LEAF_MAXC] = octs;
        }
        P.leaf_rec = ctx->arena.alloc<int32_t>(std::max<size_t>(rec.size(), 1));
        if (!rec.empty())
            FB_HIP(hipMemcpyAsync(P.leaf_rec, rec.data(), sizeof(int32_t) * rec.size(), hipMemcpyHostToDevice, st));
    }
    const int per_tile = 16 / ctx->nch;
    std::vector<int4> tiles;
    std::vector<int32_t> list, parents;
    P.tile_begin.assign(T.nlevels + 1, 0);
    P.par_begin.assign(T.nlevels + 1, 0);
    for (int l = 0; l < T.nlevels; ++l) {
        P.tile_begin[l] = (int)tiles.size();
        P.par_begin[l] = (int)parents.size();
        const int b0 = T.level_begin[l], b1 = T.level_begin[l + 1];
        for (int b = b0; b < b1; ++b)
            if (hb[6 * b + 5] > 0)
                parents.push_back(b);
        if (l == 0)
            continue;
        for (int o = 0; o < 8; ++o) {
            const int first = (int)list.size();
            for (int b = b0; b < b1; ++b)
                if (oct[b] == o)
                    list.push_back(b);
            for (int e = first; e < (int)list.size(); e += per_tile)
                tiles.push_back(make_int4(o, e, std::min(per_tile, (int)list.size() - e), 0));
        }
    }
    P.tile_begin[T.nlevels] = (int)tiles.size();
    P.par_begin[T.nlevels] = (int)parents.size();
    P.tiles = ctx->arena.alloc<int4>(std::max<size_t>(tiles.size(), 1));
    P.level_list = ctx->arena.alloc<int32_t>(std::max<size_t>(list.size(), 1));
    P.parents = ctx->arena.alloc<int32_t>(std::max<size_t>(parents.size(), 1));
    if (!tiles.empty()) {
        FB_HIP(hipMemcpyAsync(P.tiles, tiles.data(), sizeof(int4) * tiles.size(), hipMemcpyHostToDevice, st));
        FB_HIP(hipMemcpyAsync(P.level_list, list.data(), sizeof(int32_t) * list.size(), hipMemcpyHostToDevice, st));
    }
    if (!parents.empty())
        FB_HIP(hipMemcpyAsync(P.parents, parents.data(), sizeof(int32_t) * parents.size(), hipMemcpyHostToDevice, st));
    FB_HIP(hipStreamSynchronize(st));
}

}  // namespace

void build_translations(fmmbem_ctx *ctx, hipStream_t st)
{
    Tree &T = ctx->tree;
    M2LPlan &P = ctx->m2l;
    const int64_t n = T.n_m2l;
    P.q = 2 * ctx->prm.p_max;
    {
        const int pm = ctx->prm.p_max, fp = (pm + 1) * (pm + 1);
        P.box_oct = ctx->arena.alloc<int8_t>(T.nbox);
        P.oct64 = ctx->arena.alloc<cplx<double>>(8 * fp);
        P.oct32 = ctx->arena.alloc<cplx<float>>(8 * fp);
        k_box_octant<<<grid_for(T.nbox, 256), 256, 0, st>>>(T.nbox, T.box_i, T.keys, P.box_oct);
        FB_HIP(hipGetLastError());
        k_octant_tables<<<8, 64, 0, st>>>(pm, P.oct64, P.oct32);
        FB_HIP(hipGetLastError());
    }
    build_level_plan(ctx, st);
    if (n == 0)
        return;
    DevArena tmp(ctx->arena.al);
    try {
        uint64_t *key = tmp.alloc<uint64_t>(n), *key_sorted = tmp.alloc<uint64_t>(n);
        int32_t *idx = tmp.alloc<int32_t>(n);
        int *ovf = tmp.alloc<int>(1);
        FB_HIP(hipMemsetAsync(ovf, 0, sizeof(int), st));
        P.pair_sorted = ctx->arena.alloc<int32_t>(n);
        k_translation_keys<<<grid_for(n, 256), 256, 0, st>>>(n, T.m2l_pairs, T.box_i, T.keys, key, idx, ovf);
        FB_HIP(hipGetLastError());
        size_t bytes = 0;
        FB_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, key, key_sorted, idx, P.pair_sorted, (int)n, 0, 60,
                                                  st));
        void *t = tmp.alloc<char>(bytes);
        FB_HIP(hipcub::DeviceRadixSort::SortPairs(t, bytes, key, key_sorted, idx, P.pair_sorted, (int)n, 0, 60, st));
        std::vector<uint64_t> hk(n);
        int hovf = 0;
        FB_HIP(hipMemcpyAsync(hk.data(), key_sorted, sizeof(uint64_t) * n, hipMemcpyDeviceToHost, st));
        FB_HIP(hipMemcpyAsync(&hovf, ovf, sizeof(int), hipMemcpyDeviceToHost, st));
        FB_HIP(hipStreamSynchronize(st));
        FB_REQUIRE(hovf == 0, FMMBEM_EINTERNAL, "M2L translation key out of range");
        // distinct keys and chunks of at most M2L_CHUNK / nch pairs with one key
        // (at most 64 columns of pair x channel)
        const int chunk = M2L_CHUNK / ctx->nch;
        std::vector<uint64_t> ukeys;
        std::vector<int32_t> cbeg, cu;
        for (int64_t i = 0; i < n;) {
            int64_t j = i;
            while (j < n && hk[j] == hk[i])
                ++j;
            int u = (int)ukeys.size();
            ukeys.push_back(hk[i]);
            for (int64_t a = i; a < j; a += chunk) {
                cbeg.push_back((int32_t)a);
                cu.push_back(u);
            }
            i = j;
        }
        cbeg.push_back((int32_t)n);
        P.n_trans = (int)ukeys.size();
        P.n_chunks = (int)cu.size();
        P.chunk_begin = ctx->arena.alloc<int32_t>(cbeg.size());
        P.chunk_trans = ctx->arena.alloc<int32_t>(cu.size());
        P.trans_key = ctx->arena.alloc<uint64_t>(ukeys.size());
        FB_HIP(hipMemcpyAsync(P.chunk_begin, cbeg.data(), sizeof(int32_t) * cbeg.size(), hipMemcpyHostToDevice, st));
        FB_HIP(hipMemcpyAsync(P.chunk_trans, cu.data(), sizeof(int32_t) * cu.size(), hipMemcpyHostToDevice, st));
        FB_HIP(hipMemcpyAsync(P.trans_key, ukeys.data(), sizeof(uint64_t) * ukeys.size(), hipMemcpyHostToDevice, st));
        if (ctx->prm.m2l_stored == 2) {
            // directions (integer offsets reduced by their gcd) and distances
            std::map<std::array<int64_t, 3>, int> dir_id;
            std::vector<std::array<int64_t, 3>> dirs;
            std::vector<int32_t> tdir(ukeys.size());
            std::vector<double> tdist(ukeys.size());
            for (size_t u = 0; u < ukeys.size(); ++u) {
                const uint64_t k = ukeys[u];
                const int eT = (int)((k >> 48) & 63), eS = (int)((k >> 54) & 63), e = std::max(eT, eS);
                std::array<int64_t, 3> D;
                for (int d = 0; d < 3; ++d)
                    D[d] = (int64_t)((k >> (16 * d)) & 0xffff) - KEY_BIAS;
                const int64_t g = std::gcd(std::gcd(std::llabs(D[0]), std::llabs(D[1])), std::llabs(D[2]));
                std::array<int64_t, 3> r = {D[0] / g, D[1] / g, D[2] / g};
                auto it = dir_id.find(r);
                if (it == dir_id.end()) {
                    it = dir_id.emplace(r, (int)dirs.size()).first;
                    dirs.push_back(r);
                }
                tdir[u] = it->second;
                const double vx = std::ldexp((double)D[0], -e), vy = std::ldexp((double)D[1], -e),
                             vz = std::ldexp((double)D[2], -e);
                tdist[u] = std::sqrt(vx * vx + vy * vy + vz * vz);
            }
            std::vector<double> fwd, back;
            rotation_tables(dirs, ctx->prm.p_max, fwd, back);
            P.n_dirs = (int)dirs.size();
            P.rot_per = rot_tile_values(ctx->prm.p_max);
            std::vector<float> f32(fwd.begin(), fwd.end()), b32(back.begin(), back.end());
            std::vector<int32_t> order(cu.size());
            std::iota(order.begin(), order.end(), 0);
            std::stable_sort(order.begin(), order.end(),
                             [&](int32_t a, int32_t b) { return tdir[cu[a]] < tdir[cu[b]]; });
            const int nchk = (int)order.size();
            std::vector<int4> hdr(nchk);
            std::vector<double> hdist(nchk);
            for (int s = 0; s < nchk; ++s) {
                const int c = order[s], u = cu[c];
                const uint64_t k = ukeys[u];
                hdr[s] = int4{tdir[u], (int)((k >> 48) & 63) | (int)((k >> 54) & 63) << 8,
                              (cbeg[c + 1] - cbeg[c]) * ctx->nch, 0};
                hdist[s] = tdist[u];
            }
            P.rot_hdr = ctx->arena.alloc<int4>(nchk);
            P.rot_dist = ctx->arena.alloc<double>(nchk);
            P.rot_cols = ctx->arena.alloc<int2>((size_t)nchk * M2L_CHUNK);
            if (ctx->nch == 4)
                P.rot_gc = ctx->arena.alloc<double>((size_t)nchk * 3 * (M2L_CHUNK / 4));
            int32_t *dorder = tmp.alloc<int32_t>(nchk);
            FB_HIP(hipMemcpyAsync(P.rot_hdr, hdr.data(), sizeof(int4) * nchk, hipMemcpyHostToDevice, st));
            FB_HIP(hipMemcpyAsync(P.rot_dist, hdist.data(), sizeof(double) * nchk, hipMemcpyHostToDevice, st));
            FB_HIP(hipMemcpyAsync(dorder, order.data(), sizeof(int32_t) * nchk, hipMemcpyHostToDevice, st));
            k_rot_columns<<<nchk, M2L_CHUNK, 0, st>>>(nchk, ctx->nch, dorder, P.chunk_begin, P.pair_sorted, T.m2l_pairs,
                                                      T.box_r, P.rot_cols, P.rot_gc);
            FB_HIP(hipGetLastError());
            P.rot64_f = ctx->arena.alloc<double>(fwd.size());
            P.rot64_b = ctx->arena.alloc<double>(back.size());
            P.rot32_f = ctx->arena.alloc<float>(f32.size());
            P.rot32_b = ctx->arena.alloc<float>(b32.size());
            P.rot_bytes = (int64_t)(fwd.size() + back.size()) * (8 + 4);
            FB_HIP(hipMemcpyAsync(P.rot64_f, fwd.data(), sizeof(double) * fwd.size(), hipMemcpyHostToDevice, st));
            FB_HIP(hipMemcpyAsync(P.rot64_b, back.data(), sizeof(double) * back.size(), hipMemcpyHostToDevice, st));
            FB_HIP(hipMemcpyAsync(P.rot32_f, f32.data(), sizeof(float) * f32.size(), hipMemcpyHostToDevice, st));
            FB_HIP(hipMemcpyAsync(P.rot32_b, b32.data(), sizeof(float) * b32.size(), hipMemcpyHostToDevice, st));
            FB_HIP(hipStreamSynchronize(st));  // the host vectors go out of scope
        }
        const int64_t fq = (int64_t)(P.q + 1) * (P.q + 1);
        P.table64 = ctx->arena.alloc<cplx<double>>(fq * P.n_trans);
        P.table32 = ctx->arena.alloc<cplx<float>>(fq * P.n_trans);
        k_translation_tables<<<P.n_trans, 64, 0, st>>>(P.n_trans, P.trans_key, P.q, P.table64, P.table32);
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
