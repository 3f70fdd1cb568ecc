// Panel geometry, Morton octree and interaction lists on the device (Sec. 2.5).
//
// This file is compiled with -ffp-contract=off: the octree and lists must be
// reproducible bit for bit, so every floating-point operation below is rounded
// exactly as written (no fused multiply-add) and decisions (cell index,
// acceptance test) see the same values on any conforming implementation.
//
// Contract (the paper fixes only N_CRIT and the MAC theta; the rest is this
// implementation's reading):
//  * centroid c = ((v0 + v1) + v2) / 3, area S = |(v1 - v0) x (v2 - v0)| / 2;
//    Gauss points y = (l0 v0 + l1 v1) + l2 v2 for the 4-point rule with
//    barycentric points (1/3, 1/3, 1/3), (0.6, 0.2, 0.2) and permutations, and
//    weights q_k S_j with q = -27/48, 25/48 (x3).
//  * cube: bounding box of the centroids, side = max extent (1 + 2^-20) about
//    the box midpoint (1 if all centroids coincide); per-axis cell
//    min(floor((c - lo) * (2^21 / side)), 2^21 - 1); 63-bit Morton key with x
//    the most significant bit of each triplet; stable sort by key.
//  * boxes: root holds all panels; a box with more than ncrit panels below
//    level 21 splits into its non-empty octants (octant order); boxes are
//    numbered level by level in parent order.  Centre: centre of the cube
//    cell; radius R: largest distance from the centre to a centroid or Gauss
//    point of its panels; guard G = sqrt(8 max S_j).
//  * dual traversal from (root, root): M2L if (R_A + R_B)^2 < theta^2 d^2 and
//    (R_A + R_B + (1 + 1e-6) G_B)^2 <= d^2 (no near-singular pair of Sec. 2.3
//    can then lie in the pair); else P2P if both are leaves; else split the box
//    with the larger R (target on ties; never a leaf).  Lists sorted by
//    (target, source).
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "common.h"

namespace fmmbem {

namespace {

// outward unit normal of each sorted panel: (v1 - v0) x (v2 - v0), normalised
__global__ void k_normals(int64_t nt, const double *__restrict__ vtx, double *__restrict__ nrm)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nt)
        return;
    const double *v = vtx + 9 * i;
    const double e1[3] = {v[3] - v[0], v[4] - v[1], v[5] - v[2]};
    const double e2[3] = {v[6] - v[0], v[7] - v[1], v[8] - v[2]};
    const double a[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const double na = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    for (int d = 0; d < 3; ++d)
        nrm[d * nt + i] = a[d] / na;
}

__global__ void k_panel_geom(int64_t nt, const double *__restrict__ xyz, const int32_t *__restrict__ tri,
                             double *__restrict__ c, double *__restrict__ S, int *__restrict__ bad)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nt)
        return;
    const double *v0 = xyz + 3 * (int64_t)tri[3 * j];
    const double *v1 = xyz + 3 * (int64_t)tri[3 * j + 1];
    const double *v2 = xyz + 3 * (int64_t)tri[3 * j + 2];
    double e1[3], e2[3];
    for (int d = 0; d < 3; ++d) {
        c[d * nt + j] = ((v0[d] + v1[d]) + v2[d]) / 3.0;
        e1[d] = v1[d] - v0[d];
        e2[d] = v2[d] - v0[d];
    }
    double a0 = e1[1] * e2[2] - e1[2] * e2[1];
    double a1 = e1[2] * e2[0] - e1[0] * e2[2];
    double a2 = e1[0] * e2[1] - e1[1] * e2[0];
    double s = 0.5 * sqrt((a0 * a0 + a1 * a1) + a2 * a2);
    S[j] = s;
    if (!(s > 0.0))
        atomicAdd(bad, 1);
}

// per-block min/max of the centroids; out[block][6] = lo xyz, hi xyz
__global__ void k_bbox_partial(int64_t nt, const double *__restrict__ c, double *__restrict__ out)
{
    __shared__ double sh[6][256];
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = INFINITY;
        hi[d] = -INFINITY;
    }
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nt; j += (int64_t)gridDim.x * blockDim.x)
        for (int d = 0; d < 3; ++d) {
            double v = c[d * nt + j];
            lo[d] = fmin(lo[d], v);
            hi[d] = fmax(hi[d], v);
        }
    for (int d = 0; d < 3; ++d) {
        sh[d][threadIdx.x] = lo[d];
        sh[3 + d][threadIdx.x] = hi[d];
    }
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int d = 0; d < 3; ++d) {
                sh[d][threadIdx.x] = fmin(sh[d][threadIdx.x], sh[d][threadIdx.x + w]);
                sh[3 + d][threadIdx.x] = fmax(sh[3 + d][threadIdx.x], sh[3 + d][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int d = 0; d < 6; ++d)
            out[blockIdx.x * 6 + d] = sh[d][0];
}

__device__ __host__ inline uint64_t spread_bits(uint32_t v)
{
    uint64_t x = v & 0x1fffffu;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__device__ __host__ inline uint32_t gather_bits(uint64_t x)
{
    x &= 0x1249249249249249ull;
    x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
    x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
    x = (x ^ (x >> 8)) & 0x1f0000ff0000ffull;
    x = (x ^ (x >> 16)) & 0x1f00000000ffffull;
    x = (x ^ (x >> 32)) & 0x1fffffull;
    return (uint32_t)x;
}

__global__ void k_morton(int64_t nt, const double *__restrict__ c, double lox, double loy, double loz,
                         double scale, uint64_t *__restrict__ key, int32_t *__restrict__ idx)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nt)
        return;
    const double lo[3] = {lox, loy, loz};
    const uint32_t cmax = (1u << 21) - 1u;
    uint32_t cell[3];
    for (int d = 0; d < 3; ++d) {
        double f = floor((c[d * nt + j] - lo[d]) * scale);
        if (f < 0.0)
            f = 0.0;
        cell[d] = f > (double)cmax ? cmax : (uint32_t)f;
    }
    key[j] = (spread_bits(cell[0]) << 2) | (spread_bits(cell[1]) << 1) | spread_bits(cell[2]);
    idx[j] = (int32_t)j;
}

// gather caller-order geometry into sorted order; build Gauss points
__global__ void k_gather_geom(int64_t nt, const int32_t *__restrict__ perm, const double *__restrict__ xyz,
                              const int32_t *__restrict__ tri, const double *__restrict__ c_in,
                              const double *__restrict__ S_in, double *__restrict__ tc,
                              double *__restrict__ S, double *__restrict__ vtx, double *__restrict__ sp)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nt)
        return;
    int64_t j = perm[i];
    for (int d = 0; d < 3; ++d)
        tc[d * nt + i] = c_in[d * nt + j];
    double s = S_in[j];
    S[i] = s;
    const double *v[3] = {xyz + 3 * (int64_t)tri[3 * j], xyz + 3 * (int64_t)tri[3 * j + 1],
                          xyz + 3 * (int64_t)tri[3 * j + 2]};
    for (int a = 0; a < 3; ++a)
        for (int d = 0; d < 3; ++d)
            vtx[9 * i + 3 * a + d] = v[a][d];
    const double third = 1.0 / 3.0;
    const double L[4][3] = {{third, third, third}, {0.6, 0.2, 0.2}, {0.2, 0.6, 0.2}, {0.2, 0.2, 0.6}};
    const double q[4] = {-27.0 / 48.0, 25.0 / 48.0, 25.0 / 48.0, 25.0 / 48.0};
    int64_t ns = 4 * nt;
    for (int k = 0; k < 4; ++k) {
        int64_t si = 4 * i + k;
        for (int d = 0; d < 3; ++d)
            sp[d * ns + si] = (L[k][0] * v[0][d] + L[k][1] * v[1][d]) + L[k][2] * v[2][d];
        sp[3 * ns + si] = q[k] * s;
    }
}

// For each box of a level: the octant boundaries of its key range.
// bounds[b][0..8]: start of octant d (first position whose digit >= d), bounds[b][8] = end.
__global__ void k_split(int nb, const int32_t *__restrict__ beg, const int32_t *__restrict__ end,
                        const uint64_t *__restrict__ keys, int level, int ncrit, int32_t *__restrict__ bounds,
                        int32_t *__restrict__ nchild)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb)
        return;
    int32_t lo = beg[b], hi = end[b];
    if (hi - lo <= ncrit || level >= 21) {
        nchild[b] = 0;
        return;
    }
    int sh = 3 * (21 - (level + 1));
    int cnt = 0;
    int32_t prev = lo;
    for (int d = 0; d < 8; ++d) {
        // first position in [lo, hi) whose digit >= d
        int32_t a = lo, z = hi;
        while (a < z) {
            int32_t mid = a + (z - a) / 2;
            if ((int)((keys[mid] >> sh) & 7u) < d)
                a = mid + 1;
            else
                z = mid;
        }
        bounds[9 * b + d] = a;
        if (d > 0 && a > prev)
            ++cnt;
        prev = a;
    }
    bounds[9 * b + 8] = hi;
    if (hi > prev)
        ++cnt;
    nchild[b] = cnt;
}

// centre, radius and guard of every box; one block per box
__global__ void k_box_geom(int nbox, const int32_t *__restrict__ box_i, const uint64_t *__restrict__ keys,
                           const int32_t *__restrict__ perm_unused, const double *__restrict__ tc,
                           const double *__restrict__ S, const double *__restrict__ sp, int64_t nt,
                           double lox, double loy, double loz, double side, double *__restrict__ box_r)
{
    __shared__ double r2s[256], ss[256];
    int b = blockIdx.x;
    int lv = box_i[6 * b], lo = box_i[6 * b + 1], hi = box_i[6 * b + 2];
    uint64_t pre = keys[lo] >> (3 * (21 - lv));
    uint32_t ix = gather_bits(pre >> 2), iy = gather_bits(pre >> 1), iz = gather_bits(pre);
    double h = ldexp(side, -lv);
    double ctr[3] = {lox + ((double)ix + 0.5) * h, loy + ((double)iy + 0.5) * h, loz + ((double)iz + 0.5) * h};
    double r2max = 0.0, smax = 0.0;
    int64_t ns = 4 * nt;
    for (int p = lo + threadIdx.x; p < hi; p += blockDim.x) {
        {
            double dx = tc[p] - ctr[0], dy = tc[nt + p] - ctr[1], dz = tc[2 * nt + p] - ctr[2];
            double r2 = (dx * dx + dy * dy) + dz * dz;
            r2max = r2 > r2max ? r2 : r2max;
        }
        for (int k = 0; k < 4; ++k) {
            int64_t si = 4 * (int64_t)p + k;
            double dx = sp[si] - ctr[0], dy = sp[ns + si] - ctr[1], dz = sp[2 * ns + si] - ctr[2];
            double r2 = (dx * dx + dy * dy) + dz * dz;
            r2max = r2 > r2max ? r2 : r2max;
        }
        smax = S[p] > smax ? S[p] : smax;
    }
    r2s[threadIdx.x] = r2max;
    ss[threadIdx.x] = smax;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            r2s[threadIdx.x] = fmax(r2s[threadIdx.x], r2s[threadIdx.x + w]);
            ss[threadIdx.x] = fmax(ss[threadIdx.x], ss[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double *o = box_r + 5 * (int64_t)b;
        o[0] = ctr[0];
        o[1] = ctr[1];
        o[2] = ctr[2];
        o[3] = sqrt(r2s[0]);
        o[4] = sqrt(8.0 * ss[0]);
    }
}

// action of a frontier pair: 0 M2L, 1 P2P, 2 split target, 3 split source
__global__ void k_traverse_count(int64_t nf, const int2 *__restrict__ front, const int32_t *__restrict__ box_i,
                                 const double *__restrict__ box_r, double th2, int32_t *__restrict__ act,
                                 int32_t *__restrict__ n_m2l, int32_t *__restrict__ n_p2p,
                                 int32_t *__restrict__ n_new)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nf)
        return;
    int A = front[i].x, B = front[i].y;
    const double *ra = box_r + 5 * (int64_t)A, *rb = box_r + 5 * (int64_t)B;
    double dx = ra[0] - rb[0], dy = ra[1] - rb[1], dz = ra[2] - rb[2];
    double d2 = (dx * dx + dy * dy) + dz * dz;
    double s = ra[3] + rb[3];
    double g = s + rb[4] * (1.0 + 1e-6);
    int a, m = 0, q = 0, nn = 0;
    if (s * s < th2 * d2 && g * g <= d2) {
        a = 0;
        m = 1;
    } else {
        bool leafA = box_i[6 * (int64_t)A + 5] == 0, leafB = box_i[6 * (int64_t)B + 5] == 0;
        if (leafA && leafB) {
            a = 1;
            q = 1;
        } else if (!leafA && (leafB || ra[3] >= rb[3])) {
            a = 2;
            nn = box_i[6 * (int64_t)A + 5];
        } else {
            a = 3;
            nn = box_i[6 * (int64_t)B + 5];
        }
    }
    act[i] = a;
    n_m2l[i] = m;
    n_p2p[i] = q;
    n_new[i] = nn;
}

__global__ void k_traverse_emit(int64_t nf, const int2 *__restrict__ front, const int32_t *__restrict__ box_i,
                                const int32_t *__restrict__ act, const int32_t *__restrict__ o_m2l,
                                const int32_t *__restrict__ o_p2p, const int32_t *__restrict__ o_new,
                                uint64_t *__restrict__ m2l, int64_t m2l_base, uint64_t *__restrict__ p2p,
                                int64_t p2p_base, int2 *__restrict__ next)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nf)
        return;
    int A = front[i].x, B = front[i].y;
    int a = act[i];
    uint64_t key = ((uint64_t)(uint32_t)A << 32) | (uint32_t)B;
    if (a == 0) {
        m2l[m2l_base + o_m2l[i]] = key;
    } else if (a == 1) {
        p2p[p2p_base + o_p2p[i]] = key;
    } else if (a == 2) {
        int c0 = box_i[6 * (int64_t)A + 4], nc = box_i[6 * (int64_t)A + 5];
        for (int k = 0; k < nc; ++k)
            next[o_new[i] + k] = make_int2(c0 + k, B);
    } else {
        int c0 = box_i[6 * (int64_t)B + 4], nc = box_i[6 * (int64_t)B + 5];
        for (int k = 0; k < nc; ++k)
            next[o_new[i] + k] = make_int2(A, c0 + k);
    }
}

// CSR row pointers over boxes from sorted (target << 32 | source) keys
__global__ void k_csr_ptr(int nbox, const uint64_t *__restrict__ keys, int64_t n, int32_t *__restrict__ ptr,
                          int32_t *__restrict__ src, int32_t *__restrict__ pairs)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t <= nbox) {
        uint64_t want = (uint64_t)t << 32;
        int64_t a = 0, z = n;
        while (a < z) {
            int64_t mid = a + (z - a) / 2;
            if (keys[mid] < want)
                a = mid + 1;
            else
                z = mid;
        }
        ptr[t] = (int32_t)a;
    }
    if (t < n) {
        uint64_t k = keys[t];
        src[t] = (int32_t)(uint32_t)(k & 0xffffffffu);
        pairs[2 * t] = (int32_t)(k >> 32);
        pairs[2 * t + 1] = (int32_t)(uint32_t)(k & 0xffffffffu);
    }
}

__global__ void k_panel_leaf(int nleaf, const int32_t *__restrict__ leaves, const int32_t *__restrict__ box_i,
                             int32_t *__restrict__ panel_leaf)
{
    int l = blockIdx.x;
    if (l >= nleaf)
        return;
    int b = leaves[l];
    int lo = box_i[6 * b + 1], hi = box_i[6 * b + 2];
    for (int p = lo + threadIdx.x; p < hi; p += blockDim.x)
        panel_leaf[p] = b;
}

// FP32 leaf-relative coordinates of targets and sources
__global__ void k_relative(int64_t nt, const int32_t *__restrict__ panel_leaf, const double *__restrict__ box_r,
                           const double *__restrict__ tc, const double *__restrict__ sp, float *__restrict__ tc32,
                           float *__restrict__ sp32)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nt)
        return;
    const double *c = box_r + 5 * (int64_t)panel_leaf[i];
    for (int d = 0; d < 3; ++d)
        tc32[d * nt + i] = (float)(tc[d * nt + i] - c[d]);
    int64_t ns = 4 * nt;
    for (int k = 0; k < 4; ++k) {
        int64_t s = 4 * i + k;
        for (int d = 0; d < 3; ++d)
            sp32[d * ns + s] = (float)(sp[d * ns + s] - c[d]);
        sp32[3 * ns + s] = (float)sp[3 * ns + s];
    }
}

template <typename T> void exclusive_scan(const T *in, T *out, int64_t n, hipStream_t st, DevArena &tmp_arena)
{
    size_t bytes = 0;
    FB_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, in, out, (int)n, st));
    void *tmp = tmp_arena.alloc<char>(bytes);
    FB_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, bytes, in, out, (int)n, st));
}

// P2P work units.  A leaf's targets are cut into units of at most 64 (one
// per lane when the wave runs one phase).  A unit of n targets runs
// P = floor(64 / n) phases, so it costs the waves about S / P steps for S
// sources: a leaf of 33 to 53 targets left whole costs S (a third to half of
// the lanes idle), cut into 32 + the rest it costs S / 2 + S / floor(64 /
// rest) <= 0.83 S, and that cut is made (from 54 on it would save less than
// the second pass over the sources costs) unless the near field is stored
// (its product takes one lane per target and gains nothing from phases).
// Its sources are the leaf's P2P source leaves cut
// into chunks of at most floor(P2P_TILE / P) P consecutive sources, so that a
// chunk padded to a multiple of P still fits one tile.  The chunks are sorted
// by decreasing size so that dealing them round robin to the waves of a block
// balances the waves.  The FP32 offset of a chunk
// is the difference of the two leaf centres, rounded once from FP64.
// Launch order of the on-the-fly P2P (the units as built are in Morton
// order).  A unit's work is its wave steps, sum over its chunks of
// ceil(count / P).  Blocks are dealt to the XCDs round robin and a unit runs
// as one block of P2P_WAVES waves, so a unit with a large share of the work
// (a dense cluster of panels) ends long after the others and leaves its XCD
// idle: units above 1/1024 of the total are cut into pieces of about that
// work (contiguous chunk ranges; each writes a partial slot), the units are
// split into 8 consecutive groups of equal work, one per XCD (consecutive,
// so that a group's units share source leaves in its L2), and within a group
// the heaviest come first, so the light ones fill the end.
void schedule_p2p(std::vector<int4> &units, const std::vector<int2> &chunks, std::vector<int32_t> &dst,
                  std::vector<int4> &splits, XcdGroups &xg)
{
    auto steps = [&](int c, int P) { return (int64_t)((chunks[c].y & 0xffff) + P - 1) / P; };
    std::vector<int64_t> work(units.size(), 0);
    int64_t total = 0;
    for (size_t i = 0; i < units.size(); ++i) {
        const int P = 64 / (units[i].y - units[i].x);
        for (int c = units[i].z; c < units[i].w; ++c)
            work[i] += steps(c, P);
        total += work[i];
    }
    const int64_t cap = std::max<int64_t>(1, (total + 1023) / 1024);
    struct Item { int4 u; int32_t dst; int64_t work; };
    std::vector<Item> items;
    items.reserve(units.size() + 64);
    int32_t slot = 0;
    for (size_t i = 0; i < units.size(); ++i) {
        const int4 u = units[i];
        const int nch = u.w - u.z;
        const int64_t k = std::min<int64_t>(nch, (work[i] + cap - 1) / cap);
        if (k <= 1) {
            items.push_back({u, -1, work[i]});
            continue;
        }
        const int P = 64 / (u.y - u.x);
        splits.push_back(make_int4(u.x, u.y - u.x, slot, (int)k));
        int c = u.z;
        int64_t acc = 0;
        for (int64_t j = 0; j < k; ++j) {
            const int c0 = c;
            int64_t wj = 0;
            // at least one chunk per piece and enough left for the rest
            while (c < u.w - (k - 1 - j) && (c == c0 || acc + steps(c, P) <= (j + 1) * work[i] / k)) {
                acc += steps(c, P);
                wj += steps(c, P);
                ++c;
            }
            if (j == k - 1)
                while (c < u.w) {
                    wj += steps(c, P);
                    ++c;
                }
            items.push_back({make_int4(u.x, u.y, c0, c), slot++, wj});
        }
    }
    // 8 consecutive groups of equal work, heaviest first within each
    std::vector<int> grp(items.size());
    int64_t pre = 0;
    for (size_t i = 0; i < items.size(); ++i) {
        const int64_t mid = 2 * pre + items[i].work;  // twice the item's midpoint
        grp[i] = (int)std::min<int64_t>(7, total > 0 ? (8 * mid) / (2 * total) : 0);
        pre += items[i].work;
    }
    std::vector<int> order(items.size());
    for (size_t i = 0; i < items.size(); ++i)
        order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return grp[a] != grp[b] ? grp[a] < grp[b] : items[a].work > items[b].work;
    });
    units.resize(items.size());
    dst.assign(items.size(), -1);
    for (int x = 0; x <= 8; ++x)
        xg.b[x] = 0;
    for (size_t i = 0; i < order.size(); ++i) {
        units[i] = items[order[i]].u;
        dst[i] = items[order[i]].dst;
        xg.b[grp[order[i]] + 1]++;
    }
    for (int x = 0; x < 8; ++x)
        xg.b[x + 1] += xg.b[x];
}

void build_p2p_units(fmmbem_ctx *ctx, const std::vector<int32_t> &hp, int64_t n_p2p, hipStream_t st)
{
    Tree &T = ctx->tree;
    const std::vector<int32_t> &hb = T.h_box_i;
    const std::vector<double> &hr = T.h_box_r;
    std::vector<int> leaves = T.h_leaves;
    std::sort(leaves.begin(), leaves.end(), [&](int a, int b) { return hb[6 * a + 1] < hb[6 * b + 1]; });
    // per-leaf source lists (hp is sorted by target)
    std::vector<int64_t> first(T.nbox + 1, 0);
    for (int64_t i = 0; i < n_p2p; ++i)
        first[hp[2 * i] + 1]++;
    for (int b = 0; b < T.nbox; ++b)
        first[b + 1] += first[b];
    std::vector<int4> units;
    std::vector<int2> chunks;
    std::vector<float4> offs;
    struct Piece { int32_t begin, count, self, leaf; };
    std::vector<Piece> pieces;
    const bool split = ctx->prm.near_stored == 0;
    for (int t : leaves) {
        const int tb = hb[6 * t + 1], te = hb[6 * t + 2];
        for (int u0 = tb, nu = 0; u0 < te; u0 += nu) {
            const int rest = te - u0;
            nu = rest >= 64 ? 64 : (split && rest > 32 && rest <= 53) ? 32 : rest;
            const int cap = (P2P_TILE / (64 / nu)) * (64 / nu);  // a multiple of the unit's phase count
            pieces.clear();
            for (int64_t e = first[t]; e < first[t + 1]; ++e) {
                const int s = hp[2 * e + 1];
                const int32_t k0 = 4 * hb[6 * s + 1], k1 = 4 * hb[6 * s + 2];
                for (int32_t k = k0; k < k1; k += cap)
                    pieces.push_back({k, std::min(cap, k1 - k), s == t ? 1 : 0, s});
            }
            std::stable_sort(pieces.begin(), pieces.end(),
                             [](const Piece &a, const Piece &b) { return a.count > b.count; });
            const int32_t c0 = (int32_t)chunks.size();
            for (const Piece &pc : pieces) {
                chunks.push_back(make_int2(pc.begin, pc.count | (pc.self << 16)));
                offs.push_back(make_float4((float)(hr[5 * t] - hr[5 * pc.leaf]),
                                           (float)(hr[5 * t + 1] - hr[5 * pc.leaf + 1]),
                                           (float)(hr[5 * t + 2] - hr[5 * pc.leaf + 2]), 0.0f));
            }
            FB_REQUIRE(chunks.size() < ((size_t)1 << 31), FMMBEM_ENOMEM, "P2P chunk list exceeds 2^31 entries");
            units.push_back(make_int4(u0, u0 + nu, c0, (int32_t)chunks.size()));
        }
    }
    std::vector<int32_t> dst(units.size(), -1);
    std::vector<int4> splits;
    if (split)
        schedule_p2p(units, chunks, dst, splits, T.p2p_xcd);
    else
        for (int x = 0; x <= 8; ++x)  // consecutive groups of equal count
            T.p2p_xcd.b[x] = (int32_t)std::min<size_t>(units.size(), x * ((units.size() + 7) / 8));
    T.n_unit = (int32_t)units.size();
    T.n_chunk = (int64_t)chunks.size();
    T.n_split = (int32_t)splits.size();
    T.n_slot = 0;
    for (const int4 &r : splits)
        T.n_slot += r.w;
    DevArena &A = ctx->arena;
    T.p2p_unit = A.alloc<int4>(std::max<size_t>(units.size(), 1));
    T.p2p_chunk = A.alloc<int2>(std::max<size_t>(chunks.size(), 1));
    T.p2p_choff = A.alloc<float4>(std::max<size_t>(offs.size(), 1));
    T.p2p_dst = A.alloc<int32_t>(std::max<size_t>(dst.size(), 1));
    T.p2p_split = A.alloc<int4>(std::max<size_t>(splits.size(), 1));
    T.p2p_part = A.alloc<double>((size_t)std::max(T.n_slot, 1) * 3 * 64);
    if (!units.empty()) {
        FB_HIP(hipMemcpyAsync(T.p2p_unit, units.data(), sizeof(int4) * units.size(), hipMemcpyHostToDevice, st));
        FB_HIP(hipMemcpyAsync(T.p2p_dst, dst.data(), sizeof(int32_t) * dst.size(), hipMemcpyHostToDevice, st));
    }
    if (!splits.empty())
        FB_HIP(hipMemcpyAsync(T.p2p_split, splits.data(), sizeof(int4) * splits.size(), hipMemcpyHostToDevice, st));
    if (!chunks.empty()) {
        FB_HIP(hipMemcpyAsync(T.p2p_chunk, chunks.data(), sizeof(int2) * chunks.size(), hipMemcpyHostToDevice, st));
        FB_HIP(hipMemcpyAsync(T.p2p_choff, offs.data(), sizeof(float4) * offs.size(), hipMemcpyHostToDevice, st));
    }
    FB_HIP(hipStreamSynchronize(st));  // host vectors go out of scope
}

}  // namespace

void build_geometry_and_tree(fmmbem_ctx *ctx, const fmmbem_mesh *mesh, hipStream_t st)
{
    const int64_t nt = mesh->n_triangles, nv = mesh->n_vertices;
    const int ncrit = ctx->prm.ncrit;
    Tree &T = ctx->tree;
    Geometry &G = ctx->geo;
    DevArena &A = ctx->arena;
    DevArena tmp(ctx->arena.al);  // build-time scratch
    try {
        T.nt = nt;
        // ---- upload mesh, caller-order geometry
        double *d_xyz = tmp.alloc<double>(3 * nv);
        int32_t *d_tri = tmp.alloc<int32_t>(3 * nt);
        FB_HIP(hipMemcpyAsync(d_xyz, mesh->xyz, sizeof(double) * 3 * nv, hipMemcpyHostToDevice, st));
        FB_HIP(hipMemcpyAsync(d_tri, mesh->tri, sizeof(int32_t) * 3 * nt, hipMemcpyHostToDevice, st));
        double *c0 = tmp.alloc<double>(3 * nt);
        double *S0 = tmp.alloc<double>(nt);
        int *d_bad = tmp.alloc<int>(1);
        FB_HIP(hipMemsetAsync(d_bad, 0, sizeof(int), st));
        k_panel_geom<<<grid_for(nt, 256), 256, 0, st>>>(nt, d_xyz, d_tri, c0, S0, d_bad);
        FB_HIP(hipGetLastError());
        const int nblk = (int)std::min<int64_t>(256, grid_for(nt, 256));
        double *d_part = tmp.alloc<double>(6 * nblk);
        k_bbox_partial<<<nblk, 256, 0, st>>>(nt, c0, d_part);
        FB_HIP(hipGetLastError());
        std::vector<double> part(6 * nblk);
        int bad = 0;
        FB_HIP(hipMemcpyAsync(part.data(), d_part, sizeof(double) * 6 * nblk, hipMemcpyDeviceToHost, st));
        FB_HIP(hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, st));
        FB_HIP(hipStreamSynchronize(st));
        FB_REQUIRE(bad == 0, FMMBEM_EINVAL, std::to_string(bad) + " triangle(s) with zero area");
        double lo[3], hi[3];
        for (int d = 0; d < 3; ++d) {
            lo[d] = part[d];
            hi[d] = part[3 + d];
            for (int b = 1; b < nblk; ++b) {
                lo[d] = std::min(lo[d], part[6 * b + d]);
                hi[d] = std::max(hi[d], part[6 * b + 3 + d]);
            }
        }
        double ext = 0.0;
        for (int d = 0; d < 3; ++d) {
            double e = hi[d] - lo[d];
            if (e > ext)
                ext = e;
        }
        double side = ext > 0.0 ? ext * (1.0 + std::ldexp(1.0, -20)) : 1.0;
        double clo[3];
        for (int d = 0; d < 3; ++d)
            clo[d] = (lo[d] + hi[d]) * 0.5 - side * 0.5;
        double scale = std::ldexp(1.0, 21) / side;
        for (int d = 0; d < 3; ++d)
            T.cube[d] = clo[d];
        T.cube[3] = side;

        // ---- Morton keys, stable radix sort
        uint64_t *k_in = tmp.alloc<uint64_t>(nt);
        int32_t *i_in = tmp.alloc<int32_t>(nt);
        T.keys = A.alloc<uint64_t>(nt);
        T.perm = A.alloc<int32_t>(nt);
        k_morton<<<grid_for(nt, 256), 256, 0, st>>>(nt, c0, clo[0], clo[1], clo[2], scale, k_in, i_in);
        FB_HIP(hipGetLastError());
        {
            size_t bytes = 0;
            FB_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, k_in, T.keys, i_in, T.perm, (int)nt, 0, 63, st));
            void *t = tmp.alloc<char>(bytes);
            FB_HIP(hipcub::DeviceRadixSort::SortPairs(t, bytes, k_in, T.keys, i_in, T.perm, (int)nt, 0, 63, st));
        }
        // ---- sorted geometry and Gauss points
        const int64_t ns = 4 * nt;
        G.tc = A.alloc<double>(3 * nt);
        G.S = A.alloc<double>(nt);
        G.vtx = A.alloc<double>(9 * nt);
        G.sp = A.alloc<double>(4 * ns);
        k_gather_geom<<<grid_for(nt, 256), 256, 0, st>>>(nt, T.perm, d_xyz, d_tri, c0, S0, G.tc, G.S, G.vtx, G.sp);
        FB_HIP(hipGetLastError());
        G.nrm = A.alloc<double>(3 * nt);
        k_normals<<<grid_for(nt, 256), 256, 0, st>>>(nt, G.vtx, G.nrm);
        FB_HIP(hipGetLastError());

        // ---- boxes level by level (octant search on the device, records on the host)
        std::vector<int32_t> hb;  // [nbox][6]
        hb.insert(hb.end(), {0, 0, (int32_t)nt, -1, -1, 0});
        T.level_begin.assign(1, 0);
        int32_t *d_beg = tmp.alloc<int32_t>(nt + 1), *d_end = tmp.alloc<int32_t>(nt + 1);
        int32_t *d_bounds = tmp.alloc<int32_t>(9 * (nt + 1)), *d_nch = tmp.alloc<int32_t>(nt + 1);
        int level = 0;
        while (true) {
            int lb = T.level_begin.back();
            int le = (int)(hb.size() / 6);
            int nb = le - lb;
            if (nb == 0)
                break;
            T.level_begin.push_back(le);
            std::vector<int32_t> beg(nb), end(nb);
            for (int b = 0; b < nb; ++b) {
                beg[b] = hb[6 * (lb + b) + 1];
                end[b] = hb[6 * (lb + b) + 2];
            }
            FB_HIP(hipMemcpyAsync(d_beg, beg.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice, st));
            FB_HIP(hipMemcpyAsync(d_end, end.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice, st));
            k_split<<<grid_for(nb, 128), 128, 0, st>>>(nb, d_beg, d_end, T.keys, level, ncrit, d_bounds, d_nch);
            FB_HIP(hipGetLastError());
            std::vector<int32_t> bounds(9 * nb), nch(nb);
            FB_HIP(hipMemcpyAsync(bounds.data(), d_bounds, sizeof(int32_t) * 9 * nb, hipMemcpyDeviceToHost, st));
            FB_HIP(hipMemcpyAsync(nch.data(), d_nch, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, st));
            FB_HIP(hipStreamSynchronize(st));
            for (int b = 0; b < nb; ++b) {
                if (nch[b] == 0)
                    continue;
                int parent = lb + b;
                hb[6 * parent + 4] = (int32_t)(hb.size() / 6);
                hb[6 * parent + 5] = nch[b];
                for (int d = 0; d < 8; ++d) {
                    int32_t a = bounds[9 * b + d], z = bounds[9 * b + d + 1];
                    if (z > a)
                        hb.insert(hb.end(), {level + 1, a, z, parent, -1, 0});
                }
            }
            ++level;
        }
        T.nbox = (int32_t)(hb.size() / 6);
        T.nlevels = level;
        T.h_box_i = hb;
        T.box_i = A.alloc<int32_t>(hb.size());
        FB_HIP(hipMemcpyAsync(T.box_i, hb.data(), sizeof(int32_t) * hb.size(), hipMemcpyHostToDevice, st));
        T.box_r = A.alloc<double>(5 * (int64_t)T.nbox);
        k_box_geom<<<T.nbox, 256, 0, st>>>(T.nbox, T.box_i, T.keys, T.perm, G.tc, G.S, G.sp, nt, clo[0], clo[1],
                                          clo[2], side, T.box_r);
        FB_HIP(hipGetLastError());
        T.h_leaves.clear();
        T.max_leaf = 0;
        for (int b = 0; b < T.nbox; ++b)
            if (hb[6 * b + 5] == 0) {
                T.h_leaves.push_back(b);
                T.max_leaf = std::max(T.max_leaf, hb[6 * b + 2] - hb[6 * b + 1]);
            }
        T.nleaf = (int32_t)T.h_leaves.size();
        T.leaves = A.alloc<int32_t>(T.nleaf);
        FB_HIP(hipMemcpyAsync(T.leaves, T.h_leaves.data(), sizeof(int32_t) * T.nleaf, hipMemcpyHostToDevice, st));
        T.panel_leaf = A.alloc<int32_t>(nt);
        k_panel_leaf<<<T.nleaf, 64, 0, st>>>(T.nleaf, T.leaves, T.box_i, T.panel_leaf);
        FB_HIP(hipGetLastError());

        // ---- dual traversal, level-synchronous frontier
        const double th2 = ctx->prm.theta * ctx->prm.theta;
        int64_t cap_front = std::max<int64_t>(1024, 8 * (int64_t)T.nbox);
        int2 *front = tmp.alloc<int2>(cap_front), *next = nullptr;
        int64_t cap_m2l = std::max<int64_t>(1024, 64 * (int64_t)T.nbox), cap_p2p = std::max<int64_t>(1024, 32 * (int64_t)T.nleaf);
        uint64_t *m2l = tmp.alloc<uint64_t>(cap_m2l), *p2p = tmp.alloc<uint64_t>(cap_p2p);
        int64_t n_m2l = 0, n_p2p = 0, nf = 1;
        int2 root = make_int2(0, 0);
        FB_HIP(hipMemcpyAsync(front, &root, sizeof(int2), hipMemcpyHostToDevice, st));
        while (nf > 0) {
            int32_t *act = tmp.alloc<int32_t>(nf), *cm = tmp.alloc<int32_t>(nf + 1), *cp = tmp.alloc<int32_t>(nf + 1),
                    *cn = tmp.alloc<int32_t>(nf + 1);
            int32_t *om = tmp.alloc<int32_t>(nf + 1), *op = tmp.alloc<int32_t>(nf + 1), *on = tmp.alloc<int32_t>(nf + 1);
            k_traverse_count<<<grid_for(nf, 256), 256, 0, st>>>(nf, front, T.box_i, T.box_r, th2, act, cm, cp, cn);
            FB_HIP(hipGetLastError());
            exclusive_scan(cm, om, nf, st, tmp);
            exclusive_scan(cp, op, nf, st, tmp);
            exclusive_scan(cn, on, nf, st, tmp);
            int32_t last[6];
            FB_HIP(hipMemcpyAsync(&last[0], om + nf - 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            FB_HIP(hipMemcpyAsync(&last[1], cm + nf - 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            FB_HIP(hipMemcpyAsync(&last[2], op + nf - 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            FB_HIP(hipMemcpyAsync(&last[3], cp + nf - 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            FB_HIP(hipMemcpyAsync(&last[4], on + nf - 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            FB_HIP(hipMemcpyAsync(&last[5], cn + nf - 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            FB_HIP(hipStreamSynchronize(st));
            int64_t add_m = last[0] + last[1], add_p = last[2] + last[3], n_next = last[4] + last[5];
            if (n_m2l + add_m > cap_m2l) {
                int64_t nc = std::max(2 * cap_m2l, n_m2l + add_m);
                uint64_t *nb2 = tmp.alloc<uint64_t>(nc);
                FB_HIP(hipMemcpyAsync(nb2, m2l, sizeof(uint64_t) * n_m2l, hipMemcpyDeviceToDevice, st));
                m2l = nb2;
                cap_m2l = nc;
            }
            if (n_p2p + add_p > cap_p2p) {
                int64_t nc = std::max(2 * cap_p2p, n_p2p + add_p);
                uint64_t *nb2 = tmp.alloc<uint64_t>(nc);
                FB_HIP(hipMemcpyAsync(nb2, p2p, sizeof(uint64_t) * n_p2p, hipMemcpyDeviceToDevice, st));
                p2p = nb2;
                cap_p2p = nc;
            }
            next = tmp.alloc<int2>(std::max<int64_t>(1, n_next));
            k_traverse_emit<<<grid_for(nf, 256), 256, 0, st>>>(nf, front, T.box_i, act, om, op, on, m2l, n_m2l, p2p,
                                                               n_p2p, next);
            FB_HIP(hipGetLastError());
            n_m2l += add_m;
            n_p2p += add_p;
            front = next;
            nf = n_next;
            FB_REQUIRE(n_m2l < ((int64_t)1 << 31) && n_p2p < ((int64_t)1 << 31), FMMBEM_ENOMEM,
                       "interaction lists exceed 2^31 pairs");
        }
        T.n_m2l = n_m2l;
        T.n_p2p = n_p2p;
        // sort lists by (target, source) and build CSR
        auto finish_list = [&](uint64_t *keys_in, int64_t n, int32_t *&ptr, int32_t *&src, int32_t *&pairs) {
            uint64_t *sorted = tmp.alloc<uint64_t>(std::max<int64_t>(n, 1));
            if (n > 0) {
                size_t bytes = 0;
                FB_HIP(hipcub::DeviceRadixSort::SortKeys(nullptr, bytes, keys_in, sorted, (int)n, 0, 64, st));
                void *t = tmp.alloc<char>(bytes);
                FB_HIP(hipcub::DeviceRadixSort::SortKeys(t, bytes, keys_in, sorted, (int)n, 0, 64, st));
            }
            ptr = A.alloc<int32_t>(T.nbox + 1);
            src = A.alloc<int32_t>(std::max<int64_t>(n, 1));
            pairs = A.alloc<int32_t>(2 * std::max<int64_t>(n, 1));
            int64_t nthr = std::max<int64_t>(n, T.nbox + 1);
            k_csr_ptr<<<grid_for(nthr, 256), 256, 0, st>>>(T.nbox, sorted, n, ptr, src, pairs);
            FB_HIP(hipGetLastError());
        };
        finish_list(m2l, n_m2l, T.m2l_ptr, T.m2l_src, T.m2l_pairs);
        finish_list(p2p, n_p2p, T.p2p_ptr, T.p2p_src, T.p2p_pairs);

        // FP32 leaf-relative coordinates
        G.tc32 = A.alloc<float>(3 * nt);
        G.sp32 = A.alloc<float>(4 * ns);
        k_relative<<<grid_for(nt, 256), 256, 0, st>>>(nt, T.panel_leaf, T.box_r, G.tc, G.sp, G.tc32, G.sp32);
        FB_HIP(hipGetLastError());

        // host copies: box geometry, P2P work count
        T.h_box_r.resize(5 * (size_t)T.nbox);
        FB_HIP(hipMemcpyAsync(T.h_box_r.data(), T.box_r, sizeof(double) * 5 * T.nbox, hipMemcpyDeviceToHost, st));
        std::vector<int32_t> hp(2 * std::max<int64_t>(n_p2p, 1));
        if (n_p2p)
            FB_HIP(hipMemcpyAsync(hp.data(), T.p2p_pairs, sizeof(int32_t) * 2 * n_p2p, hipMemcpyDeviceToHost, st));
        FB_HIP(hipStreamSynchronize(st));
        T.p2p_interactions = 0;
        for (int64_t i = 0; i < n_p2p; ++i) {
            int a = hp[2 * i], b = hp[2 * i + 1];
            T.p2p_interactions += (int64_t)(hb[6 * a + 2] - hb[6 * a + 1]) * 4 * (hb[6 * b + 2] - hb[6 * b + 1]);
        }
        build_p2p_units(ctx, hp, n_p2p, st);
        tmp.release();
    } catch (...) {
        (void)hipStreamSynchronize(st);
        tmp.release();
        throw;
    }
}

}  // namespace fmmbem
