/*
 * Oracle: CPU reference octree and interaction lists.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.c).  The product builds the same tree
 * and lists on the GPU, from its own code; tests compare the two bit for bit.
 *
 * Method (Sec. 2.5): recursive subdivision of space into an octree until a box
 * holds at most N_CRIT panels, multipoles about box centres, and a multipole
 * acceptance criterion (MAC) theta, the largest allowed ratio of cluster size
 * to distance, that decides between the expansion path and direct (P2P)
 * evaluation.  The paper leaves the details open; the contract read here:
 *
 *  - keys: the cube around the panel centroids has side
 *    max_extent * (1 + 2^-20) about the bounding-box midpoint (side 1 when all
 *    centroids coincide); cell = min(floor((x - lo) * (2^21 / side)), 2^21 - 1)
 *    per axis, bits interleaved x,y,z from the most significant bit down,
 *    giving 63-bit Morton keys; panels are sorted stably by key.
 *  - boxes: the root holds every panel; a box with more than N_CRIT panels
 *    below level 21 is split into its non-empty octants, in octant order;
 *    boxes are numbered level by level, each level in parent order.
 *  - box centre: the centre of its cube cell; radius R: the largest distance
 *    from the centre to a centroid or a far-rule Gauss point of its panels;
 *    guard G = sqrt(8 * max S_j) over its panels.
 *  - dual traversal from (root, root): a pair (A, B) with
 *    (R_A + R_B)^2 < theta^2 |c_A - c_B|^2 and
 *    (R_A + R_B + (1 + 1e-6) G_B)^2 <= |c_A - c_B|^2 is an M2L pair; else two
 *    leaves form a P2P pair; else the box with the larger R (the target on a
 *    tie, never a leaf) is replaced by its children.  The second test keeps
 *    every near-singular (target, panel) pair of Sec. 2.3 inside a P2P pair.
 *  - lists are sorted by (target box, source box).
 * All arithmetic is FP64 with the operation order written here and no fused
 * multiply-add (compiled with -ffp-contract=off).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t nt;
    int32_t nbox, nlevels;
    int32_t *perm;        /* sorted position -> input panel */
    uint64_t *keys;       /* sorted keys */
    int32_t *bi;          /* [nbox][6]: level, begin, end, parent, child0, nchild */
    double *br;           /* [nbox][5]: cx, cy, cz, R, G */
    int64_t n_m2l, n_p2p;
    int32_t *m2l, *p2p;   /* [n][2] (target, source) */
    double cube[4];       /* lo x, lo y, lo z, side */
} or_tree;

typedef struct {
    uint64_t key;
    int32_t idx;
} kv_t;

static int kv_cmp(const void *a, const void *b)
{
    const kv_t *x = (const kv_t *)a, *y = (const kv_t *)b;
    if (x->key != y->key)
        return x->key < y->key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

static int pair_cmp(const void *a, const void *b)
{
    const int32_t *x = (const int32_t *)a, *y = (const int32_t *)b;
    if (x[0] != y[0])
        return x[0] < y[0] ? -1 : 1;
    return x[1] < y[1] ? -1 : (x[1] > y[1]);
}

typedef struct {
    int32_t *a;
    int64_t n, cap;
} pairvec;

static int pv_push(pairvec *v, int32_t t, int32_t s)
{
    if (v->n == v->cap) {
        int64_t nc = v->cap ? 2 * v->cap : 1024;
        int32_t *na = (int32_t *)realloc(v->a, sizeof(int32_t) * 2 * (size_t)nc);
        if (!na)
            return -1;
        v->a = na;
        v->cap = nc;
    }
    v->a[2 * v->n] = t;
    v->a[2 * v->n + 1] = s;
    v->n++;
    return 0;
}

static uint64_t spread3(uint32_t v)
{
    /* bit b of v goes to bit 3b */
    uint64_t r = 0;
    for (int b = 0; b < 21; ++b)
        r |= (uint64_t)((v >> b) & 1u) << (3 * b);
    return r;
}

static uint32_t compact3(uint64_t k)
{
    uint32_t r = 0;
    for (int b = 0; b < 21; ++b)
        r |= (uint32_t)((k >> (3 * b)) & 1u) << b;
    return r;
}

void or_tree_free(or_tree *t)
{
    if (!t)
        return;
    free(t->perm);
    free(t->keys);
    free(t->bi);
    free(t->br);
    free(t->m2l);
    free(t->p2p);
    free(t);
}

or_tree *or_tree_build(int64_t nt, const double *xyz, const int32_t *tri, int32_t ncrit, double theta)
{
    if (nt < 1 || ncrit < 1)
        return NULL;
    or_tree *T = (or_tree *)calloc(1, sizeof(or_tree));
    double *c = (double *)malloc(sizeof(double) * 3 * (size_t)nt);
    double *S = (double *)malloc(sizeof(double) * (size_t)nt);
    double *gp = (double *)malloc(sizeof(double) * 12 * (size_t)nt); /* Gauss points */
    kv_t *kv = (kv_t *)malloc(sizeof(kv_t) * (size_t)nt);
    if (!T || !c || !S || !gp || !kv)
        return NULL;
    T->nt = nt;
    const double third = 1.0 / 3.0;
    const double L[4][3] = {{third, third, third}, {0.6, 0.2, 0.2}, {0.2, 0.6, 0.2}, {0.2, 0.2, 0.6}};
    for (int64_t j = 0; j < nt; ++j) {
        const double *v0 = xyz + 3 * (int64_t)tri[3 * j], *v1 = xyz + 3 * (int64_t)tri[3 * j + 1],
                     *v2 = xyz + 3 * (int64_t)tri[3 * j + 2];
        double e1[3], e2[3];
        for (int d = 0; d < 3; ++d) {
            c[3 * j + d] = ((v0[d] + v1[d]) + v2[d]) / 3.0;
            e1[d] = v1[d] - v0[d];
            e2[d] = v2[d] - v0[d];
        }
        double a0 = e1[1] * e2[2] - e1[2] * e2[1];
        double a1 = e1[2] * e2[0] - e1[0] * e2[2];
        double a2 = e1[0] * e2[1] - e1[1] * e2[0];
        S[j] = 0.5 * sqrt((a0 * a0 + a1 * a1) + a2 * a2);
        for (int k = 0; k < 4; ++k)
            for (int d = 0; d < 3; ++d)
                gp[12 * j + 3 * k + d] = (L[k][0] * v0[d] + L[k][1] * v1[d]) + L[k][2] * v2[d];
    }
    /* cube */
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d)
        lo[d] = hi[d] = c[d];
    for (int64_t j = 1; j < nt; ++j)
        for (int d = 0; d < 3; ++d) {
            double v = c[3 * j + d];
            if (v < lo[d]) lo[d] = v;
            if (v > hi[d]) hi[d] = v;
        }
    double ext = 0.0;
    for (int d = 0; d < 3; ++d) {
        double e = hi[d] - lo[d];
        if (e > ext) ext = e;
    }
    double side = ext > 0.0 ? ext * (1.0 + ldexp(1.0, -20)) : 1.0;
    double clo[3];
    for (int d = 0; d < 3; ++d)
        clo[d] = (lo[d] + hi[d]) * 0.5 - side * 0.5;
    double scale = ldexp(1.0, 21) / side;
    for (int d = 0; d < 3; ++d)
        T->cube[d] = clo[d];
    T->cube[3] = side;
    const uint32_t cmax = (1u << 21) - 1u;
    for (int64_t j = 0; j < nt; ++j) {
        uint32_t cell[3];
        for (int d = 0; d < 3; ++d) {
            double f = floor((c[3 * j + d] - clo[d]) * scale);
            if (f < 0.0) f = 0.0;
            cell[d] = f > (double)cmax ? cmax : (uint32_t)f;
        }
        kv[j].key = (spread3(cell[0]) << 2) | (spread3(cell[1]) << 1) | spread3(cell[2]);
        kv[j].idx = (int32_t)j;
    }
    qsort(kv, (size_t)nt, sizeof(kv_t), kv_cmp);
    T->perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)nt);
    T->keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)nt);
    for (int64_t j = 0; j < nt; ++j) {
        T->perm[j] = kv[j].idx;
        T->keys[j] = kv[j].key;
    }
    free(kv);

    /* boxes, level by level */
    int64_t cap = 1024, nb = 1;
    int32_t *bi = (int32_t *)malloc(sizeof(int32_t) * 6 * (size_t)cap);
    bi[0] = 0; bi[1] = 0; bi[2] = (int32_t)nt; bi[3] = -1; bi[4] = -1; bi[5] = 0;
    int64_t lev_begin = 0, lev_end = 1;
    int32_t level = 0;
    while (lev_begin < lev_end) {
        for (int64_t b = lev_begin; b < lev_end; ++b) {
            int32_t beg = bi[6 * b + 1], end = bi[6 * b + 2];
            if (end - beg <= ncrit || level >= 21)
                continue;
            int sh = 3 * (21 - (level + 1));
            int32_t p = beg;
            int first = 1;
            while (p < end) {
                uint64_t dig = (T->keys[p] >> sh) & 7u;
                int32_t q = p;
                while (q < end && ((T->keys[q] >> sh) & 7u) == dig)
                    ++q;
                if (nb == cap) {
                    cap *= 2;
                    bi = (int32_t *)realloc(bi, sizeof(int32_t) * 6 * (size_t)cap);
                }
                int32_t *nbx = bi + 6 * nb;
                nbx[0] = level + 1; nbx[1] = p; nbx[2] = q; nbx[3] = (int32_t)b; nbx[4] = -1; nbx[5] = 0;
                if (first) {
                    bi[6 * b + 4] = (int32_t)nb;
                    first = 0;
                }
                bi[6 * b + 5]++;
                ++nb;
                p = q;
            }
        }
        lev_begin = lev_end;
        lev_end = nb;
        ++level;
    }
    T->nbox = (int32_t)nb;
    T->nlevels = level;
    T->bi = bi;
    T->br = (double *)malloc(sizeof(double) * 5 * (size_t)nb);
    for (int64_t b = 0; b < nb; ++b) {
        int32_t lv = bi[6 * b], beg = bi[6 * b + 1], end = bi[6 * b + 2];
        uint64_t pre = T->keys[beg] >> (3 * (21 - lv));
        uint32_t ix = compact3(pre >> 2), iy = compact3(pre >> 1), iz = compact3(pre);
        double h = ldexp(side, -lv);
        double ctr[3] = {clo[0] + ((double)ix + 0.5) * h, clo[1] + ((double)iy + 0.5) * h,
                         clo[2] + ((double)iz + 0.5) * h};
        double r2max = 0.0, smax = 0.0;
        for (int32_t p = beg; p < end; ++p) {
            int64_t j = T->perm[p];
            const double *pts[5] = {c + 3 * j, gp + 12 * j, gp + 12 * j + 3, gp + 12 * j + 6, gp + 12 * j + 9};
            for (int k = 0; k < 5; ++k) {
                double dx = pts[k][0] - ctr[0], dy = pts[k][1] - ctr[1], dz = pts[k][2] - ctr[2];
                double r2 = (dx * dx + dy * dy) + dz * dz;
                if (r2 > r2max) r2max = r2;
            }
            if (S[j] > smax) smax = S[j];
        }
        double *o = T->br + 5 * b;
        o[0] = ctr[0]; o[1] = ctr[1]; o[2] = ctr[2];
        o[3] = sqrt(r2max);
        o[4] = sqrt(8.0 * smax);
    }
    free(c); free(S); free(gp);

    /* dual traversal with an explicit stack */
    pairvec m2l = {0}, p2p = {0}, st = {0};
    pv_push(&st, 0, 0);
    double th2 = theta * theta;
    while (st.n > 0) {
        st.n--;
        int32_t A = st.a[2 * st.n], B = st.a[2 * st.n + 1];
        const double *ra = T->br + 5 * (int64_t)A, *rb = T->br + 5 * (int64_t)B;
        double dx = ra[0] - rb[0], dy = ra[1] - rb[1], dz = ra[2] - rb[2];
        double d2 = (dx * dx + dy * dy) + dz * dz;
        double s = ra[3] + rb[3];
        double g = s + rb[4] * (1.0 + 1e-6);
        if (s * s < th2 * d2 && g * g <= d2) {
            pv_push(&m2l, A, B);
            continue;
        }
        int leafA = bi[6 * (int64_t)A + 5] == 0, leafB = bi[6 * (int64_t)B + 5] == 0;
        if (leafA && leafB) {
            pv_push(&p2p, A, B);
            continue;
        }
        int splitA = !leafA && (leafB || ra[3] >= rb[3]);
        if (splitA) {
            int32_t c0 = bi[6 * (int64_t)A + 4], nc = bi[6 * (int64_t)A + 5];
            for (int32_t k = 0; k < nc; ++k)
                pv_push(&st, c0 + k, B);
        } else {
            int32_t c0 = bi[6 * (int64_t)B + 4], nc = bi[6 * (int64_t)B + 5];
            for (int32_t k = 0; k < nc; ++k)
                pv_push(&st, A, c0 + k);
        }
    }
    free(st.a);
    if (m2l.n)
        qsort(m2l.a, (size_t)m2l.n, 2 * sizeof(int32_t), pair_cmp);
    if (p2p.n)
        qsort(p2p.a, (size_t)p2p.n, 2 * sizeof(int32_t), pair_cmp);
    T->m2l = m2l.a;
    T->n_m2l = m2l.n;
    T->p2p = p2p.a;
    T->n_p2p = p2p.n;
    return T;
}

/* sizes: nbox, nlevels, n_m2l, n_p2p */
void or_tree_sizes(const or_tree *T, int64_t *out)
{
    out[0] = T->nbox;
    out[1] = T->nlevels;
    out[2] = T->n_m2l;
    out[3] = T->n_p2p;
}

void or_tree_get(const or_tree *T, int32_t *perm, uint64_t *keys, int32_t *bi, double *br,
                 int32_t *m2l, int32_t *p2p, double *cube)
{
    if (perm) memcpy(perm, T->perm, sizeof(int32_t) * (size_t)T->nt);
    if (keys) memcpy(keys, T->keys, sizeof(uint64_t) * (size_t)T->nt);
    if (bi) memcpy(bi, T->bi, sizeof(int32_t) * 6 * (size_t)T->nbox);
    if (br) memcpy(br, T->br, sizeof(double) * 5 * (size_t)T->nbox);
    if (m2l && T->n_m2l) memcpy(m2l, T->m2l, sizeof(int32_t) * 2 * (size_t)T->n_m2l);
    if (p2p && T->n_p2p) memcpy(p2p, T->p2p, sizeof(int32_t) * 2 * (size_t)T->n_p2p);
    if (cube) memcpy(cube, T->cube, sizeof(double) * 4);
}
