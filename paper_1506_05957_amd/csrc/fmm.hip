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
#include <algorithm>
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
// charges: packed sources of this mat-vec, position and charge together so
// that P2P can stream them with one wave-uniform (scalar) load per source.
// FP64: absolute position; FP32: position relative to the leaf centre.
template <typename R, bool STOKES> struct Src;
template <> struct Src<double, false> { double x, y, z, q; };
template <> struct Src<float, false> { float x, y, z, q; };
template <> struct Src<double, true> { double x, y, z, f0, f1, f2, pad0, pad1; };
template <> struct Src<float, true> { float x, y, z, f0, f1, f2, pad0, pad1; };

// KIND: FMMBEM_LAPLACE_SL (charges w x), FMMBEM_STOKES_SL (forces w t) or
// FMMBEM_LAPLACE_DL (dipoles w x n_j of the source panel, n outward).
template <int KIND> constexpr bool vec_src() { return KIND != FMMBEM_LAPLACE_SL; }

// With xs (the stored near field), the first thread of every panel also
// copies the panel's input value(s) to xs in sorted order.  With nz.partn (the
// last Arnoldi step's partial sums of |w|^2), the input is w / |w|: every block
// sums the partials in the fixed order of the Arnoldi kernels, the first
// thread of every panel writes the normalised values to xout, and block 0
// stores |w|^2 to nz.nrm2_out (the normalisation of the Arnoldi step, done
// here instead of in its own launch).
template <typename R, int KIND>
__global__ __launch_bounds__(DOT_BLOCK) void k_charges(int64_t nt, const int32_t *__restrict__ perm,
                                                       const double *__restrict__ sp, const float *__restrict__ sp32,
                                                       const double *__restrict__ nrm, const double *__restrict__ xin,
                                                       Src<R, vec_src<KIND>()> *__restrict__ src,
                                                       double *__restrict__ xs, NormIn nz, double *__restrict__ xout)
{
    constexpr int NQ = KIND == FMMBEM_STOKES_SL ? 3 : 1;
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ns = 4 * nt;
    double scale = 1.0;
    if (nz.partn) {  // every thread of the block takes part in the sum
        __shared__ double tot;
        block_sums(nz.partn, nz.nb, 1, &tot);
        __syncthreads();
        scale = 1.0 / sqrt(tot);
        if (blockIdx.x == 0 && threadIdx.x == 0 && nz.nrm2_out)
            *nz.nrm2_out = tot;
    }
    if (s >= ns)
        return;
    const int64_t o = perm[s >> 2];
    double xv[NQ];
#pragma unroll
    for (int a = 0; a < NQ; ++a)
        xv[a] = nz.partn ? xin[NQ * o + a] * scale : xin[NQ * o + a];
    if ((s & 3) == 0) {
#pragma unroll
        for (int a = 0; a < NQ; ++a) {
            if (xs)
                xs[NQ * (s >> 2) + a] = xv[a];
            if (nz.partn)
                xout[NQ * o + a] = xv[a];
        }
    }
    const double w = sp[3 * ns + s];
    Src<R, vec_src<KIND>()> v;
    if constexpr (sizeof(R) == 8) {
        v.x = sp[s];
        v.y = sp[ns + s];
        v.z = sp[2 * ns + s];
    } else {
        v.x = sp32[s];
        v.y = sp32[ns + s];
        v.z = sp32[2 * ns + s];
    }
    if constexpr (KIND == FMMBEM_LAPLACE_SL) {
        v.q = (R)(w * xv[0]);
    } else if constexpr (KIND == FMMBEM_STOKES_SL) {
        v.f0 = (R)(w * xv[0]);
        v.f1 = (R)(w * xv[1]);
        v.f2 = (R)(w * xv[2]);
        v.pad0 = v.pad1 = 0;
    } else {
        const int64_t i = s >> 2;
        const double wx = w * xv[0];
        v.f0 = (R)(wx * nrm[i]);
        v.f1 = (R)(wx * nrm[nt + i]);
        v.f2 = (R)(wx * nrm[2 * nt + i]);
        v.pad0 = v.pad1 = 0;
    }
    src[s] = v;
}

// ---------------------------------------------------------------------------
// Sources of a leaf are staged through LDS in tiles of P2M_TILE: one coalesced
// copy per tile, so that the per-source loop reads them from LDS instead of
// waiting on a global load each time.
constexpr int P2M_TILE = 256;

template <typename S>
__device__ inline void stage_sources(const S *__restrict__ src, int64_t first, int count, S *__restrict__ tile)
{
    static_assert(sizeof(S) % 16 == 0, "sources are whole 16-byte words");
    constexpr int W = sizeof(S) / 16;
    const int4 *g = reinterpret_cast<const int4 *>(src + first);
    int4 *t = reinterpret_cast<int4 *>(tile);
    for (int k = threadIdx.x; k < count * W; k += blockDim.x)
        t[k] = g[k];
}

// P2M: one block per leaf.  Thread = (order m, source slice): it accumulates
// q conj(R_n^m((y - c) / s)) over the sources of its slice for n = m..p, and
// the slices are summed in a fixed order.  PM is a compile-time bound on p so
// that the accumulators stay in registers.
//
// The harmonics of one source come from one branch-free sweep n = 1..PM whose
// step coefficients depend on (n, m) only and are set up once per thread:
//   C_n = al_n (x + i y) C_{n-1} + be_n z C_{n-1} - ga_n r^2 C_{n-2},  C_0 = 1,
// with al_n = -1/(2n) for n <= m (the diagonal R_n^n), and for n > m
// be_n = (2n - 1)/((n - m)(n + m)), ga_n = 1/((n - m)(n + m)) (ga = 0 at
// n = m + 1, where R_{m-1}^m = 0), so that C_n = R_n^n below the column and
// R_n^m on it.  Entries below the column are accumulated too and never written.
// Channels are taken CG at a time (Stokes: 4 in FP32, 2 in FP64), so that
// every harmonic serves CG channels.
template <typename R, int NCH, int PM>
__global__ __launch_bounds__(256) void k_p2m(int p, int ncs, const int32_t *__restrict__ leaves,
                                             const int32_t *__restrict__ box_i, const double *__restrict__ box_r,
                                             double side, const Src<R, NCH == 4> *__restrict__ src,
                                             cplx<R> *__restrict__ M)
{
    constexpr int CG = NCH == 1 ? 1 : (sizeof(R) == 4 ? 4 : 2);
    using S = Src<R, NCH == 4>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    S *tile = reinterpret_cast<S *>(smem_raw);                                   // [P2M_TILE]
    cplx<R> *red = reinterpret_cast<cplx<R> *>(smem_raw + sizeof(S) * P2M_TILE);  // [nsl][nc]
    const int b = leaves[blockIdx.x];
    const int lv = box_i[6 * b], pb = box_i[6 * b + 1], pe = box_i[6 * b + 2];
    const double s = ldexp(side, -(lv + 1));
    const double *c = box_r + 5 * (int64_t)b;
    const int nm = p + 1, nsl = (int)blockDim.x / nm;
    const int m = threadIdx.x % nm, sl = threadIdx.x / nm;
    const bool active = sl < nsl;
    const int nc = ncoef(p);
    const R is = (R)(1.0 / s);
    R al[PM + 1], be[PM + 1], ga[PM + 1];
#pragma unroll
    for (int n = 1; n <= PM; ++n) {
        const R f = (n > m && n <= p) ? inv_int<R>((n - m) * (n + m)) : R(0);
        al[n] = n <= m ? -inv_int<R>(2 * n) : R(0);
        be[n] = R(2 * n - 1) * f;
        ga[n] = n >= m + 2 ? f : R(0);
    }
    for (int c0 = 0; c0 < NCH; c0 += CG) {
        R are[CG][PM + 1], aim[CG][PM + 1];
#pragma unroll
        for (int g = 0; g < CG; ++g)
#pragma unroll
            for (int n = 0; n <= PM; ++n)
                are[g][n] = aim[g][n] = 0;
        for (int64_t t0 = 4 * (int64_t)pb; t0 < 4 * (int64_t)pe; t0 += P2M_TILE) {
            const int cnt = (int)std::min<int64_t>(P2M_TILE, 4 * (int64_t)pe - t0);
            __syncthreads();  // the previous tile has been read
            stage_sources(src, t0, cnt, tile);
            __syncthreads();
            if (!active)
                continue;
            for (int si = sl; si < cnt; si += nsl) {
                const S sv = tile[si];
                R x, y, z;  // relative to the leaf centre
                if constexpr (sizeof(R) == 8) {
                    x = sv.x - c[0];
                    y = sv.y - c[1];
                    z = sv.z - c[2];
                } else {
                    x = sv.x;
                    y = sv.y;
                    z = sv.z;
                }
                R qq[CG];
                if constexpr (NCH == 1) {
                    qq[0] = sv.q;
                } else {
                    const R q4 = (sv.f0 * x + sv.f1 * y) + sv.f2 * z;
                    const R all[4] = {sv.f0, sv.f1, sv.f2, q4};
#pragma unroll
                    for (int g = 0; g < CG; ++g)
                        qq[g] = all[(c0 + g) & 3];
                }
                x *= is;
                y *= is;
                z *= is;
                const R r2 = x * x + y * y + z * z;
                R cr = 1, ci = 0, pr = 0, pi = 0;
#pragma unroll
                for (int g = 0; g < CG; ++g)
                    are[g][0] += qq[g];
#pragma unroll
                for (int n = 1; n <= PM; ++n) {
                    const R A = al[n] * x + be[n] * z, B = al[n] * y, G = ga[n] * r2;
                    const R nr = (A * cr - B * ci) - G * pr, ni = (A * ci + B * cr) - G * pi;
                    pr = cr;
                    pi = ci;
                    cr = nr;
                    ci = ni;
#pragma unroll
                    for (int g = 0; g < CG; ++g) {
                        are[g][n] += qq[g] * cr;
                        aim[g][n] -= qq[g] * ci;
                    }
                }
            }
        }
#pragma unroll
        for (int g = 0; g < CG; ++g) {
            if (active) {
#pragma unroll
                for (int n = 0; n <= PM; ++n)
                    if (n <= p && n >= m)
                        red[sl * nc + cidx(n, m)] = cplx<R>{are[g][n], aim[g][n]};
            }
            __syncthreads();
            for (int t = threadIdx.x; t < nc; t += blockDim.x) {
                R sr = 0, si2 = 0;
                for (int k = 0; k < nsl; ++k) {
                    sr += red[k * nc + t].re;
                    si2 += red[k * nc + t].im;
                }
                M[((int64_t)b * NCH + c0 + g) * ncs + t] = cplx<R>{sr, si2};
            }
            __syncthreads();
        }
    }
}

// P2M at the high orders, where the per-thread accumulators of k_p2m (2 (p+1)
// values per channel and the step coefficients) no longer fit the registers
// of several waves.  One block per leaf; the leaf's sources go through in
// tiles of TS = floor(blockDim / (p + 1)).  Phase 1: thread (s, m) runs the
// recurrence of k_p2m for source s and order m and writes conj(R_n^m), n =
// m..p, to the tile's harmonics in LDS.  Phase 2: thread (coefficient,
// channel) adds q conj(R) over the tile's sources in source order into one
// accumulator that it keeps across the tiles.  The charges of a tile sit
// beside the harmonics (Stokes: f and f . (y - c)).
template <typename R, int NCH>
__global__ __launch_bounds__(256) void k_p2m_tile(int p, int ncs, const int32_t *__restrict__ leaves,
                                                  const int32_t *__restrict__ box_i, const double *__restrict__ box_r,
                                                  double side, const Src<R, NCH == 4> *__restrict__ src,
                                                  cplx<R> *__restrict__ M)
{
    using S = Src<R, NCH == 4>;
    constexpr int ITEMS = 4;  // (coefficient, channel) items per thread: nc NCH <= 4 * 256 up to p = 20
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int nm = p + 1, nc = ncoef(p);
    const int ts = (int)blockDim.x / nm;
    cplx<R> *H = reinterpret_cast<cplx<R> *>(smem_raw);  // [ts][nc]
    R *Q = reinterpret_cast<R *>(smem_raw + sizeof(cplx<R>) * (size_t)ts * nc);  // [ts][NCH]
    // 1/k for k <= p^2: a thread's column recurrence takes 1/((n - m)(n + m))
    // with its own m, a read per step that from the constant table would be a
    // per-lane memory load waited on at every step
    R *inv = Q + (size_t)ts * NCH;  // [p^2 + 1]
    for (int k = threadIdx.x; k <= p * p; k += blockDim.x)
        inv[k] = inv_int<R>(k);
    const int b = leaves[blockIdx.x];
    const int lv = box_i[6 * b], pb = box_i[6 * b + 1], pe = box_i[6 * b + 2];
    const double s = ldexp(side, -(lv + 1));
    const double *c = box_r + 5 * (int64_t)b;
    const R is = (R)(1.0 / s);
    // s fastest: a wave holds a few neighbouring orders m, whose diagonal and
    // column recurrences run about as many steps as each other (with m
    // fastest every wave would run the longest diagonal and the longest column)
    const int sl = threadIdx.x % ts, m = threadIdx.x / ts;
    R ar[ITEMS], ai[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
        ar[k] = ai[k] = 0;
    const int64_t s0 = 4 * (int64_t)pb, s1 = 4 * (int64_t)pe;
    for (int64_t t0 = s0; t0 < s1; t0 += ts) {
        const int cnt = (int)std::min<int64_t>(ts, s1 - t0);
        __syncthreads();  // the previous tile has been read
        if (sl < cnt && m < nm) {
            const S sv = src[t0 + sl];
            R x, y, z;  // relative to the leaf centre
            if constexpr (sizeof(R) == 8) {
                x = sv.x - c[0];
                y = sv.y - c[1];
                z = sv.z - c[2];
            } else {
                x = sv.x;
                y = sv.y;
                z = sv.z;
            }
            if (m == 0) {
                if constexpr (NCH == 1) {
                    Q[sl] = sv.q;
                } else {
                    Q[4 * sl] = sv.f0;
                    Q[4 * sl + 1] = sv.f1;
                    Q[4 * sl + 2] = sv.f2;
                    Q[4 * sl + 3] = (sv.f0 * x + sv.f1 * y) + sv.f2 * z;
                }
            }
            x *= is;
            y *= is;
            z *= is;
            const R r2 = x * x + y * y + z * z;
            cplx<R> *h = H + (int64_t)sl * nc;
            // the diagonal R_m^m, then the column R_n^m, n > m
            R cr = 1, ci = 0;
            for (int n = 1; n <= m; ++n) {
                const R al = -inv[2 * n];
                const R A = al * x, B = al * y;
                const R nr = A * cr - B * ci, ni = A * ci + B * cr;
                cr = nr;
                ci = ni;
            }
            h[cidx(m, m)] = cplx<R>{cr, -ci};
            R pr = 0, pi = 0;
            for (int n = m + 1; n <= p; ++n) {
                const R f = inv[(n - m) * (n + m)];
                const R A = R(2 * n - 1) * f * z, G = n >= m + 2 ? f * r2 : R(0);
                const R nr = A * cr - G * pr, ni = A * ci - G * pi;
                pr = cr;
                pi = ci;
                cr = nr;
                ci = ni;
                h[cidx(n, m)] = cplx<R>{cr, -ci};
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const int it = threadIdx.x + k * (int)blockDim.x;
            if (it < nc * NCH) {
                const int ch = it / nc, idx = it - ch * nc;
                for (int j = 0; j < cnt; ++j) {
                    const cplx<R> hv = H[(int64_t)j * nc + idx];
                    const R q = Q[NCH * j + ch];
                    ar[k] += q * hv.re;
                    ai[k] += q * hv.im;
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int it = threadIdx.x + k * (int)blockDim.x;
        if (it < nc * NCH) {
            const int ch = it / nc, idx = it - ch * nc;
            M[((int64_t)b * NCH + ch) * ncs + idx] = cplx<R>{ar[k], ai[k]};
        }
    }
}

template <typename R, int NCH> size_t p2m_tile_shm(int p)
{
    const int ts = 256 / (p + 1);
    return sizeof(cplx<R>) * (size_t)ts * ncoef(p) + sizeof(R) * ((size_t)ts * NCH + (size_t)p * p + 1);
}

// P2M of dipole sources (the double layer): a moment d = w x n at y has
// the multipole sum conj(d . grad R_n^m(y - c)), and with the gradient
// identities of the factorial-normalised harmonics
//   d . grad R_n^m = (dx - i dy)/2 R_{n-1}^{m+1} - (dx + i dy)/2 R_{n-1}^{m-1}
//                    + dz R_{n-1}^m;
// in the scaled form (u = (y - c)/s) the sum picks up a factor 1/s.  Thread =
// (order m, source slice); it runs the columns m - 1, m, m + 1 of R(u) up to
// degree p - 1 together (column -1 from R_k^-1 = -conj(R_k^1)).
template <typename R, int PM>
__global__ __launch_bounds__(256) void k_p2m_dipole(int p, int ncs, const int32_t *__restrict__ leaves,
                                                    const int32_t *__restrict__ box_i, const double *__restrict__ box_r,
                                                    double side, const Src<R, true> *__restrict__ src,
                                                    cplx<R> *__restrict__ M)
{
    using S = Src<R, true>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    S *tile = reinterpret_cast<S *>(smem_raw);                                   // [P2M_TILE]
    cplx<R> *red = reinterpret_cast<cplx<R> *>(smem_raw + sizeof(S) * P2M_TILE);  // [nsl][nc]
    const int b = leaves[blockIdx.x];
    const int lv = box_i[6 * b], pb = box_i[6 * b + 1], pe = box_i[6 * b + 2];
    const double s = ldexp(side, -(lv + 1));
    const double *c = box_r + 5 * (int64_t)b;
    const int nm = p + 1, nsl = (int)blockDim.x / nm;
    const int m = threadIdx.x % nm, sl = threadIdx.x / nm;
    const bool active = sl < nsl;
    const int nc = ncoef(p);
    const R is = (R)(1.0 / s);
    // columns run: m - 1 (|m - 1| = 1 when m = 0), m, m + 1
    const int colA = m >= 1 ? m - 1 : 1, colB = m, colC = m + 1;
    R are[PM + 1], aim[PM + 1];
#pragma unroll
    for (int n = 0; n <= PM; ++n)
        are[n] = aim[n] = 0;
    for (int64_t t0 = 4 * (int64_t)pb; t0 < 4 * (int64_t)pe; t0 += P2M_TILE) {
        const int cnt = (int)std::min<int64_t>(P2M_TILE, 4 * (int64_t)pe - t0);
        __syncthreads();  // the previous tile has been read
        stage_sources(src, t0, cnt, tile);
        __syncthreads();
        if (!active)
            continue;
        for (int si = sl; si < cnt; si += nsl) {
            const S sv = tile[si];
            R x, y, z;  // relative to the leaf centre, then scaled
            if constexpr (sizeof(R) == 8) {
                x = sv.x - c[0];
                y = sv.y - c[1];
                z = sv.z - c[2];
            } else {
                x = sv.x;
                y = sv.y;
                z = sv.z;
            }
            x *= is;
            y *= is;
            z *= is;
            const R r2 = x * x + y * y + z * z;
            // diagonal values R_k^k, kept for k = colA, colB, colC
            R dre = 1, dim = 0, aRe = 0, aIm = 0, bRe = 0, bIm = 0, cRe = 0, cIm = 0;
            for (int k = 0; k <= colC; ++k) {
                if (k == colA) {
                    aRe = dre;
                    aIm = dim;
                }
                if (k == colB) {
                    bRe = dre;
                    bIm = dim;
                }
                if (k == colC) {
                    cRe = dre;
                    cIm = dim;
                }
                const R f = -inv_int<R>(2 * (k + 1));
                const R a = f * (x * dre - y * dim), bb = f * (x * dim + y * dre);
                dre = a;
                dim = bb;
            }
            // running (current, previous) of the three columns
            R Ac = 0, Ai = 0, Ap = 0, Api = 0, Bc = 0, Bi = 0, Bp = 0, Bpi = 0, Cc = 0, Ci = 0, Cp = 0, Cpi = 0;
            const R hx = R(0.5) * sv.f0, hy = R(0.5) * sv.f1, dz = sv.f2;
#pragma unroll
            for (int k = 0; k < PM; ++k) {
                if (k < p) {
                    // advance each column to degree k
                    if (k == colA) {
                        Ac = aRe;
                        Ai = aIm;
                    } else if (k > colA) {
                        const R f = inv_int<R>((k - colA) * (k + colA)), a = R(2 * k - 1) * z;
                        const R nr = (a * Ac - r2 * Ap) * f, ni = (a * Ai - r2 * Api) * f;
                        Ap = Ac;
                        Api = Ai;
                        Ac = nr;
                        Ai = ni;
                    }
                    if (k == colB) {
                        Bc = bRe;
                        Bi = bIm;
                    } else if (k > colB) {
                        const R f = inv_int<R>((k - colB) * (k + colB)), a = R(2 * k - 1) * z;
                        const R nr = (a * Bc - r2 * Bp) * f, ni = (a * Bi - r2 * Bpi) * f;
                        Bp = Bc;
                        Bpi = Bi;
                        Bc = nr;
                        Bi = ni;
                    }
                    if (k == colC) {
                        Cc = cRe;
                        Ci = cIm;
                    } else if (k > colC) {
                        const R f = inv_int<R>((k - colC) * (k + colC)), a = R(2 * k - 1) * z;
                        const R nr = (a * Cc - r2 * Cp) * f, ni = (a * Ci - r2 * Cpi) * f;
                        Cp = Cc;
                        Cpi = Ci;
                        Cc = nr;
                        Ci = ni;
                    }
                    // R_k^{m-1}, R_k^m, R_k^{m+1} (zero below their column's order)
                    R m1r = k >= colA ? Ac : R(0);
                    const R m1i = k >= colA ? Ai : R(0);
                    if (m == 0)  // R_k^-1 = -conj(R_k^1): real part negated, imaginary part kept
                        m1r = -m1r;
                    const R z0r = k >= colB ? Bc : R(0), z0i = k >= colB ? Bi : R(0);
                    const R p1r = k >= colC ? Cc : R(0), p1i = k >= colC ? Ci : R(0);
                    // D = (hx - i hy) R^{m+1} - (hx + i hy) R^{m-1} + dz R^m, degree n = k + 1
                    const R Dr = (hx * p1r + hy * p1i) - (hx * m1r - hy * m1i) + dz * z0r;
                    const R Di = (hx * p1i - hy * p1r) - (hx * m1i + hy * m1r) + dz * z0i;
                    are[k + 1] += is * Dr;
                    aim[k + 1] -= is * Di;
                }
            }
        }
    }
    if (active) {
#pragma unroll
        for (int n = 0; n <= PM; ++n)
            if (n <= p && n >= m)
                red[sl * nc + cidx(n, m)] = cplx<R>{are[n], aim[n]};
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nc; t += blockDim.x) {
        R sr = 0, si2 = 0;
        for (int k = 0; k < nsl; ++k) {
            sr += red[k * nc + t].re;
            si2 += red[k * nc + t].im;
        }
        M[(int64_t)b * ncs + t] = cplx<R>{sr, si2};
    }
}

// ---------------------------------------------------------------------------
// M2M and L2L as products with the octant operators: the child C
// sits at delta = (c_C - c_P) / s_P, one of the 8 offsets (+-1/2, +-1/2, +-1/2),
// and in the scaled expansions
//   M2M: M_n^m(P) += sum_{j <= n} 2^-j sum_mm conj(R_{n-j}^{m-mm}(delta)) M_j^mm(C)
//   L2L: L_j^k(C) += 2^-(j+1) sum_{n >= j} sum_m L_n^m(P) conj(R_{n-j}^{m-k}(delta))
// are fixed real linear maps of the stored coefficients, one per octant
// (k_octant_mfma, below, applies them on the matrix cores).  M2M writes
// per-child terms that k_m2m_sum adds up per parent in child order; L2L adds
// into the child.  Stokes: the fourth channel changes centre with the first
// three (M2M: + d . Z, L2L: - d . Z, d = c_C - c_P).

// M_P = sum of the per-child terms Z_C over the children of P, in child order
template <typename R, int NCH>
__global__ void k_m2m_sum(int p, int ncs, int npar, const int32_t *__restrict__ parents,
                          const int32_t *__restrict__ box_i, const cplx<R> *__restrict__ Z, cplx<R> *__restrict__ M)
{
    const int nc = ncoef(p);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)npar * NCH * nc)
        return;
    const int i = (int)(t / (NCH * nc)), rem = (int)(t - (int64_t)i * NCH * nc);
    const int ch = rem / nc, c = rem - ch * nc;
    const int P = parents[i];
    const int c0 = box_i[6 * P + 4], nch = box_i[6 * P + 5];  // 1..8 children
    // the (at most 8) children's terms read together, added in child order
    cplx<R> v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
        v[u] = Z[((int64_t)(c0 + min(u, nch - 1)) * NCH + ch) * ncs + c];
    R sr = 0, si = 0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
        if (u < nch) {
            sr += v[u].re;
            si += v[u].im;
        }
    M[((int64_t)P * NCH + ch) * ncs + c] = cplx<R>{sr, si};
}

// ---------------------------------------------------------------------------
// M2L, in two passes.  Pass 1, one block per chunk of pairs sharing a
// translation (D, eT, eS), computes per pair the scaled translation
//   L_k^l = (-1)^k 2^(-eT (k+1)) sum_{n,m} 2^(-eS n) M_n^m I_{n+k}^{m+l}(D 2^-e)
// (sigma the larger half-size) and writes it to Y[pair]; pass 2 sums Y over
// each target's pairs in list order.
// Pass 1 is a dense product per chunk, on the matrix cores.  With
// X = a + ib a stored coefficient (m >= 0) and X_n^-m = (-1)^m conj(X), the
// terms of m and -m combine into a real map: for output (k, l) and input
// (n, m), with P = I_{n+k}^{m+l}, Q = (-1)^m I_{n+k}^{l-m} (Q = 0 for m = 0),
// S = P + Q and D = P - Q,
//   Re L += a S.re - b D.im,   Im L += a S.im + b D.re,
// times (-1)^k 2^(-eT (k+1)) 2^(-eS n).  Rows of the real operator A are
// (k, l, re/im), inputs (n, m, re/im), columns (pair, channel): Y = A X.
// The chunk's inputs (at most 64 columns) are staged in LDS in windows of 64,
// every load issued unguarded at a clamped address and several at a time;
// wave w takes the 16-row tiles w, w + nwave, ... (accumulators held across
// the windows); each lane generates its element of A for every 16x16x4 step
// from the key's table in LDS, branch free, and the step runs all (at most 4)
// column tiles of the chunk.  Lane layout
// (both precisions): A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k; the
// result D[i][j] is element i % 4 of lane j + 16 (i / 4) in FP32 and element
// i / 4 of lane j + 16 (i % 4) in FP64.  Stokes: column j is channel j mod 4
// of its pair, so the lanes of the fourth channel take the pair's first three
// channels from their neighbours and move its centre from c_S to c_T as they
// write it out, Y_3 + (c_S - c_T) . (Y_0, Y_1, Y_2) (the FP64 direct kernels
// leave that to the sum of Y).
template <typename R> struct Acc4;
template <> struct Acc4<double> { typedef double type __attribute__((ext_vector_type(4))); };
template <> struct Acc4<float> { typedef float type __attribute__((ext_vector_type(4))); };

__device__ __forceinline__ Acc4<double>::type mfma_16x16x4(double a, double b, Acc4<double>::type c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ Acc4<float>::type mfma_16x16x4(float a, float b, Acc4<float>::type c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// M2M and L2L with the octant operators on the matrix cores.  A block takes a
// tile of 16 columns (boxes x channels) of one level and octant and a chunk
// of 64 output rows, as 16x16x4 steps.  Wave w takes rows 16 w .. +15
// of the chunk over the inputs that the triangular structure leaves (M2M:
// degree <= the tile's last row's; L2L: >= its first row's; the operators
// hold exact zeros elsewhere), so no wave sums another's partials: A from the
// operator (rows contiguous per input, several reads in flight), B from the
// staged inputs, one 8-byte LDS read per lane and step (a vector form with
// lane = row read 16 broadcast inputs per step and was bound by LDS).  The
// rows are then put back through LDS and written, one lane per row, with the
// Stokes change of centre.  Dynamic LDS: octant_mfma_shm.
template <typename R> size_t octant_mfma_shm(int p)
{
    const size_t Dp4 = (2 * (size_t)ncoef(p) + 3) & ~(size_t)3;
    return sizeof(R) * 16 * std::max<size_t>(Dp4, 64);
}

template <typename R, int NCH, bool L2L>
__global__ __launch_bounds__(256) void k_octant_mfma(int p, int ncs, int D, const R *__restrict__ ops,
                                                     const int4 *__restrict__ tiles, int tile0,
                                                     const int32_t *__restrict__ list,
                                                     const int32_t *__restrict__ box_i,
                                                     const double *__restrict__ box_r, const cplx<R> *__restrict__ X,
                                                     cplx<R> *__restrict__ Y)
{
    constexpr int NCOL = 16;
    constexpr int BPT = NCOL / NCH;  // boxes per tile
    constexpr int PF = 8;            // operator reads in flight
    extern __shared__ __align__(16) unsigned char smem_raw[];
    R *xs = reinterpret_cast<R *>(smem_raw);   // [Dp4][NCOL] (inputs past Dp zero), then
    R *out = reinterpret_cast<R *>(smem_raw);  // [NCOL][64] the chunk's rows
    __shared__ int64_t colofs[NCOL];  // first real of each column's input, -1 past the tile
    const int4 tl = tiles[tile0 + blockIdx.x];
    const int o = tl.x, e0 = tl.y, cnt = tl.z;
    const int Dp = 2 * ncoef(p), Dp4 = (Dp + 3) & ~3;
    if ((int)threadIdx.x < NCOL) {
        const int col = threadIdx.x, b = col / NCH, ch = col - b * NCH;
        int64_t ofs = -1;
        if (b < cnt) {
            const int box = list[e0 + b];
            const int from = L2L ? box_i[6 * box + 3] : box;
            ofs = 2 * (((int64_t)from * NCH + ch) * ncs);
        }
        colofs[col] = ofs;
    }
    __syncthreads();
    {
        // wave w stages columns 4 w .. 4 w + 3, the loads of a row issued together
        const int w0 = threadIdx.x >> 6, lane0 = threadIdx.x & 63;
        const R *Xr = reinterpret_cast<const R *>(X);
        int64_t ofs[4];
#pragma unroll
        for (int c = 0; c < 4; ++c)
            ofs[c] = colofs[4 * w0 + c];
        for (int k = lane0; k < Dp4; k += 64) {
            R v[4];
#pragma unroll
            for (int c = 0; c < 4; ++c)
                v[c] = Xr[(ofs[c] < 0 ? 0 : ofs[c]) + min(k, Dp - 1)];
#pragma unroll
            for (int c = 0; c < 4; ++c)
                xs[k * NCOL + 4 * w0 + c] = (ofs[c] < 0 || k >= Dp) ? R(0) : v[c];
        }
    }
    __syncthreads();
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int r0 = blockIdx.y * 64 + 16 * w;  // this wave's first row
    int ka = 0, kb = 0;                       // its inputs, in steps of 4
    if (r0 < Dp) {
        int n0, m0, n1, m1;
        idx_to_nm(r0 >> 1, n0, m0);
        idx_to_nm(min(r0 + 15, Dp - 1) >> 1, n1, m1);
        ka = L2L ? (2 * cidx(n0, 0)) & ~3 : 0;
        kb = L2L ? Dp4 : min(Dp4, (2 * ncoef(n1) + 3) & ~3);
    }
    const int ia = lane & 15, kk = lane >> 4;  // A[i][k] and B[k][j] in lane i (or j) + 16 k
    const R *A = ops + (int64_t)o * D * D + min(r0 + ia, Dp - 1);  // rows past Dp read row Dp - 1, not stored
    typename Acc4<R>::type acc = {0, 0, 0, 0};
    const int nst = (kb - ka) >> 2;
    if (nst > 0) {
        R ring[PF];
#pragma unroll
        for (int j = 0; j < PF; ++j)
            ring[j] = A[(int64_t)min(ka + 4 * min(j, nst - 1) + kk, Dp - 1) * D];
        auto step = [&](int t, R &slot) {
            const int k = ka + 4 * t;
            acc = mfma_16x16x4(slot, xs[(k + kk) * NCOL + ia], acc);
            slot = A[(int64_t)min(ka + 4 * min(t + PF, nst - 1) + kk, Dp - 1) * D];
        };
        const int nfull = nst - nst % PF;
        for (int t0 = 0; t0 < nfull; t0 += PF) {
#pragma unroll
            for (int j = 0; j < PF; ++j)
                step(t0 + j, ring[j]);
        }
#pragma unroll
        for (int j = 0; j < PF; ++j)
            if (nfull + j < nst)
                step(nfull + j, ring[j]);
    }
    __syncthreads();  // xs is dead from here on
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = sizeof(R) == 8 ? 4 * v + kk : 4 * kk + v;  // row of element v in this lane
        out[ia * 64 + 16 * w + i] = acc[v];
    }
    __syncthreads();
    const int r = blockIdx.y * 64 + lane;
    if (w != 0 || r >= Dp)
        return;
    R a[NCOL];
#pragma unroll
    for (int q = 0; q < NCOL; ++q)
        a[q] = out[q * 64 + lane];
#pragma unroll
    for (int bq = 0; bq < BPT; ++bq) {
        if (bq >= cnt)
            break;
        const int box = list[e0 + bq];
        R v[NCH];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
            v[ch] = a[bq * NCH + ch];
        if constexpr (NCH == 4) {
            const double *cC = box_r + 5 * (int64_t)box, *cP = box_r + 5 * (int64_t)box_i[6 * box + 3];
            const R d0 = (R)(cC[0] - cP[0]), d1 = (R)(cC[1] - cP[1]), d2 = (R)(cC[2] - cP[2]);
            const R dv = d0 * v[0] + d1 * v[1] + d2 * v[2];
            v[3] = L2L ? v[3] - dv : v[3] + dv;
        }
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            R *dst = reinterpret_cast<R *>(Y + ((int64_t)box * NCH + ch) * ncs) + r;
            if constexpr (L2L)
                *dst += v[ch];
            else
                *dst = v[ch];
        }
    }
}

template <typename R, int NCH, int RT>
__global__ __launch_bounds__(256) void k_m2l_mfma(int p, int ncs, int q_tab, const int32_t *__restrict__ chunk_begin,
                                                  const int32_t *__restrict__ chunk_trans,
                                                  const uint64_t *__restrict__ trans_key,
                                                  const int32_t *__restrict__ pair_sorted,
                                                  const int32_t *__restrict__ pairs, const cplx<R> *__restrict__ table,
                                                  const double *__restrict__ box_r, const cplx<R> *__restrict__ M,
                                                  cplx<R> *__restrict__ Y)
{
    typedef typename Acc4<R>::type acc_t;
    constexpr int NT = 4;   // column tiles of a chunk (at most 64 columns)
    constexpr int KW = 64;  // inputs per staging window
    constexpr int U = 8;    // staging loads issued together per thread
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int q = 2 * p;
    const int fq = (q + 1) * (q + 1), nc = ncoef(p), Dp = 2 * nc, Kp = (Dp + 3) & ~3, nrt = (Dp + 15) / 16;
    const int ldb = min(Kp, KW) + 1;
    int64_t *colsrc = reinterpret_cast<int64_t *>(smem_raw);  // [64]: first real of the column's input, or -1
    int64_t *coldst = colsrc + 64;                             // [64]: first real of the column's result
    R *gsh = reinterpret_cast<R *>(coldst + 64);               // [16][3]: c_S - c_T of the chunk's pairs (Stokes)
    cplx<R> *It = reinterpret_cast<cplx<R> *>(gsh + 48);       // [(q+1)^2]
    R *Bs = reinterpret_cast<R *>(It + fq);                    // [64][ldb]: a window of the chunk's inputs
    uint16_t *qnm = reinterpret_cast<uint16_t *>(Bs + 64 * ldb);  // [nc]: n | m << 8
    const int c = blockIdx.x;
    const int u = chunk_trans[c], pb = chunk_begin[c], pe = chunk_begin[c + 1];
    const uint64_t key = trans_key[u];
    const int eT = (int)((key >> 48) & 63), eS = (int)((key >> 54) & 63);
    const int ncol = (pe - pb) * NCH, nct = (ncol + 15) / 16;  // nct <= NT
    const cplx<R> *tab = table + (int64_t)u * (q_tab + 1) * (q_tab + 1);
    for (int t = threadIdx.x; t < fq; t += blockDim.x)
        It[t] = tab[t];
    for (int t = threadIdx.x; t < nc; t += blockDim.x) {
        int n, m;
        idx_to_nm(t, n, m);
        qnm[t] = (uint16_t)(n | (m << 8));
    }
    if (threadIdx.x < 64) {
        const int col = threadIdx.x;
        int64_t s = -1, d = 0;
        if (col < ncol) {
            const int pl = col / NCH, ch = col - pl * NCH;
            const int pr = pair_sorted[pb + pl];
            const int S = pairs[2 * pr + 1];
            s = 2 * (((int64_t)S * NCH + ch) * ncs);
            d = 2 * (((int64_t)pr * NCH + ch) * nc);
        }
        colsrc[col] = s;
        coldst[col] = d;
        if (NCH == 4 && col < 48) {
            const int pl = col / 3, xyz = col - 3 * pl;
            R g = 0;
            if (pl < pe - pb) {
                const int pr = pair_sorted[pb + pl];
                g = (R)(box_r[5 * (int64_t)pairs[2 * pr + 1] + xyz] - box_r[5 * (int64_t)pairs[2 * pr] + xyz]);
            }
            gsh[col] = g;
        }
    }
    const int nwave = blockDim.x >> 6;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int pin = lk & 1;  // re/im part of this lane's input (fixed: steps advance k by 4)
    const int nrw = (nrt - w + nwave - 1) / nwave;  // row tiles of this wave, <= RT (checked at launch)
    const R *Mr = reinterpret_cast<const R *>(M);
    acc_t acc[RT][NT];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int ct = 0; ct < NT; ++ct)
            acc[i][ct] = acc_t{0, 0, 0, 0};
    for (int k0 = 0; k0 < Kp; k0 += KW) {
        const int kw = min(KW, Kp - k0);
        __syncthreads();  // the column offsets written, the previous window read
        // stage inputs k0 .. k0 + kw - 1 of the chunk's column tiles, zero past Dp
        // and past the last column: lane = (column of the step, input), the
        // waves take steps of cpw columns; every load unguarded (clamped), U at a time
        {
            const int cpw = KW / kw, sub = lane / kw, kk = lane - sub * kw, nstc = nct * 16;
            const int cstep = nwave * cpw;
            const bool lv = sub < cpw;
            const int kc = min(k0 + kk, Dp - 1);
            for (int cb = w * cpw; cb < nstc; cb += U * cstep) {  // wave-uniform
                R v[U];
#pragma unroll
                for (int j = 0; j < U; ++j) {
                    const int64_t s = colsrc[min(cb + sub + j * cstep, nstc - 1)];
                    v[j] = Mr[s < 0 ? 0 : s + kc];
                }
#pragma unroll
                for (int j = 0; j < U; ++j) {
                    const int col = cb + sub + j * cstep;
                    if (lv && col < nstc)
                        Bs[col * ldb + kk] = (colsrc[col] >= 0 && k0 + kk < Dp) ? v[j] : R(0);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < RT; ++i) {
            if (i >= nrw)
                break;
            const int r = (w + i * nwave) * 16 + li;  // operator row of this lane's A elements
            const int er = qnm[min(r, Dp - 1) >> 1];
            const int k = er & 0xff, l = er >> 8;
            const int po = r & 1;
            // sign of the whole entry and the component (re/im) it takes from P and Q
            const R sall = (po == 0 && pin == 1) ? R(-1) : R(1);
            const bool take_im = (po ^ pin) != 0;
            const R f = r < Dp ? sall * (R)ldexp((k & 1) ? -1.0 : 1.0, -eT * (k + 1)) : R(0);
            const R *bl = Bs + li * ldb + lk;
#pragma unroll 2
            for (int s = 0; s < kw; s += 4) {
                const int qi = k0 + s + lk;
                const int e = qnm[min(qi, Dp - 1) >> 1];
                const int n = e & 0xff, m = e >> 8;
                const cplx<R> *row = It + (n + k) * (n + k + 1);  // I_{n+k}^{0}
                const cplx<R> P = row[l + m], Q = row[l - m];
                const R pc = take_im ? P.im : P.re, qc = take_im ? Q.im : Q.re;
                // (-1)^m from Q, and + for S (pin 0) or - for D (pin 1); no Q for m = 0
                const R qs = m == 0 ? R(0) : ((((m & 1) != 0) != (pin != 0)) ? -qc : qc);
                const R a = qi < Dp ? (R)ldexp(f * (pc + qs), -eS * n) : R(0);
                R b[NT];
#pragma unroll
                for (int ct = 0; ct < NT; ++ct)
                    b[ct] = bl[ct * 16 * ldb + s];
#pragma unroll
                for (int ct = 0; ct < NT; ++ct)
                    if (ct < nct)
                        acc[i][ct] = mfma_16x16x4(a, b[ct], acc[i][ct]);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < RT; ++i) {
        if (i >= nrw)
            break;
        const int rt = w + i * nwave;
#pragma unroll
        for (int ct = 0; ct < NT; ++ct) {
            if (ct >= nct)  // wave-uniform
                break;
            const int col = ct * 16 + li;
            R *dst = reinterpret_cast<R *>(Y) + coldst[col];
            R g0 = 0, g1 = 0, g2 = 0;
            if constexpr (NCH == 4) {
                const R *gq = gsh + 3 * (col >> 2);
                g0 = gq[0];
                g1 = gq[1];
                g2 = gq[2];
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                // output element v of this lane: row 4 lk + v (FP32 form), 4 v + lk (FP64 form)
                const int row = rt * 16 + (sizeof(R) == 8 ? 4 * v + lk : 4 * lk + v);
                R val = acc[i][ct][v];
                if constexpr (NCH == 4) {
                    // every lane shuffles (no lane is off here); the channels 0..2 of
                    // this lane's pair and rows sit in lanes 4 (li / 4) + 0..2
                    const int q0 = lane & ~3;
                    const R y0 = __shfl(val, q0), y1 = __shfl(val, q0 + 1), y2 = __shfl(val, q0 + 2);
                    if ((li & 3) == 3)
                        val += g0 * y0 + g1 * y1 + g2 * y2;
                }
                if (col < ncol && row < Dp)
                    dst[row] = val;
            }
        }
    }
}

// LDS of k_m2l_mfma: the key's table and the (n, m) index
// Stored pass-1 operators (FP64).  k_m2l_opgen writes, for translation u at
// p_max, the element of A that lane (i + 16 k) of the matrix-core step (rt, kt)
// takes, A[16 rt + i][4 kt + k], exactly as k_m2l_mfma generates it, to
// ops[((u nrt + rt) k4 + kt) 64 + lane]; entries beyond 2 ncoef(p_max) are 0.
// Grid (translation, row tile); the waves take the column steps in turn.
__global__ __launch_bounds__(256) void k_m2l_opgen(int pmax, int q_tab, int nrt, int k4,
                                                   const uint64_t *__restrict__ trans_key,
                                                   const cplx<double> *__restrict__ table, double *__restrict__ ops)
{
    const int u = blockIdx.x, rt = blockIdx.y;
    const uint64_t key = trans_key[u];
    const int eT = (int)((key >> 48) & 63), eS = (int)((key >> 54) & 63);
    const cplx<double> *It = table + (int64_t)u * (q_tab + 1) * (q_tab + 1);
    const int Dp = 2 * ncoef(pmax);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const int pin = lk & 1;
    const int r = rt * 16 + li;
    const bool rv = r < Dp;
    int k = 0, l = 0;
    if (rv)
        idx_to_nm(r >> 1, k, l);
    const int po = r & 1;
    const double sall = (po == 0 && pin == 1) ? -1.0 : 1.0;
    const bool take_im = (po ^ pin) != 0;
    const double f = rv ? sall * ldexp((k & 1) ? -1.0 : 1.0, -eT * (k + 1)) : 0.0;
    double *dst = ops + ((int64_t)u * nrt + rt) * k4 * 64 + lane;
    for (int kt = w; kt < k4; kt += blockDim.x >> 6) {
        const int qi = 4 * kt + lk;
        double a = 0.0;
        if (rv && qi < Dp) {
            int n, m;
            idx_to_nm(qi >> 1, n, m);
            const cplx<double> *row = It + (n + k) * (n + k + 1);  // I_{n+k}^{0}
            const cplx<double> P = row[l + m];
            double pc = take_im ? P.im : P.re;
            if (m > 0) {
                const cplx<double> Q = row[l - m];
                const double qc = take_im ? Q.im : Q.re;
                pc += (((m & 1) != 0) != (pin != 0)) ? -qc : qc;
            }
            a = ldexp(f * pc, -eS * n);
        }
        dst[(int64_t)kt * 64] = a;
    }
}

// Pass 1 in FP64 from the stored operators.  Block = chunk (at most 64
// columns: pairs x channels, one key); wave w runs row tiles w, w + 4, w + 8
// of the operator (three products in flight) with a four-step ring of
// operator reads (one coalesced 512-byte read per wave and step, never
// guarded: a guarded read would wait on itself), so each operator value is
// read once per chunk.  The chunk's inputs are staged in LDS one window of
// 16 steps (64 inputs) at a time for all four column tiles ([64][65]
// doubles, zero past the chunk and past 2 ncoef(p)); the window barriers
// leave the ring's reads in flight.  Column tiles past the chunk are skipped
// (a branch uniform over the block).  Row tiles past nrt repeat the last one
// and are not stored; steps past the order's own read a stored value and meet
// zero inputs.
constexpr int M2LS_RB = 3;   // row tiles per wave
constexpr int M2LS_WS = 16;  // steps per staged window
template <int NCH>
__global__ __launch_bounds__(256, 3) void k_m2l_stored(int p, int ncs, int nrt_s, int k4_s,
                                                    const int32_t *__restrict__ chunk_begin,
                                                    const int32_t *__restrict__ chunk_trans,
                                                    const int32_t *__restrict__ pair_sorted,
                                                    const int32_t *__restrict__ pairs, const double *__restrict__ ops,
                                                    const double *__restrict__ box_r,
                                                    const cplx<double> *__restrict__ M, cplx<double> *__restrict__ Y)
{
    typedef Acc4<double>::type acc_t;
    constexpr int RB = M2LS_RB, NT = 4, WS = M2LS_WS, PF = 4, ldb = 16 * NT + 1;
    constexpr int nwave = 4;  // launched with 256 threads
    static_assert(WS % PF == 0 && 4 * WS == 64, "a window is 64 inputs, whole ring groups");
    __shared__ double Bs[4 * WS * ldb];
    __shared__ int colbase[16 * NT];
    __shared__ double gsh[48];  // Stokes: c_S - c_T of the chunk's pairs
    const int nc = ncoef(p), Dp = 2 * nc, nsteps = (Dp + 3) / 4, nrt = (Dp + 15) / 16;
    const int c = blockIdx.x;
    const int u = chunk_trans[c], pb = chunk_begin[c];
    const int ncol = (chunk_begin[c + 1] - pb) * NCH, nct = (ncol + 15) / 16;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    if ((int)threadIdx.x < 16 * NT) {
        const int j = threadIdx.x;
        int cb = -1;
        if (j < ncol) {
            const int pl = j / NCH, ch = j - pl * NCH;
            cb = 2 * (pairs[2 * pair_sorted[pb + pl] + 1] * NCH + ch) * ncs;  // first real
        }
        colbase[j] = cb;
        if (NCH == 4 && j < 48) {
            const int pl = j / 3, xyz = j - 3 * pl;
            double g = 0;
            if (4 * pl < ncol) {
                const int pr = pair_sorted[pb + pl];
                g = box_r[5 * (int64_t)pairs[2 * pr + 1] + xyz] - box_r[5 * (int64_t)pairs[2 * pr] + xyz];
            }
            gsh[j] = g;
        }
    }
    __syncthreads();
    const double *Mr = reinterpret_cast<const double *>(M);
    const double *Au = ops + (int64_t)u * nrt_s * k4_s * 64 + lane;
    for (int rb0 = 0; rb0 < nrt; rb0 += nwave * RB) {  // the same trip count for every wave
        const double *At[RB];
#pragma unroll
        for (int i = 0; i < RB; ++i)
            At[i] = Au + (int64_t)min(rb0 + w + nwave * i, nrt - 1) * k4_s * 64;
        acc_t acc[RB][NT];
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
            for (int ct = 0; ct < NT; ++ct)
                acc[i][ct] = acc_t{0, 0, 0, 0};
        double ring[PF][RB];
#pragma unroll
        for (int j = 0; j < PF; ++j)
#pragma unroll
            for (int i = 0; i < RB; ++i)
                ring[j][i] = At[i][(int64_t)min(j, nsteps - 1) * 64];
        for (int w0 = 0; w0 < nsteps; w0 += WS) {
            __syncthreads();  // the previous window has been read
            // wave w stages columns 16 w .. 16 w + 15, eight reads at a time
            const int k = 4 * w0 + lane, kc = min(k, Dp - 1);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                int cb[8];
                double v[8];
#pragma unroll
                for (int c2 = 0; c2 < 8; ++c2)
                    cb[c2] = colbase[16 * w + 8 * h + c2];
#pragma unroll
                for (int c2 = 0; c2 < 8; ++c2)
                    v[c2] = Mr[max(cb[c2], 0) + kc];
#pragma unroll
                for (int c2 = 0; c2 < 8; ++c2)
                    Bs[lane * ldb + 16 * w + 8 * h + c2] = (cb[c2] >= 0 && k < Dp) ? v[c2] : 0.0;
            }
            __syncthreads();
            for (int j0 = 0; j0 < WS; j0 += PF) {
#pragma unroll
                for (int j = 0; j < PF; ++j) {
                    const int st = w0 + j0 + j;
                    const double *brow = Bs + (4 * (j0 + j) + lk) * ldb + li;
#pragma unroll
                    for (int ct = 0; ct < NT; ++ct) {
                        if (ct < nct) {
                            const double bv = brow[16 * ct];
#pragma unroll
                            for (int i = 0; i < RB; ++i)
                                acc[i][ct] = mfma_16x16x4(ring[j][i], bv, acc[i][ct]);
                        }
                    }
                    const int sn = min(st + PF, nsteps - 1);
#pragma unroll
                    for (int i = 0; i < RB; ++i)
                        ring[j][i] = At[i][(int64_t)sn * 64];
                }
            }
        }
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            const int rt = rb0 + w + nwave * i;
            if (rt >= nrt)
                continue;
#pragma unroll
            for (int ct = 0; ct < NT; ++ct) {
                if (ct >= nct)  // wave-uniform
                    break;
                const int col = ct * 16 + li;
                const int pl = col / NCH, ch = col - pl * NCH;
                double *dst = col < ncol
                                  ? reinterpret_cast<double *>(Y + ((int64_t)pair_sorted[pb + pl] * NCH + ch) * nc)
                                  : nullptr;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = rt * 16 + 4 * v + lk;  // FP64 output layout
                    double val = acc[i][ct][v];
                    if constexpr (NCH == 4) {
                        // the fourth channel moves its centre from c_S to c_T, from the
                        // pair's first three channels in the neighbouring lanes (every
                        // lane shuffles)
                        const int q0 = lane & ~3;
                        const double y0 = __shfl(val, q0), y1 = __shfl(val, q0 + 1), y2 = __shfl(val, q0 + 2);
                        if (ch == 3)
                            val += gsh[3 * pl] * y0 + gsh[3 * pl + 1] * y1 + gsh[3 * pl + 2] * y2;
                    }
                    if (col < ncol && row < Dp)
                        dst[row] = val;
                }
            }
        }
    }
}

// M2L by rotation: the translation of Sec. 2.5 in three O(p^3) steps per box
// pair instead of one O(p^4) product.  The multipole expansion is rotated so
// that the translation vector lies along +z (per degree n, a real
// 2 (n + 1) x 2 (n + 1) matrix of the direction, built on the host), translated
// along z, where order l couples only with order -l through the axis values
// I_j^0(d z) = j! / d^(j + 1), and the local expansion is rotated back.  The
// rotations depend only on the direction of the key, so keys of one direction
// share them.
//
// Block = chunk (pairs x channels of one key, at most 64 columns), taken in
// groups of 16 NT columns held in LDS as one [2 nc + 2][16 NT + 1] array (the
// two rows past the last degree are zero; the odd row stride keeps a wave's
// 64 rows of one column, as staged, on distinct banks, and leaves every
// matrix-core operand read an immediate offset from a per-lane base).  Each
// stage works in place: a wave owns whole degrees (whole orders in the axial
// stage), assigned longest first to the least loaded wave, so its writes
// follow only its own reads; the at most two rows past a degree that a 4-deep
// step reads meet zero operator entries.  Every operator value of a degree is
// read before its products.  Column tiles past the chunk are skipped.
// Scalings: the source's 2^(-eS n) when the rotated multipole is stored, the
// target's (-1)^k 2^(-eT (k + 1)) and the order's signs when the translated
// local expansion is stored.
constexpr int ROT_KA = 6;  // 4-deep steps of an order in the axial stage

__device__ __forceinline__ double scale2(double x, int e) { return ldexp(x, e); }
__device__ __forceinline__ float scale2(float x, int e) { return ldexpf(x, e); }

// degrees (or orders) of this wave: items n = hi .. 0, cost(n), assigned in
// that order to the least loaded of the NW waves (lowest index on ties)
template <int NW, typename F> __device__ __forceinline__ uint32_t rot_owned(int hi, int w, F cost)
{
    int ld[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j)
        ld[j] = 0;
    uint32_t mask = 0;
    for (int n = hi; n >= 0; --n) {
        const int c = cost(n);
        int wm = 0, mv = ld[0];
#pragma unroll
        for (int j = 1; j < NW; ++j)
            if (ld[j] < mv) {
                wm = j;
                mv = ld[j];
            }
#pragma unroll
        for (int j = 0; j < NW; ++j)
            ld[j] += wm == j ? c : 0;
        if (wm == w)
            mask |= 1u << n;
    }
    return mask;
}

__device__ __forceinline__ int rot_degree_cost(int n)
{
    const int S = 2 * (n + 1);
    return ((S + 15) >> 4) * ((S + 3) >> 2);
}

// rotate degree n in place: X_n <- A_n X_n (A_n from the direction's table T,
// lane order) on column tiles ct < nct, the result scaled by 2^es.  RTC row
// tiles and at most KMC 4-deep steps (the degree's class): every operator
// value of the degree is read first, with addresses clamped to its tiles and
// no guard, so that each product waits only for its own value
template <typename R, int NT, int RTC, int KMC>
__device__ __forceinline__ void rot_degree(int n, const R *__restrict__ T, R *X, int lane, int nct, int es)
{
    typedef typename Acc4<R>::type acc_t;
    constexpr int LD = 16 * NT + 1;
    const int li = lane & 15, lk = lane >> 4;
    int off = 0;
    for (int j = 0; j < n; ++j)
        off += rot_degree_cost(j);
    const int S = 2 * (n + 1), k4 = (S + 3) >> 2, base = n * (n + 1);
    R a[KMC][RTC];
#pragma unroll
    for (int kt = 0; kt < KMC; ++kt)
#pragma unroll
        for (int rt = 0; rt < RTC; ++rt)
            a[kt][rt] = T[((int64_t)off + rt * k4 + min(kt, k4 - 1)) * 64 + lane];
    acc_t acc[RTC][NT];
#pragma unroll
    for (int rt = 0; rt < RTC; ++rt)
#pragma unroll
        for (int ct = 0; ct < NT; ++ct)
            acc[rt][ct] = acc_t{0, 0, 0, 0};
    const R *Xl = X + (base + lk) * LD + li;
#pragma unroll
    for (int kt = 0; kt < KMC; ++kt) {
        if (kt < k4) {
            R b[NT];
#pragma unroll
            for (int ct = 0; ct < NT; ++ct)
                b[ct] = Xl[4 * kt * LD + 16 * ct];
#pragma unroll
            for (int rt = 0; rt < RTC; ++rt)
#pragma unroll
                for (int ct = 0; ct < NT; ++ct)
                    if (ct < nct)
                        acc[rt][ct] = mfma_16x16x4(a[kt][rt], b[ct], acc[rt][ct]);
        }
    }
    R *Xo = X + base * LD + li;
#pragma unroll
    for (int rt = 0; rt < RTC; ++rt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = 16 * rt + (sizeof(R) == 8 ? 4 * v + lk : 4 * lk + v);
            if (row < S)
#pragma unroll
                for (int ct = 0; ct < NT; ++ct)
                    if (ct < nct)
                        Xo[row * LD + 16 * ct] = scale2(acc[rt][ct][v], es);
        }
}

// rotate the degrees of mask in place, the result of degree n scaled by 2^(e n)
template <typename R, int NT>
__device__ __forceinline__ void rot_degrees(uint32_t mask, const R *__restrict__ T, R *X, int lane, int nct, int e)
{
    for (uint32_t mk = mask; mk;) {
        const int n = 31 - __builtin_clz(mk);
        mk &= ~(1u << n);
        if (n <= 7)
            rot_degree<R, NT, 1, 4>(n, T, X, lane, nct, e * n);
        else if (n <= 15)
            rot_degree<R, NT, 2, 8>(n, T, X, lane, nct, e * n);
        else
            rot_degree<R, NT, 3, 11>(n, T, X, lane, nct, e * n);
    }
}

// translate the orders l of mask along z in place: for k = l .. p,
//   L'_k^l = (-1)^(k + l) 2^(-eT (k + 1)) sum_{n = l .. p} g_{n + k} conj(M'_n^l),
// g_j = j! / d^(j + 1) (M' already scaled by 2^(-eS n))
template <typename R, int NT>
__device__ __forceinline__ void rot_axial(uint32_t mask, int p, const R *g, R *X, int lane, int nct, int eT)
{
    typedef typename Acc4<R>::type acc_t;
    constexpr int LD = 16 * NT + 1;
    const int li = lane & 15, lk = lane >> 4;
    for (uint32_t mk = mask; mk;) {
        const int l = 31 - __builtin_clz(mk);
        mk &= ~(1u << l);
        const int c = p + 1 - l, nrt = (c + 15) >> 4, k4 = (c + 3) >> 2;
        acc_t acc[2][2][NT];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int ri = 0; ri < 2; ++ri)
#pragma unroll
                for (int ct = 0; ct < NT; ++ct)
                    acc[rt][ri][ct] = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int kt = 0; kt < ROT_KA; ++kt) {
            if (kt >= k4)
                break;
            const int nn = l + 4 * kt + lk;
            const bool nv = nn <= p;
            const int ncl = nv ? nn : p;
            const R *Xr = X + (ncl * (ncl + 1) + 2 * l) * LD + li;
            R b[2][NT];
#pragma unroll
            for (int ri = 0; ri < 2; ++ri)
#pragma unroll
                for (int ct = 0; ct < NT; ++ct)
                    b[ri][ct] = Xr[ri * LD + 16 * ct];
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) {
                if (rt < nrt) {
                    const int ko = l + 16 * rt + li;
                    const bool ok = nv && ko <= p;
                    const R gv = g[ok ? ko + nn : 0];
                    const R a = ok ? gv : R(0);
#pragma unroll
                    for (int ri = 0; ri < 2; ++ri)
#pragma unroll
                        for (int ct = 0; ct < NT; ++ct)
                            if (ct < nct)
                                acc[rt][ri][ct] = mfma_16x16x4(a, b[ri][ct], acc[rt][ri][ct]);
                }
            }
        }
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
            if (rt >= nrt)
                break;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int ko = l + 16 * rt + (sizeof(R) == 8 ? 4 * v + lk : 4 * lk + v);
                if (ko <= p) {
                    const R sc = scale2(((ko + l) & 1) ? R(-1) : R(1), -eT * (ko + 1));
                    R *Xo = X + (ko * (ko + 1) + 2 * l) * LD + li;
#pragma unroll
                    for (int ct = 0; ct < NT; ++ct) {
                        if (ct < nct) {
                            Xo[16 * ct] = sc * acc[rt][0][ct][v];
                            Xo[LD + 16 * ct] = -sc * acc[rt][1][ct][v];
                        }
                    }
                }
            }
        }
    }
}

template <typename R, int NCH, int NT, int NW>
__global__ __launch_bounds__(64 * NW, NW / 2) void k_m2l_rot(int p, int ncs, int n_chunks, int per_xcd,
                                                 const int4 *__restrict__ hdr, const double *__restrict__ dist,
                                                 const int2 *__restrict__ cols, const double *__restrict__ gcs,
                                                 int64_t rot_per, const R *__restrict__ rotf,
                                                 const R *__restrict__ rotb, const cplx<R> *__restrict__ M,
                                                 cplx<R> *__restrict__ Y)
{
    constexpr int CW = 16 * NT, LD = CW + 1, CPW = CW / NW;
    // Stokes: column w + NW i of a group is channel w mod 4 (groups start at a
    // multiple of 4), so the waves w = 3 mod 4 write out the fourth channel of
    // every pair and move its centre from c_S to c_T there, from the pair's
    // first three channels: Y_3 + (c_S - c_T) . (Y_0, Y_1, Y_2)
    constexpr bool FIXC = NCH == 4;
    static_assert(NW % 4 == 0 && CW % NW == 0, "groups hold whole pairs, whole columns per wave");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    // consecutive positions of the order (one direction) on one XCD
    const int s = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
    if (s >= n_chunks)
        return;
    const int nc = ncoef(p), Dp = 2 * nc;
    R *g = reinterpret_cast<R *>(smem_raw);  // [2 p + 2]
    R *gc = g + 2 * p + 2;                   // [CW / 4][3] (Stokes)
    R *X = gc + (FIXC ? 3 * (CW / 4) : 0);   // [Dp + 2][LD]
    const int4 h = hdr[s];
    const int dir = h.x, eT = h.y & 255, eS = h.y >> 8, ncol = h.z;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const uint32_t dmask = rot_owned<NW>(p, w, rot_degree_cost);
    const uint32_t amask = rot_owned<NW>(p, w, [p](int l) {
        const int cl = p + 1 - l;
        return ((cl + 15) >> 4) * ((cl + 3) >> 2);
    });
    if (threadIdx.x == 0) {
        const double d = dist[s], id = 1.0 / d;
        double v = id;
        for (int j = 0; j <= 2 * p; ++j) {
            g[j] = (R)v;
            v *= (j + 1) * id;
        }
    }
    for (int t = threadIdx.x; t < 2 * LD; t += blockDim.x)
        X[Dp * LD + t] = R(0);
    const R *Tf = rotf + (int64_t)dir * rot_per, *Tb = rotb + (int64_t)dir * rot_per;
    const R *Mr = reinterpret_cast<const R *>(M);
    R *Yr = reinterpret_cast<R *>(Y);
    const int2 *cs = cols + (int64_t)s * M2L_CHUNK;
    for (int c0 = 0; c0 < ncol; c0 += CW) {
        const int nct = min(NT, (ncol - c0 + 15) >> 4);
        // wave w stages (and writes out) columns w, w + NW, ... of the group
        int2 cc[CPW];
#pragma unroll
        for (int i = 0; i < CPW; ++i)
            cc[i] = cs[c0 + w + NW * i];
        __syncthreads();  // the previous group written out
        if (FIXC && w == NW - 1 && lane < 3 * (CW / 4) && c0 + 4 * (lane / 3) < ncol)
            gc[lane] = (R)gcs[((int64_t)s * (M2L_CHUNK / 4) + (c0 >> 2)) * 3 + lane];
        // RB 64-row blocks of every column of the wave in flight together (at
        // most 32 reads: a wave holds at most 63 outstanding)
        constexpr int RB = CPW >= 32 ? 1 : 32 / CPW;
        for (int r0 = 0; r0 < Dp; r0 += 64 * RB) {
            R v[RB][CPW];
#pragma unroll
            for (int h = 0; h < RB; ++h) {
                const int rc = min(r0 + 64 * h + lane, Dp - 1);
#pragma unroll
                for (int i = 0; i < CPW; ++i)
                    v[h][i] = Mr[2 * (int64_t)(cc[i].x < 0 ? 0 : cc[i].x) * ncs + rc];
            }
#pragma unroll
            for (int h = 0; h < RB; ++h) {
                const int row = r0 + 64 * h + lane;
                if (row < Dp)
#pragma unroll
                    for (int i = 0; i < CPW; ++i)
                        X[row * LD + w + NW * i] = cc[i].x >= 0 ? v[h][i] : R(0);
            }
        }
        __syncthreads();
        rot_degrees<R, NT>(dmask, Tf, X, lane, nct, -eS);
        __syncthreads();
        rot_axial<R, NT>(amask, p, g, X, lane, nct, eT);
        __syncthreads();
        rot_degrees<R, NT>(dmask, Tb, X, lane, nct, 0);
        __syncthreads();
        for (int r0 = 0; r0 < Dp; r0 += 64) {
            const int row = r0 + lane;
            if (row < Dp) {
                const R *Xw = X + row * LD + w;
                if (FIXC && (w & 3) == 3) {
#pragma unroll
                    for (int i = 0; i < CPW; ++i) {
                        const R *gq = gc + 3 * ((w + NW * i) >> 2);
                        if (cc[i].y >= 0)
                            Yr[2 * (int64_t)cc[i].y * nc + row] = Xw[NW * i] + gq[0] * Xw[NW * i - 3] +
                                                                  gq[1] * Xw[NW * i - 2] + gq[2] * Xw[NW * i - 1];
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < CPW; ++i)
                        if (cc[i].y >= 0)
                            Yr[2 * (int64_t)cc[i].y * nc + row] = Xw[NW * i];
                }
            }
        }
    }
}

// LDS of k_m2l_rot
template <typename R, int NCH> size_t m2l_rot_shm(int p, int nt)
{
    return sizeof(R) * ((2 * (size_t)p + 2) + (NCH == 4 ? 12 * (size_t)nt : 0) +
                        (2 * (size_t)ncoef(p) + 2) * (16 * (size_t)nt + 1));
}

template <typename R> size_t m2l_mfma_shm(int p)
{
    const int q = 2 * p, Kp = (2 * ncoef(p) + 3) & ~3;
    return 2 * 64 * sizeof(int64_t) + 48 * sizeof(R) + sizeof(cplx<R>) * (size_t)(q + 1) * (q + 1) +
           sizeof(R) * 64 * (size_t)(std::min(Kp, 64) + 1) + sizeof(uint16_t) * (size_t)ncoef(p);
}

// The same pass 1 on the vector units, used for FP64 (where the generated
// operator is reused too little for the matrix cores to pay): lane = real
// output row r = (k, l, re/im) of one 64-row group; for PB pairs of the chunk
// at once (their coefficients wave-uniform, scalar loads) and every input
// (n, m), the lane forms its two operator entries (for a and b) from P and Q
// in LDS and adds them times (a, b) of each pair; Horner in n applies the
// 2^(-eS n) scaling.  Stokes: a lane holds the four channels of each pair's
// row, so it moves the fourth channel's centre from c_S to c_T as it writes,
// Y_3 + (c_S - c_T) . (Y_0, Y_1, Y_2), from the rounded Y values (the same
// arithmetic as in the sum of Y, which then leaves it out).
template <typename R> __device__ inline R mul_rn(R a, R b);
template <> __device__ inline double mul_rn<double>(double a, double b) { return __dmul_rn(a, b); }
template <> __device__ inline float mul_rn<float>(float a, float b) { return __fmul_rn(a, b); }

template <typename R, int NCH, int PB>
__global__ __launch_bounds__(256) void k_m2l_valu(int p, int ncs, int q_tab, const int32_t *__restrict__ chunk_begin,
                                                  const int32_t *__restrict__ chunk_trans,
                                                  const uint64_t *__restrict__ trans_key,
                                                  const int32_t *__restrict__ pair_sorted,
                                                  const int32_t *__restrict__ pairs, const cplx<R> *__restrict__ table,
                                                  const double *__restrict__ box_r, const cplx<R> *__restrict__ M,
                                                  cplx<R> *__restrict__ Y)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int q = 2 * p;
    const int fq = (q + 1) * (q + 1), nc = ncoef(p), Dp = 2 * nc;
    cplx<R> *It = reinterpret_cast<cplx<R> *>(smem_raw);
    const int c = blockIdx.x;
    const int u = chunk_trans[c], pb = chunk_begin[c], pe = chunk_begin[c + 1];
    const uint64_t key = trans_key[u];
    const int eT = (int)((key >> 48) & 63), eS = (int)((key >> 54) & 63);
    const cplx<R> *tab = table + (int64_t)u * (q_tab + 1) * (q_tab + 1);
    for (int t = threadIdx.x; t < fq; t += blockDim.x)
        It[t] = tab[t];
    __syncthreads();
    const int nwave = blockDim.x >> 6;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const R rS = (R)ldexp(1.0, -eS);
    const int ngrp = (Dp + 63) / 64, nbat = (pe - pb + PB - 1) / PB;
    for (int task = wv; task < ngrp * nbat; task += nwave) {
        const int g = task % ngrp, base = pb + (task / ngrp) * PB;
        const int r = g * 64 + lane;
        const bool active = r < Dp;
        int k = 0, l = 0;
        idx_to_nm(active ? r >> 1 : 0, k, l);
        const bool po = (r & 1) != 0;
        const R f = (R)ldexp((k & 1) ? -1.0 : 1.0, -eT * (k + 1));
        const cplx<R> *Mb[PB];
#pragma unroll
        for (int j = 0; j < PB; ++j) {
            const int e = base + j < pe ? base + j : base;  // a short batch repeats its first pair
            // wave-uniform: the coefficients come through the scalar cache
            const int S = __builtin_amdgcn_readfirstlane(pairs[2 * pair_sorted[e] + 1]);
            Mb[j] = M + (int64_t)S * NCH * ncs;
        }
        R acc[PB][NCH];
#pragma unroll
        for (int j = 0; j < PB; ++j)
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
                acc[j][ch] = 0;
        for (int n = p; n >= 0; --n) {
#pragma unroll
            for (int j = 0; j < PB; ++j)
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch)
                    acc[j][ch] *= rS;
            const cplx<R> *row = It + (n + k) * (n + k + 1) + l;  // I_{n+k}^{l + .}
#pragma unroll 2
            for (int m = 0; m <= n; ++m) {
                const cplx<R> P = row[m];
                R qr = 0, qi = 0;
                if (m > 0) {
                    const cplx<R> Q = row[-m];
                    const R sg = (m & 1) ? R(-1) : R(1);
                    qr = sg * Q.re;
                    qi = sg * Q.im;
                }
                // entries for a (re part of the input) and b (im part)
                const R ea = po ? P.im + qi : P.re + qr;
                const R eb = po ? P.re - qr : qi - P.im;
                const int ci = cidx(n, m);
#pragma unroll
                for (int j = 0; j < PB; ++j)
#pragma unroll
                    for (int ch = 0; ch < NCH; ++ch) {
                        const cplx<R> x = Mb[j][ch * ncs + ci];
                        acc[j][ch] += ea * x.re;
                        acc[j][ch] += eb * x.im;
                    }
            }
        }
        if (!active)
            continue;
#pragma unroll
        for (int j = 0; j < PB; ++j) {
            if (base + j >= pe)
                continue;
            const int orig = pair_sorted[base + j];
            R y[NCH];
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
                y[ch] = mul_rn(f, acc[j][ch]);
            if constexpr (NCH == 4) {
                const double *cS = box_r + 5 * (int64_t)pairs[2 * orig + 1], *cT = box_r + 5 * (int64_t)pairs[2 * orig];
                const R g0 = (R)(cS[0] - cT[0]), g1 = (R)(cS[1] - cT[1]), g2 = (R)(cS[2] - cT[2]);
                y[3] += g0 * y[0] + g1 * y[1] + g2 * y[2];
            }
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
                reinterpret_cast<R *>(Y + ((int64_t)orig * NCH + ch) * nc)[r] = y[ch];
        }
    }
}

// Pass 2: L(T) = sum of Y over T's pairs (CSR order), all boxes; block =
// (box, chunk of 256 outputs), thread = (pair slice, output), slices summed
// in a fixed order.  (Stokes: every M2L kernel has already moved the fourth
// channel of each pair from c_S to c_T.)
template <typename R, int NCH>
__global__ __launch_bounds__(256) void k_m2l_reduce(int p, int ncs, const int32_t *__restrict__ order,
                                                    const int32_t *__restrict__ ptr,
                                                    const cplx<R> *__restrict__ Y, cplx<R> *__restrict__ L)
{
    __shared__ cplx<R> red[256];
    const int T = order[blockIdx.x];  // boxes with the most pairs first
    const int nc = ncoef(p), no = NCH * nc;
    const int e0 = ptr[T], e1 = ptr[T + 1];
    {
        const int o0 = blockIdx.y * (int)blockDim.x;  // this block's outputs: o0 .. o0 + span - 1
        const int span = min((int)blockDim.x, no - o0);
        const int sl = threadIdx.x / span, t = o0 + threadIdx.x % span;
        const int nsl_here = max(1, (int)blockDim.x / span);
        const int ch = t / nc, idx = t - ch * nc;
        R sr = 0, si = 0;
        if (sl < nsl_here) {
            // U reads issued together (clamped to the last pair, the extra
            // ones dropped), then added in pair order
            constexpr int U = 8;
            for (int e = e0 + sl; e < e1; e += U * nsl_here) {
                cplx<R> v[U];
                int64_t ee[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    ee[u] = min(e + u * nsl_here, e1 - 1);
                    v[u] = Y[ee[u] * no + t];
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if (e + u * nsl_here < e1) {
                        sr += v[u].re;
                        si += v[u].im;
                    }
            }
        }
        __syncthreads();
        red[threadIdx.x] = cplx<R>{sr, si};
        __syncthreads();
        if ((int)threadIdx.x < span) {
            R ar = 0, ai = 0;
            for (int k = 0; k < nsl_here; ++k) {
                ar += red[k * span + threadIdx.x].re;
                ai += red[k * span + threadIdx.x].im;
            }
            L[((int64_t)T * NCH + ch) * ncs + idx] = cplx<R>{ar, ai};
        }
    }
}

// ---------------------------------------------------------------------------
// The combine of a mat-vec for sorted target i: y[perm i] = pref (near +
// far + sum_e S_ie x_e) over the correction entries e of row i, plus x / 2
// for the second-kind operator; yf holds the far field of the target.
// With ycorr the correction's product S x is already there (k_corr_spmv, by
// sorted target) and the entries are not visited again.
struct CombineArgs {
    const int32_t *perm, *cptr, *ccol;
    const double *cval, *x, *ynear;
    double pref;
    double *y;
    const double *ycorr;
};

template <int KIND>
__device__ inline void combine_target(const CombineArgs &A, int64_t i, const double *yf)
{
    const int64_t o = A.perm[i];
    if constexpr (KIND != FMMBEM_STOKES_SL) {
        double acc = A.ynear[i] + yf[0];
        if (A.ycorr)
            acc += A.ycorr[i];
        else
            for (int e = A.cptr[i]; e < A.cptr[i + 1]; ++e)
                acc += A.cval[e] * A.x[A.ccol[e]];
        A.y[o] = KIND == FMMBEM_LAPLACE_DL ? 0.5 * A.x[o] + A.pref * acc : A.pref * acc;
    } else if (A.ycorr) {
        A.y[3 * o] = A.pref * ((A.ynear[3 * i] + yf[0]) + A.ycorr[3 * i]);
        A.y[3 * o + 1] = A.pref * ((A.ynear[3 * i + 1] + yf[1]) + A.ycorr[3 * i + 1]);
        A.y[3 * o + 2] = A.pref * ((A.ynear[3 * i + 2] + yf[2]) + A.ycorr[3 * i + 2]);
    } else {
        double a0 = A.ynear[3 * i] + yf[0], a1 = A.ynear[3 * i + 1] + yf[1], a2 = A.ynear[3 * i + 2] + yf[2];
        for (int e = A.cptr[i]; e < A.cptr[i + 1]; ++e) {
            const int64_t jo = A.ccol[e];
            const double *v = A.cval + 9 * (int64_t)e;
            const double t0 = A.x[3 * jo], t1 = A.x[3 * jo + 1], t2 = A.x[3 * jo + 2];
            a0 += (v[0] * t0 + v[1] * t1) + v[2] * t2;
            a1 += (v[3] * t0 + v[4] * t1) + v[5] * t2;
            a2 += (v[6] * t0 + v[7] * t1) + v[8] * t2;
        }
        A.y[3 * o] = A.pref * a0;
        A.y[3 * o + 1] = A.pref * a1;
        A.y[3 * o + 2] = A.pref * a2;
    }
}

// The correction's product yc = S x by sorted target (S: the near-singular
// and self corrections, CSR by sorted target, columns in caller order; 1 or
// 3 x 3 values per entry, FP64 or their FP32 copy, the products summed in
// FP64).  Sixteen lanes per row take its entries in turn;
// the lanes' sums are joined by a fixed butterfly, so the result does not
// depend on the launch.  Launched where the far-field stream would otherwise
// wait for the near field, so that the combine reads one value per component.
template <int NQ, typename V>
__global__ __launch_bounds__(256) void k_corr_spmv(int64_t nt, const int32_t *__restrict__ ptr,
                                                   const int32_t *__restrict__ col, const V *__restrict__ val,
                                                   const double *__restrict__ x, double *__restrict__ yc)
{
    const int64_t i = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
    const int l = threadIdx.x & 15;
    double a[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        a[q] = 0.0;
    if (i < nt) {
        const int c1 = ptr[i + 1];
        for (int e = ptr[i] + l; e < c1; e += 16) {
            const int64_t jo = col[e];
            if constexpr (NQ == 1) {
                a[0] += (double)val[e] * x[jo];
            } else {
                const V *v = val + 9 * (int64_t)e;
                const double t0 = x[3 * jo], t1 = x[3 * jo + 1], t2 = x[3 * jo + 2];
                a[0] += ((double)v[0] * t0 + (double)v[1] * t1) + (double)v[2] * t2;
                a[1] += ((double)v[3] * t0 + (double)v[4] * t1) + (double)v[5] * t2;
                a[2] += ((double)v[6] * t0 + (double)v[7] * t1) + (double)v[8] * t2;
            }
        }
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1)
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            a[q] += __shfl_xor(a[q], off, 16);
    if (l == 0 && i < nt)
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            yc[NQ * i + q] = a[q];
}

// the correction's values that a mat-vec of precision R reads
template <typename R> const R *corr_values(const Correction &C);
template <> const double *corr_values<double>(const Correction &C) { return C.val; }
template <> const float *corr_values<float>(const Correction &C) { return C.val32; }

// combine_target for one channel with the target's inputs already read:
// o = perm[i], its near field yn, its correction range [c0, c1) and (double
// layer) its input xo; the same arithmetic
template <int KIND>
__device__ inline void combine_target_pre(const CombineArgs &A, int64_t o, double yn, int c0, int c1, double xo,
                                          double yf)
{
    static_assert(KIND != FMMBEM_STOKES_SL, "one channel");
    double acc = yn + yf;
    for (int e = c0; e < c1; ++e)
        acc += A.cval[e] * A.x[A.ccol[e]];
    A.y[o] = KIND == FMMBEM_LAPLACE_DL ? 0.5 * xo + A.pref * acc : A.pref * acc;
}

// The scaled regular harmonics R_n^m(x, y, z), 0 <= m <= n <= p, of one
// point, in the order m = 0..p, n = m..p: f(index of (n, m), weight * Re,
// weight * Im), the weight 2 for m > 0 standing for the -m term of a real
// field (column recurrence in n on the diagonal R_m^m).
template <typename R, typename F>
__device__ __forceinline__ void sweep_regular(int p, R x, R y, R z, F &&f)
{
    const R r2 = x * x + y * y + z * z;
    R dre = 1, dim = 0;  // R_m^m
    for (int m = 0; m <= p; ++m) {
        if (m > 0) {
            R g = -inv_int<R>(2 * m);
            R a = g * (x * dre - y * dim), bb = g * (x * dim + y * dre);
            dre = a;
            dim = bb;
        }
        const R wgt = m == 0 ? R(1) : R(2);
        R cr = dre, ci = dim, pr = 0, pi = 0;
        for (int n = m; n <= p; ++n) {
            if (n > m) {
                R g = inv_int<R>((n - m) * (n + m));
                R a = R(2 * n - 1) * z;
                R nr = (a * cr - r2 * pr) * g, ni = (a * ci - r2 * pi) * g;
                pr = cr;
                pi = ci;
                cr = nr;
                ci = ni;
            }
            f(cidx(n, m), n, wgt * cr, wgt * ci);
        }
    }
}

// a target's position relative to the centre c of its leaf, in units of the
// leaf half-size s (FP32: from the leaf-relative copy)
template <typename R>
__device__ __forceinline__ void target_rel(int64_t i, int64_t nt, double s, const double *c,
                                           const double *__restrict__ tc, const float *__restrict__ tc32, R &x,
                                           R &y, R &z)
{
    if constexpr (sizeof(R) == 8) {
        double is = 1.0 / s;
        x = (tc[i] - c[0]) * is;
        y = (tc[nt + i] - c[1]) * is;
        z = (tc[2 * nt + i] - c[2]) * is;
    } else {
        float is = (float)(1.0 / s);
        x = tc32[i] * is;
        y = tc32[nt + i] * is;
        z = tc32[2 * nt + i] * is;
    }
}

// L2P: one block per leaf; lane t of every wave takes targets t, t + 64, ...
// and the four waves split the columns m of the regular harmonics (wave w
// takes m = 4 b + w for even b and 4 b + 3 - w for odd b, near equal shares
// of the (n, m) pairs), each running the diagonal recurrence to its own
// columns.  The waves' partial sums are added in wave order through LDS and
// wave 0 combines the target's far field with its near field (joined before
// the launch).  With FAR (the low orders, where the near field takes longer
// than the far chain) the far field of every target goes to yfar in sorted
// order and a separate combine joins it with the near field, so that L2P
// itself does not wait for the near field; otherwise L2P combines.
// Stokes needs the gradients of the four local expansions as well: the
// gradient of sum L_n^m R_n^m is the expansion of order p - 1 with
//   d/dz: L_{j+1}^k,  d/dx: (L_{j+1}^{k-1} - L_{j+1}^{k+1}) / 2,
//   d/dy: (i/2) (L_{j+1}^{k-1} + L_{j+1}^{k+1}),
// formed at each (j, k) from the three neighbours of degree j + 1
// (L_{j+1}^{-1} = -conj(L_{j+1}^1)).  The leaf's expansions sit in LDS
// channel-fastest, so that one coefficient's reads share one base address.
// Dynamic LDS: l2p_shm.
constexpr int L2P_WAVES = 4;

template <typename R, int KIND> constexpr int l2p_nacc()
{
    return KIND == FMMBEM_STOKES_SL ? 3 + 12 : 1;
}

template <typename R, int KIND> size_t l2p_shm(int p)
{
    constexpr int NCH = KIND == FMMBEM_STOKES_SL ? 4 : 1;
    return sizeof(cplx<R>) * NCH * (size_t)ncoef(p) + sizeof(R) * (L2P_WAVES - 1) * l2p_nacc<R, KIND>() * 64;
}

template <typename R, int KIND, bool FAR>
__global__ __launch_bounds__(64 * L2P_WAVES, 3) void k_l2p(int p, int ncs, const int32_t *__restrict__ leaves,
                                                        const int32_t *__restrict__ box_i,
                                                        const double *__restrict__ box_r, double side, int64_t nt,
                                                        const double *__restrict__ tc,
                                                        const float *__restrict__ tc32,
                                                        const cplx<R> *__restrict__ L, CombineArgs ca,
                                                        double *__restrict__ yfar)
{
    constexpr bool STOKES = KIND == FMMBEM_STOKES_SL;
    constexpr int NCH = STOKES ? 4 : 1;
    constexpr int NV = STOKES ? 3 : 1;  // potentials evaluated
    constexpr int NA = l2p_nacc<R, KIND>();  // potentials, then gradients (channel x direction)
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int nc = ncoef(p);
    cplx<R> *E = reinterpret_cast<cplx<R> *>(smem_raw);                   // [nc][NCH]
    R *red = reinterpret_cast<R *>(smem_raw + sizeof(cplx<R>) * NCH * nc);  // [L2P_WAVES - 1][NA][64]
    const int b = leaves[blockIdx.x];
    const int lv = box_i[6 * b], tb = box_i[6 * b + 1], te = box_i[6 * b + 2];
    const double s = ldexp(side, -(lv + 1));
    const double *c = box_r + 5 * (int64_t)b;
    const cplx<R> *Lb = L + (int64_t)b * NCH * ncs;
    for (int t = threadIdx.x; t < NCH * nc; t += blockDim.x) {
        const int ch = t / nc, id = t - ch * nc;
        E[id * NCH + ch] = Lb[(int64_t)ch * ncs + id];
    }
    __syncthreads();
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    for (int i0 = tb; i0 < te; i0 += 64) {
        const int i = i0 + lane;
        const bool live = i < te;
        R x = 0, y = 0, z = 0;
        if (live)
            target_rel<R>(i, nt, s, c, tc, tc32, x, y, z);
        R acc[NA];
#pragma unroll
        for (int a = 0; a < NA; ++a)
            acc[a] = 0;
        const R r2 = x * x + y * y + z * z;
        R dre = 1, dim = 0;  // R_md^md
        int md = 0;
        for (int bk = 0;; ++bk) {
            const int m = 4 * bk + ((bk & 1) ? L2P_WAVES - 1 - w : w);
            if (m > p)
                break;
            for (; md < m; ++md) {
                const R g = -inv_int<R>(2 * (md + 1));
                const R ar = g * (x * dre - y * dim), ai = g * (x * dim + y * dre);
                dre = ar;
                dim = ai;
            }
            const R wgt = m == 0 ? R(1) : R(2);
            R cr = dre, ci = dim, pr = 0, pi = 0;
            for (int n = m; n <= p; ++n) {
                if (n > m) {
                    const R g = inv_int<R>((n - m) * (n + m));
                    const R az = R(2 * n - 1) * z;
                    const R nr = (az * cr - r2 * pr) * g, ni = (az * ci - r2 * pi) * g;
                    pr = cr;
                    pi = ci;
                    cr = nr;
                    ci = ni;
                }
                const R wr = wgt * cr, wi = wgt * ci;
                const cplx<R> *e0 = E + cidx(n, m) * NCH;
                cplx<R> v[NV];
#pragma unroll
                for (int a = 0; a < NV; ++a)
                    v[a] = e0[a];
                if constexpr (STOKES) {
                    if (n < p) {
                        // (n + 1, m - 1 .. m + 1); at m = 0 the first is folded from the third
                        const cplx<R> *e1 = E + cidx(n + 1, m) * NCH;
                        cplx<R> ea[4], ez[4], eb[4];
#pragma unroll
                        for (int ch = 0; ch < 4; ++ch) {
                            ea[ch] = e1[ch - NCH];
                            ez[ch] = e1[ch];
                            eb[ch] = e1[ch + NCH];
                        }
                        const R hr = R(0.5) * wr, hi = R(0.5) * wi;
#pragma unroll
                        for (int ch = 0; ch < 4; ++ch) {
                            const R are = m == 0 ? -eb[ch].re : ea[ch].re, aim = m == 0 ? eb[ch].im : ea[ch].im;
                            const R dr = are - eb[ch].re, di = aim - eb[ch].im;
                            const R sr = are + eb[ch].re, si = aim + eb[ch].im;
                            R *g = acc + NV + 3 * ch;
                            g[0] += dr * hr;
                            g[0] += di * hi;
                            g[1] += sr * hi;
                            g[1] -= si * hr;
                            g[2] += ez[ch].re * wr;
                            g[2] += ez[ch].im * wi;
                        }
                    }
                }
#pragma unroll
                for (int a = 0; a < NV; ++a) {
                    acc[a] += v[a].re * wr;
                    acc[a] += v[a].im * wi;
                }
            }
        }
        // the waves' partial sums, added in wave order
        if (w > 0) {
#pragma unroll
            for (int a = 0; a < NA; ++a)
                red[((w - 1) * NA + a) * 64 + lane] = acc[a];
        }
        __syncthreads();
        if (w == 0 && live) {
#pragma unroll
            for (int v = 0; v < L2P_WAVES - 1; ++v)
#pragma unroll
                for (int a = 0; a < NA; ++a)
                    acc[a] += red[(v * NA + a) * 64 + lane];
            if constexpr (!STOKES) {
                const double yf = (double)acc[0] / s;
                if constexpr (FAR)
                    yfar[i] = yf;
                else
                    combine_target<KIND>(ca, i, &yf);
            } else {
                const double is = 1.0 / s, is2 = is * is;
                const double xr[3] = {(double)x * s, (double)y * s, (double)z * s};  // x - c
                double yf[3];
                for (int dir = 0; dir < 3; ++dir) {
                    double u = (double)acc[dir] * is;
                    for (int a = 0; a < 3; ++a)
                        u -= xr[a] * (double)acc[NV + 3 * a + dir] * is2;
                    u += (double)acc[NV + 9 + dir] * is2;
                    yf[dir] = u;
                }
                if constexpr (FAR) {
                    for (int dir = 0; dir < 3; ++dir)
                        yfar[3 * i + dir] = yf[dir];
                } else {
                    combine_target<KIND>(ca, i, yf);
                }
            }
        }
        __syncthreads();  // red is rewritten by the next targets
    }
}

// ---------------------------------------------------------------------------
// P2P: one block per work unit (at most 64 targets of one leaf).  The
// NW waves of the block take the unit's source chunks round robin.  With n
// targets a wave runs P = floor(64 / n) phases: lane (ph, t) sums over the
// sources ph, ph + P, ... of the chunk, so that a small leaf still fills the
// wave.  A wave stages its chunk into its own LDS tile phase-major (phase ph's
// sources contiguous) and pads each phase to the same length with zero-charge
// sources placed far away, so every lane runs the same trip count; the next
// chunk is fetched into registers while the current one is evaluated.  The
// partial sums of the waves and phases are reduced in a fixed order, in FP64.
// FP32 works in leaf-relative coordinates: r = (t - c_T) + (c_T - c_S) - (y - c_S).
constexpr int P2P_WAVES = 8;

template <typename R, bool STOKES> __device__ __forceinline__ Src<R, STOKES> far_zero_source()
{
    // at 1e18 from every target r^2 ~ 3e36 stays finite in FP32 and the
    // contribution is an exact zero
    Src<R, STOKES> v;
    v.x = v.y = v.z = R(1e18);
    if constexpr (STOKES) {
        v.f0 = v.f1 = v.f2 = 0;
        v.pad0 = v.pad1 = 0;
    } else {
        v.q = 0;
    }
    return v;
}

template <typename R, int KIND, bool SELF>
__device__ __forceinline__ void p2p_phase(const Src<R, vec_src<KIND>()> *__restrict__ row, int nj, int k, int kstep,
                                          int i, R px, R py, R pz, R *acc)
{
#pragma unroll 4
    for (int j = 0; j < nj; ++j) {
        const Src<R, vec_src<KIND>()> sv = row[j];
        const R dx = px - sv.x, dy = py - sv.y, dz = pz - sv.z;
        const R r2 = dx * dx + dy * dy + dz * dz;
        R rinv;
        if constexpr (sizeof(R) == 8) {
            // hardware estimate (documented to 2^29 ulp, a relative error of
            // 2^-23) refined by one Newton step y (3/2 - r2 y^2 / 2), which
            // squares the relative error (times 3/2): about 2^-45 (r2 is
            // finite and > 0 for every pair the result keeps; the self pair
            // is masked below)
            double y = __builtin_amdgcn_rsq(r2);
            y = y * (1.5 - (0.5 * r2) * (y * y));
            rinv = y;
        } else {
            rinv = __builtin_amdgcn_rsqf(r2);
        }
        if constexpr (SELF) {
            rinv = (k >> 2) == i ? R(0) : rinv;  // the target's own panel: integrated by the correction
            k += kstep;
        }
        if constexpr (KIND == FMMBEM_LAPLACE_SL) {
            acc[0] += sv.q * rinv;
        } else if constexpr (KIND == FMMBEM_STOKES_SL) {
            // f / r + d (d . f) / r^3 = (f + d q) / r with q = (d . f) / r^2:
            // two fused multiply-adds per component, straight into acc
            const R q = (dx * sv.f0 + dy * sv.f1 + dz * sv.f2) * (rinv * rinv);
            acc[0] += rinv * (sv.f0 + dx * q);
            acc[1] += rinv * (sv.f1 + dy * q);
            acc[2] += rinv * (sv.f2 + dz * q);
        } else {  // dipole w x n: (w x n) . (t - y) / r^3
            acc[0] += (dx * sv.f0 + dy * sv.f1 + dz * sv.f2) * (rinv * rinv * rinv);
        }
    }
}

template <typename R, int KIND>
__global__ __launch_bounds__(64 * P2P_WAVES) void k_p2p(XcdGroups xg, const int4 *__restrict__ units,
                                                        const int2 *__restrict__ chunks,
                                                        const float4 *__restrict__ choff, int64_t nt,
                                                        const double *__restrict__ tc, const float *__restrict__ tc32,
                                                        const Src<R, vec_src<KIND>()> *__restrict__ src,
                                                        const int32_t *__restrict__ dst, double *__restrict__ part,
                                                        double *__restrict__ ynear)
{
    static_assert(P2P_TILE == 128, "two staged sources per lane");
    constexpr bool VS = vec_src<KIND>();
    constexpr int NQ = KIND == FMMBEM_STOKES_SL ? 3 : 1;
    __shared__ Src<R, VS> tile[P2P_WAVES][P2P_TILE];
    __shared__ R red[P2P_WAVES][NQ][64];
    // blocks are dealt to the 8 XCDs round robin; XCD x runs the units of
    // its group (consecutive units, which share source leaves in its L2)
    const int x = (int)(blockIdx.x % 8);
    const int g = xg.b[x] + (int)(blockIdx.x / 8);
    if (g >= xg.b[x + 1])
        return;
    const int4 u = units[g];
    const int tb = u.x, n = u.y - u.x;  // 1 <= n <= 64; chunks hold at most (128 / P) P sources
    const int P = 64 / n;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int ph = lane / n, tl = lane - ph * n;
    const bool active = ph < P;
    const int i = tb + tl;  // < tb + n for every lane
    R tx, ty, tz;
    if constexpr (sizeof(R) == 8) {
        tx = tc[i];
        ty = tc[nt + i];
        tz = tc[2 * nt + i];
    } else {
        tx = tc32[i];
        ty = tc32[nt + i];
        tz = tc32[2 * nt + i];
    }
    R acc[NQ];
#pragma unroll
    for (int a = 0; a < NQ; ++a)
        acc[a] = 0;
    Src<R, VS> *my = tile[w];
    // staged slots of this lane: t = lane and t = lane + 64, at phase t % P, position t / P
    const int ta = lane, tb2 = lane + 64;
    const int pa = ta / P, qa = ta - pa * P;
    const int pb = tb2 / P, qb = tb2 - pb * P;
    int c = u.z + w;
    int2 ch = make_int2(0, 0);
    Src<R, VS> ra = far_zero_source<R, VS>(), rb = ra;
    if (c < u.w) {
        ch = chunks[c];
        const int cnt = ch.y & 0xffff;
        if (ta < cnt)
            ra = src[ch.x + ta];
        if (tb2 < cnt)
            rb = src[ch.x + tb2];
    }
    while (c < u.w) {
        const int k0 = ch.x, cnt = ch.y & 0xffff;
        const bool self = (ch.y >> 16) != 0;
        const int nj = (cnt + P - 1) / P;  // P * nj <= 128
        // the wave's reads of its previous tile are issued before these writes
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (ta < P * nj)
            my[qa * nj + pa] = ra;  // slots past cnt keep the far zero source
        if (tb2 < P * nj)
            my[qb * nj + pb] = rb;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        R px = tx, py = ty, pz = tz;
        if constexpr (sizeof(R) == 4) {
            const float4 o = choff[c];
            px += o.x;
            py += o.y;
            pz += o.z;
        }
        // fetch the next chunk while this one is evaluated
        const int cn = c + P2P_WAVES;
        if (cn < u.w) {
            ch = chunks[cn];
            const int cnt2 = ch.y & 0xffff;
            ra = far_zero_source<R, VS>();
            rb = ra;
            if (ta < cnt2)
                ra = src[ch.x + ta];
            if (tb2 < cnt2)
                rb = src[ch.x + tb2];
        }
        if (active) {
            if (self)
                p2p_phase<R, KIND, true>(my + ph * nj, nj, k0 + ph, P, i, px, py, pz, acc);
            else
                p2p_phase<R, KIND, false>(my + ph * nj, nj, 0, 0, i, px, py, pz, acc);
        }
        c = cn;
    }
#pragma unroll
    for (int a = 0; a < NQ; ++a)
        red[w][a][lane] = active ? acc[a] : R(0);
    __syncthreads();
    // a whole unit writes its targets' sums, a piece of one its partial slot
    const int slot = dst[g];
    double *out = slot < 0 ? ynear + (int64_t)NQ * tb : part + (int64_t)slot * 3 * 64;
    for (int e = threadIdx.x; e < NQ * n; e += 64 * P2P_WAVES) {
        const int a = e / n, tt = e - a * n;
        double sum = 0.0;
        for (int v = 0; v < P2P_WAVES; ++v)
            for (int q = 0; q < P; ++q)
                sum += (double)red[v][a][q * n + tt];
        out[NQ * tt + a] = sum;
    }
}

// The targets of units cut into pieces: the pieces' partial sums added in
// piece order (one block per cut unit).
template <int NQ>
__global__ __launch_bounds__(256) void k_p2p_pieces(const int4 *__restrict__ splits, const double *__restrict__ part,
                                                    double *__restrict__ ynear)
{
    const int4 r = splits[blockIdx.x];  // first target, count, first slot, pieces
    for (int e = threadIdx.x; e < NQ * r.y; e += blockDim.x) {
        double sum = 0.0;
        for (int j = 0; j < r.w; ++j)
            sum += part[(int64_t)(r.z + j) * 3 * 64 + e];
        ynear[(int64_t)NQ * r.x + e] = sum;
    }
}

// The downward pass of one leaf in one block, for one channel at the low
// orders: the local expansion of a box is its own M2L sum (written by the
// reduce) plus the L2L of its parent's.  The block follows the leaf's chain of
// ancestors (from its record, built with the tree) down from the coarsest M2L
// target level, with the ancestors' own sums and the octant operators of the
// chain staged in LDS (every leaf recomputes its ancestors: at these orders
// that costs less than one launch per level), then evaluates the leaf's local
// expansion at its targets and combines as L2P does; a thread's first
// target's inputs are read at the start, beside the chain's.  Dynamic LDS: sizeof(R) ((nc_max - 1) D^2 +
// (nc_max + 1) D) for chains of at most nc_max boxes, D = 2 ncoef(p).
template <typename R, int KIND>
__global__ __launch_bounds__(256) void k_down_leaf(int p, int ncs, int opd, const R *__restrict__ l2l_op,
                                                   const int32_t *__restrict__ leaf_rec,
                                                   const double *__restrict__ box_r, double side, int64_t nt,
                                                   const double *__restrict__ tc, const float *__restrict__ tc32,
                                                   const cplx<R> *__restrict__ L, CombineArgs ca)
{
    static_assert(KIND != FMMBEM_STOKES_SL, "one channel");
    constexpr int MAXC = DOWN_LEAF_MAXC;
    constexpr int U = 8;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int rec[LEAF_REC];
    const int D = 2 * ncoef(p), DD = D * D;
    const int tid = threadIdx.x;
    if (tid < LEAF_REC)
        rec[tid] = leaf_rec[(int64_t)blockIdx.x * LEAF_REC + tid];
    __syncthreads();
    const int tb = rec[0], te = rec[1], lv = rec[2], nch = rec[3], octs = rec[4 + MAXC];
    const int b = rec[4];
    const double s = ldexp(side, -(lv + 1));
    const double *cb = box_r + 5 * (int64_t)b;
    // this thread's first target: its inputs are read now, beside the chain's
    const int64_t i0 = tb + tid, ic = i0 < te ? i0 : (tb < te ? tb : 0);  // a valid index to read
    R x0, y0, z0;
    target_rel<R>(ic, nt, s, cb, tc, tc32, x0, y0, z0);
    const int64_t o0 = ca.perm[ic];
    const double yn0 = ca.ycorr ? ca.ynear[ic] + ca.ycorr[ic] : ca.ynear[ic];
    const int c00 = ca.ycorr ? 0 : ca.cptr[ic], c01 = ca.ycorr ? 0 : ca.cptr[ic + 1];
    const double xo0 = KIND == FMMBEM_LAPLACE_DL ? ca.x[o0] : 0.0;
    R *own = reinterpret_cast<R *>(smem_raw);  // [nch][D]
    R *ts = own + nch * D;                     // [nch - 1][D][D]: chain[c + 1] into chain[c], input-major
    R *acc = ts + (nch - 1) * DD;              // [D]: the local expansion walked down the chain
    {
        const R *Lr = reinterpret_cast<const R *>(L);
        for (int d = tid; d < nch * D; d += blockDim.x) {
            const int c = d / D;
            own[d] = Lr[(int64_t)rec[4 + c] * 2 * ncs + (d - c * D)];
        }
        // operator entries U at a time per thread, unguarded at clamped indices
        const int ne = (nch - 1) * DD;
        for (int e0 = 0; e0 < ne; e0 += U * (int)blockDim.x) {
            R v[U];
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int e = min(e0 + j * (int)blockDim.x + tid, ne - 1);
                const int c = e / DD, rem = e - c * DD, k = rem / D, r = rem - k * D;
                const int o = (octs >> (3 * c)) & 7;
                v[j] = l2l_op[((int64_t)o * opd + k) * opd + r];
            }
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int e = e0 + j * (int)blockDim.x + tid;
                if (e < ne)
                    ts[e] = v[j];
            }
        }
    }
    __syncthreads();
    for (int d = tid; d < D; d += blockDim.x)
        acc[d] = own[(nch - 1) * D + d];
    __syncthreads();
    for (int c = nch - 2; c >= 0; --c) {
        R v = 0;
        if (tid < D) {
            const R *t = ts + c * DD + tid;
            v = own[c * D + tid];
            for (int k = 0; k < D; ++k)
                v += t[k * D] * acc[k];
        }
        __syncthreads();
        if (tid < D)
            acc[tid] = v;
        __syncthreads();
    }
    const cplx<R> *V = reinterpret_cast<const cplx<R> *>(acc);
    if (i0 < te) {
        R pot = 0;
        sweep_regular<R>(p, x0, y0, z0, [&](int id, int, R wr, R wi) { pot += V[id].re * wr + V[id].im * wi; });
        combine_target_pre<KIND>(ca, o0, yn0, c00, c01, xo0, (double)pot / s);
    }
    for (int64_t i = i0 + blockDim.x; i < te; i += blockDim.x) {  // leaves of more than 256 targets
        R x, y, z;
        target_rel<R>(i, nt, s, cb, tc, tc32, x, y, z);
        R pot = 0;
        sweep_regular<R>(p, x, y, z, [&](int id, int, R wr, R wi) { pot += V[id].re * wr + V[id].im * wi; });
        const double yf = (double)pot / s;
        combine_target<KIND>(ca, i, &yf);
    }
}

// LDS of k_down_leaf for chains of at most nc_max boxes at order p; 0 where
// the fused downward pass does not apply (more than DOWN_LEAF_MAXC boxes, or
// more than 48 KiB, or more than 256 rows)
template <typename R> size_t down_leaf_shm(int p, int nc_max)
{
    const size_t D = 2 * (size_t)ncoef(p);
    if (nc_max < 1 || nc_max > DOWN_LEAF_MAXC || D > 256)
        return 0;
    const size_t b = sizeof(R) * ((size_t)(nc_max - 1) * D * D + (size_t)(nc_max + 1) * D);
    return b <= 48 * 1024 ? b : 0;
}

// ---------------------------------------------------------------------------
// combine without a far field (no accepted box pair): y_far is zero
template <int KIND>
__global__ void k_combine(int64_t nt, CombineArgs ca, const double *__restrict__ yfar)
{
    constexpr int NQ = KIND == FMMBEM_STOKES_SL ? 3 : 1;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nt)
        combine_target<KIND>(ca, i, yfar + NQ * i);
}

// charges of this mat-vec on st (for P2M, and the sorted input of the stored
// near field); ev_fork marks them
template <typename R, int KIND>
void launch_charges(fmmbem_ctx *ctx, const double *x, hipStream_t st, const NormIn &nz)
{
    constexpr bool VS = vec_src<KIND>();
    constexpr int SO = sizeof(R) == 8 ? 0 : 5;  // stage offset of this precision
    Tree &T = ctx->tree;
    Geometry &G = ctx->geo;
    const int64_t nt = ctx->nt, ns = ctx->nsrc;
    Src<R, VS> *src = static_cast<Src<R, VS> *>(ctx->charges);
    hipEvent_t ev;
    if (ctx->side_pending)  // the charges buffer may still be read on the side stream (P2P, or P2M)
        FB_HIP(hipStreamWaitEvent(st, ctx->ev_join, 0));

    stage_begin(ctx, SO + 4, st, &ev);
    // normalising: read w, write x = w / |w|; else read x
    k_charges<R, KIND><<<grid_for(ns, DOT_BLOCK), DOT_BLOCK, 0, st>>>(
        nt, T.perm, G.sp, G.sp32, G.nrm, nz.partn ? nz.w : x, src, ctx->nearm.v64 ? ctx->nearm.xs : nullptr, nz,
        const_cast<double *>(x));
    FB_HIP(hipGetLastError());
    stage_end(ctx, SO + 4, st, ev);
    FB_HIP(hipEventRecord(ctx->ev_fork, st));
}

// the near field (P2P, or the stored near-field product) on stream ns: on the
// side stream once the charges marked by ev_fork are written (ev_join marks
// its end), or on the stream of the charges themselves
template <typename R, int KIND>
void launch_near(fmmbem_ctx *ctx, hipStream_t ns, const double *x)
{
    const bool on_side = ns == ctx->side;
    constexpr bool STOKES = KIND == FMMBEM_STOKES_SL;
    constexpr bool VS = vec_src<KIND>();
    constexpr int SO = sizeof(R) == 8 ? 0 : 5;  // stage offset of this precision
    Tree &T = ctx->tree;
    Geometry &G = ctx->geo;
    const int64_t nt = ctx->nt;
    Src<R, VS> *src = static_cast<Src<R, VS> *>(ctx->charges);
    hipEvent_t ev;
    // a wait on an event that has completed costs the host next to nothing,
    // one on a pending event about as much as several kernel launches
    if (on_side)
        FB_HIP(hipStreamWaitEvent(ns, ctx->ev_fork, 0));
    stage_begin(ctx, SO + 0, ns, &ev);
    if (ctx->nearm.v64) {
        // stored near field: 2 flops per matrix entry
        launch_near_stored(ctx, sizeof(R) == 8 ? FMMBEM_FP64 : FMMBEM_FP32, ns);
        stage_end(ctx, SO + 0, ns, ev, 2.0 * (STOKES ? 9.0 : 1.0) * (double)ctx->nearm.entries);
    } else {
        if (T.n_unit > 0) {
            k_p2p<R, KIND><<<8 * T.p2p_xcd.max_count(), 64 * P2P_WAVES, 0, ns>>>(
                T.p2p_xcd, T.p2p_unit, T.p2p_chunk, T.p2p_choff, nt, G.tc, G.tc32, src, T.p2p_dst, T.p2p_part,
                ctx->y_near);
            FB_HIP(hipGetLastError());
            if (T.n_split > 0) {
                constexpr int NQ = STOKES ? 3 : 1;
                k_p2p_pieces<NQ><<<T.n_split, 256, 0, ns>>>(T.p2p_split, T.p2p_part, ctx->y_near);
                FB_HIP(hipGetLastError());
            }
        }
        // source-target pairs actually evaluated: all P2P pairs minus the 4 self points of each target
        const double fl = STOKES ? 30.0 : KIND == FMMBEM_LAPLACE_DL ? 18.0 : 12.0;
        stage_end(ctx, SO + 0, ns, ev, fl * (double)(T.p2p_interactions - 4 * nt));
    }
    // on the side stream the correction product S x follows the near field
    // there, off the far chain (which is then the longer branch)
    const Correction &C = ctx->prm.near_stored ? ctx->nearm.rest : ctx->corr;
    ctx->corr_on_near = on_side && C.nnz > 0;
    if (ctx->corr_on_near) {
        constexpr int NQ = STOKES ? 3 : 1;
        k_corr_spmv<NQ><<<grid_for(nt, 16), 256, 0, ns>>>(nt, C.ptr, C.col_orig, corr_values<R>(C), x, ctx->y_corr);
        FB_HIP(hipGetLastError());
    }
    if (on_side) {
        FB_HIP(hipEventRecord(ctx->ev_join, ns));
        ctx->side_pending = true;
    }
}

// The upward pass of order p on st: P2M of every leaf, then M2M level by level
// (deepest first), from the charges that the near-field launch wrote before
// it.  Coefficient (n, m) of every multipole does not depend on the order of
// the pass (P2M computes each order on its own; M2M takes a parent's order n
// from children's orders <= n only), so a pass of order p serves every later
// M2L of order <= p.
template <typename R, int KIND>
void up_pass(fmmbem_ctx *ctx, int p, hipStream_t st)
{
    constexpr bool STOKES = KIND == FMMBEM_STOKES_SL;
    constexpr int NCH = STOKES ? 4 : 1;
    constexpr bool VS = vec_src<KIND>();
    constexpr int SO = sizeof(R) == 8 ? 0 : 5;  // stage offset of this precision
    Tree &T = ctx->tree;
    const int ncs = ncoef(ctx->prm.p_max);
    const double side = T.cube[3];
    Src<R, VS> *src = static_cast<Src<R, VS> *>(ctx->charges);
    cplx<R> *M = static_cast<cplx<R> *>(ctx->M);
    hipEvent_t ev;
    stage_begin(ctx, SO + 2, st, &ev);
    {
        const int nsl = 256 / (p + 1);
        const size_t shm = sizeof(cplx<R>) * (size_t)nsl * ncoef(p) + sizeof(Src<R, VS>) * P2M_TILE;
        if constexpr (KIND == FMMBEM_LAPLACE_DL) {
            if (p <= 4)
                k_p2m_dipole<R, 4><<<T.nleaf, 256, shm, st>>>(p, ncs, T.leaves, T.box_i, T.box_r, side, src, M);
            else if (p <= 8)
                k_p2m_dipole<R, 8><<<T.nleaf, 256, shm, st>>>(p, ncs, T.leaves, T.box_i, T.box_r, side, src, M);
            else if (p <= 12)
                k_p2m_dipole<R, 12><<<T.nleaf, 256, shm, st>>>(p, ncs, T.leaves, T.box_i, T.box_r, side, src, M);
            else if (p <= 16)
                k_p2m_dipole<R, 16><<<T.nleaf, 256, shm, st>>>(p, ncs, T.leaves, T.box_i, T.box_r, side, src, M);
            else
                k_p2m_dipole<R, 20><<<T.nleaf, 256, shm, st>>>(p, ncs, T.leaves, T.box_i, T.box_r, side, src, M);
        } else {
            if (p <= 4)
                k_p2m<R, NCH, 4><<<T.nleaf, 256, shm, st>>>(p, ncs, T.leaves, T.box_i, T.box_r, side, src, M);
            else if (p <= 8)
                k_p2m<R, NCH, 8><<<T.nleaf, 256, shm, st>>>(p, ncs, T.leaves, T.box_i, T.box_r, side, src, M);
            else if (NCH == 1 && p <= 12)  // one channel: the column sweep still fits (160 VGPRs in FP64)
                k_p2m<R, NCH, 12><<<T.nleaf, 256, shm, st>>>(p, ncs, T.leaves, T.box_i, T.box_r, side, src, M);
            else
                k_p2m_tile<R, NCH><<<T.nleaf, 256, p2m_tile_shm<R, NCH>(p), st>>>(p, ncs, T.leaves, T.box_i, T.box_r,
                                                                                side, src, M);
        }
        FB_HIP(hipGetLastError());
    }
    const M2LPlan &P = ctx->m2l;
    const R *m2m_op;
    if constexpr (sizeof(R) == 8)
        m2m_op = P.m2m64;
    else
        m2m_op = P.m2m32;
    const int row_chunks = (2 * ncoef(p) + 63) / 64;
    cplx<R> *Z = static_cast<cplx<R> *>(P.Z);
    // children of level l into parents of level l - 1, deepest first; levels
    // above the coarsest M2L source are never read
    for (int l = T.nlevels - 1; l >= 1 && l - 1 >= P.lmin_src; --l) {
        const int t0 = P.tile_begin[l], ntile = P.tile_begin[l + 1] - t0;
        const int q0 = P.par_begin[l - 1], npar = P.par_begin[l] - q0;
        if (ntile == 0 || npar == 0)
            continue;
        k_octant_mfma<R, NCH, false><<<dim3(ntile, row_chunks), 256, octant_mfma_shm<R>(p), st>>>(p, ncs, P.op_dim, m2m_op, P.tiles, t0,
                                                                  P.level_list, T.box_i, T.box_r, M, Z);
        FB_HIP(hipGetLastError());
        k_m2m_sum<R, NCH><<<grid_for((int64_t)npar * NCH * ncoef(p), 256), 256, 0, st>>>(
            p, ncs, npar, P.parents + q0, T.box_i, Z, M);
        FB_HIP(hipGetLastError());
    }
    stage_end(ctx, SO + 2, st, ev);
}

// The far field of order p on st, P2M through L2P (without the upward pass
// when have_up: multipoles of order >= p already computed on st), from the
// charges that the near-field launch wrote before it; st joins the side stream before L2P,
// which combines far and near field into y.  Without a far field: y_far = 0,
// join and combine.
// the correction's product into ctx->y_corr on st (see k_corr_spmv)
template <typename R, int KIND>
void corr_spmv(fmmbem_ctx *ctx, const CombineArgs &ca, hipStream_t st)
{
    if (!ca.ycorr || ctx->corr_on_near)  // none, or already behind the near field
        return;
    constexpr int NQ = KIND == FMMBEM_STOKES_SL ? 3 : 1;
    const Correction &C = ctx->prm.near_stored ? ctx->nearm.rest : ctx->corr;
    k_corr_spmv<NQ><<<grid_for(ctx->nt, 16), 256, 0, st>>>(ctx->nt, ca.cptr, ca.ccol, corr_values<R>(C), ca.x,
                                                           ctx->y_corr);
    FB_HIP(hipGetLastError());
}

// the widest column group within the LDS budget (FP64: 32 or 16 columns, two
// blocks on a CU; FP32: 64 or 32 columns, at least three); four waves: blocks
// of eight waves (fewer, larger blocks per CU) measured slower in FP32
template <typename R, int NCH>
void launch_m2l_rot(fmmbem_ctx *ctx, int p, const cplx<R> *M, cplx<R> *Y, hipStream_t st)
{
    const M2LPlan &P = ctx->m2l;
    const int ncs = ncoef(ctx->prm.p_max);
    const int per = (P.n_chunks + 7) / 8;
    constexpr int NTW = sizeof(R) == 8 ? 2 : 4, NW = 4;
    constexpr size_t budget = sizeof(R) == 8 ? 80 * 1024 : 48 * 1024;
    const R *rf, *rb;
    if constexpr (sizeof(R) == 8) {
        rf = P.rot64_f;
        rb = P.rot64_b;
    } else {
        rf = P.rot32_f;
        rb = P.rot32_b;
    }
    FB_REQUIRE(p <= 20, FMMBEM_EINVAL, "rotation M2L beyond its order limit");
    if (m2l_rot_shm<R, NCH>(p, NTW) <= budget)
        k_m2l_rot<R, NCH, NTW, NW><<<8 * per, 64 * NW, m2l_rot_shm<R, NCH>(p, NTW), st>>>(
            p, ncs, P.n_chunks, per, P.rot_hdr, P.rot_dist, P.rot_cols, P.rot_gc, P.rot_per, rf, rb, M, Y);
    else
        k_m2l_rot<R, NCH, NTW / 2, NW><<<8 * per, 64 * NW, m2l_rot_shm<R, NCH>(p, NTW / 2), st>>>(
            p, ncs, P.n_chunks, per, P.rot_hdr, P.rot_dist, P.rot_cols, P.rot_gc, P.rot_per, rf, rb, M, Y);
}

template <typename R, int KIND>
void far_chain(fmmbem_ctx *ctx, int p, const CombineArgs &ca, hipStream_t st, bool have_up, bool swap)
{
    // the chain runs on fs: the main stream st, or with swap (near field on
    // st) the side stream, whose far field the combine on st joins
    constexpr bool STOKES = KIND == FMMBEM_STOKES_SL;
    constexpr int NCH = STOKES ? 4 : 1;
    constexpr int SO = sizeof(R) == 8 ? 0 : 5;  // stage offset of this precision
    Tree &T = ctx->tree;
    Geometry &G = ctx->geo;
    const int64_t nt = ctx->nt;
    const int ncs = ncoef(ctx->prm.p_max);
    const double side = T.cube[3];
    cplx<R> *M = static_cast<cplx<R> *>(ctx->M);
    cplx<R> *L = static_cast<cplx<R> *>(ctx->L);
    hipEvent_t ev;
    const hipStream_t fs = swap ? ctx->side : st;

    if (T.n_m2l > 0) {
        if (swap && !have_up)
            FB_HIP(hipStreamWaitEvent(fs, ctx->ev_fork, 0));  // the charges
        if (!have_up)
            up_pass<R, KIND>(ctx, p, fs);
        const M2LPlan &P = ctx->m2l;
        const R *l2l_op;
        if constexpr (sizeof(R) == 8)
            l2l_op = P.l2l64;
        else
            l2l_op = P.l2l32;
        const bool rot = P.rot64_f && p >= ROT_MIN_P;
        const int row_chunks = (2 * ncoef(p) + 63) / 64;

        stage_begin(ctx, SO + 1, fs, &ev);
        {
            const cplx<R> *table;
            if constexpr (sizeof(R) == 8)
                table = P.table64;
            else
                table = P.table32;
            cplx<R> *Y = static_cast<cplx<R> *>(ctx->Y);
            if (rot) {
                launch_m2l_rot<R, NCH>(ctx, p, M, Y, fs);
            } else if constexpr (sizeof(R) == 4) {
                // one wave per 16-row tile up to four tiles (the low orders of the
                // relaxed iterations: no wave idles, one tile's accumulators per
                // wave), else four waves of up to four tiles each
                const int nrt = (2 * ncoef(p) + 15) / 16;
                FB_REQUIRE(nrt <= 16, FMMBEM_EINVAL, "FP32 M2L beyond its order limit");
                if (nrt <= 4)
                    k_m2l_mfma<R, NCH, 1><<<P.n_chunks, 64 * nrt, m2l_mfma_shm<R>(p), fs>>>(
                        p, ncs, P.q, P.chunk_begin, P.chunk_trans, P.trans_key, P.pair_sorted, T.m2l_pairs, table,
                        T.box_r, M, Y);
                else
                    k_m2l_mfma<R, NCH, 4><<<P.n_chunks, 256, m2l_mfma_shm<R>(p), fs>>>(
                        p, ncs, P.q, P.chunk_begin, P.chunk_trans, P.trans_key, P.pair_sorted, T.m2l_pairs, table,
                        T.box_r, M, Y);
            } else if (P.ops64) {
                k_m2l_stored<NCH><<<P.n_chunks, 256, 0, fs>>>(p, ncs, P.ops_nrt, P.ops_k4, P.chunk_begin,
                                                               P.chunk_trans, P.pair_sorted, T.m2l_pairs, P.ops64,
                                                               T.box_r, M, Y);
            } else {
                constexpr int PB = NCH == 1 ? 8 : 2;
                const size_t shm = sizeof(cplx<R>) * (size_t)(2 * p + 1) * (2 * p + 1);
                k_m2l_valu<R, NCH, PB><<<P.n_chunks, 256, shm, fs>>>(
                    p, ncs, P.q, P.chunk_begin, P.chunk_trans, P.trans_key, P.pair_sorted, T.m2l_pairs, table,
                    T.box_r, M, Y);
            }
            FB_HIP(hipGetLastError());
        }
        // flops per box pair and channel: the direct path counts the
        // method's complex O(p^4) translation of Sec. 2.5, 4 (p + 1)^3 (p + 2)
        // (its kernels apply it as a real (2 nc) x (2 nc) operator, 8 nc^2
        // flops); the rotation path what it applies, two real rotations of
        // 8 (n + 1)^2 flops per degree and the axial step of 4 (p + 1 - l)^2
        // per order: 20 sum_{m <= p + 1} m^2
        const double q1 = p + 1.0;
        const double fl = rot ? 20.0 * q1 * (p + 2.0) * (2.0 * p + 3.0) / 6.0 : 4.0 * q1 * q1 * q1 * (p + 2.0);
        stage_end(ctx, SO + 1, fs, ev, fl * NCH * (double)T.n_m2l);

        // the downward pass: the per-target sum of the M2L terms, then L2L and L2P
        stage_begin(ctx, SO + 3, fs, &ev);
        {
            cplx<R> *Y = static_cast<cplx<R> *>(ctx->Y);
            k_m2l_reduce<R, NCH><<<dim3(T.nbox, (NCH * ncoef(p) + 255) / 256), 256, 0, fs>>>(p, ncs, P.reduce_order,
                                                                                          T.m2l_ptr, Y, L);
            FB_HIP(hipGetLastError());
        }
        // one channel at the low orders: L2L down each leaf's chain of
        // ancestors (levels from the coarsest M2L target on) and L2P in one
        // block per leaf, where the chain and its operators fit in LDS
        bool fused = false;
        if constexpr (NCH == 1) {
            FB_REQUIRE(!swap, FMMBEM_EINTERNAL, "one channel keeps the near field on the side stream");
            const size_t dshm = down_leaf_shm<R>(p, std::max(1, T.nlevels - std::max(P.lmin_tgt, 0)));
            if (dshm > 0) {
                corr_spmv<R, KIND>(ctx, ca, st);  // while the near field may still run
                FB_HIP(hipStreamWaitEvent(st, ctx->ev_join, 0));  // the combine needs the near field
                k_down_leaf<R, KIND><<<T.nleaf, 256, dshm, st>>>(p, ncs, P.op_dim, l2l_op, P.leaf_rec, T.box_r,
                                                                 side, nt, G.tc, G.tc32, L, ca);
                FB_HIP(hipGetLastError());
                fused = true;
            }
        }
        if (!fused) {
            // parents of level l - 1 into children of level l; levels above the
            // coarsest M2L target hold no local expansion
            for (int l = std::max(1, P.lmin_tgt + 1); l < T.nlevels; ++l) {
                const int t0 = P.tile_begin[l], ntile = P.tile_begin[l + 1] - t0;
                if (ntile == 0)
                    continue;
                k_octant_mfma<R, NCH, true><<<dim3(ntile, row_chunks), 256, octant_mfma_shm<R>(p), fs>>>(
                    p, ncs, P.op_dim, l2l_op, P.tiles, t0, P.level_list, T.box_i, T.box_r, L, L);
                FB_HIP(hipGetLastError());
            }
            corr_spmv<R, KIND>(ctx, ca, fs);  // while the near field may still run
            const size_t lshm = l2p_shm<R, KIND>(p);
            if (swap || p <= L2P_FAR_MAX_P) {
                // the far field while the near field may still run, then the combine
                k_l2p<R, KIND, true><<<T.nleaf, 64 * L2P_WAVES, lshm, fs>>>(p, ncs, T.leaves, T.box_i, T.box_r, side,
                                                                           nt, G.tc, G.tc32, L, ca, ctx->y_far);
                FB_HIP(hipGetLastError());
                if (swap) {  // the far field ends the side stream's work; the combine on st joins it
                    stage_end(ctx, SO + 3, fs, ev);
                    ev = nullptr;
                    FB_HIP(hipEventRecord(ctx->ev_join, fs));
                    ctx->side_pending = true;
                }
                FB_HIP(hipStreamWaitEvent(st, ctx->ev_join, 0));
                k_combine<KIND><<<grid_for(nt, 64), 64, 0, st>>>(nt, ca, ctx->y_far);
            } else {
                FB_HIP(hipStreamWaitEvent(st, ctx->ev_join, 0));  // L2P combines with the near field
                k_l2p<R, KIND, false><<<T.nleaf, 64 * L2P_WAVES, lshm, st>>>(p, ncs, T.leaves, T.box_i, T.box_r, side,
                                                                            nt, G.tc, G.tc32, L, ca, nullptr);
            }
            FB_HIP(hipGetLastError());
        }
        stage_end(ctx, SO + 3, fs, ev);
    } else {
        FB_REQUIRE(!swap, FMMBEM_EINTERNAL, "no far field to run on the side stream");
        hipEvent_t ev4;
        stage_begin(ctx, SO + 4, st, &ev4);
        fill_zero(ctx->y_far, ctx->n, st);
        corr_spmv<R, KIND>(ctx, ca, st);
        FB_HIP(hipStreamWaitEvent(st, ctx->ev_join, 0));
        k_combine<KIND><<<grid_for(nt, 64), 64, 0, st>>>(nt, ca, ctx->y_far);
        FB_HIP(hipGetLastError());
        stage_end(ctx, SO + 4, st, ev4);
    }
}

void far_dispatch(fmmbem_ctx *ctx, int p, int prec, const CombineArgs &ca, hipStream_t st, bool have_up, bool swap)
{
    const int kind = ctx->kernel;
    if (prec == FMMBEM_FP64) {
        if (kind == FMMBEM_STOKES_SL)
            far_chain<double, FMMBEM_STOKES_SL>(ctx, p, ca, st, have_up, swap);
        else if (kind == FMMBEM_LAPLACE_DL)
            far_chain<double, FMMBEM_LAPLACE_DL>(ctx, p, ca, st, have_up, swap);
        else
            far_chain<double, FMMBEM_LAPLACE_SL>(ctx, p, ca, st, have_up, swap);
    } else {
        if (kind == FMMBEM_STOKES_SL)
            far_chain<float, FMMBEM_STOKES_SL>(ctx, p, ca, st, have_up, swap);
        else if (kind == FMMBEM_LAPLACE_DL)
            far_chain<float, FMMBEM_LAPLACE_DL>(ctx, p, ca, st, have_up, swap);
        else
            far_chain<float, FMMBEM_LAPLACE_SL>(ctx, p, ca, st, have_up, swap);
    }
}

void up_dispatch(fmmbem_ctx *ctx, int p, int prec, hipStream_t st)
{
    const int kind = ctx->kernel;
    if (prec == FMMBEM_FP64) {
        if (kind == FMMBEM_STOKES_SL)
            up_pass<double, FMMBEM_STOKES_SL>(ctx, p, st);
        else if (kind == FMMBEM_LAPLACE_DL)
            up_pass<double, FMMBEM_LAPLACE_DL>(ctx, p, st);
        else
            up_pass<double, FMMBEM_LAPLACE_SL>(ctx, p, st);
    } else {
        if (kind == FMMBEM_STOKES_SL)
            up_pass<float, FMMBEM_STOKES_SL>(ctx, p, st);
        else if (kind == FMMBEM_LAPLACE_DL)
            up_pass<float, FMMBEM_LAPLACE_DL>(ctx, p, st);
        else
            up_pass<float, FMMBEM_LAPLACE_SL>(ctx, p, st);
    }
}

void charges_dispatch(fmmbem_ctx *ctx, int prec, const double *x, hipStream_t st, const NormIn &nz = NormIn{})
{
    const int kind = ctx->kernel;
    if (prec == FMMBEM_FP64) {
        if (kind == FMMBEM_STOKES_SL)
            launch_charges<double, FMMBEM_STOKES_SL>(ctx, x, st, nz);
        else if (kind == FMMBEM_LAPLACE_DL)
            launch_charges<double, FMMBEM_LAPLACE_DL>(ctx, x, st, nz);
        else
            launch_charges<double, FMMBEM_LAPLACE_SL>(ctx, x, st, nz);
    } else {
        if (kind == FMMBEM_STOKES_SL)
            launch_charges<float, FMMBEM_STOKES_SL>(ctx, x, st, nz);
        else if (kind == FMMBEM_LAPLACE_DL)
            launch_charges<float, FMMBEM_LAPLACE_DL>(ctx, x, st, nz);
        else
            launch_charges<float, FMMBEM_LAPLACE_SL>(ctx, x, st, nz);
    }
}

void near_dispatch(fmmbem_ctx *ctx, int prec, hipStream_t ns, const double *x)
{
    const int kind = ctx->kernel;
    if (prec == FMMBEM_FP64) {
        if (kind == FMMBEM_STOKES_SL)
            launch_near<double, FMMBEM_STOKES_SL>(ctx, ns, x);
        else if (kind == FMMBEM_LAPLACE_DL)
            launch_near<double, FMMBEM_LAPLACE_DL>(ctx, ns, x);
        else
            launch_near<double, FMMBEM_LAPLACE_SL>(ctx, ns, x);
    } else {
        if (kind == FMMBEM_STOKES_SL)
            launch_near<float, FMMBEM_STOKES_SL>(ctx, ns, x);
        else if (kind == FMMBEM_LAPLACE_DL)
            launch_near<float, FMMBEM_LAPLACE_DL>(ctx, ns, x);
        else
            launch_near<float, FMMBEM_LAPLACE_SL>(ctx, ns, x);
    }
}

}  // namespace

bool near_on_main(const fmmbem_ctx *ctx, int p, int prec)
{
    return ctx->kernel == FMMBEM_STOKES_SL && !ctx->prm.near_stored && prec == FMMBEM_FP32 && p <= L2P_FAR_MAX_P &&
           ctx->tree.n_m2l > 0 && ctx->tree.n_unit > 0;
}

void prefetch_charges(fmmbem_ctx *ctx, int prec, const double *x, hipStream_t st, const NormIn &nz, bool near_main)
{
    charges_dispatch(ctx, prec, x, st, nz);
    ctx->spec_x = x;
    ctx->spec_prec = prec;
    ctx->spec_up_p = -1;
    ctx->spec_near = false;
    ctx->spec_swap = near_main && ctx->kernel == FMMBEM_STOKES_SL && !ctx->prm.near_stored && ctx->tree.n_m2l > 0;
}

void prefetch_near(fmmbem_ctx *ctx, hipStream_t st)
{
    FB_REQUIRE(ctx->spec_x != nullptr, FMMBEM_EINTERNAL, "near field prefetched without the charges");
    near_dispatch(ctx, ctx->spec_prec, ctx->spec_swap ? st : ctx->side, ctx->spec_x);
    ctx->spec_near = true;
}

void prefetch_up(fmmbem_ctx *ctx, int prec, int p_up, hipStream_t st)
{
    FB_REQUIRE(ctx->spec_x != nullptr && ctx->spec_prec == prec, FMMBEM_EINTERNAL,
               "upward pass prefetched without the charges");
    FB_REQUIRE(p_up >= 1 && p_up <= ctx->prm.p_max && (prec == FMMBEM_FP64 || p_up <= P_MAX_FP32),
               FMMBEM_EINVAL, "upward pass order out of range");
    if (ctx->tree.n_m2l > 0) {
        if (ctx->spec_swap) {  // on the side stream, where the far chain will follow it
            FB_HIP(hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0));
            up_dispatch(ctx, p_up, prec, ctx->side);
            FB_HIP(hipEventRecord(ctx->ev_join, ctx->side));
            ctx->side_pending = true;
        } else {
            up_dispatch(ctx, p_up, prec, st);
        }
        ctx->spec_up_p = p_up;
    }
}

void run_matvec(fmmbem_ctx *ctx, int p, int prec, const double *x, double *y, hipStream_t st)
{
    const int kind = ctx->kernel;
    // charges prefetched for exactly this input and precision are used as
    // they are, and so are the multipoles of an upward pass prefetched with
    // them at an order >= p; anything else is dropped
    const bool have_charges = ctx->spec_x == x && ctx->spec_prec == prec;
    const bool have_up = have_charges && ctx->spec_up_p >= p;
    const bool have_near = have_charges && ctx->spec_near;
    // the order of the streams: as prefetched, else chosen here
    const bool swap = have_charges ? ctx->spec_swap : near_on_main(ctx, p, prec);
    ctx->spec_x = nullptr;
    ctx->spec_prec = -1;
    ctx->spec_up_p = -1;
    ctx->spec_near = false;
    ctx->spec_swap = false;
    bool up_here = false;
    if (!have_charges) {
        charges_dispatch(ctx, prec, x, st);  // (joins the side stream first if it still runs)
        // the upward pass before the near field's fork, as the prefetch
        // orders them: the host's wait on the still pending fork event then
        // no longer delays its launches (the GPU is full either way while
        // both run, so this gains only that delay)
        if (!swap && ctx->tree.n_m2l > 0) {
            up_dispatch(ctx, p, prec, st);
            up_here = true;
        }
    } else {
        (void)hipEventQuery(ctx->ev_fork);  // refresh its state: usually complete by now
    }
    if (!have_near)
        near_dispatch(ctx, prec, swap ? st : ctx->side, x);
    // stored near field: its blocks already hold the corrections of their pairs
    const Correction &C = ctx->prm.near_stored ? ctx->nearm.rest : ctx->corr;
    const double pref = kind == FMMBEM_STOKES_SL   ? -1.0 / (8.0 * M_PI * ctx->prm.mu)
                        : kind == FMMBEM_LAPLACE_DL ? -1.0 / (4.0 * M_PI)
                                                    : 1.0 / (4.0 * M_PI);
    const CombineArgs ca{ctx->tree.perm, C.ptr, C.col_orig, C.val, x, ctx->y_near, pref, y,
                         C.nnz > 0 ? ctx->y_corr : nullptr};
    far_dispatch(ctx, p, prec, ca, st, have_up || up_here, swap);  // ends with the join and the combine on st
    ctx->side_pending = false;
    ctx->corr_on_near = false;
}

void build_m2l_operators(fmmbem_ctx *ctx, hipStream_t st)
{
    M2LPlan &P = ctx->m2l;
    if (P.n_trans == 0)
        return;
    const int Dp = 2 * ncoef(ctx->prm.p_max);
    P.ops_nrt = (Dp + 15) / 16;
    P.ops_k4 = (Dp + 3) / 4;
    const int64_t per = (int64_t)P.ops_nrt * P.ops_k4 * 64;
    P.ops64 = ctx->arena.alloc<double>((size_t)per * P.n_trans);
    P.ops_bytes = (int64_t)sizeof(double) * per * P.n_trans;
    k_m2l_opgen<<<dim3(P.n_trans, P.ops_nrt), 256, 0, st>>>(ctx->prm.p_max, P.q, P.ops_nrt, P.ops_k4, P.trans_key,
                                                           P.table64, P.ops64);
    FB_HIP(hipGetLastError());
}

}  // namespace fmmbem
