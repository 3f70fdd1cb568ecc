// Rotation operators for the M2L pass by rotation (Sec. 2.5's translation
// done as rotate, translate along z, rotate back), built on the host at
// context build.
//
// For a rotation Q, the regular harmonics of degree n mix among themselves:
//   R_n^m(Q y) = sum_{m'} W^n_{m m'} R_n^{m'}(y),  |m|, |m'| <= n.
// With Q taking the translation direction to +z, the multipole expansion in
// the rotated frame has coefficients M'_n = conj(W^n) M_n, the translation
// along z couples each order m only with itself (I_j^m(d z) = delta_m0 j!/d^(j+1)),
// and the local expansion goes back by L_k = conj(W^k)^T L'_k.
//
// W^n comes from the harmonics themselves: on a circle of polar angle t0 with
// N equally spaced azimuths phi_j, R_n^{m'}(y_j) = R_n^{m'}(t0, 0) e^{i m' phi_j},
// so a discrete Fourier transform in phi of R_n^m(Q y_j) gives
// W^n_{m m'} R_n^{m'}(t0, 0); two circles (t0 = 1 and 2) are combined by least
// squares per m' so that no small R_n^{m'}(t0, 0) is divided by alone.  N =
// 2 p_max + 1 resolves every |m'| <= n <= p_max without aliasing.
//
// The kernels work on the stored real coefficients (m >= 0, re/im interleaved,
// X_n^{-m} = (-1)^m conj(X_n^m)), so each W^n is folded into a real
// 2(n+1) x 2(n+1) matrix (forward: M -> M', backward: L' -> L) and stored in
// the matrix-core lane order of k_m2l_rot: per degree, row tiles of 16 x
// column steps of 4, 64 values per (tile, step), value of lane i + 16 k =
// A[16 rt + i][4 kt + k] (0 outside the matrix).
#include <array>
#include <cmath>
#include <complex>
#include <map>
#include <numeric>
#include <thread>
#include <vector>

#include "common.h"

namespace fmmbem {

namespace {

using cd = std::complex<double>;

// R_n^m(x), 0 <= m <= n <= p, index n (n + 1) / 2 + m, by the Cartesian
// recurrences of the factorial normalisation
void regular_all(int p, double x, double y, double z, std::vector<cd> &R)
{
    R.assign((size_t)ncoef(p), cd(0.0, 0.0));
    const double r2 = x * x + y * y + z * z;
    R[0] = 1.0;
    for (int m = 1; m <= p; ++m)
        R[cidx(m, m)] = -cd(x, y) / (2.0 * m) * R[cidx(m - 1, m - 1)];
    for (int m = 0; m <= p; ++m)
        for (int n = m + 1; n <= p; ++n) {
            const cd prev2 = n - 2 >= m ? R[cidx(n - 2, m)] : cd(0.0, 0.0);
            R[cidx(n, m)] = ((2.0 * n - 1.0) * z * R[cidx(n - 1, m)] - r2 * prev2) / (double)((n - m) * (n + m));
        }
}

// R_n^m for negative m as well
cd regular_at(const std::vector<cd> &R, int n, int m)
{
    if (m >= 0)
        return R[cidx(n, m)];
    const cd v = std::conj(R[cidx(n, -m)]);
    return (m & 1) ? -v : v;
}

// the rotation taking unit vector u to +z: R_y(-theta) R_z(-phi)
std::array<double, 9> rotation_to_z(double ux, double uy, double uz)
{
    const double th = std::acos(std::max(-1.0, std::min(1.0, uz))), ph = std::atan2(uy, ux);
    const double cz = std::cos(-ph), sz = std::sin(-ph), cy = std::cos(-th), sy = std::sin(-th);
    // Rz = [[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]], Ry = [[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]]
    return {cy * cz, -cy * sz, sy, sz, cz, 0.0, -sy * cz, sy * sz, cy};
}

// W^n for n <= p of rotation Q: W[n][(m + n) (2n + 1) + (m' + n)].  Rows
// m >= 0 are transformed; the others follow from R_n^{-m} = (-1)^m
// conj(R_n^m) and Q real: W_{-m,-m'} = (-1)^(m + m') conj(W_{m m'}).
void rotation_w(int p, const std::array<double, 9> &Q, std::vector<std::vector<cd>> &W)
{
    const int N = 2 * p + 1;
    const double circles[2] = {1.0, 2.0};
    std::vector<std::vector<cd>> acc(p + 1);
    std::vector<std::vector<double>> wsum(p + 1);
    for (int n = 0; n <= p; ++n) {
        acc[n].assign((size_t)(n + 1) * (2 * n + 1), cd(0.0, 0.0));
        wsum[n].assign(2 * n + 1, 0.0);
    }
    // e^{-i m' phi_j}, m' = -p..p
    std::vector<cd> E((size_t)N * N);
    for (int mp = -p; mp <= p; ++mp)
        for (int j = 0; j < N; ++j)
            E[(size_t)(mp + p) * N + j] = std::polar(1.0, -2.0 * M_PI * (double)mp * j / N);
    std::vector<cd> R0, Rj, v((size_t)ncoef(p) * N);  // v[(n, m)][j] = R_n^m(Q y_j)
    for (double t0 : circles) {
        const double st = std::sin(t0), ct = std::cos(t0);
        regular_all(p, st, 0.0, ct, R0);
        for (int j = 0; j < N; ++j) {
            const double ph = 2.0 * M_PI * j / N;
            const double y0 = st * std::cos(ph), y1 = st * std::sin(ph), y2 = ct;
            regular_all(p, Q[0] * y0 + Q[1] * y1 + Q[2] * y2, Q[3] * y0 + Q[4] * y1 + Q[5] * y2,
                        Q[6] * y0 + Q[7] * y1 + Q[8] * y2, Rj);
            for (int c = 0; c < ncoef(p); ++c)
                v[(size_t)c * N + j] = Rj[c];
        }
        for (int n = 0; n <= p; ++n) {
            const int w = 2 * n + 1;
            for (int mp = -n; mp <= n; ++mp) {
                const cd a = regular_at(R0, n, mp);
                wsum[n][mp + n] += std::norm(a);
                const cd *e = &E[(size_t)(mp + p) * N];
                for (int m = 0; m <= n; ++m) {
                    const cd *vm = &v[(size_t)cidx(n, m) * N];
                    cd g(0.0, 0.0);  // (1/N) sum_j R_n^m(Q y_j) e^{-i m' phi_j} = W_{m m'} a_{m'}
                    for (int j = 0; j < N; ++j)
                        g += vm[j] * e[j];
                    acc[n][(size_t)m * w + (mp + n)] += g / (double)N * std::conj(a);
                }
            }
        }
    }
    W.assign(p + 1, {});
    for (int n = 0; n <= p; ++n) {
        const int w = 2 * n + 1;
        W[n].resize((size_t)w * w);
        for (int m = 0; m <= n; ++m)
            for (int mp = -n; mp <= n; ++mp) {
                const cd x = acc[n][(size_t)m * w + (mp + n)] / wsum[n][mp + n];
                W[n][(size_t)(m + n) * w + (mp + n)] = x;
                if (m > 0) {
                    const cd y = std::conj(x);
                    W[n][(size_t)(-m + n) * w + (-mp + n)] = ((m + mp) & 1) ? -y : y;
                }
            }
    }
}

// Real form of x -> conj(W) x (forward, rows m, columns m') or x -> conj(W)^T x
// (backward, rows l', columns l) on stored coefficients: out[2 a + {0, 1}] =
// re/im of output order a, in[2 b + {0, 1}] = re/im of input order b >= 0,
// the input's negative orders folded in by X^{-b} = (-1)^b conj(X^b).
void fold_real(int n, const std::vector<cd> &Wn, bool back, std::vector<double> &A)
{
    const int S = 2 * (n + 1), w = 2 * n + 1;
    A.assign((size_t)S * S, 0.0);
    auto W = [&](int r, int c) { return Wn[(size_t)(r + n) * w + (c + n)]; };
    for (int a = 0; a <= n; ++a)
        for (int b = 0; b <= n; ++b) {
            // coefficient of input order b (and of -b) in output order a
            const cd w1 = back ? W(b, a) : W(a, b);
            const double pr = w1.real(), q = w1.imag();
            double *r0 = &A[(size_t)(2 * a) * S], *r1 = &A[(size_t)(2 * a + 1) * S];
            if (b == 0) {
                r0[0] += pr;
                r0[1] += q;
                r1[0] += -q;
                r1[1] += pr;
            } else {
                const cd w2 = back ? W(-b, a) : W(a, -b);
                const double r = w2.real(), s = w2.imag(), sg = (b & 1) ? -1.0 : 1.0;
                r0[2 * b] += pr + sg * r;
                r0[2 * b + 1] += q - sg * s;
                r1[2 * b] += -q - sg * s;
                r1[2 * b + 1] += pr - sg * r;
            }
        }
}

}  // namespace

int64_t rot_tile_values(int p)
{
    int64_t v = 0;
    for (int n = 0; n <= p; ++n) {
        const int S = 2 * (n + 1);
        v += (int64_t)((S + 15) / 16) * ((S + 3) / 4) * 64;
    }
    return v;
}

void rotation_tables(const std::vector<std::array<int64_t, 3>> &dirs, int p, std::vector<double> &fwd,
                     std::vector<double> &back)
{
    const int64_t per = rot_tile_values(p);
    fwd.assign((size_t)per * dirs.size(), 0.0);
    back.assign((size_t)per * dirs.size(), 0.0);
    // directions in parallel on the host's cores
    const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (unsigned t = 0; t < nth; ++t)
        pool.emplace_back([&, t] {
            std::vector<std::vector<cd>> W;
            std::vector<double> A;
            for (size_t d = t; d < dirs.size(); d += nth) {
                const double dx = (double)dirs[d][0], dy = (double)dirs[d][1], dz = (double)dirs[d][2];
                const double len = std::sqrt(dx * dx + dy * dy + dz * dz);
                rotation_w(p, rotation_to_z(dx / len, dy / len, dz / len), W);
                for (int kind = 0; kind < 2; ++kind) {
                    double *dst = (kind == 0 ? fwd.data() : back.data()) + (int64_t)d * per;
                    for (int n = 0; n <= p; ++n) {
                        fold_real(n, W[n], kind == 1, A);
                        const int S = 2 * (n + 1), nrt = (S + 15) / 16, k4 = (S + 3) / 4;
                        for (int rt = 0; rt < nrt; ++rt)
                            for (int kt = 0; kt < k4; ++kt)
                                for (int lane = 0; lane < 64; ++lane) {
                                    const int i = 16 * rt + (lane & 15), k = 4 * kt + (lane >> 4);
                                    dst[((int64_t)rt * k4 + kt) * 64 + lane] = (i < S && k < S) ? A[(size_t)i * S + k] : 0.0;
                                }
                        dst += (int64_t)nrt * k4 * 64;
                    }
                }
            }
        });
    for (auto &th : pool)
        th.join();
}

}  // namespace fmmbem
