// Quadrature tables for the panel integrals (Sec. 2.3), generated at build time.
//
// Gauss-Legendre nodes come from the Golub-Welsch construction: they are the
// eigenvalues of the symmetric tridiagonal Jacobi matrix of the Legendre
// polynomials (zero diagonal, off-diagonal k / sqrt(4 k^2 - 1)), and the
// weight of node j is 2 * (first component of its unit eigenvector)^2.  The
// eigen-decomposition is a cyclic Jacobi rotation sweep, ample for n <= 64.
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"

namespace fmmbem {

void gauss_legendre_gw(int n, double *x, double *w)
{
    std::vector<double> A((size_t)n * n, 0.0), V((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
        V[(size_t)i * n + i] = 1.0;
    for (int k = 1; k < n; ++k) {
        double b = k / std::sqrt(4.0 * k * k - 1.0);
        A[(size_t)(k - 1) * n + k] = A[(size_t)k * n + (k - 1)] = b;
    }
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q)
                off += A[(size_t)p * n + q] * A[(size_t)p * n + q];
        if (off < 1e-34)
            break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = A[(size_t)p * n + q];
                if (apq == 0.0)
                    continue;
                double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
                double tau = (aqq - app) / (2.0 * apq);
                double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
                for (int k = 0; k < n; ++k) {  // A <- A J (columns p, q)
                    double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = c * akp - s * akq;
                    A[(size_t)k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {  // A <- J^T A (rows p, q)
                    double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = c * apk - s * aqk;
                    A[(size_t)q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {  // V <- V J
                    double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = c * vkp - s * vkq;
                    V[(size_t)k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    // sort ascending by eigenvalue
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i)
        order[i] = i;
    for (int i = 1; i < n; ++i)
        for (int j = i; j > 0 && A[(size_t)order[j] * n + order[j]] < A[(size_t)order[j - 1] * n + order[j - 1]]; --j)
            std::swap(order[j], order[j - 1]);
    for (int i = 0; i < n; ++i) {
        int j = order[i];
        x[i] = A[(size_t)j * n + j];
        w[i] = 2.0 * V[(size_t)0 * n + j] * V[(size_t)0 * n + j];
    }
    // symmetrise (the rule is symmetric about 0)
    for (int i = 0; i < n / 2; ++i) {
        double a = 0.5 * (x[n - 1 - i] - x[i]);
        double ww = 0.5 * (w[i] + w[n - 1 - i]);
        x[i] = -a;
        x[n - 1 - i] = a;
        w[i] = w[n - 1 - i] = ww;
    }
    if (n % 2)
        x[n / 2] = 0.0;
}

// Near-singular rule: Gauss-Legendre in (s, t) on the unit square mapped onto
// the triangle by (s, t) -> barycentric (1 - s, s (1 - t), s t); the Jacobian
// of the map is 2 s times the area, so the area-normalised weight is
// 2 s w_s w_t with w_s, w_t the weights on [0, 1].
void near_rule_table(int n1d, double *bary, double *w)
{
    std::vector<double> g(n1d), gw(n1d);
    gauss_legendre_gw(n1d, g.data(), gw.data());
    int k = 0;
    for (int a = 0; a < n1d; ++a) {
        double s = 0.5 + 0.5 * g[a];
        double ws = 0.5 * gw[a];
        for (int b = 0; b < n1d; ++b) {
            double t = 0.5 + 0.5 * g[b];
            double wt = 0.5 * gw[b];
            bary[3 * k] = 1.0 - s;
            bary[3 * k + 1] = s - s * t;
            bary[3 * k + 2] = s * t;
            w[k] = 2.0 * s * ws * wt;
            ++k;
        }
    }
}

}  // namespace fmmbem
