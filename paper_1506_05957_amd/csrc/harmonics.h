// Solid harmonics for the spherical-harmonic FMM (Sec. 2.5, Eq. 15-16).
//
// Normalisation (chosen so that every translation is a plain complex
// convolution with no coefficient tables), for x = (r, theta, phi):
//   R_n^m(x) = r^n P_n^m(cos theta) e^{i m phi} / (n + m)!        (regular)
//   I_n^m(x) = (n - m)! P_n^m(cos theta) e^{i m phi} / r^{n + 1}  (irregular)
// with P_n^m the associated Legendre functions including the Condon-Shortley
// phase, and R_n^{-m} = (-1)^m conj(R_n^m), I_n^{-m} = (-1)^m conj(I_n^m).
// They satisfy
//   1/|x - y|       = sum_{n,m} conj(R_n^m(y)) I_n^m(x)              (|y| < |x|)
//   R_n^m(a + b)    = sum_{k,l} R_k^l(a) R_{n-k}^{m-l}(b)
//   I_n^m(d + u)    = sum_{k,l} (-1)^k conj(R_k^l(u)) I_{n+k}^{m+l}(d) (|u| < |d|)
//   dR_n^m/dz = R_{n-1}^m,  dR_n^m/dx = (R_{n-1}^{m+1} - R_{n-1}^{m-1}) / 2,
//   dR_n^m/dy = -(i/2) (R_{n-1}^{m-1} + R_{n-1}^{m+1}),
// and both families follow Cartesian recurrences (no trigonometry, no pole):
//   R_0^0 = 1, R_m^m = -(x + iy) / (2m) R_{m-1}^{m-1},
//   R_n^m = ((2n - 1) z R_{n-1}^m - r^2 R_{n-2}^m) / ((n - m)(n + m)),
//   I_0^0 = 1/r, I_m^m = -(2m - 1)(x + iy) / r^2 I_{m-1}^{m-1},
//   I_n^m = ((2n - 1) z I_{n-1}^m - ((n - 1)^2 - m^2) I_{n-2}^m) / r^2.
// Expansions: multipole  phi(x) = sum M_n^m I_n^m(x - c),  M_n^m = sum q conj(R_n^m(y - c));
//             local      phi(x) = sum L_n^m conj(R_n^m(x - c)).
// Coefficients are stored for m >= 0 only, index n (n + 1) / 2 + m.
#pragma once

#include <hip/hip_runtime.h>

namespace fmmbem {

template <typename R> struct cplx {
    R re, im;
};

template <typename R> struct InvTable {
    R v[402];
};

template <typename R> constexpr InvTable<R> make_inv_table()
{
    InvTable<R> t{};
    t.v[0] = R(0);
    for (int k = 1; k < 402; ++k)
        t.v[k] = R(1) / R(k);
    return t;
}

}  // namespace fmmbem
