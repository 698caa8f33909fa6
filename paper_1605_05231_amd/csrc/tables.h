// Host-side FP64 / long-double tables: Kaiser-Bessel kernel and its Fourier
// transform (deapodization), twiddles, min-max coefficients, and the
// per-tap polynomial fits of the interpolation weights.
#pragma once

#include <stdint.h>

#include <complex>
#include <vector>

namespace tables {

// Modified Bessel function I0 by its power series sum (x^2/4)^k / (k!)^2.
long double bessel_i0(long double x);

// Kaiser-Bessel kernel psi(u) = I0(beta sqrt(1 - (2u/J)^2)) / I0(beta), |u| <= J/2.
long double kb_psi(long double u, int J, long double beta);

// Its continuous Fourier transform at f cycles per grid unit:
// (J / I0(beta)) sinh(z)/z with z = sqrt(beta^2 - (pi J f)^2) (sin(z)/z past the zero).
long double kb_psi_hat(long double f, int J, long double beta);

// Deapodization s(m) = 1 / Psi(m / K), m = -N/2 .. N/2-1.
std::vector<double> deapod(int64_t N, int64_t K, int J, double beta);

// tw[i] = exp(-2 pi i i / L), i < L, rounded once from long double.
template <typename T>
std::vector<T> twiddles(int64_t L);  // interleaved re, im (2L values)

// Min-max coefficients of one axis for offset frac in [0, 1):
// c = T^-1 r with T[j,l] = sum_m s(m)^2 e^{i gamma (j-l) m},
// r[j] = sum_m s(m) e^{-i gamma u_j m}, u_j = J/2 - 1 - j + frac.
struct MinMax {
  int64_t N, K;
  int J;
  std::vector<long double> s;  // scaling
  std::vector<std::complex<long double>> Tlu;  // LU factors of T (row-major J x J)
  std::vector<int> piv;
  MinMax(int64_t N, int64_t K, int J, const std::vector<double>& s);
  void coeffs(long double frac, std::complex<long double>* c) const;
};

// Fit per-tap polynomials P_a(z), z = 2 frac - 1 in [-1, 1], of degree deg to
// the weight functions w_a(frac) (Chebyshev interpolation, converted to the
// monomial basis).  re/im: J x (deg+1) coefficients.  Returns the maximum
// absolute error measured on a fine grid in long double.
long double fit_kb(int J, double beta, int deg, std::vector<long double>& re);
// The same for the normalised KB-windowed sinc weights of the radial ->
// umbrella resampling: w_a = sinc(u_a) psi(u_a) / sum_b sinc(u_b) psi(u_b).
long double fit_window_sinc(int J, double beta, int deg, std::vector<long double>& re);
long double fit_minmax(const MinMax& mm, int deg, std::vector<long double>& re,
                       std::vector<long double>& im);

}  // namespace tables
