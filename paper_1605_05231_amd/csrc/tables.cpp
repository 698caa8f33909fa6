// Host-side tables in extended precision; see tables.h.
#include "tables.h"

#include <cmath>

namespace tables {

static const long double PI_L = 3.141592653589793238462643383279502884L;

long double bessel_i0(long double x) {
  const long double y = 0.25L * x * x;
  long double term = 1.0L, sum = 1.0L;
  for (int k = 1; k < 500; ++k) {
    term *= y / ((long double)k * (long double)k);
    sum += term;
    if (term < 1e-22L * sum) break;
  }
  return sum;
}

long double kb_psi(long double u, int J, long double beta) {
  const long double a = 2.0L * u / (long double)J;
  long double r = 1.0L - a * a;
  if (r < 0.0L) {
    if (r > -1e-15L) r = 0.0L;
    else return 0.0L;
  }
  return bessel_i0(beta * std::sqrt(r)) / bessel_i0(beta);
}

long double kb_psi_hat(long double f, int J, long double beta) {
  const long double pj = PI_L * (long double)J * f;
  const long double z2 = beta * beta - pj * pj;
  long double v;
  if (z2 > 0) {
    const long double z = std::sqrt(z2);
    v = std::sinh(z) / z;
  } else if (z2 < 0) {
    const long double z = std::sqrt(-z2);
    v = std::sin(z) / z;
  } else {
    v = 1.0L;
  }
  return v * (long double)J / bessel_i0(beta);
}

std::vector<double> deapod(int64_t N, int64_t K, int J, double beta) {
  std::vector<double> s(N);
  for (int64_t i = 0; i < N; ++i) {
    const long double m = (long double)(i - N / 2);
    s[i] = (double)(1.0L / kb_psi_hat(m / (long double)K, J, beta));
  }
  return s;
}

template <typename T>
std::vector<T> twiddles(int64_t L) {
  std::vector<T> tw(2 * L);
  for (int64_t i = 0; i < L; ++i) {
    const long double a = 2.0L * PI_L * (long double)i / (long double)L;
    tw[2 * i] = (T)std::cos(a);
    tw[2 * i + 1] = (T)(-std::sin(a));
  }
  return tw;
}
template std::vector<float> twiddles<float>(int64_t);
template std::vector<double> twiddles<double>(int64_t);

MinMax::MinMax(int64_t N_, int64_t K_, int J_, const std::vector<double>& s_)
    : N(N_), K(K_), J(J_), s(s_.begin(), s_.end()), Tlu(J_ * J_), piv(J_) {
  const long double gamma = 2.0L * PI_L / (long double)K;
  for (int j = 0; j < J; ++j)
    for (int l = 0; l < J; ++l) {
      std::complex<long double> acc = 0;
      for (int64_t i = 0; i < N; ++i) {
        const long double m = (long double)(i - N / 2);
        const long double ph = gamma * (long double)(j - l) * m;
        acc += s[i] * s[i] * std::complex<long double>(std::cos(ph), std::sin(ph));
      }
      Tlu[j * J + l] = acc;
    }
  // LU with partial pivoting
  for (int k = 0; k < J; ++k) {
    int p = k;
    for (int i = k + 1; i < J; ++i)
      if (std::abs(Tlu[i * J + k]) > std::abs(Tlu[p * J + k])) p = i;
    piv[k] = p;
    if (p != k)
      for (int c = 0; c < J; ++c) std::swap(Tlu[k * J + c], Tlu[p * J + c]);
    for (int i = k + 1; i < J; ++i) {
      Tlu[i * J + k] /= Tlu[k * J + k];
      for (int c = k + 1; c < J; ++c) Tlu[i * J + c] -= Tlu[i * J + k] * Tlu[k * J + c];
    }
  }
}

void MinMax::coeffs(long double frac, std::complex<long double>* c) const {
  const long double gamma = 2.0L * PI_L / (long double)K;
  std::vector<std::complex<long double>> r(J);
  for (int j = 0; j < J; ++j) {
    const long double u = (long double)J / 2 - 1 - j + frac;
    std::complex<long double> acc = 0;
    for (int64_t i = 0; i < N; ++i) {
      const long double m = (long double)(i - N / 2);
      const long double ph = -gamma * u * m;
      acc += s[i] * std::complex<long double>(std::cos(ph), std::sin(ph));
    }
    r[j] = acc;
  }
  for (int k = 0; k < J; ++k)
    if (piv[k] != k) std::swap(r[k], r[piv[k]]);
  for (int i = 0; i < J; ++i)
    for (int k = 0; k < i; ++k) r[i] -= Tlu[i * J + k] * r[k];
  for (int i = J - 1; i >= 0; --i) {
    for (int k = i + 1; k < J; ++k) r[i] -= Tlu[i * J + k] * r[k];
    r[i] /= Tlu[i * J + i];
  }
  for (int j = 0; j < J; ++j) c[j] = r[j];
}

// Chebyshev nodes z_k = cos(pi (k + 1/2) / n), k < n.
static long double cheb_node(int k, int n) {
  return std::cos(PI_L * ((long double)k + 0.5L) / n);
}

// Interpolating polynomial through values fv[k] at the n Chebyshev nodes,
// returned in the monomial basis (coefficient of z^k at index k).
static std::vector<long double> cheb_from_values(const std::vector<long double>& fv) {
  const int n = (int)fv.size();
  std::vector<long double> cc(n, 0.0L);
  for (int j = 0; j < n; ++j) {
    long double acc = 0;
    for (int k = 0; k < n; ++k)
      acc += fv[k] * std::cos(PI_L * (long double)j * ((long double)k + 0.5L) / n);
    cc[j] = acc * 2.0L / n;
  }
  cc[0] *= 0.5L;
  // monomial coefficients of T_j: T_0 = 1, T_1 = z, T_j = 2 z T_{j-1} - T_{j-2}
  std::vector<std::vector<long double>> Tm(n, std::vector<long double>(n, 0.0L));
  Tm[0][0] = 1.0L;
  if (n > 1) Tm[1][1] = 1.0L;
  for (int j = 2; j < n; ++j)
    for (int k = 0; k < n; ++k)
      Tm[j][k] = (k > 0 ? 2.0L * Tm[j - 1][k - 1] : 0.0L) - Tm[j - 2][k];
  std::vector<long double> mono(n, 0.0L);
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k) mono[k] += cc[j] * Tm[j][k];
  return mono;
}

static long double horner(const long double* c, int deg, long double z) {
  long double acc = c[deg];
  for (int d = deg - 1; d >= 0; --d) acc = acc * z + c[d];
  return acc;
}

long double fit_kb(int J, double beta, int deg, std::vector<long double>& re) {
  re.assign((size_t)J * (deg + 1), 0.0L);
  long double err = 0;
  for (int a = 0; a < J; ++a) {
    auto f = [&](long double z) {
      const long double frac = 0.5L * (z + 1.0L);
      return kb_psi((long double)J / 2 - 1 - a + frac, J, beta);
    };
    std::vector<long double> fv(deg + 1);
    for (int k = 0; k <= deg; ++k) fv[k] = f(cheb_node(k, deg + 1));
    auto c = cheb_from_values(fv);
    for (int k = 0; k <= deg; ++k) re[(size_t)a * (deg + 1) + k] = c[k];
    for (int i = 0; i <= 400; ++i) {
      const long double z = -1.0L + 2.0L * i / 400;
      err = std::max(err, std::fabs(horner(c.data(), deg, z) - f(z)));
    }
  }
  return err;
}

long double fit_window_sinc(int J, double beta, int deg, std::vector<long double>& re) {
  re.assign((size_t)J * (deg + 1), 0.0L);
  // w_a(frac) = sinc(u_a) I0(beta sqrt(1 - (2 u_a / J)^2)) / sum_b (same at u_b),
  // u_a = J/2 - 1 - a + frac: the normalised window of the radial resampling
  auto weights = [&](long double frac, std::vector<long double>& wv) {
    long double sum = 0;
    for (int a = 0; a < J; ++a) {
      const long double u = (long double)J / 2 - 1 - a + frac;
      const long double sc = u == 0 ? 1.0L : std::sin(PI_L * u) / (PI_L * u);
      const long double r = 1.0L - (2.0L * u / J) * (2.0L * u / J);
      const long double ps = r >= 0 ? bessel_i0((long double)beta * std::sqrt(r)) : 0.0L;
      wv[a] = sc * ps;
      sum += wv[a];
    }
    for (int a = 0; a < J; ++a) wv[a] /= sum;
  };
  const int n = deg + 1;
  std::vector<long double> wv(J);
  std::vector<std::vector<long double>> fv(J, std::vector<long double>(n));
  for (int k = 0; k < n; ++k) {
    weights(0.5L * (cheb_node(k, n) + 1.0L), wv);
    for (int a = 0; a < J; ++a) fv[a][k] = wv[a];
  }
  for (int a = 0; a < J; ++a) {
    auto c = cheb_from_values(fv[a]);
    for (int k = 0; k <= deg; ++k) re[(size_t)a * (deg + 1) + k] = c[k];
  }
  long double err = 0;
  for (int i = 0; i <= 400; ++i) {
    const long double z = -1.0L + 2.0L * i / 400;
    weights(0.5L * (z + 1.0L), wv);
    for (int a = 0; a < J; ++a)
      err = std::max(err, std::fabs(horner(&re[(size_t)a * (deg + 1)], deg, z) - wv[a]));
  }
  return err;
}

long double fit_minmax(const MinMax& mm, int deg, std::vector<long double>& re,
                       std::vector<long double>& im) {
  const int J = mm.J;
  re.assign((size_t)J * (deg + 1), 0.0L);
  im.assign((size_t)J * (deg + 1), 0.0L);
  // sample all taps at the Chebyshev nodes once
  const int n = deg + 1;
  std::vector<std::complex<long double>> vals((size_t)n * J);
  for (int k = 0; k < n; ++k) mm.coeffs(0.5L * (cheb_node(k, n) + 1.0L), &vals[(size_t)k * J]);
  long double err = 0;
  for (int a = 0; a < J; ++a) {
    std::vector<long double> fr(n), fi(n);
    for (int k = 0; k < n; ++k) {
      fr[k] = vals[(size_t)k * J + a].real();
      fi[k] = vals[(size_t)k * J + a].imag();
    }
    auto cr = cheb_from_values(fr);
    auto ci = cheb_from_values(fi);
    for (int k = 0; k <= deg; ++k) {
      re[(size_t)a * (deg + 1) + k] = cr[k];
      im[(size_t)a * (deg + 1) + k] = ci[k];
    }
  }
  // error check at off-node points
  std::vector<std::complex<long double>> cv(J);
  for (int i = 0; i <= 64; ++i) {
    const long double z = -1.0L + 2.0L * (i + 0.37L) / 65.37L;
    mm.coeffs(0.5L * (z + 1.0L), cv.data());
    for (int a = 0; a < J; ++a) {
      const long double er = horner(&re[(size_t)a * (deg + 1)], deg, z) - cv[a].real();
      const long double ei = horner(&im[(size_t)a * (deg + 1)], deg, z) - cv[a].imag();
      err = std::max(err, std::sqrt(er * er + ei * ei));
    }
  }
  return err;
}

}  // namespace tables
