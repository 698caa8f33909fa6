// Radial -> umbrella resampling kernel (method 2, eq 2.15): one thread per
// umbrella sample.  The plane through the source that meets the detector in
// the sample's line is built in FP64, mapped to (phi, theta, rho) index
// coordinates of the radial grid, and the J^3 taps around it are gathered
// with the normalised KB-windowed sinc weights: per-tap polynomials in
// z = 2 frac - 1 fitted on the host (Chebyshev interpolation, degree 15 FP32 /
// 23 FP64, used when the fit meets 1e-7 / 1e-13), else evaluated directly in
// FP64.  phi wraps; theta and rho taps off the grid contribute nothing.
#include "cx.h"
#include "umbrella.h"

namespace kumb {

constexpr int NT = 256;

// Per axis: the J taps k0+1..k0+J around index coordinate t (k0 = floor(t -
// J/2)) and their weights sinc(u) psi(u) / sum_taps, u = t - kappa, psi the
// Kaiser-Bessel window I0(beta sqrt(1 - (2u/J)^2)) / I0(beta), all in FP64
// (I0 by its power series, 32 terms: enough for beta <= 4J/3 <= 11).
template <typename T, int J>
__device__ __forceinline__ void taps(double t, double beta, double inv_i0b, int& k0, T (&w)[J]) {
  const double tj = t - 0.5 * (double)J;
  const double f = floor(tj);
  k0 = (int)f;
  const double frac = tj - f;
  double wd[J], sum = 0.0;
#pragma unroll
  for (int a = 0; a < J; ++a) {
    const double u = 0.5 * (double)J - 1.0 - (double)a + frac;
    const double r = 1.0 - (2.0 * u / (double)J) * (2.0 * u / (double)J);
    double ps = 0.0;
    if (r > 0.0) {
      const double q = 0.25 * beta * beta * r;
      double term = 1.0, i0 = 1.0;
      for (int k = 1; k <= 32; ++k) {
        term *= q / (double)(k * k);
        i0 += term;
      }
      ps = i0 * inv_i0b;
    } else if (r == 0.0) {
      ps = inv_i0b;
    }
    const double sc = u == 0.0 ? 1.0 : sinpi(u) / (3.14159265358979323846 * u);
    wd[a] = sc * ps;
    sum += wd[a];
  }
  const double inv = 1.0 / sum;
#pragma unroll
  for (int a = 0; a < J; ++a) w[a] = (T)(wd[a] * inv);
}

// The same from the per-tap polynomials.
template <typename T, int J, int DEG>
__device__ __forceinline__ void taps_poly(double t, const TapPoly<T, DEG>& P, int& k0,
                                          T (&w)[J]) {
  const double tj = t - 0.5 * (double)J;
  const double f = floor(tj);
  k0 = (int)f;
  const T z = (T)(2.0 * (tj - f) - 1.0);
#pragma unroll
  for (int a = 0; a < J; ++a) {
    T acc = P.c[a][DEG];
#pragma unroll
    for (int d = DEG - 1; d >= 0; --d) acc = acc * z + P.c[a][d];
    w[a] = acc;
  }
}

template <typename T, int J, int DEG, bool POLY>
__global__ __launch_bounds__(NT) void k_umbrella(const cx<T>* __restrict__ D,
                                                 cx<T>* __restrict__ out, UmbrellaGeom g,
                                                 TapPoly<T, DEG> P) {
#pragma clang fp contract(off)
  const int64_t total = (int64_t)g.n_proj * g.n_alpha * g.n_t;
  const int64_t p = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (p >= total) return;
  double tp, tt, tr;
  umbrella_coords(g, p, tp, tt, tr);
  int kp, kt, kr;
  T wp[J], wt[J], wr[J];
  if constexpr (POLY) {
    taps_poly<T, J, DEG>(tp, P, kp, wp);
    taps_poly<T, J, DEG>(tt, P, kt, wt);
    taps_poly<T, J, DEG>(tr, P, kr, wr);
  } else {
    taps<T, J>(tp, g.beta, g.inv_i0beta, kp, wp);
    taps<T, J>(tt, g.beta, g.inv_i0beta, kt, wt);
    taps<T, J>(tr, g.beta, g.inv_i0beta, kr, wr);
  }
  cx<T> acc = {0, 0};
#pragma unroll
  for (int a = 0; a < J; ++a) {
    int ia = (kp + 1 + a) % g.n_phi;
    if (ia < 0) ia += g.n_phi;
    cx<T> acc_a = {0, 0};
#pragma unroll
    for (int b = 0; b < J; ++b) {
      const int ib = kt + 1 + b;
      if (ib < 0 || ib >= g.n_theta) continue;
      const cx<T>* row = D + ((int64_t)ia * g.n_theta + ib) * g.n_r;
      cx<T> acc_b = {0, 0};
#pragma unroll
      for (int c = 0; c < J; ++c) {
        const int ic = kr + 1 + c;
        if (ic < 0 || ic >= g.n_r) continue;
        const cx<T> v = row[ic];
        acc_b.x += wr[c] * v.x;
        acc_b.y += wr[c] * v.y;
      }
      acc_a.x += wt[b] * acc_b.x;
      acc_a.y += wt[b] * acc_b.y;
    }
    acc.x += wp[a] * acc_a.x;
    acc.y += wp[a] * acc_a.y;
  }
  out[p] = acc;
}

template <typename T>
struct PolyOf;
template <>
struct PolyOf<float> {
  static constexpr int DEG = NUFFTCT_UMB_DEG_F32;
  static const TapPoly<float, DEG>& get(const nufftct_umbrella& u) { return u.tp32; }
};
template <>
struct PolyOf<double> {
  static constexpr int DEG = NUFFTCT_UMB_DEG_F64;
  static const TapPoly<double, DEG>& get(const nufftct_umbrella& u) { return u.tp64; }
};

template <typename T, int J>
hipError_t launch(const nufftct_umbrella& u, const void* in, void* out, hipStream_t st) {
  constexpr int DEG = PolyOf<T>::DEG;
  const int64_t total = (int64_t)u.g.n_proj * u.g.n_alpha * u.g.n_t;
  const dim3 grd((unsigned)((total + NT - 1) / NT));
  if (u.poly)
    hipLaunchKernelGGL((k_umbrella<T, J, DEG, true>), grd, dim3(NT), 0, st, (const cx<T>*)in,
                       (cx<T>*)out, u.g, PolyOf<T>::get(u));
  else
    hipLaunchKernelGGL((k_umbrella<T, J, DEG, false>), grd, dim3(NT), 0, st, (const cx<T>*)in,
                       (cx<T>*)out, u.g, PolyOf<T>::get(u));
  return hipGetLastError();
}

}  // namespace kumb

template <typename T>
hipError_t launch_umbrella(const nufftct_umbrella& u, const void* in, void* out, hipStream_t s) {
  switch (u.J) {
    case 2: return kumb::launch<T, 2>(u, in, out, s);
    case 3: return kumb::launch<T, 3>(u, in, out, s);
    case 4: return kumb::launch<T, 4>(u, in, out, s);
    case 5: return kumb::launch<T, 5>(u, in, out, s);
    case 6: return kumb::launch<T, 6>(u, in, out, s);
    case 7: return kumb::launch<T, 7>(u, in, out, s);
    case 8: return kumb::launch<T, 8>(u, in, out, s);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_umbrella<float>(const nufftct_umbrella&, const void*, void*, hipStream_t);
template hipError_t launch_umbrella<double>(const nufftct_umbrella&, const void*, void*, hipStream_t);
