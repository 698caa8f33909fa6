// Radial -> umbrella resampling kernel (method 2, eq 2.15): one thread per
// umbrella sample.  The plane through the source that meets the detector in
// the sample's line is built in FP64, mapped to (phi, theta, rho) index
// coordinates of the radial grid, and the J^3 taps around it are gathered
// with the normalised KB-windowed sinc weights, evaluated directly in FP64.
// phi wraps; theta and rho taps off the grid contribute nothing.
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

template <typename T, int J>
__global__ __launch_bounds__(NT) void k_umbrella(const cx<T>* __restrict__ D,
                                                 cx<T>* __restrict__ out, UmbrellaGeom g) {
#pragma clang fp contract(off)
  const int64_t total = (int64_t)g.n_proj * g.n_alpha * g.n_t;
  const int64_t p = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (p >= total) return;
  double tp, tt, tr;
  umbrella_coords(g, p, tp, tt, tr);
  int kp, kt, kr;
  T wp[J], wt[J], wr[J];
  taps<T, J>(tp, g.beta, g.inv_i0beta, kp, wp);
  taps<T, J>(tt, g.beta, g.inv_i0beta, kt, wt);
  taps<T, J>(tr, g.beta, g.inv_i0beta, kr, wr);
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

template <typename T, int J>
hipError_t launch(const nufftct_umbrella& u, const void* in, void* out, hipStream_t st) {
  const int64_t total = (int64_t)u.g.n_proj * u.g.n_alpha * u.g.n_t;
  const dim3 grd((unsigned)((total + NT - 1) / NT));
  hipLaunchKernelGGL((k_umbrella<T, J>), grd, dim3(NT), 0, st, (const cx<T>*)in, (cx<T>*)out,
                     u.g);
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
