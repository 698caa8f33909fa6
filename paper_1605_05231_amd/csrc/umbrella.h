// Radial -> umbrella resampling of the derivative-Radon space (Section 2.1.3:
// method 2, eq 2.15, and method 1, eq 2.11): shared declarations of the host
// object, the scan geometry and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plan.h"

// Circular cone-beam scan and radial grid, in voxel units.
struct UmbrellaGeom {
  int n_proj, n_alpha, n_t;  // output: projections x detector-line angles x offsets
  int n_phi, n_theta, n_r;   // input: radial grid [phi][theta][rho]
  double R_s, D_sd, dt;      // source radius, source-detector distance, line-offset step
  double theta0, inv_dtheta, inv_dphi;
  double beta, inv_i0beta;   // Kaiser-Bessel window of the method-2 weights
};

// Method 2: per-tap polynomial fits (in z = 2 frac - 1) of the normalised
// windowed-sinc weights, by precision.
#define NUFFTCT_UMB_DEG_F32 15
#define NUFFTCT_UMB_DEG_F64 23
template <typename T, int DEG>
struct TapPoly {
  T c[NUFFTCT_MAXJ][DEG + 1];
};

struct nufftct_umbrella {
  UmbrellaGeom g{};
  int J = 0, precision = 0;
  int method = 2;
  // method 2: weights from the fits when they meet the precision's bound
  // (1e-7 FP32, 1e-13 FP64), else evaluated directly in FP64
  bool poly = false;
  TapPoly<float, NUFFTCT_UMB_DEG_F32> tp32{};
  TapPoly<double, NUFFTCT_UMB_DEG_F64> tp64{};
  // method 1 (eq 2.11): oversampled grid K_d = 2 N_d per axis [phi][theta][rho]
  int64_t K[3] = {0, 0, 0};
  void* d_tw_n[3] = {nullptr, nullptr, nullptr};  // twiddles of length N_d (plan precision)
  void* d_tw_k[3] = {nullptr, nullptr, nullptr};  // twiddles of length K_d
  double* d_sc[3] = {nullptr, nullptr, nullptr};  // s_d(m) / N_d, index m + N_d/2
  void* d_grid = nullptr;                         // K_0 K_1 K_2 complex workspace
  size_t grid_bytes = 0;
  WeightPoly<float, NUFFTCT_DEG_F32> wp32{};      // KB weights of the T_sparse taps
  WeightPoly<double, NUFFTCT_DEG_F64> wp64{};
};

// Index coordinates (t_phi, t_theta, t_rho) on the radial grid of umbrella
// sample p = (k * n_alpha + i) * n_t + j: the plane through source k and the
// detector line u cos(alpha_i) + v sin(alpha_i) = t_j, built in FP64.
__device__ __forceinline__ void umbrella_coords(const UmbrellaGeom& g, int64_t p, double& tp,
                                                double& tt, double& tr) {
#pragma clang fp contract(off)
  const int j = (int)(p % g.n_t);
  const int i = (int)((p / g.n_t) % g.n_alpha);
  const int k = (int)(p / ((int64_t)g.n_t * g.n_alpha));
  const double pi = 3.14159265358979323846;
  const double lam = 2.0 * pi * (double)k / (double)g.n_proj;
  const double al = pi * (double)i / (double)g.n_alpha;
  const double t = (double)(j - g.n_t / 2) * g.dt;
  const double cl = cos(lam), sl = sin(lam), ca = cos(al), sa = sin(al);
  // u = (-sl, cl, 0), v = (0, 0, 1); e = -sa u + ca v; w = ca u + sa v
  const double e0 = sa * sl, e1 = -sa * cl, e2 = ca;
  const double w0 = -ca * sl, w1 = ca * cl, w2 = sa;
  // q = c - s + t w = -D_sd shat + t w
  const double q0 = -g.D_sd * cl + t * w0, q1 = -g.D_sd * sl + t * w1, q2 = t * w2;
  double n0 = e1 * q2 - e2 * q1, n1 = e2 * q0 - e0 * q2, n2 = e0 * q1 - e1 * q0;
  const double nn = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
  n0 /= nn;
  n1 /= nn;
  n2 /= nn;
  const double rho = g.R_s * (n0 * cl + n1 * sl);
  const double theta = acos(fmin(1.0, fmax(-1.0, n2)));
  double phi = atan2(n1, n0);
  if (phi < 0.0) phi += 2.0 * pi;
  tp = phi * g.inv_dphi;
  tt = (theta - g.theta0) * g.inv_dtheta;
  tr = rho + 0.5 * (double)g.n_r;
}

template <typename T>
hipError_t launch_umbrella(const nufftct_umbrella& u, const void* in, void* out, hipStream_t s);
// method 1: radial samples -> oversampled grid F P F^-1 D (three axis passes)
template <typename T>
hipError_t launch_resample1_grid(const nufftct_umbrella& u, const void* in, void* grid,
                                 hipStream_t s);
// method 1: oversampled grid -> umbrella samples (J^3 KB taps, T_sparse)
template <typename T>
hipError_t launch_resample1_gather(const nufftct_umbrella& u, const void* grid, void* out,
                                   hipStream_t s);
bool resample1_length_supported(int64_t n);
