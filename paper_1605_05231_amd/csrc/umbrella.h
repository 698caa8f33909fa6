// Radial -> umbrella resampling of the derivative-Radon space (method 2 of
// Section 2.1.3, eq 2.15): shared declarations of the host object and the
// kernel launcher.
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
  double beta, inv_i0beta;   // Kaiser-Bessel window of the weights
};

struct nufftct_umbrella {
  UmbrellaGeom g{};
  int J = 0, precision = 0;
};

template <typename T>
hipError_t launch_umbrella(const nufftct_umbrella& u, const void* in, void* out, hipStream_t s);
