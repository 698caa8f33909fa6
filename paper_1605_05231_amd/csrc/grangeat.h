// Umbrella derivative-Radon values -> cone-beam projections: the Grangeat
// step in reverse (Section 2.2.2; its steps' costs in eq 2.21-2.24).  Shared
// declarations of the host object and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plan.h"

struct nufftct_grangeat {
  int n_proj = 0, n_alpha = 0, n = 0;  // projections, detector-line angles, detector pixels per side
  int J = 0, precision = 0;
  int K = 0;                           // 2n: padded line length and NUFFT grid side
  double R = 0, D = 0, side = 0;       // source radius, source-detector distance, detector side
  // FP64 tables (device)
  double* d_pw = nullptr;   // n: -R^2 / (R^2 + s'_j^2) * delta' (de-postweighting and the DFT's ds')
  double* d_dcw = nullptr;  // n: the k = 0 weight per sample, signed for the centred layout
  double* d_h = nullptr;    // 2n: the derivative-data inversion filter, c = -i h P
  double* d_sv = nullptr;   // n: virtual-detector coordinates s'_j
  double* d_s = nullptr;    // n: deapodization 1/Psi(m/K) at m = j - n/2
  void* d_tw = nullptr;     // K twiddles (plan precision)
  // gather form of the KB spreading (the same for every projection)
  int32_t* d_off = nullptr;  // K^2 + 1 cell offsets
  int32_t* d_pt = nullptr;   // entries: polar point p = i * 2n + m
  void* d_w = nullptr;       // entries: weight w_u w_v (plan precision)
  int64_t n_entries = 0;
  // workspaces
  void* d_c = nullptr;       // spectra [i][m][k]: n_alpha * 2n * n_proj complex
  void* d_rows = nullptr;    // after the first inverse FFT pass: [k][kappa_v][a], n_proj * K * n complex
  size_t c_bytes = 0, rows_bytes = 0;
};

// U[k][i][j] -> c[(i * 2n + m) * n_proj + k] (de-postweighting, radial FFT, filter)
template <typename T>
hipError_t launch_grangeat_radial(const nufftct_grangeat& g, const void* umb, void* c,
                                  hipStream_t s);
// c -> X[k][b][a] (KB spreading in gather form, inverse 2D FFT, crop, scaling)
template <typename T>
hipError_t launch_grangeat_backproject(const nufftct_grangeat& g, const void* c, void* x,
                                       hipStream_t s);
bool grangeat_length_supported(int64_t n);
