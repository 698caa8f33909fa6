// Internal plan structure and the launchers each kernel file provides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/nufftct.h"
#include "cx.h"
#include "host_plan.h"

// Degree of the per-tap weight polynomials (piecewise Horner form of the
// interpolation kernel on each unit interval), per precision.
#define NUFFTCT_DEG_F32 11
#define NUFFTCT_DEG_F64 17
#define NUFFTCT_MAXJ 8

// Per-tap polynomial coefficients of the weights in z = 2*frac - 1, where
// frac = (t - J/2) - floor(t - J/2).  Real part only for KB; complex for min-max.
template <typename T, int DEG>
struct WeightPoly {
  T re[NUFFTCT_MAXJ][DEG + 1];
  T im[NUFFTCT_MAXJ][DEG + 1];
};

// Elements between consecutive planes (steps of axis 0) of the oversampled
// grid: cell (j0, j1, j2) lives at j0 * grid_plane + j1 * K + j2.  A plane of
// 2 MiB or more is followed by a short pad: with a power-of-two plane stride,
// the column reads of the axis-0 FFT pass all fall on the same few memory
// channels (at K = 512 the pass streams at ~3.6 TB/s unpadded, ~5 TB/s with
// 256 B (FP32) / 768 B (FP64) of pad); smaller planes stay unpadded.
__host__ __device__ constexpr int64_t grid_plane(int64_t K, int cx_bytes) {
  return K * K * cx_bytes >= (int64_t(2) << 20) ? K * K + (cx_bytes == 8 ? 32 : 48) : K * K;
}
template <typename T>
__host__ __device__ constexpr int64_t grid_plane_of(int64_t K) {
  return grid_plane(K, (int)sizeof(cx<T>));
}

// Geometry of the non-uniform points, read by the interpolation/spreading kernels.
struct PointGeom {
  const double* dirs;  // radial plans: n_lines x 3 unit directions
  const double* pts;   // point plans: M x 3 omega values
  double dr;           // 2 pi / n_r (radial plans)
  double gamma;        // 2 pi / K
  double inv_gamma;    // 1 / gamma, rounded once
  double inv_nr;       // 1 / n_r (radial plans)
  int n_r;             // radial line length; 0 for point plans
  int K;
};


struct nufftct_plan {
  int64_t N = 0, K = 0, M = 0, n_r = 0, n_lines = 0;
  int J = 0, kernel = 0, precision = 0;
  double beta = 0;
  bool radial = false;

  // tiling of the grid for interpolation / spreading (tile divides K)
  int tile = 16;      // tile edge in grid cells
  int nb = 0;         // tiles per axis
  int max_pts = 4096; // points per task
  // squared radius (in grid cells, centred) of the ball holding every tap of
  // every point; +inf when it would not prune anything
  double ball_r2 = 1e300;

  // device memory owned by the plan
  double* d_dirs = nullptr;
  double* d_pts = nullptr;
  double* d_s = nullptr;        // deapodization s(m), N doubles
  void* d_tw_K = nullptr;       // twiddles for length K (plan precision)
  void* d_tw_r = nullptr;       // twiddles for length n_r
  int32_t* d_perm = nullptr;       // M point ids sorted by tile (interpolation order)
  int32_t* d_perm_s = nullptr;     // the same, spreading order within each task
  TileTask* d_tasks = nullptr;     // tasks: a bin and <= max_pts of its points
  int64_t ntasks = 0;
  XcdSplit xsplit{};               // per-XCD task ranges of equal point count
  int32_t* d_bin_tasks = nullptr;  // nb^3 + 1 offsets: tasks of bin b are [o[b], o[b+1])
  int32_t* d_merge_order = nullptr;  // nb^3 tiles in merge dispatch order, heaviest first
  int32_t* d_spread_order = nullptr; // ntasks: spreading dispatch order (per XCD range, largest first)
  void* d_partials = nullptr;      // per task, its spread halo tile (S^3 complex)
  float* d_bound = nullptr;        // per task, max over halo cells of sum |w| (fixed-point scale)
  int32_t* d_multi = nullptr;      // count, then the ids of the tasks the general spreading kernel takes
  double* d_line_w = nullptr;      // radial plans: per-line reconstruction weights (optional)
  void* d_grid = nullptr;       // K planes of grid_plane complex cells
  void* d_tmp = nullptr;        // M complex workspace
  size_t grid_bytes = 0, tmp_bytes = 0, partial_bytes = 0;

  // weight polynomials (host copies passed by value to kernels)
  WeightPoly<float, NUFFTCT_DEG_F32> wp32;
  WeightPoly<double, NUFFTCT_DEG_F64> wp64;

  // timing
  bool timing = false;
  struct Ev { hipEvent_t a, b; int stage; };
  std::vector<Ev> events;
  double stage_ms[8] = {0};
  int64_t stage_cnt[8] = {0};

  PointGeom geom() const {
    PointGeom g;
    g.dirs = d_dirs;
    g.pts = d_pts;
    g.dr = n_r ? (2.0 * M_PI) / (double)n_r : 0.0;
    g.gamma = (2.0 * M_PI) / (double)K;
    g.inv_gamma = 1.0 / g.gamma;
    g.inv_nr = n_r ? 1.0 / (double)n_r : 0.0;
    g.n_r = radial ? (int)n_r : 0;
    g.K = (int)K;
    return g;
  }
};

// ---- launchers (return hipSuccess or the launch error) ----
// FFT stages (k_fft_*.hip), templated on the real type
// prune: skip grid cells outside the ball that holds every tap (forward and
// adjoint paths); the single-stage entry point produces and reads full grids
template <typename T>
hipError_t launch_pad_fft(const nufftct_plan& p, const void* vol, void* grid, hipStream_t s,
                          bool prune);
template <typename T>
hipError_t launch_ifft_crop(const nufftct_plan& p, void* grid, void* vol, hipStream_t s,
                            bool prune);
template <typename T>
// line_w (device, one weight per line, or NULL) scales the adjoint's output
// lines by line_w[l] * w_scale
hipError_t launch_radial(const nufftct_plan& p, const void* in, void* out, bool adjoint,
                         bool deriv, hipStream_t s, const double* line_w = nullptr,
                         double w_scale = 1.0);
// interpolation / spreading (k_grid.hip)
template <typename T>
hipError_t launch_interp(const nufftct_plan& p, const void* grid, void* out, hipStream_t s);
// det: FP64 plans spread in fixed point (bitwise reproducible); FP32 always does
template <typename T>
hipError_t launch_spread(const nufftct_plan& p, const void* in, void* grid, hipStream_t s,
                         bool det = false);
// at plan creation: per task, the bound on the summed weight magnitudes at
// any halo cell that sets the spreading's fixed-point scale
template <typename T>
hipError_t launch_spread_bound(const nufftct_plan& p, hipStream_t s);
hipError_t launch_zero(void* ptr, size_t bytes, hipStream_t s);
template <typename T>
hipError_t launch_merge(const nufftct_plan& p, void* grid, hipStream_t s, bool prune);

bool fft_length_supported(int64_t L);
// a radial plan with its tiling given (tile edge, points per task; 0 = the
// usual choice)
int plan_create_radial_tiled(nufftct_plan** out, int64_t N, int64_t K, int J, int kernel,
                             double beta, int precision, const double* dirs, int64_t n_lines,
                             int64_t n_r, int tile, int max_pts, void* stream);
// record this thread's error message (read back by nufftct_last_error); returns code
int set_last_error(int code, const std::string& msg);
