// Internal plan structure and the launchers each kernel file provides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/nufftct.h"

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

// Geometry of the non-uniform points, read by the interpolation/spreading kernels.
struct PointGeom {
  const double* dirs;  // radial plans: n_lines x 3 unit directions
  const double* pts;   // point plans: M x 3 omega values
  double dr;           // 2 pi / n_r (radial plans)
  double gamma;        // 2 pi / K
  int n_r;             // radial line length; 0 for point plans
  int K;
};

struct TileTask {
  int32_t bin;    // linear tile index (b0 * nb + b1) * nb + b2
  int32_t start;  // first entry in the permutation
  int32_t count;  // number of points
  int32_t pad;
};

// Spreading is owner-computes: every output tile is produced by the task(s)
// that own it.  A tile's points are those of its own bin plus those of the 7
// lower-neighbour bins whose footprints spill into it; each such group is a
// contiguous segment of the permutation (points are sorted by bin, then by
// spill class).
struct SpreadSeg {
  int32_t start;  // first entry in the permutation
  int32_t count;
  int32_t delta;  // source bin = tile - (d0, d1, d2), packed d0*4 + d1*2 + d2
  int32_t pad;
};

struct SpreadTask {
  int32_t tile;       // linear output tile index
  int32_t seg_begin;  // segments [seg_begin, seg_end)
  int32_t seg_end;
  int32_t p_lo;       // sub-range of the tile's concatenated segment points
  int32_t p_hi;
  int32_t slot;       // -1: write the grid directly; else partial-tile slot
  int32_t pad0, pad1;
};

struct HeavyTile {
  int32_t tile;
  int32_t slot_begin;  // partial tiles [slot_begin, slot_end) summed in order
  int32_t slot_end;
  int32_t pad;
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

  // device memory owned by the plan
  double* d_dirs = nullptr;
  double* d_pts = nullptr;
  double* d_s = nullptr;        // deapodization s(m), N doubles
  void* d_tw_K = nullptr;       // twiddles for length K (plan precision)
  void* d_tw_r = nullptr;       // twiddles for length n_r
  int32_t* d_perm = nullptr;    // M point ids sorted by tile, then spill class
  TileTask* d_tasks = nullptr;  // interpolation tasks (bin, <= max_pts points)
  int64_t ntasks = 0;
  SpreadSeg* d_sp_segs = nullptr;
  SpreadTask* d_sp_tasks = nullptr;
  HeavyTile* d_heavy = nullptr;
  void* d_partials = nullptr;   // partial tiles of split output tiles
  int64_t n_sp_tasks = 0, n_heavy = 0, n_slots = 0;
  void* d_grid = nullptr;       // K^3 complex workspace
  void* d_tmp = nullptr;        // M complex workspace
  size_t grid_bytes = 0, tmp_bytes = 0;

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
    g.n_r = radial ? (int)n_r : 0;
    g.K = (int)K;
    return g;
  }
};

// ---- launchers (return hipSuccess or the launch error) ----
// FFT stages (k_fft_*.hip), templated on the real type
template <typename T>
hipError_t launch_pad_fft(const nufftct_plan& p, const void* vol, void* grid, hipStream_t s);
template <typename T>
hipError_t launch_ifft_crop(const nufftct_plan& p, void* grid, void* vol, hipStream_t s);
template <typename T>
hipError_t launch_radial(const nufftct_plan& p, const void* in, void* out, bool adjoint,
                         bool deriv, hipStream_t s);
// interpolation / spreading (k_grid.hip)
template <typename T>
hipError_t launch_interp(const nufftct_plan& p, const void* grid, void* out, hipStream_t s);
template <typename T>
hipError_t launch_spread(const nufftct_plan& p, const void* in, void* grid, hipStream_t s);
hipError_t launch_zero(void* ptr, size_t bytes, hipStream_t s);
template <typename T>
hipError_t launch_reduce_partials(const nufftct_plan& p, void* grid, hipStream_t s);

bool fft_length_supported(int64_t L);
// record this thread's error message (read back by nufftct_last_error); returns code
int set_last_error(int code, const std::string& msg);
