// Host logic of plan creation that needs no GPU (see host_plan.cpp).
#pragma once

#include <stdint.h>

#include <vector>

// A task of the interpolation and spreading kernels: one tile ("bin") of the
// grid and a run of the points whose first tap lies in it.
struct TileTask {
  int32_t bin;     // linear tile index (b0 * nb + b1) * nb + b2
  int32_t start;   // first entry in the permutation
  int32_t count;   // number of points
  int32_t npairs;  // spreading order: its first 2 npairs entries are npairs
                   // pairs of points that share their first tap cell
  int32_t ntwins;  // both orders: their first 2 ntwins entries are ntwins
                   // pairs of points at the same frequency (to FP64
                   // rounding), whose weights serve both points
};

namespace hostplan {

struct BinParams {
  int64_t M = 0, K = 0, n_r = 0;
  int J = 0, tile = 16, nb = 0, max_pts = 4096;
  bool radial = false;
  bool fp32 = true;         // interpolation order for FP32 pair reads
  bool pair_spread = true;  // spreading pairs points that share a first tap cell
  bool twins = false;       // interpolation pairs points at the same frequency
};

struct Binning {
  std::vector<int32_t> perm;       // interpolation order
  std::vector<int32_t> perm_s;     // spreading order (same tasks)
  std::vector<TileTask> tasks;
  std::vector<int32_t> bin_tasks;  // nbins + 1 offsets into tasks
};

// First tap per axis (centred grid index in [0, K)): t = om / gamma,
// k0 = floor(t - J/2), first = (k0 + 1 + K/2) mod K, in FP64 without
// contraction.
void host_first_taps(const double* om, int J, int64_t K, double gamma, int (&first)[3]);
// omega of point i: radial plans r_c * dirs[l], point plans the point itself
void point_omega(const BinParams& p, const std::vector<double>& geom, int64_t i,
                 double (&om)[3]);
void build_bins(const BinParams& p, const std::vector<double>& geom, Binning& B);

}  // namespace hostplan
