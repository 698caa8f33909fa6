// Descriptors of the batched stage launches of an uneven batch (shared by the
// host code that builds them and the kernels that read them).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cx.h"
#include "plan.h"

// volumes per batched launch (the kernel argument carries their pointers)
#define NUFFTCT_BATCH_MAXV 64

struct BatchArgs {
  const void* in[NUFFTCT_BATCH_MAXV];
  void* out[NUFFTCT_BATCH_MAXV];
  double r2[NUFFTCT_BATCH_MAXV];    // ball radius^2 of each volume's taps (FFT passes)
  int64_t n[NUFFTCT_BATCH_MAXV];    // lines (radial stage)
};

// A volume's plan data for the point stages (device array, built at batch creation).
struct BatchPointVol {
  const int32_t* perm;        // interpolation order
  const int32_t* perm_s;      // spreading order
  const TileTask* tasks;
  const int32_t* torder;      // spreading dispatch order
  const float* bound;         // fixed-point bound per task
  int32_t* multi;             // list of tasks for the general spreading kernel
  const int32_t* bin_tasks;
  const int32_t* merge_order;
  void* grid;                 // K^3 workspace
  void* tmp;                  // M workspace (values ahead of / after the radial stage)
  void* partials;             // spreading halo partials
  XcdSplit xs;
  PointGeom g;
  int nb, K, R;
  double r2;
};

// FFT / radial stages of one size class: `nv` volumes (<= NUFFTCT_BATCH_MAXV)
// of transform length K = L and radial length n_r, sharing N, the twiddles
// and the deapodization table.
template <typename T>
struct BatchClass {
  int N, K, n_r, nv;
  int64_t max_lines;          // largest line count of the class
  const double* s;            // deapodization
  const cx<T>* tw_K;
  const cx<T>* tw_r;
};

// Point stages of one tile group: `nv` (<= NUFFTCT_BATCH_MAXV) volumes whose
// plan data sit at `vols` (device); their block ranges start at
// start_tasks[v] (interpolation, spreading) and start_tiles[v] (merge), with
// start_*[nv] the total (kernel arguments: a block finds its volume without a
// chain of memory reads).
struct BatchStarts {
  int32_t s[NUFFTCT_BATCH_MAXV + 1];
};

struct BatchGroup {
  const BatchPointVol* vols;
  BatchStarts start_tasks, start_tiles;
  int64_t max_tasks;          // largest task count of the group (general spreading blocks)
  int nv, J, tile;
};

// One stage of one size class: what = 0 forward FFT passes (in = volumes, out =
// grids), 1 inverse FFT passes (in = grids, out = volumes), 2 radial stage,
// 3 its adjoint (in / out = the per-call buffers, n = line counts).
template <typename T>
hipError_t launch_batch_class(const BatchClass<T>& c, const BatchArgs& a, int what, bool deriv,
                              hipStream_t s);
// One point stage of one tile group: what = 0 interpolation (grid -> tmp),
// 1 spreading, its general-task pass and the merge (tmp -> grid); det: FP64
// fixed point.  poly: the plans' WeightPoly of this precision (all alike).
template <typename T>
hipError_t launch_batch_group(const BatchGroup& g, int what, bool det, const void* poly,
                              hipStream_t s);
