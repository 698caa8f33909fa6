// Batches of independent volumes of uneven size: one plan per volume, driven
// stage by stage on one stream, and HIP-graph capture/replay of a whole
// batched forward or adjoint.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "plan.h"

struct nufftct_batch {
  std::vector<nufftct_plan*> plans;
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  hipGraph_t graph[2] = {nullptr, nullptr};
};

static int bfail(int code, const std::string& msg) { return set_last_error(code, msg); }

static void free_batch(nufftct_batch* b) {
  if (!b) return;
  for (int d = 0; d < 2; ++d) {
    if (b->exec[d]) hipGraphExecDestroy(b->exec[d]);
    if (b->graph[d]) hipGraphDestroy(b->graph[d]);
  }
  for (auto* p : b->plans) nufftct_plan_destroy(p);
  delete b;
}

// Run one direction over all volumes.  Volumes are visited grouped by grid
// size so that consecutive launches reuse the same kernels.
static int run_dir(nufftct_batch* b, int dir, const void* const* src, void* const* dst, int flags,
                   void* stream) {
  std::vector<int> order(b->plans.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return b->plans[x]->K < b->plans[y]->K; });
  for (int i : order) {
    if (!src[i] || !dst[i]) return bfail(NUFFTCT_EINVAL, "null buffer for volume " + std::to_string(i));
    int rc = dir == 0 ? nufftct_forward(b->plans[i], src[i], dst[i], flags, stream)
                      : nufftct_adjoint(b->plans[i], src[i], dst[i], flags, stream);
    if (rc) return bfail(rc, "volume " + std::to_string(i) + ": " + nufftct_last_error());
  }
  return NUFFTCT_OK;
}

extern "C" {

int nufftct_batch_create(nufftct_batch** out, int nvol, const int64_t* N, const int64_t* K, int J,
                         int kernel, double beta, int precision, const double* const* dirs,
                         const int64_t* n_lines, const int64_t* n_r, void* stream) {
  if (!out) return bfail(NUFFTCT_EINVAL, "out is NULL");
  *out = nullptr;
  if (nvol < 1 || !N || !K || !dirs || !n_lines || !n_r)
    return bfail(NUFFTCT_EINVAL, "nvol must be >= 1 and the size arrays non-NULL");
  nufftct_batch* b = new (std::nothrow) nufftct_batch();
  if (!b) return bfail(NUFFTCT_ENOMEM, "host allocation failed");
  for (int i = 0; i < nvol; ++i) {
    nufftct_plan* p = nullptr;
    int rc = nufftct_plan_create_radial(&p, N[i], K[i], J, kernel, beta, precision, dirs[i],
                                        n_lines[i], n_r[i], stream);
    if (rc) {
      std::string m = "volume " + std::to_string(i) + ": " + nufftct_last_error();
      free_batch(b);
      return bfail(rc, m);
    }
    b->plans.push_back(p);
  }
  *out = b;
  return NUFFTCT_OK;
}

int nufftct_batch_forward(nufftct_batch* b, const void* const* vols, void* const* outs, int flags,
                          void* stream) {
  if (!b || !vols || !outs) return bfail(NUFFTCT_EINVAL, "null argument");
  return run_dir(b, 0, vols, outs, flags, stream);
}

int nufftct_batch_adjoint(nufftct_batch* b, const void* const* ins, void* const* vols, int flags,
                          void* stream) {
  if (!b || !ins || !vols) return bfail(NUFFTCT_EINVAL, "null argument");
  return run_dir(b, 1, (const void* const*)ins, vols, flags, stream);
}

int nufftct_batch_graph_capture(nufftct_batch* b, int dir, const void* const* src,
                                void* const* dst, int flags, void* stream) {
  if (!b || !src || !dst || (dir != 0 && dir != 1))
    return bfail(NUFFTCT_EINVAL, "null argument or bad direction");
  if (!stream) return bfail(NUFFTCT_EINVAL, "graph capture needs a non-null stream");
  hipStream_t st = (hipStream_t)stream;
  std::vector<bool> timing(b->plans.size());
  for (size_t i = 0; i < b->plans.size(); ++i) {
    timing[i] = b->plans[i]->timing;
    b->plans[i]->timing = false;
  }
  hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return bfail(NUFFTCT_EHIP, std::string("begin capture: ") + hipGetErrorString(e));
  int rc = run_dir(b, dir, src, dst, flags, stream);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(st, &g);
  for (size_t i = 0; i < b->plans.size(); ++i) b->plans[i]->timing = timing[i];
  if (rc) {
    if (g) hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return bfail(NUFFTCT_EHIP, std::string("end capture: ") + hipGetErrorString(e));
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    hipGraphDestroy(g);
    return bfail(NUFFTCT_EHIP, std::string("instantiate: ") + hipGetErrorString(e));
  }
  if (b->exec[dir]) hipGraphExecDestroy(b->exec[dir]);
  if (b->graph[dir]) hipGraphDestroy(b->graph[dir]);
  b->exec[dir] = ex;
  b->graph[dir] = g;
  return NUFFTCT_OK;
}

int nufftct_batch_graph_launch(nufftct_batch* b, int dir, void* stream) {
  if (!b || (dir != 0 && dir != 1)) return bfail(NUFFTCT_EINVAL, "null batch or bad direction");
  if (!b->exec[dir]) return bfail(NUFFTCT_EINVAL, "no graph captured for this direction");
  hipError_t e = hipGraphLaunch(b->exec[dir], (hipStream_t)stream);
  if (e != hipSuccess) return bfail(NUFFTCT_EHIP, std::string("graph launch: ") + hipGetErrorString(e));
  return NUFFTCT_OK;
}

int nufftct_batch_destroy(nufftct_batch* b) {
  free_batch(b);
  return NUFFTCT_OK;
}

}  // extern "C"
