// Batches of independent volumes of uneven size: one plan per volume (each
// with its own workspace), the volumes spread over a few worker streams that
// fork from and join back into the caller's stream, and HIP-graph
// capture/replay of a whole batched forward or adjoint (the fork/join becomes
// parallel branches of the graph).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "plan.h"

// worker streams per batch: small volumes leave most of the GPU idle, so a
// few of them run side by side
#define NUFFTCT_BATCH_LANES 4

struct nufftct_batch {
  std::vector<nufftct_plan*> plans;
  std::vector<int> lane_of;          // worker stream of each volume
  std::vector<hipStream_t> lanes;    // default priority, non-blocking
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
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
  for (auto e : b->join) hipEventDestroy(e);
  if (b->fork) hipEventDestroy(b->fork);
  for (auto s : b->lanes) hipStreamDestroy(s);
  delete b;
}

// Longest-processing-time assignment of volumes to lanes, by a cost of
// K^3 log K (FFTs) plus M J^3 (interpolation or spreading).
static void assign_lanes(nufftct_batch* b) {
  const int n = (int)b->plans.size(), L = (int)b->lanes.size();
  std::vector<double> cost(n), load(L, 0.0);
  for (int i = 0; i < n; ++i) {
    const nufftct_plan* p = b->plans[i];
    const double K3 = (double)p->K * p->K * p->K;
    cost[i] = K3 * std::log2((double)p->K) + (double)p->M * p->J * p->J * p->J;
  }
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  b->lane_of.assign(n, 0);
  for (int i : order) {
    const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    b->lane_of[i] = l;
    load[l] += cost[i];
  }
}

// Run one direction over all volumes: fork the worker streams from the
// caller's stream, run each volume on its lane, join them back.
static int run_dir(nufftct_batch* b, int dir, const void* const* src, void* const* dst, int flags,
                   void* stream) {
  const int n = (int)b->plans.size();
  for (int i = 0; i < n; ++i)
    if (!src[i] || !dst[i]) return bfail(NUFFTCT_EINVAL, "null buffer for volume " + std::to_string(i));
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipEventRecord(b->fork, st);
  for (size_t l = 0; l < b->lanes.size() && e == hipSuccess; ++l)
    e = hipStreamWaitEvent(b->lanes[l], b->fork, 0);
  if (e != hipSuccess) return bfail(NUFFTCT_EHIP, std::string("fork: ") + hipGetErrorString(e));
  int rc = NUFFTCT_OK;
  for (int i = 0; i < n && rc == NUFFTCT_OK; ++i) {
    void* ls = (void*)b->lanes[b->lane_of[i]];
    rc = dir == 0 ? nufftct_forward(b->plans[i], src[i], dst[i], flags, ls)
                  : nufftct_adjoint(b->plans[i], src[i], dst[i], flags, ls);
    if (rc) rc = bfail(rc, "volume " + std::to_string(i) + ": " + nufftct_last_error());
  }
  // join even after a failure, so that no lane is left forked (or capturing)
  for (size_t l = 0; l < b->lanes.size(); ++l) {
    hipError_t e1 = hipEventRecord(b->join[l], b->lanes[l]);
    if (e1 == hipSuccess) e1 = hipStreamWaitEvent(st, b->join[l], 0);
    if (e1 != hipSuccess && rc == NUFFTCT_OK)
      rc = bfail(NUFFTCT_EHIP, std::string("join: ") + hipGetErrorString(e1));
  }
  return rc;
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
  const int L = std::min(nvol, NUFFTCT_BATCH_LANES);
  hipError_t e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  for (int l = 0; l < L && e == hipSuccess; ++l) {
    hipStream_t s = nullptr;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) break;
    b->lanes.push_back(s);
    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) b->join.push_back(ev);
  }
  if (e != hipSuccess) {
    free_batch(b);
    return bfail(NUFFTCT_EHIP, std::string("worker streams: ") + hipGetErrorString(e));
  }
  assign_lanes(b);
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
