// Batches of independent volumes of uneven size: one plan per volume (each
// with its own workspace and tables).  Kaiser-Bessel batches with the radial
// stage run every stage as one launch across the volumes on the caller's
// stream of its size class (volumes of equal N, K, N_r; k_batch_impl.h): a few
// launches per class and direction whatever the number of volumes, the
// classes on a few worker streams that fork from and join back into the
// caller's stream, so that one class's FFT passes overlap another's point
// stages.  Other batches (min-max weights, no radial stage) run volume by
// volume on those streams.  Either way a whole batched forward or adjoint can
// be captured into a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "batch_desc.h"
#include "plan.h"

// worker streams per batch: small volumes leave most of the GPU idle, so a
// few of them run side by side
#define NUFFTCT_BATCH_LANES 4

struct BatchGroupInfo {
  int tile;
  std::vector<int> vols;               // at most NUFFTCT_BATCH_MAXV
  BatchPointVol* d_vols = nullptr;
  BatchStarts start_tasks{}, start_tiles{};
  int64_t max_tasks = 0;
};

struct BatchClassInfo {
  int N, K, n_r;
  std::vector<int> vols;
  std::vector<BatchGroupInfo> groups;  // its volumes by tile size
  int lane = 0;
  double cost = 0;
};

struct nufftct_batch {
  std::vector<nufftct_plan*> plans;
  bool batched = false;                 // one launch per stage and unit
  std::vector<BatchClassInfo> classes;  // units: volumes of one (N, K, n_r) class
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
  for (auto& c : b->classes)
    for (auto& g : c.groups) {
      if (g.d_vols) hipFree(g.d_vols);
    }
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

static double volume_cost(const nufftct_plan* p) {
  const double K3 = (double)p->K * p->K * p->K;
  return K3 * std::log2((double)p->K) + (double)p->M * p->J * p->J * p->J;
}

// The units of the batched launches: the volumes of one size class, a class
// being cut into several units when it alone would outweigh an even share of
// the worker streams (its volumes dealt longest first over them), so that the
// streams end together, and volumes of 192^3 grids or more each a unit of
// their own; each unit's tile groups with the point stages' device
// descriptors; and the worker stream of each unit (longest first).
static int build_batched(nufftct_batch* b) {
  const int n = (int)b->plans.size();
  const int L = (int)b->lanes.size();
  struct Cls {
    int N, K, n_r;
    std::vector<int> vols;
    double cost = 0;
  };
  std::vector<Cls> cls;
  double total = 0;
  for (int i = 0; i < n; ++i) {
    const nufftct_plan* p = b->plans[i];
    Cls* c = nullptr;
    for (auto& x : cls)
      if (x.N == p->N && x.K == p->K && x.n_r == p->n_r) c = &x;
    if (!c) {
      cls.push_back(Cls{(int)p->N, (int)p->K, (int)p->n_r, {}, 0.0});
      c = &cls.back();
    }
    c->vols.push_back(i);
    c->cost += volume_cost(b->plans[i]);
    total += volume_cost(b->plans[i]);
  }
  const double share = total / (2.0 * L);
  for (auto& c : cls) {
    // a volume of a 192^3 grid or more fills the GPU alone (grouping such
    // volumes measured slower than giving each its own unit); smaller ones
    // are grouped, a class cut only when it outweighs an even share
    const int nvol = (int)c.vols.size();
    const int parts = c.K >= 192 ? nvol
                                 : std::max(1, std::min(nvol, (int)std::lround(c.cost / share)));
    std::vector<int> order = c.vols;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
      return volume_cost(b->plans[x]) > volume_cost(b->plans[y]);
    });
    const size_t first = b->classes.size();
    for (int k = 0; k < parts; ++k) {
      b->classes.emplace_back();
      BatchClassInfo& u = b->classes.back();
      u.N = c.N;
      u.K = c.K;
      u.n_r = c.n_r;
    }
    for (int i : order) {
      size_t best = first;
      for (size_t k = first; k < b->classes.size(); ++k)
        if (b->classes[k].cost < b->classes[best].cost) best = k;
      b->classes[best].vols.push_back(i);
      b->classes[best].cost += volume_cost(b->plans[i]);
    }
  }
  for (auto& u : b->classes) {
    std::sort(u.vols.begin(), u.vols.end());
    if (u.vols.size() == 1) continue;  // runs the plan's own kernels
    for (int i : u.vols) {
      BatchGroupInfo* g = nullptr;
      for (auto& x : u.groups)
        if (x.tile == b->plans[i]->tile && x.vols.size() < NUFFTCT_BATCH_MAXV) g = &x;
      if (!g) {
        u.groups.emplace_back();
        g = &u.groups.back();
        g->tile = b->plans[i]->tile;
      }
      g->vols.push_back(i);
    }
  }
  for (auto& c : b->classes)
    for (auto& g : c.groups) {
      std::vector<BatchPointVol> d(g.vols.size());
      int32_t* st = g.start_tasks.s;
      int32_t* sm = g.start_tiles.s;
      st[0] = sm[0] = 0;
      for (size_t k = 0; k < g.vols.size(); ++k) {
        const nufftct_plan* p = b->plans[g.vols[k]];
        BatchPointVol& v = d[k];
        v.perm = p->d_perm;
        v.perm_s = p->d_perm_s;
        v.tasks = p->d_tasks;
        v.torder = p->d_spread_order;
        v.bound = p->d_bound;
        v.multi = p->d_multi;
        v.bin_tasks = p->d_bin_tasks;
        v.merge_order = p->d_merge_order;
        v.grid = p->d_grid;
        v.tmp = p->d_tmp;
        v.partials = p->d_partials;
        v.xs = p->xsplit;
        v.g = p->geom();
        v.nb = p->nb;
        v.K = (int)p->K;
        v.R = p->J - 1;
        v.r2 = p->ball_r2;
        // a plan without tasks launches nothing: an empty range
        const int64_t tb = p->ntasks ? (int64_t)p->xsplit.max_len * NUFFTCT_NUM_XCD : 0;
        const int64_t mb = (int64_t)p->nb * p->nb * p->nb;
        if (st[k] + tb >= ((int64_t)1 << 31) || sm[k] + mb >= ((int64_t)1 << 31))
          return bfail(NUFFTCT_EUNSUPPORTED, "batch too large for one launch per stage");
        st[k + 1] = st[k] + (int32_t)tb;
        sm[k + 1] = sm[k] + (int32_t)mb;
        g.max_tasks = std::max<int64_t>(g.max_tasks, p->ntasks);
      }
      hipError_t e = hipMalloc((void**)&g.d_vols, d.size() * sizeof(BatchPointVol));
      if (e == hipSuccess)
        e = hipMemcpy(g.d_vols, d.data(), d.size() * sizeof(BatchPointVol), hipMemcpyHostToDevice);
      if (e != hipSuccess) return bfail(NUFFTCT_ENOMEM, std::string("batch tables: ") + hipGetErrorString(e));
    }
  // units to worker streams, largest first
  std::vector<double> load(L, 0.0);
  std::vector<int> order(b->classes.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return b->classes[x].cost > b->classes[y].cost; });
  for (int ci : order) {
    const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    b->classes[ci].lane = l;
    load[l] += b->classes[ci].cost;
  }
  b->batched = true;
  return NUFFTCT_OK;
}

// One direction of one size class, one launch per stage (the FFT and radial
// stages in chunks of at most NUFFTCT_BATCH_MAXV volumes, the point stages per
// tile group), in the order of the one-plan path, on stream st.
template <typename T>
static hipError_t run_class_t(nufftct_batch* b, const BatchClassInfo& ci, int dir,
                              const void* const* src, void* const* dst, int flags,
                              hipStream_t st) {
  const bool deriv = (flags & NUFFTCT_DERIV) != 0;
  const bool det = (flags & NUFFTCT_DETERMINISTIC) != 0;
  auto fft = [&](int what) -> hipError_t {
    for (size_t c0 = 0; c0 < ci.vols.size(); c0 += NUFFTCT_BATCH_MAXV) {
      const size_t nv = std::min<size_t>(NUFFTCT_BATCH_MAXV, ci.vols.size() - c0);
      const nufftct_plan* p0 = b->plans[ci.vols[c0]];
      BatchClass<T> c{ci.N, ci.K, ci.n_r, (int)nv, 0, p0->d_s, (const cx<T>*)p0->d_tw_K,
                      (const cx<T>*)p0->d_tw_r};
      BatchArgs a{};
      for (size_t k = 0; k < nv; ++k) {
        const int i = ci.vols[c0 + k];
        const nufftct_plan* p = b->plans[i];
        a.r2[k] = p->ball_r2;
        a.n[k] = p->n_lines;
        c.max_lines = std::max<int64_t>(c.max_lines, p->n_lines);
        switch (what) {
          case 0: a.in[k] = src[i]; a.out[k] = p->d_grid; break;   // forward FFT passes
          case 1: a.in[k] = p->d_grid; a.out[k] = dst[i]; break;   // inverse passes + crop
          case 2: a.in[k] = p->d_tmp; a.out[k] = dst[i]; break;    // radial
          default: a.in[k] = src[i]; a.out[k] = p->d_tmp; break;   // radial adjoint
        }
      }
      hipError_t e = launch_batch_class<T>(c, a, what, deriv, st);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  auto points = [&](int what) -> hipError_t {
    const void* poly = sizeof(T) == 4 ? (const void*)&b->plans[0]->wp32 : (const void*)&b->plans[0]->wp64;
    for (const auto& gi : ci.groups) {
      const int nv = (int)gi.vols.size();
      if (gi.start_tasks.s[nv] == 0 && what == 0) continue;
      BatchGroup g{gi.d_vols, gi.start_tasks, gi.start_tiles, gi.max_tasks, nv, b->plans[0]->J,
                   gi.tile};
      hipError_t e = launch_batch_group<T>(g, what, det, poly, st);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  hipError_t e;
  if (dir == 0) {
    if ((e = fft(0)) != hipSuccess) return e;
    if ((e = points(0)) != hipSuccess) return e;
    return fft(2);
  }
  if ((e = fft(3)) != hipSuccess) return e;
  if ((e = points(1)) != hipSuccess) return e;
  return fft(1);
}

// Each unit on its worker stream, forked from and joined back into the
// caller's stream: the units' FFT and point stages overlap.
static int run_batched(nufftct_batch* b, int dir, const void* const* src, void* const* dst,
                       int flags, void* stream) {
  const int n = (int)b->plans.size();
  for (int i = 0; i < n; ++i) {
    if (!src[i] || !dst[i]) return bfail(NUFFTCT_EINVAL, "null buffer for volume " + std::to_string(i));
    if (src[i] == dst[i]) return bfail(NUFFTCT_EINVAL, "input and output of volume " + std::to_string(i) + " alias");
  }
  if (flags & ~(NUFFTCT_DERIV_RADIAL | NUFFTCT_DETERMINISTIC))
    return bfail(NUFFTCT_EINVAL, "unknown flags " + std::to_string(flags));
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipEventRecord(b->fork, st);
  for (size_t l = 0; l < b->lanes.size() && e == hipSuccess; ++l)
    e = hipStreamWaitEvent(b->lanes[l], b->fork, 0);
  if (e != hipSuccess) return bfail(NUFFTCT_EHIP, std::string("fork: ") + hipGetErrorString(e));
  const bool f32 = b->plans[0]->precision == NUFFTCT_FP32;
  int rc = NUFFTCT_OK;
  for (const auto& ci : b->classes) {
    hipStream_t ls = b->lanes[ci.lane];
    if (ci.vols.size() == 1) {  // a unit of one volume: the plan's own kernels
      const int i = ci.vols[0];
      rc = dir == 0 ? nufftct_forward(b->plans[i], src[i], dst[i], flags, (void*)ls)
                    : nufftct_adjoint(b->plans[i], src[i], dst[i], flags, (void*)ls);
      if (rc) {
        rc = bfail(rc, "volume " + std::to_string(i) + ": " + nufftct_last_error());
        break;
      }
      continue;
    }
    e = f32 ? run_class_t<float>(b, ci, dir, src, dst, flags, ls)
            : run_class_t<double>(b, ci, dir, src, dst, flags, ls);
    if (e != hipSuccess) {
      rc = bfail(NUFFTCT_EHIP, std::string("batched launch: ") + hipGetErrorString(e));
      break;
    }
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

// Run one direction over all volumes: fork the worker streams from the
// caller's stream, run each volume on its lane, join them back.
static int run_dir(nufftct_batch* b, int dir, const void* const* src, void* const* dst, int flags,
                   void* stream) {
  if (b->batched && (flags & NUFFTCT_RADIAL)) return run_batched(b, dir, src, dst, flags, stream);
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

// Batch creation; with `tune`, each size class (equal N, K, n_r) takes the
// tiling the autotuner picks on its member with the most points.
static int batch_create(nufftct_batch** out, int nvol, const int64_t* N, const int64_t* K, int J,
                        int kernel, double beta, int precision, const double* const* dirs,
                        const int64_t* n_lines, const int64_t* n_r, void* stream, bool tune) {
  if (!out) return bfail(NUFFTCT_EINVAL, "out is NULL");
  *out = nullptr;
  if (nvol < 1 || !N || !K || !dirs || !n_lines || !n_r)
    return bfail(NUFFTCT_EINVAL, "nvol must be >= 1 and the size arrays non-NULL");
  nufftct_batch* b = new (std::nothrow) nufftct_batch();
  if (!b) return bfail(NUFFTCT_ENOMEM, "host allocation failed");
  std::vector<int> tile(nvol, 0), max_pts(nvol, 0);
  if (tune) {
    std::vector<bool> done(nvol, false);
    for (int i = 0; i < nvol; ++i) {
      if (done[i]) continue;
      int big = i;  // the class member with the most points
      for (int j = i; j < nvol; ++j)
        if (N[j] == N[i] && K[j] == K[i] && n_r[j] == n_r[i] && n_lines[j] > n_lines[big]) big = j;
      int t = 0, mp = 0;
      if (nufftct_autotune_radial(N[big], K[big], J, kernel, beta, precision, dirs[big],
                                  n_lines[big], n_r[big], NUFFTCT_DERIV_RADIAL, &t, &mp, nullptr,
                                  stream)) {
        std::string m = "autotuning volume " + std::to_string(big) + ": " + nufftct_last_error();
        free_batch(b);
        return bfail(NUFFTCT_EHIP, m);
      }
      for (int j = i; j < nvol; ++j)
        if (N[j] == N[i] && K[j] == K[i] && n_r[j] == n_r[i]) {
          tile[j] = t;
          max_pts[j] = mp;
          done[j] = true;
        }
    }
  }
  for (int i = 0; i < nvol; ++i) {
    nufftct_plan* p = nullptr;
    int rc = plan_create_radial_tiled(&p, N[i], K[i], J, kernel, beta, precision, dirs[i],
                                      n_lines[i], n_r[i], tile[i], max_pts[i], stream);
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
  if (kernel == NUFFTCT_KERNEL_KB) {
    int rc = build_batched(b);
    if (rc) {
      std::string m = nufftct_last_error();
      free_batch(b);
      return bfail(rc, m);
    }
  }
  *out = b;
  return NUFFTCT_OK;
}

extern "C" {

int nufftct_batch_create(nufftct_batch** out, int nvol, const int64_t* N, const int64_t* K, int J,
                         int kernel, double beta, int precision, const double* const* dirs,
                         const int64_t* n_lines, const int64_t* n_r, void* stream) {
  return batch_create(out, nvol, N, K, J, kernel, beta, precision, dirs, n_lines, n_r, stream,
                      false);
}

int nufftct_batch_create_tuned(nufftct_batch** out, int nvol, const int64_t* N, const int64_t* K,
                               int J, int kernel, double beta, int precision,
                               const double* const* dirs, const int64_t* n_lines,
                               const int64_t* n_r, void* stream) {
  return batch_create(out, nvol, N, K, J, kernel, beta, precision, dirs, n_lines, n_r, stream,
                      true);
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
