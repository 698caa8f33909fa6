// C-ABI of the NUFFT derivative-Radon projector: plan construction (FP64
// tables, point binning, workspaces), forward/adjoint orchestration, stage
// timing and error reporting.  No exceptions cross the interface.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <mutex>
#include <thread>
#include <vector>

#include "host_plan.h"
#include "plan.h"
#include "tables.h"

static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int set_last_error(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) {                                                                   \
      int code_ = (e_ == hipErrorOutOfMemory) ? NUFFTCT_ENOMEM : NUFFTCT_EHIP;                \
      return fail(code_, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__,     \
                  __LINE__);                                                                  \
    }                                                                                         \
  } while (0)

static bool is_235(int64_t L) {
  if (L <= 0) return false;
  while (L % 2 == 0) L /= 2;
  while (L % 3 == 0) L /= 3;
  while (L % 5 == 0) L /= 5;
  return L == 1;
}

bool fft_length_supported(int64_t L) {
  static const int64_t sizes[] = {16, 32, 48, 64, 80, 96, 128, 160,
                                  192, 256, 320, 384, 512, 640, 768, 1024};
  for (int64_t s : sizes)
    if (s == L) return true;
  return false;
}

static int env_int(const char* name, int dflt) {
  const char* v = getenv(name);
  if (!v || !*v) return dflt;
  return atoi(v);
}

// ---------------------------------------------------------------------------
static void free_plan(nufftct_plan* p) {
  if (!p) return;
  hipFree(p->d_dirs);
  hipFree(p->d_pts);
  hipFree(p->d_s);
  hipFree(p->d_tw_K);
  hipFree(p->d_tw_r);
  hipFree(p->d_perm);
  hipFree(p->d_perm_s);
  hipFree(p->d_tasks);
  hipFree(p->d_bin_tasks);
  hipFree(p->d_merge_order);
  hipFree(p->d_spread_order);
  hipFree(p->d_partials);
  hipFree(p->d_bound);
  hipFree(p->d_multi);
  hipFree(p->d_line_w);
  hipFree(p->d_grid);
  hipFree(p->d_tmp);
  for (auto& e : p->events) {
    hipEventDestroy(e.a);
    hipEventDestroy(e.b);
  }
  delete p;
}

template <typename T>
static int upload(void** dst, const T* src, size_t n, hipStream_t st) {
  HIP_TRY(hipMalloc(dst, n * sizeof(T) > 0 ? n * sizeof(T) : 16));
  if (n) HIP_TRY(hipMemcpyAsync(*dst, src, n * sizeof(T), hipMemcpyHostToDevice, st));
  return NUFFTCT_OK;
}

static int validate(int64_t N, int64_t K, int J, int kernel, double beta, int precision,
                    int64_t M, int64_t n_r) {
  if (N < 2 || N % 2) return fail(NUFFTCT_EINVAL, "N must be even and >= 2 (got %lld)", (long long)N);
  if (K < N || K % 2) return fail(NUFFTCT_EINVAL, "K must be even and >= N (got K=%lld, N=%lld)", (long long)K, (long long)N);
  if (J < 2 || J > NUFFTCT_MAXJ || J > K)
    return fail(NUFFTCT_EINVAL, "J must be in [2, %d] and <= K (got %d)", NUFFTCT_MAXJ, J);
  if (kernel != NUFFTCT_KERNEL_KB && kernel != NUFFTCT_KERNEL_MINMAX_KB)
    return fail(NUFFTCT_EINVAL, "unknown kernel %d", kernel);
  if (precision != NUFFTCT_FP32 && precision != NUFFTCT_FP64)
    return fail(NUFFTCT_EINVAL, "unknown precision %d", precision);
  if (!(beta <= 3.0 * J) || std::isnan(beta))
    return fail(NUFFTCT_EINVAL, "beta must be <= 3*J (got %g)", beta);
  if (M < 1 || M >= (int64_t)1 << 31)
    return fail(NUFFTCT_EINVAL, "M must be in [1, 2^31) (got %lld)", (long long)M);
  if (n_r < 0 || (n_r > 0 && (n_r % 2 || M % n_r)))
    return fail(NUFFTCT_EINVAL, "n_r must be 0 or an even divisor of M (got %lld)", (long long)n_r);
  if (!is_235(K)) return fail(NUFFTCT_EUNSUPPORTED, "K=%lld has a prime factor > 5", (long long)K);
  if (!fft_length_supported(K))
    return fail(NUFFTCT_EUNSUPPORTED, "K=%lld is not among the compiled FFT lengths", (long long)K);
  if (n_r > 0 && !is_235(n_r))
    return fail(NUFFTCT_EUNSUPPORTED, "n_r=%lld has a prime factor > 5", (long long)n_r);
  if (n_r > 0 && !fft_length_supported(n_r))
    return fail(NUFFTCT_EUNSUPPORTED, "n_r=%lld is not among the compiled FFT lengths", (long long)n_r);
  return NUFFTCT_OK;
}

// ---------------------------------------------------------------------------
// Autotuning of the tiling (tile edge, points per task).  Results live in a
// process-wide table keyed by the plan's shape and are consulted by every plan
// creation; NUFFTCT_TUNE_CACHE names an optional text file that persists them.
// The key holds a hash of the direction (or point) coordinates, so that two
// geometries with equal counts do not share a tiling.
struct TuneKey {
  int64_t N, K;
  int J, kernel, precision;
  int64_t n_lines, n_r, M;
  uint64_t geom_hash;
  bool operator==(const TuneKey& o) const {
    return N == o.N && K == o.K && J == o.J && kernel == o.kernel && precision == o.precision &&
           n_lines == o.n_lines && n_r == o.n_r && M == o.M && geom_hash == o.geom_hash;
  }
};

// FNV-1a over the bytes of the coordinates
static uint64_t geom_hash(const double* g, int64_t n) {
  uint64_t h = 1469598103934665603ull;
  const unsigned char* b = reinterpret_cast<const unsigned char*>(g);
  for (int64_t i = 0; i < n * (int64_t)sizeof(double); ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}
struct TuneVal {
  int tile, max_pts;
};
static std::mutex g_tune_mu;
static std::vector<std::pair<TuneKey, TuneVal>> g_tune;
static bool g_tune_loaded = false;

static void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = getenv("NUFFTCT_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  TuneKey k;
  TuneVal v;
  long long a[8];
  unsigned long long hsh;
  while (fscanf(f, "%lld %lld %lld %lld %lld %lld %lld %lld %llx %d %d", &a[0], &a[1], &a[2],
                &a[3], &a[4], &a[5], &a[6], &a[7], &hsh, &v.tile, &v.max_pts) == 11) {
    k = TuneKey{a[0], a[1], (int)a[2], (int)a[3], (int)a[4], a[5], a[6], a[7], (uint64_t)hsh};
    g_tune.push_back({k, v});
  }
  fclose(f);
}

static bool tune_lookup(const TuneKey& k, TuneVal* v) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  for (auto it = g_tune.rbegin(); it != g_tune.rend(); ++it)
    if (it->first == k) {
      *v = it->second;
      return true;
    }
  return false;
}

static void tune_store(const TuneKey& k, const TuneVal& v) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  tune_load_locked();
  g_tune.push_back({k, v});
  const char* path = getenv("NUFFTCT_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%lld %lld %d %d %d %lld %lld %lld %llx %d %d\n", (long long)k.N, (long long)k.K,
          k.J, k.kernel, k.precision, (long long)k.n_lines, (long long)k.n_r, (long long)k.M,
          (unsigned long long)k.geom_hash, v.tile, v.max_pts);
  fclose(f);
}

static int create(nufftct_plan** out, int64_t N, int64_t K, int J, int kernel, double beta,
                  int precision, int64_t M, int64_t n_r, bool radial, const double* geom,
                  int64_t n_geom, hipStream_t st, int tile_req, int maxpts_req) {
  if (!out) return fail(NUFFTCT_EINVAL, "out is NULL");
  *out = nullptr;
  if (!geom) return fail(NUFFTCT_EINVAL, "point/direction array is NULL");
  if (beta <= 0) beta = 2.34 * J;
  int rc = validate(N, K, J, kernel, beta, precision, M, n_r);
  if (rc) return rc;
  std::vector<double> g(geom, geom + 3 * n_geom);
  for (double v : g)
    if (!std::isfinite(v) || std::fabs(v) > 1e6)
      return fail(NUFFTCT_EINVAL, "points/directions must be finite and |v| <= 1e6");

  nufftct_plan* p = new (std::nothrow) nufftct_plan();
  if (!p) return fail(NUFFTCT_ENOMEM, "host allocation failed");
  p->N = N;
  p->K = K;
  p->J = J;
  p->kernel = kernel;
  p->beta = beta;
  p->precision = precision;
  p->M = M;
  p->n_r = n_r;
  p->radial = radial;
  p->n_lines = radial ? n_geom : (n_r ? M / n_r : 0);
  // tile edge: divides K, J - 1 <= tile, and the spread's FP64 halo tile of
  // (tile + J - 1)^3 cells fits in LDS
  // order of precedence: explicit request (autotuner) > environment > tuned
  // table > default
  TuneKey tkey{N, K, J, kernel, precision, p->n_lines, n_r, M, geom_hash(geom, 3 * n_geom)};
  TuneVal tuned{0, 0};
  const bool have_tuned = tune_lookup(tkey, &tuned);
  {
    auto halo_bytes = [&](int t) { return (t + J - 1) * (t + J - 1) * (t + J - 1) * 16; };
    int t = precision == NUFFTCT_FP32 ? 16 : 8;
    if (have_tuned) t = tuned.tile;
    t = env_int("NUFFTCT_TILE", t);
    if (tile_req) t = tile_req;
    if (t != 8 && t != 16) t = 16;
    if (t == 16 && (K % 16 || halo_bytes(16) > 160 * 1024)) t = 8;
    if (K % t || J - 1 > t || halo_bytes(t) > 160 * 1024) {
      free_plan(p);
      return fail(NUFFTCT_EINVAL, "no tile edge fits K=%lld, J=%d", (long long)K, J);
    }
    p->tile = t;
  }
  p->nb = (int)(K / p->tile);
  {
    int mp = have_tuned ? tuned.max_pts : 4096;
    mp = env_int("NUFFTCT_MAXPTS", mp);
    if (maxpts_req) mp = maxpts_req;
    p->max_pts = std::max(256, mp);
  }

  auto bail = [&](int code) {
    free_plan(p);
    return code;
  };

  // deapodization and twiddles
  std::vector<double> s = tables::deapod(N, K, J, beta);
  if ((rc = upload((void**)&p->d_s, s.data(), s.size(), st))) return bail(rc);
  if (precision == NUFFTCT_FP32) {
    auto tk = tables::twiddles<float>(K);
    if ((rc = upload(&p->d_tw_K, tk.data(), tk.size(), st))) return bail(rc);
    if (n_r) {
      auto tr = tables::twiddles<float>(n_r);
      if ((rc = upload(&p->d_tw_r, tr.data(), tr.size(), st))) return bail(rc);
    }
  } else {
    auto tk = tables::twiddles<double>(K);
    if ((rc = upload(&p->d_tw_K, tk.data(), tk.size(), st))) return bail(rc);
    if (n_r) {
      auto tr = tables::twiddles<double>(n_r);
      if ((rc = upload(&p->d_tw_r, tr.data(), tr.size(), st))) return bail(rc);
    }
  }

  // weight polynomials
  {
    const int deg = precision == NUFFTCT_FP32 ? NUFFTCT_DEG_F32 : NUFFTCT_DEG_F64;
    std::vector<long double> re, im;
    long double err;
    if (kernel == NUFFTCT_KERNEL_KB) {
      err = tables::fit_kb(J, beta, deg, re);
      im.assign(re.size(), 0.0L);
    } else {
      tables::MinMax mm(N, K, J, s);
      err = tables::fit_minmax(mm, deg, re, im);
    }
    const long double tol = precision == NUFFTCT_FP32 ? 1e-7L : 1e-12L;
    if (!(err <= tol)) {
      free_plan(p);
      return fail(NUFFTCT_EUNSUPPORTED, "weight polynomial fit error %Lg exceeds %Lg", err, tol);
    }
    std::memset(&p->wp32, 0, sizeof(p->wp32));
    std::memset(&p->wp64, 0, sizeof(p->wp64));
    for (int a = 0; a < J; ++a)
      for (int k = 0; k <= deg; ++k) {
        const long double r = re[(size_t)a * (deg + 1) + k], i = im[(size_t)a * (deg + 1) + k];
        if (precision == NUFFTCT_FP32) {
          p->wp32.re[a][k] = (float)r;
          p->wp32.im[a][k] = (float)i;
        } else {
          p->wp64.re[a][k] = (double)r;
          p->wp64.im[a][k] = (double)i;
        }
      }
  }

  // geometry
  if (radial) {
    if ((rc = upload((void**)&p->d_dirs, g.data(), g.size(), st))) return bail(rc);
  } else {
    if ((rc = upload((void**)&p->d_pts, g.data(), g.size(), st))) return bail(rc);
  }

  // ball holding every tap: |t| <= t_max for every point, taps within
  // J sqrt(3)/2 of t; one extra cell of margin
  {
    double tmax = 0.0;
    if (radial) {
      for (int64_t l = 0; l < n_geom; ++l) {
        const double nn = std::sqrt(g[3 * l] * g[3 * l] + g[3 * l + 1] * g[3 * l + 1] +
                                    g[3 * l + 2] * g[3 * l + 2]);
        tmax = std::max(tmax, nn * M_PI * (double)K / (2.0 * M_PI));
      }
    } else {
      for (int64_t i = 0; i < M; ++i) {
        const double nn = std::sqrt(g[3 * i] * g[3 * i] + g[3 * i + 1] * g[3 * i + 1] +
                                    g[3 * i + 2] * g[3 * i + 2]);
        tmax = std::max(tmax, nn * (double)K / (2.0 * M_PI));
      }
    }
    const double R = tmax * (1.0 + 1e-12) + 0.5 * std::sqrt(3.0) * J + 1.0;
    p->ball_r2 = R < 0.5 * std::sqrt(3.0) * (double)K ? R * R : 1e300;
  }

  // binning
  {
    hostplan::Binning B;
    hostplan::BinParams bp;
    bp.M = p->M;
    bp.K = p->K;
    bp.n_r = p->n_r;
    bp.J = J;
    bp.tile = p->tile;
    bp.nb = p->nb;
    bp.max_pts = p->max_pts;
    bp.radial = p->radial;
    bp.fp32 = precision == NUFFTCT_FP32;
    // the FP32 spreading with Kaiser-Bessel weights sums paired points'
    // contributions; the other kernels spread one point at a time
    bp.pair_spread = bp.fp32 && kernel != NUFFTCT_KERNEL_MINMAX_KB;
    // the FP32 interpolation serves the two points of a frequency sampled
    // twice with one evaluation (their frequencies agree to FP64 rounding,
    // far below the FP32 result's precision); the Kaiser-Bessel spreading
    // also spreads such a pair with one set of weights
    bp.twins = bp.fp32;
    hostplan::build_bins(bp, g, B);
    p->ntasks = (int64_t)B.tasks.size();
    {
      // cut the task list into NUFFTCT_NUM_XCD contiguous ranges of equal point count
      int64_t total = 0;
      for (const auto& t : B.tasks) total += t.count;
      int64_t acc = 0;
      size_t i = 0;
      p->xsplit.start[0] = 0;
      for (int x = 1; x < NUFFTCT_NUM_XCD; ++x) {
        const int64_t target = total * x / NUFFTCT_NUM_XCD;
        while (i < B.tasks.size() && acc + B.tasks[i].count / 2 < target) acc += B.tasks[i++].count;
        p->xsplit.start[x] = (int32_t)i;
      }
      p->xsplit.start[NUFFTCT_NUM_XCD] = (int32_t)B.tasks.size();
      p->xsplit.max_len = 0;
      for (int x = 0; x < NUFFTCT_NUM_XCD; ++x)
        p->xsplit.max_len = std::max(p->xsplit.max_len, p->xsplit.start[x + 1] - p->xsplit.start[x]);
      p->xsplit.max_len = std::max(p->xsplit.max_len, 1);
    }
    if ((rc = upload((void**)&p->d_perm, B.perm.data(), B.perm.size(), st))) return bail(rc);
    if ((rc = upload((void**)&p->d_perm_s, B.perm_s.data(), B.perm_s.size(), st))) return bail(rc);
    if ((rc = upload((void**)&p->d_tasks, B.tasks.data(), B.tasks.size(), st))) return bail(rc);
    if ((rc = upload((void**)&p->d_bin_tasks, B.bin_tasks.data(), B.bin_tasks.size(), st)))
      return bail(rc);
    {
      // merge dispatch order: the tiles that sum the most partial cells first,
      // so that the dense centre's long per-cell task loops do not form the tail
      const int nb = p->nb, T = p->tile, R = J - 1;
      const int64_t nt = (int64_t)nb * nb * nb;
      std::vector<int64_t> cost(nt, 0);
      for (int64_t t = 0; t < nt; ++t) {
        const int t2 = (int)(t % nb), t1 = (int)((t / nb) % nb), t0 = (int)(t / ((int64_t)nb * nb));
        for (int delta = 0; delta < 8; ++delta) {
          const int d0 = (delta >> 2) & 1, d1 = (delta >> 1) & 1, d2 = delta & 1;
          const int64_t sb = (((int64_t)((t0 - d0 + nb) % nb) * nb + (t1 - d1 + nb) % nb) * nb) +
                             (t2 - d2 + nb) % nb;
          const int64_t cells = (int64_t)(d0 ? R : T) * (d1 ? R : T) * (d2 ? R : T);
          cost[t] += (int64_t)(B.bin_tasks[sb + 1] - B.bin_tasks[sb]) * cells;
        }
      }
      std::vector<int32_t> order(nt);
      for (int64_t t = 0; t < nt; ++t) order[t] = (int32_t)t;
      std::stable_sort(order.begin(), order.end(),
                       [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
      if ((rc = upload((void**)&p->d_merge_order, order.data(), order.size(), st))) return bail(rc);
    }
    {
      // spreading dispatch order: inside each XCD's task range the largest
      // tasks first, so that the last ones to start are short
      std::vector<int32_t> torder(B.tasks.size());
      for (size_t t = 0; t < torder.size(); ++t) torder[t] = (int32_t)t;
      for (int x = 0; x < NUFFTCT_NUM_XCD; ++x)
        std::stable_sort(torder.begin() + p->xsplit.start[x], torder.begin() + p->xsplit.start[x + 1],
                         [&](int32_t a, int32_t b) { return B.tasks[a].count > B.tasks[b].count; });
      if ((rc = upload((void**)&p->d_spread_order, torder.data(), torder.size(), st))) return bail(rc);
    }
    const size_t cxb = precision == NUFFTCT_FP32 ? 8 : 16;
    // per-task stride: the halo's S^3 cells rounded up to 16 (the merge's
    // loads then start on 128-byte lines)
    const size_t S = (size_t)(p->tile + J - 1);
    const size_t pstride = (S * S * S + 15) / 16 * 16;
    const size_t pbytes = (size_t)std::max<int64_t>(p->ntasks, 1) * pstride * cxb;
    hipError_t e = hipMalloc(&p->d_partials, pbytes);
    if (e != hipSuccess) {
      free_plan(p);
      return fail(NUFFTCT_ENOMEM, "spread partial tiles of %zu bytes: %s", pbytes, hipGetErrorString(e));
    }
    p->partial_bytes = pbytes;
    // host vectors go out of scope after the copies complete
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      free_plan(p);
      return fail(NUFFTCT_EHIP, "plan upload failed: %s", hipGetErrorString(e));
    }
  }

  // workspaces
  const size_t cxb = precision == NUFFTCT_FP32 ? 8 : 16;
  p->grid_bytes = ((size_t)K * (size_t)grid_plane(K, (int)cxb) * cxb + 255) / 256 * 256;
  p->tmp_bytes = (size_t)M * cxb;
  {
    hipError_t e = hipMalloc(&p->d_grid, p->grid_bytes);
    if (e != hipSuccess) {
      free_plan(p);
      return fail(NUFFTCT_ENOMEM, "workspace of %zu bytes: %s", p->grid_bytes, hipGetErrorString(e));
    }
    e = hipMalloc(&p->d_tmp, p->tmp_bytes);
    if (e != hipSuccess) {
      free_plan(p);
      return fail(NUFFTCT_ENOMEM, "workspace of %zu bytes: %s", p->tmp_bytes, hipGetErrorString(e));
    }
  }
  // per-task bounds that set the fixed-point spreading's scale (FP32 always,
  // FP64 in deterministic mode)
  {
    const size_t bbytes = (size_t)std::max<int64_t>(p->ntasks, 1) * sizeof(float);
    hipError_t e = hipMalloc(&p->d_bound, bbytes);
    const size_t mbytes = (size_t)(std::max<int64_t>(p->ntasks, 1) + 1) * sizeof(int32_t);
    if (e == hipSuccess) e = hipMalloc(&p->d_multi, mbytes);
    if (e == hipSuccess) e = hipMemsetAsync(p->d_multi, 0, mbytes, st);  // the empty list
    if (e != hipSuccess) {
      free_plan(p);
      return fail(NUFFTCT_ENOMEM, "spread bounds of %zu bytes: %s", bbytes, hipGetErrorString(e));
    }
    e = precision == NUFFTCT_FP32 ? launch_spread_bound<float>(*p, st)
                                  : launch_spread_bound<double>(*p, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      free_plan(p);
      return fail(NUFFTCT_EHIP, "spread bound kernel failed: %s", hipGetErrorString(e));
    }
  }
  *out = p;
  g_err.clear();
  return NUFFTCT_OK;
}

// ---------------------------------------------------------------------------
// stage execution with optional event timing
struct StageTimer {
  nufftct_plan* p;
  hipStream_t st;
  int stage;
  hipEvent_t a = nullptr, b = nullptr;
  // (timing is best effort: a stage whose events cannot be created or
  // recorded goes untimed, and the launch itself is unaffected)
  StageTimer(nufftct_plan* p_, hipStream_t st_, int stage_) : p(p_), st(st_), stage(stage_) {
    if (!p->timing) return;
    if (hipEventCreate(&a) != hipSuccess) a = nullptr;
    if (a && hipEventCreate(&b) != hipSuccess) b = nullptr;
    if (a && b && hipEventRecord(a, st) == hipSuccess) return;
    release();
  }
  void done() {
    if (!a || !b) return;
    if (hipEventRecord(b, st) == hipSuccess) {
      p->events.push_back({a, b, stage});
      a = b = nullptr;
    } else {
      release();
    }
  }
  void release() {
    if (a) hipEventDestroy(a);
    if (b) hipEventDestroy(b);
    a = b = nullptr;
  }
  ~StageTimer() { release(); }
};

// prune: grid cells outside the taps' ball are neither produced nor read
// (the operator paths); the single-stage entry point works on full grids
// internal flag (never accepted from callers): the adjoint radial stage scales
// line l by w_l / (8 pi^2), the direct reconstruction of Section 2.3
constexpr int FLAG_LINE_WEIGHTS = 1 << 16;
// 3D inverse Fourier transform in spherical coordinates over whole lines,
// with the radial sum's 2 pi: 1 / (2 (2 pi)^3) * 2 pi
constexpr double RECON_SCALE = 1.0 / (8.0 * M_PI * M_PI);

template <typename T>
static hipError_t run_stage(nufftct_plan* p, int stage, const void* in, void* out, int flags,
                            hipStream_t st, bool prune) {
  StageTimer tm(p, st, stage);
  hipError_t e = hipSuccess;
  switch (stage) {
    case NUFFTCT_STAGE_PAD_FFT:
      e = launch_pad_fft<T>(*p, in, out, st, prune);
      break;
    case NUFFTCT_STAGE_INTERP:
      e = launch_interp<T>(*p, in, out, st);
      break;
    case NUFFTCT_STAGE_RADIAL:
      e = launch_radial<T>(*p, in, out, false, (flags & NUFFTCT_DERIV) != 0, st);
      break;
    case NUFFTCT_STAGE_RADIAL_ADJ:
      e = launch_radial<T>(*p, in, out, true, (flags & NUFFTCT_DERIV) != 0, st,
                           (flags & FLAG_LINE_WEIGHTS) ? p->d_line_w : nullptr, RECON_SCALE);
      break;
    case NUFFTCT_STAGE_SPREAD: {
      // halo partials per task, then the owner-computes merge writes every
      // grid cell (timed on its own slot)
      e = launch_spread<T>(*p, in, out, st, (flags & NUFFTCT_DETERMINISTIC) != 0);
      tm.done();
      StageTimer tr(p, st, NUFFTCT_TIMING_MERGE);
      if (e == hipSuccess) e = launch_merge<T>(*p, out, st, prune);
      tr.done();
      break;
    }
    case NUFFTCT_STAGE_IFFT_CROP:
      // in-place on `in` (a K^3 grid the caller or the plan owns)
      e = launch_ifft_crop<T>(*p, const_cast<void*>(in), out, st, prune);
      break;
    default:
      e = hipErrorInvalidValue;
  }
  tm.done();
  return e;
}

static int check_call(nufftct_plan* p, const void* a, void* b, int flags) {
  if (!p) return fail(NUFFTCT_EINVAL, "plan is NULL");
  if (!a || !b) return fail(NUFFTCT_EINVAL, "data pointer is NULL");
  if (a == b) return fail(NUFFTCT_EINVAL, "input and output must not alias");
  if (flags & ~(NUFFTCT_DERIV_RADIAL | NUFFTCT_DETERMINISTIC))
    return fail(NUFFTCT_EINVAL, "unknown flags %d", flags);
  if ((flags & NUFFTCT_DERIV) && !(flags & NUFFTCT_RADIAL))
    return fail(NUFFTCT_EINVAL, "NUFFTCT_DERIV requires NUFFTCT_RADIAL");
  if ((flags & NUFFTCT_RADIAL) && p->n_r == 0)
    return fail(NUFFTCT_EINVAL, "plan has no radial lines (n_r = 0)");
  return NUFFTCT_OK;
}

#define STAGE_TRY(expr)                                                                     \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail(NUFFTCT_EHIP, "launch failed: %s", hipGetErrorString(e_)); \
  } while (0)

template <typename T>
static int forward_impl(nufftct_plan* p, const void* vol, void* out, int flags, hipStream_t st) {
  STAGE_TRY(run_stage<T>(p, NUFFTCT_STAGE_PAD_FFT, vol, p->d_grid, flags, st, true));
  if (flags & NUFFTCT_RADIAL) {
    STAGE_TRY(run_stage<T>(p, NUFFTCT_STAGE_INTERP, p->d_grid, p->d_tmp, flags, st, true));
    STAGE_TRY(run_stage<T>(p, NUFFTCT_STAGE_RADIAL, p->d_tmp, out, flags, st, true));
  } else {
    STAGE_TRY(run_stage<T>(p, NUFFTCT_STAGE_INTERP, p->d_grid, out, flags, st, true));
  }
  return NUFFTCT_OK;
}

// ---------------------------------------------------------------------------
// Forward operator with its workspace (the K^3 spectrum grid, then the M
// interpolated values ahead of the radial stage) in one static device array
// instead of the plan's: nothing is allocated per call, so that callers who
// cannot call hipMalloc (code under graph capture, tight serving loops) can
// use it.  The array is a host-side stand-in in host code; its device address
// is taken once per device with hipGetSymbolAddress and used everywhere.
#define NUFFTCT_STATIC_SCRATCH_BYTES (64ull << 20)
static __device__ __align__(256) unsigned char scratch[NUFFTCT_STATIC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64] = {nullptr};

static int scratch_address(void** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(NUFFTCT_EUNSUPPORTED, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return NUFFTCT_OK;
}

template <typename T>
static int forward_noalloc_impl(nufftct_plan* p, const void* vol, void* out, int flags,
                                hipStream_t st, unsigned char* ws) {
  void* grid = ws;
  void* tmp = ws + p->grid_bytes;  // grid_bytes is a multiple of 256
  STAGE_TRY(launch_pad_fft<T>(*p, vol, grid, st, true));
  if (flags & NUFFTCT_RADIAL) {
    STAGE_TRY(launch_interp<T>(*p, grid, tmp, st));
    STAGE_TRY(launch_radial<T>(*p, tmp, out, false, (flags & NUFFTCT_DERIV) != 0, st));
  } else {
    STAGE_TRY(launch_interp<T>(*p, grid, out, st));
  }
  return NUFFTCT_OK;
}

template <typename T>
static int adjoint_impl(nufftct_plan* p, const void* in, void* vol, int flags, hipStream_t st) {
  const void* src = in;
  if (flags & NUFFTCT_RADIAL) {
    STAGE_TRY(run_stage<T>(p, NUFFTCT_STAGE_RADIAL_ADJ, in, p->d_tmp, flags, st, true));
    src = p->d_tmp;
  }
  STAGE_TRY(run_stage<T>(p, NUFFTCT_STAGE_SPREAD, src, p->d_grid, flags, st, true));
  STAGE_TRY(run_stage<T>(p, NUFFTCT_STAGE_IFFT_CROP, p->d_grid, vol, flags, st, true));
  return NUFFTCT_OK;
}

// ---------------------------------------------------------------------------
extern "C" {

int nufftct_plan_create(nufftct_plan** out, int64_t N, int64_t K, int J, int kernel, double beta,
                        int precision, const double* points, int64_t M, int64_t n_r,
                        void* stream) {
  return create(out, N, K, J, kernel, beta, precision, M, n_r, false, points, M,
                (hipStream_t)stream, 0, 0);
}

int nufftct_plan_create_radial(nufftct_plan** out, int64_t N, int64_t K, int J, int kernel,
                               double beta, int precision, const double* dirs, int64_t n_lines,
                               int64_t n_r, void* stream) {
  if (n_lines < 1) {
    if (out) *out = nullptr;
    return fail(NUFFTCT_EINVAL, "n_lines must be >= 1");
  }
  if (n_r < 4) {
    if (out) *out = nullptr;
    return fail(NUFFTCT_EINVAL, "n_r must be >= 4 for a radial plan");
  }
  if (n_lines > ((int64_t)1 << 31) / n_r) {
    if (out) *out = nullptr;
    return fail(NUFFTCT_EINVAL, "n_lines * n_r must be < 2^31");
  }
  return create(out, N, K, J, kernel, beta, precision, n_lines * n_r, n_r, true, dirs, n_lines,
                (hipStream_t)stream, 0, 0);
}

}  // extern "C"

int plan_create_radial_tiled(nufftct_plan** out, int64_t N, int64_t K, int J, int kernel,
                             double beta, int precision, const double* dirs, int64_t n_lines,
                             int64_t n_r, int tile, int max_pts, void* stream) {
  if (n_lines < 1 || n_r < 4 || n_lines > ((int64_t)1 << 31) / n_r) {
    if (out) *out = nullptr;
    return fail(NUFFTCT_EINVAL, "bad radial geometry");
  }
  return create(out, N, K, J, kernel, beta, precision, n_lines * n_r, n_r, true, dirs, n_lines,
                (hipStream_t)stream, tile, max_pts);
}

extern "C" {

int nufftct_autotune_radial(int64_t N, int64_t K, int J, int kernel, double beta, int precision,
                            const double* dirs, int64_t n_lines, int64_t n_r, int flags,
                            int* best_tile, int* best_max_pts, double* best_ms, void* stream) {
  if (n_lines < 1 || n_r < 4 || !dirs) return fail(NUFFTCT_EINVAL, "bad radial geometry");
  if (flags & ~NUFFTCT_DERIV_RADIAL) return fail(NUFFTCT_EINVAL, "unknown flags %d", flags);
  hipStream_t st = (hipStream_t)stream;
  const int64_t M = n_lines * n_r;
  const size_t cxb = precision == NUFFTCT_FP64 ? 16 : 8;
  void* vol = nullptr;
  void* out = nullptr;
  HIP_TRY(hipMalloc(&vol, (size_t)N * N * N * cxb));
  if (hipMalloc(&out, (size_t)M * cxb) != hipSuccess) {
    hipFree(vol);
    return fail(NUFFTCT_ENOMEM, "autotune buffers");
  }
  // Inputs: pseudo-random values in [-1, 1) for the volume and, separately,
  // for the adjoint's input.  The spreading's cost depends on the spread of
  // magnitudes within a task (tasks spanning many binades take an extra
  // pass); random data keep that spread ordinary, where a constant volume, or
  // the forward output of one, would not.
  hipEvent_t e0 = nullptr, e1 = nullptr;
  void* din = nullptr;
  hipError_t he = hipMalloc(&din, (size_t)M * cxb);
  {
    uint64_t st64 = 0x9e3779b97f4a7c15ull;
    auto next = [&]() {  // xorshift64*
      st64 ^= st64 >> 12;
      st64 ^= st64 << 25;
      st64 ^= st64 >> 27;
      return (double)((st64 * 2685821657736338717ull) >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    };
    auto fill = [&](void* dst, size_t ncomplex) {
      const size_t nval = 2 * ncomplex;
      if (precision == NUFFTCT_FP64) {
        std::vector<double> h(nval);
        for (auto& v : h) v = next();
        hipError_t e = hipMemcpyAsync(dst, h.data(), nval * sizeof(double), hipMemcpyHostToDevice, st);
        return e == hipSuccess ? hipStreamSynchronize(st) : e;  // before h goes out of scope
      }
      std::vector<float> h(nval);
      for (auto& v : h) v = (float)next();
      hipError_t e = hipMemcpyAsync(dst, h.data(), nval * sizeof(float), hipMemcpyHostToDevice, st);
      return e == hipSuccess ? hipStreamSynchronize(st) : e;
    };
    if (he == hipSuccess) he = fill(vol, (size_t)N * N * N);
    if (he == hipSuccess) he = fill(din, (size_t)M);
  }
  if (he == hipSuccess) he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  if (he != hipSuccess) {
    if (e0) hipEventDestroy(e0);
    hipFree(vol);
    hipFree(out);
    hipFree(din);
    return fail(NUFFTCT_EHIP, "autotune set-up: %s", hipGetErrorString(he));
  }
  const int tiles[2] = {16, 8};
  const int mps[6] = {1024, 2048, 4096, 8192, 12288, 16384};
  double best = 1e30;
  TuneVal bv{0, 0};
  for (int t : tiles)
    for (int mp : mps) {
      nufftct_plan* p = nullptr;
      if (create(&p, N, K, J, kernel, beta, precision, M, n_r, true, dirs, n_lines, st, t, mp))
        continue;  // e.g. the tile does not fit this (K, J) or memory ran out
      if (p->tile != t) {  // the tile was adjusted: already covered by another candidate
        free_plan(p);
        continue;
      }
      int rc = nufftct_forward(p, vol, out, flags, stream);
      if (!rc) rc = nufftct_adjoint(p, din, vol, flags, stream);
      if (!rc && hipEventRecord(e0, st) != hipSuccess) rc = NUFFTCT_EHIP;
      for (int r = 0; r < 2 && !rc; ++r) {
        rc = nufftct_forward(p, vol, out, flags, stream);
        if (!rc) rc = nufftct_adjoint(p, din, vol, flags, stream);
      }
      if (!rc && hipEventRecord(e1, st) != hipSuccess) rc = NUFFTCT_EHIP;
      float ms = 0;
      if (!rc && hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess &&
          ms / 2 < best) {
        best = ms / 2;
        bv = TuneVal{t, mp};
      }
      const hipError_t se = hipStreamSynchronize(st);
      free_plan(p);
      if (se != hipSuccess) {  // a fault of a candidate: stop tuning
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        hipFree(vol);
        hipFree(out);
        hipFree(din);
        return fail(NUFFTCT_EHIP, "autotune candidate failed: %s", hipGetErrorString(se));
      }
    }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipFree(vol);
  hipFree(out);
  hipFree(din);
  if (bv.tile == 0) return fail(NUFFTCT_EHIP, "no autotune candidate ran");
  tune_store(TuneKey{N, K, J, kernel, precision, n_lines, n_r, M, geom_hash(dirs, 3 * n_lines)}, bv);
  if (best_tile) *best_tile = bv.tile;
  if (best_max_pts) *best_max_pts = bv.max_pts;
  if (best_ms) *best_ms = best;
  g_err.clear();
  return NUFFTCT_OK;
}

int nufftct_forward(nufftct_plan* p, const void* vol, void* out, int flags, void* stream) {
  int rc = check_call(p, vol, out, flags);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  return p->precision == NUFFTCT_FP32 ? forward_impl<float>(p, vol, out, flags, st)
                                      : forward_impl<double>(p, vol, out, flags, st);
}

int nufftct_forward_noalloc(nufftct_plan* p, const void* vol, void* out, int flags, void* stream) {
  int rc = check_call(p, vol, out, flags);
  if (rc) return rc;
  const size_t need = p->grid_bytes + ((flags & NUFFTCT_RADIAL) ? p->tmp_bytes : 0);
  if (need > NUFFTCT_STATIC_SCRATCH_BYTES)
    return fail(NUFFTCT_EINVAL,
                "nufftct_forward_noalloc: the plan needs %zu bytes of workspace (K^3 grid%s), "
                "more than the %llu-byte static scratch array",
                need, (flags & NUFFTCT_RADIAL) ? " and M values" : "",
                (unsigned long long)NUFFTCT_STATIC_SCRATCH_BYTES);
  void* ws = nullptr;
  if ((rc = scratch_address(&ws))) return rc;
  hipStream_t st = (hipStream_t)stream;
  return p->precision == NUFFTCT_FP32
             ? forward_noalloc_impl<float>(p, vol, out, flags, st, (unsigned char*)ws)
             : forward_noalloc_impl<double>(p, vol, out, flags, st, (unsigned char*)ws);
}

int nufftct_adjoint(nufftct_plan* p, const void* in, void* vol, int flags, void* stream) {
  int rc = check_call(p, in, vol, flags);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  return p->precision == NUFFTCT_FP32 ? adjoint_impl<float>(p, in, vol, flags, st)
                                      : adjoint_impl<double>(p, in, vol, flags, st);
}

int nufftct_radial_quadrature(const double* phi, int64_t n_phi, const double* theta,
                              int64_t n_theta, double* w) {
  if (!phi || !theta || !w) return fail(NUFFTCT_EINVAL, "null array");
  if (n_phi < 1 || n_theta < 1) return fail(NUFFTCT_EINVAL, "n_phi and n_theta must be >= 1");
  for (int64_t i = 0; i < n_phi; ++i)
    if (!std::isfinite(phi[i])) return fail(NUFFTCT_EINVAL, "phi must be finite");
  for (int64_t i = 0; i < n_theta; ++i)
    if (!std::isfinite(theta[i])) return fail(NUFFTCT_EINVAL, "theta must be finite");
  for (int64_t i = 1; i < n_theta; ++i)
    if (!(theta[i] > theta[i - 1])) return fail(NUFFTCT_EINVAL, "theta must increase");
  const double tau = 2.0 * M_PI;
  auto wrap = [&](double v) {  // into [0, 2 pi)
    v = std::fmod(v, tau);
    return v < 0 ? v + tau : v;
  };
  for (int64_t a = 0; a < n_phi; ++a) {
    // periodic midpoint spacing: half the way to each neighbour
    double da = tau;
    if (n_phi > 1) {
      const double next = phi[(a + 1) % n_phi], prev = phi[(a + n_phi - 1) % n_phi];
      da = 0.5 * (wrap(next - phi[a]) + wrap(phi[a] - prev));
    }
    for (int64_t b = 0; b < n_theta; ++b) {
      // trapezoid rule in theta over [theta_0, theta_last]
      double db = 2.0;  // one polar angle: the sine integral of the whole sphere
      if (n_theta > 1) {
        db = 0.0;
        if (b > 0) db += 0.5 * (theta[b] - theta[b - 1]);
        if (b + 1 < n_theta) db += 0.5 * (theta[b + 1] - theta[b]);
      }
      w[a * n_theta + b] = da * db * std::sin(theta[b]);
    }
  }
  g_err.clear();
  return NUFFTCT_OK;
}

int nufftct_set_line_weights(nufftct_plan* p, const double* w, void* stream) {
  if (!p) return fail(NUFFTCT_EINVAL, "plan is NULL");
  if (!w) return fail(NUFFTCT_EINVAL, "weights are NULL");
  if (p->n_r == 0 || p->n_lines < 1) return fail(NUFFTCT_EINVAL, "plan has no radial lines (n_r = 0)");
  for (int64_t l = 0; l < p->n_lines; ++l)
    if (!std::isfinite(w[l])) return fail(NUFFTCT_EINVAL, "weight of line %lld is not finite", (long long)l);
  hipStream_t st = (hipStream_t)stream;
  if (!p->d_line_w) {
    hipError_t e = hipMalloc(&p->d_line_w, (size_t)p->n_lines * sizeof(double));
    if (e != hipSuccess) {
      p->d_line_w = nullptr;
      return fail(NUFFTCT_ENOMEM, "line weights: %s", hipGetErrorString(e));
    }
  }
  HIP_TRY(hipMemcpyAsync(p->d_line_w, w, (size_t)p->n_lines * sizeof(double), hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  g_err.clear();
  return NUFFTCT_OK;
}

int nufftct_reconstruct(nufftct_plan* p, const void* in, void* vol, void* stream) {
  int rc = check_call(p, in, vol, NUFFTCT_DERIV_RADIAL);
  if (rc) return rc;
  if (!p->d_line_w) return fail(NUFFTCT_EINVAL, "no line weights set (nufftct_set_line_weights)");
  hipStream_t st = (hipStream_t)stream;
  const int flags = NUFFTCT_DERIV_RADIAL | FLAG_LINE_WEIGHTS;
  return p->precision == NUFFTCT_FP32 ? adjoint_impl<float>(p, in, vol, flags, st)
                                      : adjoint_impl<double>(p, in, vol, flags, st);
}

int nufftct_stage(nufftct_plan* p, int stage, const void* in, void* out, int flags, void* stream) {
  if (!p) return fail(NUFFTCT_EINVAL, "plan is NULL");
  if (!in || !out) return fail(NUFFTCT_EINVAL, "data pointer is NULL");
  if (in == out) return fail(NUFFTCT_EINVAL, "input and output must not alias");
  if (stage < 0 || stage > NUFFTCT_STAGE_IFFT_CROP) return fail(NUFFTCT_EINVAL, "unknown stage %d", stage);
  if ((stage == NUFFTCT_STAGE_RADIAL || stage == NUFFTCT_STAGE_RADIAL_ADJ) && p->n_r == 0)
    return fail(NUFFTCT_EINVAL, "plan has no radial lines (n_r = 0)");
  hipStream_t st = (hipStream_t)stream;
  // the caller's grids are compact (K^3 cells); the plan's grid has planes
  // grid_plane cells apart, which may include a pad
  const size_t cxb = p->precision == NUFFTCT_FP32 ? 8 : 16;
  const size_t plane = (size_t)p->K * p->K * cxb, pitch = (size_t)grid_plane(p->K, (int)cxb) * cxb;
  const bool padded = pitch != plane;
  const bool grid_in = stage == NUFFTCT_STAGE_INTERP || stage == NUFFTCT_STAGE_IFFT_CROP;
  const bool grid_out = stage == NUFFTCT_STAGE_PAD_FFT || stage == NUFFTCT_STAGE_SPREAD;
  const void* src = in;
  void* dst = out;
  if (grid_in && (padded || stage == NUFFTCT_STAGE_IFFT_CROP)) {
    // (the inverse passes run in place: the caller's grid stays intact)
    HIP_TRY(hipMemcpy2DAsync(p->d_grid, pitch, in, plane, plane, (size_t)p->K, hipMemcpyDeviceToDevice, st));
    src = p->d_grid;
  }
  if (grid_out && padded) dst = p->d_grid;
  hipError_t e = p->precision == NUFFTCT_FP32 ? run_stage<float>(p, stage, src, dst, flags, st, false)
                                              : run_stage<double>(p, stage, src, dst, flags, st, false);
  if (e != hipSuccess) return fail(NUFFTCT_EHIP, "launch failed: %s", hipGetErrorString(e));
  if (dst != out)
    HIP_TRY(hipMemcpy2DAsync(out, plane, p->d_grid, pitch, plane, (size_t)p->K, hipMemcpyDeviceToDevice, st));
  return NUFFTCT_OK;
}

int nufftct_plan_destroy(nufftct_plan* p) {
  if (!p) return NUFFTCT_OK;
  free_plan(p);
  return NUFFTCT_OK;
}

int nufftct_plan_info(const nufftct_plan* p, int64_t* N, int64_t* K, int* J, int64_t* M,
                      int64_t* n_r, int* precision, int64_t* workspace_bytes) {
  if (!p) return fail(NUFFTCT_EINVAL, "plan is NULL");
  if (N) *N = p->N;
  if (K) *K = p->K;
  if (J) *J = p->J;
  if (M) *M = p->M;
  if (n_r) *n_r = p->n_r;
  if (precision) *precision = p->precision;
  if (workspace_bytes) *workspace_bytes = (int64_t)(p->grid_bytes + p->tmp_bytes + p->partial_bytes);
  return NUFFTCT_OK;
}

int nufftct_plan_tiling(const nufftct_plan* p, int* tile, int* max_pts) {
  if (!p) return fail(NUFFTCT_EINVAL, "plan is NULL");
  if (tile) *tile = p->tile;
  if (max_pts) *max_pts = p->max_pts;
  return NUFFTCT_OK;
}

int nufftct_set_timing(nufftct_plan* p, int enable) {
  if (!p) return fail(NUFFTCT_EINVAL, "plan is NULL");
  p->timing = enable != 0;
  return NUFFTCT_OK;
}

int nufftct_get_stage_times(nufftct_plan* p, double* ms, int64_t* count, int n) {
  if (!p) return fail(NUFFTCT_EINVAL, "plan is NULL");
  for (auto& e : p->events) {
    HIP_TRY(hipEventSynchronize(e.b));
    float t = 0;
    HIP_TRY(hipEventElapsedTime(&t, e.a, e.b));
    p->stage_ms[e.stage] += t;
    p->stage_cnt[e.stage] += 1;
    hipEventDestroy(e.a);
    hipEventDestroy(e.b);
  }
  p->events.clear();
  for (int s = 0; s < n && s < 8; ++s) {
    if (ms) ms[s] = p->stage_ms[s];
    if (count) count[s] = p->stage_cnt[s];
  }
  for (int s = 0; s < 8; ++s) {
    p->stage_ms[s] = 0;
    p->stage_cnt[s] = 0;
  }
  return NUFFTCT_OK;
}

const char* nufftct_last_error(void) { return g_err.c_str(); }

const char* nufftct_version(void) { return "nufftct 0.1 (gfx950)"; }

}  // extern "C"
