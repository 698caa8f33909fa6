// Host side of the radial -> umbrella resampling (Section 2.1.3: method 2,
// eq 2.15, and method 1, eq 2.11): argument checks, the scan and grid
// constants, the method-1 tables and workspace, and the C ABI entry points.
#include "umbrella.h"

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "tables.h"

static int ufail(int code, const std::string& msg) { return set_last_error(code, msg); }

static int make_umbrella(nufftct_umbrella** out, int64_t n_proj, int64_t n_alpha, int64_t n_t,
                         double source_radius, double source_detector, double detector_side,
                         int64_t n_phi, int64_t n_theta, double theta0, double dtheta,
                         int64_t n_r, int J, int precision) {
  if (!out) return ufail(NUFFTCT_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_proj < 1 || n_alpha < 1 || n_t < 1 || n_phi < 1 || n_theta < 1 || n_r < 2)
    return ufail(NUFFTCT_EINVAL, "sample counts must be >= 1 (n_r >= 2)");
  if (n_proj * n_alpha > ((int64_t)1 << 31) / n_t)
    return ufail(NUFFTCT_EINVAL, "n_proj * n_alpha * n_t must be < 2^31");
  if (n_phi * n_theta > ((int64_t)1 << 31) / n_r)
    return ufail(NUFFTCT_EINVAL, "n_phi * n_theta * n_r must be < 2^31");
  if (!(source_radius > 0) || !(source_detector > 0) || !(detector_side > 0) ||
      !std::isfinite(source_radius) || !std::isfinite(source_detector) ||
      !std::isfinite(detector_side))
    return ufail(NUFFTCT_EINVAL, "scan distances must be finite and > 0");
  if (!std::isfinite(theta0) || !(dtheta > 0) || !std::isfinite(dtheta))
    return ufail(NUFFTCT_EINVAL, "theta0 must be finite and dtheta > 0");
  if (J < 2 || J > NUFFTCT_MAXJ) return ufail(NUFFTCT_EINVAL, "J must be in [2, 8]");
  if (precision != NUFFTCT_FP32 && precision != NUFFTCT_FP64)
    return ufail(NUFFTCT_EINVAL, "unknown precision");
  nufftct_umbrella* u = new (std::nothrow) nufftct_umbrella();
  if (!u) return ufail(NUFFTCT_ENOMEM, "host allocation failed");
  u->J = J;
  u->precision = precision;
  UmbrellaGeom& g = u->g;
  g.n_proj = (int)n_proj;
  g.n_alpha = (int)n_alpha;
  g.n_t = (int)n_t;
  g.n_phi = (int)n_phi;
  g.n_theta = (int)n_theta;
  g.n_r = (int)n_r;
  g.R_s = source_radius;
  g.D_sd = source_detector;
  g.dt = detector_side / (double)n_t;
  g.theta0 = theta0;
  g.inv_dtheta = 1.0 / dtheta;
  g.inv_dphi = (double)n_phi / (2.0 * M_PI);
  // method-2 weights: the sinc truncated by the KB window of width J,
  // beta = 4J/3, normalised over the J taps (evaluated in the kernel)
  g.beta = 4.0 * J / 3.0;
  g.inv_i0beta = (double)(1.0L / tables::bessel_i0((long double)g.beta));
  *out = u;
  return NUFFTCT_OK;
}

static void free_umbrella(nufftct_umbrella* u) {
  if (!u) return;
  for (int d = 0; d < 3; ++d) {
    if (u->d_tw_n[d]) hipFree(u->d_tw_n[d]);
    if (u->d_tw_k[d]) hipFree(u->d_tw_k[d]);
    if (u->d_sc[d]) hipFree(u->d_sc[d]);
  }
  if (u->d_grid) hipFree(u->d_grid);
  delete u;
}

template <typename V>
static hipError_t to_device(void** dst, const std::vector<V>& v) {
  hipError_t e = hipMalloc(dst, v.size() * sizeof(V));
  if (e != hipSuccess) {
    *dst = nullptr;
    return e;
  }
  return hipMemcpy(*dst, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice);
}

// Method-1 tables: per axis the twiddles of lengths N_d and K_d = 2 N_d, the
// scaling s_d(m) / N_d (the KB deapodization of the projector's NUFFT, over
// the inverse DFT's 1/N_d), the KB weight polynomials, and the grid workspace.
template <typename T>
static int build_method1(nufftct_umbrella* u) {
  const int64_t n[3] = {u->g.n_phi, u->g.n_theta, u->g.n_r};
  const double beta = 2.34 * u->J;
  for (int d = 0; d < 3; ++d) {
    const int64_t N = n[d], K = 2 * N;
    u->K[d] = K;
    if (to_device(&u->d_tw_n[d], tables::twiddles<T>(N)) != hipSuccess ||
        to_device(&u->d_tw_k[d], tables::twiddles<T>(K)) != hipSuccess)
      return ufail(NUFFTCT_ENOMEM, "twiddle tables: device allocation or copy failed");
    std::vector<double> sc = tables::deapod(N, K, u->J, beta);
    for (auto& v : sc) v /= (double)N;
    if (to_device((void**)&u->d_sc[d], sc) != hipSuccess)
      return ufail(NUFFTCT_ENOMEM, "scaling tables: device allocation or copy failed");
  }
  const int deg = sizeof(T) == 4 ? NUFFTCT_DEG_F32 : NUFFTCT_DEG_F64;
  std::vector<long double> re;
  const long double err = tables::fit_kb(u->J, beta, deg, re);
  const long double tol = sizeof(T) == 4 ? 1e-7L : 1e-12L;
  if (!(err <= tol)) return ufail(NUFFTCT_EUNSUPPORTED, "KB weight polynomial fit error too large");
  for (int a = 0; a < u->J; ++a)
    for (int k = 0; k <= deg; ++k) {
      const long double r = re[(size_t)a * (deg + 1) + k];
      if (sizeof(T) == 4) u->wp32.re[a][k] = (float)r;
      else u->wp64.re[a][k] = (double)r;
    }
  const size_t cells = (size_t)u->K[0] * (size_t)u->K[1] * (size_t)u->K[2];
  u->grid_bytes = cells * 2 * sizeof(T);
  if (hipMalloc(&u->d_grid, u->grid_bytes) != hipSuccess) {
    u->d_grid = nullptr;
    return ufail(NUFFTCT_ENOMEM, "grid workspace: device allocation failed");
  }
  return NUFFTCT_OK;
}

extern "C" {

int nufftct_umbrella_create(nufftct_umbrella** out, int64_t n_proj, int64_t n_alpha, int64_t n_t,
                            double source_radius, double source_detector, double detector_side,
                            int64_t n_phi, int64_t n_theta, double theta0, double dtheta,
                            int64_t n_r, int J, int precision, void* stream) {
  (void)stream;
  int rc = make_umbrella(out, n_proj, n_alpha, n_t, source_radius, source_detector, detector_side,
                         n_phi, n_theta, theta0, dtheta, n_r, J, precision);
  if (rc) return rc;
  // per-tap polynomial weights (the same function the kernel would evaluate)
  nufftct_umbrella* u = *out;
  const bool f32 = precision == NUFFTCT_FP32;
  const int deg = f32 ? NUFFTCT_UMB_DEG_F32 : NUFFTCT_UMB_DEG_F64;
  std::vector<long double> re;
  const long double err = tables::fit_window_sinc(J, u->g.beta, deg, re);
  u->poly = err <= (f32 ? 1e-7L : 1e-13L);
  for (int a = 0; a < J; ++a)
    for (int k = 0; k <= deg; ++k) {
      const long double c = re[(size_t)a * (deg + 1) + k];
      if (f32) u->tp32.c[a][k] = (float)c;
      else u->tp64.c[a][k] = (double)c;
    }
  return NUFFTCT_OK;
}

int nufftct_umbrella1_create(nufftct_umbrella** out, int64_t n_proj, int64_t n_alpha,
                             int64_t n_t, double source_radius, double source_detector,
                             double detector_side, int64_t n_phi, int64_t n_theta,
                             double theta0, double dtheta, int64_t n_r, int J, int precision,
                             void* stream) {
  (void)stream;
  if (out) *out = nullptr;
  const int64_t n[3] = {n_phi, n_theta, n_r};
  for (int d = 0; d < 3; ++d)
    if (n[d] >= 1 && !resample1_length_supported(n[d]))
      return ufail(n[d] % 2 ? NUFFTCT_EINVAL : NUFFTCT_EUNSUPPORTED,
                   "method 1: n_phi, n_theta, n_r must each be one of the compiled even lengths "
                   "8..512 with 2n = 2^a 3^b 5^c (got " + std::to_string(n[d]) + ")");
  nufftct_umbrella* u = nullptr;
  int rc = make_umbrella(&u, n_proj, n_alpha, n_t, source_radius, source_detector, detector_side,
                         n_phi, n_theta, theta0, dtheta, n_r, J, precision);
  if (rc) return rc;
  u->method = 1;
  rc = precision == NUFFTCT_FP32 ? build_method1<float>(u) : build_method1<double>(u);
  if (rc) {
    free_umbrella(u);
    return rc;
  }
  *out = u;
  return NUFFTCT_OK;
}

int nufftct_umbrella_resample(nufftct_umbrella* u, const void* radial, void* out, void* stream) {
  if (!u) return ufail(NUFFTCT_EINVAL, "resampler is NULL");
  if (!radial || !out) return ufail(NUFFTCT_EINVAL, "data pointer is NULL");
  if (radial == out) return ufail(NUFFTCT_EINVAL, "input and output must not alias");
  hipStream_t st = (hipStream_t)stream;
  const bool f32 = u->precision == NUFFTCT_FP32;
  hipError_t e;
  if (u->method == 1) {
    e = f32 ? launch_resample1_grid<float>(*u, radial, u->d_grid, st)
            : launch_resample1_grid<double>(*u, radial, u->d_grid, st);
    if (e == hipSuccess)
      e = f32 ? launch_resample1_gather<float>(*u, u->d_grid, out, st)
              : launch_resample1_gather<double>(*u, u->d_grid, out, st);
  } else {
    e = f32 ? launch_umbrella<float>(*u, radial, out, st) : launch_umbrella<double>(*u, radial, out, st);
  }
  if (e != hipSuccess) return ufail(NUFFTCT_EHIP, std::string("launch failed: ") + hipGetErrorString(e));
  return NUFFTCT_OK;
}

int nufftct_umbrella_grid_shape(const nufftct_umbrella* u, int64_t* K3) {
  if (!u || !K3) return ufail(NUFFTCT_EINVAL, "NULL argument");
  if (u->method != 1) return ufail(NUFFTCT_EINVAL, "only method 1 has an oversampled grid");
  for (int d = 0; d < 3; ++d) K3[d] = u->K[d];
  return NUFFTCT_OK;
}

int nufftct_umbrella_stage(nufftct_umbrella* u, int stage, const void* in, void* out,
                           void* stream) {
  if (!u) return ufail(NUFFTCT_EINVAL, "resampler is NULL");
  if (u->method != 1) return ufail(NUFFTCT_EINVAL, "only method 1 has stages");
  if (!in || !out) return ufail(NUFFTCT_EINVAL, "data pointer is NULL");
  if (in == out) return ufail(NUFFTCT_EINVAL, "input and output must not alias");
  hipStream_t st = (hipStream_t)stream;
  const bool f32 = u->precision == NUFFTCT_FP32;
  hipError_t e;
  if (stage == NUFFTCT_UMB_STAGE_GRID)
    e = f32 ? launch_resample1_grid<float>(*u, in, out, st) : launch_resample1_grid<double>(*u, in, out, st);
  else if (stage == NUFFTCT_UMB_STAGE_GATHER)
    e = f32 ? launch_resample1_gather<float>(*u, in, out, st)
            : launch_resample1_gather<double>(*u, in, out, st);
  else
    return ufail(NUFFTCT_EINVAL, "unknown stage");
  if (e != hipSuccess) return ufail(NUFFTCT_EHIP, std::string("launch failed: ") + hipGetErrorString(e));
  return NUFFTCT_OK;
}

int nufftct_umbrella_destroy(nufftct_umbrella* u) {
  free_umbrella(u);
  return NUFFTCT_OK;
}

}  // extern "C"
