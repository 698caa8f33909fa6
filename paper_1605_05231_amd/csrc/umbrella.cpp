// Host side of the radial -> umbrella resampling (method 2, eq 2.15): argument
// checks, the scan and grid constants, and the C ABI entry points.
#include "umbrella.h"

#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "tables.h"

static int ufail(int code, const std::string& msg) { return set_last_error(code, msg); }

extern "C" {

int nufftct_umbrella_create(nufftct_umbrella** out, int64_t n_proj, int64_t n_alpha, int64_t n_t,
                            double source_radius, double source_detector, double detector_side,
                            int64_t n_phi, int64_t n_theta, double theta0, double dtheta,
                            int64_t n_r, int J, int precision, void* stream) {
  (void)stream;
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
  // weights: the sinc truncated by the KB window of width J, beta = 4J/3,
  // normalised over the J taps (evaluated in the kernel)
  g.beta = 4.0 * J / 3.0;
  g.inv_i0beta = (double)(1.0L / tables::bessel_i0((long double)g.beta));
  *out = u;
  return NUFFTCT_OK;
}

int nufftct_umbrella_resample(nufftct_umbrella* u, const void* radial, void* out, void* stream) {
  if (!u) return ufail(NUFFTCT_EINVAL, "resampler is NULL");
  if (!radial || !out) return ufail(NUFFTCT_EINVAL, "data pointer is NULL");
  if (radial == out) return ufail(NUFFTCT_EINVAL, "input and output must not alias");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = u->precision == NUFFTCT_FP32 ? launch_umbrella<float>(*u, radial, out, st)
                                              : launch_umbrella<double>(*u, radial, out, st);
  if (e != hipSuccess) return ufail(NUFFTCT_EHIP, std::string("launch failed: ") + hipGetErrorString(e));
  return NUFFTCT_OK;
}

int nufftct_umbrella_destroy(nufftct_umbrella* u) {
  delete u;
  return NUFFTCT_OK;
}

}  // extern "C"
