// Host side of the reverse Grangeat step (Section 2.2.2): argument checks,
// the FP64 tables, the gather form of the KB spreading of the polar points,
// workspaces, and the C ABI entry points.
#include "grangeat.h"

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "tables.h"

static int gfail(int code, const std::string& msg) { return set_last_error(code, msg); }

static void free_grangeat(nufftct_grangeat* g) {
  if (!g) return;
  void* ptrs[] = {g->d_pw, g->d_dcw, g->d_h, g->d_sv, g->d_s, g->d_tw, g->d_off,
                  g->d_pt, g->d_w,   g->d_c, g->d_rows};
  for (void* p : ptrs)
    if (p) hipFree(p);
  delete g;
}

template <typename V>
static bool to_device(void** dst, const std::vector<V>& v) {
  if (hipMalloc(dst, v.size() * sizeof(V) > 0 ? v.size() * sizeof(V) : 16) != hipSuccess) {
    *dst = nullptr;
    return false;
  }
  return v.empty() ||
         hipMemcpy(*dst, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice) == hipSuccess;
}

// The polar points omega_{i,m} = pi (m - n)/n (cos alpha_i, sin alpha_i),
// alpha_i = pi i / n_alpha, each spread onto the K x K grid ([kappa_v][kappa_u],
// cell kappa at kappa mod K) with the J x J KB taps of the neighbour rule
// (s = omega / (2 pi / K) - J/2, taps floor(s) + 1 .. + J, offsets from the
// same s), listed per cell in point order.  The Nyquist points (m = 0) carry
// nothing and are left out.
#pragma clang fp contract(off)
template <typename T>
static bool build_gather(nufftct_grangeat* g, double beta) {
  const int n = g->n, K = g->K, J = g->J, L = 2 * n;
  const double gamma = (2.0 * M_PI) / (double)K;
  struct Tap {
    int kap[NUFFTCT_MAXJ];
    double w[NUFFTCT_MAXJ];
  };
  auto axis = [&](double om, Tap& tp) {
    const double s = om / gamma - 0.5 * (double)J;
    const double k0 = std::floor(s);
    const double frac = s - k0;
    for (int j = 1; j <= J; ++j) {
      int64_t kk = ((int64_t)k0 + j) % K;
      if (kk < 0) kk += K;
      tp.kap[j - 1] = (int)kk;
      tp.w[j - 1] = (double)tables::kb_psi((long double)(0.5 * (double)J - (double)j + frac), J,
                                           (long double)beta);
    }
  };
  const int64_t cells = (int64_t)K * K;
  std::vector<int32_t> count(cells + 1, 0);
  std::vector<Tap> tu((size_t)g->n_alpha * L), tv((size_t)g->n_alpha * L);
  for (int i = 0; i < g->n_alpha; ++i) {
    const double al = M_PI * (double)i / (double)g->n_alpha;
    const double ca = std::cos(al), sa = std::sin(al);
    for (int m = 1; m < L; ++m) {
      const double r = M_PI * (double)(m - n) / (double)n;
      const size_t p = (size_t)i * L + m;
      axis(ca * r, tu[p]);
      axis(sa * r, tv[p]);
      for (int b = 0; b < J; ++b)
        for (int a = 0; a < J; ++a) ++count[(int64_t)tv[p].kap[b] * K + tu[p].kap[a] + 1];
    }
  }
  for (int64_t c = 0; c < cells; ++c) count[c + 1] += count[c];
  g->n_entries = count[cells];
  std::vector<int32_t> pt((size_t)g->n_entries);
  std::vector<T> w((size_t)g->n_entries);
  std::vector<int32_t> fill(count.begin(), count.end() - 1);
  for (int i = 0; i < g->n_alpha; ++i)
    for (int m = 1; m < L; ++m) {
      const size_t p = (size_t)i * L + m;
      for (int b = 0; b < J; ++b)
        for (int a = 0; a < J; ++a) {
          const int64_t cell = (int64_t)tv[p].kap[b] * K + tu[p].kap[a];
          const int32_t e = fill[cell]++;
          pt[e] = (int32_t)p;
          w[e] = (T)(tv[p].w[b] * tu[p].w[a]);
        }
    }
  return to_device((void**)&g->d_off, count) && to_device((void**)&g->d_pt, pt) &&
         to_device(&g->d_w, w);
}

// FP64 tables (see the kernel file for their use).
template <typename T>
static bool build_tables(nufftct_grangeat* g, double beta) {
  const int n = g->n, L = 2 * n;
  const double delta = g->side / (double)n;
  const double dv = delta * g->R / g->D;  // virtual-detector pitch delta'
  const double R2 = g->R * g->R;
  const double dalpha = M_PI / (double)g->n_alpha;
  const double dk = 1.0 / ((double)L * dv);
  std::vector<double> sv(n), pw(n), dcw(n), h(L);
  for (int j = 0; j < n; ++j) {
    sv[j] = (double)(j - n / 2) * dv;
    pw[j] = -(R2 / (R2 + sv[j] * sv[j])) * dv;
    // k = 0 bin: dalpha dk^2 / 6 * P(alpha, 0), P(alpha, 0) = -sum_j s'_j q_j
    // (q_j = p'_j delta' is what the line holds), signed by (-1)^jc
    const double wdc = -sv[j] * (dalpha * dk * dk / 6.0);
    dcw[j] = ((j - n / 2) & 1) ? -wdc : wdc;
  }
  for (int m = 0; m < L; ++m) {
    const int kc = m - n;
    h[m] = m == 0 ? 0.0 : (double)((kc > 0) - (kc < 0)) / (2.0 * M_PI) * dalpha * dk;
  }
  return to_device((void**)&g->d_sv, sv) && to_device((void**)&g->d_pw, pw) &&
         to_device((void**)&g->d_dcw, dcw) && to_device((void**)&g->d_h, h) &&
         to_device((void**)&g->d_s, tables::deapod(n, g->K, g->J, beta)) &&
         to_device(&g->d_tw, tables::twiddles<T>(g->K));
}
#pragma clang fp contract(on)

extern "C" {

int nufftct_grangeat_create(nufftct_grangeat** out, int64_t n_proj, int64_t n_alpha, int64_t n,
                            double source_radius, double source_detector, double detector_side,
                            int J, int precision, void* stream) {
  (void)stream;
  if (!out) return gfail(NUFFTCT_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_proj < 1 || n_alpha < 1 || n < 2)
    return gfail(NUFFTCT_EINVAL, "n_proj, n_alpha must be >= 1 and n >= 2");
  if (!grangeat_length_supported(n))
    return gfail(n % 2 ? NUFFTCT_EINVAL : NUFFTCT_EUNSUPPORTED,
                 "n must be one of the compiled detector sizes 16 24 32 48 64 96 128 160 192 "
                 "256 320 384 512 (got " + std::to_string(n) + ")");
  if (n_proj > (int64_t)1 << 20 || n_alpha > 65535)
    return gfail(NUFFTCT_EINVAL, "n_proj must be <= 2^20 and n_alpha <= 65535");
  if (n_alpha * 2 * n * n_proj >= (int64_t)1 << 31 || n_alpha * 2 * n * 64 >= (int64_t)1 << 31)
    return gfail(NUFFTCT_EINVAL, "n_alpha * 2n * max(n_proj, 64) must be < 2^31");
  if (!(source_radius > 0) || !(source_detector > 0) || !(detector_side > 0) ||
      !std::isfinite(source_radius) || !std::isfinite(source_detector) ||
      !std::isfinite(detector_side))
    return gfail(NUFFTCT_EINVAL, "scan distances must be finite and > 0");
  if (J < 2 || J > NUFFTCT_MAXJ) return gfail(NUFFTCT_EINVAL, "J must be in [2, 8]");
  if (precision != NUFFTCT_FP32 && precision != NUFFTCT_FP64)
    return gfail(NUFFTCT_EINVAL, "unknown precision");
  nufftct_grangeat* g = new (std::nothrow) nufftct_grangeat();
  if (!g) return gfail(NUFFTCT_ENOMEM, "host allocation failed");
  g->n_proj = (int)n_proj;
  g->n_alpha = (int)n_alpha;
  g->n = (int)n;
  g->K = 2 * (int)n;
  g->J = J;
  g->precision = precision;
  g->R = source_radius;
  g->D = source_detector;
  g->side = detector_side;
  const double beta = 2.34 * J;
  const bool f32 = precision == NUFFTCT_FP32;
  const size_t cxb = f32 ? 8 : 16;
  bool ok = f32 ? build_tables<float>(g, beta) && build_gather<float>(g, beta)
                : build_tables<double>(g, beta) && build_gather<double>(g, beta);
  g->c_bytes = (size_t)n_alpha * 2 * n * n_proj * cxb;
  g->rows_bytes = (size_t)n_proj * 2 * n * n * cxb;
  if (ok && hipMalloc(&g->d_c, g->c_bytes) != hipSuccess) {
    g->d_c = nullptr;
    ok = false;
  }
  if (ok && hipMalloc(&g->d_rows, g->rows_bytes) != hipSuccess) {
    g->d_rows = nullptr;
    ok = false;
  }
  if (!ok) {
    free_grangeat(g);
    return gfail(NUFFTCT_ENOMEM, "device allocation or copy failed");
  }
  *out = g;
  return NUFFTCT_OK;
}

int nufftct_grangeat_project(nufftct_grangeat* g, const void* umbrella, void* out, void* stream) {
  if (!g) return gfail(NUFFTCT_EINVAL, "object is NULL");
  if (!umbrella || !out) return gfail(NUFFTCT_EINVAL, "data pointer is NULL");
  if (umbrella == out) return gfail(NUFFTCT_EINVAL, "input and output must not alias");
  hipStream_t st = (hipStream_t)stream;
  const bool f32 = g->precision == NUFFTCT_FP32;
  hipError_t e = f32 ? launch_grangeat_radial<float>(*g, umbrella, g->d_c, st)
                     : launch_grangeat_radial<double>(*g, umbrella, g->d_c, st);
  if (e == hipSuccess)
    e = f32 ? launch_grangeat_backproject<float>(*g, g->d_c, out, st)
            : launch_grangeat_backproject<double>(*g, g->d_c, out, st);
  if (e != hipSuccess) return gfail(NUFFTCT_EHIP, std::string("launch failed: ") + hipGetErrorString(e));
  return NUFFTCT_OK;
}

int nufftct_grangeat_stage(nufftct_grangeat* g, int stage, const void* in, void* out,
                           void* stream) {
  if (!g) return gfail(NUFFTCT_EINVAL, "object is NULL");
  if (!in || !out) return gfail(NUFFTCT_EINVAL, "data pointer is NULL");
  if (in == out) return gfail(NUFFTCT_EINVAL, "input and output must not alias");
  hipStream_t st = (hipStream_t)stream;
  const bool f32 = g->precision == NUFFTCT_FP32;
  hipError_t e;
  if (stage == NUFFTCT_GR_STAGE_SPECTRA)
    e = f32 ? launch_grangeat_radial<float>(*g, in, out, st)
            : launch_grangeat_radial<double>(*g, in, out, st);
  else if (stage == NUFFTCT_GR_STAGE_BACKPROJECT)
    e = f32 ? launch_grangeat_backproject<float>(*g, in, out, st)
            : launch_grangeat_backproject<double>(*g, in, out, st);
  else
    return gfail(NUFFTCT_EINVAL, "unknown stage");
  if (e != hipSuccess) return gfail(NUFFTCT_EHIP, std::string("launch failed: ") + hipGetErrorString(e));
  return NUFFTCT_OK;
}

int nufftct_grangeat_info(const nufftct_grangeat* g, int64_t* n_entries) {
  if (!g || !n_entries) return gfail(NUFFTCT_EINVAL, "NULL argument");
  *n_entries = g->n_entries;
  return NUFFTCT_OK;
}

int nufftct_grangeat_destroy(nufftct_grangeat* g) {
  free_grangeat(g);
  return NUFFTCT_OK;
}

}  // extern "C"
