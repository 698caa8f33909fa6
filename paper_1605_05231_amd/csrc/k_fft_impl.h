// Deapodize/zero-pad + oversampled 3D FFT, inverse 3D FFT + crop/deapodize,
// and the radial derivative DFT stage, as LDS-tiled kernels for gfx950.
//
// Grid layout: K^3 complex, last axis fastest, planes of axis 0 grid_plane
// cells apart (K^2, padded for large planes), stored CENTRED: cell j of an
// axis holds frequency kappa = j - K/2.  The centring costs nothing: the
// padded input is multiplied by (-1)^(m0+m1+m2), which shifts the spectrum of
// an unnormalised FFT by K/2 (folded into the deapodization factor).
//
// Forward (F1+F2, eq 2.10-2.11 with P the deapodization):
//   pass x : for each voxel row (n0,n1): load N values, scale by
//            s(m0)s(m1)s(m2)(-1)^(m0+m1+m2), place at (m2 mod K), FFT along
//            axis 2, store the K outputs at row ((m0 mod K), (m1 mod K)).
//   pass y : for the N populated planes (m0 mod K): FFT along axis 1 loading
//            only the N populated rows (zero-pruned), storing all K.
//   pass z : for every (j1, j2): FFT along axis 0 loading the N populated
//            planes, storing all K.
// Adjoint (A2+A1) mirrors it with inverse FFTs, storing only the N needed
// outputs of each pass and fusing the crop and deapodization into pass x.
// Both directions also skip the grid cells outside the ball that contains
// every tap of every point (see k_fft_strided).
#pragma once

#include "cx.h"
#include "fft_lds.h"
#include "plan.h"
#include "stage.h"

namespace kfft {

constexpr int NT = 512;    // threads of a line-major workgroup
constexpr int NTS = 1024;  // threads of a strided-pass workgroup

template <typename T, int L>
constexpr int nl_line() {  // lines per tile for line-major passes
  constexpr int target = sizeof(T) == 4 ? 4096 : 2048;
  return target / L > 0 ? target / L : 1;
}

// columns per tile for strided passes: FP32 16 adjacent columns (128-byte row
// segments); 8 or 32 measured slower
template <typename T, int L>
constexpr int nl_col() {
  if constexpr (sizeof(T) == 4) return L <= 512 ? 16 : 8;
  return L <= 512 ? 8 : 4;
}

__device__ __forceinline__ int centred_of(int e, int K) { return e < K / 2 ? e : e - K; }

__device__ __forceinline__ int wrap_of(int m, int K) { return m >= 0 ? m : m + K; }

// ---------------------------------------------------------------------------
// forward pass x (deapodize + pad + FFT along the contiguous axis)
// (each kernel below is a device body taking its block indices, wrapped by a
// one-plan kernel here and by the batch kernels of k_batch_impl.h)
template <typename T, int L>
__device__ __forceinline__ void pad_fft_x_body(int64_t bx, const cx<T>* __restrict__ vol,
                                               cx<T>* __restrict__ grid,
                                               const double* __restrict__ s,
                                               const cx<T>* __restrict__ tw, int N) {
  constexpr int NL = nl_line<T, L>();
  constexpr int K = L;
  __shared__ cx<T> buf[fft::tile_elems<true, L, NL>()];
  __shared__ cx<T> twl[L];
  for (int i = threadIdx.x; i < L; i += NT) twl[i] = tw[i];
  const cx<T>* twp = twl;
  const int tid = threadIdx.x;
  const int64_t nlines = (int64_t)N * N;
  const int64_t line0 = bx * NL;
  const int h = N / 2;
  stage::tile<T, NL * L, NT>(
      tid,
      [&](int idx) {
        const int line = idx / L, e = idx % L;
        const int64_t gl = line0 + line;
        cx<T> v = {0, 0};
        const int m2 = centred_of(e, K);
        if (gl < nlines && m2 >= -h && m2 < h) {
          const int n0 = (int)gl / N, n1 = (int)gl % N, n2 = m2 + h;  // N^2 < 2^31
          const cx<T> xv = vol[gl * N + n2];
          double f = s[n0] * s[n1] * s[n2];
          if ((n0 + n1 + n2 + 3 * h) & 1) f = -f;
          v.x = (T)((double)xv.x * f);
          v.y = (T)((double)xv.y * f);
        }
        return v;
      },
      [&](int idx, cx<T> v) { buf[fft::addr<true, L, NL>(idx / L, idx % L)] = v; });
  __syncthreads();
  fft::run<T, L, NL, NT, true, -1>(buf, twp, tid);
  for (int idx = tid; idx < NL * L; idx += NT) {
    const int line = idx / L, e = idx % L;
    const int64_t gl = line0 + line;
    if (gl < nlines) {
      const int n0 = (int)gl / N, n1 = (int)gl % N;
      const int q0 = wrap_of(n0 - h, K), q1 = wrap_of(n1 - h, K);
      grid[(int64_t)q0 * grid_plane_of<T>(K) + (int64_t)q1 * K + e] = buf[fft::addr<true, L, NL>(line, e)];
    }
  }
}

template <typename T, int L>
__global__ __launch_bounds__(NT) void k_pad_fft_x(const cx<T>* __restrict__ vol,
                                                  cx<T>* __restrict__ grid,
                                                  const double* __restrict__ s,
                                                  const cx<T>* __restrict__ tw, int N) {
  pad_fft_x_body<T, L>(blockIdx.x, vol, grid, s, tw, N);
}

// ---------------------------------------------------------------------------
// strided pass (axis 1 or 0): NLC adjacent columns per workgroup.
//   outer index o: pruned -> plane (o - N/2) mod K for o < N; else o < K
//   load_pruned : only rows whose centred index lies in [-N/2, N/2) are read
//   store_pruned: only those rows are written
// Ball pruning (r2 = R^2, +inf disables it): only cells whose centred
// frequency (kappa = j - K/2 on each transformed axis) satisfies
// kappa_row^2 + [kappa_outer^2] + kappa_col^2 <= R^2 are ever read by the
// interpolation or non-zero after the spread (every tap lies within J sqrt(3)/2
// of a point with |t| <= R0).  ball = 1: store only such rows (forward);
// ball = 2: load only such rows, the rest being zero (adjoint).  outer_in_ball
// says whether the outer index is a transformed (centred) axis.
template <typename T, int L, int S>
__device__ __forceinline__ void fft_strided_body(int bx, int by, int gx, cx<T>* __restrict__ grid,
                                                 const cx<T>* __restrict__ tw, int N,
                                                 int64_t row_stride, int64_t outer_stride,
                                                 int outer_pruned, int load_pruned,
                                                 int store_pruned, double r2, int ball,
                                                 int outer_in_ball) {
  constexpr int NL = nl_col<T, L>();
  constexpr int K = L;
  __shared__ cx<T> buf[fft::tile_elems<false, L, NL>()];
  // the twiddle table in LDS: every stage's twiddle reads become LDS reads
  // (broadcast across the columns of a butterfly row)
  __shared__ cx<T> twl[L];
  for (int i = threadIdx.x; i < L; i += NTS) twl[i] = tw[i];
  const cx<T>* twp = twl;
  const int tid = threadIdx.x;
  const int h = N / 2;
  const int o = by;
  const int qo = outer_pruned ? wrap_of(o - h, K) : o;
  // workgroups go round-robin over the 8 XCDs: give each XCD a contiguous
  // run of column groups, so that the groups sharing a cache line of a row
  // meet in one L2
  int cg = bx;
  if ((gx & (NUFFTCT_NUM_XCD - 1)) == 0)
    cg = (cg % NUFFTCT_NUM_XCD) * (gx / NUFFTCT_NUM_XCD) + cg / NUFFTCT_NUM_XCD;
  const int col0 = cg * NL;
  cx<T>* base = grid + (int64_t)qo * outer_stride + col0;
  // squared distance of this block's nearest column from the ball's axis
  const double ko = outer_in_ball ? (double)(qo - K / 2) : 0.0;
  double kc_min = 0.0;
  if (col0 > K / 2) kc_min = (double)(col0 - K / 2);
  else if (col0 + NL - 1 < K / 2) kc_min = (double)(K / 2 - (col0 + NL - 1));
  const bool block_out = ball && ko * ko + kc_min * kc_min > r2;
  if (block_out) {
    // nothing of this block is ever needed; the adjoint still owes zeros to
    // the rows the next pass reads
    if (ball == 2) {
      for (int idx = tid; idx < NL * L; idx += NTS) {
        const int line = idx % NL, e = idx / NL;
        const int m = centred_of(e, K);
        if (!store_pruned || (m >= -h && m < h)) base[e * row_stride + line] = cx<T>{0, 0};
      }
    }
    return;
  }
  stage::tile<T, NL * L, NTS>(
      tid,
      [&](int idx) {
        const int line = idx % NL, e = idx / NL;
        cx<T> v = {0, 0};
        const int m = centred_of(e, K);
        bool ld = !load_pruned || (m >= -h && m < h);
        if (ball == 2) {
          const double kr = (double)(e - K / 2), kc = (double)(col0 + line - K / 2);
          ld = ld && kr * kr + ko * ko + kc * kc <= r2;
        }
        if (ld) v = base[e * row_stride + line];
        return v;
      },
      [&](int idx, cx<T> v) { buf[idx] = v; });  // column-major address e*NL + line
  __syncthreads();
  fft::run<T, L, NL, NTS, false, S>(buf, twp, tid);
  for (int idx = tid; idx < NL * L; idx += NTS) {
    const int line = idx % NL, e = idx / NL;
    const int m = centred_of(e, K);
    bool stv = !store_pruned || (m >= -h && m < h);
    if (ball == 1) {
      const double kr = (double)(e - K / 2), kc = (double)(col0 + line - K / 2);
      stv = stv && kr * kr + ko * ko + kc * kc <= r2;
    }
    if (stv) base[e * row_stride + line] = buf[idx];
  }
}

template <typename T, int L, int S>
__global__ __launch_bounds__(NTS) void k_fft_strided(cx<T>* __restrict__ grid,
                                                    const cx<T>* __restrict__ tw, int N,
                                                    int64_t row_stride, int64_t outer_stride,
                                                    int outer_pruned, int load_pruned,
                                                    int store_pruned, double r2, int ball,
                                                    int outer_in_ball) {
  fft_strided_body<T, L, S>(blockIdx.x, blockIdx.y, gridDim.x, grid, tw, N, row_stride,
                            outer_stride, outer_pruned, load_pruned, store_pruned, r2, ball,
                            outer_in_ball);
}

// ---------------------------------------------------------------------------
// adjoint pass x (inverse FFT along the contiguous axis + crop + deapodize)
template <typename T, int L>
__device__ __forceinline__ void ifft_crop_x_body(int64_t bx, const cx<T>* __restrict__ grid,
                                                 cx<T>* __restrict__ vol,
                                                 const double* __restrict__ s,
                                                 const cx<T>* __restrict__ tw, int N) {
  constexpr int NL = nl_line<T, L>();
  constexpr int K = L;
  __shared__ cx<T> buf[fft::tile_elems<true, L, NL>()];
  __shared__ cx<T> twl[L];
  for (int i = threadIdx.x; i < L; i += NT) twl[i] = tw[i];
  const cx<T>* twp = twl;
  const int tid = threadIdx.x;
  const int64_t nlines = (int64_t)N * N;
  const int64_t line0 = bx * NL;
  const int h = N / 2;
  stage::tile<T, NL * L, NT>(
      tid,
      [&](int idx) {
        const int line = idx / L, e = idx % L;
        const int64_t gl = line0 + line;
        cx<T> v = {0, 0};
        if (gl < nlines) {
          const int n0 = (int)gl / N, n1 = (int)gl % N;
          const int q0 = wrap_of(n0 - h, K), q1 = wrap_of(n1 - h, K);
          v = grid[(int64_t)q0 * grid_plane_of<T>(K) + (int64_t)q1 * K + e];
        }
        return v;
      },
      [&](int idx, cx<T> v) { buf[fft::addr<true, L, NL>(idx / L, idx % L)] = v; });
  __syncthreads();
  fft::run<T, L, NL, NT, true, +1>(buf, twp, tid);
  for (int idx = tid; idx < NL * N; idx += NT) {
    const int line = idx / N, n2 = idx % N;
    const int64_t gl = line0 + line;
    if (gl < nlines) {
      const int n0 = (int)gl / N, n1 = (int)gl % N;
      const int e = wrap_of(n2 - h, K);
      const cx<T> v = buf[fft::addr<true, L, NL>(line, e)];
      double f = s[n0] * s[n1] * s[n2];
      if ((n0 + n1 + n2 + 3 * h) & 1) f = -f;
      cx<T> o;
      o.x = (T)((double)v.x * f);
      o.y = (T)((double)v.y * f);
      vol[gl * N + n2] = o;
    }
  }
}

template <typename T, int L>
__global__ __launch_bounds__(NT) void k_ifft_crop_x(const cx<T>* __restrict__ grid,
                                                    cx<T>* __restrict__ vol,
                                                    const double* __restrict__ s,
                                                    const cx<T>* __restrict__ tw, int N) {
  ifft_crop_x_body<T, L>(blockIdx.x, grid, vol, s, tw, N);
}

// ---------------------------------------------------------------------------
// radial stage (eq 2.17-2.18): per line of L = N_r samples
//   forward: D_j = (1/L) sum_c f_c G_c exp(+i r_c rho_j)
//          = (-1)^j (-1)^(L/2) / L * IDFT[(-1)^c f_c G_c]_j
//   adjoint: G~_c = conj(f_c) (-1)^c (-1)^(L/2) / L * DFT[(-1)^j d_j]_c
template <typename T, int L, bool ADJ>
__device__ __forceinline__ void radial_body(int64_t bx, const cx<T>* __restrict__ in,
                                            cx<T>* __restrict__ out,
                                            const cx<T>* __restrict__ tw, int64_t nlines,
                                            int deriv, double dr,
                                            const double* __restrict__ line_w,
                                            double w_scale) {
  constexpr int NL = nl_line<T, L>();
  __shared__ cx<T> buf[fft::tile_elems<true, L, NL>()];
  __shared__ cx<T> twl[L];
  for (int i = threadIdx.x; i < L; i += NT) twl[i] = tw[i];
  const cx<T>* twp = twl;
  const int tid = threadIdx.x;
  const int64_t line0 = bx * NL;
  const T post = (T)(((L / 2) & 1 ? -1.0 : 1.0) / (double)L);
  stage::tile<T, NL * L, NT>(
      tid,
      [&](int idx) {
        const int line = idx / L, e = idx % L;
        const int64_t gl = line0 + line;
        cx<T> v = {0, 0};
        if (gl < nlines) {
          v = in[gl * L + e];
          if (!ADJ && deriv) {  // multiply by f_c = i r_c, f_0 = 0
            const T r = e == 0 ? (T)0 : (T)((double)(e - L / 2) * dr);
            v = cx<T>{-r * v.y, r * v.x};
          }
          if (e & 1) v = cx<T>{-v.x, -v.y};
        }
        return v;
      },
      [&](int idx, cx<T> v) { buf[fft::addr<true, L, NL>(idx / L, idx % L)] = v; });
  __syncthreads();
  fft::run<T, L, NL, NT, true, ADJ ? -1 : +1>(buf, twp, tid);
  for (int idx = tid; idx < NL * L; idx += NT) {
    const int line = idx / L, e = idx % L;
    const int64_t gl = line0 + line;
    if (gl < nlines) {
      cx<T> v = buf[fft::addr<true, L, NL>(line, e)];
      T sc = (e & 1) ? -post : post;
      // adjoint with per-line weights (the direct reconstruction): the line's
      // weight times the reconstruction constant, rounded once
      if (ADJ && line_w) sc *= (T)(line_w[gl] * w_scale);
      v = cx<T>{v.x * sc, v.y * sc};
      if (ADJ && deriv) {  // multiply by conj(f_c) = -i r_c, f_0 = 0
        const T r = e == 0 ? (T)0 : (T)((double)(e - L / 2) * dr);
        v = cx<T>{r * v.y, -r * v.x};
      }
      out[gl * L + e] = v;
    }
  }
}

template <typename T, int L, bool ADJ>
__global__ __launch_bounds__(NT) void k_radial(const cx<T>* __restrict__ in,
                                               cx<T>* __restrict__ out,
                                               const cx<T>* __restrict__ tw, int64_t nlines,
                                               int deriv, double dr,
                                               const double* __restrict__ line_w,
                                               double w_scale) {
  radial_body<T, L, ADJ>(blockIdx.x, in, out, tw, nlines, deriv, dr, line_w, w_scale);
}

#define KFFT_SIZES(X) \
  X(16) X(32) X(48) X(64) X(80) X(96) X(128) X(160) X(192) X(256) X(320) X(384) X(512) X(640) X(768) X(1024)

template <typename T>
hipError_t pad_fft(const nufftct_plan& p, const void* vol, void* grid, hipStream_t st,
                   bool prune) {
  const int N = (int)p.N, K = (int)p.K;
  const double r2 = prune ? p.ball_r2 : 1e300;
  const int ball = prune && r2 < 1e299 ? 1 : 0;
  const cx<T>* tw = (const cx<T>*)p.d_tw_K;
  cx<T>* g = (cx<T>*)grid;
  switch (K) {
#define CASE(LL)                                                                              \
  case LL: {                                                                                  \
    constexpr int NLx = nl_line<T, LL>();                                                     \
    constexpr int NLc = nl_col<T, LL>();                                                      \
    const int64_t nlines = (int64_t)N * N;                                                    \
    hipLaunchKernelGGL((k_pad_fft_x<T, LL>), dim3((unsigned)((nlines + NLx - 1) / NLx)),      \
                       dim3(NT), 0, st, (const cx<T>*)vol, g, p.d_s, tw, N);                  \
    hipLaunchKernelGGL((k_fft_strided<T, LL, -1>), dim3(LL / NLc, N), dim3(NTS), 0, st, g, tw, \
                       N, (int64_t)LL, grid_plane_of<T>(LL), 1, 1, 0, r2, ball, 0);          \
    hipLaunchKernelGGL((k_fft_strided<T, LL, -1>), dim3(LL / NLc, LL), dim3(NTS), 0, st, g,    \
                       tw, N, grid_plane_of<T>(LL), (int64_t)LL, 0, 1, 0, r2, ball, 1);      \
    return hipGetLastError();                                                                 \
  }
    KFFT_SIZES(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t ifft_crop(const nufftct_plan& p, void* grid, void* vol, hipStream_t st, bool prune) {
  const int N = (int)p.N, K = (int)p.K;
  const double r2 = prune ? p.ball_r2 : 1e300;
  const int ball = prune && r2 < 1e299 ? 2 : 0;
  const cx<T>* tw = (const cx<T>*)p.d_tw_K;
  cx<T>* g = (cx<T>*)grid;
  switch (K) {
#define CASE(LL)                                                                              \
  case LL: {                                                                                  \
    constexpr int NLx = nl_line<T, LL>();                                                     \
    constexpr int NLc = nl_col<T, LL>();                                                      \
    const int64_t nlines = (int64_t)N * N;                                                    \
    hipLaunchKernelGGL((k_fft_strided<T, LL, +1>), dim3(LL / NLc, LL), dim3(NTS), 0, st, g,    \
                       tw, N, grid_plane_of<T>(LL), (int64_t)LL, 0, 0, 1, r2, ball, 1);      \
    hipLaunchKernelGGL((k_fft_strided<T, LL, +1>), dim3(LL / NLc, N), dim3(NTS), 0, st, g, tw, \
                       N, (int64_t)LL, grid_plane_of<T>(LL), 1, 0, 1, r2, ball, 0);          \
    hipLaunchKernelGGL((k_ifft_crop_x<T, LL>), dim3((unsigned)((nlines + NLx - 1) / NLx)),    \
                       dim3(NT), 0, st, (const cx<T>*)g, (cx<T>*)vol, p.d_s, tw, N);          \
    return hipGetLastError();                                                                 \
  }
    KFFT_SIZES(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t radial(const nufftct_plan& p, const void* in, void* out, bool adj, bool deriv,
                  hipStream_t st, const double* line_w, double w_scale) {
  const int64_t nl = p.M / p.n_r;
  const cx<T>* tw = (const cx<T>*)p.d_tw_r;
  const double dr = (2.0 * M_PI) / (double)p.n_r;
  switch ((int)p.n_r) {
#define CASE(LL)                                                                               \
  case LL: {                                                                                   \
    constexpr int NLx = nl_line<T, LL>();                                                      \
    dim3 grd((unsigned)((nl + NLx - 1) / NLx));                                                \
    if (adj)                                                                                   \
      hipLaunchKernelGGL((k_radial<T, LL, true>), grd, dim3(NT), 0, st, (const cx<T>*)in,      \
                         (cx<T>*)out, tw, nl, (int)deriv, dr, line_w, w_scale);                \
    else                                                                                       \
      hipLaunchKernelGGL((k_radial<T, LL, false>), grd, dim3(NT), 0, st, (const cx<T>*)in,     \
                         (cx<T>*)out, tw, nl, (int)deriv, dr, nullptr, 1.0);                   \
    return hipGetLastError();                                                                  \
  }
    KFFT_SIZES(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace kfft

#define KFFT_INSTANTIATE(T)                                                                \
  template <>                                                                              \
  hipError_t launch_pad_fft<T>(const nufftct_plan& p, const void* vol, void* grid,         \
                               hipStream_t s, bool prune) {                                \
    return kfft::pad_fft<T>(p, vol, grid, s, prune);                                       \
  }                                                                                        \
  template <>                                                                              \
  hipError_t launch_ifft_crop<T>(const nufftct_plan& p, void* grid, void* vol,             \
                                 hipStream_t s, bool prune) {                              \
    return kfft::ifft_crop<T>(p, grid, vol, s, prune);                                     \
  }                                                                                        \
  template <>                                                                              \
  hipError_t launch_radial<T>(const nufftct_plan& p, const void* in, void* out, bool adj,  \
                              bool deriv, hipStream_t s, const double* line_w,             \
                              double w_scale) {                                            \
    return kfft::radial<T>(p, in, out, adj, deriv, s, line_w, w_scale);                    \
  }
