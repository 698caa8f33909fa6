// Umbrella derivative-Radon values -> cone-beam projections (the Grangeat
// step in reverse, Section 2.2.2), as LDS-tiled kernels for gfx950.
//
// Per projection k, from its n_alpha x n umbrella samples U[k][i][j]:
//   k_gr_radial: per detector-line angle i, the line j = 0..n-1 times the
//     de-postweight and ds' (one FP64 table), zero-padded to 2n, FFT, times the
//     inversion filter -i h_m; the k = 0 bin takes the Euler-Maclaurin weight
//     times P(alpha_i, 0) = -sum s'_j q_j (a fixed-order wave reduction).
//     A workgroup takes NK projections of one angle, so its stores of the
//     spectra c[(i 2n + m) n_proj + k] are runs of NK consecutive k.
//   k_gr_rows: the KB spreading of the n_alpha x 2n polar points onto the
//     K x K grid (K = 2n) in gather form: the points and weights that reach
//     each cell are the same for every projection (a CSR list made on the
//     host), so a workgroup gathers one grid row for NK projections (NK lanes
//     per cell, reading each list entry's NK spectra as one 128-byte
//     segment), then runs the inverse FFT along the row in LDS and keeps the
//     n columns of the crop.
//   k_gr_cols: the inverse FFT along the columns (NLC adjacent columns per
//     tile), the crop to n rows, and the deapodization and de-preweighting
//     s(m_u) s(m_v) sqrt(R^2 + u'^2 + v'^2) / R in FP64, rounded once.
// No atomics: every output is a fixed-order sum.
#pragma once

#include "cx.h"
#include "fft_lds.h"
#include "grangeat.h"
#include "stage.h"

namespace kgr {

constexpr int NT = 256;       // radial and row workgroups
constexpr int NT_COL = 512;   // column workgroups

template <typename T>
constexpr int nk() {  // projections per radial / row workgroup
  return sizeof(T) == 4 ? 8 : 4;
}

template <typename T, int K>
constexpr int nk_rows() {  // projections per row workgroup: 128-byte spectra segments
  if constexpr (sizeof(T) == 4) return K <= 512 ? 16 : 8;
  return K <= 512 ? 8 : 4;
}

template <typename T, int K>
constexpr int nlc() {  // adjacent columns per column tile
  if constexpr (sizeof(T) == 4) return K <= 512 ? 16 : 8;
  return K <= 512 ? 8 : 4;
}

template <typename T, int NN>
__global__ __launch_bounds__(NT) void k_gr_radial(const cx<T>* __restrict__ U,
                                                  cx<T>* __restrict__ c,
                                                  const double* __restrict__ pw,
                                                  const double* __restrict__ dcw,
                                                  const double* __restrict__ h,
                                                  const cx<T>* __restrict__ tw, int n_proj,
                                                  int n_alpha) {
  constexpr int L = 2 * NN, NK = nk<T>();
  __shared__ cx<T> buf[fft::tile_elems<true, L, NK>()];
  __shared__ cx<T> twl[L];
  __shared__ cx<T> dcs[NK];
  const int tid = threadIdx.x;
  for (int q = tid; q < L; q += NT) twl[q] = tw[q];
  const int i = blockIdx.y;
  const int k0 = blockIdx.x * NK;
  // line `line` holds q_j (-1)^jc at (jc mod 2n), jc = j - n/2, zeros elsewhere
  stage::tile<T, NK * L, NT>(
      tid,
      [&](int idx) {
        const int line = idx / L, e = idx % L;
        const int jc = e < L / 2 ? e : e - L;
        const int k = k0 + line;
        cx<T> v = {0, 0};
        if (k < n_proj && jc >= -NN / 2 && jc < NN / 2) {
          const int j = jc + NN / 2;
          const cx<T> u = U[((int64_t)k * n_alpha + i) * NN + j];
          const double f = (jc & 1) ? -pw[j] : pw[j];
          v = cx<T>{(T)((double)u.x * f), (T)((double)u.y * f)};
        }
        return v;
      },
      [&](int idx, cx<T> v) { buf[fft::addr<true, L, NK>(idx / L, idx % L)] = v; });
  __syncthreads();
  // the k = 0 bin: one wave per line, lanes in a fixed order, then a fixed
  // shuffle tree (dcw carries the (-1)^jc of the layout)
  {
    const int lane = tid & 63, wave = tid >> 6;
    for (int line = wave; line < NK; line += NT / 64) {
      double sx = 0.0, sy = 0.0;
      for (int j = lane; j < NN; j += 64) {
        const int jc = j - NN / 2;
        const cx<T> v = buf[fft::addr<true, L, NK>(line, jc < 0 ? jc + L : jc)];
        sx += dcw[j] * (double)v.x;
        sy += dcw[j] * (double)v.y;
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        sx += __shfl_down(sx, o, 64);
        sy += __shfl_down(sy, o, 64);
      }
      if (lane == 0) dcs[line] = cx<T>{(T)sx, (T)sy};
    }
  }
  __syncthreads();
  fft::run<T, L, NK, NT, true, -1>(buf, twl, tid);
  for (int idx = tid; idx < NK * L; idx += NT) {
    const int m = idx / NK, line = idx % NK;
    const int k = k0 + line;
    if (k < n_proj) {
      cx<T> v;
      if (m == NN) {
        v = dcs[line];
      } else {
        const cx<T> P = buf[fft::addr<true, L, NK>(line, m)];
        const double hm = h[m];
        v = cx<T>{(T)(hm * (double)P.y), (T)(-hm * (double)P.x)};  // -i h P
      }
      c[((int64_t)i * L + m) * n_proj + k] = v;
    }
  }
}

template <typename T, int NN>
__global__ __launch_bounds__(NT) void k_gr_rows(const cx<T>* __restrict__ c,
                                                cx<T>* __restrict__ rows,
                                                const int32_t* __restrict__ off,
                                                const int32_t* __restrict__ pt,
                                                const T* __restrict__ w,
                                                const cx<T>* __restrict__ tw, int n_proj,
                                                int n_groups) {
  constexpr int K = 2 * NN, NK = nk_rows<T, K>();
  constexpr int CPP = NT / NK;  // cells per pass: NK lanes (one per projection) per cell
  __shared__ cx<T> buf[fft::tile_elems<true, K, NK>()];
  __shared__ cx<T> twl[K];
  const int tid = threadIdx.x;
  for (int q = tid; q < K; q += NT) twl[q] = tw[q];
  // workgroups go round-robin over the XCDs: give each XCD a contiguous run of
  // rows of one projection group, so the rows sharing polar points (every
  // point reaches J rows) meet in one L2
  int b = blockIdx.x;
  const int nb = gridDim.x;
  if ((nb & (NUFFTCT_NUM_XCD - 1)) == 0) b = (b % NUFFTCT_NUM_XCD) * (nb / NUFFTCT_NUM_XCD) + b / NUFFTCT_NUM_XCD;
  const int grp = b / K, kv = b % K;
  if (grp >= n_groups) return;
  const int k0 = grp * NK;
  const int nk_here = n_proj - k0 < NK ? n_proj - k0 : NK;
  // lane q of a cell's NK lanes gathers projection k0 + q: the lanes read the
  // NK consecutive spectra of a list entry as one segment
  const int q = tid % NK;
  const bool live = q < nk_here;
  for (int cu0 = 0; cu0 < K; cu0 += CPP) {
    const int ku = cu0 + tid / NK;
    cx<T> acc = {0, 0};
    if (ku < K) {
      const int cell = kv * K + ku;
      const int e1 = off[cell + 1];
      const cx<T>* src = c + k0 + q;
      int e = off[cell];
      // UF entries at a time: their list reads, then their spectra reads, are
      // in flight together (one at a time the loop waits on each pair of
      // dependent loads); the sums keep the list order
      constexpr int UF = 4;
      for (; e + UF <= e1; e += UF) {
        int p[UF];
        T we[UF];
#pragma unroll
        for (int r = 0; r < UF; ++r) {
          p[r] = pt[e + r];
          we[r] = w[e + r];
        }
        cx<T> v[UF];
#pragma unroll
        for (int r = 0; r < UF; ++r) v[r] = live ? src[(int64_t)p[r] * n_proj] : cx<T>{0, 0};
#pragma unroll
        for (int r = 0; r < UF; ++r) {
          acc.x += we[r] * v[r].x;
          acc.y += we[r] * v[r].y;
        }
      }
      for (; e < e1; ++e) {
        const T we = w[e];
        const cx<T> v = live ? src[(int64_t)pt[e] * n_proj] : cx<T>{0, 0};
        acc.x += we * v.x;
        acc.y += we * v.y;
      }
      buf[fft::addr<true, K, NK>(q, ku)] = acc;
    }
  }
  __syncthreads();
  fft::run<T, K, NK, NT, true, +1>(buf, twl, tid);
  for (int idx = tid; idx < NK * NN; idx += NT) {
    const int qq = idx / NN, a = idx % NN;
    if (qq < nk_here) {
      const int col = a - NN / 2 < 0 ? a - NN / 2 + K : a - NN / 2;
      rows[((int64_t)(k0 + qq) * K + kv) * NN + a] = buf[fft::addr<true, K, NK>(qq, col)];
    }
  }
}

template <typename T, int NN>
__global__ __launch_bounds__(NT_COL) void k_gr_cols(const cx<T>* __restrict__ rows,
                                                    cx<T>* __restrict__ X,
                                                    const double* __restrict__ s,
                                                    const double* __restrict__ sv,
                                                    const cx<T>* __restrict__ tw, double R) {
  constexpr int K = 2 * NN, NL = nlc<T, K>();
  __shared__ cx<T> buf[NL * K];
  __shared__ cx<T> twl[K];
  const int tid = threadIdx.x;
  for (int q = tid; q < K; q += NT_COL) twl[q] = tw[q];
  const int a0 = blockIdx.x * NL;
  const int k = blockIdx.y;
  const cx<T>* base = rows + (int64_t)k * K * NN + a0;
  stage::tile<T, NL * K, NT_COL>(
      tid,
      [&](int idx) {
        const int line = idx % NL, e = idx / NL;
        return a0 + line < NN ? base[(int64_t)e * NN + line] : cx<T>{0, 0};
      },
      [&](int idx, cx<T> v) { buf[idx] = v; });  // column-major: e * NL + line
  __syncthreads();
  fft::run<T, K, NL, NT_COL, false, +1>(buf, twl, tid);
  const double R2 = R * R, invR = 1.0 / R;
  for (int idx = tid; idx < NL * NN; idx += NT_COL) {
    const int line = idx % NL, b = idx / NL;
    const int a = a0 + line;
    if (a < NN) {
      const int row = b - NN / 2 < 0 ? b - NN / 2 + K : b - NN / 2;
      const cx<T> v = buf[row * NL + line];
      const double f = s[a] * s[b] * sqrt(R2 + sv[a] * sv[a] + sv[b] * sv[b]) * invR;
      X[((int64_t)k * NN + b) * NN + a] = cx<T>{(T)((double)v.x * f), (T)((double)v.y * f)};
    }
  }
}

// Compiled detector sizes n (K = 2n).
#define KGR_SIZES(X) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(160) X(192) X(256) X(320) X(384) X(512)

template <typename T>
hipError_t radial(const nufftct_grangeat& g, const void* umb, void* c, hipStream_t st) {
  constexpr int NK = nk<T>();
  const dim3 grd((unsigned)((g.n_proj + NK - 1) / NK), (unsigned)g.n_alpha);
  switch (g.n) {
#define CASE(NN)                                                                              \
  case NN:                                                                                    \
    hipLaunchKernelGGL((k_gr_radial<T, NN>), grd, dim3(NT), 0, st, (const cx<T>*)umb,         \
                       (cx<T>*)c, g.d_pw, g.d_dcw, g.d_h, (const cx<T>*)g.d_tw, g.n_proj,     \
                       g.n_alpha);                                                            \
    return hipGetLastError();
    KGR_SIZES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t backproject(const nufftct_grangeat& g, const void* c, void* x, hipStream_t st) {
  switch (g.n) {
#define CASE(NN)                                                                                \
  case NN: {                                                                                    \
    constexpr int NL = nlc<T, 2 * NN>();                                                        \
    constexpr int NKR = nk_rows<T, 2 * NN>();                                                   \
    const int ngr = (g.n_proj + NKR - 1) / NKR;                                                 \
    hipLaunchKernelGGL((k_gr_rows<T, NN>), dim3((unsigned)(ngr * 2 * NN)), dim3(NT), 0, st,     \
                       (const cx<T>*)c, (cx<T>*)g.d_rows, g.d_off, g.d_pt, (const T*)g.d_w,     \
                       (const cx<T>*)g.d_tw, g.n_proj, ngr);                                    \
    hipError_t e = hipGetLastError();                                                           \
    if (e != hipSuccess) return e;                                                              \
    hipLaunchKernelGGL((k_gr_cols<T, NN>), dim3((unsigned)((NN + NL - 1) / NL), g.n_proj),      \
                       dim3(NT_COL), 0, st, (const cx<T>*)g.d_rows, (cx<T>*)x, g.d_s, g.d_sv,   \
                       (const cx<T>*)g.d_tw, g.R);                                              \
    return hipGetLastError();                                                                   \
  }
    KGR_SIZES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace kgr

#define KGR_INSTANTIATE(T)                                                                   \
  template <>                                                                                \
  hipError_t launch_grangeat_radial<T>(const nufftct_grangeat& g, const void* umb, void* c, \
                                       hipStream_t s) {                                      \
    return kgr::radial<T>(g, umb, c, s);                                                     \
  }                                                                                          \
  template <>                                                                                \
  hipError_t launch_grangeat_backproject<T>(const nufftct_grangeat& g, const void* c,       \
                                            void* x, hipStream_t s) {                        \
    return kgr::backproject<T>(g, c, x, s);                                                  \
  }
