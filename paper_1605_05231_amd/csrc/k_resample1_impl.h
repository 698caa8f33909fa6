// Radial -> umbrella resampling, method 1 (Section 2.1.3, eq 2.11):
// x~ = T_sparse F P F^-1 x in the (phi, theta, rho) index space of the radial
// grid, as LDS-tiled kernels for gfx950.
//
// The operator F P F^-1 is separable, so it runs as one pass per axis, each
// pass taking every line of that axis through
//   inverse DFT of length N (exp(+i..)), then the scaling s(m)/N at the
//   centred frequency m in [-N/2, N/2) placed at (m mod K), zeros elsewhere
//   (K = 2N), then the forward FFT of length K,
// all inside LDS: each line is read once and written once.  The passes run in
// place on the one K_0 x K_1 x K_2 grid ([phi][theta][rho], rho fastest, cell
// kappa at kappa mod K): the rho pass reads the radial samples and writes its
// lines at their final rows; the theta and phi passes read the N populated
// rows of their columns and write all K rows of the same columns, and no two
// workgroups share a column, so nothing is read after another workgroup wrote
// it.  Traffic: the input once, then 2, 4 and 8 times its size written and
// 2 and 4 times read back: 21 times the radial data per resampling.
//
// T_sparse: one thread per umbrella sample gathers the J^3 Kaiser-Bessel taps
// around grid coordinate 2 t (t the sample's index coordinates), wrapped on
// every axis; weights from the per-tap polynomial fits of the projector's NUFFT.
#pragma once

#include "cx.h"
#include "fft_lds.h"
#include "stage.h"
#include "umbrella.h"

namespace krs1 {

constexpr int NT_ROW = 512;   // threads of a rho-pass workgroup
constexpr int NT_COL = 1024;  // threads of a theta / phi pass workgroup
constexpr int NT_GATHER = 256;

template <typename T, int N>
constexpr int nl_row() {  // lines per rho-pass tile
  constexpr int target = sizeof(T) == 4 ? 4096 : 2048;
  return target / (2 * N) > 0 ? target / (2 * N) : 1;
}

template <typename T, int N>
constexpr int nl_col() {  // adjacent columns per theta / phi pass tile
  if constexpr (sizeof(T) == 4) return 2 * N <= 512 ? 16 : 8;
  return 2 * N <= 512 ? 8 : 4;
}

// After the inverse DFT of length N sits in the tile, move it to the K-length
// layout of the same tile (fft::addr, line- or column-major): frequency e
// (centred m = e or e - N) goes to m mod K scaled by sc[m + N/2] (FP64, rounded
// once), and the N cells between the two halves are zeroed.  The values pass
// through registers, so the two layouts may share the buffer.  Threads walk
// the tile in its own storage order (conflict-free LDS access).
template <typename T, int N, int NL, int NTH, bool LM>
__device__ __forceinline__ void pad_scale(cx<T>* buf, const double* __restrict__ sc, int tid) {
  constexpr int K = 2 * N;
  constexpr int E = NL * N;
  constexpr int PER = (E + NTH - 1) / NTH;
  cx<T> r[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int idx = tid + i * NTH;
    if (E % NTH == 0 || idx < E) {
      const int line = LM ? idx / N : idx % NL, e = LM ? idx % N : idx / NL;
      r[i] = buf[fft::addr<LM, N, NL>(line, e)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int idx = tid + i * NTH;
    if (E % NTH == 0 || idx < E) {
      const int line = LM ? idx / N : idx % NL, e = LM ? idx % N : idx / NL;
      const bool lo = e < N / 2;
      const double f = sc[lo ? e + N / 2 : e - N / 2];  // index m + N/2
      const cx<T> v = {(T)((double)r[i].x * f), (T)((double)r[i].y * f)};
      buf[fft::addr<LM, K, NL>(line, lo ? e : e + N)] = v;
      buf[fft::addr<LM, K, NL>(line, N / 2 + e)] = cx<T>{0, 0};
    }
  }
  __syncthreads();
}

// rho pass: line l = (a, b) of the radial samples (contiguous, length N) ->
// grid row (a K_1 + b), all K = 2N cells.
template <typename T, int N>
__global__ __launch_bounds__(NT_ROW) void k_rs1_row(const cx<T>* __restrict__ in,
                                                    cx<T>* __restrict__ grid,
                                                    const double* __restrict__ sc,
                                                    const cx<T>* __restrict__ tw_n,
                                                    const cx<T>* __restrict__ tw_k,
                                                    int64_t nlines, int n_mid, int k_mid) {
  constexpr int K = 2 * N, NL = nl_row<T, N>();
  __shared__ cx<T> buf[fft::tile_elems<true, K, NL>()];
  __shared__ cx<T> twn[N];
  __shared__ cx<T> twk[K];
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += NT_ROW) twn[i] = tw_n[i];
  for (int i = tid; i < K; i += NT_ROW) twk[i] = tw_k[i];
  const int64_t line0 = (int64_t)blockIdx.x * NL;
  stage::tile<T, NL * N, NT_ROW>(
      tid,
      [&](int idx) {
        const int64_t gl = line0 + idx / N;
        return gl < nlines ? in[gl * N + idx % N] : cx<T>{0, 0};
      },
      [&](int idx, cx<T> v) { buf[fft::addr<true, N, NL>(idx / N, idx % N)] = v; });
  __syncthreads();
  fft::run<T, N, NL, NT_ROW, true, +1>(buf, twn, tid);
  pad_scale<T, N, NL, NT_ROW, true>(buf, sc, tid);
  fft::run<T, K, NL, NT_ROW, true, -1>(buf, twk, tid);
  for (int idx = tid; idx < NL * K; idx += NT_ROW) {
    const int line = idx / K, e = idx % K;
    const int64_t gl = line0 + line;
    if (gl < nlines) {
      const int64_t row = (gl / n_mid) * k_mid + gl % n_mid;
      grid[row * K + e] = buf[fft::addr<true, K, NL>(line, e)];
    }
  }
}

// theta / phi pass, in place: NL adjacent columns of one outer slab; rows
// 0..N-1 hold the input, rows 0..K-1 receive the output.
template <typename T, int N>
__global__ __launch_bounds__(NT_COL) void k_rs1_col(cx<T>* __restrict__ grid,
                                                    const double* __restrict__ sc,
                                                    const cx<T>* __restrict__ tw_n,
                                                    const cx<T>* __restrict__ tw_k,
                                                    int64_t row_stride, int64_t outer_stride,
                                                    int64_t ncols) {
  constexpr int K = 2 * N, NL = nl_col<T, N>();
  __shared__ cx<T> buf[NL * K];
  __shared__ cx<T> twn[N];
  __shared__ cx<T> twk[K];
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += NT_COL) twn[i] = tw_n[i];
  for (int i = tid; i < K; i += NT_COL) twk[i] = tw_k[i];
  // workgroups go round-robin over the XCDs: give each XCD a contiguous run of
  // column groups, so that the groups sharing a row's cache lines meet in one L2
  int64_t cg = blockIdx.x;
  if ((gridDim.x & (NUFFTCT_NUM_XCD - 1)) == 0)
    cg = (cg % NUFFTCT_NUM_XCD) * (gridDim.x / NUFFTCT_NUM_XCD) + cg / NUFFTCT_NUM_XCD;
  const int64_t col0 = cg * NL;
  cx<T>* base = grid + (int64_t)blockIdx.y * outer_stride + col0;
  const int nc = ncols - col0 < NL ? (int)(ncols - col0) : NL;
  stage::tile<T, NL * N, NT_COL>(
      tid,
      [&](int idx) {
        const int line = idx % NL, e = idx / NL;
        return line < nc ? base[e * row_stride + line] : cx<T>{0, 0};
      },
      [&](int idx, cx<T> v) { buf[idx] = v; });  // column-major: e * NL + line
  __syncthreads();
  fft::run<T, N, NL, NT_COL, false, +1>(buf, twn, tid);
  pad_scale<T, N, NL, NT_COL, false>(buf, sc, tid);
  fft::run<T, K, NL, NT_COL, false, -1>(buf, twk, tid);
  for (int idx = tid; idx < NL * K; idx += NT_COL) {
    const int line = idx % NL, e = idx / NL;
    if (line < nc) base[e * row_stride + line] = buf[idx];
  }
}

// Per-tap KB weights at offset frac (polynomials in z = 2 frac - 1).
template <typename T, int J, int DEG>
__device__ __forceinline__ void kb_weights(const WeightPoly<T, DEG>& P, double frac, T (&w)[J]) {
  const T z = (T)(2.0 * frac - 1.0);
#pragma unroll
  for (int a = 0; a < J; ++a) {
    T acc = P.re[a][DEG];
#pragma unroll
    for (int d = DEG - 1; d >= 0; --d) acc = acc * z + P.re[a][d];
    w[a] = acc;
  }
}

// First tap (already wrapped into [0, K)) and weights around grid coordinate tg.
template <typename T, int J, int DEG>
__device__ __forceinline__ int axis_taps(double tg, int K, const WeightPoly<T, DEG>& P,
                                         T (&w)[J]) {
  const double s = tg - 0.5 * (double)J;
  const double f = floor(s);
  kb_weights<T, J, DEG>(P, s - f, w);
  int k = (int)fmod(f + 1.0, (double)K);
  if (k < 0) k += K;
  return k;
}

template <typename T, int J, int DEG>
__global__ __launch_bounds__(NT_GATHER) void k_rs1_gather(const cx<T>* __restrict__ grid,
                                                          cx<T>* __restrict__ out,
                                                          UmbrellaGeom g, int K0, int K1, int K2,
                                                          WeightPoly<T, DEG> P) {
  const int64_t total = (int64_t)g.n_proj * g.n_alpha * g.n_t;
  const int64_t p = (int64_t)blockIdx.x * NT_GATHER + threadIdx.x;
  if (p >= total) return;
  double tp, tt, tr;
  umbrella_coords(g, p, tp, tt, tr);
  // grid coordinate t K/N = 2 t on every axis (exact)
  T w0[J], w1[J], w2[J];
  const int f0 = axis_taps<T, J, DEG>(2.0 * tp, K0, P, w0);
  const int f1 = axis_taps<T, J, DEG>(2.0 * tt, K1, P, w1);
  const int f2 = axis_taps<T, J, DEG>(2.0 * tr, K2, P, w2);
  int i2[J];
#pragma unroll
  for (int c = 0; c < J; ++c) i2[c] = f2 + c < K2 ? f2 + c : f2 + c - K2;
  cx<T> acc = {0, 0};
#pragma unroll
  for (int a = 0; a < J; ++a) {
    const int i0 = f0 + a < K0 ? f0 + a : f0 + a - K0;
    cx<T> acc_a = {0, 0};
#pragma unroll
    for (int b = 0; b < J; ++b) {
      const int i1 = f1 + b < K1 ? f1 + b : f1 + b - K1;
      const cx<T>* row = grid + ((int64_t)i0 * K1 + i1) * K2;
      cx<T> acc_b = {0, 0};
#pragma unroll
      for (int c = 0; c < J; ++c) {
        const cx<T> v = row[i2[c]];
        acc_b.x += w2[c] * v.x;
        acc_b.y += w2[c] * v.y;
      }
      acc_a.x += w1[b] * acc_b.x;
      acc_a.y += w1[b] * acc_b.y;
    }
    acc.x += w0[a] * acc_a.x;
    acc.y += w0[a] * acc_a.y;
  }
  out[p] = acc;
}

// Compiled axis lengths N (K = 2N): even, with 2N = 2^a 3^b 5^c.
#define KRS1_SIZES(X)                                                                          \
  X(8) X(12) X(16) X(20) X(24) X(30) X(32) X(36) X(40) X(48) X(60) X(64) X(72) X(80) X(90)     \
  X(96) X(120) X(128) X(144) X(160) X(180) X(192) X(240) X(256) X(288) X(320) X(360) X(384)    \
  X(480) X(512)

template <typename T, int N>
hipError_t row_pass(const nufftct_umbrella& u, const void* in, void* grid, hipStream_t st) {
  constexpr int NL = nl_row<T, N>();
  const int64_t nlines = (int64_t)u.g.n_phi * u.g.n_theta;
  hipLaunchKernelGGL((k_rs1_row<T, N>), dim3((unsigned)((nlines + NL - 1) / NL)), dim3(NT_ROW),
                     0, st, (const cx<T>*)in, (cx<T>*)grid, u.d_sc[2], (const cx<T>*)u.d_tw_n[2],
                     (const cx<T>*)u.d_tw_k[2], nlines, u.g.n_theta, (int)u.K[1]);
  return hipGetLastError();
}

// axis 1 (theta): outer slabs a < N_0, columns K_2, rows of stride K_2;
// axis 0 (phi): one slab, columns K_1 K_2, rows of stride K_1 K_2
template <typename T, int N>
hipError_t col_pass(const nufftct_umbrella& u, int axis, void* grid, hipStream_t st) {
  constexpr int NL = nl_col<T, N>();
  const int64_t row_stride = axis == 1 ? u.K[2] : u.K[1] * u.K[2];
  const int64_t outer_stride = axis == 1 ? u.K[1] * u.K[2] : 0;
  const int64_t ncols = row_stride;
  const unsigned nouter = axis == 1 ? (unsigned)u.g.n_phi : 1u;
  const int64_t ngroups = (ncols + NL - 1) / NL;
  hipLaunchKernelGGL((k_rs1_col<T, N>), dim3((unsigned)ngroups, nouter), dim3(NT_COL), 0, st,
                     (cx<T>*)grid, u.d_sc[axis], (const cx<T>*)u.d_tw_n[axis],
                     (const cx<T>*)u.d_tw_k[axis], row_stride, outer_stride, ncols);
  return hipGetLastError();
}

template <typename T>
hipError_t grid_passes(const nufftct_umbrella& u, const void* in, void* grid, hipStream_t st) {
  hipError_t e = hipErrorInvalidValue;
  switch (u.g.n_r) {
#define CASE(NN) \
  case NN: e = row_pass<T, NN>(u, in, grid, st); break;
    KRS1_SIZES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  for (int axis = 1; axis >= 0; --axis) {
    const int n = axis == 1 ? u.g.n_theta : u.g.n_phi;
    switch (n) {
#define CASE(NN) \
  case NN: e = col_pass<T, NN>(u, axis, grid, st); break;
      KRS1_SIZES(CASE)
#undef CASE
      default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T, int DEG>
struct PolyOf;
template <>
struct PolyOf<float, NUFFTCT_DEG_F32> {
  static const WeightPoly<float, NUFFTCT_DEG_F32>& get(const nufftct_umbrella& u) { return u.wp32; }
};
template <>
struct PolyOf<double, NUFFTCT_DEG_F64> {
  static const WeightPoly<double, NUFFTCT_DEG_F64>& get(const nufftct_umbrella& u) { return u.wp64; }
};

template <typename T, int J>
hipError_t gather_j(const nufftct_umbrella& u, const void* grid, void* out, hipStream_t st) {
  constexpr int DEG = sizeof(T) == 4 ? NUFFTCT_DEG_F32 : NUFFTCT_DEG_F64;
  const int64_t total = (int64_t)u.g.n_proj * u.g.n_alpha * u.g.n_t;
  hipLaunchKernelGGL((k_rs1_gather<T, J, DEG>), dim3((unsigned)((total + NT_GATHER - 1) / NT_GATHER)),
                     dim3(NT_GATHER), 0, st, (const cx<T>*)grid, (cx<T>*)out, u.g, (int)u.K[0],
                     (int)u.K[1], (int)u.K[2], PolyOf<T, DEG>::get(u));
  return hipGetLastError();
}

template <typename T>
hipError_t gather(const nufftct_umbrella& u, const void* grid, void* out, hipStream_t st) {
  switch (u.J) {
    case 2: return gather_j<T, 2>(u, grid, out, st);
    case 3: return gather_j<T, 3>(u, grid, out, st);
    case 4: return gather_j<T, 4>(u, grid, out, st);
    case 5: return gather_j<T, 5>(u, grid, out, st);
    case 6: return gather_j<T, 6>(u, grid, out, st);
    case 7: return gather_j<T, 7>(u, grid, out, st);
    case 8: return gather_j<T, 8>(u, grid, out, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace krs1

#define KRS1_INSTANTIATE(T)                                                                  \
  template <>                                                                                \
  hipError_t launch_resample1_grid<T>(const nufftct_umbrella& u, const void* in, void* grid, \
                                      hipStream_t s) {                                       \
    return krs1::grid_passes<T>(u, in, grid, s);                                             \
  }                                                                                          \
  template <>                                                                                \
  hipError_t launch_resample1_gather<T>(const nufftct_umbrella& u, const void* grid,         \
                                        void* out, hipStream_t s) {                          \
    return krs1::gather<T>(u, grid, out, s);                                                 \
  }
