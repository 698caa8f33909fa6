// One launch per stage across the volumes of an uneven batch (gfx950).
//
// The FFT and radial stages are compiled per transform length, so they run
// once per size class (volumes of equal N, K and N_r): blockIdx.z picks the
// volume, and the per-call buffer pointers (and each volume's ball radius
// or line count) travel in the kernel arguments.  The point stages
// (interpolation, spreading and its general-task pass, merge) do not depend
// on K at compile time, so one launch covers every volume of a tile size: the
// volumes' block ranges are laid end to end (each a multiple of 8 long, so a
// block's XCD is the one its plan would give it), a block finds its volume
// in a table of range starts and reads the volume's plan data from a device
// array.  Each block then runs exactly the body the one-plan kernel runs.
#pragma once

#include "k_fft_impl.h"
#include "k_grid_impl.h"

#include "batch_desc.h"

namespace kbatch {

// volume of global block b: the last v with start.s[v] <= b (start[nv] = total)
__device__ __forceinline__ int find_vol(const BatchStarts& start, int nv, int64_t b) {
  int lo = 0, hi = nv - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start.s[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <typename T, int L>
__global__ __launch_bounds__(kfft::NT) void k_pad_fft_x_b(BatchArgs a, const double* __restrict__ s,
                                                          const cx<T>* __restrict__ tw, int N) {
  const int v = blockIdx.z;
  kfft::pad_fft_x_body<T, L>(blockIdx.x, (const cx<T>*)a.in[v], (cx<T>*)a.out[v], s, tw, N);
}

template <typename T, int L, int S>
__global__ __launch_bounds__(kfft::NTS) void k_fft_strided_b(BatchArgs a,
                                                             const cx<T>* __restrict__ tw, int N,
                                                             int64_t row_stride,
                                                             int64_t outer_stride,
                                                             int outer_pruned, int load_pruned,
                                                             int store_pruned, int ball,
                                                             int outer_in_ball) {
  // the grids: the outputs of the forward passes, the inputs of the inverse ones
  const int v = blockIdx.z;
  cx<T>* grid = S < 0 ? (cx<T>*)a.out[v] : (cx<T>*)a.in[v];
  kfft::fft_strided_body<T, L, S>(blockIdx.x, blockIdx.y, gridDim.x, grid, tw, N,
                                  row_stride, outer_stride, outer_pruned, load_pruned,
                                  store_pruned, a.r2[v], ball, outer_in_ball);
}

template <typename T, int L>
__global__ __launch_bounds__(kfft::NT) void k_ifft_crop_x_b(BatchArgs a,
                                                            const double* __restrict__ s,
                                                            const cx<T>* __restrict__ tw, int N) {
  const int v = blockIdx.z;
  kfft::ifft_crop_x_body<T, L>(blockIdx.x, (const cx<T>*)a.in[v], (cx<T>*)a.out[v], s, tw, N);
}

template <typename T, int L, bool ADJ>
__global__ __launch_bounds__(kfft::NT) void k_radial_b(BatchArgs a, const cx<T>* __restrict__ tw,
                                                       int deriv, double dr) {
  const int v = blockIdx.z;
  if ((int64_t)blockIdx.x * kfft::nl_line<T, L>() >= a.n[v]) return;  // past this volume's lines
  kfft::radial_body<T, L, ADJ>(blockIdx.x, (const cx<T>*)a.in[v], (cx<T>*)a.out[v], tw, a.n[v],
                               deriv, dr, nullptr, 1.0);
}

template <typename T, int J, int TILE, bool CW, int DEG>
__global__ __launch_bounds__(kgrid::GridCfg<T>::NT_INTERP)
__attribute__((amdgpu_waves_per_eu(kgrid::GridCfg<T>::INTERP_WAVES))) void k_interp_b(
    const BatchPointVol* __restrict__ vols, BatchStarts start, int nv,
    WeightPoly<T, DEG> P) {
  const int v = find_vol(start, nv, blockIdx.x);
  const BatchPointVol& d = vols[v];
  kgrid::interp_body<T, J, TILE, CW, DEG>((int64_t)blockIdx.x - start.s[v], (const cx<T>*)d.grid,
                                          (cx<T>*)d.tmp, d.perm, d.tasks, d.xs, d.g, d.nb, P);
}

template <typename T, int J, int TILE, bool CW, int DEG, bool FIXED>
__global__ __launch_bounds__(kgrid::GridCfg<T>::NT_SPREAD)
__attribute__((amdgpu_waves_per_eu(kgrid::GridCfg<T>::SPREAD_WAVES))) void k_spread_b(
    const BatchPointVol* __restrict__ vols, BatchStarts start, int nv,
    WeightPoly<T, DEG> P) {
  const int v = find_vol(start, nv, blockIdx.x);
  const BatchPointVol& d = vols[v];
  int64_t task_id = xcd_task((int64_t)blockIdx.x - start.s[v], d.xs);
  if (task_id < 0) return;
  if (d.torder) task_id = d.torder[task_id];
  kgrid::spread_task<T, J, TILE, CW, DEG, FIXED, false>(task_id, (const cx<T>*)d.tmp,
                                                        (cx<T>*)d.partials, d.perm_s, d.tasks,
                                                        d.bound, d.multi, d.g, d.nb, P);
}

// the listed tasks of every volume, volume by volume; the list lengths are
// read together first, so that the usual empty lists cost one memory latency
template <typename T, int J, int TILE, bool CW, int DEG>
__global__ __launch_bounds__(kgrid::GridCfg<T>::NT_SPREAD) void k_spread_rest_b(
    const BatchPointVol* __restrict__ vols, int nv, WeightPoly<T, DEG> P) {
  __shared__ int counts[NUFFTCT_BATCH_MAXV];
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  if ((int)threadIdx.x < nv) {
    counts[threadIdx.x] = vols[threadIdx.x].multi[0];
    if (counts[threadIdx.x] > (int)blockIdx.x) atomicOr(&any, 1);
  }
  __syncthreads();
  if (!any) return;
  for (int v = 0; v < nv; ++v) {
    const BatchPointVol& d = vols[v];
    const int count = counts[v];
    for (int i = blockIdx.x; i < count; i += gridDim.x) {
      kgrid::spread_task<T, J, TILE, CW, DEG, true, true>(d.multi[1 + i], (const cx<T>*)d.tmp,
                                                          (cx<T>*)d.partials, d.perm_s, d.tasks,
                                                          d.bound, d.multi, d.g, d.nb, P);
      __syncthreads();  // the next task reuses the LDS
    }
  }
}

// a batch's merge arguments: those of the volume of block b
struct MergeBatchArgs {
  const BatchPointVol* vols;
  BatchStarts start;
  int nv;
  __device__ __forceinline__ kgrid::MergeArgs resolve(unsigned b, unsigned& bx) const {
    const int v = find_vol(start, nv, b);
    const BatchPointVol& d = vols[v];
    bx = b - (unsigned)start.s[v];
    return kgrid::MergeArgs{(const cx<float>*)d.partials, d.bin_tasks, d.merge_order,
                            (cx<float>*)d.grid, d.nb, d.K, d.R, d.r2, d.multi};
  }
};

template <typename T, int TILE>
__global__ __launch_bounds__(TILE * TILE * TILE < 1024 ? TILE * TILE * TILE : 1024) void k_merge_b(
    const BatchPointVol* __restrict__ vols, BatchStarts start, int nv) {
  const int v = find_vol(start, nv, blockIdx.x);
  const BatchPointVol& d = vols[v];
  kgrid::merge_body<T, TILE>(blockIdx.x - start.s[v], (const cx<T>*)d.partials, d.bin_tasks,
                             d.merge_order, (cx<T>*)d.grid, d.nb, d.K, d.R, d.r2, d.multi);
}

// ---- launchers -------------------------------------------------------------
template <typename T, int L>
hipError_t fwd_fft(const BatchClass<T>& c, const BatchArgs& a, hipStream_t st) {
  constexpr int NLx = kfft::nl_line<T, L>();
  constexpr int NLc = kfft::nl_col<T, L>();
  const int64_t nlines = (int64_t)c.N * c.N;
  hipLaunchKernelGGL((k_pad_fft_x_b<T, L>), dim3((unsigned)((nlines + NLx - 1) / NLx), 1, c.nv),
                     dim3(kfft::NT), 0, st, a, c.s, c.tw_K, c.N);
  hipLaunchKernelGGL((k_fft_strided_b<T, L, -1>), dim3(L / NLc, c.N, c.nv), dim3(kfft::NTS), 0, st,
                     a, c.tw_K, c.N, (int64_t)L, grid_plane_of<T>(L), 1, 1, 0, 1, 0);
  hipLaunchKernelGGL((k_fft_strided_b<T, L, -1>), dim3(L / NLc, L, c.nv), dim3(kfft::NTS), 0, st,
                     a, c.tw_K, c.N, grid_plane_of<T>(L), (int64_t)L, 0, 1, 0, 1, 1);
  return hipGetLastError();
}

template <typename T, int L>
hipError_t adj_fft(const BatchClass<T>& c, const BatchArgs& a, hipStream_t st) {
  constexpr int NLx = kfft::nl_line<T, L>();
  constexpr int NLc = kfft::nl_col<T, L>();
  const int64_t nlines = (int64_t)c.N * c.N;
  hipLaunchKernelGGL((k_fft_strided_b<T, L, +1>), dim3(L / NLc, L, c.nv), dim3(kfft::NTS), 0, st,
                     a, c.tw_K, c.N, grid_plane_of<T>(L), (int64_t)L, 0, 0, 1, 2, 1);
  hipLaunchKernelGGL((k_fft_strided_b<T, L, +1>), dim3(L / NLc, c.N, c.nv), dim3(kfft::NTS), 0, st,
                     a, c.tw_K, c.N, (int64_t)L, grid_plane_of<T>(L), 1, 0, 1, 2, 0);
  hipLaunchKernelGGL((k_ifft_crop_x_b<T, L>), dim3((unsigned)((nlines + NLx - 1) / NLx), 1, c.nv),
                     dim3(kfft::NT), 0, st, a, c.s, c.tw_K, c.N);
  return hipGetLastError();
}

template <typename T, int L>
hipError_t radial(const BatchClass<T>& c, const BatchArgs& a, bool adj, bool deriv,
                  hipStream_t st) {
  constexpr int NLx = kfft::nl_line<T, L>();
  const dim3 grd((unsigned)((c.max_lines + NLx - 1) / NLx), 1, c.nv);
  const double dr = (2.0 * M_PI) / (double)L;
  if (adj)
    hipLaunchKernelGGL((k_radial_b<T, L, true>), grd, dim3(kfft::NT), 0, st, a, c.tw_r, (int)deriv,
                       dr);
  else
    hipLaunchKernelGGL((k_radial_b<T, L, false>), grd, dim3(kfft::NT), 0, st, a, c.tw_r,
                       (int)deriv, dr);
  return hipGetLastError();
}

// what: 0 forward FFT passes (in = volumes, out = grids), 1 inverse FFT passes
// (in = grids, out = volumes; r2 in a.r2), 2 radial, 3 radial adjoint
template <typename T>
hipError_t class_stage(const BatchClass<T>& c, const BatchArgs& a, int what, bool deriv,
                       hipStream_t st) {
  if (what >= 2) {
    switch (c.n_r) {
#define CASE(LL) \
  case LL: return radial<T, LL>(c, a, what == 3, deriv, st);
      KFFT_SIZES(CASE)
#undef CASE
      default: return hipErrorInvalidValue;
    }
  }
  switch (c.K) {
#define CASE(LL) \
  case LL: return what == 0 ? fwd_fft<T, LL>(c, a, st) : adj_fft<T, LL>(c, a, st);
    KFFT_SIZES(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int J, int TILE>
hipError_t point_stage(const BatchGroup& g, int what, bool det, const WeightPoly<T, kgrid::PolyOf<T>::DEG>& P,
                       hipStream_t st) {
  if constexpr (!kgrid::tile_fits<T, J, TILE>()) {
    return hipErrorInvalidValue;
  } else {
    constexpr int DEG = kgrid::PolyOf<T>::DEG;
    if (what == 0) {
      hipLaunchKernelGGL((k_interp_b<T, J, TILE, false, DEG>), dim3((unsigned)g.start_tasks.s[g.nv]),
                         dim3(kgrid::GridCfg<T>::NT_INTERP), 0, st, g.vols, g.start_tasks, g.nv, P);
      return hipGetLastError();
    }
    constexpr bool F32 = sizeof(T) == 4;
    // FP32 always spreads in fixed point; FP64 in deterministic mode only
    const bool fixed = F32 || det;
    const bool any = g.start_tasks.s[g.nv] > 0;  // no tasks: the merge alone writes the zeros
    if (fixed && any) {
      hipLaunchKernelGGL((k_spread_b<T, J, TILE, false, DEG, true>), dim3((unsigned)g.start_tasks.s[g.nv]),
                         dim3(kgrid::GridCfg<T>::NT_SPREAD), 0, st, g.vols, g.start_tasks, g.nv, P);
      const unsigned nbr = (unsigned)std::min<int64_t>(g.max_tasks, kgrid::NB_REST);
      hipLaunchKernelGGL((k_spread_rest_b<T, J, TILE, false, DEG>), dim3(nbr),
                         dim3(kgrid::GridCfg<T>::NT_SPREAD), 0, st, g.vols, g.nv, P);
    }
    if constexpr (!F32) {
      if (!fixed && any)
        hipLaunchKernelGGL((k_spread_b<T, J, TILE, false, DEG, false>), dim3((unsigned)g.start_tasks.s[g.nv]),
                           dim3(kgrid::GridCfg<T>::NT_SPREAD), 0, st, g.vols, g.start_tasks, g.nv, P);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (F32 && TILE == 16)
      hipLaunchKernelGGL((kgrid::k_merge_pairs<16, 2, MergeBatchArgs>),
                         dim3((unsigned)g.start_tiles.s[g.nv]), dim3(1024), 0, st,
                         MergeBatchArgs{g.vols, g.start_tiles, g.nv});
    else
      hipLaunchKernelGGL((k_merge_b<T, TILE>), dim3((unsigned)g.start_tiles.s[g.nv]),
                         dim3(TILE * TILE * TILE < 1024 ? TILE * TILE * TILE : 1024), 0, st, g.vols,
                         g.start_tiles, g.nv);
    return hipGetLastError();
  }
}

// what: 0 interpolation, 1 spreading (+ general pass, merge); det: FP64 fixed point
template <typename T>
hipError_t group_stage(const BatchGroup& g, int what, bool det,
                       const WeightPoly<T, kgrid::PolyOf<T>::DEG>& P, hipStream_t st) {
#define TILES(JJ)                                                        \
  case JJ:                                                               \
    return g.tile == 16 ? point_stage<T, JJ, 16>(g, what, det, P, st)   \
                        : g.tile == 8 ? point_stage<T, JJ, 8>(g, what, det, P, st) \
                                      : hipErrorInvalidValue;
  switch (g.J) {
    TILES(2) TILES(3) TILES(4) TILES(5) TILES(6) TILES(7) TILES(8)
    default: return hipErrorInvalidValue;
  }
#undef TILES
}

}  // namespace kbatch

#define KBATCH_INSTANTIATE(T)                                                                  \
  template <>                                                                                  \
  hipError_t launch_batch_class<T>(const BatchClass<T>& c, const BatchArgs& a, int what,      \
                                   bool deriv, hipStream_t s) {                                \
    return kbatch::class_stage<T>(c, a, what, deriv, s);                                       \
  }                                                                                            \
  template <>                                                                                  \
  hipError_t launch_batch_group<T>(const BatchGroup& g, int what, bool det, const void* poly,  \
                                   hipStream_t s) {                                            \
    return kbatch::group_stage<T>(g, what, det,                                                \
                                  *(const WeightPoly<T, kgrid::PolyOf<T>::DEG>*)poly, s);      \
  }
