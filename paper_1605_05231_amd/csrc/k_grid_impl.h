// J^3 interpolation (gather) and spreading (scatter) between the centred K^3
// spectrum grid and the non-uniform points, LDS-tiled for gfx950.
//
// The sparse interpolator T_sparse of eq 2.11 (Section 2.1.3) with the
// neighbour rule t = omega_d / (2 pi / K), k0 = floor(t - J/2), taps
// k0+1..k0+J per axis, and its transpose (the NUFFT transpose).
//
// Points are binned on the host by the tile of their first tap (tile edge
// TILE cells dividing K) and processed tile by tile.  Interpolation: one
// workgroup per task (a bin and up to max_pts of its points) stages the tile
// plus its (J-1)-cell halo, S^3 cells with S = TILE + J - 1, in LDS once;
// every point then reads its J^3 taps there.  Spreading is owner-computes
// (see k_spread): no global atomics, every grid cell written once.
// The tap index math runs in FP64 without contraction so that it reproduces
// the host binning bit for bit; in the interpolation a point whose taps still
// fall outside the staged tile takes a global-memory path.
//
// Weights: per tap a, w_a = P_a(z), a polynomial in z = 2 frac - 1 fitted on
// the host in FP64 to the kernel on that tap's unit interval (Kaiser-Bessel
// real; min-max complex), evaluated with Horner's rule.
#pragma once

#include "cx.h"
#include "plan.h"

namespace kgrid {

constexpr int NT = 256;

template <typename T>
__device__ __forceinline__ void lds_add(T* a, T v) {
  [[clang::atomic(no_remote_memory, no_fine_grained_memory, ignore_denormal_mode)]] {
    __hip_atomic_fetch_add(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

// First tap (centred, wrapped to [0, K)) and fractional offset per axis.
__device__ __forceinline__ void point_taps(const PointGeom& g, int p, int J, int (&first)[3],
                                           double (&frac)[3]) {
#pragma clang fp contract(off)
  double om[3];
  if (g.n_r) {
    const int l = p / g.n_r;
    const int c = p - l * g.n_r;
    const double r = (double)(c - g.n_r / 2) * g.dr;
    om[0] = r * g.dirs[3 * (int64_t)l + 0];
    om[1] = r * g.dirs[3 * (int64_t)l + 1];
    om[2] = r * g.dirs[3 * (int64_t)l + 2];
  } else {
    om[0] = g.pts[3 * (int64_t)p + 0];
    om[1] = g.pts[3 * (int64_t)p + 1];
    om[2] = g.pts[3 * (int64_t)p + 2];
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double t = om[d] / g.gamma;
    const double tj = t - 0.5 * (double)J;
    const double k0 = floor(tj);
    frac[d] = tj - k0;
    int64_t f = (int64_t)k0 + 1 + g.K / 2;
    f %= g.K;
    if (f < 0) f += g.K;
    first[d] = (int)f;
  }
}

template <typename T, int J, int DEG, bool CW>
__device__ __forceinline__ void axis_weights(const WeightPoly<T, DEG>& P, double frac,
                                             T (&wr)[J], T (&wi)[J]) {
  const T z = (T)(2.0 * frac - 1.0);
#pragma unroll
  for (int a = 0; a < J; ++a) {
    T acc = P.re[a][DEG];
#pragma unroll
    for (int d = DEG - 1; d >= 0; --d) acc = acc * z + P.re[a][d];
    wr[a] = acc;
    if constexpr (CW) {
      T ai = P.im[a][DEG];
#pragma unroll
      for (int d = DEG - 1; d >= 0; --d) ai = ai * z + P.im[a][d];
      wi[a] = ai;
    } else {
      wi[a] = (T)0;
    }
  }
}

__device__ __forceinline__ int wrapK(int c, int K) { return c >= K ? c - K : c; }

// ---------------------------------------------------------------------------
template <typename T, int J, int TILE, bool CW, int DEG>
__global__ __launch_bounds__(NT) void k_interp(const cx<T>* __restrict__ grid,
                                               cx<T>* __restrict__ out,
                                               const int32_t* __restrict__ perm,
                                               const TileTask* __restrict__ tasks,
                                               int64_t ntasks, int64_t per_xcd, PointGeom g,
                                               int nb, WeightPoly<T, DEG> P) {
  constexpr int S = TILE + J - 1;
  __shared__ cx<T> tile[S * S * S];
  const int64_t task_id = xcd_task(blockIdx.x, per_xcd);
  if (task_id >= ntasks) return;
  const TileTask tk = tasks[task_id];
  const int K = g.K;
  const int b2 = tk.bin % nb, b1 = (tk.bin / nb) % nb, b0 = tk.bin / (nb * nb);
  const int o0 = b0 * TILE, o1 = b1 * TILE, o2 = b2 * TILE;
  for (int idx = threadIdx.x; idx < S * S * S; idx += NT) {
    const int i2 = idx % S, i1 = (idx / S) % S, i0 = idx / (S * S);
    const int c0 = wrapK(o0 + i0, K), c1 = wrapK(o1 + i1, K), c2 = wrapK(o2 + i2, K);
    tile[idx] = grid[((int64_t)c0 * K + c1) * K + c2];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < tk.count; i += NT) {
    const int p = perm[tk.start + i];
    int first[3];
    double frac[3];
    point_taps(g, p, J, first, frac);
    T w0r[J], w0i[J], w1r[J], w1i[J], w2r[J], w2i[J];
    axis_weights<T, J, DEG, CW>(P, frac[0], w0r, w0i);
    axis_weights<T, J, DEG, CW>(P, frac[1], w1r, w1i);
    axis_weights<T, J, DEG, CW>(P, frac[2], w2r, w2i);
    const int l0 = first[0] - o0, l1 = first[1] - o1, l2 = first[2] - o2;
    const bool inside = (unsigned)l0 < (unsigned)TILE && (unsigned)l1 < (unsigned)TILE &&
                        (unsigned)l2 < (unsigned)TILE;
    cx<T> acc = {0, 0};
#pragma unroll
    for (int a = 0; a < J; ++a) {
      cx<T> acc_a = {0, 0};
#pragma unroll
      for (int b = 0; b < J; ++b) {
        cx<T> acc_b = {0, 0};
        if (inside) {
          const cx<T>* row = &tile[((l0 + a) * S + (l1 + b)) * S + l2];
#pragma unroll
          for (int c = 0; c < J; ++c) {
            const cx<T> v = row[c];
            if constexpr (CW) {
              acc_b = cadd(acc_b, cmul(v, cx<T>{w2r[c], w2i[c]}));
            } else {
              acc_b.x += w2r[c] * v.x;
              acc_b.y += w2r[c] * v.y;
            }
          }
        } else {
          const int c0 = wrapK(first[0] + a, K), c1 = wrapK(first[1] + b, K);
          const cx<T>* row = grid + ((int64_t)c0 * K + c1) * K;
#pragma unroll
          for (int c = 0; c < J; ++c) {
            const cx<T> v = row[wrapK(first[2] + c, K)];
            if constexpr (CW) {
              acc_b = cadd(acc_b, cmul(v, cx<T>{w2r[c], w2i[c]}));
            } else {
              acc_b.x += w2r[c] * v.x;
              acc_b.y += w2r[c] * v.y;
            }
          }
        }
        if constexpr (CW) {
          acc_a = cadd(acc_a, cmul(acc_b, cx<T>{w1r[b], w1i[b]}));
        } else {
          acc_a.x += w1r[b] * acc_b.x;
          acc_a.y += w1r[b] * acc_b.y;
        }
      }
      if constexpr (CW) {
        acc = cadd(acc, cmul(acc_a, cx<T>{w0r[a], w0i[a]}));
      } else {
        acc.x += w0r[a] * acc_a.x;
        acc.y += w0r[a] * acc_a.y;
      }
    }
    out[p] = acc;
  }
}

// ---------------------------------------------------------------------------
// Owner-computes spreading: one task per output tile (or per chunk of a heavy
// tile's points).  The tile (TILE^3 cells, no halo) accumulates in LDS the
// contributions of every point whose footprint reaches it: the points of its
// own bin and the spilling points of the 7 lower-neighbour bins, listed as
// segments of the permutation.  The finished tile is written with plain
// coalesced stores, zeros included, so the grid needs no clearing and no
// global atomics; a split tile writes a partial that k_reduce_partials sums
// in a fixed order.
template <typename T, int J, int TILE, bool CW, int DEG>
__global__ __launch_bounds__(NT) void k_spread(const cx<T>* __restrict__ in,
                                               cx<T>* __restrict__ grid,
                                               cx<double>* __restrict__ partials,
                                               const int32_t* __restrict__ perm,
                                               const SpreadTask* __restrict__ tasks,
                                               const SpreadSeg* __restrict__ segs,
                                               int64_t ntasks, int64_t per_xcd, PointGeom g,
                                               int nb, WeightPoly<T, DEG> P) {
  constexpr int TT = TILE * TILE * TILE;
  constexpr int RP = TILE + 1;  // padded row pitch (breaks r2-only bank mapping)
  // FP64 accumulators: LDS f64 atomic adds run several times faster than f32
  // ones on gfx950 and make the per-tile sums exact to FP32 output precision
  __shared__ cx<double> tile[TILE * TILE * RP];
  const int64_t task_id = xcd_task(blockIdx.x, per_xcd);
  if (task_id >= ntasks) return;
  const SpreadTask tk = tasks[task_id];
  const int K = g.K;
  const int t2 = tk.tile % nb, t1 = (tk.tile / nb) % nb, t0 = tk.tile / (nb * nb);
  for (int idx = threadIdx.x; idx < TILE * TILE * RP; idx += NT) tile[idx] = cx<double>{0, 0};
  __syncthreads();
  int base = 0;
  for (int s = tk.seg_begin; s < tk.seg_end; ++s) {
    const SpreadSeg sg = segs[s];
    const int lo = max(tk.p_lo, base) - base;
    const int hi = min(tk.p_hi, base + sg.count) - base;
    base += sg.count;
    if (lo >= hi) continue;
    const int d0 = (sg.delta >> 2) & 1, d1 = (sg.delta >> 1) & 1, d2 = sg.delta & 1;
    // origin of the source bin's tile
    const int so0 = ((t0 - d0 + nb) % nb) * TILE;
    const int so1 = ((t1 - d1 + nb) % nb) * TILE;
    const int so2 = ((t2 - d2 + nb) % nb) * TILE;
    for (int i = lo + (int)threadIdx.x; i < hi; i += NT) {
      const int p = perm[sg.start + i];
      const cx<T> v = in[p];
      int first[3];
      double frac[3];
      point_taps(g, p, J, first, frac);
      T w0r[J], w0i[J], w1r[J], w1i[J], w2r[J], w2i[J];
      axis_weights<T, J, DEG, CW>(P, frac[0], w0r, w0i);
      axis_weights<T, J, DEG, CW>(P, frac[1], w1r, w1i);
      axis_weights<T, J, DEG, CW>(P, frac[2], w2r, w2i);
      // first tap relative to this tile's origin (negative when it lies in the
      // lower neighbour tile)
      int q0 = first[0] - so0, q1 = first[1] - so1, q2 = first[2] - so2;
      q0 += q0 < 0 ? K : 0;
      q1 += q1 < 0 ? K : 0;
      q2 += q2 < 0 ? K : 0;
      const int l0 = q0 - d0 * TILE, l1 = q1 - d1 * TILE, l2 = q2 - d2 * TILE;
#pragma unroll
      for (int a = 0; a < J; ++a) {
        const int r0 = l0 + a;
        if ((unsigned)r0 >= (unsigned)TILE) continue;
        // conj(w) for the transpose
        const cx<T> va = CW ? cmulc(v, cx<T>{w0r[a], w0i[a]}) : cx<T>{w0r[a] * v.x, w0r[a] * v.y};
#pragma unroll
        for (int b = 0; b < J; ++b) {
          const int r1 = l1 + b;
          if ((unsigned)r1 >= (unsigned)TILE) continue;
          const cx<T> vb =
              CW ? cmulc(va, cx<T>{w1r[b], w1i[b]}) : cx<T>{w1r[b] * va.x, w1r[b] * va.y};
          cx<double>* row = &tile[(r0 * TILE + r1) * RP];
#pragma unroll
          for (int c = 0; c < J; ++c) {
            const int r2 = l2 + c;
            if ((unsigned)r2 >= (unsigned)TILE) continue;
            const cx<T> u =
                CW ? cmulc(vb, cx<T>{w2r[c], w2i[c]}) : cx<T>{w2r[c] * vb.x, w2r[c] * vb.y};
            lds_add(&row[r2].x, (double)u.x);
            lds_add(&row[r2].y, (double)u.y);
          }
        }
      }
    }
  }
  __syncthreads();
  if (tk.slot < 0) {
    const int o0 = t0 * TILE, o1 = t1 * TILE, o2 = t2 * TILE;
    for (int idx = threadIdx.x; idx < TT; idx += NT) {
      const int i2 = idx % TILE, i1 = (idx / TILE) % TILE, i0 = idx / (TILE * TILE);
      const cx<double> v = tile[(i0 * TILE + i1) * RP + i2];
      grid[((int64_t)(o0 + i0) * K + (o1 + i1)) * K + (o2 + i2)] = cx<T>{(T)v.x, (T)v.y};
    }
  } else {
    cx<double>* dst = partials + (int64_t)tk.slot * TT;
    for (int idx = threadIdx.x; idx < TT; idx += NT) {
      const int i2 = idx % TILE, i1 = (idx / TILE) % TILE, i0 = idx / (TILE * TILE);
      dst[idx] = tile[(i0 * TILE + i1) * RP + i2];
    }
  }
}

// Sum the partial tiles of each split output tile, in slot order, into the grid.
template <typename T>
__global__ __launch_bounds__(NT) void k_reduce_partials(const cx<double>* __restrict__ partials,
                                                        cx<T>* __restrict__ grid,
                                                        const HeavyTile* __restrict__ heavy,
                                                        int nb, int K, int TILE) {
  const HeavyTile h = heavy[blockIdx.x];
  const int TT = TILE * TILE * TILE;
  const int t2 = h.tile % nb, t1 = (h.tile / nb) % nb, t0 = h.tile / (nb * nb);
  for (int idx = threadIdx.x; idx < TT; idx += NT) {
    cx<double> acc = {0, 0};
    for (int s = h.slot_begin; s < h.slot_end; ++s) acc = cadd(acc, partials[(int64_t)s * TT + idx]);
    const int i2 = idx % TILE, i1 = (idx / TILE) % TILE, i0 = idx / (TILE * TILE);
    grid[((int64_t)(t0 * TILE + i0) * K + (t1 * TILE + i1)) * K + (t2 * TILE + i2)] =
        cx<T>{(T)acc.x, (T)acc.y};
  }
}

// ---------------------------------------------------------------------------
template <typename T>
struct PolyOf;
template <>
struct PolyOf<float> {
  static constexpr int DEG = NUFFTCT_DEG_F32;
  static const WeightPoly<float, DEG>& get(const nufftct_plan& p) { return p.wp32; }
};
template <>
struct PolyOf<double> {
  static constexpr int DEG = NUFFTCT_DEG_F64;
  static const WeightPoly<double, DEG>& get(const nufftct_plan& p) { return p.wp64; }
};

template <typename T, int J, int TILE>
constexpr bool tile_fits() {
  return (TILE + J - 1) * (TILE + J - 1) * (TILE + J - 1) * (int)sizeof(cx<T>) <= 96 * 1024 &&
         J - 1 <= TILE;
}

template <typename T, int J, int TILE, bool CW, bool SPREAD>
hipError_t launch_one(const nufftct_plan& p, const void* src, void* dst, hipStream_t st) {
  if constexpr (!tile_fits<T, J, TILE>()) {
    return hipErrorInvalidValue;
  } else {
    constexpr int DEG = PolyOf<T>::DEG;
    const auto& P = PolyOf<T>::get(p);
    const int64_t per = (p.ntasks + NUFFTCT_NUM_XCD - 1) / NUFFTCT_NUM_XCD;
    const dim3 grd((unsigned)(per * NUFFTCT_NUM_XCD));
    const PointGeom g = p.geom();
    if (SPREAD) {
      const int64_t sper = (p.n_sp_tasks + NUFFTCT_NUM_XCD - 1) / NUFFTCT_NUM_XCD;
      hipLaunchKernelGGL((k_spread<T, J, TILE, CW, DEG>), dim3((unsigned)(sper * NUFFTCT_NUM_XCD)),
                         dim3(NT), 0, st, (const cx<T>*)src, (cx<T>*)dst, (cx<double>*)p.d_partials,
                         p.d_perm, p.d_sp_tasks, p.d_sp_segs, p.n_sp_tasks, sper, g, p.nb, P);
    } else {
      hipLaunchKernelGGL((k_interp<T, J, TILE, CW, DEG>), grd, dim3(NT), 0, st,
                         (const cx<T>*)src, (cx<T>*)dst, p.d_perm, p.d_tasks, p.ntasks, per, g,
                         p.nb, P);
    }
    return hipGetLastError();
  }
}

template <typename T, int J, bool CW, bool SPREAD>
hipError_t by_tile(const nufftct_plan& p, const void* src, void* dst, hipStream_t st) {
  switch (p.tile) {
    case 8: return launch_one<T, J, 8, CW, SPREAD>(p, src, dst, st);
    case 16: return launch_one<T, J, 16, CW, SPREAD>(p, src, dst, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, bool CW, bool SPREAD>
hipError_t by_j(const nufftct_plan& p, const void* src, void* dst, hipStream_t st) {
  switch (p.J) {
    case 2: return by_tile<T, 2, CW, SPREAD>(p, src, dst, st);
    case 3: return by_tile<T, 3, CW, SPREAD>(p, src, dst, st);
    case 4: return by_tile<T, 4, CW, SPREAD>(p, src, dst, st);
    case 5: return by_tile<T, 5, CW, SPREAD>(p, src, dst, st);
    case 6: return by_tile<T, 6, CW, SPREAD>(p, src, dst, st);
    case 7: return by_tile<T, 7, CW, SPREAD>(p, src, dst, st);
    case 8: return by_tile<T, 8, CW, SPREAD>(p, src, dst, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, bool SPREAD>
hipError_t run(const nufftct_plan& p, const void* src, void* dst, hipStream_t st) {
  if (p.ntasks == 0) return hipSuccess;
  if (p.kernel == NUFFTCT_KERNEL_MINMAX_KB) return by_j<T, true, SPREAD>(p, src, dst, st);
  return by_j<T, false, SPREAD>(p, src, dst, st);
}

template <typename T>
hipError_t reduce(const nufftct_plan& p, void* grid, hipStream_t st) {
  if (p.n_heavy == 0) return hipSuccess;
  hipLaunchKernelGGL((k_reduce_partials<T>), dim3((unsigned)p.n_heavy), dim3(NT), 0, st,
                     (const cx<double>*)p.d_partials, (cx<T>*)grid, p.d_heavy, p.nb, (int)p.K, p.tile);
  return hipGetLastError();
}

}  // namespace kgrid

#define KGRID_INSTANTIATE(T)                                                                \
  template <>                                                                               \
  hipError_t launch_interp<T>(const nufftct_plan& p, const void* grid, void* out,           \
                              hipStream_t s) {                                              \
    return kgrid::run<T, false>(p, grid, out, s);                                           \
  }                                                                                         \
  template <>                                                                               \
  hipError_t launch_spread<T>(const nufftct_plan& p, const void* in, void* grid,            \
                              hipStream_t s) {                                              \
    return kgrid::run<T, true>(p, in, grid, s);                                             \
  }                                                                                         \
  template <>                                                                               \
  hipError_t launch_reduce_partials<T>(const nufftct_plan& p, void* grid, hipStream_t s) {  \
    return kgrid::reduce<T>(p, grid, s);                                                    \
  }
