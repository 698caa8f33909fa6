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
// every point then reads its J^3 taps there.  Spreading uses the same tasks:
// each accumulates its halo tile in LDS and stores it as a partial; an
// owner-computes merge sums the partials into the grid.  No global atomics;
// every grid cell is written once.
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

// Launch shapes per precision (measured on gfx950):
//   FP32 interpolation: two 512-thread workgroups per CU (LDS-bound) within
//     128 VGPRs, which leaves room for a one-ahead prefetch of the next
//     point's id only (not of its geometry);
//   FP32 spreading: one 8-byte accumulator per halo cell (74 KB for tile 16,
//     J = 6), so two 512-thread workgroups share a CU within 128 VGPRs;
//   FP64: 256-thread interpolation with the next point's geometry prefetched,
//     1024-thread spreading.
template <typename T>
struct GridCfg;
template <>
struct GridCfg<float> {
  static constexpr int NT_INTERP = 512, INTERP_WAVES = 4, NT_SPREAD = 512, SPREAD_WAVES = 4;
  static constexpr bool PREFETCH_GEOM = false;
};
template <>
struct GridCfg<double> {
  static constexpr int NT_INTERP = 256, INTERP_WAVES = 1, NT_SPREAD = 1024, SPREAD_WAVES = 1;
  static constexpr bool PREFETCH_GEOM = true;
};
// threads of the plan-time spreading-bound kernel (FP32 plans only)
constexpr int NT_BOUND = 512;

template <typename T>
__device__ __forceinline__ void lds_add(T* a, T v) {
  [[clang::atomic(no_remote_memory, no_fine_grained_memory, ignore_denormal_mode)]] {
    __hip_atomic_fetch_add(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

// Raw geometry of one point as loaded from memory: the multiplier r and the
// direction (radial plans: r = r_c, a = nhat_l) or r = 1 and a = omega (point
// plans), so that omega = r * a in FP64 either way (exact for r = 1).  Loading
// it is separated from using it so that the next point's loads can be issued
// one iteration ahead.
struct PtRaw {
  int p;
  double r, a0, a1, a2;
};

__device__ __forceinline__ PtRaw point_of(const PointGeom& g, int pid) {
#pragma clang fp contract(off)
  PtRaw q;
  q.p = pid;
  if (g.n_r) {
    // line and sample of the point: q.p / n_r through a double reciprocal,
    // corrected by one either way
    int l = (int)((double)q.p * g.inv_nr);
    int c = q.p - l * g.n_r;
    if (c < 0) {
      --l;
      c += g.n_r;
    } else if (c >= g.n_r) {
      ++l;
      c -= g.n_r;
    }
    q.r = (double)(c - g.n_r / 2) * g.dr;
    q.a0 = g.dirs[3 * (int64_t)l + 0];
    q.a1 = g.dirs[3 * (int64_t)l + 1];
    q.a2 = g.dirs[3 * (int64_t)l + 2];
  } else {
    q.r = 1.0;
    q.a0 = g.pts[3 * (int64_t)q.p + 0];
    q.a1 = g.pts[3 * (int64_t)q.p + 1];
    q.a2 = g.pts[3 * (int64_t)q.p + 2];
  }
  return q;
}

__device__ __forceinline__ PtRaw fetch_point(const PointGeom& g, const int32_t* __restrict__ perm,
                                             int idx) {
  return point_of(g, perm[idx]);
}

// First tap (centred, wrapped to [0, K)) and fractional offset per axis, with
// the host binning's FP64 arithmetic (no contraction): t = omega / gamma,
// k0 = floor(t - J/2).  FAST: t is first formed as omega * (1/gamma), which
// differs from the quotient by a few ulps at most; where that leaves the
// fractional part farther than 1e-9 from an integer, floor() cannot differ
// and the result stands (the fraction then differs from the exact one by
// ~1e-13, far below FP32 resolution); otherwise the exact quotient is taken.
template <bool FAST>
__device__ __forceinline__ void point_taps(const PointGeom& g, const PtRaw& q, int J,
                                           int (&first)[3], double (&frac)[3]) {
#pragma clang fp contract(off)
  const double om[3] = {q.r * q.a0, q.r * q.a1, q.r * q.a2};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double tj, k0;
    bool exact = !FAST;
    if (FAST) {
      tj = om[d] * g.inv_gamma - 0.5 * (double)J;
      k0 = floor(tj);
      const double fr = tj - k0;
      exact = fr < 1e-9 || fr > 1.0 - 1e-9;
    }
    if (exact) {
      const double t = om[d] / g.gamma;
      tj = t - 0.5 * (double)J;
      k0 = floor(tj);
    }
    frac[d] = tj - k0;
    // |omega| is bounded at plan creation, so k0 fits an int; wrap without a
    // 64-bit modulo in the common case
    int f = (int)k0 + 1 + g.K / 2;
    if ((unsigned)f >= (unsigned)g.K) {
      f %= g.K;
      if (f < 0) f += g.K;
    }
    first[d] = f;
  }
}

template <typename T, int J, int DEG, bool CW>
__device__ __forceinline__ void axis_weights(const WeightPoly<T, DEG>& P, double frac,
                                             T (&wr)[J], T (&wi)[J]) {
  const T z = (T)(2.0 * frac - 1.0);
  if constexpr (!CW) {
    // The Kaiser-Bessel kernel is even, so tap J-1-a at z is tap a at -z:
    // with P_a(z) = E(z^2) + z O(z^2), w_a = E + z O and w_{J-1-a} = E - z O,
    // half the polynomial work of evaluating every tap.
    const T z2 = z * z;
#pragma unroll
    for (int a = 0; a < (J + 1) / 2; ++a) {
      constexpr int TOPE = DEG & ~1, TOPO = (DEG - 1) | 1;  // highest even / odd power
      T e = P.re[a][TOPE];
#pragma unroll
      for (int d = TOPE - 2; d >= 0; d -= 2) e = e * z2 + P.re[a][d];
      T o = P.re[a][TOPO];
#pragma unroll
      for (int d = TOPO - 2; d >= 1; d -= 2) o = o * z2 + P.re[a][d];
      wr[a] = e + z * o;
      wi[a] = (T)0;
      if (J - 1 - a != a) {  // (the middle tap of an odd J is its own mirror)
        wr[J - 1 - a] = e - z * o;
        wi[J - 1 - a] = (T)0;
      }
    }
    return;
  }
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

// floor(x + 1/2) as a 32-bit integer in one instruction (|x| < 2^31); the
// compiler's round-to-nearest conversion takes two
__device__ __forceinline__ int round_int(float x) {
  int r;
  asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
  return r;
}

// Innermost pitch of the interpolation's staged halo tile: for FP32, S rounded
// up to even, so that a row's start parity equals its first tap's parity and
// pairs of complex values can be read as aligned 16-byte words.
template <typename T>
constexpr int interp_pitch(int S) { return sizeof(T) == 4 ? S + (S & 1) : S; }

// Read J consecutive complex values of a staged row starting at element rs.
template <typename T, int J>
__device__ __forceinline__ void read_row(const cx<T>* tile, int rs, cx<T> (&v)[J]) {
#pragma unroll
  for (int k = 0; k < J; ++k) v[k] = tile[rs + k];
}

// The same row read as aligned 16-byte pairs (FP32 only; the row pitch is
// even), halving the LDS instructions of the gather: rs the row's first
// element (read singly when odd, as is an odd tail), h the index of the
// first aligned pair at or after it, EVEN the parity of rs.
template <typename T, int J, bool EVEN>
__device__ __forceinline__ void read_row_pairs(const cx<T>* tile, int rs, int h, cx<T> (&v)[J]) {
  static_assert(sizeof(T) == 4, "pair reads are for FP32 complex values");
  const float4* q = reinterpret_cast<const float4*>(tile);
  constexpr int k0 = EVEN ? 0 : 1;
  if constexpr (!EVEN) v[0] = tile[rs];
#pragma unroll
  for (int k = k0; k + 1 < J; k += 2) {
    const float4 w = q[h + (k - k0) / 2];
    v[k] = cx<T>{w.x, w.y};
    v[k + 1] = cx<T>{w.z, w.w};
  }
  if constexpr (((J - k0) & 1) != 0) v[J - 1] = tile[rs + J - 1];
}

template <typename T, int J, bool CW>
__device__ __forceinline__ cx<T> wmac(cx<T> acc, cx<T> v, T wr, T wi) {
  if constexpr (CW) return cadd(acc, cmul(v, cx<T>{wr, wi}));
  return cx<T>{acc.x + wr * v.x, acc.y + wr * v.y};
}

// Separable J^3 gather of one point.  MODE 0: taps inside the staged tile
// are read from LDS one value at a time, others from the global grid;
// MODE 1 / 2: every tap is inside and the first tap's cell is even / odd,
// rows are read with pair reads.
template <typename T, int J, int S, int S2, bool CW, int MODE>
__device__ __forceinline__ cx<T> gather(const cx<T>* tile, const cx<T>* __restrict__ grid, int K,
                                        const int (&first)[3], int l0, int l1, int l2, bool inside,
                                        const T (&w0r)[J], const T (&w0i)[J], const T (&w1r)[J],
                                        const T (&w1i)[J], const T (&w2r)[J], const T (&w2i)[J]) {
  cx<T> acc = {0, 0};
  // pair reads: the first tap's staged element and the index of the first
  // 16-byte pair at or after it; with S2 even, every other row of the
  // footprint starts a constant number of pairs further, so the reads'
  // addresses differ only by immediate offsets
  const int rs0 = (l0 * S + l1) * S2 + l2;
  const int h0 = (rs0 + (MODE == 2 ? 1 : 0)) >> 1;
  // the outermost tap loop stays rolled: full unrolling lets the compiler
  // hoist every row read of a point and spill
#pragma unroll 1
  for (int a = 0; a < J; ++a) {
    cx<T> acc_a = {0, 0};
#pragma unroll
    for (int b = 0; b < J; ++b) {
      cx<T> acc_b = {0, 0};
      cx<T> rv[J];
      if constexpr (MODE != 0) {
        static_assert(S2 % 2 == 0, "pair reads need an even row pitch");
        const int row = (a * S + b) * S2;
        read_row_pairs<T, J, MODE == 1>(tile, rs0 + row, h0 + (a * S + b) * (S2 / 2), rv);
      } else if (inside) {
        read_row<T, J>(tile, ((l0 + a) * S + (l1 + b)) * S2 + l2, rv);
      } else {
        const int c0 = wrapK(first[0] + a, K), c1 = wrapK(first[1] + b, K);
        const cx<T>* row = grid + (int64_t)c0 * grid_plane_of<T>(K) + (int64_t)c1 * K;
#pragma unroll
        for (int c = 0; c < J; ++c) rv[c] = row[wrapK(first[2] + c, K)];
      }
#pragma unroll
      for (int c = 0; c < J; ++c) acc_b = wmac<T, J, CW>(acc_b, rv[c], w2r[c], w2i[c]);
      acc_a = wmac<T, J, CW>(acc_a, acc_b, w1r[b], w1i[b]);
    }
    acc = wmac<T, J, CW>(acc, acc_a, w0r[a], w0i[a]);
  }
  return acc;
}

// Layout of a task's halo partial in memory.  The halo (S^3 cells, S = TILE +
// R, R = J - 1) is cut per axis into the task's own TILE cells and the R cells
// that belong to the next bin; the 8 resulting blocks are stored one after
// another, block delta = 4 d0 + 2 d1 + d2 (d = 1: the outer part on that
// axis), each row-major over its own extents.  Block delta is exactly what
// bin (own + delta) adds to its cells [0, e0) x [0, e1) x [0, e2) (e = TILE or
// R), so the merge reads every block as one contiguous, line-aligned run.
// Per-task stride: S^3 rounded up to 16 cells (128 B for FP32).
__host__ __device__ constexpr int part_ext(int d, int tile, int r) { return d ? r : tile; }
__host__ __device__ constexpr int part_size(int delta, int tile, int r) {
  return part_ext((delta >> 2) & 1, tile, r) * part_ext((delta >> 1) & 1, tile, r) *
         part_ext(delta & 1, tile, r);
}
__host__ __device__ constexpr int part_base(int delta, int tile, int r) {
  int b = 0;
  for (int k = 0; k < delta; ++k) b += part_size(k, tile, r);
  return b;
}
__host__ __device__ constexpr int part_stride(int tile, int r) {
  return ((tile + r) * (tile + r) * (tile + r) + 15) / 16 * 16;
}
// offset in a task's partial of halo cell (q0, q1, q2)
__host__ __device__ inline int part_offset(int q0, int q1, int q2, int tile, int r) {
  const int d0 = q0 >= tile, d1 = q1 >= tile, d2 = q2 >= tile;
  const int delta = 4 * d0 + 2 * d1 + d2;
  const int e1 = part_ext(d1, tile, r), e2 = part_ext(d2, tile, r);
  return part_base(delta, tile, r) + ((q0 - d0 * tile) * e1 + (q1 - d1 * tile)) * e2 +
         (q2 - d2 * tile);
}

// ---------------------------------------------------------------------------
// (the kernels below are device bodies taking their block index, wrapped by
// one-plan kernels here and by the batch kernels of k_batch_impl.h)
// Stage the S^3 halo tile at grid cell (o0, o1, o2) into LDS (rows of pitch
// S2): a thread's elements idx = tid + k NT, all CH loads in flight before
// their LDS writes, coordinates stepped by NT's own digits in base S (no
// division per element).  WRAP: the halo crosses the grid's end, so every
// coordinate wraps; otherwise the elements' grid offsets are stepped too.
template <typename T, int S, int S2, int NT, int CH, bool WRAP>
__device__ __forceinline__ void stage_halo(cx<T>* tile, const cx<T>* __restrict__ grid, int K,
                                           int o0, int o1, int o2) {
  constexpr int NE = S * S * S;
  constexpr int D0 = NT / (S * S), D1 = (NT / S) % S, D2 = NT % S;
  const int P = (int)grid_plane_of<T>(K);
  const cx<T>* gt = grid + (int64_t)o0 * P + (int64_t)o1 * K + o2;
#pragma unroll 1
  for (int i = threadIdx.x; i < NE; i += CH * NT) {
    cx<T> v[CH];
    int lds[CH];
    int i2 = i % S, i1 = (i / S) % S, i0 = i / (S * S);
    int go = i0 * P + i1 * K + i2, li = (i0 * S + i1) * S2 + i2;
#pragma unroll
    for (int k = 0; k < CH; ++k) {
      lds[k] = li;
      if (i + k * NT < NE) {
        if constexpr (!WRAP) {
          v[k] = gt[go];
        } else {
          const int c0 = wrapK(o0 + i0, K), c1 = wrapK(o1 + i1, K), c2 = wrapK(o2 + i2, K);
          v[k] = grid[(int64_t)c0 * P + (int64_t)c1 * K + c2];
        }
      }
      i2 += D2;
      go += D0 * P + D1 * K + D2;
      li += (D0 * S + D1) * S2 + D2;
      if (i2 >= S) {
        i2 -= S;
        ++i1;
        go += K - S;
        li += S2 - S;
      }
      i1 += D1;
      if (i1 >= S) {
        i1 -= S;
        ++i0;
        go += P - S * K;
      }
      i0 += D0;
    }
#pragma unroll
    for (int k = 0; k < CH; ++k)
      if (i + k * NT < NE) tile[lds[k]] = v[k];
  }
}

template <typename T, int J, int TILE, bool CW, int DEG>
__device__ __forceinline__ void interp_body(int64_t bx, const cx<T>* __restrict__ grid,
                                            cx<T>* __restrict__ out,
                                            const int32_t* __restrict__ perm,
                                            const TileTask* __restrict__ tasks,
                                            const XcdSplit& xs, const PointGeom& g, int nb,
                                            const WeightPoly<T, DEG>& P) {
  constexpr int NT_INTERP = GridCfg<T>::NT_INTERP;
  constexpr int S = TILE + J - 1;
  constexpr int S2 = interp_pitch<T>(S);
  __shared__ float4 tile_mem[(S * S * S2 * (int)sizeof(cx<T>) + 15) / 16];
  cx<T>* tile = reinterpret_cast<cx<T>*>(tile_mem);
  const int64_t task_id = xcd_task(bx, xs);
  if (task_id < 0) return;
  const TileTask tk = tasks[task_id];
  const int K = g.K;
  const int b2 = tk.bin % nb, b1 = (tk.bin / nb) % nb, b0 = tk.bin / (nb * nb);
  const int o0 = b0 * TILE, o1 = b1 * TILE, o2 = b2 * TILE;
  {
    // CH loads per thread in flight before their LDS writes (a loop that
    // writes each cell as it arrives waits on every load in turn): the whole
    // tile in one round trip where 20 loads per thread cover it (J <= 7 at
    // 16^3 tiles; 8 per round measured 10 % slower at c3)
    constexpr int NE = S * S * S;
    constexpr int CH = (NE + NT_INTERP - 1) / NT_INTERP < 20 ? (NE + NT_INTERP - 1) / NT_INTERP : 20;
    const bool edge = o0 + S > K || o1 + S > K || o2 + S > K;
    if (edge)
      stage_halo<T, S, S2, NT_INTERP, CH, true>(tile, grid, K, o0, o1, o2);
    else
      stage_halo<T, S, S2, NT_INTERP, CH, false>(tile, grid, K, o0, o1, o2);
  }
  __syncthreads();
  // Units of the task's interpolation order: unit u < ntwins is the pair of
  // points at entries 2u, 2u + 1 (one frequency sampled twice: one
  // evaluation, two outputs), unit u >= ntwins the point at entry ntwins + u.
  const int nt = tk.ntwins, nunits = tk.count - nt;
  auto entry = [&](int u) { return tk.start + (u < nt ? 2 * u : nt + u); };
  // the next unit one iteration ahead: its whole geometry (FP64), or only its
  // id (FP32, whose register budget has no room for the geometry)
  PtRaw nxt;
  int pnxt = 0;
  if ((int)threadIdx.x < nunits) {
    if constexpr (GridCfg<T>::PREFETCH_GEOM) nxt = fetch_point(g, perm, entry(threadIdx.x));
    else pnxt = perm[entry(threadIdx.x)];
  }
  for (int i = threadIdx.x; i < nunits; i += NT_INTERP) {
    PtRaw cur;
    if constexpr (GridCfg<T>::PREFETCH_GEOM) {
      cur = nxt;
      if (i + NT_INTERP < nunits) nxt = fetch_point(g, perm, entry(i + NT_INTERP));
    } else {
      cur = point_of(g, pnxt);
      if (i + NT_INTERP < nunits) pnxt = perm[entry(i + NT_INTERP)];
    }
    const int p = cur.p;
    const int p2 = i < nt ? perm[tk.start + 2 * i + 1] : -1;  // the unit's second point
    int first[3];
    double frac[3];
    point_taps<sizeof(T) == 4>(g, cur, J, first, frac);
    T w0r[J], w0i[J], w1r[J], w1i[J], w2r[J], w2i[J];
    axis_weights<T, J, DEG, CW>(P, frac[0], w0r, w0i);
    axis_weights<T, J, DEG, CW>(P, frac[1], w1r, w1i);
    axis_weights<T, J, DEG, CW>(P, frac[2], w2r, w2i);
    const int l0 = first[0] - o0, l1 = first[1] - o1, l2 = first[2] - o2;
    const bool inside = (unsigned)l0 < (unsigned)TILE && (unsigned)l1 < (unsigned)TILE &&
                        (unsigned)l2 < (unsigned)TILE;
    // The host orders each task's points even cells first, so whole waves
    // usually agree on the parity and take a pair-read path.
    cx<T> acc;
    bool done = false;
    if constexpr (sizeof(T) == 4) {
      const bool even = (l2 & 1) == 0;
      if (__all(inside && even)) {
        acc = gather<T, J, S, S2, CW, 1>(tile, grid, K, first, l0, l1, l2, inside, w0r, w0i, w1r,
                                         w1i, w2r, w2i);
        done = true;
      } else if (__all(inside && !even)) {
        acc = gather<T, J, S, S2, CW, 2>(tile, grid, K, first, l0, l1, l2, inside, w0r, w0i, w1r,
                                         w1i, w2r, w2i);
        done = true;
      }
    }
    if (!done)
      acc = gather<T, J, S, S2, CW, 0>(tile, grid, K, first, l0, l1, l2, inside, w0r, w0i, w1r,
                                       w1i, w2r, w2i);
    out[p] = acc;
    if (p2 >= 0) out[p2] = acc;
  }
}

template <typename T, int J, int TILE, bool CW, int DEG>
__global__ __launch_bounds__(GridCfg<T>::NT_INTERP)
__attribute__((amdgpu_waves_per_eu(GridCfg<T>::INTERP_WAVES))) void k_interp(const cx<T>* __restrict__ grid,
                                               cx<T>* __restrict__ out,
                                               const int32_t* __restrict__ perm,
                                               const TileTask* __restrict__ tasks,
                                               XcdSplit xs, PointGeom g,
                                               int nb, WeightPoly<T, DEG> P) {
  interp_body<T, J, TILE, CW, DEG>(blockIdx.x, grid, out, perm, tasks, xs, g, nb, P);
}

// One contribution u (already on the fixed-point scale when FIXED) to halo
// cell `cell` of the task's LDS accumulators: FP32 packs the rounded
// components into one 64-bit word (q_re 2^32 + q_im, the high half less the
// borrow of a negative q_im); FP64 fixed point adds each rounded component
// to its own 64-bit word; FP64 floating point adds to planar accumulators.
template <typename T, int SS, bool FIXED>
__device__ __forceinline__ void add_cell(unsigned long long* accp, double* acc, int cell, cx<T> u) {
  if constexpr (sizeof(T) == 4) {
    const int qr = round_int(u.x), qi = round_int(u.y);
    const unsigned int hi = (unsigned int)qr + (unsigned int)(qi >> 31);
    lds_add(&accp[cell], ((unsigned long long)hi << 32) | (unsigned int)qi);
  } else if constexpr (FIXED) {
    lds_add(&accp[cell], (unsigned long long)(long long)rint((double)u.x));
    lds_add(&accp[SS + cell], (unsigned long long)(long long)rint((double)u.y));
  } else {
    lds_add(&acc[cell], (double)u.x);
    lds_add(&acc[SS + cell], (double)u.y);
  }
}

// The J^3 contributions of one point (value v, tap (0,0,0) at halo cell
// `base`), with conj(w) for the transpose.
template <typename T, int J, int S, int SS, bool CW, bool FIXED>
__device__ __forceinline__ void spread_one(unsigned long long* accp, double* acc, cx<T> v, int base,
                                           const T (&w0r)[J], const T (&w0i)[J],
                                           const T (&w1r)[J], const T (&w1i)[J],
                                           const T (&w2r)[J], const T (&w2i)[J]) {
#pragma unroll
  for (int a = 0; a < J; ++a) {
    const cx<T> va = CW ? cmulc(v, cx<T>{w0r[a], w0i[a]}) : cx<T>{w0r[a] * v.x, w0r[a] * v.y};
#pragma unroll
    for (int b = 0; b < J; ++b) {
      const cx<T> vb =
          CW ? cmulc(va, cx<T>{w1r[b], w1i[b]}) : cx<T>{w1r[b] * va.x, w1r[b] * va.y};
      const int row = base + (a * S + b) * S;
#pragma unroll
      for (int c = 0; c < J; ++c) {
        const cx<T> u =
            CW ? cmulc(vb, cx<T>{w2r[c], w2i[c]}) : cx<T>{w2r[c] * vb.x, w2r[c] * vb.y};
        add_cell<T, SS, FIXED>(accp, acc, row + c, u);
      }
    }
  }
}

// Two points with the same first tap cell and real weights w and x: each of
// the J^3 cells receives w v + x v2 in one atomic.
template <typename T, int J, int S, int SS, bool FIXED>
__device__ __forceinline__ void spread_pair(unsigned long long* accp, double* acc, cx<T> v,
                                            cx<T> v2, int base, const T (&w0r)[J],
                                            const T (&w1r)[J], const T (&w2r)[J],
                                            const T (&x0r)[J], const T (&x1r)[J],
                                            const T (&x2r)[J]) {
#pragma unroll
  for (int a = 0; a < J; ++a) {
    const cx<T> va = {w0r[a] * v.x, w0r[a] * v.y}, xa = {x0r[a] * v2.x, x0r[a] * v2.y};
#pragma unroll
    for (int b = 0; b < J; ++b) {
      const cx<T> vb = {w1r[b] * va.x, w1r[b] * va.y}, xb = {x1r[b] * xa.x, x1r[b] * xa.y};
      const int row = base + (a * S + b) * S;
#pragma unroll
      for (int c = 0; c < J; ++c) {
        const cx<T> u = {w2r[c] * vb.x + x2r[c] * xb.x, w2r[c] * vb.y + x2r[c] * xb.y};
        add_cell<T, SS, FIXED>(accp, acc, row + c, u);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Spreading, phase 1: one workgroup per task accumulates all J^3 taps of its
// points into the task's halo tile (S^3 cells, S = TILE + J - 1) in LDS, then
// writes the halo tile to the task's partial slot with plain stores.  Every
// point is visited once and every tap lands inside the halo.
//
// LDS accumulation (f32 LDS atomic adds run ~8x slower than 64-bit ones on
// gfx950), fixed point in integers, order-independent and so bitwise
// reproducible:
//   FP32 path: both components in one 64-bit word.  With the task's scale
//     s = 2^30 / (vmax B) (2^29 for complex weights), vmax the largest
//     component of the task's values and B the plan-time bound on
//     sum_points prod_axes |w| at any cell of the halo (k_spread_bound),
//     every cell's sums of the rounded contributions q = floor(s u + 1/2)
//     stay inside [-2^31, 2^31).  Each tap adds the word q_re 2^32 + q_im
//     (two's complement) with one ds_add_u64; the low half of a sum is the
//     sum of q_im and the rest the sum of q_re, the carries between them being
//     exact.  The per-contribution error is <= 0.5 / s.
//   FP64 form, deterministic mode: one 64-bit word per component, scale
//     2^62 / (vmax B) (2^61 for complex weights), one ds_add_u64 each.
//   FP64 form, default: FP64 atomic adds (ds_add_f64) on planar real /
//     imaginary accumulators (order-dependent rounding).
// The fixed-point kernels run in two passes.  The main kernel spreads every
// task whose values need nothing more than that single scale; a task whose
// non-zero magnitudes span 2^CLASS_BITS or more, whose scale is not a normal
// number (magnitudes near the ends of the range), or that holds a NaN or an
// infinity goes on a list, and a second kernel spreads the listed tasks in
// full:
//   Magnitude classes: the error bound follows the largest magnitude that
//     shares the scale, so such a task is spread in several passes, one per
//     class of binades (each class holds the occupied binades within
//     CLASS_BITS of its top) with its own scale 2^-c f (2^c the class's bound,
//     applied exactly with ldexp, so tiny and huge magnitudes keep their
//     precision); the passes after the first add their decoded sums to the
//     partial.  A value's contributions are then accurate to
//     <= 2^(CLASS_BITS - 31) B times twice its own magnitude.
//   Non-finite values take no part in the integer sums; the cells of their
//     J^3 footprints are flagged and written as NaN.
constexpr int CLASS_BITS = 16;
constexpr int MAX_CLASSES = 96;  // finite non-zero doubles span 2098 binades: 175 classes at most
                                 // of which the class list keeps the top 96 (floats need 22)

template <typename T>
struct Mag;
template <>
struct Mag<float> {  // magnitudes of FP32 values by their bit patterns
  using U = unsigned;
  static constexpr float MAXV = 3.402823466e38f;
  static constexpr int EXP_OFF = 126, EXP_WORDS = 8;  // exponents [-126, 128]
  static constexpr double RANGE = 1073741824.0;        // 2^30
  // binary exponent e with a < 2^e (a in [2^(e-1), 2^e) for normal values;
  // denormals and zero give the smallest binade's bound)
  __device__ static int exp_of(float a) { return (int)(__float_as_uint(a) >> 23) - 126; }
  __device__ static U bits(float a) { return __float_as_uint(a); }
  __device__ static float from(U b) { return __uint_as_float(b); }
  __device__ static float ldexp2(float x, int e) { return ldexpf(x, e); }  // exact
  static constexpr U NONE = 0xffffffffu;
};
template <>
struct Mag<double> {
  using U = unsigned long long;
  static constexpr double MAXV = 1.7976931348623157e308;
  static constexpr int EXP_OFF = 1022, EXP_WORDS = 64;  // exponents [-1022, 1024]
  static constexpr double RANGE = 4611686018427387904.0;  // 2^62
  __device__ static int exp_of(double a) {
    return (int)(__double_as_longlong(a) >> 52) - 1022;
  }
  __device__ static U bits(double a) { return (U)__double_as_longlong(a); }
  __device__ static double from(U b) { return __longlong_as_double((long long)b); }
  __device__ static double ldexp2(double x, int e) { return ldexp(x, e); }
  static constexpr U NONE = ~0ull;
};

template <int J, int S>
__device__ __forceinline__ void flag_footprint(unsigned* flags, int base) {
  for (int a = 0; a < J; ++a)
    for (int b = 0; b < J; ++b)
      for (int c = 0; c < J; ++c) {
        const int cell = base + (a * S + b) * S + c;
        atomicOr(&flags[cell >> 5], 1u << (cell & 31));
      }
}

// The spreading of one task.  FIXED: integer accumulation (FP32 always, FP64
// in deterministic mode).  REST = false (main kernel): tasks that one scale
// serves; the others append their id to mlist (count in mlist[0], ids after
// it) and return.  REST = true: a listed task in full.  The two are separate
// kernels so that the general multi-pass code costs the usual single pass no
// registers.
template <typename T, int J, int TILE, bool CW, int DEG, bool FIXED, bool REST>
__device__ __forceinline__ void spread_task(int64_t task_id, const cx<T>* __restrict__ in,
                                            cx<T>* __restrict__ partials,
                                            const int32_t* __restrict__ perm,
                                            const TileTask* __restrict__ tasks,
                                            const float* __restrict__ bound,
                                            int32_t* __restrict__ mlist, const PointGeom& g,
                                            int nb, const WeightPoly<T, DEG>& P) {
  constexpr int NT_SPREAD = GridCfg<T>::NT_SPREAD;
  constexpr bool WIDE = sizeof(T) == 8;  // FP64: one word per component
  constexpr int S = TILE + J - 1;
  constexpr int SS = S * S * S;
  constexpr int R = J - 1;
  using MG = Mag<T>;
  using U = typename MG::U;
  // FP32: one packed 64-bit word per cell.  FP64: planar accumulators (all
  // real parts, then all imaginary parts), so that a wave's 64-bit atomics
  // spread over every LDS bank instead of half of them.
  __shared__ double acc[FIXED && !WIDE ? SS : 2 * SS];
  __shared__ unsigned s_nan[FIXED && REST ? (SS + 31) / 32 : 1];
  __shared__ unsigned s_occ[FIXED && REST ? MG::EXP_WORDS : 1];
  __shared__ int s_ctop[FIXED && REST ? MAX_CLASSES : 1];
  __shared__ U s_maxbits, s_minbits;
  __shared__ int s_bad, s_ncls;
  unsigned long long* accp = reinterpret_cast<unsigned long long*>(acc);
  const TileTask tk = tasks[task_id];
  const int b2 = tk.bin % nb, b1 = (tk.bin / nb) % nb, b0 = tk.bin / (nb * nb);
  const int o0 = b0 * TILE, o1 = b1 * TILE, o2 = b2 * TILE;
  for (int idx = threadIdx.x; idx < (FIXED && !WIDE ? SS : 2 * SS); idx += NT_SPREAD) acc[idx] = 0.0;
  // magnitude statistics of the task's values (fixed point)
  T vmax = 0, scale = 1;
  double inv = 1.0, bnd = 1.0;
  int emax = 0, emin = 0, ncls = 1;
  bool bad = false, multi = false;
  if constexpr (FIXED) {
    if constexpr (REST)
      for (int idx = threadIdx.x; idx < (SS + 31) / 32; idx += NT_SPREAD) s_nan[idx] = 0u;
    if (threadIdx.x == 0) {
      s_maxbits = 0;
      s_minbits = MG::NONE;
      s_bad = 0;
    }
    if (REST && threadIdx.x < (REST ? MG::EXP_WORDS : 0)) s_occ[threadIdx.x] = 0u;
    __syncthreads();
    bnd = (double)bound[task_id];
    if constexpr (!REST) {
      // the largest magnitude sets the scale; the smallest non-zero one and
      // the non-finite values are found on the way through the points, and a
      // task that needs more than this one scale is then listed instead of
      // written.  Four points per step
      T m = 0, ssum = 0;  // (ssum is NaN or infinite if a value is, or if it overflows)
      for (int i0 = threadIdx.x; i0 < tk.count; i0 += 4 * NT_SPREAD) {
        int id[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int i = i0 + k * NT_SPREAD;
          id[k] = i < tk.count ? perm[tk.start + i] : -1;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (id[k] >= 0) {
            const cx<T> v = in[id[k]];
            m = fmax(m, fmax(fabs(v.x), fabs(v.y)));  // (NaN operands are ignored)
            ssum += fabs(v.x) + fabs(v.y);
          }
      }
      if (!(ssum <= (T)MG::MAXV)) s_bad = 1;
      if constexpr (WIDE)
        __hip_atomic_fetch_max(&s_maxbits, MG::bits(m), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      else
        atomicMax(&s_maxbits, MG::bits(m));
      __syncthreads();
      vmax = MG::from(s_maxbits);
      emax = vmax > (T)0 ? MG::exp_of(vmax) : 0;
      // one scale for the whole task, a normal number, and finite values: else
      // the task is listed
      const double sd = vmax > (T)0 && bnd > 0.0 ? (CW ? 0.5 : 1.0) * MG::RANGE / ((double)vmax * bnd) : 1.0;
      if (s_bad || !(sd >= (sizeof(T) == 4 ? 1.17549435e-38 : 2.2250738585072014e-308) && sd <= (double)MG::MAXV)) {
        if (threadIdx.x == 0) mlist[1 + atomicAdd(&mlist[0], 1)] = (int32_t)task_id;
        return;
      }
      scale = (T)sd;
    } else {
      U mx = 0, mn = MG::NONE;  // bits of the largest and smallest non-zero magnitudes
      bool nf = false;
      // SC points per step, every load issued unconditionally (lanes past the
      // end reload the step's first point and ignore it)
      constexpr int SC = 8;
      for (int i0 = threadIdx.x; i0 < tk.count; i0 += SC * NT_SPREAD) {
        int id[SC];
#pragma unroll
        for (int k = 0; k < SC; ++k) {
          const int i = i0 + k * NT_SPREAD;
          id[k] = perm[tk.start + (i < tk.count ? i : i0)];
        }
        cx<T> v[SC];
#pragma unroll
        for (int k = 0; k < SC; ++k) v[k] = in[id[k]];
#pragma unroll
        for (int k = 0; k < SC; ++k) {
          const bool ok = i0 + k * NT_SPREAD < tk.count;
          const T ax = fabs(v[k].x), ay = fabs(v[k].y), a = ax > ay ? ax : ay;
          const bool fin = ax <= (T)MG::MAXV && ay <= (T)MG::MAXV;  // false for NaN and infinities
          nf = nf || (ok && !fin);
          const bool pos = ok && fin && a > (T)0;
          const U ab = MG::bits(a);  // non-negative values order like their bit patterns
          mx = pos && ab > mx ? ab : mx;
          mn = pos && ab < mn ? ab : mn;
        }
      }
      if constexpr (WIDE) {
        __hip_atomic_fetch_max(&s_maxbits, mx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_fetch_min(&s_minbits, mn, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      } else {
        atomicMax(&s_maxbits, mx);
        atomicMin(&s_minbits, mn);
      }
      if (nf) s_bad = 1;
      __syncthreads();
      vmax = MG::from(s_maxbits);
      bad = s_bad != 0;
      emax = vmax > (T)0 ? MG::exp_of(vmax) : 0;
      emin = vmax > (T)0 ? MG::exp_of(MG::from(s_minbits)) : 0;
      multi = vmax > (T)0 && emax - emin >= CLASS_BITS;
      // the occupied binades, then the classes: each starts at the highest
      // occupied binade below the previous class and spans CLASS_BITS of them
      for (int i0 = threadIdx.x; i0 < tk.count; i0 += NT_SPREAD) {
        const cx<T> v = in[perm[tk.start + i0]];
        const T a = fabs(v.x) > fabs(v.y) ? fabs(v.x) : fabs(v.y);
        if (a > (T)0 && a <= (T)MG::MAXV) {
          const int e = MG::exp_of(a) + MG::EXP_OFF;
          atomicOr(&s_occ[e >> 5], 1u << (e & 31));
        }
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        int n = 0, e = emax;
        while (vmax > (T)0 && e >= emin && n < MAX_CLASSES) {
          s_ctop[n++] = e;
          e -= CLASS_BITS;
          while (e >= emin && !((s_occ[(e + MG::EXP_OFF) >> 5] >> ((e + MG::EXP_OFF) & 31)) & 1u)) --e;
        }
        s_ncls = n > 0 ? n : 1;
        if (n == 0) s_ctop[0] = 0;
      }
      __syncthreads();
      ncls = s_ncls;
    }
  } else {
    __syncthreads();
  }
  // units: a pair of points that share their first tap cell (entries 2u and
  // 2u + 1, u < npairs), then single points (entry npairs + u)
  // FP32 with real weights: both points' contributions to a cell summed
  // before one atomic; otherwise (min-max weights, or FP64, whose register
  // budget it would exceed) the points of a unit are spread one by one.
  // The first ntwins pairs (FP32, either weights) sample one frequency
  // twice: their weights are evaluated once and spread the sum of the two
  // values.
  constexpr bool PAIRED = !CW && sizeof(T) == 4;
  const int np = tk.npairs, nunits = tk.count - np, nt = tk.ntwins;
  cx<T>* dst = partials + task_id * (int64_t)part_stride(TILE, R);
  // no accumulation is needed when every value is zero or non-finite
  const bool work = !FIXED || vmax > (T)0;
  for (int cls = 0; cls < (REST ? ncls : 1); ++cls) {
    // REST: the class's scale, v -> ldexp(v, -ctop) f, and its decoding
    int ctop = 0, clo = 0;
    T f = 1;
    if constexpr (FIXED && REST) {
      if (cls > 0) {
        __syncthreads();  // the previous pass's write-out has read the accumulators
        for (int idx = threadIdx.x; idx < (WIDE ? 2 * SS : SS); idx += NT_SPREAD) acc[idx] = 0.0;
        __syncthreads();
      }
      ctop = s_ctop[cls];
      clo = multi ? ctop - CLASS_BITS : -(1 << 20);
      // class bound / 2^ctop: the exact maximum for the first class
      const double u = cls == 0 ? (double)MG::ldexp2(vmax, -emax) : 1.0;
      if (vmax > (T)0 && bnd > 0.0) {
        f = (T)((CW ? 0.5 : 1.0) * MG::RANGE / (u * bnd));
        inv = ldexp(1.0 / (double)f, ctop);
      }
    }
    // the scaled value: 0 for values of other classes or non-finite ones
    auto prep = [&](cx<T> v) -> cx<T> {
      if constexpr (!FIXED) {
        return v;
      } else if constexpr (!REST) {
        return cx<T>{v.x * scale, v.y * scale};
      } else {
        const T ax = fabs(v.x), ay = fabs(v.y);
        if (!(ax <= (T)MG::MAXV) || !(ay <= (T)MG::MAXV)) return cx<T>{0, 0};
        if (multi) {
          const T a = ax > ay ? ax : ay;
          const int e = a > (T)0 ? MG::exp_of(a) : clo;
          if (e > ctop || e <= clo) return cx<T>{0, 0};
        }
        return cx<T>{MG::ldexp2(v.x, -ctop) * f, MG::ldexp2(v.y, -ctop) * f};
      }
    };
    auto nonfinite = [](cx<T> v) { return !(fabs(v.x) <= (T)MG::MAXV) || !(fabs(v.y) <= (T)MG::MAXV); };
    PtRaw nxt, nxt2;
    cx<T> vnxt = {0, 0}, vnxt2 = {0, 0};
    auto fetch_unit = [&](int u) {  // one unit ahead (its second point if paired)
      const int e = u < np ? 2 * u : np + u;
      nxt = fetch_point(g, perm, tk.start + e);
      vnxt = in[nxt.p];
      vnxt2 = cx<T>{0, 0};
      if (sizeof(T) == 4 && u < nt) {
        nxt2.p = perm[tk.start + e + 1];  // (a twin's geometry is the first point's)
        vnxt2 = in[nxt2.p];
      } else if (PAIRED && u < np) {
        nxt2 = fetch_point(g, perm, tk.start + e + 1);
        vnxt2 = in[nxt2.p];
      }
    };
    const bool go = work || (REST && bad);
    T tmn = (T)INFINITY;  // main kernel: the smallest non-zero magnitude
    cx<T> vs1 = {0, 0}, vs2 = {0, 0};
    if (go && (int)threadIdx.x < nunits) fetch_unit(threadIdx.x);
    for (int u = threadIdx.x; go && u < nunits; u += NT_SPREAD) {
      PtRaw cur = nxt, cur2 = nxt2;
      cx<T> v = vnxt, v2 = vnxt2;
      const bool pair = u < np;
      const bool twin = sizeof(T) == 4 && u < nt;
      if (u + NT_SPREAD < nunits) fetch_unit(u + NT_SPREAD);
      if (!PAIRED && pair && !twin) {
        cur2 = fetch_point(g, perm, tk.start + 2 * u + 1);
        v2 = in[cur2.p];
      }
      // (the flags are set once, in the first class's pass)
      const bool bad1 = FIXED && REST && bad && cls == 0 && nonfinite(v);
      const bool bad2 = FIXED && REST && bad && cls == 0 && pair && nonfinite(v2);
      if constexpr (FIXED && !REST) {
        // the smallest non-zero magnitude and the non-finite values, from the
        // scaled values (the second point of a unit is zero when there is
        // none); taken here rather than on arrival, where waiting for the
        // prefetched values would expose their latency
        vs1 = v;
        vs2 = v2;
      }
      v = prep(v);
      v2 = prep(v2);
      if constexpr (FIXED && REST) {
        // nothing to add (values of other classes) and nothing to flag
        const bool nz = v.x != (T)0 || v.y != (T)0 || (pair && (v2.x != (T)0 || v2.y != (T)0));
        if (!nz && !bad1 && !bad2) continue;
      }
      int first[3], first2[3] = {0, 0, 0};
      double frac[3], frac2[3] = {0.0, 0.0, 0.0};
      point_taps<sizeof(T) == 4>(g, cur, J, first, frac);
      const int l0 = first[0] - o0, l1 = first[1] - o1, l2 = first[2] - o2;
      // the host bins with the same FP64 arithmetic, so every point of the task
      // lies in its tile; the check only keeps LDS accesses in bounds
      const bool in1 = (unsigned)l0 < (unsigned)TILE && (unsigned)l1 < (unsigned)TILE &&
                       (unsigned)l2 < (unsigned)TILE;
      T w0r[J], w0i[J], w1r[J], w1i[J], w2r[J], w2i[J];
      axis_weights<T, J, DEG, CW>(P, frac[0], w0r, w0i);
      axis_weights<T, J, DEG, CW>(P, frac[1], w1r, w1i);
      axis_weights<T, J, DEG, CW>(P, frac[2], w2r, w2i);
      bool same = true;  // the second point shares the first tap cell
      if (twin) {
        // the host found both points in one cell with FP64 frequencies that
        // agree to 1e-12, far below the FP32 weights' resolution
#pragma unroll
        for (int d = 0; d < 3; ++d) first2[d] = first[d];
      } else if (pair) {
        point_taps<sizeof(T) == 4>(g, cur2, J, first2, frac2);
        same = first2[0] == first[0] && first2[1] == first[1] && first2[2] == first[2];
      }
      if constexpr (FIXED && REST) {
        const int m0 = first2[0] - o0, m1 = first2[1] - o1, m2 = first2[2] - o2;
        if (bad1 && in1) flag_footprint<J, S>(s_nan, (l0 * S + l1) * S + l2);
        if (bad2 && (unsigned)m0 < (unsigned)TILE && (unsigned)m1 < (unsigned)TILE &&
            (unsigned)m2 < (unsigned)TILE)
          flag_footprint<J, S>(s_nan, (m0 * S + m1) * S + m2);
      }
      if constexpr (FIXED && !REST) {
        // (the values are finite here; zeros are left out by mapping them to +inf)
        const T a1 = fmax(fabs(vs1.x), fabs(vs1.y)), a2 = fmax(fabs(vs2.x), fabs(vs2.y));
        tmn = fmin(tmn, fmin(a1 > (T)0 ? a1 : (T)INFINITY, a2 > (T)0 ? a2 : (T)INFINITY));
      }
      if (twin) {
        const cx<T> vs = {v.x + v2.x, v.y + v2.y};
        if (in1)
          spread_one<T, J, S, SS, CW, FIXED>(accp, acc, vs, (l0 * S + l1) * S + l2, w0r, w0i,
                                             w1r, w1i, w2r, w2i);
      } else if constexpr (PAIRED) {
        // (a single point, or a pair whose first cells differ, adds a zero here)
        T x0r[J], x0i[J], x1r[J], x1i[J], x2r[J], x2i[J];
        const bool both = pair && same;
        axis_weights<T, J, DEG, CW>(P, both ? frac2[0] : frac[0], x0r, x0i);
        axis_weights<T, J, DEG, CW>(P, both ? frac2[1] : frac[1], x1r, x1i);
        axis_weights<T, J, DEG, CW>(P, both ? frac2[2] : frac[2], x2r, x2i);
        const cx<T> vq = both ? v2 : cx<T>{0, 0};
        if (in1)
          spread_pair<T, J, S, SS, FIXED>(accp, acc, v, vq, (l0 * S + l1) * S + l2, w0r, w1r, w2r,
                                          x0r, x1r, x2r);
      } else {
        if (in1)
          spread_one<T, J, S, SS, CW, FIXED>(accp, acc, v, (l0 * S + l1) * S + l2, w0r, w0i, w1r,
                                             w1i, w2r, w2i);
      }
      if (pair && !twin && (!PAIRED || !same)) {
        // the second point on its own (or first cells that differ in the
        // device's rounding of a tie)
        const int m0 = first2[0] - o0, m1 = first2[1] - o1, m2 = first2[2] - o2;
        if ((unsigned)m0 < (unsigned)TILE && (unsigned)m1 < (unsigned)TILE &&
            (unsigned)m2 < (unsigned)TILE) {
          axis_weights<T, J, DEG, CW>(P, frac2[0], w0r, w0i);
          axis_weights<T, J, DEG, CW>(P, frac2[1], w1r, w1i);
          axis_weights<T, J, DEG, CW>(P, frac2[2], w2r, w2i);
          spread_one<T, J, S, SS, CW, FIXED>(accp, acc, v2, (m0 * S + m1) * S + m2, w0r, w0i, w1r,
                                             w1i, w2r, w2i);
        }
      }
    }
    if constexpr (FIXED && !REST) {
      // a task that needs more than one scale goes to the general kernel
      const U tmb = tmn <= (T)MG::MAXV ? MG::bits(tmn) : MG::NONE;
      if constexpr (WIDE)
        __hip_atomic_fetch_min(&s_minbits, tmb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      else
        atomicMin(&s_minbits, tmb);
      __syncthreads();
      const U mnb = s_minbits;
      const bool wide_range = mnb != MG::NONE && vmax > (T)0 && emax - MG::exp_of(MG::from(mnb)) >= CLASS_BITS;
      if (wide_range) {
        if (threadIdx.x == 0) mlist[1 + atomicAdd(&mlist[0], 1)] = (int32_t)task_id;
        return;
      }
    }
    __syncthreads();
    // write the partial block by block (consecutive threads, consecutive
    // addresses), see part_offset; further classes add to what the first wrote
    const bool add = REST && cls > 0;
    if constexpr (FIXED && !REST) inv = 1.0 / (double)scale;  // (not live across the loop)
    auto decode = [&](int cell) -> cx<T> {  // the two sums of a cell
      cx<T> r;
      if constexpr (!FIXED) {
        r = cx<T>{(T)acc[cell], (T)acc[SS + cell]};
      } else if constexpr (WIDE) {
        r = cx<T>{(T)((double)(long long)accp[cell] * inv), (T)((double)(long long)accp[SS + cell] * inv)};
      } else {
        const unsigned long long w = accp[cell];
        const long long lo = (long long)(int)(unsigned int)(w & 0xffffffffull);
        const long long hi = (long long)(w - (unsigned long long)lo) >> 32;
        r = cx<T>{(T)((double)hi * inv), (T)((double)lo * inv)};
      }
      if constexpr (FIXED && REST)
        if (bad && ((s_nan[cell >> 5] >> (cell & 31)) & 1u)) r = cx<T>{(T)NAN, (T)NAN};
      return r;
    };
#pragma unroll
    for (int delta = 0; delta < 8; ++delta) {
      const int d0 = (delta >> 2) & 1, d1 = (delta >> 1) & 1, d2 = delta & 1;
      const int e1 = part_ext(d1, TILE, R), e2 = part_ext(d2, TILE, R);
      const int n = part_size(delta, TILE, R), base = part_base(delta, TILE, R);
      if constexpr (FIXED && !WIDE) {
        // blocks whose rows have an even length (and an even base): two cells
        // of a row per lane, one 16-byte store
        if ((e2 & 1) == 0) {
          constexpr int NTS2 = NT_SPREAD;
#pragma unroll
          for (int k = 0; k < (part_size(delta, TILE, R) / 2 + NTS2 - 1) / NTS2; ++k) {
            const int j = (int)threadIdx.x + k * NTS2;
            if (j < n / 2) {
              const int idx = 2 * j;
              const int r2 = idx % e2, r1 = (idx / e2) % e1, r0 = idx / (e1 * e2);
              const int cell = ((r0 + d0 * TILE) * S + (r1 + d1 * TILE)) * S + (r2 + d2 * TILE);
              const cx<T> a = decode(cell), b = decode(cell + 1);
              float4 o = make_float4(a.x, a.y, b.x, b.y);
              float4* q = reinterpret_cast<float4*>(dst + base) + j;
              if (add) {
                const float4 p = *q;
                o = make_float4(p.x + o.x, p.y + o.y, p.z + o.z, p.w + o.w);
              }
              *q = o;
            }
          }
          continue;
        }
      }
      for (int idx = threadIdx.x; idx < n; idx += NT_SPREAD) {
        const int r2 = idx % e2, r1 = (idx / e2) % e1, r0 = idx / (e1 * e2);
        const int cell = ((r0 + d0 * TILE) * S + (r1 + d1 * TILE)) * S + (r2 + d2 * TILE);
        cx<T> v = decode(cell);
        if (add) v = cadd(v, dst[base + idx]);
        dst[base + idx] = v;
      }
    }
  }
}

template <typename T, int J, int TILE, bool CW, int DEG, bool FIXED>
__global__ __launch_bounds__(GridCfg<T>::NT_SPREAD)
__attribute__((amdgpu_waves_per_eu(GridCfg<T>::SPREAD_WAVES))) void k_spread(
    const cx<T>* __restrict__ in, cx<T>* __restrict__ partials, const int32_t* __restrict__ perm,
    const TileTask* __restrict__ tasks, const int32_t* __restrict__ torder,
    const float* __restrict__ bound, int32_t* __restrict__ mlist, XcdSplit xs, PointGeom g,
    int nb, WeightPoly<T, DEG> P) {
  int64_t task_id = xcd_task(blockIdx.x, xs);
  if (task_id < 0) return;
  if (torder) task_id = torder[task_id];  // largest tasks of each XCD range first
  spread_task<T, J, TILE, CW, DEG, FIXED, false>(task_id, in, partials, perm, tasks, bound, mlist,
                                                 g, nb, P);
}

// Fixed point: the listed tasks in full (a few blocks walk the list, so that
// the usual empty list costs one small launch)
constexpr int NB_REST = 512;
template <typename T, int J, int TILE, bool CW, int DEG>
__global__ __launch_bounds__(GridCfg<T>::NT_SPREAD) void k_spread_rest(
    const cx<T>* __restrict__ in, cx<T>* __restrict__ partials, const int32_t* __restrict__ perm,
    const TileTask* __restrict__ tasks, const float* __restrict__ bound,
    int32_t* __restrict__ mlist, PointGeom g, int nb, WeightPoly<T, DEG> P) {
  const int count = mlist[0];
  for (int i = blockIdx.x; i < count; i += gridDim.x) {
    spread_task<T, J, TILE, CW, DEG, true, true>(mlist[1 + i], in, partials, perm, tasks, bound,
                                                 mlist, g, nb, P);
    __syncthreads();  // the next task reuses the LDS
  }
}

// Plan-time bound for the FP32 spreading scale: per task, the largest over
// its halo cells of sum_points prod_axes |w_axis| (the weights the spreading
// evaluates), accumulated exactly in 2^-32 units with every term rounded up,
// then rounded up to float.
template <typename T, int J, int TILE, bool CW, int DEG>
__global__ __launch_bounds__(NT_BOUND) void k_spread_bound(float* __restrict__ bound,
                                                            const int32_t* __restrict__ perm,
                                                            const TileTask* __restrict__ tasks,
                                                            XcdSplit xs, PointGeom g, int nb,
                                                            WeightPoly<T, DEG> P) {
  constexpr int S = TILE + J - 1;
  constexpr int SS = S * S * S;
  __shared__ unsigned long long acc[SS];
  __shared__ unsigned long long s_max;
  const int64_t task_id = xcd_task(blockIdx.x, xs);
  if (task_id < 0) return;
  const TileTask tk = tasks[task_id];
  const int b2 = tk.bin % nb, b1 = (tk.bin / nb) % nb, b0 = tk.bin / (nb * nb);
  const int o0 = b0 * TILE, o1 = b1 * TILE, o2 = b2 * TILE;
  for (int idx = threadIdx.x; idx < SS; idx += NT_BOUND) acc[idx] = 0ull;
  if (threadIdx.x == 0) s_max = 0ull;
  __syncthreads();
  for (int i = threadIdx.x; i < tk.count; i += NT_BOUND) {
    const PtRaw cur = fetch_point(g, perm, tk.start + i);
    int first[3];
    double frac[3];
    point_taps<sizeof(T) == 4>(g, cur, J, first, frac);
    const int l0 = first[0] - o0, l1 = first[1] - o1, l2 = first[2] - o2;
    if ((unsigned)l0 >= (unsigned)TILE || (unsigned)l1 >= (unsigned)TILE ||
        (unsigned)l2 >= (unsigned)TILE)
      continue;
    T w0r[J], w0i[J], w1r[J], w1i[J], w2r[J], w2i[J];
    axis_weights<T, J, DEG, CW>(P, frac[0], w0r, w0i);
    axis_weights<T, J, DEG, CW>(P, frac[1], w1r, w1i);
    axis_weights<T, J, DEG, CW>(P, frac[2], w2r, w2i);
    double m0[J], m1[J], m2[J];
#pragma unroll
    for (int a = 0; a < J; ++a) {
      m0[a] = sqrt((double)w0r[a] * w0r[a] + (double)w0i[a] * w0i[a]);
      m1[a] = sqrt((double)w1r[a] * w1r[a] + (double)w1i[a] * w1i[a]);
      m2[a] = sqrt((double)w2r[a] * w2r[a] + (double)w2i[a] * w2i[a]);
    }
    for (int a = 0; a < J; ++a)
      for (int b = 0; b < J; ++b) {
        const int row = ((l0 + a) * S + (l1 + b)) * S + l2;
        const double mab = m0[a] * m1[b] * 4294967296.0;  // 2^32
#pragma unroll
        for (int c = 0; c < J; ++c)
          lds_add(&acc[row + c], (unsigned long long)ceil(mab * m2[c] * (1.0 + 1e-12)));
      }
  }
  __syncthreads();
  unsigned long long m = 0ull;
  for (int idx = threadIdx.x; idx < SS; idx += NT_BOUND) m = acc[idx] > m ? acc[idx] : m;
  __hip_atomic_fetch_max(&s_max, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  __syncthreads();
  if (threadIdx.x == 0) {
    const double b = (double)s_max * (1.0 / 4294967296.0) * (1.0 + 1e-6);
    bound[task_id] = __double2float_ru(b);
  }
}

// Spreading, phase 2 (owner computes): each grid cell is the fixed-order sum
// of the halo partials that cover it -- those of every task of its own bin and
// of the lower-neighbour bins whose halos reach it (J-1 cells into the tile).
// One workgroup per tile and one thread per cell: the 8 source bins' task
// ranges are read once per workgroup into LDS, then every cell issues its
// (mostly single) partial loads independently.  With the block layout of the
// partials, the cells of a row read consecutive words of each block.
template <typename T, int TILE>
__device__ __forceinline__ void merge_body(int bx, const cx<T>* __restrict__ partials,
                                           const int32_t* __restrict__ bin_tasks,
                                           const int32_t* __restrict__ order,
                                           cx<T>* __restrict__ grid, int nb, int K, int R,
                                           double r2, int32_t* __restrict__ mlist) {
  // the spreading's list of multi-class tasks has been consumed: empty it
  if (mlist && bx == 0 && threadIdx.x == 0) mlist[0] = 0;
  constexpr int TT = TILE * TILE * TILE;
  constexpr int NTM = TT < 1024 ? TT : 1024;
  constexpr int PER = TT / NTM;
  const int64_t PS = part_stride(TILE, R);
  const int tile = order[bx];
  const int t2 = tile % nb, t1 = (tile / nb) % nb, t0 = tile / (nb * nb);
  {
    // tiles wholly outside the ball holding every tap are never read
    double d2 = 0.0;
    const int ts[3] = {t0, t1, t2};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int lo = ts[d] * TILE - K / 2, hi = lo + TILE - 1;
      const double c = lo > 0 ? (double)lo : (hi < 0 ? (double)(-hi) : 0.0);
      d2 += c * c;
    }
    if (d2 > r2) return;
  }
  __shared__ int rng[16];
  if (threadIdx.x < 8) {
    const int delta = threadIdx.x;
    const int d0 = (delta >> 2) & 1, d1 = (delta >> 1) & 1, d2 = delta & 1;
    const int sb = (((t0 - d0 + nb) % nb) * nb + (t1 - d1 + nb) % nb) * nb + (t2 - d2 + nb) % nb;
    rng[2 * delta] = bin_tasks[sb];
    rng[2 * delta + 1] = bin_tasks[sb + 1];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int idx = (int)threadIdx.x + k * NTM;
    const int i2 = idx % TILE, i1 = (idx / TILE) % TILE, i0 = idx / (TILE * TILE);
    cx<T> acc = {0, 0};
    // the first task of every source bin that reaches this cell: up to eight
    // independent loads (lanes that miss a source do not load, and a wave
    // whose lanes all miss skips it), then the further tasks of the bins that
    // have several; a fixed order
    int64_t off[8];
    bool hit[8];
#pragma unroll
    for (int delta = 0; delta < 8; ++delta) {
      const int d0 = (delta >> 2) & 1, d1 = (delta >> 1) & 1, d2 = delta & 1;
      // block delta of bin (tile - delta) covers cells [0,e0) x [0,e1) x [0,e2)
      const int e0 = part_ext(d0, TILE, R), e1 = part_ext(d1, TILE, R), e2 = part_ext(d2, TILE, R);
      hit[delta] = i0 < e0 && i1 < e1 && i2 < e2 && rng[2 * delta] < rng[2 * delta + 1];
      off[delta] = part_base(delta, TILE, R) + (i0 * e1 + i1) * e2 + i2;
    }
    cx<T> first[8];
#pragma unroll
    for (int delta = 0; delta < 8; ++delta) {
      first[delta] = cx<T>{0, 0};
      if (hit[delta]) first[delta] = partials[rng[2 * delta] * PS + off[delta]];
    }
#pragma unroll
    for (int delta = 0; delta < 8; ++delta)
      if (hit[delta]) acc = cadd(acc, first[delta]);
#pragma unroll
    for (int delta = 0; delta < 8; ++delta)
      if (hit[delta])
        for (int t = rng[2 * delta] + 1; t < rng[2 * delta + 1]; ++t)
          acc = cadd(acc, partials[t * PS + off[delta]]);
    grid[(int64_t)(t0 * TILE + i0) * grid_plane_of<T>(K) + (int64_t)(t1 * TILE + i1) * K +
         (t2 * TILE + i2)] = acc;
  }
}

template <typename T, int TILE>
__global__ __launch_bounds__(TILE * TILE * TILE < 1024 ? TILE * TILE * TILE : 1024) void k_merge(
    const cx<T>* __restrict__ partials, const int32_t* __restrict__ bin_tasks,
    const int32_t* __restrict__ order, cx<T>* __restrict__ grid, int nb, int K, int R, double r2,
    int32_t* __restrict__ mlist) {
  merge_body<T, TILE>(blockIdx.x, partials, bin_tasks, order, grid, nb, K, R, r2, mlist);
}

// FP32 merge with C adjacent cells (C = 2 or 4; i2 a multiple of C) per
// thread: the blocks whose rows are TILE long are read and the grid written
// in 16-byte pairs (part_base offsets and the per-task stride are even), the
// short-row blocks one value at a time; the per-cell summation order is the
// one of k_merge.
// Its arguments: one plan's (MergeArgs) or, in a batch, those of the
// volume a block belongs to (the argument type resolves them from the block
// index); the body is the kernel's own, so that the one-plan kernel compiles
// as a plain kernel.
struct MergeArgs {
  const cx<float>* partials;
  const int32_t* bin_tasks;
  const int32_t* order;
  cx<float>* grid;
  int nb, K, R;
  double r2;
  int32_t* mlist;
  __device__ __forceinline__ MergeArgs resolve(unsigned b, unsigned& bx) const {
    bx = b;
    return *this;
  }
};

template <int TILE, int C, typename A>
__global__ __launch_bounds__(1024) void k_merge_pairs(A args) {
  unsigned bx;
  const MergeArgs a = args.resolve(blockIdx.x, bx);
  const cx<float>* __restrict__ partials = a.partials;
  const int32_t* __restrict__ bin_tasks = a.bin_tasks;
  const int32_t* __restrict__ order = a.order;
  cx<float>* __restrict__ grid = a.grid;
  const int nb = a.nb, K = a.K, R = a.R;
  const double r2 = a.r2;
  int32_t* __restrict__ mlist = a.mlist;
  // the spreading's list of multi-class tasks has been consumed: empty it
  if (mlist && bx == 0 && threadIdx.x == 0) mlist[0] = 0;
  constexpr int TTC = TILE * TILE * TILE / C;
  constexpr int NTM = TTC < 1024 ? TTC : 1024;
  constexpr int PER = TTC / NTM;
  const int64_t PS = part_stride(TILE, R);
  const int tile = order[bx];
  const int t2 = tile % nb, t1 = (tile / nb) % nb, t0 = tile / (nb * nb);
  {
    double d2 = 0.0;
    const int ts[3] = {t0, t1, t2};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int lo = ts[d] * TILE - K / 2, hi = lo + TILE - 1;
      const double c = lo > 0 ? (double)lo : (hi < 0 ? (double)(-hi) : 0.0);
      d2 += c * c;
    }
    if (d2 > r2) return;
  }
  __shared__ int rng[16];
  if (threadIdx.x < 8) {
    const int delta = threadIdx.x;
    const int d0 = (delta >> 2) & 1, d1 = (delta >> 1) & 1, d2 = delta & 1;
    const int sb = (((t0 - d0 + nb) % nb) * nb + (t1 - d1 + nb) % nb) * nb + (t2 - d2 + nb) % nb;
    rng[2 * delta] = bin_tasks[sb];
    rng[2 * delta + 1] = bin_tasks[sb + 1];
  }
  __syncthreads();
  const float4* p4 = reinterpret_cast<const float4*>(partials);
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int idx = (int)threadIdx.x + k * NTM;
    const int i2 = C * (idx % (TILE / C)), i1 = (idx / (TILE / C)) % TILE;
    const int i0 = idx / (TILE * TILE / C);
    cx<float> acc[C];
#pragma unroll
    for (int q = 0; q < C; ++q) acc[q] = cx<float>{0, 0};
    int64_t off[8];
    bool any[8];
    int e2s[8];
#pragma unroll
    for (int delta = 0; delta < 8; ++delta) {
      const int d0 = (delta >> 2) & 1, d1 = (delta >> 1) & 1, d2 = delta & 1;
      const int e0 = part_ext(d0, TILE, R), e1 = part_ext(d1, TILE, R), e2 = part_ext(d2, TILE, R);
      any[delta] = i0 < e0 && i1 < e1 && i2 < e2 && rng[2 * delta] < rng[2 * delta + 1];
      e2s[delta] = e2;
      off[delta] = part_base(delta, TILE, R) + (i0 * e1 + i1) * e2 + i2;
    }
    // every load is issued unconditionally (masked-off lanes read element 0
    // and drop it), so that all of them are in flight together: loads under
    // divergent branches are waited for where the branches join
    cx<float> f[8][C];
#pragma unroll
    for (int delta = 0; delta < 8; ++delta) {
      const int64_t o = any[delta] ? rng[2 * delta] * PS + off[delta] : 0;
      if ((delta & 1) == 0) {  // rows of TILE cells: 16-byte reads of cell pairs
#pragma unroll
        for (int q = 0; q < C; q += 2) {
          const float4 v = p4[(o + q) >> 1];
          f[delta][q] = any[delta] ? cx<float>{v.x, v.y} : cx<float>{0, 0};
          f[delta][q + 1] = any[delta] ? cx<float>{v.z, v.w} : cx<float>{0, 0};
        }
      } else {
#pragma unroll
        for (int q = 0; q < C; ++q) {
          const bool ok = any[delta] && i2 + q < e2s[delta];
          const cx<float> v = partials[ok ? o + q : 0];
          f[delta][q] = ok ? v : cx<float>{0, 0};
        }
      }
    }
#pragma unroll
    for (int delta = 0; delta < 8; ++delta)
#pragma unroll
      for (int q = 0; q < C; ++q)
        if (any[delta] && i2 + q < e2s[delta]) acc[q] = cadd(acc[q], f[delta][q]);
#pragma unroll
    for (int delta = 0; delta < 8; ++delta)
#pragma unroll
      for (int q = 0; q < C; ++q)
        if (any[delta] && i2 + q < e2s[delta])
          for (int t = rng[2 * delta] + 1; t < rng[2 * delta + 1]; ++t)
            acc[q] = cadd(acc[q], partials[t * PS + off[delta] + q]);
    float4* g4 = reinterpret_cast<float4*>(
        grid + (int64_t)(t0 * TILE + i0) * grid_plane_of<float>(K) + (int64_t)(t1 * TILE + i1) * K +
        (t2 * TILE + i2));
#pragma unroll
    for (int q = 0; q < C; q += 2) g4[q >> 1] = make_float4(acc[q].x, acc[q].y, acc[q + 1].x, acc[q + 1].y);
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
constexpr bool tile_fits() {  // the spread's FP64 halo tile must fit in LDS
  return (TILE + J - 1) * (TILE + J - 1) * (TILE + J - 1) * 16 <= 160 * 1024 && J - 1 <= TILE;
}

// OP_SPREAD_DET: FP64 spreading in fixed point (deterministic mode); the FP32
// spreading is always fixed point
enum Op { OP_INTERP = 0, OP_SPREAD = 1, OP_BOUND = 2, OP_SPREAD_DET = 3 };

template <typename T, int J, int TILE, bool CW, int OP>
hipError_t launch_one(const nufftct_plan& p, const void* src, void* dst, hipStream_t st) {
  if constexpr (!tile_fits<T, J, TILE>() || (OP == OP_SPREAD_DET && sizeof(T) == 4)) {
    return hipErrorInvalidValue;
  } else {
    constexpr int DEG = PolyOf<T>::DEG;
    const auto& P = PolyOf<T>::get(p);
    const dim3 grd((unsigned)((int64_t)p.xsplit.max_len * NUFFTCT_NUM_XCD));
    const PointGeom g = p.geom();
    if constexpr (OP == OP_SPREAD || OP == OP_SPREAD_DET) {
      constexpr bool FX = sizeof(T) == 4 || OP == OP_SPREAD_DET;
      hipLaunchKernelGGL((k_spread<T, J, TILE, CW, DEG, FX>), grd, dim3(GridCfg<T>::NT_SPREAD), 0,
                         st, (const cx<T>*)src, (cx<T>*)p.d_partials, p.d_perm_s, p.d_tasks,
                         p.d_spread_order, p.d_bound, p.d_multi, p.xsplit, g, p.nb, P);
      if constexpr (FX) {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const unsigned nbr = (unsigned)std::min<int64_t>(p.ntasks, NB_REST);
        hipLaunchKernelGGL((k_spread_rest<T, J, TILE, CW, DEG>), dim3(nbr),
                           dim3(GridCfg<T>::NT_SPREAD), 0, st, (const cx<T>*)src,
                           (cx<T>*)p.d_partials, p.d_perm_s, p.d_tasks, p.d_bound, p.d_multi, g,
                           p.nb, P);
      }
    } else if constexpr (OP == OP_BOUND) {
      hipLaunchKernelGGL((k_spread_bound<T, J, TILE, CW, DEG>), grd, dim3(NT_BOUND), 0, st,
                         p.d_bound, p.d_perm_s, p.d_tasks, p.xsplit, g, p.nb, P);
    } else {
      hipLaunchKernelGGL((k_interp<T, J, TILE, CW, DEG>), grd, dim3(GridCfg<T>::NT_INTERP), 0, st,
                         (const cx<T>*)src, (cx<T>*)dst, p.d_perm, p.d_tasks, p.xsplit, g,
                         p.nb, P);
    }
    return hipGetLastError();
  }
}

template <typename T, int J, bool CW, int OP>
hipError_t by_tile(const nufftct_plan& p, const void* src, void* dst, hipStream_t st) {
  switch (p.tile) {
    case 8: return launch_one<T, J, 8, CW, OP>(p, src, dst, st);
    case 16: return launch_one<T, J, 16, CW, OP>(p, src, dst, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, bool CW, int OP>
hipError_t by_j(const nufftct_plan& p, const void* src, void* dst, hipStream_t st) {
  switch (p.J) {
    case 2: return by_tile<T, 2, CW, OP>(p, src, dst, st);
    case 3: return by_tile<T, 3, CW, OP>(p, src, dst, st);
    case 4: return by_tile<T, 4, CW, OP>(p, src, dst, st);
    case 5: return by_tile<T, 5, CW, OP>(p, src, dst, st);
    case 6: return by_tile<T, 6, CW, OP>(p, src, dst, st);
    case 7: return by_tile<T, 7, CW, OP>(p, src, dst, st);
    case 8: return by_tile<T, 8, CW, OP>(p, src, dst, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int OP>
hipError_t run(const nufftct_plan& p, const void* src, void* dst, hipStream_t st) {
  if (p.ntasks == 0) return hipSuccess;
  if constexpr (OP == OP_SPREAD_DET && sizeof(T) == 4) return run<T, OP_SPREAD>(p, src, dst, st);
  if (p.kernel == NUFFTCT_KERNEL_MINMAX_KB) return by_j<T, true, OP>(p, src, dst, st);
  return by_j<T, false, OP>(p, src, dst, st);
}

template <typename T>
hipError_t merge(const nufftct_plan& p, void* grid, hipStream_t st, bool prune) {
  const int R = p.J - 1;
  const double r2 = prune ? p.ball_r2 : 1e300;
  const dim3 grd((unsigned)((int64_t)p.nb * p.nb * p.nb));
  if (p.tile == 16 && sizeof(T) == 4) {
    const MergeArgs a{(const cx<float>*)p.d_partials, p.d_bin_tasks, p.d_merge_order,
                      (cx<float>*)grid, p.nb, (int)p.K, R, r2, p.d_multi};
    hipLaunchKernelGGL((k_merge_pairs<16, 2, MergeArgs>), grd, dim3(1024), 0, st, a);
    return hipGetLastError();
  }
  if (p.tile == 16)
    hipLaunchKernelGGL((k_merge<T, 16>), grd, dim3(1024), 0, st, (const cx<T>*)p.d_partials,
                       p.d_bin_tasks, p.d_merge_order, (cx<T>*)grid, p.nb, (int)p.K, R, r2,
                       p.d_multi);
  else if (p.tile == 8)
    hipLaunchKernelGGL((k_merge<T, 8>), grd, dim3(512), 0, st, (const cx<T>*)p.d_partials,
                       p.d_bin_tasks, p.d_merge_order, (cx<T>*)grid, p.nb, (int)p.K, R, r2,
                       p.d_multi);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace kgrid

#define KGRID_INSTANTIATE(T)                                                                \
  template <>                                                                               \
  hipError_t launch_interp<T>(const nufftct_plan& p, const void* grid, void* out,           \
                              hipStream_t s) {                                              \
    return kgrid::run<T, kgrid::OP_INTERP>(p, grid, out, s);                                           \
  }                                                                                         \
  template <>                                                                               \
  hipError_t launch_spread<T>(const nufftct_plan& p, const void* in, void* grid,            \
                              hipStream_t s, bool det) {                                    \
    return det ? kgrid::run<T, kgrid::OP_SPREAD_DET>(p, in, grid, s)                        \
               : kgrid::run<T, kgrid::OP_SPREAD>(p, in, grid, s);                           \
  }                                                                                         \
  template <>                                                                               \
  hipError_t launch_spread_bound<T>(const nufftct_plan& p, hipStream_t s) {                 \
    return kgrid::run<T, kgrid::OP_BOUND>(p, nullptr, nullptr, s);                          \
  }                                                                                         \
  template <>                                                                               \
  hipError_t launch_merge<T>(const nufftct_plan& p, void* grid, hipStream_t s, bool prune) { \
    return kgrid::merge<T>(p, grid, s, prune);                                              \
  }
