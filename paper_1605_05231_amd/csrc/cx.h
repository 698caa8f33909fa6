// Complex arithmetic and small device helpers shared by the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.x * s, a.y * s}; }
// a * (S i), S = +1 or -1
template <int S, typename T>
__device__ __forceinline__ cx<T> cmul_si(cx<T> a) {
  return S > 0 ? cx<T>{-a.y, a.x} : cx<T>{a.y, -a.x};
}

// number of XCDs of gfx950; workgroups are dispatched round-robin across them
#define NUFFTCT_NUM_XCD 8

// Contiguous task ranges, one per XCD, cut on the host so that each range
// holds about the same number of points.  Block b runs on XCD b % 8 and takes
// the (b / 8)-th task of that XCD's range, so neighbouring tiles (which share
// halo cells) go through the same L2 and every XCD gets an equal share of work.
struct XcdSplit {
  int32_t start[NUFFTCT_NUM_XCD + 1];
  int32_t max_len;  // longest range; the grid has 8 * max_len blocks
};

// Task of block b, or -1 when b is past the end of its XCD's range.
__device__ __forceinline__ int64_t xcd_task(int64_t b, const XcdSplit& xs) {
  const int x = (int)(b % NUFFTCT_NUM_XCD);
  const int64_t t = xs.start[x] + b / NUFFTCT_NUM_XCD;
  return t < xs.start[x + 1] ? t : -1;
}
