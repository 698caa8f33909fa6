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

// Map a linear block index to a task so that each XCD receives a contiguous
// range of tasks (neighbouring tiles share their halos through that XCD's L2).
__device__ __forceinline__ int64_t xcd_task(int64_t b, int64_t per_xcd) {
  return (b % NUFFTCT_NUM_XCD) * per_xcd + b / NUFFTCT_NUM_XCD;
}
