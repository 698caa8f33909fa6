// Interpolation / spreading kernels instantiated for FP32 (complex64), and
// the fill kernel used to clear workspaces (kept as a kernel so that it can
// be captured in HIP graphs).
// FP32 spreading keeps one 8-byte accumulator per halo cell (74 KB for
// tile 16, J = 6), so two workgroups share a CU; 512 threads each within
// 128 VGPRs (measured faster than 1024 threads within 64).
#ifndef NUFFTCT_SPREAD32_NT
#define NUFFTCT_SPREAD32_NT 512
#endif
#ifndef NUFFTCT_SPREAD32_WAVES
#define NUFFTCT_SPREAD32_WAVES 4
#endif
#define NUFFTCT_SPREAD_NT NUFFTCT_SPREAD32_NT
#define NUFFTCT_SPREAD_WAVES_PER_EU NUFFTCT_SPREAD32_WAVES
// FP32 interpolation: two 512-thread workgroups per CU (LDS-bound) within
// 128 VGPRs, which leaves room for a one-ahead prefetch of the next point's id
// only (not of its geometry).
#ifndef NUFFTCT_INTERP32_NT
#define NUFFTCT_INTERP32_NT 512
#endif
#ifndef NUFFTCT_INTERP32_WAVES
#define NUFFTCT_INTERP32_WAVES 4
#endif
#ifndef NUFFTCT_INTERP32_PREFETCH
#define NUFFTCT_INTERP32_PREFETCH 2
#endif
#define NUFFTCT_INTERP_NT NUFFTCT_INTERP32_NT
#define NUFFTCT_INTERP_WAVES_PER_EU NUFFTCT_INTERP32_WAVES
#define NUFFTCT_INTERP_PREFETCH NUFFTCT_INTERP32_PREFETCH
#include "k_grid_impl.h"
KGRID_INSTANTIATE(float)

__global__ void k_zero(float4* __restrict__ p, int64_t n16) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n16; i += stride) p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

hipError_t launch_zero(void* ptr, size_t bytes, hipStream_t s) {
  const int64_t n16 = (int64_t)(bytes / 16);
  if (n16 == 0) return hipSuccess;
  int64_t blocks = (n16 + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, (float4*)ptr, n16);
  return hipGetLastError();
}
