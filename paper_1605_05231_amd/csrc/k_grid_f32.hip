// Interpolation / spreading kernels instantiated for FP32 (complex64), and
// the fill kernel used to clear workspaces (kept as a kernel so that it can
// be captured in HIP graphs).
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
