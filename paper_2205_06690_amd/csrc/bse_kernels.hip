// A-matrix contraction, spectrum and utility kernels for gfx950.
#include "bse_kernels.h"

namespace bse {

// flags[b] = 1 if row b of w has a non-finite value
__global__ void k_finite_check(const double* __restrict__ w, size_t ng, int* __restrict__ flags) {
  const int b = blockIdx.y;
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  int mine = 0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < ng; i += (size_t)gridDim.x * blockDim.x)
    if (!isfinite(w[(size_t)b * ng + i])) mine = 1;
  if (mine) atomicOr(&bad, 1);
  __syncthreads();
  if (threadIdx.x == 0 && bad) atomicOr(&flags[b], 1);
}

__global__ void k_fill_nan(double* __restrict__ w, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) w[i] = __builtin_nan("");
}

hipError_t launch_finite_check(const double* w, int B, size_t ng, int* flags, hipStream_t st) {
  hipError_t e = hipMemsetAsync(flags, 0, sizeof(int) * B, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_finite_check, dim3(64, B), dim3(256), 0, st, w, ng, flags);
  return hipGetLastError();
}

hipError_t launch_fill_nan(double* w, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_nan, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, w, n);
  return hipGetLastError();
}

}  // namespace bse
