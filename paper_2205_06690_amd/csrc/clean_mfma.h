// FP32 matrix-core kernels of the cleaning projection.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>

namespace bse {
hipError_t launch_coef_mfma(const float2* d, int F, const float* phi, int S, size_t ng, int chunk,
                            float* part, double dv, double2* coef, hipStream_t st);
hipError_t launch_edot(const float2* d, const float2* E, int F, int L, int S, size_t ng,
                       double2* gpart, double dv, double2* coef, hipStream_t st);
hipError_t launch_update_mfma(float2* d, int F, const float* phi, int S, const float2* E, int L,
                              size_t ng, const double2* coef, float* coefT, hipStream_t st);
size_t coef_part_floats(int F, int S, size_t ng, int chunk);
size_t edot_part_entries(int F, size_t ng);
}  // namespace bse
