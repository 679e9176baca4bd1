// Launchers of the A-matrix, spectrum and utility kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>

namespace bse {
hipError_t launch_finite_check(const double* w, int B, size_t ng, int* flags, hipStream_t st);
hipError_t launch_fill_nan(double* w, size_t n, hipStream_t st);
}  // namespace bse
