// Grid contractions of Eq. 1 on the BF16 matrix cores with operands split
// once from FP64 (three-term products, FP32 tile sums, FP64 chunk sums).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>

#include "prop_kernels.h"   // LaunchEvents

namespace bse {
// x [n] FP64 -> bf16 pairs h, l (bit patterns), x ~ h + l
hipError_t launch_split64(const double* x, size_t n, unsigned short* h, unsigned short* l,
                          hipStream_t st);
// products phi_p phi_q (FP64) for K pairs pq[K][2] -> bf16 pairs [K][ng]
hipError_t launch_products_split(const double* phi, const int* pq, int K, size_t ng, unsigned short* h,
                                 unsigned short* l, hipStream_t st);
// C[M][N] = scale sum_r A[m][r] B[n][r]; A, B as bf16 pairs [rows][K];
// K a multiple of 64; part holds contract_part_floats(M, N, K) floats
// ev / ev_reduce (nullable): start and stop events recorded in the dispatch
// packets of the GEMM and of the chunk reduction
hipError_t launch_contract_x3(const unsigned short* ah, const unsigned short* al, int M,
                              const unsigned short* bh, const unsigned short* bl, int N, size_t K,
                              double scale, float* part, double* C, hipStream_t st,
                              const LaunchEvents* ev = nullptr, const LaunchEvents* ev_reduce = nullptr);
size_t contract_part_floats(int M, int N, size_t K);
}  // namespace bse
