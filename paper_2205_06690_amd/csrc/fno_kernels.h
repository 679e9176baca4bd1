// Launchers of the Fourier-operator surrogate kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>

namespace bse {
bool fno_grid_supported(int n);
void fno_configure(int n);
// V[F][K] = DFT of real fields on the kept modes (times c_k/ng if ck)
hipError_t fno_fft_fwd(int n, const float* in, int F, const float2* tw, int m, int ck, float2* work,
                       float2* V, hipStream_t st);
// out[F][ng] (=, or += when accumulate) = Re unnormalised inverse DFT of U on the kept modes
// (U times c_k/ng if ck)
hipError_t fno_fft_inv(int n, const float2* U, int F, const float2* tw, int m, int ck, float2* work,
                       float* out, int accumulate, hipStream_t st);
// per-mode channel mix U[b][o][k] = sum_i V[b][i][k] R[k][i][o] and its two
// backward products; path 0: matrix cores (up to 32 channels), 1: vector FMA
hipError_t fno_spec_mix(const float2* V, const float2* R, int B, int C, int K, float2* U, int path,
                        hipStream_t st);
hipError_t fno_spec_mix_bwd(const float2* V, const float2* GU, const float2* R, int B, int C, int K,
                            float2* GV, float2* GR, int path, hipStream_t st);
hipError_t fno_pointwise(const float* in, int Cin, const float* Wm, const float* bias, int Cout,
                         const float* add, int B, size_t ng, int act, float* zout, float* out,
                         hipStream_t st);
hipError_t fno_pointwise_bwd(const float* gz, int Cout, const float* Wm, int Cin, int B, size_t ng,
                             float* gin, hipStream_t st);
hipError_t fno_gelu_bwd(float* gh, const float* z, size_t n, hipStream_t st);
size_t fno_outer_part_len(int Co, int Ci, int B, size_t ng);
hipError_t fno_outer(const float* A, int Co, const float* X, int Ci, int B, size_t ng, float* part,
                     float* gW, float* gb, hipStream_t st);
hipError_t fno_proj_bwd(const float* gy, const float* Q, int C, int B, size_t ng, float* gh, hipStream_t st);
int fno_loss_blocks(size_t ng);
hipError_t fno_loss_partial(const float* y, const float* t, int B, size_t ng, double* part, hipStream_t st);
hipError_t fno_loss_grad(const float* y, const float* t, const double* tn, int B, size_t ng, float* gy,
                         hipStream_t st);
hipError_t fno_adam(float* master, float* compute, const float* g, float* m, float* v, size_t n,
                    float lr, float b1, float b2, float eps, int step, int bf16, hipStream_t st);
hipError_t fno_round_copy(const float* src, float* dst, size_t n, int bf16, hipStream_t st);
// dst[b][c] = sample idx[b] of src[.][C][n^3] under a symmetry of the cube:
// output axis k is input axis perm[k], and the output axes in flip_mask
// (bit k) run backwards
hipError_t fno_gather_sym(const float* src, const int* idx, int B, int C, int n, const int perm[3],
                          int flip_mask, float* dst, hipStream_t st);
}  // namespace bse
