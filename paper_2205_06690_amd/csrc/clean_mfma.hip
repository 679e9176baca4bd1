// Cleaning projection of the perturbed stochastic orbitals (Eq. 15,
// linearised) on the FP32 matrix cores of gfx950.
//
//   coefficients  C[f][s] = h^3 sum_r phi_s(r) d_f(r)       (split-K GEMM)
//   update        d_f(r) -= sum_s C[f][s] phi_s(r) + c_f E_l(r)
//
// Complex fields are viewed as two real rows (2f: real part, 2f+1:
// imaginary part), the occupied orbitals are real, so both products are real
// GEMMs: rows x states over K = grid points, and rows x points over
// K = states.  v_mfma_f32_16x16x4f32: lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; the 16x16 result sits in lane l as D[4(l/16)+v][l%16],
// v = 0..3.
#include <hip/hip_runtime.h>

#include "clean_mfma.h"

namespace bse {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int CM_BM = 128, CM_BN = 128, CM_BK = 32, CM_PAD = 4;

// part[kc][row][s] (row < 2F, s < S) = sum over chunk kc of A[row][r] phi_s(r).
// Global loads of stage k+1 are issued into registers before the matrix-core
// work of stage k.
__global__ void __launch_bounds__(256) k_coef_mfma(const float2* __restrict__ d, int F,
                                                   const float* __restrict__ phi, int S,
                                                   size_t ng, int chunk,
                                                   float* __restrict__ part) {
  __shared__ float As[CM_BK][CM_BM + CM_PAD];
  __shared__ float Bs[CM_BK][CM_BN + CM_PAD];
  constexpr int NA = (CM_BM / 2) * CM_BK / 256;  // float2 per thread
  constexpr int NB = CM_BN * CM_BK / 256;        // float per thread
  const int R = 2 * F;
  const int r0 = blockIdx.x * CM_BM;
  const int s0 = blockIdx.y * CM_BN;
  const int kc = blockIdx.z;
  const size_t k0 = (size_t)kc * chunk;
  const size_t k1 = min(ng, k0 + (size_t)chunk);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int f0 = r0 / 2;
  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  float2 ra[NA];
  float rb[NB];
  auto load = [&](size_t kb) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = tid + i * 256;
      const int ff = e / CM_BK, p = e % CM_BK;
      const int f = f0 + ff;
      const size_t r = kb + p;
      ra[i] = (f < F && r < k1) ? d[(size_t)f * ng + r] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int e = tid + i * 256;
      const int ss = e / CM_BK, p = e % CM_BK;
      const int s = s0 + ss;
      const size_t r = kb + p;
      rb[i] = (s < S && r < k1) ? phi[(size_t)s * ng + r] : 0.f;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = tid + i * 256;
      const int ff = e / CM_BK, p = e % CM_BK;
      As[p][2 * ff] = ra[i].x;
      As[p][2 * ff + 1] = ra[i].y;
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int e = tid + i * 256;
      const int ss = e / CM_BK, p = e % CM_BK;
      Bs[p][ss] = rb[i];
    }
  };
  load(k0);
  for (size_t kb = k0; kb < k1; kb += CM_BK) {
    __syncthreads();
    store();
    __syncthreads();
    if (kb + CM_BK < k1) load(kb + CM_BK);
#pragma unroll
    for (int k4 = 0; k4 < CM_BK / 4; ++k4) {
      const int kk = k4 * 4 + (lane >> 4);
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][wm * 64 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
  float* out = part + (size_t)kc * R * S;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = r0 + wm * 64 + i * 16 + 4 * (lane >> 4) + v;
        const int col = s0 + wn * 64 + j * 16 + (lane & 15);
        if (row < R && col < S) out[(size_t)row * S + col] = acc[i][j][v];
      }
}

// coefT[s][row] = (float) re/im of coef[f][s], row = 2f + c
__global__ void k_coef_transpose(const double2* __restrict__ coef, int F, int S,
                                 float* __restrict__ coefT) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= F * S) return;
  const int f = i % F, s = i / F;
  const double2 c = coef[(size_t)f * (S + 1) + s];
  coefT[(size_t)s * 2 * F + 2 * f] = (float)c.x;
  coefT[(size_t)s * 2 * F + 2 * f + 1] = (float)c.y;
}

// coef[f][s] = dv * (sum_kc part[kc][2f][s] + i sum_kc part[kc][2f+1][s]),
// stored with row stride S+1 (slot S holds the E dot).
__global__ void k_coef_reduce(const float* __restrict__ part, int nchunk, int F, int S, double dv,
                              double2* __restrict__ coef) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= F * S) return;
  const int f = i / S, s = i % S;
  const size_t RS = (size_t)2 * F * S;
  double x = 0, y = 0;
  for (int k = 0; k < nchunk; ++k) {
    x += part[k * RS + (size_t)(2 * f) * S + s];
    y += part[k * RS + (size_t)(2 * f + 1) * S + s];
  }
  coef[(size_t)f * (S + 1) + s] = make_double2(x * dv, y * dv);
}

// partial <E_l, d_f> over blocks of 1024 points: gpart[f][blk]
__global__ void __launch_bounds__(256) k_edot(const float2* __restrict__ d, const float2* __restrict__ E,
                                              int L, size_t ng, double2* __restrict__ gpart) {
  const int f = blockIdx.y, l = f % L;
  const size_t base = (size_t)blockIdx.x * 1024;
  double x = 0, y = 0;
  for (int q = 0; q < 4; ++q) {
    const size_t r = base + threadIdx.x + q * 256;
    if (r < ng) {
      const float2 a = d[(size_t)f * ng + r];
      const float2 e = E[(size_t)l * ng + r];
      x += (double)e.x * a.x + (double)e.y * a.y;
      y += (double)e.x * a.y - (double)e.y * a.x;
    }
  }
  __shared__ double rx[256], ry[256];
  rx[threadIdx.x] = x;
  ry[threadIdx.x] = y;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      rx[threadIdx.x] += rx[threadIdx.x + s];
      ry[threadIdx.x] += ry[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) gpart[(size_t)f * gridDim.x + blockIdx.x] = make_double2(rx[0], ry[0]);
}

__global__ void k_edot_reduce(const double2* __restrict__ gpart, int nblk, int F, int S, double dv,
                              double2* __restrict__ coef) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= F) return;
  double x = 0, y = 0;
  for (int k = 0; k < nblk; ++k) {
    x += gpart[(size_t)f * nblk + k].x;
    y += gpart[(size_t)f * nblk + k].y;
  }
  coef[(size_t)f * (S + 1) + S] = make_double2(x * dv, y * dv);
}

// d_f(r) -= sum_s C[f][s] phi_s(r) + c_f E_l(r); rows 2f/2f+1 = re/im of C
// (coefT[s][row], FP32).  Block: 128 rows (64 fields) x 128 points, K =
// states in stages of 32 with register prefetch.
__global__ void __launch_bounds__(256) k_update_mfma(float2* __restrict__ d, int F,
                                                     const float* __restrict__ phi, int S,
                                                     const float2* __restrict__ E, int L,
                                                     size_t ng, const float* __restrict__ coefT,
                                                     const double2* __restrict__ coef) {
  __shared__ float As[CM_BK][CM_BM + CM_PAD];
  __shared__ float Bs[CM_BK][CM_BN + CM_PAD];
  constexpr int NA = CM_BM * CM_BK / 256;
  constexpr int NB = CM_BN * CM_BK / 256;
  const int R = 2 * F;
  const size_t p0 = (size_t)blockIdx.x * CM_BN;
  const int r0 = blockIdx.y * CM_BM;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  float ra[NA], rb[NB];
  auto load = [&](int sb) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = tid + i * 256;
      const int ss = e / CM_BM, rr = e % CM_BM;
      const int s = sb + ss, row = r0 + rr;
      ra[i] = (s < S && row < R) ? coefT[(size_t)s * R + row] : 0.f;
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int e = tid + i * 256;
      const int ss = e / CM_BN, p = e % CM_BN;
      const int s = sb + ss;
      const size_t r = p0 + p;
      rb[i] = (s < S && r < ng) ? phi[(size_t)s * ng + r] : 0.f;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = tid + i * 256;
      As[e / CM_BM][e % CM_BM] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int e = tid + i * 256;
      Bs[e / CM_BN][e % CM_BN] = rb[i];
    }
  };
  load(0);
  for (int sb = 0; sb < S; sb += CM_BK) {
    __syncthreads();
    store();
    __syncthreads();
    if (sb + CM_BK < S) load(sb + CM_BK);
#pragma unroll
    for (int k4 = 0; k4 < CM_BK / 4; ++k4) {
      const int kk = k4 * 4 + (lane >> 4);
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][wm * 64 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
  // epilogue: lane holds rows 4q..4q+3 = fields 2q, 2q+1 (re, im) at one point
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = r0 + wm * 64 + i * 16 + 4 * (lane >> 4);
      const size_t r = p0 + wn * 64 + j * 16 + (lane & 15);
      if (r >= ng) continue;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int f = row / 2 + h;
        if (2 * f >= R) continue;
        const int l = f % L;
        const float cr = (float)coef[(size_t)f * (S + 1) + S].x;
        const float2 e = E[(size_t)l * ng + r];
        float2 v = d[(size_t)f * ng + r];
        v.x -= acc[i][j][2 * h] + cr * e.x;
        v.y -= acc[i][j][2 * h + 1] + cr * e.y;
        d[(size_t)f * ng + r] = v;
      }
    }
}

hipError_t launch_coef_mfma(const float2* d, int F, const float* phi, int S, size_t ng, int chunk,
                            float* part, double dv, double2* coef, hipStream_t st) {
  const int nchunk = (int)((ng + chunk - 1) / chunk);
  dim3 g((2 * F + CM_BM - 1) / CM_BM, (S + CM_BN - 1) / CM_BN, nchunk);
  hipLaunchKernelGGL(k_coef_mfma, g, dim3(256), 0, st, d, F, phi, S, ng, chunk, part);
  hipLaunchKernelGGL(k_coef_reduce, dim3((F * S + 255) / 256), dim3(256), 0, st, part, nchunk, F, S,
                     dv, coef);
  return hipGetLastError();
}

hipError_t launch_edot(const float2* d, const float2* E, int F, int L, int S, size_t ng,
                       double2* gpart, double dv, double2* coef, hipStream_t st) {
  const int nblk = (int)((ng + 1023) / 1024);
  hipLaunchKernelGGL(k_edot, dim3(nblk, F), dim3(256), 0, st, d, E, L, ng, gpart);
  hipLaunchKernelGGL(k_edot_reduce, dim3((F + 255) / 256), dim3(256), 0, st, gpart, nblk, F, S, dv,
                     coef);
  return hipGetLastError();
}

hipError_t launch_update_mfma(float2* d, int F, const float* phi, int S, const float2* E, int L,
                              size_t ng, const double2* coef, float* coefT, hipStream_t st) {
  hipLaunchKernelGGL(k_coef_transpose, dim3((F * S + 255) / 256), dim3(256), 0, st, coef, F, S, coefT);
  dim3 g((unsigned)((ng + CM_BN - 1) / CM_BN), (2 * F + CM_BM - 1) / CM_BM);
  hipLaunchKernelGGL(k_update_mfma, g, dim3(256), 0, st, d, F, phi, S, E, L, ng, coefT, coef);
  return hipGetLastError();
}

size_t coef_part_floats(int F, int S, size_t ng, int chunk) {
  return (size_t)((ng + chunk - 1) / chunk) * 2 * F * S;
}
size_t edot_part_entries(int F, size_t ng) { return (size_t)F * ((ng + 1023) / 1024); }

}  // namespace bse
