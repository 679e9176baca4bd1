// Fourier-operator screening surrogate: forward, backward and Adam kernels
// for gfx950 (FP32 activations and accumulation, weights rounded to BF16).
//
// Spectral convolution on the kept modes K = {kx, ky in [-m, m), kz in
// [0, m)}: a truncated 3-D DFT (full y-z plane transforms, then x lines of
// the kept (ky, kz) columns only, gathered to [field][K]), a per-mode
// complex channel mix, and the adjoint path (scatter to the kept columns,
// inverse x lines, inverse y-z planes, real part).  The DFT machinery is the
// LDS four-step line transform of fft_lines.h.
#include <hip/hip_runtime.h>

#include "fft_lines.h"
#include "fno_kernels.h"

namespace bse {

template <int N> constexpr int fplane_stride() { return N + 1; }
template <int N> __device__ __forceinline__ int fplane_idx(int e) {
  return (e / N) * fplane_stride<N>() + (e % N);
}
// the twiddle table copied into LDS (the transforms then read it through the
// LDS counter, not behind the vector-memory loads of the data)
template <int N>
__device__ __forceinline__ void fno_tw_lds(float2* t, const float2* __restrict__ tw, int tid, int nthr) {
  for (int i = tid; i < N; i += nthr) t[i] = tw[i];
}

// scrambled slot of natural frequency index k (inverse of scr2k)
template <int N> __device__ __forceinline__ int k2scr(int k) {
  constexpr int N1 = Fac<N>::N1, N2 = Fac<N>::N2;
  return (k % N1) * N2 + k / N1;
}

// ---------------------------------------------------------------------------
// truncated forward DFT: real fields [F][ng] -> V[F][K] (times c_k/ng if
// ck_scale, else times 1)
// ---------------------------------------------------------------------------
template <int N>
__global__ void __launch_bounds__(256) k_fno_yz_fwd_t(const float* __restrict__ in,
                                                     float2* __restrict__ work,
                                                     const float2* __restrict__ tw) {
  extern __shared__ unsigned char smem_raw[];
  float2* s = reinterpret_cast<float2*>(smem_raw);
  constexpr int P = N * N, S = fplane_stride<N>(), NT = 256;
  const size_t ng = (size_t)N * N * N;
  const int x = blockIdx.x, f = blockIdx.y, tid = threadIdx.x;
  const float* src = in + (size_t)f * ng + (size_t)x * P;
  float2* twl = s + N * S;
  fno_tw_lds<N>(twl, tw, tid, NT);
  for (int e = tid; e < P; e += NT) s[fplane_idx<N>(e)] = make_float2(src[e], 0.f);
  __syncthreads();
  NoMul nm;
  stageA_fwd<N>(s, N, S, 1, twl, tid, NT, true);
  __syncthreads();
  stageB<N, 0>(s, N, S, 1, twl, tid, NT, true, nm);
  __syncthreads();
  stageA_fwd<N>(s, N, 1, S, twl, tid, NT, true);
  __syncthreads();
  stageB<N, 0>(s, N, 1, S, twl, tid, NT, true, nm);
  __syncthreads();
  float2* dst = work + (size_t)f * ng + (size_t)x * P;
  for (int e = tid; e < P; e += NT) dst[e] = s[fplane_idx<N>(e)];
}

// kept columns: 2m x m (ky, kz); block = (field, group of KC columns)
constexpr int KC = 16;
template <int N>
__global__ void __launch_bounds__(256) k_fno_x_gather(const float2* __restrict__ work,
                                                      const float2* __restrict__ tw, int m,
                                                      int ck_scale, float2* __restrict__ V) {
  __shared__ float2 s[N * KC];
  __shared__ float2 twl[N];
  fno_tw_lds<N>(twl, tw, threadIdx.x, 256);
  const size_t ng = (size_t)N * N * N;
  const int f = blockIdx.y, tid = threadIdx.x;
  const int ncol = 2 * m * m;
  const int K = 2 * m * 2 * m * m;
  const int col0 = blockIdx.x * KC;
  // load x lines of KC kept columns (zero past the last column)
  for (int e = tid; e < N * KC; e += 256) {
    const int x = e / KC, c = e % KC;
    const int col = col0 + c;
    float2 v = make_float2(0.f, 0.f);
    if (col < ncol) {
      const int jy = col / m, kz = col % m;
      const int ky = jy - m;                     // signed
      const int ys = k2scr<N>((ky + N) % N), zs = k2scr<N>(kz);
      v = work[(size_t)f * ng + (size_t)x * N * N + (size_t)ys * N + zs];
    }
    s[x * KC + c] = v;
  }
  __syncthreads();
  NoMul nm;
  stageA_fwd<N>(s, KC, 1, KC, twl, tid, 256, true);
  __syncthreads();
  stageB<N, 0>(s, KC, 1, KC, twl, tid, 256, true, nm);
  __syncthreads();
  const float inv = 1.0f / (float)ng;
  for (int e = tid; e < 2 * m * KC; e += 256) {
    const int jx = e / KC, c = e % KC;
    const int col = col0 + c;
    if (col >= ncol) continue;
    const int jy = col / m, kz = col % m;
    const int kx = jx - m;
    float2 v = s[k2scr<N>((kx + N) % N) * KC + c];
    if (ck_scale) {
      const float sc = (kz == 0 ? 1.0f : 2.0f) * inv;
      v.x *= sc;
      v.y *= sc;
    }
    // mode index: kx-major, then ky, then kz
    V[(size_t)f * K + ((size_t)jx * 2 * m + jy) * m + kz] = v;
  }
}

// ---------------------------------------------------------------------------
// adjoint: U[F][K] (times c_k/ng if ck_scale) -> real fields [F][ng]
// (out = result, or out += result when accumulate)
// ---------------------------------------------------------------------------
template <int N>
__global__ void __launch_bounds__(256) k_fno_x_scatter(const float2* __restrict__ U,
                                                       const float2* __restrict__ tw, int m,
                                                       int ck_scale, float2* __restrict__ work) {
  __shared__ float2 s[N * KC];
  __shared__ float2 twl[N];
  fno_tw_lds<N>(twl, tw, threadIdx.x, 256);
  const size_t ng = (size_t)N * N * N;
  const int f = blockIdx.y, tid = threadIdx.x;
  const int ncol = 2 * m * m;
  const int K = 2 * m * 2 * m * m;
  const int col0 = blockIdx.x * KC;
  for (int e = tid; e < N * KC; e += 256) s[e] = make_float2(0.f, 0.f);
  __syncthreads();
  const float inv = 1.0f / (float)ng;
  for (int e = tid; e < 2 * m * KC; e += 256) {
    const int jx = e / KC, c = e % KC;
    const int col = col0 + c;
    if (col >= ncol) continue;
    const int jy = col / m, kz = col % m;
    const int kx = jx - m;
    float2 v = U[(size_t)f * K + ((size_t)jx * 2 * m + jy) * m + kz];
    if (ck_scale) {
      const float sc = (kz == 0 ? 1.0f : 2.0f) * inv;
      v.x *= sc;
      v.y *= sc;
    }
    s[k2scr<N>((kx + N) % N) * KC + c] = v;
  }
  __syncthreads();
  NoMul nm;
  stageB<N, 1>(s, KC, 1, KC, twl, tid, 256, true, nm);
  __syncthreads();
  stageC_inv<N>(s, KC, 1, KC, tid, 256, true);
  __syncthreads();
  for (int e = tid; e < N * KC; e += 256) {
    const int x = e / KC, c = e % KC;
    const int col = col0 + c;
    if (col >= ncol) continue;
    const int jy = col / m, kz = col % m;
    const int ky = jy - m;
    const int ys = k2scr<N>((ky + N) % N), zs = k2scr<N>(kz);
    work[(size_t)f * ng + (size_t)x * N * N + (size_t)ys * N + zs] = s[x * KC + c];
  }
}

template <int N>
__global__ void __launch_bounds__(256) k_fno_yz_inv(const float2* __restrict__ work,
                                                    const float2* __restrict__ tw,
                                                    float* __restrict__ out, int accumulate) {
  extern __shared__ unsigned char smem_raw[];
  float2* s = reinterpret_cast<float2*>(smem_raw);
  constexpr int P = N * N, S = fplane_stride<N>(), NT = 256;
  const size_t ng = (size_t)N * N * N;
  const int x = blockIdx.x, f = blockIdx.y, tid = threadIdx.x;
  const float2* src = work + (size_t)f * ng + (size_t)x * P;
  float2* twl = s + N * S;
  fno_tw_lds<N>(twl, tw, tid, NT);
  for (int e = tid; e < P; e += NT) s[fplane_idx<N>(e)] = src[e];
  __syncthreads();
  NoMul nm;
  stageB<N, 1>(s, N, S, 1, twl, tid, NT, true, nm);
  __syncthreads();
  stageC_inv<N>(s, N, S, 1, tid, NT, true);
  __syncthreads();
  stageB<N, 1>(s, N, 1, S, twl, tid, NT, true, nm);
  __syncthreads();
  stageC_inv<N>(s, N, 1, S, tid, NT, true);
  __syncthreads();
  float* dst = out + (size_t)f * ng + (size_t)x * P;
  for (int e = tid; e < P; e += NT) {
    const float v = s[fplane_idx<N>(e)].x;
    dst[e] = accumulate ? dst[e] + v : v;
  }
}

// ---------------------------------------------------------------------------
// spectral channel mix
// ---------------------------------------------------------------------------
// U[b][o][k] = sum_i V[b][i][k] R[k][i][o]
__global__ void k_spec_mix(const float2* __restrict__ V, const float2* __restrict__ R, int B, int C,
                           int K, float2* __restrict__ U) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t tot = (size_t)B * K * C;
  if (idx >= tot) return;
  const int o = (int)(idx % C);
  const int k = (int)((idx / C) % K);
  const int b = (int)(idx / ((size_t)C * K));
  float ax = 0.f, ay = 0.f;
  for (int i = 0; i < C; ++i) {
    const float2 v = V[((size_t)b * C + i) * K + k];
    const float2 r = R[((size_t)k * C + i) * C + o];
    ax += v.x * r.x - v.y * r.y;
    ay += v.x * r.y + v.y * r.x;
  }
  U[((size_t)b * C + o) * K + k] = make_float2(ax, ay);
}

// GV[b][i][k] = sum_o GU[b][o][k] conj(R[k][i][o])
__global__ void k_spec_mix_bwd_v(const float2* __restrict__ GU, const float2* __restrict__ R, int B,
                                 int C, int K, float2* __restrict__ GV) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t tot = (size_t)B * K * C;
  if (idx >= tot) return;
  const int i = (int)(idx % C);
  const int k = (int)((idx / C) % K);
  const int b = (int)(idx / ((size_t)C * K));
  float ax = 0.f, ay = 0.f;
  for (int o = 0; o < C; ++o) {
    const float2 g = GU[((size_t)b * C + o) * K + k];
    const float2 r = R[((size_t)k * C + i) * C + o];
    ax += g.x * r.x + g.y * r.y;
    ay += g.y * r.x - g.x * r.y;
  }
  GV[((size_t)b * C + i) * K + k] = make_float2(ax, ay);
}

// GR[k][i][o] = sum_b conj(V[b][i][k]) GU[b][o][k]
__global__ void k_spec_mix_bwd_r(const float2* __restrict__ V, const float2* __restrict__ GU, int B,
                                 int C, int K, float2* __restrict__ GR) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t tot = (size_t)K * C * C;
  if (idx >= tot) return;
  const int o = (int)(idx % C);
  const int i = (int)((idx / C) % C);
  const int k = (int)(idx / ((size_t)C * C));
  float ax = 0.f, ay = 0.f;
  for (int b = 0; b < B; ++b) {
    const float2 v = V[((size_t)b * C + i) * K + k];
    const float2 g = GU[((size_t)b * C + o) * K + k];
    ax += v.x * g.x + v.y * g.y;
    ay += v.x * g.y - v.y * g.x;
  }
  GR[idx] = make_float2(ax, ay);
}

// ---------------------------------------------------------------------------
// The same three products on the matrix cores (v_mfma_f32_16x16x4f32, FP32
// operands and accumulation), one wave per Fourier mode k, for channel
// counts up to 32 (padded with zeros to CP, a multiple of 16).  A complex
// product X Y is the real product of [Xr | Xi] with the 2 x 2 block form of
// Y, so the real and imaginary parts of an output are two column tiles of
// one real GEMM.  Lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] of
// a 16 x 4 by 4 x 16 step and holds D[4 (l / 16) + j][l % 16], j < 4.
// Every output is written once (no atomics): results do not depend on
// scheduling.
// ---------------------------------------------------------------------------
typedef float mf4 __attribute__((ext_vector_type(4)));

// U_k = V_k R_k: rows b (16 per pass), columns [Ur | Ui], contraction over
// [i re | i im] with blocks [[Rr, Ri], [-Ri, Rr]]
template <int CP>
__global__ void __launch_bounds__(256) k_spec_mix_mfma(const float2* __restrict__ V,
                                                       const float2* __restrict__ R, int B, int C, int K,
                                                       float2* __restrict__ U) {
  constexpr int S = CP / 4, T = CP / 16;
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= K) return;
  const int lr = lane & 15, lk = lane >> 4;
  const float2* Rk = R + (size_t)k * C * C;
  float2 r[S][T];
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int i = 4 * s + lk, o = 16 * t + lr;
      r[s][t] = (i < C && o < C) ? Rk[(size_t)i * C + o] : make_float2(0.f, 0.f);
    }
  for (int b0 = 0; b0 < B; b0 += 16) {
    const int b = b0 + lr;
    float2 v[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int i = 4 * s + lk;
      v[s] = (b < B && i < C) ? V[((size_t)b * C + i) * K + k] : make_float2(0.f, 0.f);
    }
    mf4 acc[2 * T];
#pragma unroll
    for (int t = 0; t < 2 * T; ++t) acc[t] = mf4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int part = 0; part < 2; ++part)
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const float a = part == 0 ? v[s].x : v[s].y;
#pragma unroll
        for (int t = 0; t < T; ++t) {
          const float2 rr = r[s][t];
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, part == 0 ? rr.x : -rr.y, acc[t], 0, 0, 0);
          acc[T + t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, part == 0 ? rr.y : rr.x, acc[T + t], 0, 0, 0);
        }
      }
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = b0 + 4 * lk + j, o = 16 * t + lr;
        if (row < B && o < C) U[((size_t)row * C + o) * K + k] = make_float2(acc[t][j], acc[T + t][j]);
      }
  }
}

// GV_k = GU_k conj(R_k)^T: rows b, columns [GVr | GVi] over i, contraction
// over [o re | o im] with blocks [[Rr^T, -Ri^T], [Ri^T, Rr^T]]
template <int CP>
__global__ void __launch_bounds__(256) k_spec_mix_bwd_v_mfma(const float2* __restrict__ GU,
                                                             const float2* __restrict__ R, int B, int C,
                                                             int K, float2* __restrict__ GV) {
  constexpr int S = CP / 4, T = CP / 16;
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= K) return;
  const int lr = lane & 15, lk = lane >> 4;
  const float2* Rk = R + (size_t)k * C * C;
  float2 r[S][T];                       // r[s][t] = R[i = 16 t + lr][o = 4 s + lk]
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int o = 4 * s + lk, i = 16 * t + lr;
      r[s][t] = (i < C && o < C) ? Rk[(size_t)i * C + o] : make_float2(0.f, 0.f);
    }
  for (int b0 = 0; b0 < B; b0 += 16) {
    const int b = b0 + lr;
    float2 g[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int o = 4 * s + lk;
      g[s] = (b < B && o < C) ? GU[((size_t)b * C + o) * K + k] : make_float2(0.f, 0.f);
    }
    mf4 acc[2 * T];
#pragma unroll
    for (int t = 0; t < 2 * T; ++t) acc[t] = mf4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int part = 0; part < 2; ++part)
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const float a = part == 0 ? g[s].x : g[s].y;
#pragma unroll
        for (int t = 0; t < T; ++t) {
          const float2 rr = r[s][t];
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, part == 0 ? rr.x : rr.y, acc[t], 0, 0, 0);
          acc[T + t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, part == 0 ? -rr.y : rr.x, acc[T + t], 0, 0, 0);
        }
      }
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int row = b0 + 4 * lk + j, i = 16 * t + lr;
        if (row < B && i < C) GV[((size_t)row * C + i) * K + k] = make_float2(acc[t][j], acc[T + t][j]);
      }
  }
}

// GR_k = V_k^H GU_k: rows i, columns [GRr | GRi] over o, contraction over
// [b re | b im] (four batch entries per step) with blocks
// [[GUr, GUi], [GUi, -GUr]]
template <int CP>
__global__ void __launch_bounds__(256) k_spec_mix_bwd_r_mfma(const float2* __restrict__ V,
                                                             const float2* __restrict__ GU, int B, int C,
                                                             int K, float2* __restrict__ GR) {
  constexpr int T = CP / 16;
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= K) return;
  const int lr = lane & 15, lk = lane >> 4;
  mf4 acc[T][2 * T];
#pragma unroll
  for (int m = 0; m < T; ++m)
#pragma unroll
    for (int t = 0; t < 2 * T; ++t) acc[m][t] = mf4{0.f, 0.f, 0.f, 0.f};
  for (int b0 = 0; b0 < B; b0 += 4) {
    const int b = b0 + lk;
    float2 va[T], gb[T];
#pragma unroll
    for (int m = 0; m < T; ++m) {
      const int i = 16 * m + lr;
      va[m] = (b < B && i < C) ? V[((size_t)b * C + i) * K + k] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int o = 16 * t + lr;
      gb[t] = (b < B && o < C) ? GU[((size_t)b * C + o) * K + k] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int part = 0; part < 2; ++part)
#pragma unroll
      for (int m = 0; m < T; ++m) {
        const float a = part == 0 ? va[m].x : va[m].y;
#pragma unroll
        for (int t = 0; t < T; ++t) {
          const float2 g = gb[t];
          acc[m][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, part == 0 ? g.x : g.y, acc[m][t], 0, 0, 0);
          acc[m][T + t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, part == 0 ? g.y : -g.x, acc[m][T + t], 0, 0, 0);
        }
      }
  }
#pragma unroll
  for (int m = 0; m < T; ++m)
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = 16 * m + 4 * lk + j, o = 16 * t + lr;
        if (i < C && o < C) GR[((size_t)k * C + i) * C + o] = make_float2(acc[m][t][j], acc[m][T + t][j]);
      }
}

// ---------------------------------------------------------------------------
// pointwise channel layers
// ---------------------------------------------------------------------------
__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.3989422804014327f;
}

// out[b][o][r] = sum_i Wm[o][i] in[b][i][r] + bias[o] (+ add[b][o][r]);
// act: 0 none, 1 gelu (pre-activation kept in zout when non-null).
// CIN/COUT > 0: compile-time channel counts (inputs stay in registers).
constexpr int PW_MAXC = 64;
template <int CIN, int COUT>
__global__ void __launch_bounds__(256) k_pointwise(const float* __restrict__ in, int Cin_,
                                                   const float* __restrict__ Wm,
                                                   const float* __restrict__ bias, int Cout_,
                                                   const float* __restrict__ add, size_t ng, int act,
                                                   float* __restrict__ zout, float* __restrict__ out) {
  const int Cin = CIN > 0 ? CIN : Cin_;
  const int Cout = COUT > 0 ? COUT : Cout_;
  __shared__ float sw[PW_MAXC * PW_MAXC];
  __shared__ float sb[PW_MAXC];
  for (int e = threadIdx.x; e < Cin * Cout; e += 256) sw[e] = Wm[e];
  for (int e = threadIdx.x; e < Cout; e += 256) sb[e] = bias ? bias[e] : 0.f;
  __syncthreads();
  const size_t r = (size_t)blockIdx.x * 256 + threadIdx.x;
  const int b = blockIdx.y;
  if (r >= ng) return;
  float xin[CIN > 0 ? CIN : PW_MAXC];
#pragma unroll
  for (int i = 0; i < (CIN > 0 ? CIN : PW_MAXC); ++i)
    if (i < Cin) xin[i] = in[((size_t)b * Cin + i) * ng + r];
#pragma unroll 4
  for (int o = 0; o < Cout; ++o) {
    float acc = sb[o];
#pragma unroll
    for (int i = 0; i < (CIN > 0 ? CIN : PW_MAXC); ++i)
      if (i < Cin) acc += sw[o * Cin + i] * xin[i];
    const size_t oi = ((size_t)b * Cout + o) * ng + r;
    if (add) acc += add[oi];
    if (zout) zout[oi] = acc;
    out[oi] = act ? gelu_f(acc) : acc;
  }
}

// gin[b][i][r] += sum_o Wm[o][i] gz[b][o][r]
template <int COUT>
__global__ void __launch_bounds__(256) k_pointwise_bwd(const float* __restrict__ gz, int Cout_,
                                                       const float* __restrict__ Wm, int Cin,
                                                       size_t ng, float* __restrict__ gin) {
  const int Cout = COUT > 0 ? COUT : Cout_;
  __shared__ float sw[PW_MAXC * PW_MAXC];
  for (int e = threadIdx.x; e < Cin * Cout; e += 256) sw[e] = Wm[e];
  __syncthreads();
  const size_t r = (size_t)blockIdx.x * 256 + threadIdx.x;
  const int b = blockIdx.y;
  if (r >= ng) return;
  float g[COUT > 0 ? COUT : PW_MAXC];
#pragma unroll
  for (int o = 0; o < (COUT > 0 ? COUT : PW_MAXC); ++o)
    if (o < Cout) g[o] = gz[((size_t)b * Cout + o) * ng + r];
#pragma unroll 4
  for (int i = 0; i < Cin; ++i) {
    float acc = 0.f;
#pragma unroll
    for (int o = 0; o < (COUT > 0 ? COUT : PW_MAXC); ++o)
      if (o < Cout) acc += sw[o * Cin + i] * g[o];
    gin[((size_t)b * Cin + i) * ng + r] += acc;
  }
}

// gz = gh * gelu'(z)   (in place on gh)
__global__ void k_gelu_bwd(float* __restrict__ gh, const float* __restrict__ z, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) gh[i] *= gelu_grad_f(z[i]);
}

// partial outer products over points:
//   part[blk][o][i] = sum_{r in blk} A[b][o][r] X[b][i][r],  part[blk][Co*Ci + o] = sum A
// X == nullptr: only the sums.  One block = 1024 points of one sample.
constexpr int OP_PTS = 1024, OP_TILE = 64;
__global__ void __launch_bounds__(256) k_outer_partial(const float* __restrict__ A, int Co,
                                                       const float* __restrict__ X, int Ci,
                                                       size_t ng, int nblk_per_b,
                                                       float* __restrict__ part) {
  __shared__ float sa[PW_MAXC][OP_TILE + 1];
  __shared__ float sx[PW_MAXC][OP_TILE + 1];
  const int b = blockIdx.x / nblk_per_b;
  const size_t r0 = (size_t)(blockIdx.x % nblk_per_b) * OP_PTS;
  const int tid = threadIdx.x;
  const int npair = Co * (X ? Ci : 0);
  float acc[16];
  float accs = 0.f;
  for (int q = 0; q < 16; ++q) acc[q] = 0.f;
  for (size_t t0 = r0; t0 < r0 + OP_PTS && t0 < ng; t0 += OP_TILE) {
    for (int e = tid; e < Co * OP_TILE; e += 256) {
      const int c = e / OP_TILE, p = e % OP_TILE;
      const size_t r = t0 + p;
      sa[c][p] = r < ng ? A[((size_t)b * Co + c) * ng + r] : 0.f;
    }
    if (X)
      for (int e = tid; e < Ci * OP_TILE; e += 256) {
        const int c = e / OP_TILE, p = e % OP_TILE;
        const size_t r = t0 + p;
        sx[c][p] = r < ng ? X[((size_t)b * Ci + c) * ng + r] : 0.f;
      }
    __syncthreads();
    for (int q = 0; q < 16; ++q) {
      const int pr = tid + q * 256;
      if (pr >= npair) break;
      const int o = pr / Ci, i = pr % Ci;
      float s = 0.f;
      for (int p = 0; p < OP_TILE; ++p) s += sa[o][p] * sx[i][p];
      acc[q] += s;
    }
    if (tid < Co) {
      float s = 0.f;
      for (int p = 0; p < OP_TILE; ++p) s += sa[tid][p];
      accs += s;
    }
    __syncthreads();
  }
  float* out = part + (size_t)blockIdx.x * (npair + Co);
  for (int q = 0; q < 16; ++q) {
    const int pr = tid + q * 256;
    if (pr < npair) out[pr] = acc[q];
  }
  if (tid < Co) out[npair + tid] = accs;
}

__global__ void k_sum_partials(const float* __restrict__ part, int nblk, int len, float* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= len) return;
  double s = 0;
  for (int k = 0; k < nblk; ++k) s += part[(size_t)k * len + j];
  out[j] = (float)s;
}

// gh[b][i][r] = Q[i] gy[b][r]
__global__ void k_proj_bwd(const float* __restrict__ gy, const float* __restrict__ Q, int C, size_t ng,
                           float* __restrict__ gh) {
  const size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (r >= ng) return;
  const float g = gy[(size_t)b * ng + r];
  for (int i = 0; i < C; ++i) gh[((size_t)b * C + i) * ng + r] = Q[i] * g;
}

// per-sample sums: sq[b] = sum (y - t)^2, tt[b] = sum t^2 (partials per block)
__global__ void __launch_bounds__(256) k_loss_partial(const float* __restrict__ y, const float* __restrict__ t,
                                                      size_t ng, int nblk_per_b, double* __restrict__ part) {
  const int b = blockIdx.x / nblk_per_b;
  const size_t r0 = (size_t)(blockIdx.x % nblk_per_b) * 4096;
  double a = 0, c = 0;
  for (size_t r = r0 + threadIdx.x; r < r0 + 4096 && r < ng; r += 256) {
    const double d = (double)y[(size_t)b * ng + r] - (double)t[(size_t)b * ng + r];
    const double tv = t[(size_t)b * ng + r];
    a += d * d;
    c += tv * tv;
  }
  __shared__ double ra[256], rc[256];
  ra[threadIdx.x] = a;
  rc[threadIdx.x] = c;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      ra[threadIdx.x] += ra[threadIdx.x + s];
      rc[threadIdx.x] += rc[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * (size_t)blockIdx.x] = ra[0];
    part[2 * (size_t)blockIdx.x + 1] = rc[0];
  }
}

// gy = (2/B) (y - t) / tn[b]
__global__ void k_loss_grad(const float* __restrict__ y, const float* __restrict__ t,
                            const double* __restrict__ tn, int B, size_t ng, float* __restrict__ gy) {
  const size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (r >= ng) return;
  const size_t i = (size_t)b * ng + r;
  gy[i] = (float)(2.0 / B * ((double)y[i] - (double)t[i]) / tn[b]);
}

// Adam on the FP32 master copy; the compute copy holds the BF16-rounded values
__global__ void k_adam(float* __restrict__ master, float* __restrict__ compute,
                       const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       size_t n, float lr, float b1, float b2, float eps, float c1, float c2,
                       int bf16) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float p = master[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  master[i] = p;
  compute[i] = bf16 ? (float)(__bf16)p : p;
}

__global__ void k_round_copy(const float* __restrict__ src, float* __restrict__ dst, size_t n, int bf16) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = bf16 ? (float)(__bf16)src[i] : src[i];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int N>
struct FnoLaunch {
  static hipError_t fwd(const float* in, int F, const float2* tw, int m, int ck, float2* work,
                        float2* V, hipStream_t st) {
    const size_t sm = sizeof(float2) * (N * fplane_stride<N>() + N);
    hipLaunchKernelGGL(k_fno_yz_fwd_t<N>, dim3(N, F), dim3(256), sm, st, in, work, tw);
    const int ncol = 2 * m * m;
    hipLaunchKernelGGL(k_fno_x_gather<N>, dim3((ncol + KC - 1) / KC, F), dim3(256), 0, st, work,
                       tw, m, ck, V);
    return hipGetLastError();
  }
  static hipError_t inv(const float2* U, int F, const float2* tw, int m, int ck, float2* work,
                        float* out, int accumulate, hipStream_t st) {
    const size_t ng = (size_t)N * N * N;
    hipError_t e = hipMemsetAsync(work, 0, sizeof(float2) * ng * F, st);
    if (e != hipSuccess) return e;
    const int ncol = 2 * m * m;
    hipLaunchKernelGGL(k_fno_x_scatter<N>, dim3((ncol + KC - 1) / KC, F), dim3(256), 0, st, U, tw,
                       m, ck, work);
    const size_t sm = sizeof(float2) * (N * fplane_stride<N>() + N);
    hipLaunchKernelGGL(k_fno_yz_inv<N>, dim3(N, F), dim3(256), sm, st, work, tw, out, accumulate);
    return hipGetLastError();
  }
  static void configure() {
    const int sm = (int)(sizeof(float2) * (N * fplane_stride<N>() + N));
    (void)hipFuncSetAttribute((const void*)k_fno_yz_fwd_t<N>, hipFuncAttributeMaxDynamicSharedMemorySize, sm);
    (void)hipFuncSetAttribute((const void*)k_fno_yz_inv<N>, hipFuncAttributeMaxDynamicSharedMemorySize, sm);
  }
};

bool fno_grid_supported(int n) { return n == 16 || n == 32 || n == 64; }

#define FNO_DISPATCH(n, CALL)                 \
  switch (n) {                                \
    case 16: return FnoLaunch<16>::CALL;      \
    case 32: return FnoLaunch<32>::CALL;      \
    case 64: return FnoLaunch<64>::CALL;      \
    default: return hipErrorInvalidValue;     \
  }

hipError_t fno_fft_fwd(int n, const float* in, int F, const float2* tw, int m, int ck, float2* work,
                       float2* V, hipStream_t st) {
  FNO_DISPATCH(n, fwd(in, F, tw, m, ck, work, V, st));
}
hipError_t fno_fft_inv(int n, const float2* U, int F, const float2* tw, int m, int ck, float2* work,
                       float* out, int accumulate, hipStream_t st) {
  FNO_DISPATCH(n, inv(U, F, tw, m, ck, work, out, accumulate, st));
}
void fno_configure(int n) {
  switch (n) {
    case 16: FnoLaunch<16>::configure(); break;
    case 32: FnoLaunch<32>::configure(); break;
    case 64: FnoLaunch<64>::configure(); break;
    default: break;
  }
}

static inline unsigned nb(size_t n) { return (unsigned)((n + 255) / 256); }

// path 0: the matrix-core products for up to 32 channels (the vector-FMA
// ones above beyond); path 1: the vector-FMA products only
hipError_t fno_spec_mix(const float2* V, const float2* R, int B, int C, int K, float2* U, int path,
                        hipStream_t st) {
  const int g_spec_mix_path = path;
  const unsigned nw = (unsigned)((K + 3) / 4);
  if (g_spec_mix_path == 0 && C <= 16)
    hipLaunchKernelGGL(k_spec_mix_mfma<16>, dim3(nw), dim3(256), 0, st, V, R, B, C, K, U);
  else if (g_spec_mix_path == 0 && C <= 32)
    hipLaunchKernelGGL(k_spec_mix_mfma<32>, dim3(nw), dim3(256), 0, st, V, R, B, C, K, U);
  else
    hipLaunchKernelGGL(k_spec_mix, dim3(nb((size_t)B * K * C)), dim3(256), 0, st, V, R, B, C, K, U);
  return hipGetLastError();
}
hipError_t fno_spec_mix_bwd(const float2* V, const float2* GU, const float2* R, int B, int C, int K,
                            float2* GV, float2* GR, int path, hipStream_t st) {
  const int g_spec_mix_path = path;
  const unsigned nw = (unsigned)((K + 3) / 4);
  if (g_spec_mix_path == 0 && C <= 16) {
    hipLaunchKernelGGL(k_spec_mix_bwd_v_mfma<16>, dim3(nw), dim3(256), 0, st, GU, R, B, C, K, GV);
    hipLaunchKernelGGL(k_spec_mix_bwd_r_mfma<16>, dim3(nw), dim3(256), 0, st, V, GU, B, C, K, GR);
  } else if (g_spec_mix_path == 0 && C <= 32) {
    hipLaunchKernelGGL(k_spec_mix_bwd_v_mfma<32>, dim3(nw), dim3(256), 0, st, GU, R, B, C, K, GV);
    hipLaunchKernelGGL(k_spec_mix_bwd_r_mfma<32>, dim3(nw), dim3(256), 0, st, V, GU, B, C, K, GR);
  } else {
    hipLaunchKernelGGL(k_spec_mix_bwd_v, dim3(nb((size_t)B * K * C)), dim3(256), 0, st, GU, R, B, C, K, GV);
    hipLaunchKernelGGL(k_spec_mix_bwd_r, dim3(nb((size_t)K * C * C)), dim3(256), 0, st, V, GU, B, C, K, GR);
  }
  return hipGetLastError();
}
hipError_t fno_pointwise(const float* in, int Cin, const float* Wm, const float* bias, int Cout,
                         const float* add, int B, size_t ng, int act, float* zout, float* out,
                         hipStream_t st) {
  if (Cin > PW_MAXC || Cout > PW_MAXC) return hipErrorInvalidValue;
  const dim3 g(nb(ng), B);
  if (Cin == 3 && Cout == 32)
    hipLaunchKernelGGL((k_pointwise<3, 32>), g, dim3(256), 0, st, in, Cin, Wm, bias, Cout, add, ng, act, zout, out);
  else if (Cin == 32 && Cout == 32)
    hipLaunchKernelGGL((k_pointwise<32, 32>), g, dim3(256), 0, st, in, Cin, Wm, bias, Cout, add, ng, act, zout, out);
  else if (Cin == 32 && Cout == 1)
    hipLaunchKernelGGL((k_pointwise<32, 1>), g, dim3(256), 0, st, in, Cin, Wm, bias, Cout, add, ng, act, zout, out);
  else
    hipLaunchKernelGGL((k_pointwise<0, 0>), g, dim3(256), 0, st, in, Cin, Wm, bias, Cout, add, ng, act, zout, out);
  return hipGetLastError();
}
hipError_t fno_pointwise_bwd(const float* gz, int Cout, const float* Wm, int Cin, int B, size_t ng,
                             float* gin, hipStream_t st) {
  if (Cin > PW_MAXC || Cout > PW_MAXC) return hipErrorInvalidValue;
  if (Cout == 32)
    hipLaunchKernelGGL((k_pointwise_bwd<32>), dim3(nb(ng), B), dim3(256), 0, st, gz, Cout, Wm, Cin, ng, gin);
  else
    hipLaunchKernelGGL((k_pointwise_bwd<0>), dim3(nb(ng), B), dim3(256), 0, st, gz, Cout, Wm, Cin, ng, gin);
  return hipGetLastError();
}
hipError_t fno_gelu_bwd(float* gh, const float* z, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_gelu_bwd, dim3(nb(n)), dim3(256), 0, st, gh, z, n);
  return hipGetLastError();
}
size_t fno_outer_part_len(int Co, int Ci, int B, size_t ng) {
  const size_t nblk = (size_t)B * ((ng + OP_PTS - 1) / OP_PTS);
  return (nblk + 1) * (size_t)(Co * Ci + Co);   // partials plus the reduced row
}
// gW[o][i] (Co x Ci) and gb[o] = sums over points of A x X, A
hipError_t fno_outer(const float* A, int Co, const float* X, int Ci, int B, size_t ng, float* part,
                     float* gW, float* gb, hipStream_t st) {
  if (Co > PW_MAXC || Ci > PW_MAXC || Co * (X ? Ci : 0) > 16 * 256) return hipErrorInvalidValue;
  const int nbb = (int)((ng + OP_PTS - 1) / OP_PTS);
  const int nblk = B * nbb;
  hipLaunchKernelGGL(k_outer_partial, dim3(nblk), dim3(256), 0, st, A, Co, X, Ci, ng, nbb, part);
  const int npair = Co * (X ? Ci : 0);
  const int len = npair + Co;
  // reduce into a contiguous [npair | Co] block, then split
  float* red = part + (size_t)nblk * len;
  hipLaunchKernelGGL(k_sum_partials, dim3(nb(len)), dim3(256), 0, st, part, nblk, len, red);
  if (npair && gW) {
    hipError_t e = hipMemcpyAsync(gW, red, sizeof(float) * npair, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
  }
  if (gb) {
    hipError_t e = hipMemcpyAsync(gb, red + npair, sizeof(float) * Co, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}
hipError_t fno_proj_bwd(const float* gy, const float* Q, int C, int B, size_t ng, float* gh, hipStream_t st) {
  hipLaunchKernelGGL(k_proj_bwd, dim3(nb(ng), B), dim3(256), 0, st, gy, Q, C, ng, gh);
  return hipGetLastError();
}
int fno_loss_blocks(size_t ng) { return (int)((ng + 4095) / 4096); }
hipError_t fno_loss_partial(const float* y, const float* t, int B, size_t ng, double* part, hipStream_t st) {
  const int nbb = fno_loss_blocks(ng);
  hipLaunchKernelGGL(k_loss_partial, dim3(B * nbb), dim3(256), 0, st, y, t, ng, nbb, part);
  return hipGetLastError();
}
hipError_t fno_loss_grad(const float* y, const float* t, const double* tn, int B, size_t ng, float* gy,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_loss_grad, dim3(nb(ng), B), dim3(256), 0, st, y, t, tn, B, ng, gy);
  return hipGetLastError();
}
hipError_t fno_adam(float* master, float* compute, const float* g, float* m, float* v, size_t n,
                    float lr, float b1, float b2, float eps, int step, int bf16, hipStream_t st) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(nb(n)), dim3(256), 0, st, master, compute, g, m, v, n, lr, b1, b2,
                     eps, c1, c2, bf16);
  return hipGetLastError();
}
hipError_t fno_round_copy(const float* src, float* dst, size_t n, int bf16, hipStream_t st) {
  hipLaunchKernelGGL(k_round_copy, dim3(nb(n)), dim3(256), 0, st, src, dst, n, bf16);
  return hipGetLastError();
}

// training batches under the symmetries of the cube: output point (o0, o1,
// o2), after the flips o_k -> n - 1 - o_k, reads input point i with
// i[perm[k]] = o_k
__global__ void k_gather_sym(const float* __restrict__ src, const int* __restrict__ idx, int C, int n,
                             int p0, int p1, int p2, int fmask, float* __restrict__ dst) {
  const size_t ng = (size_t)n * n * n;
  const size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= ng) return;
  const int c = blockIdx.y, b = blockIdx.z;
  int oc[3] = {(int)(o / ((size_t)n * n)), (int)((o / n) % n), (int)(o % n)};
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if ((fmask >> k) & 1) oc[k] = n - 1 - oc[k];
  int ic[3];
  ic[p0] = oc[0];
  ic[p1] = oc[1];
  ic[p2] = oc[2];
  const size_t i = ((size_t)ic[0] * n + ic[1]) * n + ic[2];
  dst[((size_t)b * C + c) * ng + o] = src[((size_t)idx[b] * C + c) * ng + i];
}

hipError_t fno_gather_sym(const float* src, const int* idx, int B, int C, int n, const int perm[3],
                          int flip_mask, float* dst, hipStream_t st) {
  const size_t ng = (size_t)n * n * n;
  hipLaunchKernelGGL(k_gather_sym, dim3((unsigned)((ng + 255) / 256), C, B), dim3(256), 0, st, src, idx, C, n,
                     perm[0], perm[1], perm[2], flip_mask, dst);
  return hipGetLastError();
}

}  // namespace bse
