// Grid contractions of the Tamm-Dancoff matrix (Eq. 1) on the gfx950 matrix
// cores: C[m][n] = scale sum_r A[m][r] B[n][r] over the grid points r, with
// both operands split once from FP64 into bf16 pairs x = hi + lo and the
// three-term product a_hi b_hi + a_hi b_lo + a_lo b_hi.
//
//   exchange (ia|jb): A = rho_ia = phi_i phi_a, B = v[rho_jb]
//   direct (ab|W|ij): A = phi_a phi_b,          B = W_ij
//
// Tiles of 128 x 128 outputs over chunks of the grid (split K), staged in
// LDS 64 points at a time with the next stage's loads in flight; FP32 sums
// per tile and chunk, FP64 sums over chunks.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include "contract_mfma.h"
#include "mfma_tiles.h"

#include <algorithm>

namespace bse {

// hi/lo of x [n] (FP64)
__global__ void k_split64(const double* __restrict__ x, size_t n, unsigned short* __restrict__ h,
                          unsigned short* __restrict__ l) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    split_hl64(x[i], h[i], l[i]);
}

// hi/lo of the products phi_p phi_q (FP64) for the K index pairs pq[K][2]
__global__ void k_products_split(const double* __restrict__ phi, const int* __restrict__ pq, int K,
                                 size_t ng, unsigned short* __restrict__ h,
                                 unsigned short* __restrict__ l) {
  const size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (r >= ng || k >= K) return;
  const int p = pq[2 * k], q = pq[2 * k + 1];
  split_hl64(phi[(size_t)p * ng + r] * phi[(size_t)q * ng + r], h[(size_t)k * ng + r],
             l[(size_t)k * ng + r]);
}

// One 32-point step of a wave's 64 x 64 outputs: the A fragments of its four
// row blocks stay in registers while the B fragments stream, one column block
// at a time, so that fewer registers are live than with all of B loaded (two
// blocks per SIMD).  Each accumulator sees the same three products in the same
// order as in mma_stage.
template <int P>
__device__ __forceinline__ void mma_step_bstream(const __bf16 (*Ah)[P], const __bf16 (*Al)[P],
                                                 const __bf16 (*Bh)[P], const __bf16 (*Bl)[P],
                                                 int lane, int wm, int wn, f4 (&acc)[4][4], int ko) {
  const int kk = ko + 8 * (lane >> 4);
  bf8 fah[4], fal[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = wm * 64 + i * 16 + (lane & 15);
    fah[i] = *reinterpret_cast<const bf8*>(&Ah[row][kk]);
    fal[i] = *reinterpret_cast<const bf8*>(&Al[row][kk]);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int col = wn * 64 + j * 16 + (lane & 15);
    const bf8 fbh = *reinterpret_cast<const bf8*>(&Bh[col][kk]);
    const bf8 fbl = *reinterpret_cast<const bf8*>(&Bl[col][kk]);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fal[i], fbh, acc[i][j], 0, 0, 0);
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fah[i], fbl, acc[i][j], 0, 0, 0);
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fah[i], fbh, acc[i][j], 0, 0, 0);
    }
  }
}

// part[kc][m][n] = sum over chunk kc of A[m][r] B[n][r], staged KS grid
// points at a time.  Tile order (with remap): column tile fastest, then row
// tile, then chunk, renumbered so that each XCD works through a contiguous
// range and the tiles of one chunk share their row and column panels in L2.
template <int KS>
__global__ void __launch_bounds__(256, 2) k_contract_x3(const unsigned short* __restrict__ ah,
                                                     const unsigned short* __restrict__ al, int M,
                                                     const unsigned short* __restrict__ bh,
                                                     const unsigned short* __restrict__ bl, int N,
                                                     size_t K, size_t chunk, int ntm, int ntn,
                                                     unsigned ntile, int remap,
                                                     float* __restrict__ part) {
  constexpr int P = KS + 8;            // padded LDS row (bf16), a multiple of 8
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_c[];
  __bf16 (*Ah)[P] = reinterpret_cast<__bf16 (*)[P]>(smem_c);
  __bf16 (*Al)[P] = Ah + XT;
  __bf16 (*Bh)[P] = Al + XT;
  __bf16 (*Bl)[P] = Bh + XT;
  const unsigned t = remap ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
  if (t >= ntile) return;
  const int tn = (int)(t % ntn), tm = (int)((t / ntn) % ntm), kc = (int)(t / ((unsigned)ntn * ntm));
  const int m0 = tm * XT, n0 = tn * XT;
  const size_t k0 = (size_t)kc * chunk, k1 = min(K, k0 + chunk);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  // loader: QR lanes per row, each one 16-byte piece of the row's KS
  // values, so that a load instruction covers whole 128-byte lines of
  // RPP rows; pass c takes rows r0 + RPP c of the 2 XT staged rows (A's,
  // then B's).  Rows past M (columns past N) load the last row: their
  // outputs are never stored.
  constexpr int QR = KS / 8, RPP = 256 / QR, NC = 2 * XT / RPP;
  static_assert(2 * XT % RPP == 0 && XT % RPP == 0, "passes fill A's rows, then B's");
  const int qp = tid % QR, r0 = tid / QR;
  const unsigned short* gh[NC];
  const unsigned short* gl[NC];
  __bf16* lh[NC];
  __bf16* ll[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int r = r0 + RPP * c;
    if (r < XT) {
      const size_t m = (size_t)min(M - 1, m0 + r);
      gh[c] = ah + m * K + 8 * qp;
      gl[c] = al + m * K + 8 * qp;
      lh[c] = &Ah[r][8 * qp];
      ll[c] = &Al[r][8 * qp];
    } else {
      const size_t n = (size_t)min(N - 1, n0 + r - XT);
      gh[c] = bh + n * K + 8 * qp;
      gl[c] = bl + n * K + 8 * qp;
      lh[c] = &Bh[r - XT][8 * qp];
      ll[c] = &Bl[r - XT][8 * qp];
    }
  }
  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  typedef unsigned u4v __attribute__((ext_vector_type(4)));
  u4v rh[NC], rl[NC];
  auto load = [&](size_t kb) __attribute__((always_inline)) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      rh[c] = *reinterpret_cast<const u4v*>(gh[c] + kb);
      rl[c] = *reinterpret_cast<const u4v*>(gl[c] + kb);
    }
  };
  auto store = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      *reinterpret_cast<u4v*>(lh[c]) = rh[c];
      *reinterpret_cast<u4v*>(ll[c]) = rl[c];
    }
  };
  load(k0);
  for (size_t kb = k0; kb < k1; kb += KS) {
    __syncthreads();
    store();
    __syncthreads();
    if (kb + KS < k1) load(kb + KS);
#pragma unroll
    for (int ko = 0; ko < KS; ko += XK) mma_step_bstream<P>(Ah, Al, Bh, Bl, lane, wm, wn, acc, ko);
  }
  float* out = part + (size_t)kc * M * N;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm * 64 + i * 16 + 4 * (lane >> 4) + v;
        const int n = n0 + wn * 64 + j * 16 + (lane & 15);
        if (m < M && n < N) out[(size_t)m * N + n] = acc[i][j][v];
      }
}

// C[m][n] = scale sum_kc part[kc][m][n] in FP64.  A block sums 32 outputs in
// CR_SL slices of the chunks (slice j: kc = j, j + CR_SL, ...) and adds the
// slices in order: a fixed summation order with enough loads in flight to
// stream the partials.
constexpr int CR_SL = 8;
__global__ void __launch_bounds__(256) k_contract_reduce(const float* __restrict__ part, int nchunk,
                                                         size_t MN, double scale,
                                                         double* __restrict__ C) {
  __shared__ double red[CR_SL][32];
  const int o = threadIdx.x & 31, j = threadIdx.x >> 5;
  const size_t i = (size_t)blockIdx.x * 32 + o;
  double acc = 0;
  if (i < MN)
    for (int k = j; k < nchunk; k += CR_SL) acc += part[(size_t)k * MN + i];
  red[j][o] = acc;
  __syncthreads();
  if (j == 0 && i < MN) {
    double s = 0;
#pragma unroll
    for (int q = 0; q < CR_SL; ++q) s += red[q][o];
    C[i] = s * scale;
  }
}

static unsigned round8u(unsigned n) { return (n + 7u) & ~7u; }

template <int KS> constexpr size_t contract_lds() { return 4ull * XT * (KS + 8) * sizeof(unsigned short); }

// Stages of 64 points; chunks of 2048 points keep the row and column panels
// of the tiles running together small enough to be served from cache (at
// M = N = 800, K = 112^3: 9.5 ms with 33472-point chunks and 32-point
// stages, 7.1 ms with 2048 and 64).
constexpr int CK_STAGE = 64;
constexpr size_t CK_CHUNK = 2048;

void contract_plan(int M, int N, size_t K, size_t* chunk, int* nchunk) {
  (void)M;
  (void)N;
  const size_t c = std::min(K, CK_CHUNK);
  *chunk = c;
  *nchunk = (int)((K + c - 1) / c);
}

size_t contract_part_floats(int M, int N, size_t K) {
  size_t c;
  int nc;
  contract_plan(M, N, K, &c, &nc);
  return (size_t)nc * M * N;
}

hipError_t launch_split64(const double* x, size_t n, unsigned short* h, unsigned short* l,
                          hipStream_t st) {
  const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_split64, dim3(blocks), dim3(256), 0, st, x, n, h, l);
  return hipGetLastError();
}

hipError_t launch_products_split(const double* phi, const int* pq, int K, size_t ng, unsigned short* h,
                                 unsigned short* l, hipStream_t st) {
  hipLaunchKernelGGL(k_products_split, dim3((unsigned)((ng + 255) / 256), K), dim3(256), 0, st, phi, pq,
                     K, ng, h, l);
  return hipGetLastError();
}

hipError_t launch_contract_x3(const unsigned short* ah, const unsigned short* al, int M,
                              const unsigned short* bh, const unsigned short* bl, int N, size_t K,
                              double scale, float* part, double* C, hipStream_t st,
                              const LaunchEvents* ev, const LaunchEvents* ev_reduce) {
  if (M <= 0 || N <= 0 || K % CK_STAGE != 0) return hipErrorInvalidValue;
  size_t chunk;
  int nchunk;
  contract_plan(M, N, K, &chunk, &nchunk);
  const int ntm = (M + XT - 1) / XT, ntn = (N + XT - 1) / XT;
  const unsigned ntile = (unsigned)ntm * ntn * nchunk;
  (void)hipFuncSetAttribute((const void*)k_contract_x3<CK_STAGE>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)contract_lds<CK_STAGE>());
  if (ev)
    hipExtLaunchKernelGGL(k_contract_x3<CK_STAGE>, dim3(round8u(ntile)), dim3(256),
                          (uint32_t)contract_lds<CK_STAGE>(), st, ev->start, ev->stop, 0, ah, al, M, bh, bl,
                          N, K, chunk, ntm, ntn, ntile, 1, part);
  else
    hipLaunchKernelGGL(k_contract_x3<CK_STAGE>, dim3(round8u(ntile)), dim3(256), contract_lds<CK_STAGE>(),
                       st, ah, al, M, bh, bl, N, K, chunk, ntm, ntn, ntile, 1, part);
  const size_t MN = (size_t)M * N;
  const dim3 gr((unsigned)((MN + 31) / 32));
  if (ev_reduce)
    hipExtLaunchKernelGGL(k_contract_reduce, gr, dim3(256), 0, st, ev_reduce->start, ev_reduce->stop, 0, part,
                          nchunk, MN, scale, C);
  else
    hipLaunchKernelGGL(k_contract_reduce, gr, dim3(256), 0, st, part, nchunk, MN, scale, C);
  return hipGetLastError();
}

}  // namespace bse
