// Shared pieces of the BF16x3 matrix-core kernels (gfx950): 128 x 128
// tiles staged in LDS in stages of 32 K values, hi/lo splits, and the
// XCD-aware tile numbering.
//
// v_mfma_f32_16x16x32_bf16: lane l supplies row (l%16) of A and column (l%16)
// of B, each as 8 consecutive K values starting at 8(l/16); the 16x16 result
// sits in lane l as D[4(l/16)+v][l%16], v = 0..3.
#pragma once
#include <hip/hip_runtime.h>

namespace bse {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int XT = 128;       // tile rows and columns
constexpr int XK = 32;        // K per stage: one 16x16x32 step
constexpr int XKP = XK + 8;   // padded LDS row in bf16 (80 bytes, 16-byte aligned)

__device__ __forceinline__ void split_hl(float x, unsigned short& h, unsigned short& l) {
  const __bf16 bh = (__bf16)x;
  const __bf16 bl = (__bf16)(x - (float)bh);
  h = __builtin_bit_cast(unsigned short, bh);
  l = __builtin_bit_cast(unsigned short, bl);
}

// Workgroup ids are dealt round-robin to the 8 XCDs; renumber them so that
// each XCD works through a contiguous range of tiles (nb is a multiple of 8)
// and tiles that share an operand tile share that XCD's L2.
__device__ __forceinline__ unsigned xcd_tile(unsigned id, unsigned nb) {
  return (id & 7u) * (nb >> 3) + (id >> 3);
}

// One stage of MFMA work on staged 128-row tiles: the 32 K values starting
// at koff of LDS rows of P bf16; wave (wm, wn) owns a 64 x 64 block of
// 4 x 4 result tiles.
template <int P>
__device__ __forceinline__ void mma_stage(const __bf16 (*Ah)[P], const __bf16 (*Al)[P],
                                          const __bf16 (*Bh)[P], const __bf16 (*Bl)[P],
                                          int lane, int wm, int wn, f4 (&acc)[4][4], int koff = 0) {
  const int kk = koff + 8 * (lane >> 4);
  bf8 ah[4], al[4], bh[4], bl[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = wm * 64 + i * 16 + (lane & 15);
    ah[i] = *reinterpret_cast<const bf8*>(&Ah[row][kk]);
    al[i] = *reinterpret_cast<const bf8*>(&Al[row][kk]);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int col = wn * 64 + j * 16 + (lane & 15);
    bh[j] = *reinterpret_cast<const bf8*>(&Bh[col][kk]);
    bl[j] = *reinterpret_cast<const bf8*>(&Bl[col][kk]);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
    }
}

// x = hi + lo from an FP64 value: hi = bf16(x), lo = bf16(x - hi)
__device__ __forceinline__ void split_hl64(double x, unsigned short& h, unsigned short& l) {
  const __bf16 bh = (__bf16)(float)x;
  const __bf16 bl = (__bf16)(float)(x - (double)(float)bh);
  h = __builtin_bit_cast(unsigned short, bh);
  l = __builtin_bit_cast(unsigned short, bl);
}

}  // namespace bse
