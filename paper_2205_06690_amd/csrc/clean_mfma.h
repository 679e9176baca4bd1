// Matrix-core kernels of the cleaning projection (three-term BF16 split,
// FP32 tile sums, FP64 sums over point chunks).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>

namespace bse {
constexpr int CLEAN_CHUNK_E = 1024;   // points per split-K chunk, the L unperturbed orbitals
// points per split-K chunk of the perturbed set's coefficient GEMM: about
// 2048 blocks of 128 x 128 tiles whatever the batch and grid
int clean_chunk_d(int F, int S, size_t ng);

// mid-step to end-of-step conversion applied on the fly: d <- ph (d - i hdt u_b H_l)
struct MidArgs {
  int on;
  const float* u;      // [B][ng]
  const float2* H;     // [L][ng]
  const float2* ph;    // [ng]
  int L;
  float half_dt;
  size_t ng;
};

// occupied orbitals split into bf16 pairs (bit patterns), in the two layouts
// the GEMMs read: h/l [S][ng] and th/tl [ng][Sp], Sp = S rounded up to 32
struct PhiSplit {
  const unsigned short *h, *l, *th, *tl;
  int S, Sp;
};
struct PhiSplitBufs {
  unsigned short *h, *l, *th, *tl;
};
int clean_sp(int S);
hipError_t launch_phi_split(const float* phi, int S, size_t ng, PhiSplitBufs b, hipStream_t st);

// coef[f][s] = dv sum_r phi_s d_f (s < S); with gpart non-null also
// coef[f][S] = dv <E_l, d_f> (gpart: [F][nchunk] partials).  mid.on requires
// gpart.  ng and chunk must be multiples of 32.
hipError_t launch_coef_x3(const float2* d, int F, const PhiSplit& ps, size_t ng, int chunk,
                          float* part, double dv, double2* coef, hipStream_t st, const MidArgs& mid,
                          const float2* E, int L, double2* gpart);
// d_f -= sum_s C[f][s] phi_s + c_f E_l (after the end of the step when mid.on);
// scratch holds the split coefficient rows (clean_scratch_floats)
hipError_t launch_update_x3(float2* d, int F, const PhiSplit& ps, const float2* E, int L, size_t ng,
                            const double2* coef, float* scratch, hipStream_t st, const MidArgs& mid);
// for batches of up to F = B L fields
size_t clean_scratch_floats(int F, int L, int S, size_t ng);
// for batches of up to F = B L fields
size_t edot_part_entries(int F, int L, int S, size_t ng);
}  // namespace bse
