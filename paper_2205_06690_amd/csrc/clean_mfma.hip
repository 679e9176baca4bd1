// Cleaning projection of the perturbed stochastic orbitals (Eq. 15,
// linearised) on the gfx950 matrix cores, in three-term BF16 arithmetic.
//
//   coefficients  C[f][s] = h^3 sum_r phi_s(r) d_f(r)       (split-K GEMM)
//   update        d_f(r) -= sum_s C[f][s] phi_s(r) + c_f E_l(r)
//
// Complex fields are viewed as two real rows (2f: real part, 2f+1:
// imaginary part); the occupied orbitals are real, so both products are real
// GEMMs: rows x states over K = grid points, and rows x points over
// K = states.  Each FP32 operand x is split as x = hi + lo with hi = bf16(x),
// lo = bf16(x - hi), and a.b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi (the
// dropped lo.lo term is ~2^-16 of the product); products accumulate in FP32
// per tile, tiles over K chunks in FP64.  The occupied orbitals are split
// once per orbital set, in both layouts the two GEMMs read.
//
// v_mfma_f32_16x16x32_bf16: lane l supplies row (l%16) of A and column (l%16)
// of B, each as 8 consecutive K values starting at 8(l/16); the 16x16 result
// sits in lane l as D[4(l/16)+v][l%16], v = 0..3.
//
// The end of the time step (d <- Ph (d - i dt/2 u_b H_l), Strang splitting)
// is applied on the fly by the coefficient GEMM's loader and again by the
// update's epilogue, so the perturbed set is read once by each GEMM and
// written once.
#include <hip/hip_runtime.h>

#include "clean_mfma.h"
#include "mfma_tiles.h"

#include <algorithm>

namespace bse {

int clean_sp(int S) { return (S + XK - 1) / XK * XK; }

__device__ __forceinline__ float2 cm(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// end of the step for one value: ph (v - i hdt u h)
__device__ __forceinline__ float2 finish1(float2 v, float2 h, float u, float2 p, float hdt) {
  const float cu = hdt * u;
  return cm(p, make_float2(v.x + cu * h.y, v.y - cu * h.x));
}

__device__ __forceinline__ float2 finish_mid(const MidArgs& m, int f, size_t r, float2 v) {
  const int b = f / m.L, l = f % m.L;
  return finish1(v, m.H[(size_t)l * m.ng + r], m.u[(size_t)b * m.ng + r], m.ph[r], m.half_dt);
}


// phi [S][ng] FP32 -> hi/lo in [S][ng] and, zero-padded to Sp states, [ng][Sp]
__global__ void k_phi_split(const float* __restrict__ phi, int S, int Sp, size_t ng,
                            unsigned short* __restrict__ h, unsigned short* __restrict__ l,
                            unsigned short* __restrict__ th, unsigned short* __restrict__ tl) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ng * (size_t)Sp) return;
  const size_t r = i / Sp;
  const int s = (int)(i % Sp);
  const float x = s < S ? phi[(size_t)s * ng + r] : 0.f;
  unsigned short a, b;
  split_hl(x, a, b);
  th[i] = a;
  tl[i] = b;
  if (s < S) {
    h[(size_t)s * ng + r] = a;
    l[(size_t)s * ng + r] = b;
  }
}

// part[kc][row][s] (row < 2F, s < S) = sum over chunk kc of D[row][r] phi_s(r),
// D = d, finished on the fly when MID.  With EDOT the column-tile-0 blocks
// also accumulate <E_l, d_f> over their chunk into gpart[f][kc] (E = Ph H_l
// computed in registers when MID, read from E otherwise).  Global loads of
// stage k+1 are in flight during the matrix-core work of stage k.
template <bool MID, bool EDOT>
__global__ void __launch_bounds__(256) k_coef_x3(const float2* __restrict__ d, int F, PhiSplit ps,
                                                 size_t ng, int chunk, int nrt, int nct, int nchunk,
                                                 unsigned ntile, MidArgs mid,
                                                 const float2* __restrict__ E, int L,
                                                 float* __restrict__ part,
                                                 double2* __restrict__ gpart) {
  __shared__ __attribute__((aligned(16))) __bf16 Ah[XT][XKP];
  __shared__ __attribute__((aligned(16))) __bf16 Al[XT][XKP];
  __shared__ __attribute__((aligned(16))) __bf16 Bh[XT][XKP];
  __shared__ __attribute__((aligned(16))) __bf16 Bl[XT][XKP];
  const unsigned t = xcd_tile(blockIdx.x, gridDim.x);
  if (t >= ntile) return;
  // column tile fastest: the column tiles of one row tile run together on one
  // XCD and read its d tile (and the finish inputs) from L2, not HBM
  const int ct = (int)(t % nct), rt = (int)((t / nct) % nrt), kc = (int)(t / ((unsigned)nrt * nct));
  const int R = 2 * F, S = ps.S;
  const int r0 = rt * XT, s0 = ct * XT, f0 = r0 / 2;
  const size_t k0 = (size_t)kc * chunk;
  const size_t k1 = min(ng, k0 + (size_t)chunk);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  const bool do_e = EDOT && ct == 0;
  // loader: fields f0 + qa + 16i at points pa, pa+1; state s0 + sb at points hb..hb+15
  const int qa = tid >> 4, pa = (tid & 15) * 2;
  const int sb = tid >> 1, hb = (tid & 1) * 16;
  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  float4 ra[4], rh[4];
  float2 ru[4];
  float4 rp = make_float4(0.f, 0.f, 0.f, 0.f);
  uint4 rbh[2], rbl[2];
  double ex[4], ey[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) ex[i] = ey[i] = 0.0;
  const uint4 z4 = make_uint4(0u, 0u, 0u, 0u);
  auto load = [&](size_t kb) {
    const size_t r = kb + pa;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int f = f0 + qa + 16 * i;
      if (f < F) {
        ra[i] = *reinterpret_cast<const float4*>(d + (size_t)f * ng + r);
        if (MID) {
          rh[i] = *reinterpret_cast<const float4*>(mid.H + (size_t)(f % L) * ng + r);
          ru[i] = *reinterpret_cast<const float2*>(mid.u + (size_t)(f / L) * ng + r);
        } else if (do_e) {
          rh[i] = *reinterpret_cast<const float4*>(E + (size_t)(f % L) * ng + r);
        }
      } else {
        ra[i] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
    if (MID) rp = *reinterpret_cast<const float4*>(mid.ph + r);
    const int s = s0 + sb;
    if (s < S) {
      const uint4* qh = reinterpret_cast<const uint4*>(ps.h + (size_t)s * ng + kb + hb);
      const uint4* ql = reinterpret_cast<const uint4*>(ps.l + (size_t)s * ng + kb + hb);
      rbh[0] = qh[0];
      rbh[1] = qh[1];
      rbl[0] = ql[0];
      rbl[1] = ql[1];
    } else {
      rbh[0] = rbh[1] = rbl[0] = rbl[1] = z4;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int ff = qa + 16 * i;
      const int f = f0 + ff;
      float2 v0 = make_float2(ra[i].x, ra[i].y), v1 = make_float2(ra[i].z, ra[i].w);
      if (f < F) {
        float2 e0, e1;
        if (MID) {
          const float2 h0 = make_float2(rh[i].x, rh[i].y), h1 = make_float2(rh[i].z, rh[i].w);
          const float2 p0 = make_float2(rp.x, rp.y), p1 = make_float2(rp.z, rp.w);
          v0 = finish1(v0, h0, ru[i].x, p0, mid.half_dt);
          v1 = finish1(v1, h1, ru[i].y, p1, mid.half_dt);
          e0 = cm(p0, h0);
          e1 = cm(p1, h1);
        } else {
          e0 = make_float2(rh[i].x, rh[i].y);
          e1 = make_float2(rh[i].z, rh[i].w);
        }
        if (do_e) {
          ex[i] += (double)e0.x * v0.x + (double)e0.y * v0.y + (double)e1.x * v1.x + (double)e1.y * v1.y;
          ey[i] += (double)e0.x * v0.y - (double)e0.y * v0.x + (double)e1.x * v1.y - (double)e1.y * v1.x;
        }
      }
      unsigned short h0r, l0r, h1r, l1r, h0i, l0i, h1i, l1i;
      split_hl(v0.x, h0r, l0r);
      split_hl(v1.x, h1r, l1r);
      split_hl(v0.y, h0i, l0i);
      split_hl(v1.y, h1i, l1i);
      *reinterpret_cast<unsigned*>(&Ah[2 * ff][pa]) = (unsigned)h0r | ((unsigned)h1r << 16);
      *reinterpret_cast<unsigned*>(&Al[2 * ff][pa]) = (unsigned)l0r | ((unsigned)l1r << 16);
      *reinterpret_cast<unsigned*>(&Ah[2 * ff + 1][pa]) = (unsigned)h0i | ((unsigned)h1i << 16);
      *reinterpret_cast<unsigned*>(&Al[2 * ff + 1][pa]) = (unsigned)l0i | ((unsigned)l1i << 16);
    }
    *reinterpret_cast<uint4*>(&Bh[sb][hb]) = rbh[0];
    *reinterpret_cast<uint4*>(&Bh[sb][hb + 8]) = rbh[1];
    *reinterpret_cast<uint4*>(&Bl[sb][hb]) = rbl[0];
    *reinterpret_cast<uint4*>(&Bl[sb][hb + 8]) = rbl[1];
  };
  load(k0);
  for (size_t kb = k0; kb < k1; kb += XK) {
    __syncthreads();
    store();
    __syncthreads();
    if (kb + XK < k1) load(kb + XK);
    mma_stage<XKP>(Ah, Al, Bh, Bl, lane, wm, wn, acc);
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
  if (do_e) {
    // the 16 lanes sharing qa hold the same 4 fields at different points
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double x = ex[i], y = ey[i];
      for (int off = 8; off > 0; off >>= 1) {
        x += __shfl_down(x, off, 16);
        y += __shfl_down(y, off, 16);
      }
      const int f = f0 + qa + 16 * i;
      if ((tid & 15) == 0 && f < F) gpart[(size_t)f * nchunk + kc] = make_double2(x, y);
    }
  }
}

// coef[f][s] = dv * (sum_kc part[kc][2f][s] + i sum_kc part[kc][2f+1][s]),
// stored with row stride S+1 (slot S holds the E dot).  A block sums 32
// outputs in RED_SL slices of the chunks (slice j: kc = j, j + RED_SL, ...),
// then adds the slices in order: a fixed summation order with enough loads
// in flight to stream the partials.
constexpr int RED_SL = 8;
__global__ void __launch_bounds__(256) k_coef_reduce(const float* __restrict__ part, int nchunk, int F,
                                                     int S, double dv, double2* __restrict__ coef) {
  __shared__ double2 red[RED_SL][32];
  const int o = threadIdx.x & 31, j = threadIdx.x >> 5;
  const int i = blockIdx.x * 32 + o;
  const bool live = i < F * S;
  const int f = live ? i / S : 0, s = live ? i % S : 0;
  const size_t RS = (size_t)2 * F * S;
  double x = 0, y = 0;
  if (live)
    for (int k = j; k < nchunk; k += RED_SL) {
      x += part[k * RS + (size_t)(2 * f) * S + s];
      y += part[k * RS + (size_t)(2 * f + 1) * S + s];
    }
  red[j][o] = make_double2(x, y);
  __syncthreads();
  if (j == 0 && live) {
    double sx = 0, sy = 0;
#pragma unroll
    for (int q = 0; q < RED_SL; ++q) {
      sx += red[q][o].x;
      sy += red[q][o].y;
    }
    coef[(size_t)f * (S + 1) + s] = make_double2(sx * dv, sy * dv);
  }
}

// coef[f][S] = dv sum_k gpart[f][k]: one wave per field, lanes over k, then a
// fixed shuffle tree
__global__ void __launch_bounds__(256) k_edot_reduce(const double2* __restrict__ gpart, int nblk, int F,
                                                     int S, double dv, double2* __restrict__ coef) {
  const int f = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (f >= F) return;
  double x = 0, y = 0;
  for (int k = lane; k < nblk; k += 64) {
    const double2 g = gpart[(size_t)f * nblk + k];
    x += g.x;
    y += g.y;
  }
  for (int off = 32; off > 0; off >>= 1) {
    x += __shfl_down(x, off, 64);
    y += __shfl_down(y, off, 64);
  }
  if (lane == 0) coef[(size_t)f * (S + 1) + S] = make_double2(x * dv, y * dv);
}

// coefficient rows for the update: ct[row][s], row 2f = Re C[f][s], 2f+1 =
// Im C[f][s], split hi/lo, zero for s >= S
__global__ void k_coef_split(const double2* __restrict__ coef, int F, int S, int Sp,
                             unsigned short* __restrict__ cth, unsigned short* __restrict__ ctl) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 2 * F * Sp) return;
  const int row = i / Sp, s = i % Sp, f = row / 2;
  float x = 0.f;
  if (s < S) {
    const double2 c = coef[(size_t)f * (S + 1) + s];
    x = (float)((row & 1) ? c.y : c.x);
  }
  split_hl(x, cth[i], ctl[i]);
}

// d_f(r) = fin(d_f(r)) - sum_s C[f][s] phi_s(r) - c_f E_l(r), fin the end of
// the step when MID.  Block: 128 rows (64 fields) x 128 points, K = states
// in stages of 32; row tile fastest so that the row tiles of one point tile
// (sharing its phi^T tile) run together on one XCD.
template <bool MID>
__global__ void __launch_bounds__(256, 3) k_update_x3(float2* __restrict__ d, int F, PhiSplit ps,
                                                   const float2* __restrict__ E, int L, size_t ng,
                                                   const unsigned short* __restrict__ cth,
                                                   const unsigned short* __restrict__ ctl,
                                                   const double2* __restrict__ coef, int nrt,
                                                   unsigned ntile, MidArgs mid) {
  // operand tiles during the K loop; afterwards the same LDS holds half of
  // the result tile (64 rows x 128 points, rows padded) at a time
  constexpr int TP = XT + 4;
  static_assert(4 * XT * XKP * sizeof(__bf16) >= 64 * TP * sizeof(float), "result half fits");
  __shared__ __attribute__((aligned(16))) __bf16 lds_u[4 * XT * XKP];
  __bf16 (*Ah)[XKP] = reinterpret_cast<__bf16 (*)[XKP]>(lds_u);
  __bf16 (*Al)[XKP] = Ah + XT;
  __bf16 (*Bh)[XKP] = Al + XT;
  __bf16 (*Bl)[XKP] = Bh + XT;
  float* T = reinterpret_cast<float*>(lds_u);
  const unsigned t = xcd_tile(blockIdx.x, gridDim.x);
  if (t >= ntile) return;
  const int rt = (int)(t % nrt);
  const size_t p0 = (size_t)(t / nrt) * XT;
  const int r0 = rt * XT;
  const int R = 2 * F, S = ps.S, Sp = ps.Sp;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  // loader: 4 lanes per row, 16 bytes each, 64 rows a pass; passes 0 and 1
  // take coefficient rows, 2 and 3 points of phi^T.  Rows past R (points
  // past ng) load the last one: their results are never stored.  go, lo:
  // element offsets in the global operand and in LDS (hi arrays; lo arrays
  // one operand tile further)
  const int qp = tid & 3, rw = tid >> 2;
  unsigned go[4], lo[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int r = rw + 64 * (c & 1);
    if (c < 2) {
      go[c] = (unsigned)min(R - 1, r0 + r) * (unsigned)Sp + 8 * qp;
      lo[c] = r * XKP + 8 * qp;
    } else {
      go[c] = (unsigned)min(ng - 1, p0 + r) * (unsigned)Sp + 8 * qp;
      lo[c] = 2 * XT * XKP + r * XKP + 8 * qp;
    }
  }
  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  typedef unsigned u4v __attribute__((ext_vector_type(4)));
  u4v rh[4], rl[4];
  auto load = [&](int kb) __attribute__((always_inline)) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const unsigned short* gh = c < 2 ? cth : ps.th;
      const unsigned short* gl = c < 2 ? ctl : ps.tl;
      rh[c] = *reinterpret_cast<const u4v*>(gh + go[c] + kb);
      rl[c] = *reinterpret_cast<const u4v*>(gl + go[c] + kb);
    }
  };
  auto store = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      *reinterpret_cast<u4v*>(lds_u + lo[c]) = rh[c];
      *reinterpret_cast<u4v*>(lds_u + lo[c] + XT * XKP) = rl[c];
    }
  };
  load(0);
  for (int kb = 0; kb < Sp; kb += XK) {
    __syncthreads();
    store();
    __syncthreads();
    if (kb + XK < Sp) load(kb + XK);
    mma_stage<XKP>(Ah, Al, Bh, Bl, lane, wm, wn, acc);
  }
  // epilogue, two halves of 32 fields: the waves owning the half write their
  // results to LDS, then every thread streams 4 fields x 4 consecutive points
  // (16-byte accesses; a wave covers 128 points of two fields)
  const int pg = tid & 31, fs = tid >> 5;
  const size_t pr = p0 + 4 * pg;
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    __syncthreads();
    if (wm == half) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            T[(i * 16 + 4 * (lane >> 4) + v) * TP + wn * 64 + j * 16 + (lane & 15)] = acc[i][j][v];
    }
    __syncthreads();
    if (pr >= ng) continue;
    float4 p01 = make_float4(0.f, 0.f, 0.f, 0.f), p23 = p01;
    if (MID) {
      p01 = *reinterpret_cast<const float4*>(mid.ph + pr);
      p23 = *reinterpret_cast<const float4*>(mid.ph + pr + 2);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int fl = fs + 8 * q;                 // field within the half
      const int f = r0 / 2 + half * 32 + fl;
      if (2 * f >= R) continue;
      const int l = f % L;
      const float cr = (float)coef[(size_t)f * (S + 1) + S].x;
      float2* dp = d + (size_t)f * ng + pr;
      float4 d01 = reinterpret_cast<const float4*>(dp)[0];
      float4 d23 = reinterpret_cast<const float4*>(dp)[1];
      float4 e01, e23;
      if (MID) {
        const float2* hp = mid.H + (size_t)l * ng + pr;
        const float4 h01 = reinterpret_cast<const float4*>(hp)[0];
        const float4 h23 = reinterpret_cast<const float4*>(hp)[1];
        const float4 uu = *reinterpret_cast<const float4*>(mid.u + (size_t)(f / L) * ng + pr);
        const float2 hv[4] = {make_float2(h01.x, h01.y), make_float2(h01.z, h01.w),
                              make_float2(h23.x, h23.y), make_float2(h23.z, h23.w)};
        const float2 pv[4] = {make_float2(p01.x, p01.y), make_float2(p01.z, p01.w),
                              make_float2(p23.x, p23.y), make_float2(p23.z, p23.w)};
        const float uv[4] = {uu.x, uu.y, uu.z, uu.w};
        float2 dv[4] = {make_float2(d01.x, d01.y), make_float2(d01.z, d01.w),
                        make_float2(d23.x, d23.y), make_float2(d23.z, d23.w)};
        float2 ev[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          dv[k] = finish1(dv[k], hv[k], uv[k], pv[k], mid.half_dt);
          ev[k] = cm(pv[k], hv[k]);
        }
        d01 = make_float4(dv[0].x, dv[0].y, dv[1].x, dv[1].y);
        d23 = make_float4(dv[2].x, dv[2].y, dv[3].x, dv[3].y);
        e01 = make_float4(ev[0].x, ev[0].y, ev[1].x, ev[1].y);
        e23 = make_float4(ev[2].x, ev[2].y, ev[3].x, ev[3].y);
      } else {
        const float2* ep = E + (size_t)l * ng + pr;
        e01 = reinterpret_cast<const float4*>(ep)[0];
        e23 = reinterpret_cast<const float4*>(ep)[1];
      }
      const float4 are = *reinterpret_cast<const float4*>(&T[(2 * fl) * TP + 4 * pg]);
      const float4 aim = *reinterpret_cast<const float4*>(&T[(2 * fl + 1) * TP + 4 * pg]);
      d01.x -= are.x + cr * e01.x;
      d01.y -= aim.x + cr * e01.y;
      d01.z -= are.y + cr * e01.z;
      d01.w -= aim.y + cr * e01.w;
      d23.x -= are.z + cr * e23.x;
      d23.y -= aim.z + cr * e23.y;
      d23.z -= are.w + cr * e23.z;
      d23.w -= aim.w + cr * e23.w;
      reinterpret_cast<float4*>(dp)[0] = d01;
      reinterpret_cast<float4*>(dp)[1] = d23;
    }
  }
}

static unsigned round8(unsigned n) { return (n + 7u) & ~7u; }

hipError_t launch_phi_split(const float* phi, int S, size_t ng, PhiSplitBufs b, hipStream_t st) {
  const int Sp = clean_sp(S);
  const size_t n = ng * (size_t)Sp;
  hipLaunchKernelGGL(k_phi_split, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, phi, S, Sp, ng,
                     b.h, b.l, b.th, b.tl);
  return hipGetLastError();
}

hipError_t launch_coef_x3(const float2* d, int F, const PhiSplit& ps, size_t ng, int chunk,
                          float* part, double dv, double2* coef, hipStream_t st, const MidArgs& mid,
                          const float2* E, int L, double2* gpart) {
  if (F <= 0 || ps.S <= 0 || ng % XK || chunk % XK || chunk <= 0) return hipErrorInvalidValue;
  if (mid.on && !gpart) return hipErrorInvalidValue;
  const int nrt = (2 * F + XT - 1) / XT, nct = (ps.S + XT - 1) / XT;
  const int nchunk = (int)((ng + chunk - 1) / chunk);
  const unsigned ntile = (unsigned)nrt * nct * nchunk;
  const dim3 g(round8(ntile)), b(256);
  if (mid.on)
    hipLaunchKernelGGL((k_coef_x3<true, true>), g, b, 0, st, d, F, ps, ng, chunk, nrt, nct, nchunk,
                       ntile, mid, E, L, part, gpart);
  else if (gpart)
    hipLaunchKernelGGL((k_coef_x3<false, true>), g, b, 0, st, d, F, ps, ng, chunk, nrt, nct, nchunk,
                       ntile, mid, E, L, part, gpart);
  else
    hipLaunchKernelGGL((k_coef_x3<false, false>), g, b, 0, st, d, F, ps, ng, chunk, nrt, nct, nchunk,
                       ntile, mid, E, L, part, gpart);
  if (gpart)
    hipLaunchKernelGGL(k_edot_reduce, dim3((F + 3) / 4), dim3(256), 0, st, gpart, nchunk, F, ps.S, dv,
                       coef);
  hipLaunchKernelGGL(k_coef_reduce, dim3((F * ps.S + 31) / 32), dim3(256), 0, st, part, nchunk, F, ps.S,
                     dv, coef);
  return hipGetLastError();
}

hipError_t launch_update_x3(float2* d, int F, const PhiSplit& ps, const float2* E, int L, size_t ng,
                            const double2* coef, float* scratch, hipStream_t st, const MidArgs& mid) {
  if (F <= 0 || ps.S <= 0 || ps.Sp != clean_sp(ps.S)) return hipErrorInvalidValue;
  // the loader's 32-bit element offsets into phi^T and the coefficient rows
  if (ng * (size_t)ps.Sp > 0xFFFFFFFFull || (size_t)2 * F * ps.Sp > 0xFFFFFFFFull) return hipErrorInvalidValue;
  const int Sp = ps.Sp;
  unsigned short* cth = reinterpret_cast<unsigned short*>(scratch);
  unsigned short* ctl = cth + (size_t)2 * F * Sp;
  hipLaunchKernelGGL(k_coef_split, dim3((2 * F * Sp + 255) / 256), dim3(256), 0, st, coef, F, ps.S, Sp,
                     cth, ctl);
  const int nrt = (2 * F + XT - 1) / XT;
  const size_t npt = (ng + XT - 1) / XT;
  const unsigned ntile = (unsigned)(nrt * npt);
  const dim3 g(round8(ntile)), b(256);
  if (mid.on)
    hipLaunchKernelGGL(k_update_x3<true>, g, b, 0, st, d, F, ps, E, L, ng, cth, ctl, coef, nrt, ntile,
                       mid);
  else
    hipLaunchKernelGGL(k_update_x3<false>, g, b, 0, st, d, F, ps, E, L, ng, cth, ctl, coef, nrt, ntile,
                       mid);
  return hipGetLastError();
}

// K chunks for about 8192 blocks: the blocks of one chunk share its field
// and orbital panels, and the shorter their K runs the less they drift apart
// and miss each other's panels in L2 (112^3, 210 fields, 260 states: 2.78 ms
// with 2048 blocks, 2.39 ms with 8192, the partial sums 4x larger)
int clean_chunk_d(int F, int S, size_t ng) {
  const size_t tiles = (size_t)((2 * F + XT - 1) / XT) * ((S + XT - 1) / XT);
  const size_t nc = std::max<size_t>(1, (8192 + tiles - 1) / tiles);
  const size_t c = ((ng + nc - 1) / nc + XK - 1) / XK * XK;
  return (int)std::min<size_t>(c, 1u << 30);
}

// coefficient partials of F fields: nchunk(F) x 2F x S floats
static size_t coef_part_d(int F, int S, size_t ng) {
  const size_t cd = (size_t)clean_chunk_d(F, S, ng);
  return (ng + cd - 1) / cd * 2 * (size_t)F * S;
}

// F = B L fields for batches of up to B pairs: the chunk count depends on the
// batch, so the partials are sized by the largest need over every batch size
size_t clean_scratch_floats(int F, int L, int S, size_t ng) {
  size_t a = 0;
  for (int f = L; f <= F; f += L) a = std::max(a, coef_part_d(f, S, ng));
  const size_t b = (ng + CLEAN_CHUNK_E - 1) / CLEAN_CHUNK_E * 2 * (size_t)L * S;
  const size_t c = (size_t)2 * F * clean_sp(S);   // two bf16 arrays of 2F x Sp
  return std::max(a, std::max(b, c));
}

size_t edot_part_entries(int F, int L, int S, size_t ng) {
  size_t m = 0;
  for (int f = L; f <= F; f += L) {
    const size_t cd = (size_t)clean_chunk_d(f, S, ng);
    m = std::max(m, (size_t)f * ((ng + cd - 1) / cd));
  }
  return m;
}

}  // namespace bse
