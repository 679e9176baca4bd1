// Propagation, Poisson and cleaning kernels of the stochastic TD-Hartree
// action of W (Method: "Stochastic evaluation of the action of W",
// Eqs. 10-15), for gfx950.
//
// Field layout: complex interleaved (float2/double2), [field][x][y][z] with
// z fastest, n = N per axis.  The kinetic propagator exp(-i T dt) is
// separable into exp(-i kx^2 dt/2) exp(-i ky^2 dt/2) exp(-i kz^2 dt/2); the
// x factor is applied by prop_x on tiles [N x TC] of x-lines, the y and z
// factors by prop_yz on whole contiguous y-z planes.  The Coulomb solve is a
// full 3-D transform: forward y-z planes, x-lines with the 4 pi/k^2
// multiplier between the forward and inverse halves, inverse y-z planes.
#include <hip/hip_ext.h>

#include "fft_lines.h"
#include "prop_kernels.h"
#include "clean_mfma.h"

#include <algorithm>
#include <type_traits>

namespace bse {

// The twiddle and kinetic-phase tables are staged in LDS behind the data
// region: the transforms then read them through the LDS counter instead of
// the in-order vector-memory counter, which would otherwise make the first
// table read wait for the whole in-flight prefetch of the next plane.
template <int N, typename C>
__device__ __forceinline__ void stage_tables(C* t, const C* __restrict__ tw, const C* __restrict__ kp,
                                             int tid, int nthr) {
  for (int i = tid; i < N; i += nthr) {
    t[i] = tw[i];
    if (kp) t[N + i] = kp[i];
  }
}

// ---------------------------------------------------------------------------
// prop_x: pre-kinetic pointwise step fused with the x factor of exp(-iT dt)
// ---------------------------------------------------------------------------
// mode PX_ETA0: out = Pf * in                                  (unperturbed set)
// mode PX_FULL: out = Pf * (d - i dt u_b H_l)                  (mid-step state)
// mode PX_HALF: out = Ph * (d - i dt/2 u_b (Ph H_l))           (cleaned end state)
// The pair variant (ETA = false) runs one block per (tile, pair) over the L
// orbitals of the pair: u_b and the phase tile stay in registers, and the
// loads of orbital l+1 are in flight while orbital l is transformed.
template <int N, int TC, typename T>
__device__ __forceinline__ void kinetic_x_tile(cplx<T>* s, const cplx<T>* __restrict__ tw,
                                               const cplx<T>* __restrict__ kp, int tid, int nthr) {
  using C = cplx<T>;
  stageA_fwd<N>(s, TC, 1, TC, tw, tid, nthr, true);
  __syncthreads();
  stageB<N, 2>(s, TC, 1, TC, tw, tid, nthr, true,
               [kp](int, C v, int k) { return cmul(v, kp[k]); });
  __syncthreads();
  stageC_inv<N>(s, TC, 1, TC, tid, nthr, true);
  __syncthreads();
}

// Each thread owns work items (column c, j2) of the four-step transform of
// its x-lines: the N1 values x = j1 N2 + j2 are loaded from HBM straight into
// registers (coalesced over c), transformed (stage A) and written to LDS;
// stage B runs through LDS; stage C reads its N1 slots back and the results
// go straight to HBM.  The pair variant keeps u_b in registers across the L
// orbitals and has the next orbital's loads in flight during the transform.
// The (field, tile) of a workgroup.  Order 0: a 2-D grid (fields, tiles),
// field fastest, so that the fields of one tile run close together.  Order
// 1: a 1-D grid renumbered so that XCD x (workgroup ids are dealt round-robin
// to the eight XCDs, x = id mod 8) walks its own contiguous range of
// (tile, field) with the field fastest: the fields of a tile then share one
// XCD's L2 for the tile's shared operands (the unperturbed orbitals, the
// phase tables) instead of each of the eight L2s fetching them.
__device__ __forceinline__ bool field_tile(int order, int nf, int ntile, int& f, int& tile) {
  if (order == 0) {
    f = blockIdx.x;
    tile = blockIdx.y;
    return true;
  }
  const unsigned id = blockIdx.x, per = gridDim.x >> 3;
  const unsigned v = (id & 7u) * per + (id >> 3);
  if (v >= (unsigned)nf * (unsigned)ntile) return false;
  f = (int)(v % (unsigned)nf);
  tile = (int)(v / (unsigned)nf);
  return true;
}
inline dim3 field_tile_grid(int order, int nf, int ntile) {
  if (order == 0) return dim3(nf, ntile);
  const unsigned n = (unsigned)nf * (unsigned)ntile;
  return dim3(8 * ((n + 7) / 8));
}

// One (field or pair fb, tile of TC columns) of the x pass, by a block of
// 256 threads on LDS s (x_lds bytes); shared by the per-system kernel and the
// work-list kernel of uneven batches.
template <int N, int TC, typename T, bool ETA>
__device__ __forceinline__ void prop_x_item(const PropXArgs<T>& a, int fb, int tile, cplx<T>* s) {
  using C = cplx<T>;
  constexpr int NTH = 256;
  constexpr int N1 = Fac<N>::N1, N2 = Fac<N>::N2;
  constexpr int IT = TC * N2 / NTH;
  static_assert(TC * N2 % NTH == 0, "work items must fill the block");
  const size_t ng = (size_t)N * N * N;
  const int c0 = tile * TC;
  const int tid = threadIdx.x;
  C* tws = s + N * TC;
  stage_tables<N>(tws, a.tw, a.kph, tid, NTH);
  __syncthreads();
  const C* tw = tws;
  const C* kp = tws + N;
  // global offset of element j1 of item it
  auto gidx = [&](int it, int j1) -> size_t {
    const int w = tid + it * NTH;
    const int c = w % TC, j2 = w / TC;
    return (size_t)(j1 * N2 + j2) * N * N + c0 + c;
  };
  // stage A from registers: DFT_N1, twiddle, write slot k1 N2 + j2 of line c
  auto stage_a = [&](int it, C* v) {
    const int w = tid + it * NTH;
    const int c = w % TC, j2 = w / TC;
    Dft<N1, -1, C>::run(v);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) {
      C x = v[k1];
      if (k1 > 0 && j2 > 0) x = cmul(x, tw[(j2 * k1) % N]);
      s[(k1 * N2 + j2) * TC + c] = x;
    }
  };
  // stage C to registers: read slots, inverse DFT_N1 -> x = j1 N2 + j2
  auto stage_c = [&](int it, C* v) {
    const int w = tid + it * NTH;
    const int c = w % TC, j2 = w / TC;
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) v[k1] = s[(k1 * N2 + j2) * TC + c];
    Dft<N1, +1, C>::run(v);
  };
  auto mul = [kp](int, C v, int k) { return cmul(v, kp[k]); };
  if (ETA) {
    const size_t fo = (size_t)fb * ng;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      C v[N1];
#pragma unroll
      for (int j1 = 0; j1 < N1; ++j1) {
        const size_t g = gidx(it, j1);
        v[j1] = cmul(a.pf[g], a.din[fo + g]);
      }
      stage_a(it, v);
    }
    __syncthreads();
    stageB<N, 2>(s, TC, 1, TC, tw, tid, NTH, true, mul);
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      C v[N1];
      stage_c(it, v);
#pragma unroll
      for (int j1 = 0; j1 < N1; ++j1) a.dout[fo + gidx(it, j1)] = v[j1];
    }
    return;
  }
  const int b = fb;
  const bool half = a.mode == PX_HALF;
  const T cu = half ? (T)0.5 * a.dt : a.dt;
  const C* __restrict__ ptab = half ? a.ph : a.pf;
  T uu[IT][N1];
  C dn[IT][N1], hn[IT][N1];
#pragma unroll
  for (int it = 0; it < IT; ++it)
#pragma unroll
    for (int j1 = 0; j1 < N1; ++j1) {
      const size_t g = gidx(it, j1);
      uu[it][j1] = cu * a.u[(size_t)b * ng + g];
      dn[it][j1] = a.din[(size_t)b * a.L * ng + g];
      hn[it][j1] = a.H[g];
    }
  for (int l = 0; l < a.L; ++l) {
    const size_t fo = ((size_t)b * a.L + l) * ng;
    C v[IT][N1];
#pragma unroll
    for (int it = 0; it < IT; ++it)
#pragma unroll
      for (int j1 = 0; j1 < N1; ++j1) {
        const C p = ptab[gidx(it, j1)];
        C h = hn[it][j1];
        if (half) h = cmul(p, h);
        const C x = cmk<C>(dn[it][j1].x + uu[it][j1] * h.y, dn[it][j1].y - uu[it][j1] * h.x);
        v[it][j1] = cmul(p, x);
      }
    if (l + 1 < a.L) {
#pragma unroll
      for (int it = 0; it < IT; ++it)
#pragma unroll
        for (int j1 = 0; j1 < N1; ++j1) {
          const size_t g = gidx(it, j1);
          dn[it][j1] = a.din[fo + ng + g];
          hn[it][j1] = a.H[(size_t)(l + 1) * ng + g];
        }
    }
    __syncthreads();  // the previous orbital's stage C has read its slots
#pragma unroll
    for (int it = 0; it < IT; ++it) stage_a(it, v[it]);
    __syncthreads();
    stageB<N, 2>(s, TC, 1, TC, tw, tid, NTH, true, mul);
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      stage_c(it, v[it]);
#pragma unroll
      for (int j1 = 0; j1 < N1; ++j1) a.dout[fo + gidx(it, j1)] = v[it][j1];
    }
  }
}

template <int N, int TC, typename T, bool ETA>
__global__ void __launch_bounds__(256) k_prop_x(PropXArgs<T> a) {
  extern __shared__ unsigned char smem_raw[];
  // the blocks of one tile run close together and share its H and phase
  // tiles in L2 (field_tile)
  int fb, tile;
  if (!field_tile(a.order, a.nf, N * N / TC, fb, tile)) return;
  prop_x_item<N, TC, T, ETA>(a, fb, tile, reinterpret_cast<cplx<T>*>(smem_raw));
}

// ---------------------------------------------------------------------------
// prop_yz: y and z factors of exp(-iT dt) on a whole y-z plane, plus the
// induced density dn_b = 4 sum_l Re(conj(H_l) d_{b,l}) of the post-kinetic
// state (linearised Eq. 11 source).  The pair variant loops over the L
// orbitals with the next plane's loads in flight during the transform.
// ---------------------------------------------------------------------------
// Plane layout in LDS: row y at y * (N + 1), so that lanes walking over y
// (stride N + 1 complex values) spread over the LDS banks.
template <int N> constexpr int plane_stride() { return N + 1; }
template <int N> __device__ __forceinline__ int plane_idx(int e) {
  return (e / N) * plane_stride<N>() + (e % N);
}

template <int N, typename T, int NT>
__device__ __forceinline__ void kinetic_yz_plane(cplx<T>* s, const cplx<T>* __restrict__ tw,
                                                 const cplx<T>* __restrict__ kp, int tid) {
  using C = cplx<T>;
  constexpr int S = plane_stride<N>();
  auto mul = [kp](int, C v, int k) { return cmul(v, kp[k]); };
  // z lines: line = y (stride S), elements contiguous; lanes walk over y
  stageA_fwd<N>(s, N, S, 1, tw, tid, NT, true);
  __syncthreads();
  stageB<N, 2>(s, N, S, 1, tw, tid, NT, true, mul);
  __syncthreads();
  stageC_inv<N>(s, N, S, 1, tid, NT, true);
  __syncthreads();
  // y lines: line = z (stride 1), elements S apart; lanes walk over z
  stageA_fwd<N>(s, N, 1, S, tw, tid, NT, true);
  __syncthreads();
  stageB<N, 2>(s, N, 1, S, tw, tid, NT, true, mul);
  __syncthreads();
  stageC_inv<N>(s, N, 1, S, tid, NT, true);
  __syncthreads();
}

// One (plane x, pair b) of the pair variant of the plane pass: the L
// orbitals of the pair with the next one's loads in flight, and the induced
// density of the pair; a block of NT threads on LDS s (yz_lds bytes).
// Shared by the per-system kernel and the work-list kernel.
template <int N, typename T, int NT>
__device__ __forceinline__ void prop_yz_pair_item(const PropYZArgs<T>& a, int x, int b, cplx<T>* s) {
  using C = cplx<T>;
  constexpr int P = N * N;
  constexpr int PER = (P + NT - 1) / NT;
  constexpr bool PREF_H = PER <= 8;
  const int ng = N * N * N;
  const int tid = threadIdx.x;
  const size_t poff = (size_t)x * P;
  C* tws = s + N * plane_stride<N>();
  stage_tables<N>(tws, a.tw, a.kph, tid, NT);
  T acc[PER];
  C dn[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    acc[i] = 0;
    const int e = tid + i * NT;
    if (e < P) dn[i] = a.d[((size_t)b * a.L) * ng + poff + e];
  }
  for (int l = 0; l < a.L; ++l) {
    C* d = a.d + ((size_t)b * a.L + l) * ng + poff;
    const C* __restrict__ h = a.H + (size_t)l * ng + poff;
    C hc[PREF_H ? PER : 1];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = tid + i * NT;
      if (e < P) s[plane_idx<N>(e)] = dn[i];
    }
    __syncthreads();
    // loads of the next orbital and of this orbital's unperturbed plane are
    // in flight during the transform
    if (l + 1 < a.L) {
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = tid + i * NT;
        if (e < P) dn[i] = d[ng + e];
      }
    }
    if (PREF_H) {
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = tid + i * NT;
        if (e < P) hc[PREF_H ? i : 0] = h[e];
      }
    }
    kinetic_yz_plane<N, T, NT>(s, tws, tws + N, tid);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = tid + i * NT;
      if (e < P) {
        const C v = s[plane_idx<N>(e)];
        const C hh = PREF_H ? hc[PREF_H ? i : 0] : h[e];
        d[e] = v;
        acc[i] += hh.x * v.x + hh.y * v.y;
      }
    }
  }
  T* dn_out = a.dens + (size_t)b * ng + poff;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = tid + i * NT;
    if (e < P) dn_out[e] = (T)4 * acc[i];
  }
}

template <int N, typename T, int NT, bool DENS>
__global__ void __launch_bounds__(NT) k_prop_yz(PropYZArgs<T> a) {
  using C = cplx<T>;
  extern __shared__ unsigned char smem_raw[];
  C* s = reinterpret_cast<C*>(smem_raw);
  // grid: (x planes, fields or pairs) with the plane fastest: blocks running
  // together stream consecutive planes of one field (measured faster than
  // sharing the H planes across pairs, which the x pass gains from)
  if (DENS) {
    prop_yz_pair_item<N, T, NT>(a, blockIdx.x, blockIdx.y, s);
    return;
  }
  constexpr int P = N * N;
  const int ng = N * N * N;
  const int x = blockIdx.x;
  const int tid = threadIdx.x;
  const size_t poff = (size_t)x * P;
  C* tws = s + N * plane_stride<N>();
  stage_tables<N>(tws, a.tw, a.kph, tid, NT);
  C* d = a.d + (size_t)blockIdx.y * ng + poff;
  for (int e = tid; e < P; e += NT) s[plane_idx<N>(e)] = d[e];
  __syncthreads();
  kinetic_yz_plane<N, T, NT>(s, tws, tws + N, tid);
  for (int e = tid; e < P; e += NT) d[e] = s[plane_idx<N>(e)];
}

// ---------------------------------------------------------------------------
// The y and z factors as two line passes, for grids whose y-z plane would
// leave one block per compute unit (112^3 in FP32: 101 KB of LDS, and the
// lone block's barriers idle the CU): a z-line pass over tiles of PZ_TL
// contiguous lines, then a y-line pass over tiles of PY_TZ z columns of one
// x plane, which also forms the induced density of a pair's L orbitals.
// One more HBM pass, in exchange for several small blocks per CU.
// ---------------------------------------------------------------------------
constexpr int PZ_TL = 32, PY_TZ = 16, PY_ES = PY_TZ + 1, PY_NT = 128;

template <int N, typename T>
__global__ void __launch_bounds__(256) k_prop_z(PropYZArgs<T> a) {
  using C = cplx<T>;
  extern __shared__ unsigned char smem_raw[];
  C* s = reinterpret_cast<C*>(smem_raw);
  constexpr int TL = PZ_TL, S = N + 1, E = TL * N;
  const size_t ng = (size_t)N * N * N;
  const int tid = threadIdx.x;
  C* d = a.d + (size_t)blockIdx.y * ng + (size_t)blockIdx.x * E;
  C* tws = s + TL * S;
  stage_tables<N>(tws, a.tw, a.kph, tid, 256);
  for (int e = tid; e < E; e += 256) s[(e / N) * S + e % N] = d[e];
  __syncthreads();
  const C* kp = tws + N;
  auto mul = [kp](int, C v, int k) { return cmul(v, kp[k]); };
  // z lines: line = (x, y) row (stride S), elements contiguous
  stageA_fwd<N>(s, TL, S, 1, tws, tid, 256, true);
  __syncthreads();
  stageB<N, 2>(s, TL, S, 1, tws, tid, 256, true, mul);
  __syncthreads();
  stageC_inv<N>(s, TL, S, 1, tid, 256, true);
  __syncthreads();
  for (int e = tid; e < E; e += 256) d[e] = s[(e / N) * S + e % N];
}

// y lines of one tile: line = z column c (stride 1), element y at y * PY_ES
template <int N, typename T>
__device__ __forceinline__ void kinetic_y_tile(cplx<T>* s, const cplx<T>* __restrict__ tw,
                                               const cplx<T>* __restrict__ kp, int tid) {
  using C = cplx<T>;
  auto mul = [kp](int, C v, int k) { return cmul(v, kp[k]); };
  stageA_fwd<N>(s, PY_TZ, 1, PY_ES, tw, tid, PY_NT, true);
  __syncthreads();
  stageB<N, 2>(s, PY_TZ, 1, PY_ES, tw, tid, PY_NT, true, mul);
  __syncthreads();
  stageC_inv<N>(s, PY_TZ, 1, PY_ES, tid, PY_NT, true);
  __syncthreads();
}

// grid (fields or pairs, tiles): the pairs of one tile run together and
// share its unperturbed-orbital tiles in L2
template <int N, typename T, bool DENS>
__global__ void __launch_bounds__(PY_NT) k_prop_y(PropYZArgs<T> a) {
  using C = cplx<T>;
  extern __shared__ unsigned char smem_raw[];
  C* s = reinterpret_cast<C*>(smem_raw);
  constexpr int TZ = PY_TZ, E = N * TZ, PER = E / PY_NT;
  static_assert(N % TZ == 0 && E % PY_NT == 0, "tiles must divide the grid");
  const size_t ng = (size_t)N * N * N;
  int b, tile;
  if (!field_tile(a.order, a.nf, N * (N / TZ), b, tile)) return;
  const int tid = threadIdx.x;
  const int x = tile / (N / TZ), z0 = (tile % (N / TZ)) * TZ;
  const size_t off = (size_t)x * N * N + z0;
  C* tws = s + N * PY_ES;
  stage_tables<N>(tws, a.tw, a.kph, tid, PY_NT);
  // element e of the tile: y = e / TZ, column c = e % TZ
  auto gi = [](int e) { return (size_t)(e / TZ) * N + (e % TZ); };
  auto li = [](int e) { return (e / TZ) * PY_ES + (e % TZ); };
  if (!DENS) {
    C* d = a.d + (size_t)b * ng + off;
    for (int e = tid; e < E; e += PY_NT) s[li(e)] = d[gi(e)];
    __syncthreads();
    kinetic_y_tile<N, T>(s, tws, tws + N, tid);
    for (int e = tid; e < E; e += PY_NT) d[gi(e)] = s[li(e)];
    return;
  }
  T acc[PER];
  C dn[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    acc[i] = 0;
    dn[i] = a.d[((size_t)b * a.L) * ng + off + gi(tid + i * PY_NT)];
  }
  for (int l = 0; l < a.L; ++l) {
    C* d = a.d + ((size_t)b * a.L + l) * ng + off;
    const C* __restrict__ h = a.H + (size_t)l * ng + off;
    C hc[PER];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) s[li(tid + i * PY_NT)] = dn[i];
    __syncthreads();
    // the next orbital's tile and this orbital's unperturbed tile load
    // during the transform
    if (l + 1 < a.L) {
#pragma unroll
      for (int i = 0; i < PER; ++i) dn[i] = d[ng + gi(tid + i * PY_NT)];
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) hc[i] = h[gi(tid + i * PY_NT)];
    kinetic_y_tile<N, T>(s, tws, tws + N, tid);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = tid + i * PY_NT;
      const C v = s[li(e)];
      d[gi(e)] = v;
      acc[i] += hc[i].x * v.x + hc[i].y * v.y;
    }
  }
  T* dn_out = a.dens + (size_t)b * ng + off;
#pragma unroll
  for (int i = 0; i < PER; ++i) dn_out[gi(tid + i * PY_NT)] = (T)4 * acc[i];
}

// ---------------------------------------------------------------------------
// prop_yz_reg: the y and z factors of exp(-iT dt) on a whole y-z plane in one
// HBM pass where the plane fills most of the LDS (112^3 in FP32), plus the
// induced density as in prop_yz.  A line of N = 16 R points lives in the
// registers of 16 lanes of one row (lane j holds the points 16 j1 + j, j1 <
// R).  Its transform is the four-step factorisation with the R-point DFTs
// inside each lane and the 16-point DFTs across the 16 lanes as radix-2
// butterflies on cross-lane moves (decimation in frequency forward, leaving
// lane j with frequency k1 + R rev4(j); decimation in time back), the
// kinetic phase applied in between.  The LDS holds the plane only to turn
// z-lines into y-lines and back: three barriers per field, the next field's
// loads in flight during the transforms.  One block per CU.
// ---------------------------------------------------------------------------
constexpr int YZR_NT = 896;   // 56 rows of 16 lanes: two lines of each plane per row at N = 112

// the value of lane (l ^ H) of the same 16-lane row (H = 1, 2, 4, 8): DPP
// quad permutations for 1 and 2, the row rotation by 8 for 8, and a
// ds_swizzle in bit-mask mode (lane l reads lane l ^ 4) for 4
template <int H> __device__ __forceinline__ float xlane(float v) {
  const int iv = __builtin_bit_cast(int, v);
  int r;
  if constexpr (H == 1) {
    r = __builtin_amdgcn_mov_dpp(iv, 0xB1, 0xF, 0xF, false);     // quad_perm(1, 0, 3, 2)
  } else if constexpr (H == 2) {
    r = __builtin_amdgcn_mov_dpp(iv, 0x4E, 0xF, 0xF, false);     // quad_perm(2, 3, 0, 1)
  } else if constexpr (H == 8) {
    r = __builtin_amdgcn_mov_dpp(iv, 0x128, 0xF, 0xF, false);    // row_ror:8
  } else {
    r = __builtin_amdgcn_ds_swizzle(iv, 0x1F | (4 << 10));      // and 0x1f, or 0, xor 4
  }
  return __builtin_bit_cast(float, r);
}
template <int H> __device__ __forceinline__ float2 xlane2(float2 v) {
  return make_float2(xlane<H>(v.x), xlane<H>(v.y));
}

// One radix-2 stage of span H across the row, the same operations on every
// lane.  Decimation in frequency: the lower lane of a pair keeps a + b, the
// upper one (a - b) w, w = W_{2H}^(j mod H): t = other + sg mine, then t we
// (sg = +1, we = 1 on the lower lane; sg = -1, we = w on the upper one).
template <int H, int R>
__device__ __forceinline__ void xstage_fwd(float2 (&v)[R], float sg, float2 we) {
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const float2 o = xlane2<H>(v[k]);
    v[k] = cmul(make_float2(fmaf(sg, v[k].x, o.x), fmaf(sg, v[k].y, o.y)), we);
  }
}
// Its inverse without the factor 1/2, a = A + B conj(w), b = A - B conj(w):
// each lane scales its own value by m (1 on the lower lane, conj(w) on the
// upper one), then new = other + sg mine.
template <int H, int R>
__device__ __forceinline__ void xstage_inv(float2 (&v)[R], float sg, float2 m) {
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const float2 u = cmul(v[k], m);
    const float2 o = xlane2<H>(u);
    v[k] = make_float2(fmaf(sg, u.x, o.x), fmaf(sg, u.y, o.y));
  }
}

// The span-2 stage, whose twiddle W_4^(j mod 2) is 1 or -i (forward) and its
// conjugate 1 or +i (inverse): the product by -i or +i as two selects with a
// negation instead of a complex multiply (rot: upper lane with j odd).
template <int R>
__device__ __forceinline__ void xstage_fwd_q(float2 (&v)[R], float sg, bool rot) {
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const float2 o = xlane2<2>(v[k]);
    const float2 t = make_float2(fmaf(sg, v[k].x, o.x), fmaf(sg, v[k].y, o.y));
    v[k] = rot ? make_float2(t.y, -t.x) : t;
  }
}
template <int R>
__device__ __forceinline__ void xstage_inv_q(float2 (&v)[R], float sg, bool rot) {
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const float2 u = rot ? make_float2(-v[k].y, v[k].x) : v[k];
    const float2 o = xlane2<2>(u);
    v[k] = make_float2(fmaf(sg, u.x, o.x), fmaf(sg, u.y, o.y));
  }
}

// per-lane constants of the four cross-lane stages
struct XConst {
  float s8, s4, s2, s1;            // +1 on the lower lane of the stage's pairs, -1 on the upper
  float2 w8, w4;                   // the forward twiddle on upper lanes, 1 on lower ones
  bool q2;                         // upper lane of the span-2 stage with j odd: twiddle -i
};

// exp(-i k^2 dt/2) along one line held by a row (1/N of the inverse in kp)
template <int N>
__device__ __forceinline__ void kin_line_reg(float2 (&v)[N / 16], int j, int rj, const float2* tw,
                                             const float2* kp, const XConst& xc) {
  constexpr int R = N / 16;
  Dft<R, -1, float2>::run(v);
#pragma unroll
  for (int k1 = 1; k1 < R; ++k1) v[k1] = cmul(v[k1], tw[j * k1]);
  const float2 one = make_float2(1.f, 0.f);
  xstage_fwd<8>(v, xc.s8, xc.w8);
  xstage_fwd<4>(v, xc.s4, xc.w4);
  xstage_fwd_q(v, xc.s2, xc.q2);
  xstage_fwd<1>(v, xc.s1, one);
#pragma unroll
  for (int k1 = 0; k1 < R; ++k1) v[k1] = cmul(v[k1], kp[k1 + R * rj]);
  xstage_inv<1>(v, xc.s1, one);
  xstage_inv_q(v, xc.s2, xc.q2);
  xstage_inv<4>(v, xc.s4, make_float2(xc.w4.x, -xc.w4.y));
  xstage_inv<8>(v, xc.s8, make_float2(xc.w8.x, -xc.w8.y));
#pragma unroll
  for (int k1 = 1; k1 < R; ++k1) v[k1] = cmulc(v[k1], tw[j * k1]);
  Dft<R, +1, float2>::run(v);
}

template <int N, bool DENS>
__global__ void __launch_bounds__(YZR_NT) k_prop_yz_reg(PropYZArgs<float> a) {
  using C = float2;
  constexpr int R = N / 16, G = YZR_NT / 16, LPG = N / G, S = N + 1;
  static_assert(N % 16 == 0 && N % G == 0, "rows of 16 lanes must tile the plane");
  extern __shared__ unsigned char smem_raw[];
  C* pl = reinterpret_cast<C*>(smem_raw);          // plane [N][S]
  C* tws = pl + N * S;                              // tw[N], then kph[N]
  // the density sums of the pair variant, each thread's own slots (no
  // sharing, no barriers): [LPG R][YZR_NT]
  float* accl = reinterpret_cast<float*>(tws + 2 * N);
  const int tid = threadIdx.x, g = tid >> 4, j = tid & 15;
  // (plane x, field b): a 2-D grid (planes, fields), or the XCD-grouped
  // 1-D order with the fields of a plane consecutive on one XCD, so that
  // they share its L2 for the plane's unperturbed orbitals (field_tile)
  int x, b;
  if (a.order == 0) {
    x = blockIdx.x;
    b = blockIdx.y;
  } else if (!field_tile(1, a.nf, N, b, x)) {
    return;
  }
  const size_t ng = (size_t)N * N * N;
  const size_t off = (size_t)x * N * N;
  stage_tables<N>(tws, a.tw, a.kph, tid, YZR_NT);
  const int rj = ((j & 1) << 3) | ((j & 2) << 1) | ((j & 4) >> 1) | ((j & 8) >> 3);
  // z-layout element (q, j1) of the plane: y = g + G q, z = 16 j1 + j
  const int zb = g * N + j;
  auto zo = [&](int q, int j1) { return zb + G * N * q + 16 * j1; };
  const int nf = DENS ? a.L : 1;
  const size_t f0 = DENS ? (size_t)b * a.L : (size_t)b;
  C dr[LPG][R];
  {
    const C* src = a.d + f0 * ng + off;
#pragma unroll
    for (int q = 0; q < LPG; ++q)
#pragma unroll
      for (int j1 = 0; j1 < R; ++j1) dr[q][j1] = src[zo(q, j1)];
  }
  if (DENS) {
#pragma unroll
    for (int e = 0; e < LPG * R; ++e) accl[e * YZR_NT + tid] = 0.f;
  }
  __syncthreads();   // tables staged
  const C* tw = tws;
  const C* kp = tws + N;
  XConst xc;
  {
    const C one = make_float2(1.f, 0.f);
    xc.s8 = (j & 8) ? -1.f : 1.f;
    xc.s4 = (j & 4) ? -1.f : 1.f;
    xc.s2 = (j & 2) ? -1.f : 1.f;
    xc.s1 = (j & 1) ? -1.f : 1.f;
    xc.w8 = (j & 8) ? tw[(j & 7) * R] : one;
    xc.w4 = (j & 4) ? tw[(j & 3) * 2 * R] : one;
    xc.q2 = (j & 3) == 3;
  }
  for (int l = 0; l < nf; ++l) {
    C* d = a.d + (f0 + l) * ng + off;
    const C* h = DENS ? a.H + (size_t)l * ng + off : nullptr;
    __syncthreads();   // the previous field's z lines have left the LDS
#pragma unroll
    for (int q = 0; q < LPG; ++q)
#pragma unroll
      for (int j1 = 0; j1 < R; ++j1) pl[(g + G * q) * S + 16 * j1 + j] = dr[q][j1];
    __syncthreads();
    // y lines: column z = g + G q, lane j holds y = 16 j1 + j
#pragma unroll
    for (int q = 0; q < LPG; ++q) {
      C v[R];
#pragma unroll
      for (int j1 = 0; j1 < R; ++j1) v[j1] = pl[(16 * j1 + j) * S + g + G * q];
      kin_line_reg<N>(v, j, rj, tw, kp, xc);
#pragma unroll
      for (int j1 = 0; j1 < R; ++j1) pl[(16 * j1 + j) * S + g + G * q] = v[j1];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < LPG; ++q) {
      C v[R];
#pragma unroll
      for (int j1 = 0; j1 < R; ++j1) v[j1] = pl[(g + G * q) * S + 16 * j1 + j];
      // this line's unperturbed values and the next field's loads of this
      // line slot in flight during its transform
      C hr[R];
      if (DENS) {
#pragma unroll
        for (int j1 = 0; j1 < R; ++j1) hr[j1] = h[zo(q, j1)];
      }
      if (l + 1 < nf) {
        const C* nx = d + ng;
#pragma unroll
        for (int j1 = 0; j1 < R; ++j1) dr[q][j1] = nx[zo(q, j1)];
      }
      kin_line_reg<N>(v, j, rj, tw, kp, xc);
#pragma unroll
      for (int j1 = 0; j1 < R; ++j1) {
        d[zo(q, j1)] = v[j1];
        if (DENS) accl[(q * R + j1) * YZR_NT + tid] += hr[j1].x * v[j1].x + hr[j1].y * v[j1].y;
      }
    }
  }
  if (DENS) {
    float* dn = a.dens + (size_t)b * ng + off;
#pragma unroll
    for (int q = 0; q < LPG; ++q)
#pragma unroll
      for (int j1 = 0; j1 < R; ++j1) dn[zo(q, j1)] = 4.f * accl[(q * R + j1) * YZR_NT + tid];
  }
}

// ---------------------------------------------------------------------------
// prop_yz_rt: the same plane pass with the 16-point DFTs taken out of the
// lanes' cross-lane butterflies.  Lines, loads, stores and the 7-point DFTs
// stay as in prop_yz_reg (16 lanes of a row hold a line, 7 points each);
// after the 7-point DFTs and their twiddles, the 8 lines a wave holds (4
// rows x 2 slots) are 56 vectors of 16 points (one per (line, k1)), which
// go through a scratch area of the wave's own, one vector to a lane: the
// 16-point DFT, the kinetic phase and the inverse DFT in registers, then
// back to the lines.  The plane is kept transposed, [z][y], so that a
// wave's y-lines are the rows it alone reads and writes: its scratch is
// those rows, and the y half-step needs no block barrier.  Scratch element
// jj of vector vi sits at slot jj ^ f(vi), f(vi) = (vi ^ (vi >> 4)) mod 16,
// which keeps the lanes of a wave on distinct banks.  A wave's LDS
// operations run in program order, so its scratch needs no wait between the
// writes of one lane and the reads of another, only that the compiler keeps
// their order (a wave barrier).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int rt_swz(int vi) { return (vi ^ (vi >> 4)) & 15; }

template <int N, bool DENS>
__global__ void __launch_bounds__(YZR_NT) k_prop_yz_rt(PropYZArgs<float> a) {
  using C = float2;
  constexpr int R = N / 16, G = YZR_NT / 16, LPG = N / G, S = N + 1;
  constexpr int NVQ = 4 * R;                        // vectors per wave and slot
  static_assert(N % 16 == 0 && N % G == 0 && LPG == 2, "two line slots of 16 lanes per row");
  static_assert(LPG * NVQ <= 64, "one vector per lane");
  static_assert(NVQ * 16 <= 4 * S, "a slot's vectors fit in the wave's four rows");
  extern __shared__ unsigned char smem_raw[];
  C* pl = reinterpret_cast<C*>(smem_raw);           // plane, transposed: [z][y], rows of S
  C* tws = pl + N * S;                              // tw[N], then kph[N]
  float* accl = reinterpret_cast<float*>(tws + 2 * N);
  const int tid = threadIdx.x, g = tid >> 4, j = tid & 15;
  const int lane = tid & 63, wv = tid >> 6, rr = (tid >> 4) & 3;
  // this wave's scratch: slot q's vectors in rows 4 wv .. 4 wv + 3 + G q
  C* scr0 = pl + (4 * wv) * S;
  C* scr1 = pl + (4 * wv + G) * S;
  int x, b;
  if (a.order == 0) {
    x = blockIdx.x;
    b = blockIdx.y;
  } else if (!field_tile(1, a.nf, N, b, x)) {
    return;
  }
  const size_t ng = (size_t)N * N * N;
  const size_t off = (size_t)x * N * N;
  stage_tables<N>(tws, a.tw, a.kph, tid, YZR_NT);
  const int zb = g * N + j;
  auto zo = [&](int q, int j1) { return zb + G * N * q + 16 * j1; };
  const int nf = DENS ? a.L : 1;
  const size_t f0 = DENS ? (size_t)b * a.L : (size_t)b;
  C dr[LPG][R];
  {
    const C* src = a.d + f0 * ng + off;
#pragma unroll
    for (int q = 0; q < LPG; ++q)
#pragma unroll
      for (int j1 = 0; j1 < R; ++j1) dr[q][j1] = src[zo(q, j1)];
  }
  if (DENS) {
#pragma unroll
    for (int e = 0; e < LPG * R; ++e) accl[e * YZR_NT + tid] = 0.f;
  }
  __syncthreads();   // tables staged
  const C* tw = tws;
  const C* kp = tws + N;
  // the vector a lane transforms: slot vq, frequency vk1 (of row lane & 3)
  const int vq = lane / NVQ, vloc = lane % NVQ, vk1 = vloc >> 2;
  const bool vlive = lane < LPG * NVQ;
  C* vscr = (vq ? scr1 : scr0) + vloc * 16;
  const int vsw = rt_swz(lane);
  auto order = [&]() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  auto fwd7 = [&](C (&v)[R]) {
    Dft<R, -1, float2>::run(v);
#pragma unroll
    for (int k1 = 1; k1 < R; ++k1) v[k1] = cmul(v[k1], tw[j * k1]);
  };
  auto inv7 = [&](C (&v)[R]) {
#pragma unroll
    for (int k1 = 1; k1 < R; ++k1) v[k1] = cmulc(v[k1], tw[j * k1]);
    Dft<R, +1, float2>::run(v);
  };
  // vector (q, k1, row rr) is lane (q NVQ + 4 k1 + rr) of the 16-point stage
  auto xfer_out = [&](C (&v)[LPG][R]) {
#pragma unroll
    for (int q = 0; q < LPG; ++q)
#pragma unroll
      for (int k1 = 0; k1 < R; ++k1) {
        const int vl = 4 * k1 + rr;
        (q ? scr1 : scr0)[vl * 16 + (j ^ rt_swz(q * NVQ + vl))] = v[q][k1];
      }
  };
  auto xfer_in_q = [&](C (&vq_)[R], int q) {
#pragma unroll
    for (int k1 = 0; k1 < R; ++k1) {
      const int vl = 4 * k1 + rr;
      vq_[k1] = (q ? scr1 : scr0)[vl * 16 + (j ^ rt_swz(q * NVQ + vl))];
    }
  };
  auto xfer_in = [&](C (&v)[LPG][R]) {
#pragma unroll
    for (int q = 0; q < LPG; ++q)
#pragma unroll
      for (int k1 = 0; k1 < R; ++k1) {
        const int vl = 4 * k1 + rr;
        v[q][k1] = (q ? scr1 : scr0)[vl * 16 + (j ^ rt_swz(q * NVQ + vl))];
      }
  };
  auto dft16_kin = [&]() {
    if (vlive) {
      C y[16];
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) y[jj] = vscr[jj ^ vsw];
      Dft<16, -1, float2>::run(y);
#pragma unroll
      for (int k2 = 0; k2 < 16; ++k2) y[k2] = cmul(y[k2], kp[vk1 + R * k2]);
      Dft<16, +1, float2>::run(y);
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) vscr[jj ^ vsw] = y[jj];
    }
  };
  auto stage16 = [&](C (&v)[LPG][R]) {
    xfer_out(v);
    order();
    dft16_kin();
    order();
    xfer_in(v);
  };
  for (int l = 0; l < nf; ++l) {
    C* d = a.d + (f0 + l) * ng + off;
    const C* h = DENS ? a.H + (size_t)l * ng + off : nullptr;
    __syncthreads();   // the previous field's scratch is done with the plane
    // point (y = g + G q, z = 16 j1 + j) to row z, column y
#pragma unroll
    for (int q = 0; q < LPG; ++q)
#pragma unroll
      for (int j1 = 0; j1 < R; ++j1) pl[(16 * j1 + j) * S + g + G * q] = dr[q][j1];
    __syncthreads();
    // y lines: row z = g + G q (this wave's), lane j holds y = 16 j1 + j
    C v[LPG][R];
#pragma unroll
    for (int q = 0; q < LPG; ++q) {
#pragma unroll
      for (int j1 = 0; j1 < R; ++j1) v[q][j1] = pl[(g + G * q) * S + 16 * j1 + j];
      fwd7(v[q]);
    }
    order();           // the rows are read before they turn into scratch
    stage16(v);
    order();
#pragma unroll
    for (int q = 0; q < LPG; ++q) {
      inv7(v[q]);
#pragma unroll
      for (int j1 = 0; j1 < R; ++j1) pl[(g + G * q) * S + 16 * j1 + j] = v[q][j1];
    }
    __syncthreads();
    // z lines: column y = g + G q, lane j holds z = 16 j1 + j
#pragma unroll
    for (int q = 0; q < LPG; ++q) {
#pragma unroll
      for (int j1 = 0; j1 < R; ++j1) v[q][j1] = pl[(16 * j1 + j) * S + g + G * q];
    }
#pragma unroll
    for (int q = 0; q < LPG; ++q) fwd7(v[q]);
    __syncthreads();   // every wave has read its columns: rows turn into scratch
    xfer_out(v);
    order();
    dft16_kin();
    order();
    // one slot at a time back from the scratch (fewer live registers); the
    // next field's loads go out between the slots, in flight during the
    // second slot's transform and stores
#pragma unroll
    for (int q = 0; q < LPG; ++q) {
      xfer_in_q(v[q], q);
      C hr[R];
      if (DENS) {
#pragma unroll
        for (int j1 = 0; j1 < R; ++j1) hr[j1] = h[zo(q, j1)];
      }
      inv7(v[q]);
#pragma unroll
      for (int j1 = 0; j1 < R; ++j1) {
        d[zo(q, j1)] = v[q][j1];
        if (DENS) accl[(q * R + j1) * YZR_NT + tid] += hr[j1].x * v[q][j1].x + hr[j1].y * v[q][j1].y;
      }
      if (q == 0 && l + 1 < nf) {
        const C* nx = d + ng;
#pragma unroll
        for (int qq = 0; qq < LPG; ++qq)
#pragma unroll
          for (int j1 = 0; j1 < R; ++j1) dr[qq][j1] = nx[zo(qq, j1)];
      }
    }
  }
  if (DENS) {
    float* dn = a.dens + (size_t)b * ng + off;
#pragma unroll
    for (int q = 0; q < LPG; ++q)
#pragma unroll
      for (int j1 = 0; j1 < R; ++j1) dn[zo(q, j1)] = 4.f * accl[(q * R + j1) * YZR_NT + tid];
  }
}

// ---------------------------------------------------------------------------
// Coulomb potential v[rho] of real densities, two packed per complex field
// (the 4 pi/k^2 kernel is real and even, so re and im stay independent).
// ---------------------------------------------------------------------------
// One packed input value: with checking on, a non-finite density value is
// replaced by 0 and remembered, so that a failed pair cannot reach the pair
// that shares its transform.
template <typename C, typename T>
__device__ __forceinline__ C load_pair(T v0, T v1, bool check, int& bad0, int& bad1) {
  if (check) {
    if (!isfinite(v0)) { v0 = (T)0; bad0 = 1; }
    if (!isfinite(v1)) { v1 = (T)0; bad1 = 1; }
  }
  return cmk<C>(v0, v1);
}
__device__ __forceinline__ void flag_bad(int* flags, int b0, int b1, int bad0, int bad1) {
  if (bad0) atomicOr(&flags[b0], 1);
  if (bad1) atomicOr(&flags[b1], 1);
}

template <int N, typename T, int NT>
__global__ void __launch_bounds__(NT) k_poisson_yz_fwd(PoisArgs<T> a) {
  using C = cplx<T>;
  extern __shared__ unsigned char smem_raw[];
  C* s = reinterpret_cast<C*>(smem_raw);
  constexpr int P = N * N;
  constexpr int S = plane_stride<N>();
  const int ng = N * N * N;
  const int x = blockIdx.x, m = blockIdx.y, tid = threadIdx.x;
  const int b0 = 2 * m, b1 = 2 * m + 1;
  const T* r0 = a.rho + (size_t)b0 * ng + (size_t)x * P;
  const T* r1 = (b1 < a.B) ? a.rho + (size_t)b1 * ng + (size_t)x * P : nullptr;
  C* tw = s + N * S;
  stage_tables<N, C>(tw, a.tw, nullptr, tid, NT);
  const T i0 = a.pscale ? (T)(1.0 / a.pscale[b0]) : (T)1;
  const T i1 = (a.pscale && r1) ? (T)(1.0 / a.pscale[b1]) : (T)1;
  int bad0 = 0, bad1 = 0;
  for (int e = tid; e < P; e += NT)
    s[plane_idx<N>(e)] = load_pair<C>(r0[e] * i0, r1 ? r1[e] * i1 : (T)0, a.flags != nullptr, bad0, bad1);
  flag_bad(a.flags, b0, b1, bad0, bad1);
  __syncthreads();
  NoMul nm;
  stageA_fwd<N>(s, N, S, 1, tw, tid, NT, true);
  __syncthreads();
  stageB<N, 0>(s, N, S, 1, tw, tid, NT, true, nm);
  __syncthreads();
  stageA_fwd<N>(s, N, 1, S, tw, tid, NT, true);
  __syncthreads();
  stageB<N, 0>(s, N, 1, S, tw, tid, NT, true, nm);
  __syncthreads();
  C* w = a.work + (size_t)m * ng + (size_t)x * P;
  for (int e = tid; e < P; e += NT) w[e] = s[plane_idx<N>(e)];
}

template <int N, int TC, typename T>
__global__ void __launch_bounds__(256) k_poisson_x(PoisArgs<T> a) {
  using C = cplx<T>;
  extern __shared__ unsigned char smem_raw[];
  C* s = reinterpret_cast<C*>(smem_raw);
  const int ng = N * N * N;
  const int c0 = blockIdx.x * TC, m = blockIdx.y, tid = threadIdx.x, nthr = blockDim.x;
  C* w = a.work + (size_t)m * ng;
  C* tw = s + N * TC;
  T* k2 = reinterpret_cast<T*>(tw + N);
  for (int i = tid; i < N; i += nthr) {
    tw[i] = a.tw[i];
    k2[i] = a.k2[i];
  }
  for (int e = tid; e < N * TC; e += nthr) {
    const int x = e / TC, c = e % TC;
    s[x * TC + c] = w[(size_t)x * N * N + c0 + c];
  }
  __syncthreads();
  stageA_fwd<N>(s, TC, 1, TC, tw, tid, nthr, true);
  __syncthreads();
  const T scale = a.vscale;
  const bool kin = a.kinetic != 0;
  auto mul = [k2, c0, scale, kin](int line, C v, int kx) {
    const int c = c0 + line;
    const int ky = scr2k<N>(c / N), kz = scr2k<N>(c % N);
    const T kk = k2[kx] + k2[ky] + k2[kz];
    const T f = kin ? scale * (T)0.5 * kk : ((kx == 0 && ky == 0 && kz == 0) ? (T)0 : scale / kk);
    return cscale(v, f);
  };
  stageB<N, 2>(s, TC, 1, TC, tw, tid, nthr, true, mul);
  __syncthreads();
  stageC_inv<N>(s, TC, 1, TC, tid, nthr, true);
  __syncthreads();
  for (int e = tid; e < N * TC; e += nthr) {
    const int x = e / TC, c = e % TC;
    w[(size_t)x * N * N + c0 + c] = s[x * TC + c];
  }
}

template <int N, typename T, int NT>
__global__ void __launch_bounds__(NT) k_poisson_yz_inv(PoisArgs<T> a) {
  using C = cplx<T>;
  extern __shared__ unsigned char smem_raw[];
  C* s = reinterpret_cast<C*>(smem_raw);
  constexpr int P = N * N;
  constexpr int S = plane_stride<N>();
  const int ng = N * N * N;
  const int x = blockIdx.x, m = blockIdx.y, tid = threadIdx.x;
  const C* w = a.work + (size_t)m * ng + (size_t)x * P;
  C* tw = s + N * S;
  stage_tables<N, C>(tw, a.tw, nullptr, tid, NT);
  for (int e = tid; e < P; e += NT) s[plane_idx<N>(e)] = w[e];
  __syncthreads();
  NoMul nm;
  stageB<N, 1>(s, N, S, 1, tw, tid, NT, true, nm);
  __syncthreads();
  stageC_inv<N>(s, N, S, 1, tid, NT, true);
  __syncthreads();
  stageB<N, 1>(s, N, 1, S, tw, tid, NT, true, nm);
  __syncthreads();
  stageC_inv<N>(s, N, 1, S, tid, NT, true);
  __syncthreads();
  const int b0 = 2 * m, b1 = 2 * m + 1;
  const size_t o0 = (size_t)b0 * ng + (size_t)x * P;
  const size_t o1 = (size_t)b1 * ng + (size_t)x * P;
  const bool has1 = b1 < a.B;
  const double c0 = a.pscale ? a.pscale[b0] : 1.0, c1 = (a.pscale && has1) ? a.pscale[b1] : 1.0;
  for (int e = tid; e < P; e += NT) {
    C v = s[plane_idx<N>(e)];
    if (a.pscale) v = cmk<C>((T)(c0 * v.x), (T)(c1 * v.y));
    if (a.out) {
      a.out[o0 + e] = v.x;
      if (has1) a.out[o1 + e] = v.y;
    }
    if (a.out64) {
      a.out64[o0 + e] = (double)v.x;
      if (has1) a.out64[o1 + e] = (double)v.y;
    }
    if (a.acc) {
      a.acc[o0 + e] += a.wn * (double)v.x;
      if (has1) a.acc[o1 + e] += a.wn * (double)v.y;
    }
  }
}

// Poisson for grids whose y-z plane does not fit in LDS (FP64 at 112^3): the
// plane passes are split into a z-line pass over tiles of PL_TL contiguous
// lines and a y-line pass over tiles of PL_TL z columns of one x plane.  The
// transforms, the scrambled spectrum order and the epilogue are those of the
// plane passes.
constexpr int PL_TL = 16;

// dir 0: pair of real densities -> work, forward z half; dir 1: work ->
// inverse z half -> outputs
template <int N, typename T>
__global__ void __launch_bounds__(256) k_poisson_z(PoisArgs<T> a, int dir) {
  using C = cplx<T>;
  extern __shared__ unsigned char smem_raw[];
  C* s = reinterpret_cast<C*>(smem_raw);
  constexpr int TL = PL_TL, S = N + 1, E = TL * N;
  const int ng = N * N * N;
  const int m = blockIdx.y, tid = threadIdx.x;
  const size_t base = (size_t)blockIdx.x * TL * N;   // lines (x, y) = blockIdx.x * TL ...
  C* tw = s + TL * S;
  stage_tables<N, C>(tw, a.tw, nullptr, tid, 256);
  const int b0 = 2 * m, b1 = 2 * m + 1;
  const bool has1 = b1 < a.B;
  NoMul nm;
  if (dir == 0) {
    const T* r0 = a.rho + (size_t)b0 * ng + base;
    const T* r1 = has1 ? a.rho + (size_t)b1 * ng + base : nullptr;
    const T i0 = a.pscale ? (T)(1.0 / a.pscale[b0]) : (T)1;
    const T i1 = (a.pscale && has1) ? (T)(1.0 / a.pscale[b1]) : (T)1;
    int bad0 = 0, bad1 = 0;
    for (int e = tid; e < E; e += 256)
      s[(e / N) * S + e % N] = load_pair<C>(r0[e] * i0, r1 ? r1[e] * i1 : (T)0, a.flags != nullptr, bad0, bad1);
    flag_bad(a.flags, b0, b1, bad0, bad1);
    __syncthreads();
    stageA_fwd<N>(s, TL, S, 1, tw, tid, 256, true);
    __syncthreads();
    stageB<N, 0>(s, TL, S, 1, tw, tid, 256, true, nm);
    __syncthreads();
    C* w = a.work + (size_t)m * ng + base;
    for (int e = tid; e < E; e += 256) w[e] = s[(e / N) * S + e % N];
    return;
  }
  const C* w = a.work + (size_t)m * ng + base;
  for (int e = tid; e < E; e += 256) s[(e / N) * S + e % N] = w[e];
  __syncthreads();
  stageB<N, 1>(s, TL, S, 1, tw, tid, 256, true, nm);
  __syncthreads();
  stageC_inv<N>(s, TL, S, 1, tid, 256, true);
  __syncthreads();
  const size_t o0 = (size_t)b0 * ng + base, o1 = (size_t)b1 * ng + base;
  const double c0 = a.pscale ? a.pscale[b0] : 1.0, c1 = (a.pscale && has1) ? a.pscale[b1] : 1.0;
  for (int e = tid; e < E; e += 256) {
    C v = s[(e / N) * S + e % N];
    if (a.pscale) v = cmk<C>((T)(c0 * v.x), (T)(c1 * v.y));
    if (a.out) {
      a.out[o0 + e] = v.x;
      if (has1) a.out[o1 + e] = v.y;
    }
    if (a.out64) {
      a.out64[o0 + e] = (double)v.x;
      if (has1) a.out64[o1 + e] = (double)v.y;
    }
    if (a.acc) {
      a.acc[o0 + e] += a.wn * (double)v.x;
      if (has1) a.acc[o1 + e] += a.wn * (double)v.y;
    }
  }
}

// y lines of PL_TL consecutive z columns of one x plane, work in place;
// dir 0: forward half, dir 1: inverse half
template <int N, typename T>
__global__ void __launch_bounds__(256) k_poisson_y(PoisArgs<T> a, int dir) {
  using C = cplx<T>;
  extern __shared__ unsigned char smem_raw[];
  C* s = reinterpret_cast<C*>(smem_raw);
  constexpr int TL = PL_TL, E = TL * N;
  const int ng = N * N * N;
  const int x = blockIdx.x / (N / TL), z0 = (blockIdx.x % (N / TL)) * TL;
  const int m = blockIdx.y, tid = threadIdx.x;
  C* w = a.work + (size_t)m * ng + (size_t)x * N * N + z0;
  C* tw = s + E;
  stage_tables<N, C>(tw, a.tw, nullptr, tid, 256);
  for (int e = tid; e < E; e += 256) s[e] = w[(size_t)(e / TL) * N + e % TL];
  __syncthreads();
  NoMul nm;
  if (dir == 0) {
    stageA_fwd<N>(s, TL, 1, TL, tw, tid, 256, true);
    __syncthreads();
    stageB<N, 0>(s, TL, 1, TL, tw, tid, 256, true, nm);
  } else {
    stageB<N, 1>(s, TL, 1, TL, tw, tid, 256, true, nm);
    __syncthreads();
    stageC_inv<N>(s, TL, 1, TL, tid, 256, true);
  }
  __syncthreads();
  for (int e = tid; e < E; e += 256) w[(size_t)(e / TL) * N + e % TL] = s[e];
}

// ---------------------------------------------------------------------------
// pointwise helpers
// ---------------------------------------------------------------------------
// rho_b = phi_i phi_j (FP64)
__global__ void k_pair_density(const double* __restrict__ phi, const int* __restrict__ pq,
                               int B, size_t ng, double* __restrict__ rho) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (i >= ng || b >= B) return;
  const int p = pq[2 * b], q = pq[2 * b + 1];
  rho[(size_t)b * ng + i] = phi[(size_t)p * ng + i] * phi[(size_t)q * ng + i];
}

// eta_l(0) = L^-1/2 sum_s xi[l, s] phi_s  (Eq. 14), FP64, and H_0 = conj(Ph) eta(0)
template <typename T>
__global__ void k_stoch_orbitals(const double* __restrict__ phi, const signed char* __restrict__ xi,
                                 int L, int n_occ, int deterministic, size_t ng, double inv_sqrt_l,
                                 const cplx<T>* __restrict__ ph, double* __restrict__ eta0,
                                 cplx<T>* __restrict__ H0) {
  using C = cplx<T>;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int l = blockIdx.y;
  if (i >= ng) return;
  double v = 0.0;
  if (deterministic) {
    v = phi[(size_t)l * ng + i];
  } else {
    for (int s = 0; s < n_occ; ++s) v += (double)xi[(size_t)l * n_occ + s] * phi[(size_t)s * ng + i];
    v *= inv_sqrt_l;
  }
  eta0[(size_t)l * ng + i] = v;
  const C p = ph[i];
  H0[(size_t)l * ng + i] = cmk<C>((T)(v * (double)p.x), (T)(-v * (double)p.y));
}

// d_{b,l}(0) = -i q_b eta_l(0)
template <typename T>
__global__ void k_kick(const double* __restrict__ q, const double* __restrict__ eta0, int L,
                       size_t ng, cplx<T>* __restrict__ d) {
  using C = cplx<T>;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int f = blockIdx.y;
  if (i >= ng) return;
  const int b = f / L, l = f % L;
  const double v = q[(size_t)b * ng + i] * eta0[(size_t)l * ng + i];
  d[(size_t)f * ng + i] = cmk<C>((T)0, (T)(-v));
}

// end-of-step state from the mid-step one: d <- Ph (d - i dt/2 u_b H_l) and
// E_l = Ph H_l (from_mid = 1); E_l = Ph H_l only (0); at t = 0 E_l is the
// real eta_l(0) itself (2).
template <typename T>
__global__ void k_clean_finish(cplx<T>* __restrict__ d, const T* __restrict__ u,
                               const cplx<T>* __restrict__ H, const cplx<T>* __restrict__ ph,
                               const double* __restrict__ eta0, cplx<T>* __restrict__ E, int L,
                               size_t ng, T dt, int from_mid) {
  using C = cplx<T>;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int f = blockIdx.y;
  if (i >= ng) return;
  const int b = f / L, l = f % L;
  if (from_mid == 2) {
    if (f < L) E[(size_t)l * ng + i] = cmk<C>((T)eta0[(size_t)l * ng + i], (T)0);
    return;
  }
  const C p = ph[i];
  const C h = H[(size_t)l * ng + i];
  if (f < L) E[(size_t)l * ng + i] = cmul(p, h);
  if (from_mid == 1) {
    C v = d[(size_t)f * ng + i];
    const T cu = (T)0.5 * dt * u[(size_t)b * ng + i];
    v = cmk<C>(v.x + cu * h.y, v.y - cu * h.x);
    d[(size_t)f * ng + i] = cmul(p, v);
  }
}

// dn_b = 4 sum_l Re(conj(E_l) d_{b,l})
template <typename T>
__global__ void k_density_end(const cplx<T>* __restrict__ d, const cplx<T>* __restrict__ E,
                              int L, size_t ng, T* __restrict__ dens) {
  using C = cplx<T>;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (i >= ng) return;
  T acc = 0;
  for (int l = 0; l < L; ++l) {
    const C v = d[((size_t)b * L + l) * ng + i];
    const C e = E[(size_t)l * ng + i];
    acc += e.x * v.x + e.y * v.y;
  }
  dens[(size_t)b * ng + i] = (T)4 * acc;
}

// ---------------------------------------------------------------------------
// cleaning (Eq. 15, linearised): d <- Q d - Re<E_l, Q d>/||eta_l(0)||^2 E_l
// ---------------------------------------------------------------------------
// partial coefficients over a chunk of grid points:
//   part[chunk][f][s] = sum_{r in chunk} phi_s(r) d_f(r)   (s < S)
//   part[chunk][f][S] = sum_{r in chunk} conj(E_l(f)) d_f(r)
// tile: 32 fields x 32 states per block, 256 threads, 2x2 per thread.
constexpr int CT_F = 32, CT_S = 32, CT_R = 32;
template <typename T>
__global__ void __launch_bounds__(256) k_clean_coef(const cplx<T>* __restrict__ d, int F,
                                                    const T* __restrict__ phi, int S,
                                                    const cplx<T>* __restrict__ E, int L,
                                                    size_t ng, int chunk,
                                                    cplx<double>* __restrict__ part) {
  using C = cplx<T>;
  __shared__ C sd[CT_F][CT_R + 1];
  __shared__ T sp[CT_S][CT_R + 1];
  const int f0 = blockIdx.x * CT_F;
  const int s0 = blockIdx.y * CT_S;  // s == S row block also carries the E dot
  const int kc = blockIdx.z;
  const size_t r0 = (size_t)kc * chunk;
  const size_t r1 = min(ng, r0 + (size_t)chunk);
  const int tid = threadIdx.x;
  const int tf = tid / 16, ts = tid % 16;
  C acc[2][2];
  C acce[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    acce[i] = cmk<C>(0, 0);
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = cmk<C>(0, 0);
  }
  const bool do_e = (s0 == 0);
  for (size_t rb = r0; rb < r1; rb += CT_R) {
    for (int e = tid; e < CT_F * CT_R; e += 256) {
      const int ff = e / CT_R, rr = e % CT_R;
      const int f = f0 + ff;
      const size_t r = rb + rr;
      sd[ff][rr] = (f < F && r < r1) ? d[(size_t)f * ng + r] : cmk<C>(0, 0);
    }
    for (int e = tid; e < CT_S * CT_R; e += 256) {
      const int ss = e / CT_R, rr = e % CT_R;
      const int s = s0 + ss;
      const size_t r = rb + rr;
      sp[ss][rr] = (s < S && r < r1) ? phi[(size_t)s * ng + r] : (T)0;
    }
    __syncthreads();
#pragma unroll 8
    for (int rr = 0; rr < CT_R; ++rr) {
      const C d0 = sd[tf * 2][rr], d1 = sd[tf * 2 + 1][rr];
      const T p0 = sp[ts * 2][rr], p1 = sp[ts * 2 + 1][rr];
      acc[0][0] = cmk<C>(acc[0][0].x + d0.x * p0, acc[0][0].y + d0.y * p0);
      acc[0][1] = cmk<C>(acc[0][1].x + d0.x * p1, acc[0][1].y + d0.y * p1);
      acc[1][0] = cmk<C>(acc[1][0].x + d1.x * p0, acc[1][0].y + d1.y * p0);
      acc[1][1] = cmk<C>(acc[1][1].x + d1.x * p1, acc[1][1].y + d1.y * p1);
    }
    if (do_e && ts == 0) {
      for (int i = 0; i < 2; ++i) {
        const int f = f0 + tf * 2 + i;
        if (f >= F) continue;
        const int l = f % L;
        for (int rr = 0; rr < CT_R; ++rr) {
          const size_t r = rb + rr;
          if (r >= r1) break;
          const C ee = E[(size_t)l * ng + r];
          acce[i] = cadd(acce[i], cmulc(sd[tf * 2 + i][rr], ee));
        }
      }
    }
    __syncthreads();
  }
  cplx<double>* out = part + (size_t)kc * F * (S + 1);
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int f = f0 + tf * 2 + i;
    if (f >= F) continue;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int s = s0 + ts * 2 + j;
      if (s < S) out[(size_t)f * (S + 1) + s] = cmk<cplx<double>>(acc[i][j].x, acc[i][j].y);
    }
    if (do_e && ts == 0) out[(size_t)f * (S + 1) + S] = cmk<cplx<double>>(acce[i].x, acce[i].y);
  }
}

// reduce partials over chunks; coef[f][s] = h^3 sum (s < S); coef[f][S] = h^3 <E,d>
__global__ void k_clean_reduce(const cplx<double>* __restrict__ part, int nchunk, int FS,
                               double dv, cplx<double>* __restrict__ coef) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= FS) return;
  double x = 0, y = 0;
  for (int k = 0; k < nchunk; ++k) {
    const cplx<double> v = part[(size_t)k * FS + i];
    x += v.x;
    y += v.y;
  }
  coef[i] = cmk<cplx<double>>(x * dv, y * dv);
}

// renormalisation factor per field: c_f = Re(<E,d> - sum_s conj(De[l][s]) C[f][s]) / N0_l;
// one wave per field, lanes over s, a fixed shuffle tree
__global__ void __launch_bounds__(256) k_clean_renorm(cplx<double>* __restrict__ coef, int F, int S,
                                                      const cplx<double>* __restrict__ coefE,
                                                      const double* __restrict__ n0, int L, int renorm) {
  const int f = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (f >= F) return;
  const int l = f % L;
  cplx<double>* c = coef + (size_t)f * (S + 1);
  double r = 0;
  for (int s = lane; s < S; s += 64) {
    const cplx<double> de = coefE[(size_t)l * (S + 1) + s];
    const cplx<double> cc = c[s];
    r += de.x * cc.x + de.y * cc.y;
  }
  for (int off = 32; off > 0; off >>= 1) r += __shfl_down(r, off, 64);
  if (lane == 0) {
    const double v = c[S].x - r;
    c[S] = cmk<cplx<double>>(renorm ? v / n0[l] : 0.0, 0.0);
  }
}

// d_f(r) -= sum_s C[f][s] phi_s(r) + c_f E_l(r)
// block: 64 grid points x up to 16 fields of one chunk; coefficients staged in LDS
template <typename T>
__global__ void __launch_bounds__(256) k_clean_update(cplx<T>* __restrict__ d, int F,
                                                      const T* __restrict__ phi, int S,
                                                      const cplx<T>* __restrict__ E, int L,
                                                      size_t ng,
                                                      const cplx<double>* __restrict__ coef) {
  using C = cplx<T>;
  constexpr int FB = 16, RB = 64, SB = 128;
  __shared__ C sc[FB][SB + 1];
  __shared__ T sphi[32][RB];
  const size_t r0 = (size_t)blockIdx.x * RB;
  const int fb0 = blockIdx.y * FB;
  const int tid = threadIdx.x;
  const int rr = tid % RB, fq = tid / RB;  // 4 field groups of 4
  const size_t r = r0 + rr;
  C acc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = cmk<C>(0, 0);
  for (int sb = 0; sb < S; sb += SB) {
    const int sn = min(SB, S - sb);
    __syncthreads();
    for (int e = tid; e < FB * sn; e += 256) {
      const int ff = e / sn, ss = e % sn;
      const int f = fb0 + ff;
      const cplx<double> v = (f < F) ? coef[(size_t)f * (S + 1) + sb + ss] : cmk<cplx<double>>(0, 0);
      sc[ff][ss] = cmk<C>((T)v.x, (T)v.y);
    }
    for (int s2 = 0; s2 < sn; s2 += 32) {
      const int sm = min(32, sn - s2);
      __syncthreads();
      for (int e = tid; e < 32 * RB; e += 256) {
        const int ss = e / RB, q = e % RB;
        sphi[ss][q] = (ss < sm && r0 + q < ng) ? phi[(size_t)(sb + s2 + ss) * ng + r0 + q] : (T)0;
      }
      __syncthreads();
      for (int ss = 0; ss < sm; ++ss) {
        const T p = sphi[ss][rr];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const C c = sc[fq * 4 + i][s2 + ss];
          acc[i] = cmk<C>(acc[i].x + c.x * p, acc[i].y + c.y * p);
        }
      }
    }
  }
  if (r >= ng) return;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int f = fb0 + fq * 4 + i;
    if (f >= F) continue;
    const int l = f % L;
    const T cr = (T)coef[(size_t)f * (S + 1) + S].x;
    const C e = E[(size_t)l * ng + r];
    C v = d[(size_t)f * ng + r];
    v = cmk<C>(v.x - acc[i].x - cr * e.x, v.y - acc[i].y - cr * e.y);
    d[(size_t)f * ng + r] = v;
  }
}

// out[b] = q[b] + wpol[b]
__global__ void k_add(const double* __restrict__ a, const double* __restrict__ b, size_t n,
                      double* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] + b[i];
}

// ||eta_l(0)||^2 h^3 partial sums
__global__ void k_norms(const double* __restrict__ eta0, size_t ng, double dv, double* __restrict__ out) {
  const int l = blockIdx.x;
  __shared__ double red[256];
  double acc = 0;
  for (size_t i = threadIdx.x; i < ng; i += 256) {
    const double v = eta0[(size_t)l * ng + i];
    acc += v * v;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[l] = red[0] * dv;
}

__global__ void k_add_f32(const double* __restrict__ a, const double* __restrict__ b, size_t n,
                          float* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)(a[i] + b[i]);
}

// The unperturbed set evolves by a unitary map, so its norms stay those of
// eta_l(0).  First pass: NORM_NB blocks per orbital sum |H_l|^2 over their
// share of the points (FP64) into part[l][blk]; second pass (one block):
// the partials of each orbital added in block order and, on a drift beyond
// tol (or a non-finite sum), every pair of the batch marked.
constexpr int NORM_NB = 64;
template <typename T>
__global__ void __launch_bounds__(256) k_norm_part(const cplx<T>* __restrict__ H, size_t ng,
                                                   double* __restrict__ part) {
  const int l = blockIdx.y, blk = blockIdx.x;
  const size_t per = (ng + NORM_NB - 1) / NORM_NB;
  const size_t i0 = (size_t)blk * per, i1 = i0 + per < ng ? i0 + per : ng;
  __shared__ double red[256];
  double acc = 0;
  for (size_t i = i0 + threadIdx.x; i < i1; i += 256) {
    const cplx<T> v = H[(size_t)l * ng + i];
    acc += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)l * NORM_NB + blk] = red[0];
}

__global__ void __launch_bounds__(256) k_norm_check(const double* __restrict__ part, int L, double dv,
                                                    const double* __restrict__ n0, double tol,
                                                    int* __restrict__ flags, int B) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int l = threadIdx.x; l < L; l += 256) {
    double acc = 0;
    for (int k = 0; k < NORM_NB; ++k) acc += part[(size_t)l * NORM_NB + k];
    const double r = acc * dv / n0[l] - 1.0;
    if (!(fabs(r) <= tol)) atomicOr(&bad, 1);
  }
  __syncthreads();
  if (bad)
    for (int b = threadIdx.x; b < B; b += 256) atomicOr(&flags[b], 2);
}

template <typename W>
__global__ void k_nan_flagged(W* __restrict__ w, size_t ng, const int* __restrict__ flags) {
  const int b = blockIdx.y;
  if (!flags[b]) return;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < ng; i += (size_t)gridDim.x * blockDim.x)
    w[(size_t)b * ng + i] = (W)__builtin_nan("");
}

template <typename T>
__global__ void k_to_real(const double* __restrict__ in, size_t n, T* __restrict__ out) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (T)in[i];
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
template <int N> constexpr int yz_threads() { return N >= 64 ? 512 : 256; }
template <int N> constexpr int x_tc() { return N <= 16 ? 64 : 32; }

// tile width of the x pass and block size of the plane passes are tunable;
// a variant is valid when the work items fill the block
template <int N, int TC> constexpr bool x_valid() {
  return (N * N) % TC == 0 && (TC * Fac<N>::N2) % 256 == 0;
}

// dynamic LDS of the propagation passes: data region + twiddle and phase tables
template <int N, int TC, typename T> constexpr size_t x_lds() {
  return sizeof(cplx<T>) * ((size_t)N * TC + 2 * N);
}
template <int N, typename T> constexpr size_t yz_lds() {
  return sizeof(cplx<T>) * ((size_t)N * plane_stride<N>() + 2 * N);
}

// ---------------------------------------------------------------------------
// Work-list passes of uneven batches: for one grid size, a persistent grid
// (as many blocks as the CUs hold) walks the items of every listed system,
// each with its own pairs and buffers.  An item computes exactly what the
// per-system kernel computes for it (the tile shape changes only which
// thread does what), so results equal the per-system passes bit for bit.
// One instantiation per grid size keeps each one's registers those of its
// per-system kernel.
// ---------------------------------------------------------------------------
// The items of a persistent list launch: workgroup ids are dealt
// round-robin to the eight XCDs, so XCD c = id mod 8 takes the c-th eighth of
// the items, walked by its own workgroups in order; consecutive items (the
// fields of one tile, the planes of one pair) then share that XCD's L2.  The
// grid is a multiple of 8.  Within a workgroup the items only grow, so its
// entry index only moves forward.
struct ListWalk {
  unsigned it, hi, step;
  __device__ ListWalk(unsigned total) {
    const unsigned c = blockIdx.x & 7u, per = (total + 7u) / 8u;
    step = gridDim.x >> 3;
    it = c * per + (blockIdx.x >> 3);
    hi = min(total, c * per + per);
  }
};
template <typename E>
__device__ __forceinline__ int list_advance(const E* __restrict__ list, int nsys, int k, unsigned it) {
  while (k + 1 < nsys && list[k + 1].first <= it) ++k;
  return k;
}

template <int N>
__global__ void __launch_bounds__(256) k_prop_x_list(const XListSys* __restrict__ list, int nsys, unsigned total) {
  extern __shared__ unsigned char smem_raw[];
  float2* s = reinterpret_cast<float2*>(smem_raw);
  int k = 0;
  for (ListWalk w(total); w.it < w.hi; w.it += w.step) {
    k = list_advance(list, nsys, k, w.it);
    const XListSys e = list[k];
    const unsigned loc = w.it - e.first;
    prop_x_item<N, x_tc<N>(), float, false>(e.a, (int)(loc % (unsigned)e.a.nf), (int)(loc / (unsigned)e.a.nf), s);
    __syncthreads();   // the next item restages the tables and the tile
  }
}

template <int N>
__global__ void __launch_bounds__(yz_threads<N>()) k_prop_yz_list(const YZListSys* __restrict__ list, int nsys,
                                                                 unsigned total) {
  extern __shared__ unsigned char smem_raw[];
  float2* s = reinterpret_cast<float2*>(smem_raw);
  int k = 0;
  for (ListWalk w(total); w.it < w.hi; w.it += w.step) {
    k = list_advance(list, nsys, k, w.it);
    const YZListSys e = list[k];
    const unsigned loc = w.it - e.first;
    prop_yz_pair_item<N, float, yz_threads<N>()>(e.a, (int)(loc % (unsigned)N), (int)(loc / (unsigned)N), s);
    __syncthreads();
  }
}

bool prop_list_grid(int n) { return n == 16 || n == 24 || n == 32 || n == 48 || n == 64; }
unsigned prop_x_list_items(int n, int pairs) {
  const int tc = n <= 16 ? 64 : 32;   // x_tc
  return (unsigned)pairs * (unsigned)(n * n / tc);
}
unsigned prop_yz_list_items(int n, int pairs) { return (unsigned)n * (unsigned)pairs; }

// blocks of a persistent list launch: what the CUs hold at once, a multiple
// of the 8 XCDs
static hipError_t list_grid(const void* k, int block, size_t lds, unsigned total, unsigned* grid) {
  int dev = 0, ncu = 0, per = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, block, lds);
  if (e != hipSuccess) return e;
  const unsigned g = std::min((total + 7u) / 8u * 8u, (unsigned)(std::max(1, per) * ncu));
  *grid = std::max(8u, g / 8u * 8u);
  return hipSuccess;
}

template <int N>
static hipError_t prop_list_go(const XListSys* xl, const YZListSys* yl, int nsys, unsigned total, hipStream_t st) {
  const void* k;
  int block;
  size_t lds;
  if (xl) {
    k = (const void*)k_prop_x_list<N>;
    block = 256;
    lds = x_lds<N, x_tc<N>(), float>();
  } else {
    k = (const void*)k_prop_yz_list<N>;
    block = yz_threads<N>();
    lds = yz_lds<N, float>();
  }
  hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  unsigned g = 0;
  if (e == hipSuccess) e = list_grid(k, block, lds, total, &g);
  if (e != hipSuccess) return e;
  if (xl)
    hipLaunchKernelGGL(k_prop_x_list<N>, dim3(g), dim3(256), lds, st, xl, nsys, total);
  else
    hipLaunchKernelGGL(k_prop_yz_list<N>, dim3(g), dim3(yz_threads<N>()), lds, st, yl, nsys, total);
  return hipGetLastError();
}

static hipError_t prop_list(int n, const XListSys* xl, const YZListSys* yl, int nsys, unsigned total,
                            hipStream_t st) {
  if (nsys < 1 || total == 0) return hipErrorInvalidValue;
  switch (n) {
    case 16: return prop_list_go<16>(xl, yl, nsys, total, st);
    case 24: return prop_list_go<24>(xl, yl, nsys, total, st);
    case 32: return prop_list_go<32>(xl, yl, nsys, total, st);
    case 48: return prop_list_go<48>(xl, yl, nsys, total, st);
    case 64: return prop_list_go<64>(xl, yl, nsys, total, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_prop_x_list(int n, const XListSys* list, int nsys, unsigned total, hipStream_t st) {
  return prop_list(n, list, nullptr, nsys, total, st);
}
hipError_t launch_prop_yz_list(int n, const YZListSys* list, int nsys, unsigned total, hipStream_t st) {
  return prop_list(n, nullptr, list, nsys, total, st);
}

template <int N, typename T>
struct Launch {
  // plain launch, or one that records ev's events in its own dispatch
  template <typename K, typename A>
  static void go(K kern, dim3 grid, dim3 block, size_t sm, hipStream_t st, const LaunchEvents* ev, const A& a) {
    if (ev)
      hipExtLaunchKernelGGL(kern, grid, block, (uint32_t)sm, st, ev->start, ev->stop, 0, a);
    else
      hipLaunchKernelGGL(kern, grid, block, sm, st, a);
  }
  template <int TC>
  static hipError_t prop_x_tc(const PropXArgs<T>& a, int F, hipStream_t st, const LaunchEvents* ev) {
    if constexpr (!x_valid<N, TC>()) {
      return hipErrorInvalidValue;
    } else {
      PropXArgs<T> b = a;
      b.nf = F;
      const dim3 grid = field_tile_grid(a.order, F, N * N / TC);
      size_t sm = x_lds<N, TC, T>();
      if (a.mode == PX_ETA0)
        go(k_prop_x<N, TC, T, true>, grid, dim3(256), sm, st, ev, b);
      else
        go(k_prop_x<N, TC, T, false>, grid, dim3(256), sm, st, ev, b);
      return hipGetLastError();
    }
  }
  // F: fields (unperturbed set) or pairs (perturbed set); tc 0 = default
  static hipError_t prop_x(const PropXArgs<T>& a, int F, hipStream_t st, int tc, const LaunchEvents* ev) {
    if (tc == 0) tc = x_tc<N>();
    switch (tc) {
      case 16: return prop_x_tc<16>(a, F, st, ev);
      case 32: return prop_x_tc<32>(a, F, st, ev);
      case 64: return prop_x_tc<64>(a, F, st, ev);
      default: return hipErrorInvalidValue;
    }
  }
  template <int NT>
  static hipError_t prop_yz_nt(const PropYZArgs<T>& a, int nb, hipStream_t st, const LaunchEvents* ev) {
    size_t sm = yz_lds<N, T>();
    if (a.density)
      go(k_prop_yz<N, T, NT, true>, dim3(N, nb), dim3(NT), sm, st, ev, a);
    else
      go(k_prop_yz<N, T, NT, false>, dim3(N, nb), dim3(NT), sm, st, ev, a);
    return hipGetLastError();
  }
  static constexpr bool yz_split() { return yz_lds<N, T>() > 80 * 1024; }
  // the register-line plane pass (prop_yz_reg) replaces the two line passes
  static constexpr bool yz_reg() { return std::is_same<T, float>::value && N == 112; }
  // the plane, the twiddle and phase tables, the density sums
  static constexpr size_t yz_reg_lds() {
    return sizeof(float2) * ((size_t)N * (N + 1) + 2 * N) + sizeof(float) * (size_t)N * N;
  }
  static hipError_t prop_yz_reg(const PropYZArgs<T>& a, int nb, hipStream_t st, const LaunchEvents* ev) {
    if constexpr (yz_reg()) {
      PropYZArgs<T> ar = a;
      ar.nf = nb;
      const dim3 gr = a.order ? field_tile_grid(1, nb, N) : dim3(N, nb);
      if (a.fused == 2) {
        if (a.density)
          go(k_prop_yz_rt<N, true>, gr, dim3(YZR_NT), yz_reg_lds(), st, ev, ar);
        else
          go(k_prop_yz_rt<N, false>, gr, dim3(YZR_NT), yz_reg_lds(), st, ev, ar);
      } else if (a.density)
        go(k_prop_yz_reg<N, true>, gr, dim3(YZR_NT), yz_reg_lds(), st, ev, ar);
      else
        go(k_prop_yz_reg<N, false>, gr, dim3(YZR_NT), yz_reg_lds(), st, ev, ar);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  // the two line passes: ev times the z pass, ev2 the y pass
  static hipError_t prop_zy(const PropYZArgs<T>& a, int nb, hipStream_t st, const LaunchEvents* ev,
                            const LaunchEvents* ev2) {
    if constexpr (N % PY_TZ == 0 && (N * N) % PZ_TL == 0 && (N * PY_TZ) % PY_NT == 0) {
      const int F = a.density ? nb * a.L : nb;
      const size_t smz = sizeof(cplx<T>) * ((size_t)PZ_TL * (N + 1) + 2 * N);
      const size_t smy = sizeof(cplx<T>) * ((size_t)N * PY_ES + 2 * N);
      go(k_prop_z<N, T>, dim3(N * N / PZ_TL, F), dim3(256), smz, st, ev, a);
      PropYZArgs<T> ay = a;
      ay.nf = nb;
      const dim3 gy = field_tile_grid(a.order, nb, N * (N / PY_TZ));
      if (a.density)
        go(k_prop_y<N, T, true>, gy, dim3(PY_NT), smy, st, ev2, ay);
      else
        go(k_prop_y<N, T, false>, gy, dim3(PY_NT), smy, st, ev2, ay);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  static hipError_t prop_yz(const PropYZArgs<T>& a, int nb, hipStream_t st, int nt, const LaunchEvents* ev,
                            const LaunchEvents* ev2) {
    if (a.fused && yz_reg()) return prop_yz_reg(a, nb, st, ev);   // 1 cross-lane, 2 transposed
    if constexpr (yz_split()) return prop_zy(a, nb, st, ev, ev2);
    if (nt == 0) nt = yz_threads<N>();
    switch (nt) {
      case 256: return prop_yz_nt<256>(a, nb, st, ev);
      case 512: return prop_yz_nt<512>(a, nb, st, ev);
      default: return hipErrorInvalidValue;
    }
  }
  static hipError_t poisson(const PoisArgs<T>& a, hipStream_t st) {
    constexpr int NT = yz_threads<N>();
    constexpr int TC = x_tc<N>();
    const int M = (a.B + 1) / 2;
    const size_t smp = yz_lds<N, T>();
    const size_t smx = x_lds<N, TC, T>();
    if constexpr (yz_lds<N, T>() > 80 * 1024) {
      // the plane does not fit, or would leave one block per CU: separate
      // z-line and y-line passes
      static_assert(N % PL_TL == 0, "line tiles must divide the grid");
      const size_t smz = sizeof(cplx<T>) * ((size_t)PL_TL * (N + 1) + N);
      const size_t smy = sizeof(cplx<T>) * ((size_t)PL_TL * N + N);
      const dim3 gz(N * N / PL_TL, M), gy(N * (N / PL_TL), M);
      hipLaunchKernelGGL((k_poisson_z<N, T>), gz, dim3(256), smz, st, a, 0);
      hipLaunchKernelGGL((k_poisson_y<N, T>), gy, dim3(256), smy, st, a, 0);
      hipLaunchKernelGGL((k_poisson_x<N, TC, T>), dim3(N * N / TC, M), dim3(256), smx, st, a);
      hipLaunchKernelGGL((k_poisson_y<N, T>), gy, dim3(256), smy, st, a, 1);
      hipLaunchKernelGGL((k_poisson_z<N, T>), gz, dim3(256), smz, st, a, 1);
    } else {
      hipLaunchKernelGGL((k_poisson_yz_fwd<N, T, NT>), dim3(N, M), dim3(NT), smp, st, a);
      hipLaunchKernelGGL((k_poisson_x<N, TC, T>), dim3(N * N / TC, M), dim3(256), smx, st, a);
      hipLaunchKernelGGL((k_poisson_yz_inv<N, T, NT>), dim3(N, M), dim3(NT), smp, st, a);
    }
    return hipGetLastError();
  }
  template <int TC> static void conf_x() {
    if constexpr (x_valid<N, TC>()) {
      const int smx = (int)x_lds<N, TC, T>();
      (void)hipFuncSetAttribute((const void*)k_prop_x<N, TC, T, true>, hipFuncAttributeMaxDynamicSharedMemorySize, smx);
      (void)hipFuncSetAttribute((const void*)k_prop_x<N, TC, T, false>, hipFuncAttributeMaxDynamicSharedMemorySize, smx);
    }
  }
  template <int NT> static void conf_yz() {
    if constexpr (yz_lds<N, T>() > 160 * 1024) return;   // the plane kernels never run
    const int smp = (int)yz_lds<N, T>();
    (void)hipFuncSetAttribute((const void*)k_prop_yz<N, T, NT, true>, hipFuncAttributeMaxDynamicSharedMemorySize, smp);
    (void)hipFuncSetAttribute((const void*)k_prop_yz<N, T, NT, false>, hipFuncAttributeMaxDynamicSharedMemorySize, smp);
  }
  static void configure() {
    constexpr int NT = yz_threads<N>();
    constexpr int TC = x_tc<N>();
    const int smp = (int)yz_lds<N, T>();
    const int smx = (int)x_lds<N, TC, T>();
    conf_x<16>();
    conf_x<32>();
    conf_x<64>();
    conf_yz<256>();
    conf_yz<512>();
    if constexpr (yz_lds<N, T>() <= 160 * 1024) {
      (void)hipFuncSetAttribute((const void*)k_poisson_yz_fwd<N, T, NT>, hipFuncAttributeMaxDynamicSharedMemorySize, smp);
      (void)hipFuncSetAttribute((const void*)k_poisson_yz_inv<N, T, NT>, hipFuncAttributeMaxDynamicSharedMemorySize, smp);
    }
    (void)hipFuncSetAttribute((const void*)k_poisson_x<N, TC, T>, hipFuncAttributeMaxDynamicSharedMemorySize, smx);
    if constexpr (yz_reg()) {
      (void)hipFuncSetAttribute((const void*)k_prop_yz_reg<N, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)yz_reg_lds());
      (void)hipFuncSetAttribute((const void*)k_prop_yz_reg<N, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)yz_reg_lds());
      (void)hipFuncSetAttribute((const void*)k_prop_yz_rt<N, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)yz_reg_lds());
      (void)hipFuncSetAttribute((const void*)k_prop_yz_rt<N, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)yz_reg_lds());
    }
  }
};

// a grid is supported when its line transforms are instantiated and its y-z
// step fits: the plane pass needs the padded plane in LDS, the line passes
// (taken where the plane would leave one block per CU) only their tiles
template <typename T>
bool grid_supported(int n) {
  bool split;
  switch (n) {
    case 16: split = Launch<16, T>::yz_split(); break;
    case 24: split = Launch<24, T>::yz_split(); break;
    case 32: split = Launch<32, T>::yz_split(); break;
    case 48: split = Launch<48, T>::yz_split(); break;
    case 64: split = Launch<64, T>::yz_split(); break;
    case 112: split = Launch<112, T>::yz_split(); break;
    default: return false;
  }
  return split || sizeof(cplx<T>) * ((size_t)n * (n + 1) + 2 * (size_t)n) <= 160 * 1024;
}

#define BSE_DISPATCH_N(n, T, CALL)                \
  switch (n) {                                    \
    case 16: return Launch<16, T>::CALL;          \
    case 24: return Launch<24, T>::CALL;          \
    case 32: return Launch<32, T>::CALL;          \
    case 48: return Launch<48, T>::CALL;          \
    case 64: return Launch<64, T>::CALL;          \
    case 112: return Launch<112, T>::CALL;        \
    default: return hipErrorInvalidValue;         \
  }

template <typename T>
hipError_t launch_prop_x(int n, const PropXArgs<T>& a, int F, hipStream_t st, int tc, const LaunchEvents* ev) {
  BSE_DISPATCH_N(n, T, prop_x(a, F, st, tc, ev));
}
template <typename T>
hipError_t launch_prop_yz(int n, const PropYZArgs<T>& a, int nb, hipStream_t st, int nt,
                          const LaunchEvents* ev, const LaunchEvents* ev2) {
  BSE_DISPATCH_N(n, T, prop_yz(a, nb, st, nt, ev, ev2));
}
template <typename T>
bool prop_yz_split(int n) {
  switch (n) {
    case 16: return Launch<16, T>::yz_split();
    case 24: return Launch<24, T>::yz_split();
    case 32: return Launch<32, T>::yz_split();
    case 48: return Launch<48, T>::yz_split();
    case 64: return Launch<64, T>::yz_split();
    case 112: return Launch<112, T>::yz_split();
    default: return false;
  }
}
template <typename T>
bool prop_yz_fused(int n) {
  return n == 112 && Launch<112, T>::yz_reg();
}
template <typename T>
hipError_t launch_poisson(int n, const PoisArgs<T>& a, hipStream_t st) {
  BSE_DISPATCH_N(n, T, poisson(a, st));
}
template <typename T>
void configure_kernels(int n) {
  switch (n) {
    case 16: Launch<16, T>::configure(); break;
    case 24: Launch<24, T>::configure(); break;
    case 32: Launch<32, T>::configure(); break;
    case 48: Launch<48, T>::configure(); break;
    case 64: Launch<64, T>::configure(); break;
    case 112: Launch<112, T>::configure(); break;
    default: break;
  }
}

static inline dim3 pw_grid(size_t ng, int y) { return dim3((unsigned)((ng + 255) / 256), y); }

hipError_t launch_pair_density(const double* phi, const int* pq, int B, size_t ng, double* rho,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_pair_density, pw_grid(ng, B), dim3(256), 0, st, phi, pq, B, ng, rho);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_stoch_orbitals(const double* phi, const signed char* xi, int L, int n_occ,
                                 int deterministic, size_t ng, const cplx<T>* ph, double* eta0,
                                 cplx<T>* H0, hipStream_t st) {
  hipLaunchKernelGGL((k_stoch_orbitals<T>), pw_grid(ng, L), dim3(256), 0, st, phi, xi, L, n_occ,
                     deterministic, ng, 1.0 / sqrt((double)L), ph, eta0, H0);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_kick(const double* q, const double* eta0, int L, int F, size_t ng, cplx<T>* d,
                       hipStream_t st) {
  hipLaunchKernelGGL((k_kick<T>), pw_grid(ng, F), dim3(256), 0, st, q, eta0, L, ng, d);
  return hipGetLastError();
}
// E_l = Ph H_l (or eta_l(0) at t = 0) for the L unperturbed orbitals only
template <typename T>
__global__ void k_clean_e(const cplx<T>* __restrict__ H, const cplx<T>* __restrict__ ph,
                          const double* __restrict__ eta0, cplx<T>* __restrict__ E, size_t ng, int t0) {
  using C = cplx<T>;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int l = blockIdx.y;
  if (i >= ng) return;
  if (t0) E[(size_t)l * ng + i] = cmk<C>((T)eta0[(size_t)l * ng + i], (T)0);
  else E[(size_t)l * ng + i] = cmul(ph[i], H[(size_t)l * ng + i]);
}

template <typename T>
hipError_t launch_clean(const CleanArgs<T>& a, hipStream_t st) {
  const int S = a.S;
  if constexpr (std::is_same<T, float>::value) {
    // 1. E; the mid-step to end-of-step conversion of d is fused into the
    //    matrix-core kernels (loader of the coefficient GEMM, epilogue of
    //    the update) instead of a pass of its own
    hipLaunchKernelGGL((k_clean_e<T>), pw_grid(a.ng, a.L), dim3(256), 0, st, a.H, a.ph, a.eta0, a.E,
                       a.ng, a.from_mid == 2 ? 1 : 0);
    MidArgs mid{};
    mid.on = a.from_mid == 1 ? 1 : 0;
    mid.u = a.u;
    mid.H = a.H;
    mid.ph = a.ph;
    mid.L = a.L;
    mid.half_dt = 0.5f * a.dt;
    mid.ng = a.ng;
    const MidArgs off{};
    const PhiSplit ps{a.phih, a.phil, a.phith, a.phitl, S, clean_sp(S)};
    // 2. coefficients and <E_l, d_f> on the matrix cores
    hipError_t e = launch_coef_x3(a.d, a.F, ps, a.ng, clean_chunk_d(a.F, S, a.ng), a.part32, a.dv, a.coef, st, mid,
                                  a.E, a.L, a.gpart);
    if (e != hipSuccess) return e;
    e = launch_coef_x3(a.E, a.L, ps, a.ng, CLEAN_CHUNK_E, a.part32, a.dv, a.coefE, st, off, a.E, a.L,
                       nullptr);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_clean_renorm, dim3((a.F + 3) / 4), dim3(256), 0, st, a.coef, a.F, S,
                       a.coefE, a.n0, a.L, a.renorm);
    // 3. update on the matrix cores
    e = launch_update_x3(a.d, a.F, ps, a.E, a.L, a.ng, a.coef, a.part32, st, mid);
    if (e != hipSuccess) return e;
  } else {
    // 1. end-of-step state and E = Ph H
    hipLaunchKernelGGL((k_clean_finish<T>), pw_grid(a.ng, a.F), dim3(256), 0, st, a.d, a.u, a.H,
                       a.ph, a.eta0, a.E, a.L, a.ng, a.dt, a.from_mid);
    // 2. coefficients of d against phi_s and E_l, and of E_l against phi_s
    const int nchunk = (int)((a.ng + a.chunk - 1) / a.chunk);
    dim3 g1((a.F + CT_F - 1) / CT_F, (S + CT_S - 1) / CT_S, nchunk);
    hipLaunchKernelGGL((k_clean_coef<T>), g1, dim3(256), 0, st, a.d, a.F, a.phi, S, a.E, a.L, a.ng,
                       a.chunk, a.part);
    hipLaunchKernelGGL(k_clean_reduce, dim3((a.F * (S + 1) + 255) / 256), dim3(256), 0, st, a.part,
                       nchunk, a.F * (S + 1), a.dv, a.coef);
    dim3 g2((a.L + CT_F - 1) / CT_F, (S + CT_S - 1) / CT_S, nchunk);
    hipLaunchKernelGGL((k_clean_coef<T>), g2, dim3(256), 0, st, a.E, a.L, a.phi, S, a.E, a.L, a.ng,
                       a.chunk, a.part);
    hipLaunchKernelGGL(k_clean_reduce, dim3((a.L * (S + 1) + 255) / 256), dim3(256), 0, st, a.part,
                       nchunk, a.L * (S + 1), a.dv, a.coefE);
    hipLaunchKernelGGL(k_clean_renorm, dim3((a.F + 3) / 4), dim3(256), 0, st, a.coef, a.F, S,
                       a.coefE, a.n0, a.L, a.renorm);
    // 3. update
    dim3 g3((unsigned)((a.ng + 63) / 64), (a.F + 15) / 16);
    hipLaunchKernelGGL((k_clean_update<T>), g3, dim3(256), 0, st, a.d, a.F, a.phi, S, a.E, a.L,
                       a.ng, a.coef);
  }
  // 4. density of the cleaned state
  hipLaunchKernelGGL((k_density_end<T>), pw_grid(a.ng, a.F / a.L), dim3(256), 0, st, a.d, a.E,
                     a.L, a.ng, a.dens);
  return hipGetLastError();
}
hipError_t launch_add(const double* a, const double* b, size_t n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b, n, out);
  return hipGetLastError();
}
hipError_t launch_add_f32(const double* a, const double* b, size_t n, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_add_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, b, n, out);
  return hipGetLastError();
}
hipError_t launch_norms(const double* eta0, int L, size_t ng, double dv, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_norms, dim3(L), dim3(256), 0, st, eta0, ng, dv, out);
  return hipGetLastError();
}
size_t norm_drift_part_elems(int L) { return (size_t)L * NORM_NB; }
template <typename T>
hipError_t launch_norm_drift(const cplx<T>* H, int L, size_t ng, double dv, const double* n0, double tol,
                             int* flags, int B, double* part, hipStream_t st) {
  if (L <= 0 || B <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_norm_part<T>), dim3(NORM_NB, L), dim3(256), 0, st, H, ng, part);
  hipLaunchKernelGGL(k_norm_check, dim3(1), dim3(256), 0, st, part, L, dv, n0, tol, flags, B);
  return hipGetLastError();
}
hipError_t launch_nan_flagged(double* w, int B, size_t ng, const int* flags, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_nan_flagged<double>), dim3(64, B), dim3(256), 0, st, w, ng, flags);
  return hipGetLastError();
}
hipError_t launch_nan_flagged_f32(float* w, int B, size_t ng, const int* flags, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_nan_flagged<float>), dim3(64, B), dim3(256), 0, st, w, ng, flags);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_to_real(const double* in, size_t n, T* out, hipStream_t st) {
  hipLaunchKernelGGL((k_to_real<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, n, out);
  return hipGetLastError();
}

#define BSE_INST(T)                                                                            \
  template hipError_t launch_prop_x<T>(int, const PropXArgs<T>&, int, hipStream_t, int,        \
                                       const LaunchEvents*);                                     \
  template hipError_t launch_prop_yz<T>(int, const PropYZArgs<T>&, int, hipStream_t, int,      \
                                        const LaunchEvents*, const LaunchEvents*);               \
  template bool prop_yz_split<T>(int);                                                         \
  template bool prop_yz_fused<T>(int);                                                         \
  template hipError_t launch_poisson<T>(int, const PoisArgs<T>&, hipStream_t);                 \
  template void configure_kernels<T>(int);                                                     \
  template bool grid_supported<T>(int);                                                        \
  template hipError_t launch_stoch_orbitals<T>(const double*, const signed char*, int, int,    \
                                               int, size_t, const cplx<T>*, double*, cplx<T>*, \
                                               hipStream_t);                                   \
  template hipError_t launch_kick<T>(const double*, const double*, int, int, size_t, cplx<T>*, \
                                     hipStream_t);                                             \
  template hipError_t launch_clean<T>(const CleanArgs<T>&, hipStream_t);                       \
  template hipError_t launch_to_real<T>(const double*, size_t, T*, hipStream_t);                \
  template hipError_t launch_norm_drift<T>(const cplx<T>*, int, size_t, double, const double*,  \
                                           double, int*, int, double*, hipStream_t);

BSE_INST(float)
BSE_INST(double)

}  // namespace bse
