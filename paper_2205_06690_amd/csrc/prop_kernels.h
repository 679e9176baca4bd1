// Argument blocks and launchers of the propagation kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include "fft_lines.h"

namespace bse {

enum { PX_ETA0 = 0, PX_FULL = 1, PX_HALF = 2 };

template <typename T> struct PropXArgs {
  const cplx<T>* din;
  cplx<T>* dout;
  const cplx<T>* pf;   // exp(-i V dt)
  const cplx<T>* ph;   // exp(-i V dt/2)
  const T* u;          // [B][ng]
  const cplx<T>* H;    // unperturbed mid-step state [L][ng]
  const cplx<T>* tw;   // twiddles exp(-2 pi i m/N)
  const cplx<T>* kph;  // exp(-i k^2 dt/2) / N per frequency index
  T dt;
  int L;
  int mode;
  int order;           // workgroup order: 0 field fastest on a 2-D grid, 1 XCD-grouped (see launch_order)
  int nf;              // fields (or pairs) of the launch; set by the launcher
};

template <typename T> struct PropYZArgs {
  cplx<T>* d;
  const cplx<T>* H;
  const cplx<T>* tw;
  const cplx<T>* kph;
  T* dens;
  int L;
  int density;
  int order;           // workgroup order of the y-line pass, as PropXArgs::order
  int nf;              // fields (or pairs) of the launch; set by the launcher
  int fused;           // where prop_yz_fused(n), one pass for y and z: 1 cross-lane DFT16, 2 DFT16 per lane
};

template <typename T> struct PoisArgs {
  const T* rho;        // [B][ng] real densities
  int B;
  cplx<T>* work;       // [(B+1)/2][ng]
  const cplx<T>* tw;
  const T* k2;         // k^2 per frequency index
  T vscale;            // 4 pi / ng
  T* out;              // nullable [B][ng]
  double* out64;       // nullable [B][ng]
  double* acc;         // nullable [B][ng]: acc += wn * v[rho]
  double wn;
  int kinetic;         // 1: multiplier vscale k^2/2 (the kinetic operator) instead of vscale/k^2
  const double* pscale;  // nullable [B]: density b enters its packed transform as rho_b / pscale[b]
                         // and its potential leaves times pscale[b], so that two packed
                         // densities of very different size keep their own relative rounding
  int* flags;          // nullable [B]: a non-finite input value of density b is replaced by 0
                       // (so that it cannot reach the density packed with it) and flags[b] |= 1
};

template <typename T> struct CleanArgs {
  cplx<T>* d;          // [F][ng]
  int F, L, S;
  const T* u;
  const cplx<T>* H;
  const cplx<T>* ph;
  cplx<T>* E;          // [L][ng] workspace
  const T* phi;        // occupied orbitals [S][ng]
  size_t ng;
  T dt;
  int from_mid;
  int chunk;
  cplx<double>* part;  // [nchunk][F][S+1]
  cplx<double>* coef;  // [F][S+1]
  cplx<double>* coefE; // [L][S+1]
  const double* n0;    // [L]
  int renorm;
  double dv;
  T* dens;             // [F/L][ng]
  const double* eta0;  // [L][ng] eta_l(0), used at t = 0
  float* part32;       // matrix-core partials and split coefficients (mixed precision)
  cplx<double>* gpart; // partial <E_l, d_f> per chunk of points
  // occupied orbitals as bf16 hi/lo pairs, [S][ng] and [ng][Sp] (mixed precision)
  const unsigned short *phih, *phil, *phith, *phitl;
};

template <typename T> bool grid_supported(int n);
template <typename T> void configure_kernels(int n);
// start/stop events recorded by the kernel's own dispatch (timing without
// separate event packets on the stream)
struct LaunchEvents {
  hipEvent_t start, stop;
};
// tc: x-tile width (16, 32, 64; 0 = default); nt: plane-pass block size (256, 512; 0 = default);
// ev: nullable timing events
template <typename T> hipError_t launch_prop_x(int n, const PropXArgs<T>& a, int F, hipStream_t st, int tc = 0,
                                               const LaunchEvents* ev = nullptr);
// grids whose y-z plane would leave one block per CU (prop_yz_split) run the
// y and z factors as a z-line and a y-line pass: ev then times the z pass
// and ev2 the y pass; otherwise ev times the plane pass and ev2 is unused
template <typename T> hipError_t launch_prop_yz(int n, const PropYZArgs<T>& a, int nb, hipStream_t st, int nt = 0,
                                                const LaunchEvents* ev = nullptr,
                                                const LaunchEvents* ev2 = nullptr);
// Work lists of uneven batches (FP32): one launch of a propagation pass walks
// the items of every listed system of one grid size, (pair, x tile) for the
// x pass and (x plane, pair) for the plane pass, systems in order with
// first = the number of items before them in the list.  Grids whose plane
// pass is the LDS plane kernel (prop_list_grid); each item is computed as by
// the per-system pass.
struct XListSys {
  PropXArgs<float> a;   // the pair pass of this system (mode PX_FULL or PX_HALF, nf = pairs)
  unsigned first;
};
struct YZListSys {
  PropYZArgs<float> a;  // the pair pass with the density (nf = pairs)
  unsigned first;
};
bool prop_list_grid(int n);
// items of one system: pairs x tiles, planes x pairs
unsigned prop_x_list_items(int n, int pairs);
unsigned prop_yz_list_items(int n, int pairs);
// list: device array of nsys entries of grid size n, total = all their items
hipError_t launch_prop_x_list(int n, const XListSys* list, int nsys, unsigned total, hipStream_t st);
hipError_t launch_prop_yz_list(int n, const YZListSys* list, int nsys, unsigned total, hipStream_t st);
template <typename T> bool prop_yz_split(int n);
// grids where the y and z factors can run as one register-line plane pass
template <typename T> bool prop_yz_fused(int n);
template <typename T> hipError_t launch_poisson(int n, const PoisArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_stoch_orbitals(const double* phi, const signed char* xi, int L, int n_occ,
                                 int deterministic, size_t ng, const cplx<T>* ph, double* eta0,
                                 cplx<T>* H0, hipStream_t st);
template <typename T>
hipError_t launch_kick(const double* q, const double* eta0, int L, int F, size_t ng, cplx<T>* d,
                       hipStream_t st);
template <typename T> hipError_t launch_clean(const CleanArgs<T>& a, hipStream_t st);
template <typename T> hipError_t launch_to_real(const double* in, size_t n, T* out, hipStream_t st);
hipError_t launch_pair_density(const double* phi, const int* pq, int B, size_t ng, double* rho,
                               hipStream_t st);
hipError_t launch_add(const double* a, const double* b, size_t n, double* out, hipStream_t st);
hipError_t launch_norms(const double* eta0, int L, size_t ng, double dv, double* out, hipStream_t st);
// unitarity of the unperturbed propagation: if |dv sum |H_l|^2 / n0[l] - 1| > tol for any l, or the
// sum is not finite, flags[b] |= 2 for every b < B; part holds norm_drift_part_elems(L) doubles
size_t norm_drift_part_elems(int L);
template <typename T>
hipError_t launch_norm_drift(const cplx<T>* H, int L, size_t ng, double dv, const double* n0, double tol,
                             int* flags, int B, double* part, hipStream_t st);
// rows b < B of w[B][ng] with flags[b] != 0 become NaN
hipError_t launch_nan_flagged(double* w, int B, size_t ng, const int* flags, hipStream_t st);
hipError_t launch_nan_flagged_f32(float* w, int B, size_t ng, const int* flags, hipStream_t st);
hipError_t launch_add_f32(const double* a, const double* b, size_t n, float* out, hipStream_t st);

}  // namespace bse
