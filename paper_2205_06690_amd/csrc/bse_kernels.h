// Launchers of the A-matrix, spectrum and utility kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>

namespace bse {
// flags[b] |= 1 for every row b of w[B][ng] with a non-finite value
hipError_t launch_finite_check(const double* w, int B, size_t ng, int* flags, hipStream_t st);
hipError_t launch_fill_nan(double* w, size_t n, hipStream_t st);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t st);
template <typename T>
hipError_t launch_products(const double* phi, const int* pq, int K, size_t ng, T* out, hipStream_t st);
size_t gemm_chunk(int M, int N, size_t K);
size_t gemm_part_elems(int M, int N, size_t K);
// C[m][n] = scale * sum_r A[m][r] B[n][r]
hipError_t launch_gemm_f64(const double* A, int M, const double* B, int N, size_t K, double scale,
                           double* part, double* C, hipStream_t st);
hipError_t launch_assemble_a(const double* X, const double* D, int no, int nc, int nij,
                             const double* eps_v, const double* eps_c, double scissors, double* A,
                             hipStream_t st);
hipError_t launch_dipoles(const double* phi, const int* pq, int K, int n, double h, double* f0,
                          hipStream_t st);
hipError_t launch_gemv(const double* A, int n, const double* v, double* y, hipStream_t st);
// w -= V^T-projection onto the first m basis vectors (c = V w); c[m-1] also to *last
// Lanczos iterations k0 .. k1-1 in one launch for n <= lanczos_fused_max():
// basis V[n+1][n] (v_k0 set), al[k] = alpha_k, bq[k] = |w_k|^2
int lanczos_fused_max();
hipError_t launch_lanczos_steps(const double* A, int n, double* V, int k0, int k1, double* al, double* bq,
                                hipStream_t st);
hipError_t launch_reorth(const double* V, int n, int m, double* c, double* w, hipStream_t st,
                         double* last = nullptr);
hipError_t launch_dot(const double* a, const double* b, int n, double* out, hipStream_t st);
// out[q] = sum_k S[q][k] V[k], q < nq, k < m
hipError_t launch_ritz(const double* V, int n, int m, const double* S, int nq, double* out,
                       hipStream_t st);
// matrix-free A f (Eq. 6), FP64, fields [n_o][ng]: rho = 2 sum phi_i f_i;
// out_j = Tf_j + (V + Delta - eps_j) f_j + dv phi_j - sum_i f_i W_ij (W stack
// of pairs i <= j in row order); out_j -= sum_s C[j][s] phi_s (n_o S <= 8192)
hipError_t launch_mixed_density(const double* phv, const double* f, int n_o, size_t ng, double* rho,
                                hipStream_t st);
hipError_t launch_mixed_combine(const double* f, const double* tf, const double* vext,
                                const double* eps_v, double scissors, const double* dv,
                                const double* phv, const double* wij, int n_o, size_t ng,
                                double* out, hipStream_t st);
// C[n_o][S] = dv sum_r f_i(r) phi_s(r) for n_o <= 32 fields (ng a multiple
// of 32); part holds proj_part_elems(n_o, S) doubles
size_t proj_part_elems(int n_o, int S);
hipError_t launch_proj_coef(const double* f, int n_o, const double* phi, int S, size_t ng, double dv,
                            double* part, double* C, hipStream_t st);
hipError_t launch_project_out(double* out, int n_o, const double* phi, int S, const double* C,
                              size_t ng, hipStream_t st);
// mixed-representation Chebyshev: one step of polarisation p over len values
// with partials part[mixed_cheb_blocks()][6]; dipole start f_j = (r_axis - c) phi_j
int mixed_cheb_blocks();
hipError_t launch_mixed_cheb_update(const double* af, const double* fc, const double* fp, double* fn,
                                    size_t len, double a, double b, int first, double dv, int p,
                                    double* part, hipStream_t st);
hipError_t launch_mixed_dipole(const double* phv, int n_o, int n, double h, int axis, double* f,
                               hipStream_t st);
// Chebyshev spectrum (Eqs. 7-8): Gershgorin rows lohi[2][n]; one recursion
// step on [3][n] vectors with per-block partial residues part[cheb_blocks(n)][6];
// residues mu[3][2K], node weights D[3][M] and sigma[n_w] from the partials
hipError_t launch_gershgorin(const double* A, int n, double* lohi, hipStream_t st);
int cheb_blocks(int n);
// the dipoles f0[n][3] as the three start vectors out[3][n]
hipError_t launch_cheb_start(const double* f0, int n, double* out, hipStream_t st);
// mm[0] = min of lohi[0..n), mm[1] = max of lohi[n..2n) (the Gershgorin interval)
hipError_t launch_interval(const double* lohi, int n, double* mm, hipStream_t st);
hipError_t launch_cheb_step(const double* A, int n, const double* fc, const double* fp, double* fn,
                            double a, double b, int first, double* part, hipStream_t st);
hipError_t launch_cheb_spectrum(const double* part, int K, int nblk, double* mu, int M, double* D,
                                double a, double b, const double* w, int n_w, double sig,
                                double* out, hipStream_t st);
// frequency-resolved exciton states (Eq. 8): g[n_w][N] Chebyshev coefficients
// of the broadened delta (Gauss-Chebyshev quadrature on M nodes); F[n_w][3][n]
// = g[.][0] f0 at the start, then one recursion step per moment adding
// g[.][m_next] f^{m_next}; exciton densities dens[n_out][ng] of F[n_out][n]
hipError_t launch_cheb_coef(const double* w, int n_w, int N, int M, double a, double b, double sig,
                            double* g, hipStream_t st);
hipError_t launch_cheb_acc_init(const double* f0, int n, const double* g, int N, int n_w, double* F,
                                hipStream_t st);
hipError_t launch_cheb_step_acc(const double* A, int n, const double* fc, const double* fp, double* fn,
                                double a, double b, int first, const double* g, int N, int m_next,
                                int n_w, double* F, hipStream_t st);
// F[n_w][len] = / += g[.][m] f over grid vectors (mixed representation)
hipError_t launch_states_acc(double* F, const double* f, const double* g, int N, int m, int n_w,
                             size_t len, int init, hipStream_t st);
hipError_t launch_exciton_density(const double* phi, int v0, int c0, int n_o, int n_c, size_t ng,
                                  const double* F, int n_out, double* dens, hipStream_t st);
// out = w / sqrt(*bsq), bsq on the device
hipError_t launch_scale_norm(const double* w, int n, const double* bsq, double* out, hipStream_t st);
}  // namespace bse

namespace bse {
hipError_t launch_ground_density(const double* phi, int n_occ, size_t ng, double* n0, hipStream_t st);
// v_bndry = mean of vext + vh over the zero-index faces minus the cell mean,
// into out[0] (device); part holds boundary_part_elems(n) doubles
size_t boundary_part_elems(int n);
hipError_t launch_boundary_average(const double* vext, const double* vh, int n, double* part, double* out,
                                   hipStream_t st);
// scale[b] = RMS of row b from launch_row_dots' sums (1 for a zero row)
hipError_t launch_rms_scales(const double* dots, int B, size_t ng, double* scale, hipStream_t st);
hipError_t launch_row_dots(const double* a, const double* c, const double* d, int B, size_t ng,
                           double* out, hipStream_t st);
hipError_t launch_features(const double* q, const double* scale, const double* n0, double n0s,
                           const double* v, double vs, int B, size_t ng, float* x, hipStream_t st);
hipError_t launch_targets(const double* wpol, const double* scale, int B, size_t ng, float* t,
                          hipStream_t st);
// out[2k] = |a[rows[k]] - b[k]|^2, out[2k+1] = |b[k]|^2 over ng points, k < K
hipError_t launch_diff_norms(const double* a, const int* rows, const double* b, int K, size_t ng, double* out,
                             hipStream_t st);
hipError_t launch_assemble_w(const double* q, const double* scale, const float* y, int B, size_t ng,
                             double* wpol, double* w, hipStream_t st);
}  // namespace bse
