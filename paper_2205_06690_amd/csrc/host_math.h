// Host-side numerics of libbse, in plain C++ with no device code: the
// SplitMix64 draws of the stochastic signs (Eq. 14), the trapezoid weights
// of the damped time integral (Eq. 13), the symmetric tridiagonal eigenpairs
// of the Lanczos spectrum, and the least-squares fit of the finite-box W(k->0)
// correction.  Kept apart so that they build with the host sanitizers.
#pragma once
#include <cstdint>
#include <vector>

namespace bse_host {

// SplitMix64 finaliser of (seed, k): z = seed + (k + 1) * golden gamma, then
// the three xor-shift-multiply rounds (Steele, Lea and Flood; Vigna).
uint64_t splitmix64_draw(uint64_t seed, uint64_t k);

// xi[l][s] = +1 if the top bit of draw l * n_occ + s is 0, else -1
void stochastic_signs(uint64_t seed, int n_stoch, int n_occ, int8_t* xi);

// w[n] = c_n exp(-gamma^2 t_n^2 / 2) dt, t_n = n dt, c = 1/2 at n = 0 and
// n = N, 1 otherwise (the trapezoid rule on [0, N dt]); w has N + 1 entries
void time_weights(int n_steps, double dt, double gamma, double* w);

// Sturm counts (eigenvalues of T below x) of the symmetric tridiagonal T
// (diagonal a[m], squared off-diagonal b2[m-1]) at nx points at once.
void sturm_counts(const std::vector<double>& a, const std::vector<double>& b2, int m, const double* x,
                  int nx, int* cnt);

// The k lowest eigenpairs of the symmetric tridiagonal T (diagonal a,
// off-diagonal b; m rows): bisection on Sturm counts until each bracket is
// below tol relative to its magnitude, then inverse iteration with partial
// pivoting, vectors orthogonalised within clusters and normalised.
void tridiag_lowest(const std::vector<double>& a, const std::vector<double>& b, int m, int k,
                    std::vector<double>& theta, std::vector<std::vector<double>>& vecs, double tol = 1e-15);

// Least squares of omega[b][m] = c_m + e v[b] over n_box boxes and n_exc
// excitations; outputs eps_inv = e, c[n_exc] (nullable), w_k0[b] = e v[b].
// Returns nullptr, or a message for bad arguments (nothing written).
const char* fit_box_correction(int n_box, int n_exc, const double* omega, const double* v, double* eps_inv,
                               double* c, double* w_k0);

}  // namespace bse_host
