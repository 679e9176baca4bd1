/* libbse: MI355X (gfx950) hot path of stochastic-W Bethe-Salpeter spectra.
 *
 * The method (Method section of the paper, "Stochastic evaluation of the
 * action of W" and Eqs. 1, 7, 10-15):
 *   - a closed-shell system with 2 N_occ electrons described by eigenstates
 *     phi_s, eps_s of a zero-order Hamiltonian H0 = -1/2 Lap + V_ext on a
 *     periodic real-space grid;
 *   - the action of the static screened interaction on a pair density,
 *     W_ij(r) = q_ij(r) + W^pol_ij(r), q_ij = v[phi_i phi_j], obtained by a
 *     linear-response time-dependent Hartree propagation of L random-sign
 *     stochastic occupied orbitals (Eq. 14) kicked by q_ij, cleaned of
 *     occupied-space amplitude every M steps (Eq. 15), with the induced
 *     Coulomb potential integrated under a Gaussian damping (Eq. 13);
 *   - the Tamm-Dancoff matrix A(ia;jb) = (eps_a - eps_i + Delta) d_ij d_ab
 *     + 2 (ia|jb) - (phi_a phi_b|W|phi_i phi_j) (Eq. 1), and its lowest
 *     excitons with dipole oscillator strengths (Eq. 7).
 *
 * Conventions
 *   - Grid: cubic n x n x n, spacing h (bohr), periodic, row-major with z
 *     fastest; grid point (i,j,k) sits at (i h, j h, k h).  Integrals are
 *     sums times h^3.  Supported n: 16, 24, 32, 48, 64 and 112, in both
 *     precisions.
 *   - Orbitals: real, sum_r |phi|^2 h^3 = 1, ascending eps; orbitals
 *     0..n_occ-1 are occupied.  Units: Hartree atomic units.
 *   - The Coulomb kernel is periodic, 4 pi/|k|^2 with k = 0 removed.
 *   - The propagation is the exact linearisation (alpha -> 0) of the
 *     paper's finite-alpha kick exp(-i alpha q); Strang split-operator steps
 *     of dt; trapezoid time weights on t_n = n dt up to T = n_steps dt.
 *
 * Ownership: the library copies every host input; the caller allocates
 * every output.  Device variants borrow caller device memory and are
 * ordered on the stream given to bse_set_stream (default: the null stream).
 *
 * Errors: no exception crosses this interface.  Every call returns a
 * bse_status; on an argument error nothing is written.  bse_last_error()
 * gives a thread-local message for the last failing call.  A system
 * handle must not be used by two threads at once.
 */
#ifndef BSE_H
#define BSE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bse_system bse_system; /* opaque; owns all device memory */

typedef enum {
  BSE_OK = 0,
  BSE_ERR_ARG = -1,     /* invalid argument; nothing written */
  BSE_ERR_STATE = -2,   /* call out of order (e.g. apply_W before set_orbitals) */
  BSE_ERR_OOM = -3,     /* device allocation failed */
  BSE_ERR_DEVICE = -4,  /* HIP runtime error */
  BSE_ERR_NUMERIC = -5  /* non-finite result for some pair (see pair_status) */
} bse_status;

enum { BSE_FP64 = 0, BSE_MIXED = 1 };     /* bse_config.precision              */
enum { BSE_F64 = 0, BSE_F32 = 1 };        /* element type of a device W output */

typedef struct {
  int32_t nx, ny, nz;   /* grid points per axis (must be equal)                    */
  double h;             /* grid spacing, bohr                                      */
  int32_t n_occ;        /* occupied orbitals (2 n_occ electrons)                   */
  int32_t n_stoch;      /* L stochastic orbitals (Eq. 14); 0 = deterministic, all
                           n_occ occupied orbitals are propagated                  */
  uint64_t seed;        /* SplitMix64 seed of the signs unless bse_set_signs       */
  double dt;            /* time step, a.u.                                         */
  int32_t n_steps;      /* N; T = N dt                                             */
  double gamma;         /* Gaussian damping width of Eq. 13, Hartree               */
  int32_t clean_every;  /* M of Eq. 15 (also cleans at t = 0); 0 = never           */
  double alpha;         /* must be 0 (linearised kick)                             */
  double scissors;      /* Delta of Eq. 1, Hartree                                 */
  int32_t precision;    /* BSE_FP64: every step in FP64.  BSE_MIXED: propagation
                           and cleaning in FP32, source potentials, the time
                           integral and all outputs in FP64                        */
  int32_t device;       /* HIP device ordinal                                      */
  int32_t max_batch;    /* pairs propagated together (memory bound); >= 1          */
} bse_config;

/* Create a system from V_ext[nx*ny*nz] (host, FP64).  *out receives the
 * handle.  Allocates the device tables of the grid.
 * Passage: the Method section's statement of the problem (a closed-shell
 * system of 2 n_occ electrons whose zero-order Hamiltonian H0 = -1/2 Lap +
 * V_ext has the eigenstates phi_s, eps_s) and the propagation parameters of
 * its stochastic W subsection (Eqs. 10-15: dt, the number of steps, the
 * damping gamma of Eq. 13, the cleaning period M of Eq. 15, L of Eq. 14).
 * Errors: BSE_ERR_ARG for a non-cubic or unsupported grid, a non-positive
 * h, dt or max_batch, alpha != 0, a non-finite V_ext or a bad device
 * ordinal (*out is then NULL); BSE_ERR_OOM / BSE_ERR_DEVICE from HIP. */
bse_status bse_create_system(const bse_config* cfg, const double* v_ext, bse_system** out);

/* Orbitals phi[n_orb][nx*ny*nz] (host, FP64, h^3-normalised) and
 * eigenvalues eps[n_orb] (host, FP64, ascending).  n_orb >= n_occ; the
 * A matrix needs n_orb >= n_occ + n_c.  Builds the stochastic orbitals of
 * Eq. 14 (shared by every pair; the unperturbed set is propagated alongside
 * each batch of pairs).  Replaces earlier orbitals. */
bse_status bse_set_orbitals(bse_system* sys, int32_t n_orb, const double* phi, const double* eps);

/* Explicit signs xi[n_stoch][n_occ] (host, +-1) of Eq. 14, replacing the
 * ones drawn from cfg.seed.  Call before bse_set_orbitals. */
bse_status bse_set_signs(bse_system* sys, int32_t n_stoch, int32_t n_occ, const int8_t* xi);

/* W-action on n_pairs pair densities phi_p phi_q, pq[n_pairs][2] (host).
 * Passage: the subsection on the stochastic evaluation of the action of W
 * (W = v + W^pol; the kick by q_pq = v[phi_p phi_q], the propagation of
 * Eqs. 10-11, W^pol(t) of Eq. 12, its damped time integral Eq. 13, the
 * stochastic orbitals of Eq. 14 and the cleaning of Eq. 15).
 * w_out[n_pairs][ng] (host, FP64) receives W_pq = q_pq + W^pol_pq;
 * wpol_out (nullable) receives W^pol_pq; pair_status (nullable,
 * [n_pairs]) receives 0 or BSE_ERR_NUMERIC per pair.  A pair fails when a
 * Poisson solve of its densities meets a non-finite value, when its W is
 * not finite, or (every pair of its batch) when the unperturbed orbitals
 * lose their norm at a cleaning step (relative drift above 1e-3 in mixed
 * precision, 1e-8 in FP64); its rows are NaN-filled, the densities packed
 * with it are shielded from it, and the call returns BSE_ERR_NUMERIC after
 * finishing every other pair.  Errors: BSE_ERR_STATE before
 * bse_set_orbitals; BSE_ERR_ARG for null buffers or an orbital index out
 * of range (nothing written). */
bse_status bse_apply_W(bse_system* sys, int32_t n_pairs, const int32_t* pq, double* w_out,
                       double* wpol_out, int32_t* pair_status);

/* Device variant of bse_apply_W (same passage): pq_dev[n_pairs][2]
 * (device, int32) and w_dev[n_pairs][ng] (device, caller-owned) of element
 * type dtype: BSE_F64 (double) or BSE_F32 (float, W rounded from the FP64
 * sum q + W^pol).  Stream-ordered on the bse_set_stream stream: the call
 * first reads pq_dev back (a small copy that waits for the work already on
 * that stream) and checks every index, then enqueues the propagation and
 * returns.  A failed pair (see bse_apply_W) is NaN-filled on the device;
 * there is no status output.  Errors: BSE_ERR_STATE before
 * bse_set_orbitals; BSE_ERR_ARG for null buffers, a bad dtype or an index
 * out of range (nothing written). */
bse_status bse_apply_W_device(bse_system* sys, int32_t n_pairs, const int32_t* pq_dev, void* w_dev,
                              int32_t dtype);

/* Failure injection for tests of the error path.  target BSE_FAULT_ORBITAL:
 * writes value (any double, NaN included) into the device copy of orbital
 * `index` at grid point `point`, bypassing the input checks of
 * bse_set_orbitals (the stochastic orbitals and the precision copies made
 * there are not changed).  target BSE_FAULT_UNPERTURBED: writes value into
 * the real part of the t = 0 unperturbed stochastic orbital `index` (< L)
 * at `point` (a finite value that changes its norm trips the norm check of
 * the cleaning steps).  The next set_orbitals restores both.  Errors:
 * BSE_ERR_STATE before bse_set_orbitals; BSE_ERR_ARG for a bad target or an
 * index out of range. */
enum { BSE_FAULT_ORBITAL = 0, BSE_FAULT_UNPERTURBED = 1 };
bse_status bse_inject_fault(bse_system* sys, int32_t target, int32_t index, int64_t point, double value);

/* Tamm-Dancoff matrix (Eq. 1) for the highest n_o occupied and lowest n_c
 * virtual orbitals: A[(n_o n_c)^2] (host, FP64, row-major), row index
 * (i - (n_occ - n_o)) * n_c + (a - n_occ).  Propagates the n_o(n_o+1)/2
 * valence pairs, keeps their W_ij on the device for bse_spectrum.
 * Errors: BSE_ERR_NUMERIC when some W_ij fails the checks of bse_apply_W
 * or A has a non-finite element (no spectrum of it is then possible);
 * BSE_ERR_ARG for a window outside the orbitals set. */
bse_status bse_build_A(bse_system* sys, int32_t n_o, int32_t n_c, double* A);

/* The W_ij that the last successful bse_build_A propagated and keeps on
 * the device (the screened interaction of its direct term, Eq. 1):
 * w_out[n_o(n_o+1)/2][nx*ny*nz] (host, FP64, caller-allocated), pairs
 * (i, j), i <= j, of the valence window in row-major order of (i, j).
 * Errors: BSE_ERR_STATE before a successful bse_build_A. */
bse_status bse_valence_W(bse_system* sys, double* w_out);

/* Lowest n_exc excitons of the last A (Lanczos in FP64 on the device):
 * omega[n_exc] (Hartree), dip2[n_exc][3] = |<X_n|f0_axis>|^2 with
 * f0_ia = <phi_a| r_axis - box centre |phi_i>, and, if n_w > 0, the
 * absorption sigma[n_w] = w sum_n sum_axis dip2 g(w - omega_n) on
 * w_grid[n_w], g a normalised Gaussian of standard deviation sigma_broad
 * (Eq. 7). */
bse_status bse_spectrum(bse_system* sys, int32_t n_exc, double* omega, double* dip2, int32_t n_w,
                        const double* w_grid, double sigma_broad, double* sigma);

/* Matrix-free action of the Tamm-Dancoff operator in the mixed hole-grid
 * representation (Eq. 6, with A = Q A-bar of the preceding equations), in
 * FP64 on the device, for the valence window of the last bse_build_A (its
 * n_o orbitals and the W_ij it keeps): for each of n_vec vectors
 * f[n_vec][n_o][nx*ny*nz] (host, real, orbital j = n_occ - n_o + index),
 *   af_j = Q [ (H0 + Delta - eps_j) f_j + v[2 sum_i phi_i f_i] phi_j
 *              - sum_i f_i W_ij ],
 * H0 = -1/2 Laplacian (spectral) + V_ext, v the periodic Coulomb kernel with
 * k = 0 removed, Q = 1 - sum_{s < n_occ} |phi_s><phi_s|.  af has f's layout
 * (host, caller-allocated).  Errors: BSE_ERR_STATE before bse_build_A;
 * BSE_ERR_ARG on null pointers or n_o * n_occ > 8192. */
bse_status bse_apply_A_mixed(bse_system* sys, int32_t n_vec, const double* f, double* af);

/* The paper's spectrum algorithm (Eqs. 6-8): the Chebyshev recursion of
 * bse_chebyshev_spectrum with A applied matrix-free in the mixed
 * representation (bse_apply_A_mixed) instead of the electron-hole matrix,
 * so the excitations range over the whole virtual space of the grid.  Start
 * vectors, one per axis: f0_j = Q (r_axis - box centre) phi_j over the
 * valence window of the last bse_build_A; residues R_n = sum_j
 * <f0_j| T_n(A~) f0_j> (h^3 sum over the grid), A~ = (A - b)/a with
 * b = (e_min + e_max)/2, a = 1.01 (e_max - e_min)/2, where e_min < e_max
 * must bound the spectrum of A on the virtual space (required; the kinetic
 * part reaches 3 (pi/h)^2 / 2).  sigma[n_w], residues[3][n_mom] (nullable
 * unless n_w == 0) as in bse_chebyshev_spectrum.  FP64 on the device;
 * costs 3 n_mom / 2 applications of A.  Errors: BSE_ERR_STATE before
 * bse_build_A; BSE_ERR_ARG on bad sizes or bounds. */
bse_status bse_chebyshev_mixed(bse_system* sys, int32_t n_mom, double e_min, double e_max,
                               int32_t n_w, const double* w_grid, double sigma_broad,
                               double* sigma, double* residues);

/* Absorption by the Chebyshev expansion of the broadened delta (Eqs. 7-8)
 * on the A of the last bse_build_A, in FP64 on the device.  For each of
 * the three polarisations, with the electron-hole dipoles
 * f0_ia = <phi_a| r_axis - box centre |phi_i> as start vector, the
 * residues R_n = <f0| T_n(A~) |f0>, n < n_mom, where A~ = (A - b)/a,
 * b = (e_min + e_max)/2 and a = 1.01 (e_max - e_min)/2; then
 * sigma(w) = w sum_axis sum_n g_n(w) R_n with g_n(w) the Chebyshev
 * coefficients (in A~) of a normalised Gaussian of standard deviation
 * sigma_broad centred at w, by Gauss-Chebyshev quadrature on 2 n_mom nodes.
 * e_min < e_max: caller's bound on the spectrum of A (Hartree); otherwise
 * the Gershgorin interval of A is used.  n_mom: even, >= 2.  Outputs (host):
 * sigma[n_w] if n_w > 0, residues[3][n_mom] (nullable unless n_w == 0),
 * bounds[2] = the interval used (nullable).  Errors: BSE_ERR_STATE before
 * bse_build_A; BSE_ERR_ARG on bad sizes or a degenerate interval. */
bse_status bse_chebyshev_spectrum(bse_system* sys, int32_t n_mom, double e_min, double e_max,
                                  int32_t n_w, const double* w_grid, double sigma_broad,
                                  double* sigma, double* residues, double* bounds);

/* Allocation-free variant of bse_chebyshev_spectrum, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same arguments,
 * kernels, arithmetic and results (bit for bit), with every device buffer
 * of the call (the three recursion vectors per polarisation, the per-block
 * partial residues, the residues, the node sums, the frequency grid, the
 * Gershgorin bounds) carved from one fixed 64 MiB device array that the
 * library holds per GPU until the process ends; the start vectors and the
 * Gershgorin interval are formed on the device, so the call makes no host
 * staging copies either.  It calls no hipMalloc, hipFree or allocating
 * routine.  Limit: about 0.75 n_mom (n_o n_c) + 9 n_o n_c + 9 n_mom +
 * 2 n_w doubles must fit in the 64 MiB (e.g. n_mom up to ~13000 at
 * n_o n_c = 800); larger requests return BSE_ERR_ARG before any work.
 * Every call on a GPU shares that GPU's array: calls that overlap on one
 * GPU (two host threads, or two streams) race and must be serialised by
 * the caller.  Nothing in the array needs to start at zero (every element
 * a call reads, it has written first).  Errors: as bse_chebyshev_spectrum,
 * plus BSE_ERR_ARG for a request above the limit. */
bse_status bse_chebyshev_spectrum_noalloc(bse_system* sys, int32_t n_mom, double e_min, double e_max,
                                          int32_t n_w, const double* w_grid, double sigma_broad,
                                          double* sigma, double* residues, double* bounds);

/* Frequency-resolved exciton states (Eq. 8) and their densities, on the A
 * of the last bse_build_A, in FP64 on the device.  For each frequency
 * w_list[q] (Hartree) and each of the three dipole start vectors f0 (as in
 * bse_chebyshev_spectrum):
 *   F[q][axis] = sum_{n < n_mom} g_n(w_q) T_n(A~) f0_axis,
 * A~ = (A - b)/a, b = (e_min + e_max)/2, a = 1.01 (e_max - e_min)/2, g_n the
 * Chebyshev coefficients of a normalised Gaussian of standard deviation
 * sigma_broad centred at w_q (Gauss-Chebyshev quadrature on 2 n_mom nodes),
 * i.e. the broadened delta(A - w_q) applied to f0; its components are the
 * transition amplitudes f_ia(w) in the row order of A.  The exciton density
 * of each state is dn(r) = 2 sum_i phi_i(r) f_i(r) with f_i = sum_a F_ia phi_a
 * (the density of the mixed representation), i.e. 2 sum_ia F_ia phi_i phi_a.
 * e_min < e_max: caller's bound on the spectrum of A; otherwise the
 * Gershgorin interval.  n_mom >= 2 (the full recursion: n_mom - 1
 * applications of A); 1 <= n_w <= 8; sigma_broad > 0.  Outputs (host,
 * caller-allocated): f_out[n_w][3][n_o n_c]; dens_out[n_w][3][nx*ny*nz]
 * (nullable); bounds[2] the interval used (nullable).  Errors:
 * BSE_ERR_STATE before bse_build_A; BSE_ERR_ARG on bad sizes, null
 * required pointers or a degenerate interval. */
bse_status bse_exciton_states(bse_system* sys, int32_t n_mom, double e_min, double e_max,
                              int32_t n_w, const double* w_list, double sigma_broad,
                              double* f_out, double* dens_out, double* bounds);

/* Frequency-resolved exciton states of the mixed representation (Eq. 8 with
 * A applied matrix-free as in bse_apply_A_mixed, Eq. 6), the paper's route
 * to exciton maps: for each frequency w_list[q] and each axis, the grid
 * vectors f_j(r; w_q) = sum_{n < n_mom} g_n(w_q) T_n(A~) f0_j over the
 * valence window of the last bse_build_A, from the start vectors
 * f0_j = Q (r_axis - box centre) phi_j of bse_chebyshev_mixed, with A~, g_n
 * and the interval [e_min, e_max] (required) as in bse_chebyshev_mixed.
 * Outputs (host, caller-allocated): the electron-hole amplitudes
 * f_ia = h^3 sum_r phi_a f_i on the n_a lowest virtual orbitals (a = n_occ
 * .. n_occ + n_a - 1, any n_a up to the orbitals set, not only the n_c of
 * A) in f_out[n_w][3][n_o][n_a]; the exciton densities 2 sum_i phi_i f_i in
 * dens_out[n_w][3][nx*ny*nz] (nullable).  FP64 on the device; costs
 * 3 (n_mom - 1) applications of A.  1 <= n_w <= 8; n_a = 0 requires
 * dens_out.  Errors: BSE_ERR_STATE before bse_build_A; BSE_ERR_ARG on bad
 * sizes, a missing interval or n_o * n_occ > 8192. */
bse_status bse_exciton_states_mixed(bse_system* sys, int32_t n_mom, double e_min, double e_max,
                                    int32_t n_w, const double* w_list, double sigma_broad, int32_t n_a,
                                    double* f_out, double* dens_out);

/* Finite-box W(k->0) correction (Results section: the scissors of Eq. 1 is
 * shifted down by W(k->0) = eps_eff^-1 v_bndry, eps_eff^-1 fitted so that
 * the spectra of runs in several box sizes overlap).
 *
 * bse_boundary_potential: v_bndry of this system's box, the mean of the
 * Kohn-Sham potential V_ext + v_H[n] (n = 2 sum_{s < n_occ} phi_s^2, v_H
 * the periodic Coulomb potential without its k = 0 term) over the grid
 * points with a zero index along some axis (the three faces through the
 * origin corner; 3 n^2 - 3 n + 1 points), minus its mean over the cell.
 * FP64 on the device; *v_bndry (host) receives it.  Errors: BSE_ERR_STATE
 * before bse_set_orbitals; BSE_ERR_ARG for a null output. */
bse_status bse_boundary_potential(bse_system* sys, double* v_bndry);

/* bse_fit_box_correction: least-squares fit over n_box >= 2 boxes of the
 * n_exc >= 1 lowest excitation energies omega[n_box][n_exc] (host, Hartree,
 * e.g. from bse_spectrum of each box) to omega[b][m] = c[m] + eps_inv *
 * v_bndry[b] (a scissors moves every excitation by the same amount, so
 * spectra corrected by -W(k->0) overlap when these do).  Outputs (host):
 * *eps_inv; c[n_exc] (nullable); w_k0[n_box] = eps_inv * v_bndry[b], the
 * W(k->0) to subtract from each box's scissors.  Host arithmetic only.
 * Errors: BSE_ERR_ARG for bad sizes, null required pointers, non-finite
 * inputs, or boundary potentials that all agree to 1e-12 relative. */
bse_status bse_fit_box_correction(int32_t n_box, int32_t n_exc, const double* omega,
                                  const double* v_bndry, double* eps_inv, double* c, double* w_k0);

/* Uneven batch: the W-action for several systems at once (different grids,
 * orbital counts and pair counts, same device).  System k propagates
 * n_pairs[k] (<= its max_batch) pairs pq[k][n_pairs[k]][2] (host) and
 * writes W to w_dev[k] (device, FP64, [n_pairs[k]][ng_k]).  mode bit 0:
 * the whole propagation of every system is captured into one HIP graph and
 * launched once.  mode bit 1: the lockstep work-list schedule, every system
 * taking each time step in turn on one stream, with the perturbed sets' x
 * and plane passes of all systems as one persistent launch each per step,
 * walking the (system, pair, tile or plane) items of the whole batch;
 * mixed-precision systems on grids of 16, 24, 32, 48 or 64 points per axis
 * with the same number of steps and cleaning interval (else BSE_ERR_ARG).
 * Without bit 1 the systems run on their own streams (one graph branch each
 * with bit 0).  Returns after the work has finished.  Results equal those
 * of bse_apply_W_device per system bit for bit in every mode.  Errors:
 * BSE_ERR_ARG for a null argument, a mode outside 0..3, a system twice,
 * systems on different devices, n_pairs outside 1..max_batch or a pair
 * index out of range. */
bse_status bse_apply_W_batch(int32_t n_sys, bse_system* const* systems, const int32_t* n_pairs,
                             const int32_t* const* pq, void* const* w_dev, int32_t mode);

/* Uneven batch as a plan (the batched form of the W-action for many
 * independent systems; the paper treats pairs as independent units, and
 * here whole systems are too): bse_batch_plan_create captures the whole
 * propagation of every system (its arguments as in bse_apply_W_batch,
 * pair lists copied to the plan's own device buffers, w_dev[k] bound to the
 * plan) into one HIP graph with one branch per system and instantiates it
 * once; bse_batch_plan_run replays it.  A run is ordered after the work
 * already queued on every system's stream, every system's stream waits for
 * it, and it returns after enqueueing.  Results equal bse_apply_W_batch
 * bit for bit.  The plan uses the systems' workspaces: a run returns
 * BSE_ERR_STATE when any system's workspace or orbitals have moved since
 * the capture (a larger batch or orbitals of another size), and runs must
 * not overlap other work of the same systems.  Errors: as
 * bse_apply_W_batch. */
typedef struct bse_batch_plan bse_batch_plan;
bse_status bse_batch_plan_create(int32_t n_sys, bse_system* const* systems, const int32_t* n_pairs,
                                 const int32_t* const* pq, void* const* w_dev, bse_batch_plan** plan);
bse_status bse_batch_plan_run(bse_batch_plan* plan);
void bse_batch_plan_destroy(bse_batch_plan* plan);

/* Autotuner: times the variants of the two propagation passes for this
 * system's grid, precision and a batch of n_pairs pairs and keeps the
 * fastest for later calls: the x pass's tile width (16, 32, 64) and
 * workgroup order (bse_set_launch_order bit 0); the plane pass's block size
 * (256, 512), or where the y and z factors run as one register-line pass
 * (112^3 in mixed precision, unless bse_set_yz_schedule chose the line
 * passes) its 16-point DFT schedule (2 or 0) and workgroup order (bit 2).
 * The tile shapes and orders do not change results; the two DFT schedules
 * agree to FP32 rounding.  cache_path (nullable) is a text
 * file of "key tc nt ms_x ms_yz ox sched oz" lines (sched -1 where not
 * tuned): a matching key is used without timing, a new result is appended.
 * Overwrites the system's pair workspace. */
bse_status bse_autotune(bse_system* sys, int32_t n_pairs, const char* cache_path);
/* The tuned x-tile width and plane-pass block size (0 = built-in default,
 * or not used by the one-pass y-z kernel). */
int32_t bse_tuned_shape(bse_system* sys, int32_t* tc, int32_t* nt);

/* Stream for all later device work of this system (a hipStream_t). */
bse_status bse_set_stream(bse_system* sys, void* hip_stream);

/* Signs of Eq. 14 drawn from SplitMix64 (host only, no device needed):
 * xi[l][s] = +1 if the top bit of draw l*n_occ + s is 0, else -1. */
bse_status bse_generate_signs(uint64_t seed, int32_t n_stoch, int32_t n_occ, int8_t* xi);

/* Per-kernel timing of the last bse_apply_W / bse_apply_W_device call:
 * names[k] and avg_ms[k], calls[k] for up to cap entries; returns the
 * number of kernels timed (0 unless timing was enabled). */
int32_t bse_kernel_times(bse_system* sys, int32_t cap, const char** names, double* avg_ms,
                         int32_t* calls);
/* Per-kernel HIP-event timing (synchronisation-free events around the timed
 * launches, each pair costing a few microseconds of stream time): enable = 0
 * off; 1 the propagation passes (prop_x, prop_yz) and the grid contractions
 * (gemm_exchange, gemm_direct) only; 2 every timed section (also cleaning,
 * Poisson, exciton states).  Errors: BSE_ERR_ARG for other values. */
bse_status bse_set_timing(bse_system* sys, int32_t enable);

/* Kernel schedule of the y and z factors of the kinetic step on grids whose
 * y-z plane fills most of the LDS (112^3 in mixed precision): 2 (default)
 * one pass over whole planes, the lines in registers for the 7-point DFTs
 * and each 16-point DFT (with the kinetic phase and its inverse) in one
 * lane's registers after a transpose through the wave's own LDS; 0 the
 * same pass with the 16-point DFTs as butterflies across the 16 lanes of a
 * row; 1 a z-line pass and a y-line pass (one more HBM pass).  Results
 * agree to FP32 rounding.  Errors: BSE_ERR_ARG for other values. */
bse_status bse_set_yz_schedule(bse_system* sys, int32_t schedule);

/* Workgroup order of the propagation's x pass (bit 0 of order), y-line
 * pass (bit 1) and fused y-z plane pass (bit 2, the 112^3 FP32 schedule);
 * results do not depend on it.  Bit clear: a 2-D grid, the fields of a tile
 * (plane) consecutive so that they run close together; bit set: a 1-D grid
 * renumbered so that each of the eight XCDs (each with its own L2) walks a
 * contiguous range of (tile, field), so that the fields of a tile share one
 * L2 for its unperturbed orbitals and phase tables.  Default 5 (measured at
 * 112^3, 21 pairs: the grouped x pass fetches 1.02x its algorithmic bytes
 * instead of 1.52x and runs 1 % faster, the grouped fused pass 1.02x
 * instead of 1.20x and 1 % faster; the grouped y-line pass, 7 % slower,
 * stays in the plain order).  Errors: BSE_ERR_ARG outside 0..7. */
bse_status bse_set_launch_order(bse_system* sys, int32_t order);

/* Kernel schedule of bse_spectrum's Lanczos iteration (the arithmetic and
 * the convergence checks are the same either way; results agree to
 * rounding).  0 (default): for n_o n_c <= 384 every step up to the next
 * convergence check runs in one single-workgroup launch with its vectors
 * in LDS; larger A take path 1.  1: one chip-wide launch per operation of
 * every step.  Errors: BSE_ERR_ARG for other values. */
bse_status bse_set_lanczos_path(bse_system* sys, int32_t path);

const char* bse_last_error(void);
const char* bse_version(void);
void bse_destroy_system(bse_system* sys);

/* ---------------------------------------------------------------------------
 * Screening surrogate: a Fourier neural operator that maps the scaled
 * source potential q_ij / s_ij (s_ij its RMS) plus molecule descriptor
 * channels to W^pol_ij / s_ij on the same grid.  It is trained on pairs that
 * bse_apply_W generates and its errors are measured on them; it does not replace the
 * propagation unless its prediction passes the caller's checks.
 *
 * Network: h0 = P x + p; for l < layers: z = W_l h + b_l + S_l h,
 * h = gelu(z) (no gelu after the last layer); y = Q h + q0.  S_l keeps the
 * modes kx, ky in [-modes, modes), kz in [0, modes) (FFT index units), mixes
 * channels per mode with complex weights R_l[k][i][o], and returns
 * (1/ng) Re sum_k c_k U(k) e^{ik.r} with c_k = 1 on kz = 0, 2 elsewhere.
 * Loss: mean over the batch of ||y - t||^2 / ||t||^2; Adam (0.9, 0.999,
 * 1e-8) on FP32 master weights; the weights used by the forward and
 * backward kernels are the master weights rounded to BF16 when
 * bf16_weights != 0; activations and accumulation are FP32.
 *
 * Flat parameter vector (floats): P[width][cin], p[width], Q[width], q0[1],
 * then per layer R_l[K][width][width][2] (re, im; K = 4 modes^3, mode order
 * kx-major, then ky, then kz, signed frequencies ascending), W_l[width][width]
 * (out, in), b_l[width].
 * Buffers: x[B][cin][n^3], y and t [B][n^3], FP32, device, caller-owned.
 * ------------------------------------------------------------------------- */
typedef struct bse_fno bse_fno;
typedef struct {
  int32_t n;            /* grid points per axis: 16, 32 or 64 */
  int32_t cin;          /* input channels (<= 64)             */
  int32_t width;        /* hidden channels (<= 64)            */
  int32_t modes;        /* m, 2m <= n                         */
  int32_t layers;       /* Fourier layers                     */
  int32_t max_batch;    /* largest batch                      */
  int32_t device;
  int32_t bf16_weights; /* 1: compute with BF16-rounded weights */
  uint64_t seed;        /* initial weights                    */
} bse_fno_config;

bse_status bse_fno_create(const bse_fno_config* cfg, bse_fno** out);
int64_t bse_fno_num_params(const bse_fno* fno);
/* Set (host, FP32, flat layout above) the master weights; resets Adam. */
bse_status bse_fno_set_params(bse_fno* fno, const float* host);
/* Copy the master (which = 0) or compute (which = 1) weights to the host. */
bse_status bse_fno_get_params(bse_fno* fno, float* host, int32_t which);
bse_status bse_fno_set_stream(bse_fno* fno, void* hip_stream);
/* Kernels of the per-mode channel mix U_k = V_k R_k of every Fourier layer
 * (and of its two backward products): path 0 (default) the matrix cores
 * (FP32 operands and accumulation, width up to 32), path 1 vector FMA.  The
 * two agree to FP32 rounding.  Errors: BSE_ERR_ARG for another path. */
bse_status bse_fno_set_mix_path(bse_fno* fno, int32_t path);
/* y = network(x) for a batch of B samples; returns when done. */
bse_status bse_fno_forward(bse_fno* fno, int32_t B, const void* x_dev, void* y_dev);
/* Loss of the batch against targets t and, if grad_host is non-null, its
 * gradient (flat layout; complex weights as d/dRe, d/dIm). */
bse_status bse_fno_loss_grad(bse_fno* fno, int32_t B, const void* x_dev, const void* t_dev,
                             double* loss, float* grad_host);
/* One training step: loss, gradient, Adam update with learning rate lr. */
bse_status bse_fno_train_step(bse_fno* fno, int32_t B, const void* x_dev, const void* t_dev,
                              double lr, double* loss);
/* Training batch under a symmetry of the cube (the Hamiltonian of a box and
 * the Coulomb kernel commute with the cube's rotations and reflections, so
 * a mapped sample has the mapped target): x_dst[b] = x_src[idx[b]] and
 * t_dst[b] = t_src[idx[b]] (x [.][cin][n^3], t [.][n^3], FP32, device,
 * points z fastest) with output axis k taken from input axis perm[k] and
 * the output axes in flip_mask (bit k = axis k) reversed.  idx (host,
 * B values in 0..n_src-1) and perm (host, a permutation of 0, 1, 2).
 * Returns when done.  Errors: BSE_ERR_ARG for B outside 1..max_batch, a
 * null pointer, an index out of range, a perm that is no permutation or a
 * flip_mask outside 0..7. */
bse_status bse_fno_gather(bse_fno* fno, int32_t B, const int32_t* idx, int32_t n_src, const void* x_src,
                          const void* t_src, const int32_t* perm, int32_t flip_mask, void* x_dst, void* t_dst);
const char* bse_fno_last_error(void);
int32_t bse_fno_max_batch(const bse_fno* fno);
void bse_fno_destroy(bse_fno* fno);

/* Training samples for the surrogate from a system's pairs pq[n_pairs][2]
 * (host): x_dev[n][3][ng] (FP32) receives q/s, the ground-state density
 * 2 sum_occ phi^2 divided by its maximum, and V_ext divided by max|V_ext|,
 * with s the RMS of q; t_dev (nullable, FP32 [n][ng]) receives W^pol/s from
 * the propagation (bse_apply_W); scale_dev (nullable, FP64 [n]) receives s.
 * The grid of the system must be that of the network. */
bse_status bse_fno_make_samples(bse_system* sys, int32_t n_pairs, const int32_t* pq, void* x_dev,
                                void* t_dev, void* scale_dev);

/* Surrogate W-action with the propagation as the judge of its error: the
 * network's W = q + s * net(x) for every pair pq[n_pairs][2] (host) into
 * w_dev[n_pairs][ng] (device, FP64, caller-owned); then n_judge pairs spread
 * evenly over the list (index floor((2k+1) n_pairs / (2 n_judge)), k <
 * n_judge) are propagated (bse_apply_W) and the network's relative L2 error
 * |W_net - W| / |W| on each is measured on the device.  The network's other
 * predictions are kept only when every judged error is finite and <= tol
 * and their own sign check holds (<rho|W^pol rho> < 0 < <rho|W rho>, rho =
 * phi_p phi_q); every other pair -- all of them when the judge rejects the
 * network, or when n_judge = 0 or tol <= 0 -- gets the propagation's W, and
 * the judged pairs return their propagated W.  The unjudged pairs' errors
 * are estimated by the sample, not bounded.  accepted[n_pairs] (host,
 * nullable): 1 where w_dev holds the network's prediction, 0 where it holds
 * the propagation's; judged_err[n_judge] (host, nullable): the measured
 * errors.  Errors: BSE_ERR_ARG for null buffers, 0 > n_judge > n_pairs, a
 * non-finite tol or an index out of range. */
bse_status bse_apply_W_surrogate(bse_system* sys, bse_fno* net, int32_t n_pairs, const int32_t* pq,
                                 void* w_dev, double tol, int32_t n_judge, int32_t* accepted,
                                 double* judged_err);

#ifdef __cplusplus
}
#endif
#endif /* BSE_H */
