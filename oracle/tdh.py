"""Action of the static screened interaction on a pair density, in FP64
(oracle; test infrastructure).

Follows the "Stochastic evaluation of the action of W" subsection:

* W = v + W^pol, so W_ij(r) = q_ij(r) + W^pol_ij(r) with the source
  potential q_ij = v[phi_i phi_j].
* The occupied orbitals (all N_occ of them, or L random-sign combinations
  eta_l = L^-1/2 sum_s (+-1) phi_s, Eq. 14) are kicked by exp(-i alpha q_ij)
  and propagated with H0 + u_ij(t) (Eq. 10), u_ij the Coulomb potential of
  the density change (Eq. 11); W^pol_ij(t) = u_ij(t)/alpha (Eq. 12) and the
  static action is the Gaussian-damped time integral (Eq. 13).
* Both the perturbed and the unperturbed sets are propagated; every M steps
  (and at t = 0) the perturbed set is cleaned of occupied-space amplitude,
  eta^a <- eta^0 + Q (eta^a - eta^0), Q = 1 - sum_s |phi_s><phi_s| (Eq. 15),
  then each perturbed orbital is rescaled to its initial norm.

Readings where the paper is silent (each restated in the design notes):

* u is the potential of n^alpha(t) - n^{alpha=0}(t), the unperturbed set
  feeling V_ext only.
* Time stepping is Strang split-operator with spacing dt: half potential
  phase exp(-i (V_ext + u_n) dt/2), kinetic exp(-i T dt) in k space, new
  density -> u_{n+1}, half potential phase with u_{n+1}.  A potential phase
  does not change a density, so u_{n+1} is well defined after the kinetic
  part.
* The time integral is the trapezoid rule on t_n = n dt truncated at
  T = N dt: weights 1/2 at n = 0 and n = N, 1 otherwise.
* The cleaning at step n (n a multiple of M, and n = 0) acts on the state
  after the full step; u_n is recomputed from the cleaned state before it
  enters the time integral and the next step.
* Linearised form (``mode="linear"``): the exact d/d(alpha) at alpha = 0
  of the finite-alpha scheme above.  With delta eta = d eta^a / d alpha:
  delta eta(0) = -i q eta, density change 4 sum_l Re(conj(eta^0) delta eta),
  half phase delta eta <- e^{-i V dt/2}(delta eta - i dt/2 u eta^0), cleaning
  delta eta <- Q delta eta, and the first-order norm restoration
  delta eta <- delta eta - Re<eta^0, delta eta>/||eta_l(0)||^2 eta^0.
  The 1/alpha of Eq. 12 is absorbed.
"""
from __future__ import annotations

import math

import numpy as np

from .grid import Grid


def stochastic_orbitals(phi_occ: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """Eq. 14: eta_l = L^-1/2 sum_s xi[l, s] phi_s.  phi_occ is
    [N_occ, nx, ny, nz] real; xi is [L, N_occ] of +-1."""
    L = xi.shape[0]
    n_occ = phi_occ.shape[0]
    eta = (xi.astype(np.float64) @ phi_occ.reshape(n_occ, -1)) / math.sqrt(L)
    return eta.reshape((L,) + phi_occ.shape[1:])


def source_potential(grid: Grid, phi_i: np.ndarray, phi_j: np.ndarray) -> np.ndarray:
    """q_ij = v[phi_i phi_j]."""
    return grid.poisson(phi_i * phi_j)


def time_weights(n_steps: int, dt: float, gamma: float) -> np.ndarray:
    """Trapezoid weights of the damped integral, Eq. 13: c_n exp(-g^2 t_n^2/2) dt
    for n = 0..N."""
    t = np.arange(n_steps + 1, dtype=np.float64) * dt
    c = np.ones(n_steps + 1)
    c[0] = 0.5
    c[-1] = 0.5
    return c * np.exp(-0.5 * gamma ** 2 * t ** 2) * dt


def _project_out(grid: Grid, phi_occ2: np.ndarray, d: np.ndarray) -> np.ndarray:
    """Q d for fields d [..., nx, ny, nz]; phi_occ2 is [N_occ, ng]."""
    shp = d.shape
    d2 = d.reshape(-1, grid.ng)
    c = (d2 @ phi_occ2.T) * grid.dv          # <phi_s|d>, phi real
    return (d2 - c @ phi_occ2).reshape(shp)


def w_pol(grid: Grid, v_ext: np.ndarray, phi_occ: np.ndarray, eta0: np.ndarray,
          q: np.ndarray, *, dt: float, n_steps: int, gamma: float, clean_every: int,
          mode: str = "linear", alpha: float = 1e-6, feedback: bool = True,
          renorm: bool = True, clean_t0: bool = True, progress=None) -> np.ndarray:
    """W^pol for each source potential in q [B, nx, ny, nz].

    eta0: the propagated occupied set [L, nx, ny, nz] (stochastic orbitals,
    or the N_occ orbitals themselves for the deterministic method).
    feedback=False drops u from the propagation (independent-particle
    response) while still accumulating v[density change]; it is a test mode.
    clean_every = 0 disables cleaning (including t = 0 unless clean_t0).
    progress (nullable) is called with the step count after every step (a
    report hook for long runs; it sees no data).
    """
    if mode not in ("linear", "finite"):
        raise ValueError(mode)
    B = q.shape[0]
    phi2 = phi_occ.reshape(phi_occ.shape[0], -1)
    w = time_weights(n_steps, dt, gamma)
    ph_half = np.exp(-0.5j * v_ext * dt)
    eta_u = eta0.astype(np.complex128)                     # [L, ...]
    norm0 = np.real(grid.dot(eta_u, eta_u))                # ||eta_l(0)||^2
    wpol = np.zeros(q.shape, dtype=np.float64)
    do_clean0 = clean_t0 and clean_every > 0

    if mode == "linear":
        d = -1j * q[:, None] * eta_u[None]                 # [B, L, ...]

        def clean(d, eta):
            d = _project_out(grid, phi2, d)
            if renorm:
                r = np.real(grid.dot(eta[None], d))        # [B, L]
                d = d - (r / norm0[None, :])[..., None, None, None] * eta[None]
            return d

        def dens(d, eta):
            return 4.0 * np.sum(np.real(np.conj(eta[None]) * d), axis=1)

        if do_clean0:
            d = clean(d, eta_u)
        u = grid.poisson(dens(d, eta_u))
        wpol += w[0] * u
        for n in range(n_steps):
            uf = u if feedback else 0.0 * u
            d = ph_half * (d - 0.5j * dt * uf[:, None] * eta_u[None])
            eta_u = ph_half * eta_u
            d = grid.kinetic_propagator(d, dt)
            eta_u = grid.kinetic_propagator(eta_u, dt)
            u = grid.poisson(dens(d, eta_u))
            uf = u if feedback else 0.0 * u
            d = ph_half * (d - 0.5j * dt * uf[:, None] * eta_u[None])
            eta_u = ph_half * eta_u
            if clean_every > 0 and (n + 1) % clean_every == 0:
                d = clean(d, eta_u)
                u = grid.poisson(dens(d, eta_u))
            wpol += w[n + 1] * u
            if progress is not None:
                progress(n + 1)
        return wpol

    # finite alpha: the paper's scheme literally, divided by alpha
    ea = np.exp(-1j * alpha * q)[:, None] * eta_u[None]    # [B, L, ...]

    def clean_f(ea, eu):
        ea = eu[None] + _project_out(grid, phi2, ea - eu[None])
        if renorm:
            nr = np.real(grid.dot(ea, ea))                 # [B, L]
            ea = ea * np.sqrt(norm0[None, :] / nr)[..., None, None, None]
        return ea

    def dens_f(ea, eu):
        return 2.0 * np.sum(np.abs(ea) ** 2 - np.abs(eu[None]) ** 2, axis=1)

    if do_clean0:
        ea = clean_f(ea, eta_u)
    u = grid.poisson(dens_f(ea, eta_u))
    wpol += w[0] * u / alpha
    for n in range(n_steps):
        uf = u if feedback else 0.0 * u
        ea = np.exp(-0.5j * dt * (v_ext[None] + uf))[:, None] * ea
        eta_u = ph_half * eta_u
        ea = grid.kinetic_propagator(ea, dt)
        eta_u = grid.kinetic_propagator(eta_u, dt)
        u = grid.poisson(dens_f(ea, eta_u))
        uf = u if feedback else 0.0 * u
        ea = np.exp(-0.5j * dt * (v_ext[None] + uf))[:, None] * ea
        eta_u = ph_half * eta_u
        if clean_every > 0 and (n + 1) % clean_every == 0:
            ea = clean_f(ea, eta_u)
            u = grid.poisson(dens_f(ea, eta_u))
        wpol += w[n + 1] * u / alpha
    return wpol


def apply_w(grid: Grid, v_ext: np.ndarray, phi: np.ndarray, n_occ: int,
            pairs, eta0: np.ndarray, **kw):
    """W_ij = q_ij + W^pol_ij for each (i, j) in ``pairs``.

    phi: [n_orb, nx, ny, nz] real orbitals (h^3-normalised), the first n_occ
    occupied.  Returns (W, W^pol), each [n_pairs, nx, ny, nz]."""
    pairs = np.asarray(pairs).reshape(-1, 2)
    q = np.stack([source_potential(grid, phi[i], phi[j]) for i, j in pairs])
    wp = w_pol(grid, v_ext, phi[:n_occ], eta0, q, **kw)
    return q + wp, wp
