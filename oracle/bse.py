"""Tamm-Dancoff BSE matrix, excitons and absorption in FP64 (oracle; test
infrastructure).

* Eq. 1: A(ia; jb) = (eps_a - eps_i + Delta) delta_ij delta_ab + 2 (ia|jb)
  - (phi_a phi_b | W | phi_i phi_j), singlet, static W.  The printed
  eps_a - eps_j is read as eps_a - eps_i (equal under delta_ij); Delta is the
  scissors shift of the GW-corrected gap (Delta GW_0 paragraph).
* (ia|jb) = h^3 sum_r phi_i phi_a v[phi_j phi_b]; the direct term is
  h^3 sum_r phi_a phi_b W_ij with W_ij = q_ij + W^pol_ij (W_ji = W_ij).
* Index order of A: row (i - i0) * n_c + (a - a0) for valence i (the highest
  n_o occupied) and conduction a (the lowest n_c virtual).
* Eq. 7 in the electron-hole basis: sigma(omega) = omega <f0| delta(A - omega)
  |f0> with f0_ia = <phi_a| x |phi_i>; via the eigenpairs (Omega_n, X_n) of A
  this is omega sum_n |<X_n|f0>|^2 delta(omega - Omega_n).  The delta is a
  Gaussian of standard deviation ``sigma`` (the 0.08 eV broadening of the
  Results section read as a standard deviation); x, y, z polarisations are
  summed.  Positions are measured from the box centre.
"""
from __future__ import annotations

import math

import numpy as np

from .grid import Grid


def exchange(grid: Grid, phi_v: np.ndarray, phi_c: np.ndarray) -> np.ndarray:
    """(ia|jb) for i, j in phi_v [n_o, ...] and a, b in phi_c [n_c, ...]."""
    n_o, n_c = phi_v.shape[0], phi_c.shape[0]
    rho = (phi_v[:, None] * phi_c[None, :]).reshape(n_o * n_c, -1)
    vr = grid.poisson(rho.reshape((n_o * n_c,) + grid.shape)).reshape(n_o * n_c, -1)
    return (rho @ vr.T) * grid.dv


def direct(grid: Grid, phi_c: np.ndarray, w_ij: np.ndarray) -> np.ndarray:
    """(phi_a phi_b | W | phi_i phi_j) as D[(ia), (jb)], given the full
    symmetric stack w_ij [n_o, n_o, nx, ny, nz]."""
    n_o, n_c = w_ij.shape[0], phi_c.shape[0]
    rab = (phi_c[:, None] * phi_c[None, :]).reshape(n_c * n_c, -1)   # (a, b)
    K = (rab @ w_ij.reshape(n_o * n_o, -1).T) * grid.dv              # [(a,b),(i,j)]
    K = K.reshape(n_c, n_c, n_o, n_o)
    # D[i, a, j, b] = K[a, b, i, j]
    return np.transpose(K, (2, 0, 3, 1)).reshape(n_o * n_c, n_o * n_c)


def w_stack(n_o: int, pairs, w_pairs: np.ndarray) -> np.ndarray:
    """Full symmetric [n_o, n_o, ...] stack from W for the pairs (i <= j),
    indices relative to the valence window."""
    out = np.zeros((n_o, n_o) + w_pairs.shape[1:])
    for k, (i, j) in enumerate(pairs):
        out[i, j] = w_pairs[k]
        out[j, i] = w_pairs[k]
    return out


def build_a(grid: Grid, phi_v: np.ndarray, phi_c: np.ndarray, eps_v: np.ndarray,
            eps_c: np.ndarray, w_full: np.ndarray, scissors: float = 0.0) -> np.ndarray:
    """Eq. 1 with the W_ij stack w_full [n_o, n_o, ...]."""
    n_o, n_c = phi_v.shape[0], phi_c.shape[0]
    diag = (eps_c[None, :] - eps_v[:, None] + scissors).reshape(-1)
    A = np.diag(diag) + 2.0 * exchange(grid, phi_v, phi_c) - direct(grid, phi_c, w_full)
    return A


def dipoles(grid: Grid, phi_v: np.ndarray, phi_c: np.ndarray) -> np.ndarray:
    """f0[(ia), axis] = <phi_a| r_axis - centre |phi_i>."""
    xs = grid.coords()
    n_o, n_c = phi_v.shape[0], phi_c.shape[0]
    out = np.zeros((n_o * n_c, 3))
    rho = (phi_v[:, None] * phi_c[None, :])                        # [n_o, n_c, ...]
    for ax in range(3):
        c = 0.5 * grid.shape[ax] * grid.h
        x = xs[ax] - c
        shp = [1, 1, 1]
        shp[ax] = -1
        out[:, ax] = (np.sum(rho * x.reshape(shp), axis=(-3, -2, -1)) * grid.dv).reshape(-1)
    return out


def excitons(A: np.ndarray, f0: np.ndarray, n_exc: int):
    """Lowest n_exc eigenvalues of A and |<X_n|f0_axis>|^2 [n_exc, 3]."""
    w, X = np.linalg.eigh(A)
    d = X[:, :n_exc].T @ f0
    return w[:n_exc], d ** 2


def absorption(omega: np.ndarray, dip2: np.ndarray, w_grid: np.ndarray,
               sigma: float) -> np.ndarray:
    """Eq. 7 with Gaussian-broadened deltas, polarisations summed."""
    s = dip2.sum(axis=1)
    g = np.exp(-0.5 * ((w_grid[:, None] - omega[None, :]) / sigma) ** 2) / (
        sigma * math.sqrt(2.0 * math.pi))
    return w_grid * (g @ s)


# ---------------------------------------------------------------------------
# Chebyshev spectrum (Eqs. 7-8): sigma(omega) = omega <f0| delta(A - omega)
# |f0>, the broadened delta expanded in Chebyshev polynomials of the scaled
# A, with the residues R_n = <f0| T_n(A~) |f0> from the three-term
# recursion.  A~ = (A - b) / a maps [e_min, e_max] into [-1, 1].
# ---------------------------------------------------------------------------
def spectral_bounds(A: np.ndarray):
    """Gershgorin interval of the symmetric matrix A."""
    r = np.abs(A).sum(axis=1) - np.abs(np.diag(A))
    return float(np.min(np.diag(A) - r)), float(np.max(np.diag(A) + r))


def chebyshev_scale(e_min: float, e_max: float, margin: float = 0.01):
    """(a, b) with A~ = (A - b)/a; the interval is widened by ``margin`` of
    its half-width so that the spectrum sits strictly inside (-1, 1)."""
    b = 0.5 * (e_max + e_min)
    a = 0.5 * (e_max - e_min) * (1.0 + margin)
    return a, b


def chebyshev_residues(A: np.ndarray, f0: np.ndarray, n_mom: int, a: float, b: float):
    """R_n = <f0 | T_n(A~) | f0> for n < n_mom, one column of f0 per
    polarisation: f^0 = f0, f^1 = A~ f^0, f^{n+1} = 2 A~ f^n - f^{n-1}."""
    At = (A - b * np.eye(A.shape[0])) / a
    f_prev = f0.copy()
    R = np.zeros((n_mom, f0.shape[1]))
    R[0] = np.sum(f0 * f_prev, axis=0)
    if n_mom == 1:
        return R
    f_cur = At @ f0
    R[1] = np.sum(f0 * f_cur, axis=0)
    for n in range(2, n_mom):
        f_next = 2.0 * (At @ f_cur) - f_prev
        R[n] = np.sum(f0 * f_next, axis=0)
        f_prev, f_cur = f_cur, f_next
    return R


def chebyshev_coefficients(w_grid: np.ndarray, n_mom: int, a: float, b: float, sigma: float,
                           n_nodes: int | None = None):
    """g_n(omega): Chebyshev coefficients in A~ of the Gaussian delta of
    standard deviation ``sigma`` centred at omega, by Gauss-Chebyshev
    quadrature on ``n_nodes`` nodes (default 2 n_mom):
    g_n = (2 - delta_n0)/M sum_k G(a cos th_k + b - omega) cos(n th_k),
    th_k = pi (k + 1/2) / M."""
    M = 2 * n_mom if n_nodes is None else n_nodes
    th = math.pi * (np.arange(M) + 0.5) / M
    E = a * np.cos(th) + b
    G = np.exp(-0.5 * ((E[None, :] - w_grid[:, None]) / sigma) ** 2) / (sigma * math.sqrt(2.0 * math.pi))
    C = np.cos(np.arange(n_mom)[:, None] * th[None, :])           # [n, k]
    g = (G @ C.T) / M
    g[:, 1:] *= 2.0
    return g                                                       # [n_w, n_mom]


def chebyshev_absorption(R: np.ndarray, w_grid: np.ndarray, a: float, b: float, sigma: float,
                         n_nodes: int | None = None) -> np.ndarray:
    """Eq. 7 through Eq. 8: sigma(omega) = omega sum_pol sum_n g_n(omega) R_n."""
    g = chebyshev_coefficients(w_grid, R.shape[0], a, b, sigma, n_nodes)
    return w_grid * (g @ R.sum(axis=1))


def chebyshev_states(A: np.ndarray, f0: np.ndarray, n_mom: int, a: float, b: float,
                     w_grid: np.ndarray, sigma: float, n_nodes: int | None = None) -> np.ndarray:
    """Eq. 8: the frequency-resolved exciton states
    |f(omega)> = sum_{n < n_mom} g_n(omega) T_n(A~) |f^0>, the f^n by the
    three-term recursion in A~ = (A - b)/a, one column of f0 per
    polarisation; [n_w, n, n_pol]."""
    g = chebyshev_coefficients(np.asarray(w_grid, dtype=float), n_mom, a, b, sigma, n_nodes)
    At = (A - b * np.eye(A.shape[0])) / a
    out = g[:, 0, None, None] * f0[None]
    if n_mom == 1:
        return out
    f_prev, f_cur = f0, At @ f0
    out = out + g[:, 1, None, None] * f_cur[None]
    for n in range(2, n_mom):
        f_next = 2.0 * (At @ f_cur) - f_prev
        out = out + g[:, n, None, None] * f_next[None]
        f_prev, f_cur = f_cur, f_next
    return out


def exciton_density(phi_v: np.ndarray, phi_c: np.ndarray, F: np.ndarray) -> np.ndarray:
    """Exciton density of an electron-hole vector F [n_o n_c] (rows of A,
    valence index major): the mixed-representation density 2 sum_i phi_i f_i
    with f_i = sum_a F_ia phi_a, i.e. 2 sum_ia F_ia phi_i phi_a."""
    n_o, n_c = phi_v.shape[0], phi_c.shape[0]
    Fm = np.asarray(F, dtype=float).reshape(n_o, n_c)
    f_i = np.tensordot(Fm, phi_c, axes=(1, 0))          # [n_o, ...]
    return 2.0 * np.sum(phi_v * f_i, axis=0)


# ---------------------------------------------------------------------------
# Matrix-free action of A in the mixed hole-grid representation (Eq. 6 with
# A = Q A-bar): f_j(r) for the n_o valence orbitals j,
#   (A-bar f)_j = (H0 + Delta - eps_j) f_j + dv phi_j - sum_i f_i W_ij,
#   dv = v[dn], dn = 2 sum_i phi_i f_i,
# and Q = 1 - sum_{s < N_occ} |phi_s><phi_s| applied to every f_j.
# ---------------------------------------------------------------------------
def apply_a_mixed(grid: Grid, v_ext: np.ndarray, phi_occ: np.ndarray, eps_v: np.ndarray,
                  w_full: np.ndarray, f: np.ndarray, scissors: float = 0.0) -> np.ndarray:
    """A f for f [n_o, nx, ny, nz] (real); phi_occ [N_occ, ...] with the
    valence window as its last n_o rows; eps_v [n_o]; w_full [n_o, n_o, ...]
    the symmetric W_ij stack."""
    n_o, n_occ = f.shape[0], phi_occ.shape[0]
    phv = phi_occ[n_occ - n_o:]
    dv = grid.poisson(2.0 * np.sum(phv * f, axis=0))
    out = np.empty_like(f)
    for j in range(n_o):
        t = np.real(grid.kinetic(f[j])) + (v_ext + scissors - eps_v[j]) * f[j] + dv * phv[j]
        for i in range(n_o):
            t = t - f[i] * w_full[i, j]
        out[j] = t
    P = phi_occ.reshape(n_occ, -1)
    c = (out.reshape(n_o, -1) @ P.T) * grid.dv
    return out - (c @ P).reshape(out.shape)


def chebyshev_residues_op(apply, f0_list, n_mom: int, a: float, b: float, inner):
    """R_n[p] = inner(f0_p, T_n(A~) f0_p) for a linear operator given by
    ``apply`` (A~ = (A - b)/a), n < n_mom, by the three-term recursion."""
    R = np.zeros((n_mom, len(f0_list)))
    for p, f0 in enumerate(f0_list):
        f_prev = f0
        R[0, p] = inner(f0, f0)
        if n_mom == 1:
            continue
        f_cur = (apply(f0) - b * f0) / a
        R[1, p] = inner(f0, f_cur)
        for n in range(2, n_mom):
            f_next = 2.0 * (apply(f_cur) - b * f_cur) / a - f_prev
            R[n, p] = inner(f0, f_next)
            f_prev, f_cur = f_cur, f_next
    return R


def chebyshev_states_op(apply, f0_list, n_mom: int, a: float, b: float, w_grid: np.ndarray,
                        sigma: float, n_nodes: int | None = None) -> np.ndarray:
    """Eq. 8 for a linear operator given by ``apply``: for each start vector
    f0_p, sum_{n < n_mom} g_n(omega) T_n(A~) f0_p with A~ = (A - b)/a, by
    the three-term recursion; [n_w, n_pol, *f0.shape]."""
    g = chebyshev_coefficients(np.asarray(w_grid, dtype=float), n_mom, a, b, sigma, n_nodes)
    out = np.zeros((g.shape[0], len(f0_list)) + np.shape(f0_list[0]))
    for p, f0 in enumerate(f0_list):
        f_prev = f0
        out[:, p] = g[:, 0].reshape((-1,) + (1,) * f0.ndim) * f0
        if n_mom == 1:
            continue
        f_cur = (apply(f0) - b * f0) / a
        out[:, p] += g[:, 1].reshape((-1,) + (1,) * f0.ndim) * f_cur
        for n in range(2, n_mom):
            f_next = 2.0 * (apply(f_cur) - b * f_cur) / a - f_prev
            out[:, p] += g[:, n].reshape((-1,) + (1,) * f0.ndim) * f_next
            f_prev, f_cur = f_cur, f_next
    return out


def mixed_amplitudes(grid: Grid, phi_a: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Electron-hole amplitudes of a mixed-representation state:
    f_ia = <phi_a|f_i> = h^3 sum_r phi_a(r) f_i(r); [n_o, n_a]."""
    n_o, n_a = f.shape[0], phi_a.shape[0]
    return (f.reshape(n_o, -1) @ phi_a.reshape(n_a, -1).T) * grid.dv


def mixed_exciton_density(phi_v: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Exciton density of a mixed-representation state: 2 sum_i phi_i f_i."""
    return 2.0 * np.sum(phi_v * f, axis=0)


def mixed_dipole_start(grid: Grid, phi_occ: np.ndarray, n_o: int):
    """Start vectors of the mixed representation, one per axis:
    f0_j = Q (r_axis - box centre) phi_j for the valence window (the last
    n_o occupied orbitals); [3][n_o, nx, ny, nz]."""
    n_occ = phi_occ.shape[0]
    phv = phi_occ[n_occ - n_o:]
    P = phi_occ.reshape(n_occ, -1)
    xs = grid.coords()
    out = []
    for ax in range(3):
        shp = [1, 1, 1]
        shp[ax] = -1
        x = (xs[ax] - 0.5 * grid.shape[ax] * grid.h).reshape(shp)
        f = (phv * x).reshape(n_o, -1)
        f = f - ((f @ P.T) * grid.dv) @ P
        out.append(f.reshape((n_o,) + grid.shape))
    return out
