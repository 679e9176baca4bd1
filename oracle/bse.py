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
