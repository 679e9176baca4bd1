"""Finite-box W(k->0) correction in FP64 (oracle; test infrastructure).

The Results section shifts the scissors Delta of Eq. 1 down by W(k->0):
the calculation is repeated in several box sizes, each box gives the
average Kohn-Sham potential on its boundary v_bndry, W(k->0) is taken as
eps_eff^-1 v_bndry, and the one parameter eps_eff^-1 is fitted so that the
spectra of the different boxes overlap.  Readings:

* Kohn-Sham potential of the synthetic H0 (kinetic + V_ext, no mean-field
  term of its own): V_KS = V_ext + v_H[n] with n = 2 sum_{s < N_occ}
  phi_s^2, v_H the periodic Coulomb potential (k = 0 term removed).
* Boundary: the grid points on the three faces through the origin corner
  (index 0 on any axis; the opposite faces are their periodic images),
  3 n^2 - 3 n + 1 points for an n^3 grid.  v_bndry is their mean minus the
  mean over the whole cell, the zero that a k = 0-free potential refers to.
* Overlapping spectra: the scissors adds the same constant to every
  Tamm-Dancoff eigenvalue, so spectra corrected by -W(k->0) overlap when
  the lowest excitation energies do.  eps_eff^-1 is the least-squares slope
  of Omega_n(box) = c_n + eps_eff^-1 v_bndry(box), one intercept per
  exciton.
"""
from __future__ import annotations

import numpy as np

from .grid import Grid


def occupied_density(phi_occ: np.ndarray) -> np.ndarray:
    """n = 2 sum_s phi_s^2 over the occupied orbitals phi_occ [N_occ, ...]."""
    return 2.0 * np.sum(phi_occ * phi_occ, axis=0)


def ks_potential(grid: Grid, v_ext: np.ndarray, phi_occ: np.ndarray) -> np.ndarray:
    """V_ext + v_H[n] on the grid."""
    return v_ext + grid.poisson(occupied_density(phi_occ))


def boundary_mask(shape) -> np.ndarray:
    """True on the grid points with index 0 along some axis."""
    m = np.zeros(shape, dtype=bool)
    m[0, :, :] = True
    m[:, 0, :] = True
    m[:, :, 0] = True
    return m


def boundary_average(v: np.ndarray) -> float:
    """Mean of v over the boundary points minus its mean over the cell."""
    return float(v[boundary_mask(v.shape)].mean() - v.mean())


def boundary_potential(grid: Grid, v_ext: np.ndarray, phi_occ: np.ndarray) -> float:
    """v_bndry of one box."""
    return boundary_average(ks_potential(grid, v_ext, phi_occ))


def fit_inverse_dielectric(omega: np.ndarray, v_bndry: np.ndarray):
    """Least-squares eps_eff^-1 and intercepts c_n for
    omega[b, n] = c_n + eps_eff^-1 v_bndry[b] (b: box, n: exciton).
    Returns (eps_inv, c, w_k0) with w_k0[b] = eps_inv * v_bndry[b]."""
    omega = np.asarray(omega, dtype=np.float64)
    v = np.asarray(v_bndry, dtype=np.float64)
    n_box, n_exc = omega.shape
    if n_box < 2:
        raise ValueError("need at least two boxes")
    dv = v - v.mean()
    if not np.abs(dv).max() > 1e-12 * max(float(np.abs(v).max()), 1e-300):
        raise ValueError("boundary potentials of the boxes coincide")
    den = n_exc * float(dv @ dv)
    dom = omega - omega.mean(axis=0, keepdims=True)
    eps_inv = float(np.sum(dom * dv[:, None])) / den
    c = omega.mean(axis=0) - eps_inv * v.mean()
    return eps_inv, c, eps_inv * v
