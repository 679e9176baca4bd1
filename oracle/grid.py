"""Periodic real-space grid operators in FP64 (oracle; test infrastructure).

* Grid: n_x x n_y x n_z points, spacing h, row-major with z fastest;
  integrals are sums times h^3.
* Kinetic energy -1/2 Laplacian is Fourier spectral: |k|^2/2 with
  k = 2 pi fftfreq(n, h) on each axis (the split-operator propagation named
  in the Results section uses exactly this operator).
* Coulomb potential of a density, v[rho](r) = int |r - r'|^-1 rho(r') dr'
  (the q_ij of the "Stochastic evaluation of the action of W" subsection and
  the u_ij of Eq. 11): periodic solution of the Poisson equation,
  FFT^-1( 4 pi / |k|^2 FFT rho ), with the k = 0 component set to zero.
"""
from __future__ import annotations

import math
import os

import numpy as np

try:
    import scipy.fft as _sfft
    # FFT threads: BSE_ORACLE_THREADS if set (one-core runs), else every core
    _W = int(os.environ.get("BSE_ORACLE_THREADS", "0")) or os.cpu_count() or 1

    def fftn(x):
        return _sfft.fftn(x, axes=(-3, -2, -1), workers=_W)

    def ifftn(x):
        return _sfft.ifftn(x, axes=(-3, -2, -1), workers=_W)
except ImportError:  # pragma: no cover
    def fftn(x):
        return np.fft.fftn(x, axes=(-3, -2, -1))

    def ifftn(x):
        return np.fft.ifftn(x, axes=(-3, -2, -1))


class Grid:
    def __init__(self, shape, h: float):
        self.shape = tuple(int(s) for s in shape)
        self.h = float(h)
        self.dv = self.h ** 3
        self.ng = int(np.prod(self.shape))
        ks = [2.0 * math.pi * np.fft.fftfreq(n, d=self.h) for n in self.shape]
        self.k2 = (ks[0][:, None, None] ** 2 + ks[1][None, :, None] ** 2
                   + ks[2][None, None, :] ** 2)
        with np.errstate(divide="ignore"):
            vk = 4.0 * math.pi / self.k2
        vk[0, 0, 0] = 0.0
        self.vk = vk

    # integrals ------------------------------------------------------------
    def dot(self, f, g):
        """<f|g> = h^3 sum conj(f) g over the last three axes."""
        return np.sum(np.conj(f) * g, axis=(-3, -2, -1)) * self.dv

    # operators ------------------------------------------------------------
    def poisson(self, rho):
        """Coulomb potential of a real density (any leading batch axes)."""
        return np.real(ifftn(self.vk * fftn(rho)))

    def kinetic(self, psi):
        """-1/2 Laplacian of a field."""
        return ifftn(0.5 * self.k2 * fftn(psi))

    def kinetic_propagator(self, psi, dt: float):
        """exp(-i T dt) psi, T = -1/2 Laplacian."""
        return ifftn(np.exp(-0.5j * self.k2 * dt) * fftn(psi))

    def coords(self):
        """Grid point positions x_i = i h on each axis."""
        return [np.arange(n, dtype=np.float64) * self.h for n in self.shape]
