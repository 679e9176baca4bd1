"""Pins of the oracle's grid operators (Poisson, kinetic propagator) against
closed forms that do not use the FFT."""
import math

import numpy as np
import pytest
from scipy.special import erf

from oracle.grid import Grid


def _periodic_gaussian(grid, centre, sigma, images=3):
    """Normalised Gaussian charge, summed over periodic images, on the grid."""
    xs = grid.coords()
    rho = np.zeros(grid.shape)
    box = [n * grid.h for n in grid.shape]
    norm = (2.0 * math.pi * sigma ** 2) ** -1.5
    for a in range(-images, images + 1):
        for b in range(-images, images + 1):
            for c in range(-images, images + 1):
                dx = xs[0] - centre[0] - a * box[0]
                dy = xs[1] - centre[1] - b * box[1]
                dz = xs[2] - centre[2] - c * box[2]
                rho += norm * np.exp(-(dx[:, None, None] ** 2 + dy[None, :, None] ** 2
                                       + dz[None, None, :] ** 2) / (2 * sigma ** 2))
    return rho


def _reciprocal_sum_potential(grid, charges, pts):
    """Periodic potential of Gaussian charges (q, centre, sigma) with the
    k = 0 term removed, by explicit plane-wave summation over G != 0:
    (1/Omega) sum_G 4 pi/G^2 q exp(-G^2 sigma^2/2) cos(G.(r - R))."""
    box = grid.shape[0] * grid.h
    omega = box ** 3
    mmax = 14
    m = np.arange(-mmax, mmax + 1)
    G1 = 2 * math.pi * m / box
    Gx, Gy, Gz = np.meshgrid(G1, G1, G1, indexing="ij")
    G2 = Gx ** 2 + Gy ** 2 + Gz ** 2
    mask = G2 > 0
    Gx, Gy, Gz, G2 = Gx[mask], Gy[mask], Gz[mask], G2[mask]
    out = np.zeros(len(pts))
    for q, R, sigma in charges:
        amp = 4 * math.pi / G2 * q * np.exp(-G2 * sigma ** 2 / 2) / omega
        for k, r in enumerate(pts):
            ph = Gx * (r[0] - R[0]) + Gy * (r[1] - R[1]) + Gz * (r[2] - R[2])
            out[k] += np.sum(amp * np.cos(ph))
    return out


def test_poisson_gaussian_reciprocal_sum():
    """P1: grid Poisson of a resolved Gaussian = analytic lattice sum."""
    grid = Grid((16, 16, 16), 0.5)
    sig = 1.2
    R1 = (3.1, 4.2, 3.7)
    R2 = (5.0, 2.6, 4.4)
    rho = _periodic_gaussian(grid, R1, sig) - 0.5 * _periodic_gaussian(grid, R2, sig)
    v = grid.poisson(rho)
    rng = np.random.default_rng(3)
    idx = rng.integers(0, 16, size=(12, 3))
    pts = [(i * 0.5, j * 0.5, k * 0.5) for i, j, k in idx]
    ref = _reciprocal_sum_potential(grid, [(1.0, R1, sig), (-0.5, R2, sig)], pts)
    got = np.array([v[i, j, k] for i, j, k in idx])
    assert np.max(np.abs(got - ref)) < 1e-9 * np.max(np.abs(ref))


def test_poisson_free_space_limit():
    """P1: a neutral Gaussian pair in a large box approaches the free-space
    potential erf(r/(sqrt2 s))/r - erf(r'/(sqrt2 s))/r' (dipole images are
    O(p / box^3)); catches the 4 pi and the sign independently of the
    lattice-sum formula."""
    grid = Grid((48, 48, 48), 0.5)
    sig = 0.9
    c = 12.0
    R1 = (c - 0.8, c, c)
    R2 = (c + 0.8, c, c)
    rho = _periodic_gaussian(grid, R1, sig, images=1) - _periodic_gaussian(grid, R2, sig, images=1)
    v = grid.poisson(rho)
    xs = grid.coords()[0]
    errs = []
    for i in (16, 20, 22, 26, 28, 32):
        r = np.array([xs[i], c, c])
        d1 = np.linalg.norm(r - R1)
        d2 = np.linalg.norm(r - R2)
        f = lambda d: erf(d / (math.sqrt(2) * sig)) / d if d > 1e-12 else math.sqrt(2 / math.pi) / sig
        ref = f(d1) - f(d2)
        errs.append(abs(v[i, 24, 24] - ref) / max(abs(ref), 1e-3))
    # image-dipole fields reach ~2 % at the outer points; a wrong 4 pi or sign
    # would be off by >= 50 %
    assert max(errs) < 3e-2


def test_poisson_kzero_removed_and_linear():
    grid = Grid((12, 10, 8), 0.6)
    rng = np.random.default_rng(1)
    a = rng.standard_normal(grid.shape)
    b = rng.standard_normal(grid.shape)
    va, vb = grid.poisson(a), grid.poisson(b)
    assert abs(va.mean()) < 1e-13
    assert np.allclose(grid.poisson(2 * a - 3 * b), 2 * va - 3 * vb, atol=1e-12)
    # symmetric positive semidefinite: <a|v b> = <b|v a>, <a|v a> >= 0
    assert abs(np.sum(a * vb) - np.sum(b * va)) < 1e-10 * np.sum(np.abs(a * vb))
    assert np.sum(a * va) > 0
    # a constant density has zero potential
    assert np.abs(grid.poisson(np.ones(grid.shape))).max() < 1e-13


def test_kinetic_plane_wave_exact():
    """P2: a grid plane wave is an exact eigenvector of the kinetic step."""
    grid = Grid((12, 16, 10), 0.45)
    xs = grid.coords()
    m = (2, -3, 4)
    k = [2 * math.pi * m[a] / (grid.shape[a] * grid.h) for a in range(3)]
    pw = np.exp(1j * (k[0] * xs[0][:, None, None] + k[1] * xs[1][None, :, None]
                      + k[2] * xs[2][None, None, :]))
    dt = 0.37
    out = grid.kinetic_propagator(pw, dt)
    expect = np.exp(-0.5j * dt * sum(kk ** 2 for kk in k)) * pw
    assert np.abs(out - expect).max() < 1e-13
    # -1/2 Laplacian eigenvalue
    assert np.abs(grid.kinetic(pw) - 0.5 * sum(kk ** 2 for kk in k) * pw).max() < 1e-12


def test_kinetic_gaussian_spreading_closed_form():
    """P2: free Gaussian wavepacket, textbook closed form
    psi(x,t) ~ (1 + i t/s^2)^(-1/2) exp(-x^2 / (2 s^2 (1 + i t/s^2))) per axis."""
    n, h = 96, 0.25   # box 24: periodic images below 1e-11
    grid = Grid((n, n, n), h)
    c = n * h / 2
    s = 1.0
    xs = grid.coords()[0] - c

    def packet(t):
        z = 1 + 1j * t / s ** 2
        f = z ** -0.5 * np.exp(-xs ** 2 / (2 * s ** 2 * z))
        return f[:, None, None] * f[None, :, None] * f[None, None, :]

    psi0 = packet(0.0)
    t = 1.3
    out = psi0
    for _ in range(5):
        out = grid.kinetic_propagator(out, t / 5)
    assert np.abs(out - packet(t)).max() < 1e-10
    # unitarity
    assert abs(np.real(grid.dot(out, out)) - np.real(grid.dot(psi0, psi0))) < 1e-12
