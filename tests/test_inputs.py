"""Input generator: H0 eigensolver pins, sign generator test vector, wells."""
import math

import numpy as np

from paper_2205_06690_amd import inputs


def test_splitmix64_published_vector():
    """SplitMix64 seeded with 1234567: the first outputs of the published
    reference generator."""
    got = [inputs.splitmix64_draw(1234567, k) for k in range(5)]
    assert got == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                   4593380528125082431, 16408922859458223821]


def test_signs_balanced_and_deterministic():
    xi = inputs.stochastic_signs(9, 10, 400)
    assert xi.dtype == np.int8 and set(np.unique(xi)) == {-1, 1}
    assert abs(xi.mean()) < 0.05
    assert np.array_equal(xi, inputs.stochastic_signs(9, 10, 400))
    assert not np.array_equal(xi, inputs.stochastic_signs(10, 10, 400))


def test_free_particle_spectrum():
    """P3: V = 0 gives exactly the grid plane-wave energies k^2/2."""
    n, h = 10, 0.6
    v = np.zeros((n, n, n))
    phi, eps = inputs.eigensolve(v, h, 20)
    k = 2 * math.pi * np.fft.fftfreq(n, d=h)
    e = np.sort((k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2).ravel() / 2)
    assert np.allclose(eps, e[:20], atol=1e-10)


def test_chefsi_matches_dense():
    """P3: the iterative solver (grid above the dense limit) agrees with the
    dense eigendecomposition and returns orthonormal residual-small states."""
    spec = inputs.SystemSpec(n=14, h=0.6, n_wells=4, seed=21, n_occ=6, n_o=2, n_c=2)
    v = inputs.make_vext(spec)
    phi, eps = inputs.eigensolve(v, spec.h, 8, tol=1e-9)
    H = inputs._H0(v, spec.h)
    Hd = H(np.eye(v.size))
    w = np.linalg.eigvalsh(0.5 * (Hd + Hd.T))
    assert np.allclose(eps, w[:8], atol=1e-10)
    X = phi * math.sqrt(spec.h ** 3)
    assert np.abs(X @ X.T - np.eye(8)).max() < 1e-10
    assert np.abs(H(X) - eps[:, None] * X).max() < 1e-8


def test_wells_recipe():
    spec = inputs.CONFIGS["tiny24"]
    U, w, R = inputs.well_params(spec)
    assert len(U) == 8 and U.min() >= 1 and U.max() <= 3
    assert w.min() >= 0.8 and w.max() <= 1.5
    assert R.min() >= 0.2 * spec.box and R.max() <= 0.8 * spec.box
    v = inputs.make_vext(spec)
    assert v.shape == (24, 24, 24) and v.max() <= 0 and v.min() < -1.0
    spec3 = inputs.CONFIGS["paper112"]
    U, w, R = inputs.well_params(spec3)
    c = spec3.box / 2
    ring = np.hypot(R[:120, 0] - c, R[:120, 1] - c)
    assert np.allclose(ring, 9.0) and np.abs(R[:120, 2] - c).max() <= 1.3
    assert np.linalg.norm(R[120:] - c, axis=1).max() <= 4.0
