"""Pins of the W(k->0) box-correction oracle against closed forms, brute
force and a library least-squares solve."""
import itertools
import math

import numpy as np
import pytest

from oracle import box
from oracle.grid import Grid
from paper_2205_06690_amd import inputs


def test_boundary_mask_counts_and_brute_force_mean():
    """3 n^2 - 3 n + 1 boundary points; the mean over them equals a loop
    over every point with a zero index."""
    rng = np.random.default_rng(3)
    for n in (2, 3, 5, 8):
        v = rng.standard_normal((n, n, n))
        assert box.boundary_mask(v.shape).sum() == 3 * n * n - 3 * n + 1
        acc, cnt = 0.0, 0
        for i, j, k in itertools.product(range(n), repeat=3):
            if min(i, j, k) == 0:
                acc += v[i, j, k]
                cnt += 1
        assert math.isclose(box.boundary_average(v), acc / cnt - v.mean(), rel_tol=1e-12, abs_tol=1e-14)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_boundary_average_of_a_cosine(axis):
    """cos(2 pi i / n) along one axis: the face across that axis holds 1,
    each slice of the other two faces sums to -1, and the cell mean is 0:
    (n - 1)^2 / (3 n^2 - 3 n + 1)."""
    n = 12
    c = np.cos(2 * np.pi * np.arange(n) / n)
    shp = [1, 1, 1]
    shp[axis] = n
    v = np.broadcast_to(c.reshape(shp), (n, n, n)).copy()
    assert math.isclose(box.boundary_average(v), (n - 1) ** 2 / (3 * n * n - 3 * n + 1), rel_tol=1e-12)


def test_ks_potential_single_mode_closed_form():
    """One orbital phi = sqrt(2/V) cos(k x), k = 2 pi / L: n = (2/V)(1 + cos 2kx)
    and v_H = (2/V) (4 pi / (2k)^2) cos(2kx) exactly (one Fourier mode); with
    a sin partner the density is uniform and v_H vanishes."""
    n, h = 16, 0.5
    grid = Grid((n, n, n), h)
    L = n * h
    V = L ** 3
    k = 2 * np.pi / L
    x = np.arange(n) * h
    cx = np.cos(k * x)[:, None, None] * np.ones((n, n, n))
    sx = np.sin(k * x)[:, None, None] * np.ones((n, n, n))
    phi = np.sqrt(2.0 / V) * np.stack([cx, sx])
    assert np.allclose(grid.dot(phi, phi), 1.0, rtol=1e-12)
    v_ext = np.random.default_rng(1).standard_normal((n, n, n))
    vh = box.ks_potential(grid, v_ext, phi[:1]) - v_ext
    want = (2.0 / V) * (4 * np.pi / (2 * k) ** 2) * np.cos(2 * k * x)[:, None, None]
    assert np.abs(vh - want).max() < 1e-12 * np.abs(want).max()
    assert np.abs(box.ks_potential(grid, v_ext, phi) - v_ext).max() < 1e-13
    # its boundary value: the cosine face formula with amplitude A
    A = (2.0 / V) * (4 * np.pi / (2 * k) ** 2)
    assert math.isclose(box.boundary_average(vh), A * (n - 1) ** 2 / (3 * n * n - 3 * n + 1), rel_tol=1e-10)


def test_occupied_density_holds_two_electrons_per_orbital():
    spec = inputs.CONFIGS["tiny24"]
    sysd = inputs.make_system(spec)
    grid = Grid(spec.shape, spec.h)
    phi = sysd["phi"][:spec.n_occ].reshape((spec.n_occ,) + spec.shape)
    assert math.isclose(box.occupied_density(phi).sum() * grid.dv, 2 * spec.n_occ, rel_tol=1e-9)


def test_fit_recovers_a_planted_slope_and_matches_lstsq():
    rng = np.random.default_rng(7)
    n_box, n_exc = 4, 5
    v = rng.uniform(-0.2, 0.1, n_box)
    c = rng.uniform(0.1, 0.3, n_exc)
    om = c[None, :] + 0.3 * v[:, None]
    e, cc, wk = box.fit_inverse_dielectric(om, v)
    assert math.isclose(e, 0.3, rel_tol=1e-12)
    assert np.allclose(cc, c, rtol=1e-12) and np.allclose(wk, 0.3 * v, rtol=1e-12)
    # with noise: the same parameters as a general least-squares solve of
    # the design matrix [one-hot exciton | v_b]
    om = om + 1e-3 * rng.standard_normal(om.shape)
    e, cc, _ = box.fit_inverse_dielectric(om, v)
    X = np.zeros((n_box * n_exc, n_exc + 1))
    for b in range(n_box):
        for m in range(n_exc):
            X[b * n_exc + m, m] = 1.0
            X[b * n_exc + m, n_exc] = v[b]
    sol = np.linalg.lstsq(X, om.reshape(-1), rcond=None)[0]
    assert math.isclose(e, sol[-1], rel_tol=1e-10) and np.allclose(cc, sol[:-1], rtol=1e-10)
    # a scissors shift of every energy moves the intercepts only
    e2, cc2, _ = box.fit_inverse_dielectric(om + 0.05, v)
    assert math.isclose(e2, e, rel_tol=1e-10) and np.allclose(cc2, cc + 0.05, rtol=1e-12)


def test_fit_rejects_degenerate_inputs():
    with pytest.raises(ValueError):
        box.fit_inverse_dielectric(np.ones((1, 3)), np.ones(1))
    with pytest.raises(ValueError):
        box.fit_inverse_dielectric(np.ones((3, 3)), np.full(3, 0.2))


def test_box_series_places_the_same_molecule():
    """A box series keeps the wells (depths, widths) and moves their centres
    by half the added box length, so the molecule sits at the same offset
    from every box centre; the first box is the original system."""
    spec = inputs.CONFIGS["tiny24"]
    U0, w0, R0 = inputs.well_params(spec)
    for s in inputs.box_series(spec, [24, 28, 32]):
        U, w, R = inputs.well_params(s)
        assert np.array_equal(U, U0) and np.array_equal(w, w0)
        assert np.allclose(R - 0.5 * s.box, R0 - 0.5 * spec.box, rtol=0, atol=1e-12)
    assert np.array_equal(inputs.make_vext(inputs.box_series(spec, [24])[0]), inputs.make_vext(spec))
