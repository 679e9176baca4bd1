"""GPU Tamm-Dancoff matrix and lowest excitons against the FP64 oracle
(same inputs and signs): A element by element, excitons to 1 meV in mixed
precision, and the device Lanczos against a dense eigensolve of the same A."""
import numpy as np
import pytest

from paper_2205_06690_amd import inputs
from oracle.grid import Grid
from oracle import bse as obse
from gpu_util import say, system, oracle_w, gpu_system

pytestmark = pytest.mark.gpu
MEV = 1e-3 / inputs.HARTREE_EV


@pytest.fixture(scope="module")
def tiny_a():
    spec, sysd = system("tiny24")
    pairs = inputs.ij_pairs(spec)
    w, _ = oracle_w(spec, sysd, pairs)
    grid = Grid(spec.shape, spec.h)
    phi = sysd["phi"].reshape((-1,) + spec.shape)
    v0 = spec.n_occ - spec.n_o
    rel_pairs = [(i - v0, j - v0) for i, j in pairs]
    wf = obse.w_stack(spec.n_o, rel_pairs, w)
    phv = phi[v0:spec.n_occ]
    phc = phi[spec.n_occ:spec.n_occ + spec.n_c]
    eps = sysd["eps"]
    A = obse.build_a(grid, phv, phc, eps[v0:spec.n_occ], eps[spec.n_occ:spec.n_occ + spec.n_c], wf)
    f0 = obse.dipoles(grid, phv, phc)
    return spec, sysd, A, f0


@pytest.mark.parametrize("precision,tol_a,tol_w", [(0, 1e-11, 1e-11), (1, 2e-6, MEV)])
def test_tiny24_build_a_and_excitons(tiny_a, precision, tol_a, tol_w):
    spec, sysd, A_o, f0 = tiny_a
    s = gpu_system(spec, sysd, precision, max_batch=3)
    A = s.build_a(spec.n_o, spec.n_c)
    err_a = np.abs(A - A_o).max()
    say(f"prec {precision}: max|dA| {err_a:.3e}  max|A| {np.abs(A_o).max():.3e}")
    assert err_a < tol_a
    n_exc = 6
    om, d2 = s.spectrum(n_exc)
    om_o, d2_o = obse.excitons(A_o, f0, n_exc)
    say(f"prec {precision}: max|dOmega| {np.abs(om - om_o).max():.3e} Ha")
    assert np.abs(om - om_o).max() < tol_w
    assert np.allclose(d2.sum(1), d2_o.sum(1), rtol=1e-3, atol=1e-8)
    # Lanczos on the device equals a dense eigensolve of the same matrix
    w_dense = np.linalg.eigvalsh(A)[:n_exc]
    assert np.abs(om - w_dense).max() < 1e-10
    # absorption on a grid (Eq. 7 with Gaussian deltas)
    wg = np.linspace(om.min() - 0.05, om.max() + 0.05, 200)
    om2, d22, sg = s.spectrum(n_exc, wg, 0.003)
    assert np.allclose(sg, obse.absorption(om2, d22, wg, 0.003), rtol=1e-10, atol=1e-14)


def test_build_a_symmetric_and_errors(tiny_a):
    from paper_2205_06690_amd import bse
    spec, sysd, A_o, f0 = tiny_a
    s = gpu_system(spec, sysd, 1, max_batch=3)
    with pytest.raises(bse.BseError) as e:
        s.spectrum(3)
    assert e.value.code == bse.BSE_ERR_STATE
    with pytest.raises(bse.BseError) as e:
        s.build_a(spec.n_o, 100)
    assert e.value.code == bse.BSE_ERR_ARG
    A = s.build_a(spec.n_o, spec.n_c)
    assert np.array_equal(A, A.T)
