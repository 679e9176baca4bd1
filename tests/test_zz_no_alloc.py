"""The allocation-free Chebyshev spectrum against bse_chebyshev_spectrum:
two calls in a row on one GPU (the second with a smaller A, fewer moments
and fewer frequencies, and a given interval), each equal to the allocating
entry point bit for bit; a request above the scratch limit is refused
before any work."""
import numpy as np
import pytest

from gpu_util import say, small_spec, gpu_system

pytestmark = pytest.mark.gpu


def _system(n_o, n_c, seed):
    from paper_2205_06690_amd import inputs, bse
    spec = small_spec(n=16, h=0.6, wells=5, seed=seed, n_occ=6, n_o=n_o, n_c=n_c, n_steps=20)
    sysd = inputs.make_system(spec)
    s = gpu_system(spec, sysd, bse.BSE_FP64, max_batch=8)
    s.build_a(n_o, n_c)
    return s


def test_noalloc_chebyshev_equals_allocating_entry_twice():
    from paper_2205_06690_amd import bse
    s1 = _system(3, 4, 7)        # A of 12 x 12
    s2 = _system(2, 3, 8)        # A of 6 x 6
    sig = 0.05
    calls = [(s1, 400, np.linspace(-0.5, 2.0, 300), None),
             (s2, 100, np.linspace(-0.2, 1.0, 50), "given")]
    for k, (s, n_mom, wg, how) in enumerate(calls):
        bounds = None
        if how == "given":
            _, _, bo = s.chebyshev_spectrum(2, None)
            bounds = (bo[0] - 0.1, bo[1] + 0.1)
        sg_a, res_a, bo_a = s.chebyshev_spectrum(n_mom, wg, sig, bounds=bounds)
        sg_n, res_n, bo_n = s.chebyshev_spectrum_noalloc(n_mom, wg, sig, bounds=bounds)
        say(f"no-alloc call {k + 1}: n_mom {n_mom}, n_w {wg.size}, "
            f"max|d sigma| {np.abs(sg_n - sg_a).max():.1e}, max|d R| {np.abs(res_n - res_a).max():.1e}")
        assert np.array_equal(bo_n, bo_a)
        assert np.array_equal(res_n, res_a)
        assert np.array_equal(sg_n, sg_a)
        # residues only (no frequency grid)
        _, r2, _ = s.chebyshev_spectrum_noalloc(n_mom, None, sig, bounds=bounds)
        assert np.array_equal(r2, res_a)
    with pytest.raises(bse.BseError) as e:
        s2.chebyshev_spectrum_noalloc(20_000_000, None, sig)
    assert e.value.code == bse.BSE_ERR_ARG
    s1.close()
    s2.close()
