"""GPU W-action against the FP64 oracle on the same inputs and signs
(element-wise over the whole grid).  FP64 mode must agree to round-off,
mixed precision (FP32 propagation) to the 1e-3 relative bound on W."""
import numpy as np
import pytest

from paper_2205_06690_amd import inputs
from gpu_util import say, system, small_spec, oracle_w, gpu_system, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tiny():
    spec, sysd = system("tiny24")
    pairs = np.concatenate([inputs.ij_pairs(spec), inputs.ia_pairs(spec)])
    say(f"oracle tiny24: {len(pairs)} pairs")
    w, wp = oracle_w(spec, sysd, pairs)
    return spec, sysd, pairs, w.reshape(len(pairs), -1), wp.reshape(len(pairs), -1)


def test_tiny24_fp64(tiny):
    from paper_2205_06690_amd import bse
    spec, sysd, pairs, w_o, wp_o = tiny
    say("gpu tiny24 fp64")
    s = gpu_system(spec, sysd, bse.BSE_FP64, max_batch=4)
    w, wp = s.apply_w(pairs, want_wpol=True)
    say("fp64 rel W", rel(w, w_o).max(), "rel Wpol", rel(wp, wp_o).max())
    assert rel(w, w_o).max() < 1e-10
    assert rel(wp, wp_o).max() < 1e-8


def test_tiny24_mixed(tiny):
    from paper_2205_06690_amd import bse
    spec, sysd, pairs, w_o, wp_o = tiny
    say("gpu tiny24 mixed")
    s = gpu_system(spec, sysd, bse.BSE_MIXED, max_batch=5)
    w, wp = s.apply_w(pairs, want_wpol=True)
    say("mixed rel W", rel(w, w_o).max(), "rel Wpol", rel(wp, wp_o).max())
    assert rel(w, w_o).max() < 1e-3
    assert rel(wp, wp_o).max() < 1e-2


@pytest.mark.parametrize("precision", [0, 1])
def test_small16_deterministic(precision):
    """Deterministic mode (all occupied orbitals propagated) on a 16^3 grid."""
    spec = small_spec(n_stoch=0)
    sysd = inputs.make_system(spec)
    pairs = np.array([[4, 5], [5, 5], [3, 6]], dtype=np.int32)
    w_o, wp_o = oracle_w(spec, sysd, pairs, n_stoch=0)
    s = gpu_system(spec, sysd, precision, max_batch=2, n_stoch=0)
    w, wp = s.apply_w(pairs, want_wpol=True)
    w_o, wp_o = w_o.reshape(3, -1), wp_o.reshape(3, -1)
    say("det16 prec", precision, "rel W", rel(w, w_o).max(), "rel Wpol", rel(wp, wp_o).max())
    tol = 1e-10 if precision == 0 else 1e-3
    assert rel(w, w_o).max() < tol
