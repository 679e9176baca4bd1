"""The run parameters and energies the paper prints (Results section), as a
fixture under tests/golden/: their printed relations, and the pieces of this
code that take them -- the pair count of the W-actions, the scissors shift
on the diagonal of A (Eq. 1), the default spectral broadening."""
import json
import os

import numpy as np

from paper_2205_06690_amd import inputs
from oracle import bse as obse
from oracle.grid import Grid

G = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_run_parameters.json")))


def v(key):
    return G[key]["value"]


def test_printed_energies_are_consistent():
    # the Delta-GW0 gap is the DFT gap plus its correction; the scissors is
    # the correction combined with -W(k -> 0), which is eps_eff^-1 v_bndry
    assert abs(v("dft_gap_eV") + v("dgw0_correction_eV") - v("dgw0_gap_eV")) < 1e-9
    assert abs(v("dgw0_correction_eV") + v("minus_W_k0_eV") - v("scissors_eV")) < 1e-9
    assert v("core_hours") == v("wall_hours") * v("cores")


def test_pair_count_of_the_w_actions():
    """n_o(n_o+1)/2 valence pairs i <= j: 5050 for n_o = 100 (the printed
    5005 is an arithmetic slip of the same formula)."""
    spec = inputs.SystemSpec(n=16, h=0.5, n_wells=1, seed=0, n_occ=120, n_o=v("n_o"), n_c=1)
    pairs = inputs.ij_pairs(spec)
    n_o = v("n_o")
    assert len(pairs) == n_o * (n_o + 1) // 2 == 5050
    assert len(pairs) != v("w_actions_printed")
    assert np.all(pairs[:, 0] <= pairs[:, 1])
    assert len({tuple(p) for p in pairs}) == len(pairs)


def test_scissors_shift_on_the_diagonal_of_a():
    """With the interaction terms removed, A is diagonal with
    eps_a - eps_i + Delta, Delta the printed scissors (converted to Ha)."""
    grid = Grid((8, 8, 8), 0.5)
    phv = np.zeros((2,) + grid.shape)
    phc = np.zeros((3,) + grid.shape)
    ev, ec = np.array([-0.4, -0.3]), np.array([0.1, 0.2, 0.35])
    w = np.zeros((2, 2) + grid.shape)
    delta = v("scissors_eV") / inputs.HARTREE_EV
    A = obse.build_a(grid, phv, phc, ev, ec, w, scissors=delta)
    ref = (ec[None, :] - ev[:, None] + delta).reshape(-1)
    assert np.allclose(A, np.diag(ref), atol=1e-15)
    assert abs(delta - 0.0382189) < 1e-6


def test_default_broadening_is_the_papers():
    import inspect
    from paper_2205_06690_amd import bse as lib_bse
    sig = inspect.signature(lib_bse.System.chebyshev_spectrum).parameters["sigma"].default
    assert abs(sig * inputs.HARTREE_EV - v("broadening_eV")) < 1e-12
