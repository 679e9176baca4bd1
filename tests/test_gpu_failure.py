"""Failure handling of the W-action (the checks the cleaning steps of Eq. 15
make possible), forced from the host through bse_inject_fault so that every
kernel still runs to its normal end:

* a NaN in one conduction orbital fails exactly the pairs that contain it
  (status BSE_ERR_NUMERIC, NaN rows) while the pairs packed with them in the
  same Poisson transforms finish and equal a clean run;
* a finite change of the unperturbed set's norm trips the norm check of the
  cleaning steps and fails every pair of the batch;
* bse_build_A reports BSE_ERR_NUMERIC for a non-finite A;
* the device variant NaN-fills the failed rows in both output types, and
  rejects an index out of range without writing anything.
"""
import numpy as np
import pytest

from gpu_util import say, small_spec, gpu_system, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    from paper_2205_06690_amd import inputs
    spec = small_spec(n=16, n_occ=6, n_o=2, n_c=3, n_steps=40)
    sysd = inputs.make_system(spec)
    pairs = inputs.ia_pairs(spec)           # (4,6) (4,7) (4,8) (5,6) (5,7) (5,8)
    return spec, sysd, pairs


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_nan_in_one_orbital_fails_only_its_pairs(setup, precision):
    from paper_2205_06690_amd import bse
    spec, sysd, pairs = setup
    prec = bse.BSE_MIXED if precision == "mixed" else bse.BSE_FP64
    s = gpu_system(spec, sysd, prec, max_batch=len(pairs))
    w_clean, st0 = s.apply_w(pairs, return_status=True)
    assert np.all(st0 == 0) and np.all(np.isfinite(w_clean))
    bad_orb = spec.n_occ + 1
    s.inject_fault(bad_orb, 123, float("nan"))
    w, st = s.apply_w(pairs, return_status=True)
    bad = np.array([bad_orb in p for p in pairs])
    say(f"{precision}: statuses {st.tolist()}, bad pairs {np.flatnonzero(bad).tolist()}")
    assert np.all(st[bad] == bse.BSE_ERR_NUMERIC)
    assert np.all(st[~bad] == 0)
    assert np.all(np.isnan(w[bad]))
    assert np.all(np.isfinite(w[~bad]))
    # the good pairs, two of them packed with a failed one, equal the clean
    # run up to the rounding of the shared transforms
    e = rel(w[~bad], w_clean[~bad]).max()
    say(f"{precision}: good pairs vs clean run {e:.2e}")
    assert e < (1e-5 if precision == "mixed" else 1e-12)
    with pytest.raises(bse.BseError) as ex:
        s.apply_w(pairs)
    assert ex.value.code == bse.BSE_ERR_NUMERIC
    # set_orbitals restores the clean state
    s.set_orbitals(sysd["phi"], sysd["eps"])
    w2, st2 = s.apply_w(pairs, return_status=True)
    assert np.all(st2 == 0) and rel(w2, w_clean).max() < 1e-12
    s.close()



@pytest.mark.timeout(300)
def test_nan_at_the_paper_grid_fails_only_its_pairs():
    """The same at 112^3 in mixed precision, where the y and z factors of the
    propagation run as one pass over whole planes with the lines in
    registers: three pairs, so that one packed Poisson field holds a failed
    density with a good one and the other a failed density alone; the NaN
    sits at the centre of the box, where the orbital is large, so that the
    failed pair's sanitised source differs from the clean one."""
    import dataclasses
    from paper_2205_06690_amd import bse, inputs
    spec = dataclasses.replace(inputs.CONFIGS["paper112"], n_steps=20)
    sysd = inputs.make_system(spec)
    bad_orb = spec.n_occ + 1
    pairs = np.array([(spec.n_occ - 2, bad_orb), (spec.n_occ - 1, bad_orb + 1), (spec.n_occ - 1, bad_orb)],
                     dtype=np.int32)
    s = gpu_system(spec, sysd, bse.BSE_MIXED, max_batch=len(pairs))
    w_clean, st0 = s.apply_w(pairs, return_status=True)
    assert np.all(st0 == 0) and np.all(np.isfinite(w_clean))
    c = spec.n // 2
    s.inject_fault(bad_orb, (c * spec.n + c) * spec.n + c, float("nan"))
    w, st = s.apply_w(pairs, return_status=True)
    bad = np.array([bad_orb in p for p in pairs])
    say(f"112^3: statuses {st.tolist()}, bad pairs {np.flatnonzero(bad).tolist()}")
    assert np.all(st[bad] == bse.BSE_ERR_NUMERIC)
    assert np.all(st[~bad] == 0)
    assert np.all(np.isnan(w[bad]))
    e = rel(w[~bad], w_clean[~bad]).max()
    say(f"112^3: good pair vs clean run {e:.2e}")
    assert e < 1e-5
    s.close()


def test_unperturbed_norm_drift_fails_every_pair(setup):
    from paper_2205_06690_amd import bse
    spec, sysd, pairs = setup
    s = gpu_system(spec, sysd, bse.BSE_MIXED, max_batch=3)
    # a finite value ten times the orbital's scale: nothing is NaN, only
    # the norm of the unperturbed orbital is off
    s.inject_fault(1, 77, 3.0, unperturbed=True)
    w, st = s.apply_w(pairs, return_status=True)
    say(f"norm drift: statuses {st.tolist()}")
    assert np.all(st == bse.BSE_ERR_NUMERIC)
    assert np.all(np.isnan(w))
    s.close()


def test_build_a_reports_non_finite_a(setup):
    from paper_2205_06690_amd import bse
    spec, sysd, _ = setup
    s = gpu_system(spec, sysd, bse.BSE_MIXED, max_batch=3)
    A0 = s.build_a(spec.n_o, spec.n_c)
    assert np.all(np.isfinite(A0))
    s.inject_fault(spec.n_occ + 2, 5, float("nan"))    # a conduction orbital: exchange and direct terms
    with pytest.raises(bse.BseError) as ex:
        s.build_a(spec.n_o, spec.n_c)
    assert ex.value.code == bse.BSE_ERR_NUMERIC
    with pytest.raises(bse.BseError) as ex2:
        s.spectrum(2)
    assert ex2.value.code == bse.BSE_ERR_STATE
    # a valence orbital: W_ij itself fails
    s.set_orbitals(sysd["phi"], sysd["eps"])
    s.inject_fault(spec.n_occ - 1, 9, float("inf"))
    with pytest.raises(bse.BseError) as ex3:
        s.build_a(spec.n_o, spec.n_c)
    assert ex3.value.code == bse.BSE_ERR_NUMERIC
    s.close()


def test_device_variant_fills_failed_rows_in_both_types(setup):
    import torch
    from paper_2205_06690_amd import bse
    spec, sysd, pairs = setup
    s = gpu_system(spec, sysd, bse.BSE_MIXED, max_batch=len(pairs))
    pq = torch.from_numpy(np.ascontiguousarray(pairs, dtype=np.int32)).cuda()
    w64 = torch.zeros((len(pairs), spec.ng), dtype=torch.float64, device="cuda")
    w32 = torch.zeros((len(pairs), spec.ng), dtype=torch.float32, device="cuda")
    s.apply_w_device(pq, w64)
    s.apply_w_device(pq, w32)
    torch.cuda.synchronize()
    a64, a32 = w64.cpu().numpy(), w32.cpu().numpy().astype(np.float64)
    # the FP32 output is the FP64 sum rounded once
    assert np.array_equal(a32, a64.astype(np.float32).astype(np.float64))
    w_host = s.apply_w(pairs)
    assert np.array_equal(w_host, a64)
    bad_orb = spec.n_occ
    s.inject_fault(bad_orb, 0, float("nan"))
    s.apply_w_device(pq, w64)
    s.apply_w_device(pq, w32)
    torch.cuda.synchronize()
    bad = np.array([bad_orb in p for p in pairs])
    b64, b32 = w64.cpu().numpy(), w32.cpu().numpy()
    assert np.all(np.isnan(b64[bad])) and np.all(np.isnan(b32[bad]))
    assert np.all(np.isfinite(b64[~bad])) and np.all(np.isfinite(b32[~bad]))
    # an index out of range writes nothing
    w64.fill_(7.0)
    bad_pq = pq.clone()
    bad_pq[2, 1] = spec.n_orb
    with pytest.raises(bse.BseError) as ex:
        s.apply_w_device(bad_pq, w64)
    assert ex.value.code == bse.BSE_ERR_ARG
    torch.cuda.synchronize()
    assert bool(torch.all(w64 == 7.0))
    s.close()
