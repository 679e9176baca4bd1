"""Edge cases of the GPU path on a small system: an empty pair list, pair
order and repeated pairs, a batch of exactly max_batch pairs, the 1 x 1
Tamm-Dancoff matrix, the shortest Chebyshev recursion (two moments) for
the residues and the frequency-resolved states, and the Lanczos either
side of its single-workgroup size limit."""
import numpy as np
import pytest

from paper_2205_06690_amd import inputs
from oracle import bse as obse
from oracle.grid import Grid
from gpu_util import say, small_spec, oracle_w, gpu_system, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small():
    spec = small_spec()
    return spec, inputs.make_system(spec)


@pytest.mark.parametrize("precision", [0, 1])
def test_empty_repeated_and_reversed_pairs(small, precision):
    """No pairs: no work and no error.  rho_ij = rho_ji, so reversed and
    repeated pairs give the same W up to rounding, and a batch of exactly
    max_batch pairs equals the same pairs run one by one.  Not bit for bit:
    the Coulomb solves pack two densities into one complex transform, whose
    butterflies round each density against its partner, and in mixed
    precision the cleaning GEMM's point chunks follow the batch size."""
    spec, sysd = small
    s = gpu_system(spec, sysd, precision, max_batch=3)
    w0 = s.apply_w(np.zeros((0, 2), dtype=np.int32))
    assert w0.shape == (0, spec.ng)
    pairs = np.array([[4, 5], [5, 4], [4, 5]], dtype=np.int32)
    w = s.apply_w(pairs)
    single = np.concatenate([s.apply_w(pairs[k:k + 1]) for k in range(3)])
    e_rep = max(rel(w[1:2], w[:1]).max(), rel(w[2:3], w[:1]).max())
    e_bat = rel(w, single).max()
    say(f"edges prec {precision}: repeated/reversed {e_rep:.2e}, batch vs single {e_bat:.2e}")
    bound = 1e-12 if precision == 0 else 1e-6
    assert e_rep < bound and e_bat < bound
    w_o, _ = oracle_w(spec, sysd, pairs[:1])
    tol = 1e-10 if precision == 0 else 1e-3
    assert rel(w[:1], w_o.reshape(1, -1)).max() < tol


def test_one_by_one_a_and_two_moments(small):
    """n_o = n_c = 1: A is the scalar (e_a - e_i) + 2 (ia|ia) - (aa|W|ii);
    two moments: R_0 = |f0|^2, R_1 = f0 . A~ f0, and the states
    g_0 f0 + g_1 A~ f0, against the oracle on its own A."""
    spec, sysd = small
    s = gpu_system(spec, sysd, 0, max_batch=3)
    A = s.build_a(1, 1)
    grid = Grid(spec.shape, spec.h)
    phi = sysd["phi"].reshape((-1,) + spec.shape)
    i, a_ = spec.n_occ - 1, spec.n_occ
    w_o, _ = oracle_w(spec, sysd, np.array([[i, i]], dtype=np.int32))
    wf = w_o.reshape((1, 1) + spec.shape)
    A_o = obse.build_a(grid, phi[i:i + 1], phi[a_:a_ + 1], sysd["eps"][i:i + 1], sysd["eps"][a_:a_ + 1], wf)
    say(f"1x1 A: gpu {A[0, 0]:.12f} oracle {A_o[0, 0]:.12f}")
    assert A.shape == (1, 1) and abs(A[0, 0] - A_o[0, 0]) < 1e-10
    f0 = obse.dipoles(grid, phi[i:i + 1], phi[a_:a_ + 1])
    # the Lanczos path on one row: the exciton is A itself, its strength |f0|^2
    om1, d21 = s.spectrum(1)
    assert abs(om1[0] - A[0, 0]) < 1e-12 * max(1.0, abs(A[0, 0]))
    assert np.allclose(d21[0], f0[0] ** 2, rtol=1e-10, atol=1e-14)
    lo, hi = A_o[0, 0] - 0.1, A_o[0, 0] + 0.1
    a, b = obse.chebyshev_scale(lo, hi)
    _, R, _ = s.chebyshev_spectrum(2, None, bounds=(lo, hi))
    R_o = obse.chebyshev_residues(A_o, f0, 2, a, b)
    assert np.allclose(R, R_o.T, rtol=1e-10, atol=1e-14)
    wl = np.array([A_o[0, 0] - 0.01, A_o[0, 0]])
    F, dn, _ = s.exciton_states(2, wl, 0.02, bounds=(lo, hi))
    F_o = obse.chebyshev_states(A_o, f0, 2, a, b, wl, 0.02).transpose(0, 2, 1)
    assert np.allclose(F, F_o, rtol=1e-10, atol=1e-14)
    dn_o = obse.exciton_density(phi[i:i + 1], phi[a_:a_ + 1], F_o[1, 0])
    assert np.abs(dn[1, 0] - dn_o).max() < 1e-10 * np.abs(dn_o).max()


@pytest.mark.timeout(400)
@pytest.mark.parametrize("n_o,n_c", [(12, 32), (11, 35), (32, 32)])
def test_lanczos_at_the_single_workgroup_limit(n_o, n_c):
    """A of 384 rows (the largest the single-workgroup Lanczos takes), of
    385 (one past it: the launch-per-operation schedule) and of 1024: both
    schedules give the lowest excitons of a dense eigensolve of the same
    A."""
    spec = small_spec(n=16, h=0.6, wells=5, seed=7, n_occ=n_o, n_o=n_o, n_c=n_c, n_steps=20, n_stoch=4)
    sysd = inputs.make_system(spec)
    s = gpu_system(spec, sysd, 0, max_batch=64)
    A = s.build_a(n_o, n_c)
    assert A.shape == (n_o * n_c, n_o * n_c) and np.array_equal(A, A.T)
    n_exc = 10
    w_dense = np.linalg.eigvalsh(A)[:n_exc]
    om0, d0 = s.spectrum(n_exc)
    s.set_lanczos_path(1)
    om1, d1 = s.spectrum(n_exc)
    s.set_lanczos_path(0)
    scale = max(1.0, np.abs(w_dense).max())
    say(f"n = {n_o * n_c}: Lanczos vs dense {np.abs(om0 - w_dense).max():.2e} / {np.abs(om1 - w_dense).max():.2e}")
    assert np.abs(om0 - w_dense).max() < 1e-9 * scale
    assert np.abs(om1 - w_dense).max() < 1e-9 * scale
    assert np.allclose(d0, d1, rtol=1e-6, atol=1e-12)


@pytest.mark.timeout(300)
def test_launch_order_does_not_change_results():
    """The XCD-grouped workgroup order of the x, y-line and fused y-z passes
    (order 7) gives W bit for bit equal to the plain order (0), on a 64^3
    grid (plane pass) and on the 112^3 grid (fused y-z pass in mixed
    precision, z and y line passes in FP64)."""
    import dataclasses
    from paper_2205_06690_amd import bse, inputs
    cases = [(dataclasses.replace(inputs.CONFIGS["mid64"], n_steps=30), bse.BSE_MIXED),
             (dataclasses.replace(inputs.CONFIGS["paper112"], n_steps=20), bse.BSE_MIXED),
             (dataclasses.replace(inputs.CONFIGS["paper112"], n_steps=20), bse.BSE_FP64)]
    for spec, prec in cases:
        sysd = inputs.make_system(spec)
        pairs = inputs.ij_pairs(spec)[-5:]
        res = []
        for order in (0, 7):
            s = gpu_system(spec, sysd, prec, max_batch=len(pairs))
            s.set_launch_order(order)
            res.append(s.apply_w(pairs))
            s.close()
        say(f"launch order {spec.n}^3 precision {prec}: max|dW| {np.abs(res[0] - res[1]).max():.1e}")
        assert np.array_equal(res[0], res[1])


@pytest.mark.timeout(300)
def test_fused_yz_pass_equals_line_passes():
    """At 112^3 in mixed precision the y and z factors run as one pass over
    whole planes, the 16-point DFTs either as cross-lane butterflies
    (schedule 0) or one vector per lane through a wave's scratch (schedule
    2); the schedule of two line passes (1) computes the same propagation in
    another order of rounding: W of a 21-pair slice over 60 steps agrees to
    FP32 rounding."""
    import dataclasses
    from paper_2205_06690_amd import bse, inputs
    spec = dataclasses.replace(inputs.CONFIGS["paper112"], n_steps=60)
    sysd = inputs.make_system(spec)
    pairs = inputs.ij_pairs(spec)[-21:]
    res = {}
    for sched in (1, 0, 2):
        s = gpu_system(spec, sysd, bse.BSE_MIXED, max_batch=len(pairs))
        s.set_yz_schedule(sched)
        res[sched] = s.apply_w(pairs)
        s.close()
    for sched in (0, 2):
        e = rel(res[sched], res[1]).max()
        say(f"one-pass schedule {sched} vs line passes, 21 pairs x 60 steps: max rel W {e:.2e}")
        assert e < 2e-5

@pytest.mark.timeout(300)
def test_autotune_at_the_paper_grid(tmp_path):
    """At 112^3 in mixed precision the autotuner also picks the one-pass y-z
    kernel's DFT schedule and workgroup order: W over 20 steps stays within
    FP32 rounding of the untuned run (the schedules round differently)."""
    import dataclasses
    from paper_2205_06690_amd import bse, inputs
    spec = dataclasses.replace(inputs.CONFIGS["paper112"], n_steps=20)
    sysd = inputs.make_system(spec)
    pairs = inputs.ij_pairs(spec)[-3:]
    s = gpu_system(spec, sysd, bse.BSE_MIXED, max_batch=len(pairs))
    before = s.apply_w(pairs)
    cache = str(tmp_path / "tune112.txt")
    tc, nt = s.autotune(len(pairs), cache)
    fields = open(cache).read().split()
    say(f"112^3 autotune: x tile {tc}, x order {fields[5]}, y-z schedule {fields[6]}, y-z order {fields[7]}")
    assert tc in (16, 32, 64) and nt == 0 and fields[6] in ("0", "2") and fields[7] in ("0", "1")
    after = s.apply_w(pairs)
    e = rel(after, before).max()
    say(f"112^3 autotuned vs default: max rel W {e:.2e}")
    assert e < 2e-5
    s.close()
