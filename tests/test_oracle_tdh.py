"""Pins of the oracle's TD-Hartree action of W (Eqs. 10-15) against closed
forms (sum over states, Casida-type linear response, the damped time
integrals of Eq. 13 in closed form), exact identities (Hadamard signs,
linearity, symmetry), the finite-alpha scheme and the stochastic 1/sqrt(L)
law.  The closed forms integrate the Gaussian damping exactly in continuous
time; none of them takes the oracle's quadrature weights."""
import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import dawsn, erf, wofz

from oracle.grid import Grid
from oracle import tdh
from paper_2205_06690_amd import inputs


def tiny_system(n=8, h=0.7, wells=3, seed=5, n_occ=4):
    spec = inputs.SystemSpec(n=n, h=h, n_wells=wells, seed=seed, n_occ=n_occ, n_o=2, n_c=2)
    v = inputs.make_vext(spec)
    phi, eps = inputs.eigensolve(v, h, n ** 3)      # dense: every state
    return Grid(v.shape, h), v, phi.reshape((-1,) + v.shape), eps


def damped_integral(T, gamma):
    """int_0^T exp(-gamma^2 t^2 / 2) dt = sqrt(pi/2)/gamma erf(gamma T/sqrt 2)."""
    return math.sqrt(math.pi / 2.0) / gamma * math.erf(gamma * T / math.sqrt(2.0))


def damped_sine_integral(om, T, gamma):
    """int_0^T exp(-a t^2) sin(om t) dt, a = gamma^2/2, in closed form.

    Completing the square, -a t^2 + i om t = -a (t - i x/sqrt a)^2 - x^2 with
    x = om/(2 sqrt a), turns the integral into the imaginary part of an error
    function of complex argument.  Written with Dawson's function F (the
    T -> infinity value, F(x)/sqrt a) and the Faddeeva function
    w(z) = exp(-z^2) erfc(-i z) for the tail beyond T:
      I = F(x)/sqrt(a) - sqrt(pi)/(2 sqrt a) Im[exp(-a T^2 + i om T) w(i z)],
    z = sqrt(a) T - i x.  Accepts an array of om."""
    om = np.asarray(om, dtype=np.float64)
    a = 0.5 * gamma * gamma
    sa = math.sqrt(a)
    x = om / (2.0 * sa)
    z = sa * T - 1j * x
    tail = np.imag(np.exp(-a * T * T + 1j * om * T) * wofz(1j * z))
    return dawsn(x) / sa - math.sqrt(math.pi) / (2.0 * sa) * tail


def chi0_closed_form(grid, phi, eps, n_occ, q, T, gamma):
    """Independent-particle response, summed over every grid eigenstate:
    v[-4 sum_{s occ, a virt} F(e_a - e_s) <phi_s phi_a|q> phi_s phi_a],
    F(W) = int_0^T exp(-gamma^2 t^2/2) sin(W t) dt (continuous time)."""
    acc = np.zeros(grid.shape)
    for s in range(n_occ):
        rho = phi[s][None] * phi[n_occ:]                       # [n_virt, ...]
        qs = np.sum(rho * q[None], axis=(1, 2, 3)) * grid.dv
        F = damped_sine_integral(eps[n_occ:] - eps[s], T, gamma)
        acc += -4.0 * np.tensordot(F * qs, rho, axes=1)
    return grid.poisson(acc)


def rpa_closed_form(grid, phi, eps, n_occ, q, T, gamma):
    """Linear TD-Hartree response in the transition space (s occ, a virt):
    x'' = -D^1/2 M D^1/2 ... with M = D^1/2 (D + 4K) D^1/2,
    K_{sa,tb} = (phi_s phi_a | v | phi_t phi_b); x(0) = 0, x'(0) = -D q_sa;
    density change 4 sum x_sa phi_s phi_a; W^pol = v[int_0^T exp(-gamma^2
    t^2/2) dn(t) dt] with the damped integral of each normal mode in closed
    form."""
    nv = phi.shape[0] - n_occ
    R = (phi[:n_occ, None] * phi[None, n_occ:]).reshape(n_occ * nv, -1)
    D = (eps[None, n_occ:] - eps[:n_occ, None]).reshape(-1)
    VR = grid.poisson(R.reshape((-1,) + grid.shape)).reshape(R.shape[0], -1)
    K = (R @ VR.T) * grid.dv
    qv = (R @ q.reshape(-1)) * grid.dv
    sD = np.sqrt(D)
    M = sD[:, None] * (np.diag(D) + 4.0 * K) * sD[None, :]
    om2, F = np.linalg.eigh(0.5 * (M + M.T))
    om = np.sqrt(om2)
    Ft = damped_sine_integral(om, T, gamma)
    X = -sD * (F @ ((Ft / om) * (F.T @ (sD * qv))))
    return grid.poisson((4.0 * X @ R).reshape(grid.shape))


def test_damped_sine_closed_form_against_quadrature():
    """The closed form used by the pins equals adaptive quadrature of the
    integrand, and tends to Dawson's function, sqrt(2)/gamma F(om/(sqrt 2
    gamma)), once the damping has decayed by T."""
    for om, T, g in [(0.3, 10.0, 0.1), (2.0, 10.0, 0.1), (5.0, 30.0, 0.143), (0.05, 5.0, 0.8),
                     (12.0, 10.0, 0.429)]:
        ref = quad(lambda t: math.exp(-0.5 * g * g * t * t) * math.sin(om * t), 0.0, T,
                   limit=500, epsabs=1e-13, epsrel=1e-12)[0]
        assert abs(damped_sine_integral(om, T, g) - ref) < 1e-11 * max(1.0, abs(ref))
    for om in (0.1, 1.0, 4.0):
        g = 0.5
        inf = math.sqrt(2.0) / g * dawsn(om / (math.sqrt(2.0) * g))
        assert abs(damped_sine_integral(om, 40.0, g) - inf) < 1e-13
    assert abs(damped_integral(10.0, 0.1) - quad(lambda t: math.exp(-0.005 * t * t), 0, 10.0)[0]) < 1e-12


# (gamma, T): the paper's damping truncated at T = 10 (end weight
# exp(-1/2) = 0.61), and the default damping of the workloads (1e-4 at T)
_QUAD_CASES = [(0.1, 10.0), (math.sqrt(2 * math.log(1e4)) / 10.0, 10.0), (0.8, 3.0)]


@pytest.mark.parametrize("gamma,T", _QUAD_CASES)
def test_time_weights_integrate_the_gaussian_damping(gamma, T):
    """Eq. 13's weights summed equal int_0^T exp(-gamma^2 t^2/2) dt =
    sqrt(pi/2)/gamma erf(gamma T/sqrt 2) up to the trapezoid rule's
    Euler-Maclaurin term dt^2/12 (f'(T) - f'(0)) (f'(0) = 0 here): a wrong
    damping exponent misses the integral, a wrong end weight leaves an O(dt)
    error that this leading term does not explain."""
    fpT = -gamma * gamma * T * math.exp(-0.5 * gamma * gamma * T * T)
    exact = damped_integral(T, gamma)
    for n in (100, 200, 400):
        dt = T / n
        err = float(np.sum(tdh.time_weights(n, dt, gamma))) - exact
        lead = dt * dt / 12.0 * fpT
        # the next Euler-Maclaurin term is O(dt^4 gamma^4); 1e-13 covers rounding
        assert abs(err - lead) < 5e-3 * abs(lead) + 1e-13, (n, err, lead)


@pytest.mark.parametrize("gamma,T", _QUAD_CASES)
def test_time_weights_integrate_damped_sines(gamma, T):
    """sum_n w_n sin(om t_n) equals the damped sine integral of each mode in
    closed form up to dt^2/12 (f'(T) - f'(0)), f(t) = exp(-gamma^2 t^2/2)
    sin(om t): the quadrature the time integral of Eq. 13 applies to every
    oscillation of the response."""
    a = 0.5 * gamma * gamma
    for om in (0.05, 0.7, 2.5):
        fp0 = om
        fpT = math.exp(-a * T * T) * (om * math.cos(om * T) - 2 * a * T * math.sin(om * T))
        exact = float(damped_sine_integral(om, T, gamma))
        for n in (200, 400, 800):
            dt = T / n
            t = np.arange(n + 1) * dt
            err = float(tdh.time_weights(n, dt, gamma) @ np.sin(om * t)) - exact
            lead = dt * dt / 12.0 * (fpT - fp0)
            assert abs(err - lead) < 2e-2 * abs(lead) + 1e-13, (om, n, err, lead)


def test_time_weights_small_case_by_hand():
    """N = 2, dt = 0.5, gamma = 1: weights (1/2, e^{-1/8}, e^{-1/2}/2) dt."""
    w = tdh.time_weights(2, 0.5, 1.0)
    assert np.allclose(w, [0.25, 0.5 * math.exp(-0.125), 0.25 * math.exp(-0.5)], rtol=1e-15, atol=0)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def sys4():
    return tiny_system(n_occ=4)


def _run(grid, v, phi, n_occ, q, dt, T, gamma=None, **kw):
    n = int(round(T / dt))
    gamma = math.sqrt(2 * math.log(1e4)) / T if gamma is None else gamma
    wp = tdh.w_pol(grid, v, phi[:n_occ], phi[:n_occ], q[None], dt=dt, n_steps=n,
                   gamma=gamma, **kw)[0]
    return wp, T, gamma


@pytest.mark.parametrize("clean_every,gamma", [(0, None), (10, None), (10, 0.1)])
def test_chi0_matches_sum_over_states(sys4, clean_every, gamma):
    """P4: without Hartree feedback the propagated response equals the
    sum-over-states form integrated in continuous time, with an O(dt^2)
    error from the split operator and the quadrature together.  The
    gamma = 0.1 case (the paper's damping, truncated at T = 5 where the
    weight is still 0.88) makes the end weights of the quadrature count."""
    grid, v, phi, eps = sys4
    q = tdh.source_potential(grid, phi[2], phi[3])
    errs = []
    for dt in (0.1, 0.05, 0.025):
        wp, T, g = _run(grid, v, phi, 4, q, dt, 5.0, gamma=gamma, clean_every=clean_every,
                        feedback=False)
        errs.append(_rel(wp, chi0_closed_form(grid, phi, eps, 4, q, T, g)))
    assert errs[-1] < 2e-3
    assert 3.0 < errs[1] / errs[2] < 5.0          # second order in dt


def test_tdh_matches_casida(sys4):
    """P5: full TD-Hartree (feedback on, deterministic, cleaned every 10
    steps) equals the Casida-type transition-space solution to O(dt^2)."""
    grid, v, phi, eps = sys4
    q = tdh.source_potential(grid, phi[1], phi[3])
    errs = []
    for dt in (0.1, 0.05, 0.025):
        wp, T, g = _run(grid, v, phi, 4, q, dt, 5.0, clean_every=10)
        errs.append(_rel(wp, rpa_closed_form(grid, phi, eps, 4, q, T, g)))
    assert errs[-1] < 2e-3
    assert 3.0 < errs[1] / errs[2] < 5.0
    # the feedback matters: the independent-particle form is far away
    wp0, _, _ = _run(grid, v, phi, 4, q, 0.025, 5.0, clean_every=10, feedback=False)
    assert _rel(wp0, wp) > 20 * errs[-1]


def test_hadamard_signs_equal_deterministic():
    """P6: with L = N_occ = 8 and xi = Hadamard rows, sum_l |eta_l><eta_l| = P
    and the stochastic code path reproduces the deterministic one to
    round-off (Q-cleaning is linear; the norm restoration is not, and then
    agrees to the split-operator leakage only)."""
    grid, v, phi, eps = tiny_system(n=8, h=0.7, wells=4, seed=11, n_occ=8)
    occ = phi[:8]
    eta = tdh.stochastic_orbitals(occ, inputs.hadamard_signs(8))
    Pm = np.einsum("lr,ls->rs", eta.reshape(8, -1), eta.reshape(8, -1)) * grid.dv
    P0 = np.einsum("lr,ls->rs", occ.reshape(8, -1), occ.reshape(8, -1)) * grid.dv
    assert np.abs(Pm - P0).max() < 1e-12
    q = tdh.source_potential(grid, phi[6], phi[7])[None]
    kw = dict(dt=0.05, n_steps=100, gamma=0.8, clean_every=10)
    det = tdh.w_pol(grid, v, occ, occ, q, renorm=False, **kw)
    sto = tdh.w_pol(grid, v, occ, eta, q, renorm=False, **kw)
    assert _rel(sto, det) < 1e-12
    det_r = tdh.w_pol(grid, v, occ, occ, q, renorm=True, **kw)
    sto_r = tdh.w_pol(grid, v, occ, eta, q, renorm=True, **kw)
    assert _rel(sto_r, det_r) < 1e-3


def test_linearity_and_symmetry(sys4):
    """P8: W^pol is linear in the source; <rho_kl|W^pol rho_ij> is symmetric
    (to the time-stepping error) and <rho|W^pol rho> < 0."""
    grid, v, phi, eps = sys4
    kw = dict(dt=0.025, n_steps=200, gamma=math.sqrt(2 * math.log(1e4)) / 5.0,
              clean_every=10)
    r1, r2 = phi[2] * phi[3], phi[1] * phi[1]
    q1, q2 = grid.poisson(r1), grid.poisson(r2)
    occ = phi[:4]
    w1, w2, w12 = tdh.w_pol(grid, v, occ, occ, np.stack([q1, q2, 2 * q1 - 0.5 * q2]), **kw)
    assert _rel(w12, 2 * w1 - 0.5 * w2) < 1e-12
    a = np.sum(r2 * w1) * grid.dv
    b = np.sum(r1 * w2) * grid.dv
    assert abs(a - b) < 2e-3 * abs(a)
    assert np.sum(r1 * w1) < 0 and np.sum(r2 * w2) < 0


def _mix_orbitals(phi, n_occ, theta, rng):
    """Orthonormal orbitals that are NOT H0 eigenstates: rotate the occupied
    set into a few virtual states by angle theta."""
    ng = phi[0].size
    X = phi.reshape(phi.shape[0], -1).copy()
    out = X[:n_occ].copy()
    for s in range(n_occ):
        out[s] = math.cos(theta) * X[s] + math.sin(theta) * X[n_occ + s]
    return out.reshape((n_occ,) + phi.shape[1:])


def test_finite_alpha_limit():
    """P9: the linearised scheme is the alpha -> 0 limit of the paper's
    finite-alpha scheme (kick exp(-i alpha q), density difference of the two
    propagated sets, literal re-normalisation).  Orbitals are rotated off
    the eigenstates so that the unperturbed set leaks out of the occupied
    space and the norm restoration matters."""
    grid, v, phi, eps = tiny_system(n_occ=4)
    occ = _mix_orbitals(phi, 4, 0.3, None)
    xi = inputs.stochastic_signs(7, 3, 4)
    eta = tdh.stochastic_orbitals(occ, xi)
    q = grid.poisson(occ[2] * occ[3])[None]
    kw = dict(dt=0.05, n_steps=80, gamma=0.8, clean_every=10)
    lin = tdh.w_pol(grid, v, occ, eta, q, mode="linear", **kw)
    # alpha at the top of the paper's 1e-6..1e-4 range: below ~1e-5 the
    # FP64 density difference n^a - n^0 is dominated by cancellation
    fin = tdh.w_pol(grid, v, occ, eta, q, mode="finite", alpha=1e-4, **kw)
    fin2 = tdh.w_pol(grid, v, occ, eta, q, mode="finite", alpha=2e-4, **kw)
    e1, e2 = _rel(fin, lin), _rel(fin2, lin)
    assert e1 < 1e-5
    assert 1.5 < e2 / e1 < 2.5                     # first order in alpha
    lin_nr = tdh.w_pol(grid, v, occ, eta, q, mode="linear", renorm=False, **kw)
    assert _rel(lin_nr, lin) > 100 * e1            # the restoration is exercised


def test_stochastic_error_scales_as_inverse_sqrt_L():
    """P7: over seeds, the RMS error of the stochastic W^pol against the
    deterministic one falls as L^-1/2."""
    grid, v, phi, eps = tiny_system(n=8, h=0.7, wells=4, seed=3, n_occ=6)
    occ = phi[:6]
    q = grid.poisson(phi[4] * phi[5])[None]
    kw = dict(dt=0.05, n_steps=60, gamma=1.2, clean_every=10)
    det = tdh.w_pol(grid, v, occ, occ, q, **kw)[0]
    Ls = (2, 8, 32)
    rms = []
    for L in Ls:
        e2 = []
        for k in range(24):
            eta = tdh.stochastic_orbitals(occ, inputs.stochastic_signs(100 + k, L, 6))
            e2.append(np.sum((tdh.w_pol(grid, v, occ, eta, q, **kw)[0] - det) ** 2))
        rms.append(math.sqrt(np.mean(e2)) / np.linalg.norm(det))
    slope = np.polyfit(np.log(Ls), np.log(rms), 1)[0]
    assert -0.7 < slope < -0.3, (rms, slope)


def test_unperturbed_kick_has_no_density():
    """At t = 0 a phase kick leaves the density unchanged: with zero steps
    W^pol vanishes identically in the linearised form."""
    grid, v, phi, eps = tiny_system(n_occ=4)
    eta = tdh.stochastic_orbitals(phi[:4], inputs.stochastic_signs(1, 5, 4))
    q = grid.poisson(phi[0] * phi[3])[None]
    wp = tdh.w_pol(grid, v, phi[:4], eta, q, dt=0.05, n_steps=0, gamma=1.0, clean_every=10)
    assert np.abs(wp).max() == 0.0


@pytest.mark.parametrize("perm,flips", [((1, 2, 0), (0,)), ((0, 2, 1), (1, 2)), ((2, 1, 0), ())])
def test_response_commutes_with_cube_symmetries(sys4, perm, flips):
    """An axis permutation or reversal of the periodic cubic grid maps the
    system (V_ext, orbitals, source) onto one with the mapped response:
    W^pol of the mapped system equals the mapped W^pol (the surrogate's
    training data are augmented by exactly these maps)."""
    grid, v, phi, eps = sys4
    n_occ = 4
    q = grid.poisson(phi[1] * phi[2])

    def g(f):                                   # the map on the last three axes
        lead = f.ndim - 3
        f = np.transpose(f, tuple(range(lead)) + tuple(lead + a for a in perm))
        return np.flip(f, axis=tuple(lead + a for a in flips)) if flips else f

    wp, _, _ = _run(grid, v, phi, n_occ, q, 0.05, 2.0, clean_every=10)
    wp_g, _, _ = _run(grid, g(v).copy(), g(phi).copy(), n_occ, g(q).copy(), 0.05, 2.0, clean_every=10)
    assert _rel(wp_g, g(wp)) < 1e-12
