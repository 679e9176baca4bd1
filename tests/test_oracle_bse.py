"""Pins of the oracle's Tamm-Dancoff matrix (Eq. 1), dipoles and absorption
(Eq. 7) against closed forms for Gaussian orbitals, whose pair products are
Gaussian charges with analytic periodic Coulomb integrals."""
import math

import numpy as np
import pytest

from oracle.grid import Grid
from oracle import bse

S = 1.2          # orbital width (bohr)
N, H = 60, 0.4   # box 24 bohr: orbital tails at the boundary < 1e-9


def _orbital(grid, R):
    xs = grid.coords()
    box = grid.shape[0] * grid.h
    out = np.zeros(grid.shape)
    nrm = (math.pi * S ** 2) ** -0.75
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            for c in (-1, 0, 1):
                dx = xs[0] - R[0] - a * box
                dy = xs[1] - R[1] - b * box
                dz = xs[2] - R[2] - c * box
                out += nrm * np.exp(-(dx[:, None, None] ** 2 + dy[None, :, None] ** 2
                                      + dz[None, None, :] ** 2) / (2 * S ** 2))
    return out


def _pair(R1, R2):
    """phi_1 phi_2 = Q g_sigma(r - M): charge, centre, width."""
    R1, R2 = np.asarray(R1), np.asarray(R2)
    d2 = np.sum((R1 - R2) ** 2)
    return math.exp(-d2 / (4 * S ** 2)), 0.5 * (R1 + R2), S / math.sqrt(2)


def _coulomb(p1, p2, box):
    """Periodic Coulomb integral of two Gaussian charges, k = 0 removed:
    (1/Omega) sum_{G != 0} 4 pi/G^2 Q1 Q2 exp(-G^2 (s1^2 + s2^2)/2) cos(G.(M1 - M2))."""
    (Q1, M1, s1), (Q2, M2, s2) = p1, p2
    mmax = 28      # exp(-G^2 (s1^2+s2^2)/2) < 1e-14 beyond
    m = np.arange(-mmax, mmax + 1)
    G1 = 2 * math.pi * m / box
    Gx, Gy, Gz = np.meshgrid(G1, G1, G1, indexing="ij")
    G2 = Gx ** 2 + Gy ** 2 + Gz ** 2
    msk = G2 > 0
    d = M1 - M2
    ph = Gx[msk] * d[0] + Gy[msk] * d[1] + Gz[msk] * d[2]
    val = np.sum(4 * math.pi / G2[msk] * np.exp(-G2[msk] * (s1 ** 2 + s2 ** 2) / 2) * np.cos(ph))
    return Q1 * Q2 * val / box ** 3


@pytest.fixture(scope="module")
def gauss():
    grid = Grid((N, N, N), H)
    c = N * H / 2
    Rv = [(c - 0.7, c + 0.2, c), (c + 0.4, c - 0.5, c + 0.6)]
    Rc = [(c + 1.1, c + 0.9, c - 0.4), (c - 0.9, c - 1.0, c + 0.3), (c, c + 1.3, c + 1.0)]
    phv = np.stack([_orbital(grid, R) for R in Rv])
    phc = np.stack([_orbital(grid, R) for R in Rc])
    return grid, Rv, Rc, phv, phc


def test_exchange_closed_form(gauss):
    grid, Rv, Rc, phv, phc = gauss
    X = bse.exchange(grid, phv, phc)
    box = N * H
    nc = len(Rc)
    for i in range(2):
        for a in range(nc):
            for j in range(2):
                for b in range(nc):
                    ref = _coulomb(_pair(Rv[i], Rc[a]), _pair(Rv[j], Rc[b]), box)
                    assert abs(X[i * nc + a, j * nc + b] - ref) < 1e-8 * abs(ref) + 1e-12


def test_direct_and_assembly_with_bare_coulomb(gauss):
    """P10: with W^pol = 0 the direct term is the bare (ab|v|ij) and A is
    diag + 2 (ia|jb) - (ab|v|ij) in the (i, a) row order."""
    grid, Rv, Rc, phv, phc = gauss
    box = N * H
    nc = len(Rc)
    w_full = np.zeros((2, 2) + grid.shape)
    for i in range(2):
        for j in range(2):
            w_full[i, j] = grid.poisson(phv[i] * phv[j])
    D = bse.direct(grid, phc, w_full)
    ev = np.array([-0.5, -0.3])
    ec = np.array([0.1, 0.25, 0.4])
    A = bse.build_a(grid, phv, phc, ev, ec, w_full, scissors=0.05)
    for i in range(2):
        for a in range(nc):
            for j in range(2):
                for b in range(nc):
                    dref = _coulomb(_pair(Rc[a], Rc[b]), _pair(Rv[i], Rv[j]), box)
                    xref = _coulomb(_pair(Rv[i], Rc[a]), _pair(Rv[j], Rc[b]), box)
                    assert abs(D[i * nc + a, j * nc + b] - dref) < 1e-8 * abs(dref) + 1e-12
                    diag = (ec[a] - ev[i] + 0.05) if (i == j and a == b) else 0.0
                    aref = diag + 2 * xref - dref
                    assert abs(A[i * nc + a, j * nc + b] - aref) < 1e-8
    assert np.abs(A - A.T).max() < 1e-12


def test_dipoles_closed_form(gauss):
    grid, Rv, Rc, phv, phc = gauss
    f0 = bse.dipoles(grid, phv, phc)
    c = N * H / 2
    nc = len(Rc)
    for i in range(2):
        for a in range(nc):
            Q, M, _ = _pair(Rv[i], Rc[a])
            assert np.allclose(f0[i * nc + a], Q * (M - c), atol=1e-9)


def test_excitons_uncoupled_and_absorption_sum():
    rng = np.random.default_rng(0)
    d = np.array([0.5, 0.2, 0.9, 0.35])
    f0 = rng.standard_normal((4, 3))
    om, dip2 = bse.excitons(np.diag(d), f0, 3)
    order = np.argsort(d)[:3]
    assert np.allclose(om, d[order])
    assert np.allclose(dip2, f0[order] ** 2)
    # a coupled A: the oscillator strengths of all excitons add up to |f0|^2
    Q, _ = np.linalg.qr(rng.standard_normal((4, 4)))
    A = Q @ np.diag(d) @ Q.T
    om, dip2 = bse.excitons(A, f0, 4)
    assert np.allclose(dip2.sum(axis=0), (f0 ** 2).sum(axis=0))
    # sigma(omega)/omega integrates to the summed strengths
    wg = np.linspace(-1, 3, 40001)
    sig = bse.absorption(om, dip2, wg, 0.02)
    with np.errstate(divide="ignore", invalid="ignore"):
        integ = np.trapezoid(np.where(wg != 0, sig / wg, 0.0), wg)
    assert abs(integ - dip2.sum()) < 1e-6 * dip2.sum()


# --------------------------------------------------------------------------
# Chebyshev spectrum (Eqs. 7-8)
# --------------------------------------------------------------------------
def _sym(n, seed, lo=0.2, hi=1.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.sort(rng.uniform(lo, hi, n))
    A = (Q * lam) @ Q.T
    return 0.5 * (A + A.T), rng.standard_normal((n, 3))


def test_chebyshev_residues_closed_form():
    """R_n = sum_k |<X_k|f0>|^2 cos(n arccos((lambda_k - b)/a)) from the
    eigenpairs; a wrong factor 2, sign or start vector in the recursion
    breaks it."""
    A, f0 = _sym(30, 3)
    a, b = bse.chebyshev_scale(*bse.spectral_bounds(A))
    R = bse.chebyshev_residues(A, f0, 200, a, b)
    w, X = np.linalg.eigh(A)
    p = (X.T @ f0) ** 2
    th = np.arccos((w - b) / a)
    Rc = np.array([(np.cos(n * th)[:, None] * p).sum(axis=0) for n in range(200)])
    assert np.abs(R - Rc).max() < 1e-12 * np.abs(Rc).max()
    assert np.allclose(R[0], (f0 ** 2).sum(axis=0))


def test_chebyshev_absorption_converges_to_eigen_sum():
    """With enough moments the Chebyshev spectrum equals the Gaussian-
    broadened sum over excitons; too few moments leave a visible error."""
    A, f0 = _sym(40, 5)
    a, b = bse.chebyshev_scale(*bse.spectral_bounds(A))
    s = 0.02
    wg = np.linspace(0.1, 1.1, 150)
    w, X = np.linalg.eigh(A)
    ref = bse.absorption(w, (X.T @ f0) ** 2, wg, s)
    errs = []
    for N in (int(a / s), int(8 * a / s)):
        R = bse.chebyshev_residues(A, f0, N, a, b)
        errs.append(np.abs(bse.chebyshev_absorption(R, wg, a, b, s) - ref).max() / np.abs(ref).max())
    assert errs[0] > 1e-3
    assert errs[1] < 1e-10


def test_chebyshev_single_level():
    """A = [[E0]]: sigma(omega) = omega f^2 G(E0 - omega) exactly (the
    interval is widened around the single level)."""
    E0, f = 0.37, 1.3
    A = np.array([[E0]])
    f0 = np.array([[f, 0.0, 0.0]])
    a, b = bse.chebyshev_scale(E0 - 0.2, E0 + 0.2)
    s = 0.01
    wg = np.linspace(0.3, 0.45, 31)
    R = bse.chebyshev_residues(A, f0, 400, a, b)
    g = np.exp(-0.5 * ((wg - E0) / s) ** 2) / (s * math.sqrt(2 * math.pi))
    assert np.abs(bse.chebyshev_absorption(R, wg, a, b, s) - wg * f * f * g).max() < 1e-9 * (wg * f * f * g).max()


def test_gershgorin_bounds_contain_spectrum():
    A, _ = _sym(25, 9, lo=-0.5, hi=2.0)
    lo, hi = bse.spectral_bounds(A)
    w = np.linalg.eigvalsh(A)
    assert lo <= w[0] and w[-1] <= hi


def test_chebyshev_states_equal_gaussian_of_a():
    """Eq. 8 with enough moments is the broadened delta of A applied to
    f0: sum_k G(lambda_k - omega) X_k <X_k|f0> from the eigenpairs; too
    few moments leave a visible error."""
    A, f0 = _sym(30, 7)
    a, b = bse.chebyshev_scale(*bse.spectral_bounds(A))
    s = 0.02
    wg = np.array([0.25, 0.48, 0.61, 0.9])
    w, X = np.linalg.eigh(A)
    G = np.exp(-0.5 * ((w[None, :] - wg[:, None]) / s) ** 2) / (s * math.sqrt(2 * math.pi))
    ref = np.einsum("qk,nk,kp->qnp", G, X, X.T @ f0)
    errs = []
    for n_mom in (int(a / s), int(8 * a / s)):
        F = bse.chebyshev_states(A, f0, n_mom, a, b, wg, s)
        errs.append(np.abs(F - ref).max() / np.abs(ref).max())
    assert errs[0] > 1e-3
    assert errs[1] < 1e-10


def test_chebyshev_states_carry_the_residue_spectrum():
    """<f0|f(omega)> summed over polarisations is sigma(omega)/omega of the
    residue path (Eq. 7), itself pinned to the eigenpairs above."""
    A, f0 = _sym(20, 8)
    a, b = bse.chebyshev_scale(*bse.spectral_bounds(A))
    s, n_mom = 0.03, 400
    wg = np.linspace(0.3, 0.9, 7)
    F = bse.chebyshev_states(A, f0, n_mom, a, b, wg, s)
    R = bse.chebyshev_residues(A, f0, n_mom, a, b)
    sg = bse.chebyshev_absorption(R, wg, a, b, s)
    assert np.allclose(wg * np.einsum("np,qnp->q", f0, F), sg, rtol=1e-11, atol=1e-14)


def test_exciton_density_charge_and_dipole(gauss):
    """For Gaussian orbitals the pair products are Gaussian charges Q_ia at
    M_ia, so the exciton density of F integrates to 2 sum F_ia Q_ia and its
    dipole is 2 sum F_ia Q_ia (M_ia - c) = 2 F.f0; a transposed F, a lost
    factor 2 or a swapped orbital set breaks both."""
    grid, Rv, Rc, phv, phc = gauss
    nc = len(Rc)
    rng = np.random.default_rng(12)
    F = rng.standard_normal(len(Rv) * nc)
    dn = bse.exciton_density(phv, phc, F)
    c = N * H / 2
    q = sum(F[i * nc + a] * _pair(Rv[i], Rc[a])[0] for i in range(len(Rv)) for a in range(nc))
    dip = sum(F[i * nc + a] * _pair(Rv[i], Rc[a])[0] * (_pair(Rv[i], Rc[a])[1] - c)
              for i in range(len(Rv)) for a in range(nc))
    assert abs(np.sum(dn) * grid.dv - 2 * q) < 1e-9
    # the mixed-representation density of f_i = sum_a F_ia phi_a is the same
    f_mixed = np.tensordot(F.reshape(len(Rv), nc), phc, axes=(1, 0))
    assert np.abs(bse.mixed_exciton_density(phv, f_mixed) - dn).max() < 1e-12 * np.abs(dn).max()
    xs = grid.coords()
    for ax in range(3):
        shp = [1, 1, 1]
        shp[ax] = -1
        mom = np.sum(dn * (xs[ax] - c).reshape(shp)) * grid.dv
        assert abs(mom - 2 * dip[ax]) < 1e-9
        assert abs(mom - 2 * F @ bse.dipoles(grid, phv, phc)[:, ax]) < 1e-9


# --------------------------------------------------------------------------
# matrix-free A f in the mixed representation (Eq. 6)
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def mixed_system():
    """Eigenstates of a small well potential on 12^3: 6 occupied (the last 2
    the valence window), 4 conduction, and a symmetric synthetic W_ij stack
    (smooth, negative-definite like a screened interaction)."""
    from paper_2205_06690_amd import inputs
    spec = inputs.SystemSpec(n=12, h=0.7, n_wells=4, seed=11, n_occ=6, n_o=2, n_c=4)
    sysd = inputs.make_system(spec, use_cache=False)
    grid = Grid(spec.shape, spec.h)
    phi = sysd["phi"].reshape((-1,) + spec.shape)
    rng = np.random.default_rng(4)
    x = [np.arange(n) * spec.h for n in spec.shape]
    X, Y, Z = np.meshgrid(*x, indexing="ij")
    w = np.zeros((2, 2) + spec.shape)
    for i in range(2):
        for j in range(i, 2):
            c = rng.uniform(2, 6, 3)
            w[i, j] = w[j, i] = -0.3 * np.exp(-((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2) / 4.0)
    return spec, grid, sysd["v_ext"], phi, sysd["eps"], w


def test_apply_a_mixed_matches_eq1_in_the_conduction_space(mixed_system):
    """For f_j = sum_b c_jb phi_b, <phi_a| (A f)_i> = sum_jb A(ia; jb) c_jb
    with A from the electron-hole assembly of Eq. 1."""
    spec, grid, v, phi, eps, w = mixed_system
    phv, phc = phi[4:6], phi[6:10]
    A = bse.build_a(grid, phv, phc, eps[4:6], eps[6:10], w, scissors=0.01)
    c = np.random.default_rng(2).standard_normal((2, 4))
    f = (c @ phc.reshape(4, -1)).reshape((2,) + spec.shape)
    Af = bse.apply_a_mixed(grid, v, phi[:6], eps[4:6], w, f, scissors=0.01)
    proj = (Af.reshape(2, -1) @ phc.reshape(4, -1).T) * grid.dv                # [i, a]
    assert np.abs(proj.reshape(-1) - A @ c.reshape(-1)).max() < 1e-9


def test_apply_a_mixed_projected_and_symmetric(mixed_system):
    spec, grid, v, phi, eps, w = mixed_system
    rng = np.random.default_rng(7)
    P = phi[:6].reshape(6, -1)

    def q(g):
        g = g.reshape(2, -1)
        return (g - ((g @ P.T) * grid.dv) @ P).reshape((2,) + spec.shape)
    f = q(rng.standard_normal((2,) + spec.shape))
    g = q(rng.standard_normal((2,) + spec.shape))
    Af = bse.apply_a_mixed(grid, v, phi[:6], eps[4:6], w, f)
    Ag = bse.apply_a_mixed(grid, v, phi[:6], eps[4:6], w, g)
    assert np.abs((Af.reshape(2, -1) @ P.T) * grid.dv).max() < 1e-10
    lhs = np.sum(g * Af) * grid.dv
    rhs = np.sum(Ag * f) * grid.dv
    assert abs(lhs - rhs) < 1e-10 * max(abs(lhs), 1.0)


def test_apply_a_mixed_without_interaction(mixed_system):
    """W = 0 and no Hartree term (the density coupling is removed by taking
    a conduction state for one hole only and checking against
    eps_a - eps_j): phi_a is an eigenvector of Q(H0 - eps_j)."""
    spec, grid, v, phi, eps, w = mixed_system
    f = np.zeros((2,) + spec.shape)
    f[1] = phi[7]
    Af = bse.apply_a_mixed(grid, v, phi[:6], eps[4:6], np.zeros_like(w), f)
    # the Hartree term 2 phi_j v[phi_j f_j] is present; remove it explicitly
    dv = grid.poisson(2.0 * phi[5] * phi[7])
    hart = np.stack([dv * phi[4], dv * phi[5]])
    P = phi[:6].reshape(6, -1)
    hart = (hart.reshape(2, -1) - ((hart.reshape(2, -1) @ P.T) * grid.dv) @ P).reshape(hart.shape)
    rest = Af - hart
    assert np.abs(rest[0]).max() < 1e-9
    assert np.abs(rest[1] - (eps[7] - eps[5]) * phi[7]).max() < 1e-7 * np.abs(phi[7]).max()


def test_chebyshev_residues_operator_form_closed_form():
    """The operator form of the recursion against the eigenpair closed form."""
    A, f0 = _sym(20, 13)
    a, b = bse.chebyshev_scale(*bse.spectral_bounds(A))
    R = bse.chebyshev_residues_op(lambda v: A @ v, [f0[:, p] for p in range(3)], 120, a, b,
                                  lambda u, v: float(u @ v))
    w, X = np.linalg.eigh(A)
    p = (X.T @ f0) ** 2
    th = np.arccos((w - b) / a)
    Rc = np.array([(np.cos(n * th)[:, None] * p).sum(axis=0) for n in range(120)])
    assert np.abs(R - Rc).max() < 1e-12 * np.abs(Rc).max()


def test_chebyshev_states_operator_form_equals_matrix_form():
    """The operator recursion of Eq. 8 with A applied as a product equals
    the matrix form, itself pinned to the eigenpairs."""
    A, f0 = _sym(16, 13)
    a, b = bse.chebyshev_scale(*bse.spectral_bounds(A))
    wg = np.array([0.3, 0.55, 0.8])
    Fm = bse.chebyshev_states(A, f0, 300, a, b, wg, 0.03)               # [q, n, p]
    Fo = bse.chebyshev_states_op(lambda x: A @ x, [f0[:, p] for p in range(3)], 300, a, b, wg, 0.03)
    assert np.abs(Fo - Fm.transpose(0, 2, 1)).max() < 1e-12 * np.abs(Fm).max()


def test_mixed_amplitudes_recover_conduction_coefficients(mixed_system):
    """For f_i = sum_a c_ia phi_a over orthonormal eigenstates the
    amplitudes <phi_a|f_i> are c_ia, and zero on the occupied orbitals."""
    spec, grid, v, phi, eps, w = mixed_system
    c = np.random.default_rng(14).standard_normal((2, 4))
    f = np.tensordot(c, phi[6:10], axes=(1, 0))
    assert np.abs(bse.mixed_amplitudes(grid, phi[6:10], f) - c).max() < 1e-9
    assert np.abs(bse.mixed_amplitudes(grid, phi[:6], f)).max() < 1e-9


def test_mixed_dipole_start_projects_to_eh_dipoles(mixed_system):
    """<phi_a| f0_j> = <phi_a| x |phi_j> for conduction a (Q leaves the
    virtual components alone) and <phi_s| f0_j> = 0 for occupied s."""
    spec, grid, v, phi, eps, w = mixed_system
    f0 = bse.mixed_dipole_start(grid, phi[:6], 2)
    d = bse.dipoles(grid, phi[4:6], phi[6:10])                 # [(i, a), axis]
    for ax in range(3):
        proj = (f0[ax].reshape(2, -1) @ phi[6:10].reshape(4, -1).T) * grid.dv
        assert np.abs(proj.reshape(-1) - d[:, ax]).max() < 1e-12
        assert np.abs((f0[ax].reshape(2, -1) @ phi[:6].reshape(6, -1).T) * grid.dv).max() < 1e-12
