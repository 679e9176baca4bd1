"""Pins of the oracle's Fourier-operator surrogate: spectral-convolution
conventions on plane waves, finite-difference gradients, the first Adam
step, and gelu."""
import math

import numpy as np
from scipy.special import erf

from oracle import fno


def _plane(n, k):
    r = np.arange(n)
    ph = 2 * math.pi * (k[0] * r[:, None, None] + k[1] * r[None, :, None] + k[2] * r[None, None, :]) / n
    return np.cos(ph)


def test_spectral_identity_passes_kept_modes_and_drops_others():
    n, m, C = 8, 2, 1
    modes = fno.kept_modes(n, m)
    R = np.ones((len(modes), C, C), dtype=np.complex128)
    for k in [(1, -1, 1), (0, 1, 0), (-2, 1, 1), (1, 0, 0)]:
        v = _plane(n, k)[None, None]
        s, _ = fno.spectral_forward(v, R, n, modes)
        assert np.abs(s - v).max() < 1e-12, k
    for k in [(2, 0, 1), (0, 0, 2), (3, 1, 0)]:          # outside K
        v = _plane(n, k)[None, None]
        s, _ = fno.spectral_forward(v, R, n, modes)
        assert np.abs(s).max() < 1e-12, k


def test_spectral_multiplies_mode_by_weight():
    """A kept mode k (k_z > 0) with weight R = a + ib becomes
    a cos(k.r) - b sin(k.r)."""
    n, m = 8, 2
    modes = fno.kept_modes(n, m)
    k = (1, 1, 1)
    idx = [i for i, q in enumerate(modes) if tuple(q) == (1, 1, 1)][0]
    R = np.zeros((len(modes), 1, 1), dtype=np.complex128)
    R[idx, 0, 0] = 0.3 + 0.7j
    r = np.arange(n)
    ph = 2 * math.pi * (r[:, None, None] + r[None, :, None] + r[None, None, :]) / n
    s, _ = fno.spectral_forward(np.cos(ph)[None, None], R, n, modes)
    assert np.abs(s[0, 0] - (0.3 * np.cos(ph) - 0.7 * np.sin(ph))).max() < 1e-12


def test_gradients_match_finite_differences():
    n, m, L = 8, 2, 2
    rng = np.random.default_rng(0)
    p = fno.init_params(3, 4, m, L, seed=1)
    for k in p:
        p[k] = p[k] + 0.1 * (rng.standard_normal(p[k].shape)
                             + (1j * rng.standard_normal(p[k].shape) if np.iscomplexobj(p[k]) else 0))
    x = rng.standard_normal((2, 3, n, n, n))
    t = rng.standard_normal((2, n, n, n))
    L0, g = fno.loss_and_grad(p, x, t, n, m, L)
    eps = 1e-6
    for key in ["P", "p", "Q", "q0", "W0", "b1", "R0", "R1"]:
        flat = p[key].reshape(-1)
        for j in rng.choice(flat.size, size=min(4, flat.size), replace=False):
            for part in ([1.0, 1j] if np.iscomplexobj(flat) else [1.0]):
                q = {kk: vv.copy() for kk, vv in p.items()}
                q[key].reshape(-1)[j] += eps * part
                Lp, _ = fno.loss_and_grad(q, x, t, n, m, L)
                q[key].reshape(-1)[j] -= 2 * eps * part
                Lm, _ = fno.loss_and_grad(q, x, t, n, m, L)
                fd = (Lp - Lm) / (2 * eps)
                gj = g[key].reshape(-1)[j]
                an = gj.real if part == 1.0 else gj.imag
                assert abs(fd - an) < 1e-6 * max(1.0, abs(an)), (key, j, part, fd, an)


def test_first_adam_step_moves_by_lr_sign():
    p = {"a": np.array([1.0, -2.0, 3.0]), "c": np.array([1 + 1j])}
    g = {"a": np.array([0.5, -0.1, 2.0]), "c": np.array([-3.0 + 0.2j])}
    st = {}
    fno.adam_step(p, g, st, lr=0.01, eps=0.0)
    assert np.allclose(p["a"], [0.99, -1.99, 2.99])
    assert np.allclose(p["c"], [1.01 + 0.99j])


def test_adam_three_step_trajectory_by_hand():
    """Three Adam steps (beta1 = 0.9, beta2 = 0.999, eps = 0, lr = 0.1) of one
    parameter p = 1 with gradients 1, -2, 1/2, worked by hand in fractions:
      t = 1: m = 1/10, v = 1/1000, m^ = 1, v^ = 1, p = 0.9
      t = 2: m = -11/100, v = 4999/10^6, m^ = -11/19, v^ = 4999/1999,
             p = 0.9 + 0.1 (11/19) / sqrt(4999/1999)
      t = 3: m = -49/1000, v = 5244001/10^9, m^ = -49/271,
             v^ = 749143/428143, p = p_2 + 0.1 (49/271) / sqrt(749143/428143)
    The first step moves every parameter by lr sign(g) whatever the betas;
    the second and third tell beta1 from beta2 and check both bias
    corrections.  A complex parameter updates its real and imaginary parts
    as two independent real parameters."""
    p2 = 0.9 + 0.1 * (11 / 19) / math.sqrt(4999 / 1999)
    p3 = p2 + 0.1 * (49 / 271) / math.sqrt(749143 / 428143)
    traj = []
    p = {"a": np.array([1.0]), "c": np.array([1.0 - 1.0j])}
    st = {}
    for g in (1.0, -2.0, 0.5):
        fno.adam_step(p, {"a": np.array([g]), "c": np.array([g - 1j * g])}, st, lr=0.1, eps=0.0)
        traj.append((p["a"][0], p["c"][0]))
    for (a, c), ref in zip(traj, (0.9, p2, p3)):
        assert abs(a - ref) < 1e-14
        assert abs(c.real - ref) < 1e-14 and abs(c.imag + ref) < 1e-14
    assert abs(p3 - 0.9502794190086671) < 1e-15


def test_gelu_values_and_derivative():
    z = np.array([-3.0, -0.5, 0.0, 0.7, 2.5])
    assert np.allclose(fno.gelu(z), z * 0.5 * (1 + erf(z / math.sqrt(2))))
    d = (fno.gelu(z + 1e-6) - fno.gelu(z - 1e-6)) / 2e-6
    assert np.allclose(fno.gelu_grad(z), d, atol=1e-8)
