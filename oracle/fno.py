"""Fourier-operator screening surrogate in FP64 (oracle; test infrastructure).

The surrogate maps the source potential of a pair density (scaled to unit
RMS) together with two channels describing the molecule (ground-state
density and V_ext) to the induced part W^pol of the screened interaction,
in the same scaling.  The paper has no such network; it stands beside the
TD-Hartree propagation, which generates its training data and checks its predictions.

Network (a Fourier neural operator):
  h_0 = P x + p                                  (lift, per grid point)
  z_l = W_l h_l + b_l + S_l h_l,  h_{l+1} = gelu(z_l) for l < n_layers - 1,
                                  h_{n_layers} = z_{n_layers - 1}
  y   = Q h_{n_layers} + q0                      (projection)
with the spectral convolution, for real channel fields v_i(r),
  V_i(k) = sum_r v_i(r) e^{-i k.r}  on the kept modes K,
  U_o(k) = sum_i V_i(k) R_io(k),
  (S v)_o(r) = (1/n_g) Re sum_{k in K} c_k U_o(k) e^{i k.r},
K = {k_x, k_y in [-m, m), k_z in [0, m)} in FFT index units, c_k = 1 on the
k_z = 0 plane and 2 elsewhere (the conjugate half of the spectrum).
gelu(z) = z/2 (1 + erf(z / sqrt 2)).  Loss: mean over the batch of
||y - t||^2 / ||t||^2.  Adam with bias correction.

Backward (complex gradients G = dL/dRe + i dL/dIm):
  G_U(k) = (c_k / n_g) DFT(g_S)(k),  G_V = conj(R) G_U,  G_R += conj(V) G_U,
  g_v(r) += Re sum_{k in K} G_V(k) e^{i k.r}.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def mode_mask(n: int, m: int):
    """Boolean mask of K on the full n^3 FFT grid and the c_k weights."""
    k = np.arange(n)
    kk = np.where(k < (n + 1) // 2, k, k - n)
    inxy = (kk >= -m) & (kk < m)
    inz = (kk >= 0) & (kk < m)
    mask = inxy[:, None, None] & inxy[None, :, None] & inz[None, None, :]
    ck = np.where(kk[None, None, :] == 0, 1.0, 2.0) * np.ones((n, n, n))
    return mask, ck


def kept_modes(n: int, m: int):
    """Index arrays (ix, iy, iz) of K in FFT index units, ordered
    kx-major, then ky, then kz, each ascending in signed frequency."""
    sig = list(range(-m, m))
    out = []
    for kx in sig:
        for ky in sig:
            for kz in range(m):
                out.append((kx % n, ky % n, kz))
    return np.array(out, dtype=np.int64)


def init_params(cin: int, width: int, m: int, n_layers: int, seed: int = 0):
    rng = np.random.default_rng(seed)
    K = (2 * m) * (2 * m) * m
    p = {"P": rng.uniform(-1, 1, (width, cin)) / math.sqrt(cin),
         "p": np.zeros(width),
         "Q": rng.uniform(-1, 1, width) / math.sqrt(width),
         "q0": np.zeros(1)}
    for l in range(n_layers):
        sc = 1.0 / (width * width)
        p[f"R{l}"] = sc * (rng.uniform(0, 1, (K, width, width))
                           + 1j * rng.uniform(0, 1, (K, width, width)))
        p[f"W{l}"] = rng.uniform(-1, 1, (width, width)) / math.sqrt(width)
        p[f"b{l}"] = np.zeros(width)
    return p


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def spectral_forward(v, R, n, modes):
    """v [B, C, n, n, n] real -> (S v [B, O, n, n, n], V [B, C, K])."""
    ix, iy, iz = modes[:, 0], modes[:, 1], modes[:, 2]
    F = np.fft.fftn(v, axes=(-3, -2, -1))
    V = F[..., ix, iy, iz]                                   # [B, C, K]
    U = np.einsum("bck,kco->bok", V, R)
    ck = np.where(iz == 0, 1.0, 2.0)
    S = np.zeros(v.shape[:1] + (R.shape[2], n, n, n), dtype=np.complex128)
    S[..., ix, iy, iz] = U * ck
    s = np.real(np.fft.ifftn(S, axes=(-3, -2, -1)))          # ifftn carries the 1/n_g
    return s, V


def spectral_backward(gs, V, R, n, modes):
    """Gradient of the spectral convolution: returns (g_v, G_R)."""
    ix, iy, iz = modes[:, 0], modes[:, 1], modes[:, 2]
    ng = n ** 3
    ck = np.where(iz == 0, 1.0, 2.0)
    GU = np.fft.fftn(gs, axes=(-3, -2, -1))[..., ix, iy, iz] * ck / ng     # [B, O, K]
    GV = np.einsum("bok,kco->bck", GU, np.conj(R))
    GR = np.einsum("bck,bok->kco", np.conj(V), GU)
    full = np.zeros(gs.shape[:1] + (R.shape[1], n, n, n), dtype=np.complex128)
    full[..., ix, iy, iz] = GV
    gv = np.real(np.fft.ifftn(full, axes=(-3, -2, -1))) * ng                # unnormalised inverse
    return gv, GR


def forward(params, x, n, m, n_layers):
    """x [B, Cin, n, n, n] -> y [B, n, n, n] and the cache for backward."""
    modes = kept_modes(n, m)
    h = np.einsum("oi,bi...->bo...", params["P"], x) + params["p"][None, :, None, None, None]
    cache = {"x": x, "h": [h], "z": [], "V": []}
    for l in range(n_layers):
        s, V = spectral_forward(h, params[f"R{l}"], n, modes)
        z = (np.einsum("oi,bi...->bo...", params[f"W{l}"], h)
             + params[f"b{l}"][None, :, None, None, None] + s)
        cache["z"].append(z)
        cache["V"].append(V)
        h = gelu(z) if l < n_layers - 1 else z
        cache["h"].append(h)
    y = np.einsum("i,bi...->b...", params["Q"], h) + params["q0"][0]
    return y, cache


def loss_and_grad(params, x, t, n, m, n_layers):
    """Mean relative squared error and its gradient with respect to every
    parameter (complex parameters: dL/dRe + i dL/dIm)."""
    modes = kept_modes(n, m)
    B = x.shape[0]
    y, c = forward(params, x, n, m, n_layers)
    tn = np.sum(t ** 2, axis=(1, 2, 3))
    diff = y - t
    L = float(np.mean(np.sum(diff ** 2, axis=(1, 2, 3)) / tn))
    gy = (2.0 / B) * diff / tn[:, None, None, None]
    g = {}
    hL = c["h"][-1]
    B_, C_ = hL.shape[0], hL.shape[1]
    g["Q"] = np.einsum("br,bir->i", gy.reshape(B_, -1), hL.reshape(B_, C_, -1))
    g["q0"] = np.array([gy.sum()])
    gh = params["Q"][None, :, None, None, None] * gy[:, None]
    for l in reversed(range(n_layers)):
        z = c["z"][l]
        gz = gh * gelu_grad(z) if l < n_layers - 1 else gh
        hin = c["h"][l]
        g[f"W{l}"] = np.einsum("bor,bir->oi", gz.reshape(gz.shape[0], gz.shape[1], -1),
                               hin.reshape(hin.shape[0], hin.shape[1], -1))
        g[f"b{l}"] = gz.sum(axis=(0, 2, 3, 4))
        gv, GR = spectral_backward(gz, c["V"][l], params[f"R{l}"], n, modes)
        g[f"R{l}"] = GR
        gh = np.einsum("oi,bo...->bi...", params[f"W{l}"], gz) + gv
    g["P"] = np.einsum("bor,bir->oi", gh.reshape(gh.shape[0], gh.shape[1], -1),
                       c["x"].reshape(c["x"].shape[0], c["x"].shape[1], -1))
    g["p"] = gh.sum(axis=(0, 2, 3, 4))
    return L, g


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update in place; complex parameters update their real and
    imaginary parts as independent real parameters."""
    state["t"] = state.get("t", 0) + 1
    tt = state["t"]
    for k, gk in grads.items():
        m = state.setdefault("m_" + k, np.zeros_like(gk))
        v = state.setdefault("v_" + k, np.zeros(gk.shape, dtype=np.complex128 if np.iscomplexobj(gk) else np.float64))
        m[...] = beta1 * m + (1 - beta1) * gk
        if np.iscomplexobj(gk):
            v[...] = beta2 * v + (1 - beta2) * (gk.real ** 2 + 1j * gk.imag ** 2)
            mh = m / (1 - beta1 ** tt)
            vh = v / (1 - beta2 ** tt)
            params[k] = params[k] - lr * (mh.real / (np.sqrt(vh.real) + eps)
                                          + 1j * mh.imag / (np.sqrt(vh.imag) + eps))
        else:
            v[...] = beta2 * v + (1 - beta2) * gk ** 2
            mh = m / (1 - beta1 ** tt)
            vh = v / (1 - beta2 ** tt)
            params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    return params
