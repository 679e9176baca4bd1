"""Seeded synthetic inputs: Gaussian-well molecules, their H0 eigenpairs and
the random signs of the stochastic occupied orbitals.

This module prepares *inputs* only.  It holds none of the method's
arithmetic (no propagation, no screening, no BSE matrix): both the FP64
oracle and the GPU library receive what it returns.

* The paper's system is a closed-shell molecule described by the
  eigenstates of a zero-order Hamiltonian H0 (Method section, first
  paragraphs).  Its real H0 came from DFT with pseudopotentials; here H0 is
  -1/2 Laplacian (Fourier spectral on a periodic grid) plus a sum of
  attractive Gaussian wells, solved in FP64.
* The random signs +-1 of the stochastic orbitals (Eq. 14) are drawn from
  SplitMix64 (Steele, Lea and Flood, OOPSLA 2014; reference C code by
  S. Vigna): the k-th draw of a generator seeded with ``seed`` is
  mix(seed + (k+1)*0x9E3779B97F4A7C15) with the published finaliser, and
  sign(l, s) = +1 when the top bit of draw k = l*N_occ + s is 0, else -1.

Well recipe: V(r) = -sum_k U_k exp(-|r - R_k|^2_mic / (2 w_k^2)) with
minimum-image distances, U ~ U[1,3] Ha, w ~ U[0.8,1.5] bohr, centres
uniform in the inner 60 % of the box; numpy ``default_rng(seed)`` draws
U[:], then w[:], then R[:, 3].  The ring-plus-sphere layout puts 120 centres
on a ring of radius 9 bohr in the z = 0 plane through the box centre
(angle U[0, 2pi), z jitter U[-1.3, 1.3]) and the rest uniformly inside a
sphere of radius 4 bohr at the centre.
"""
from __future__ import annotations

import dataclasses
import hashlib
import json
import math
import os
from typing import Optional

import numpy as np

try:  # threaded FFTs when scipy is present
    import scipy.fft as _sfft

    def _rfftn(x, axes):
        return _sfft.rfftn(x, axes=axes, workers=os.cpu_count() or 1)

    def _irfftn(x, s, axes):
        return _sfft.irfftn(x, s=s, axes=axes, workers=os.cpu_count() or 1)
except ImportError:  # pragma: no cover
    def _rfftn(x, axes):
        return np.fft.rfftn(x, axes=axes)

    def _irfftn(x, s, axes):
        return np.fft.irfftn(x, s=s, axes=axes)


HARTREE_EV = 27.211386245988
MASK64 = (1 << 64) - 1
GOLDEN64 = 0x9E3779B97F4A7C15


# --------------------------------------------------------------------------
# system specification
# --------------------------------------------------------------------------
@dataclasses.dataclass
class SystemSpec:
    n: int                   # grid points per axis (cubic box)
    h: float                 # spacing, bohr
    n_wells: int
    seed: int
    n_occ: int               # closed shell with 2*n_occ electrons
    n_o: int                 # valence orbitals in the exciton window
    n_c: int                 # conduction orbitals in the exciton window
    n_stoch: int = 10        # L stochastic orbitals; 0 => deterministic
    dt: float = 0.05
    n_steps: int = 200
    clean_every: int = 10    # M
    gamma: Optional[float] = None   # Ha; None => sqrt(2 ln 1e4) / T
    layout: str = "uniform"  # "uniform" | "ring_sphere"
    depth: tuple = (1.0, 3.0)
    width: tuple = (0.8, 1.5)
    sign_seed: Optional[int] = None  # None => seed
    mol_n: Optional[int] = None      # draw the wells as in a box of mol_n points and centre
                                     # that box in this one (the same molecule in several boxes)

    @property
    def ng(self) -> int:
        return self.n ** 3

    @property
    def shape(self):
        return (self.n, self.n, self.n)

    @property
    def box(self) -> float:
        return self.n * self.h

    @property
    def t_final(self) -> float:
        return self.n_steps * self.dt

    @property
    def gamma_eff(self) -> float:
        if self.gamma is not None:
            return float(self.gamma)
        return math.sqrt(2.0 * math.log(1.0e4)) / self.t_final

    @property
    def n_orb(self) -> int:
        return self.n_occ + self.n_c

    def key(self) -> str:
        d = dataclasses.asdict(self)
        return hashlib.sha1(json.dumps(d, sort_keys=True).encode()).hexdigest()[:16]

    def potential_key(self) -> str:
        """Hash of the fields that fix V_ext (and so the orbitals)."""
        d = {k: getattr(self, k) for k in ("n", "h", "n_wells", "seed", "layout", "depth", "width")}
        if self.mol_n is not None:
            d["mol_n"] = self.mol_n
        return hashlib.sha1(json.dumps(d, sort_keys=True).encode()).hexdigest()[:16]


# The five workloads: a tiny plain-method case, a mid-size molecule, a
# paper-scale molecule (electron count of the paper's 520-electron system),
# and the generator recipes of the uneven batch and the surrogate data.
CONFIGS = {
    "tiny24": SystemSpec(n=24, h=0.5, n_wells=8, seed=0, n_occ=8, n_o=2, n_c=4,
                         n_stoch=10, dt=0.05, n_steps=200),
    "mid64": SystemSpec(n=64, h=0.4, n_wells=60, seed=1, n_occ=120, n_o=10, n_c=20,
                        n_stoch=10, dt=0.05, n_steps=400),
    "paper112": SystemSpec(n=112, h=0.5, n_wells=220, seed=2, n_occ=260, n_o=20,
                           n_c=40, n_stoch=10, dt=0.05, n_steps=600,
                           layout="ring_sphere"),
}


def box_series(spec: SystemSpec, sizes):
    """The molecule of ``spec`` in cubic boxes of ``sizes`` points per axis
    (same spacing, wells at the same place relative to the box centre): the
    several-box runs of the W(k->0) correction (Results section)."""
    return [dataclasses.replace(spec, n=int(m), mol_n=spec.n) for m in sizes]


def uneven_batch_specs(n_systems: int = 32):
    """The uneven batch: grids from {32,48,64}^3 at h = 0.4, 10-80 wells,
    N_occ 10-100, 16-200 pair densities, 400 steps, seeds 1000+m."""
    specs = []
    for m in range(n_systems):
        rng = np.random.default_rng(1000 + m)
        n = int(rng.choice([32, 48, 64]))
        n_wells = int(rng.integers(10, 81))
        n_occ = int(rng.integers(10, 101))
        n_pairs = int(rng.integers(16, 201))
        # n_o * n_c >= n_pairs with n_o <= n_occ
        n_o = max(1, min(n_occ, int(round(math.sqrt(n_pairs / 2.0)))))
        n_c = int(math.ceil(n_pairs / n_o))
        specs.append((SystemSpec(n=n, h=0.4, n_wells=n_wells, seed=1000 + m,
                                 n_occ=n_occ, n_o=n_o, n_c=n_c, n_stoch=10,
                                 dt=0.05, n_steps=400), n_pairs))
    return specs


# --------------------------------------------------------------------------
# wells
# --------------------------------------------------------------------------
def grid_coords(n: int, h: float):
    """Grid point positions x_i = i*h, i = 0..n-1 (periodic box [0, n*h))."""
    return np.arange(n, dtype=np.float64) * h


def well_params(spec: SystemSpec):
    rng = np.random.default_rng(spec.seed)
    k = spec.n_wells
    U = rng.uniform(spec.depth[0], spec.depth[1], size=k)
    w = rng.uniform(spec.width[0], spec.width[1], size=k)
    if spec.mol_n is not None:
        # the molecule of the mol_n box, moved to the centre of this one
        if spec.mol_n > spec.n:
            raise ValueError("mol_n must not exceed n")
        U, w, R = well_params(dataclasses.replace(spec, n=spec.mol_n, mol_n=None))
        return U, w, R + 0.5 * (spec.n - spec.mol_n) * spec.h
    box = spec.box
    if spec.layout == "uniform":
        R = rng.uniform(0.2, 0.8, size=(k, 3)) * box
    elif spec.layout == "ring_sphere":
        n_ring = min(120, k)
        n_sph = k - n_ring
        c = 0.5 * box
        ang = rng.uniform(0.0, 2.0 * math.pi, size=n_ring)
        zj = rng.uniform(-1.3, 1.3, size=n_ring)
        ring = np.stack([c + 9.0 * np.cos(ang), c + 9.0 * np.sin(ang), c + zj], axis=1)
        # uniform in a ball of radius 4: direction * r, r = 4 u^(1/3)
        d = rng.normal(size=(n_sph, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        r = 4.0 * rng.uniform(0.0, 1.0, size=n_sph) ** (1.0 / 3.0)
        sph = c + d * r[:, None]
        R = np.concatenate([ring, sph], axis=0)
    else:
        raise ValueError(f"unknown layout {spec.layout!r}")
    return U, w, R


def make_vext(spec: SystemSpec) -> np.ndarray:
    """V_ext on the grid, FP64, shape (n, n, n), row-major, z fastest."""
    U, w, R = well_params(spec)
    x = grid_coords(spec.n, spec.h)
    box = spec.box
    V = np.zeros(spec.shape, dtype=np.float64)
    for k in range(len(U)):
        d = [x - R[k, a] for a in range(3)]
        d = [di - box * np.round(di / box) for di in d]
        g = [np.exp(-(di ** 2) / (2.0 * w[k] ** 2)) for di in d]
        V -= U[k] * g[0][:, None, None] * g[1][None, :, None] * g[2][None, None, :]
    return V


# --------------------------------------------------------------------------
# H0 eigensolver (FP64): dense for tiny grids, Chebyshev-filtered subspace
# iteration (Zhou & Saad 2007) otherwise.
# --------------------------------------------------------------------------
def _k2half_rfft(n: int, h: float):
    k = 2.0 * math.pi * np.fft.fftfreq(n, d=h)
    kr = 2.0 * math.pi * np.fft.rfftfreq(n, d=h)
    # the last axis of an rfft holds the non-negative frequencies; the
    # Nyquist bin (even n) carries (pi/h)^2, the same as fftfreq's -n/2
    k2 = k[:, None, None] ** 2 + k[None, :, None] ** 2 + kr[None, None, :] ** 2
    return 0.5 * k2


class _H0:
    def __init__(self, v_ext: np.ndarray, h: float):
        self.shape = v_ext.shape
        self.n = v_ext.shape[0]
        self.v = v_ext.reshape(-1)
        self.t = _k2half_rfft(self.n, h)
        self.tmax = float(3.0 * (math.pi / h) ** 2 / 2.0)

    def __call__(self, X: np.ndarray) -> np.ndarray:
        m = X.shape[0]
        F = _rfftn(X.reshape((m,) + self.shape), axes=(1, 2, 3))
        F *= self.t[None]
        Y = _irfftn(F, s=self.shape, axes=(1, 2, 3)).reshape(m, -1)
        Y += self.v[None, :] * X
        return Y


def _cholqr(Y: np.ndarray) -> np.ndarray:
    for _ in range(2):
        S = Y @ Y.T
        Lc = np.linalg.cholesky(S)
        Y = np.linalg.inv(Lc) @ Y
    return Y


def _chebfilter(H, X, deg, a, b, a0):
    e = (b - a) / 2.0
    c = (b + a) / 2.0
    sigma = e / (a0 - c)
    tau = 2.0 / sigma
    Y = (H(X) - c * X) * (sigma / e)
    for _ in range(2, deg + 1):
        sn = 1.0 / (tau - sigma)
        Yn = (H(Y) - c * Y) * (2.0 * sn / e) - (sigma * sn) * X
        X, Y, sigma = Y, Yn, sn
    return Y


def eigensolve(v_ext: np.ndarray, h: float, n_states: int, *, tol: float = 1e-9,
               seed: int = 12345, max_iter: int = 200, deg: int = 16,
               verbose: bool = False):
    """Lowest ``n_states`` eigenpairs of H0 = -1/2 Lap + V_ext on the periodic
    grid.  Returns (phi [n_states, ng], eps [n_states]) with
    sum |phi|^2 h^3 = 1, ascending eps, and the sign fixed so that each
    orbital's largest-magnitude value is positive.  ``tol`` bounds the
    residual ||H0 x - eps x|| of the unit-norm vectors x."""
    H = _H0(v_ext, h)
    ng = v_ext.size
    if ng <= 2200:
        I = np.eye(ng)
        Hd = H(I)
        Hd = 0.5 * (Hd + Hd.T)
        w, U = np.linalg.eigh(Hd)
        X = U[:, :n_states].T.copy()
        eps = w[:n_states].copy()
    else:
        m = n_states + max(16, n_states // 2)
        rng = np.random.default_rng(seed)
        X = _cholqr(rng.standard_normal((m, ng)))
        HX = H(X)
        w, U = np.linalg.eigh(X @ HX.T)
        X = U.T @ X
        b = H.tmax + float(v_ext.max())
        a = float(w[-1])
        a0 = float(w[0])
        for it in range(max_iter):
            Y = _chebfilter(H, X, deg, a, b, a0)
            X = _cholqr(Y)
            HX = H(X)
            S = X @ HX.T
            S = 0.5 * (S + S.T)
            w, U = np.linalg.eigh(S)
            X = U.T @ X
            HX = U.T @ HX
            R = HX[:n_states] - w[:n_states, None] * X[:n_states]
            res = np.linalg.norm(R, axis=1).max()
            if verbose:
                print(f"chefsi it {it} res {res:.3e} eps0 {w[0]:.6f}", flush=True)
            a0 = float(w[0])
            a = float(w[-1])
            if res < tol:
                break
        else:
            raise RuntimeError(f"eigensolve did not converge (res {res:.3e})")
        X = X[:n_states]
        eps = w[:n_states].copy()
    idx = np.argmax(np.abs(X), axis=1)
    sgn = np.sign(X[np.arange(X.shape[0]), idx])
    X = X * sgn[:, None]
    phi = X / math.sqrt(h ** 3)
    return np.ascontiguousarray(phi), eps


def eigensolve_torch(v_ext: np.ndarray, h: float, n_states: int, *, tol: float = 1e-9,
                     seed: int = 12345, max_iter: int = 200, deg: int = 16, device: str = "cuda",
                     verbose: bool = False):
    """The same Chebyshev-filtered subspace iteration as ``eigensolve``, with
    the FP64 FFTs and tall-skinny products on a GPU through torch (input
    preparation only; small dense steps stay on the host in numpy)."""
    import torch
    n = v_ext.shape[0]
    ng = v_ext.size
    dev = torch.device(device)
    vt = torch.from_numpy(np.ascontiguousarray(v_ext.reshape(-1))).to(dev)
    tk = torch.from_numpy(_k2half_rfft(n, h)).to(dev)
    shape = v_ext.shape

    def H(X):
        m = X.shape[0]
        F = torch.fft.rfftn(X.reshape((m,) + shape), dim=(1, 2, 3))
        F *= tk
        Y = torch.fft.irfftn(F, s=shape, dim=(1, 2, 3)).reshape(m, ng)
        return Y + vt * X

    def cholqr(Y):
        for _ in range(2):
            S = (Y @ Y.T).cpu().numpy()
            Li = np.linalg.inv(np.linalg.cholesky(S))
            Y = torch.from_numpy(Li).to(dev) @ Y
        return Y

    m = n_states + max(16, n_states // 2)
    g = torch.Generator(device="cpu").manual_seed(seed)
    X = cholqr(torch.randn((m, ng), dtype=torch.float64, generator=g).to(dev))
    HX = H(X)
    w, U = np.linalg.eigh((X @ HX.T).cpu().numpy())
    X = torch.from_numpy(U.T.copy()).to(dev) @ X
    b = float(3.0 * (math.pi / h) ** 2 / 2.0) + float(v_ext.max())
    a, a0 = float(w[-1]), float(w[0])
    for it in range(max_iter):
        e = (b - a) / 2.0
        c = (b + a) / 2.0
        sigma = e / (a0 - c)
        tau = 2.0 / sigma
        Y = (H(X) - c * X) * (sigma / e)
        Xp = X
        for _ in range(2, deg + 1):
            sn = 1.0 / (tau - sigma)
            Yn = (H(Y) - c * Y) * (2.0 * sn / e) - (sigma * sn) * Xp
            Xp, Y, sigma = Y, Yn, sn
        X = cholqr(Y)
        HX = H(X)
        S = (X @ HX.T).cpu().numpy()
        w, U = np.linalg.eigh(0.5 * (S + S.T))
        Ut = torch.from_numpy(U.T.copy()).to(dev)
        X = Ut @ X
        HX = Ut @ HX
        wt = torch.from_numpy(w[:n_states].copy()).to(dev)
        res = float(torch.linalg.norm(HX[:n_states] - wt[:, None] * X[:n_states], dim=1).max())
        if verbose:
            print(f"chefsi(gpu) it {it} res {res:.3e}", flush=True)
        a0, a = float(w[0]), float(w[-1])
        if res < tol:
            break
    else:
        raise RuntimeError(f"eigensolve did not converge (res {res:.3e})")
    Xh = X[:n_states].cpu().numpy()
    idx = np.argmax(np.abs(Xh), axis=1)
    sgn = np.sign(Xh[np.arange(Xh.shape[0]), idx])
    phi = (Xh * sgn[:, None]) / math.sqrt(h ** 3)
    return np.ascontiguousarray(phi), w[:n_states].copy()


# --------------------------------------------------------------------------
# random signs of the stochastic orbitals
# --------------------------------------------------------------------------
def splitmix64_draw(seed: int, k: int) -> int:
    """The k-th (0-based) output of SplitMix64 seeded with ``seed``."""
    z = (seed + (k + 1) * GOLDEN64) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def stochastic_signs(seed: int, n_stoch: int, n_occ: int) -> np.ndarray:
    """xi[l, s] in {+1, -1} (int8), l < n_stoch, s < n_occ."""
    xi = np.empty((n_stoch, n_occ), dtype=np.int8)
    for l in range(n_stoch):
        for s in range(n_occ):
            xi[l, s] = 1 if (splitmix64_draw(seed, l * n_occ + s) >> 63) == 0 else -1
    return xi


def hadamard_signs(n: int) -> np.ndarray:
    """Rows of the Sylvester Hadamard matrix of order n (a power of two)."""
    Hm = np.array([[1]], dtype=np.int8)
    while Hm.shape[0] < n:
        Hm = np.block([[Hm, Hm], [Hm, -Hm]]).astype(np.int8)
    if Hm.shape[0] != n:
        raise ValueError("n must be a power of two")
    return Hm


# --------------------------------------------------------------------------
# index sets
# --------------------------------------------------------------------------
def valence_indices(spec: SystemSpec):
    return list(range(spec.n_occ - spec.n_o, spec.n_occ))


def conduction_indices(spec: SystemSpec):
    return list(range(spec.n_occ, spec.n_occ + spec.n_c))


def ij_pairs(spec: SystemSpec) -> np.ndarray:
    """The n_o(n_o+1)/2 valence pairs (i <= j) whose W_ij the A matrix needs."""
    v = valence_indices(spec)
    return np.array([(v[a], v[b]) for a in range(len(v)) for b in range(a, len(v))],
                    dtype=np.int32).reshape(-1, 2)


def ia_pairs(spec: SystemSpec) -> np.ndarray:
    """The n_o*n_c valence-conduction pair densities."""
    return np.array([(i, a) for i in valence_indices(spec) for a in conduction_indices(spec)],
                    dtype=np.int32).reshape(-1, 2)


# --------------------------------------------------------------------------
# one-stop system build with an on-disk cache
# --------------------------------------------------------------------------
def cache_dir() -> str:
    d = os.environ.get("BSE_INPUT_CACHE", os.path.join("/tmp", "bse_inputs"))
    os.makedirs(d, exist_ok=True)
    return d


def _gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def make_system(spec: SystemSpec, *, n_states: Optional[int] = None, tol: float = 1e-9,
                use_cache: bool = True, verbose: bool = False, use_gpu: Optional[bool] = None):
    """Return dict(v_ext, phi, eps, xi) for ``spec`` (FP64; phi has
    ``n_states`` (default n_occ + n_c) rows).  Grids above 2 10^4 points are
    solved with torch on a GPU when one is present (input preparation
    only), else on the CPU."""
    n_states = spec.n_orb if n_states is None else n_states
    v = make_vext(spec)
    key = f"{spec.potential_key()}_{n_states}_{tol:g}"
    path = os.path.join(cache_dir(), f"sys_{key}.npz")
    phi = eps = None
    if use_cache and os.path.exists(path):
        try:
            z = np.load(path)
            phi, eps = z["phi"], z["eps"]
        except Exception:
            phi = eps = None
    if phi is None:
        if use_gpu is None:
            use_gpu = spec.ng > 20000 and _gpu_available()
        if use_gpu:
            phi, eps = eigensolve_torch(v, spec.h, n_states, tol=tol, verbose=verbose)
        else:
            phi, eps = eigensolve(v, spec.h, n_states, tol=tol, verbose=verbose)
        if use_cache:
            tmp = path + f".tmp{os.getpid()}.npz"
            np.savez(tmp, phi=phi, eps=eps)
            os.replace(tmp, path)
    sseed = spec.seed if spec.sign_seed is None else spec.sign_seed
    L = spec.n_stoch if spec.n_stoch > 0 else spec.n_occ
    xi = stochastic_signs(sseed, L, spec.n_occ) if spec.n_stoch > 0 else None
    return {"v_ext": v, "phi": phi, "eps": eps, "xi": xi}
