"""Training and evaluation driver of the screening surrogate.

The data, the network's forward and backward passes, Adam and the
surrogate W-action with its acceptance checks all run in libbse
(bse_fno_make_samples, bse_fno_train_step, bse_fno_forward,
bse_apply_W_surrogate); this module only schedules them: which pairs of
which molecules, batch order, learning-rate schedule.  Device buffers are
torch tensors.
"""
from __future__ import annotations

import math
import time
from typing import List, Optional

import numpy as np

from . import inputs
from . import bse


def surrogate_specs(seeds, n_steps: int = 200):
    """Mid-size molecules for the surrogate: 64^3 grid, h = 0.4, 60 wells,
    N_occ = 120, valence window 10, conduction window 20, L = 10, dt = 0.05."""
    return [inputs.SystemSpec(n=64, h=0.4, n_wells=60, seed=int(s), n_occ=120, n_o=10, n_c=20,
                              n_stoch=10, dt=0.05, n_steps=n_steps) for s in seeds]


def system_pairs(spec) -> np.ndarray:
    """The 55 valence pairs and the first 150 valence-conduction pairs."""
    return np.concatenate([inputs.ij_pairs(spec), inputs.ia_pairs(spec)[:150]])


def open_system(spec, sysd, max_batch: int = 64, precision: int = bse.BSE_MIXED):
    S = bse.System(spec.n, spec.h, sysd["v_ext"], n_occ=spec.n_occ, n_stoch=spec.n_stoch,
                   seed=spec.seed, dt=spec.dt, n_steps=spec.n_steps, gamma=spec.gamma_eff,
                   clean_every=spec.clean_every, precision=precision, max_batch=max_batch)
    S.set_signs(sysd["xi"])
    S.set_orbitals(sysd["phi"], sysd["eps"])
    return S


def generate(specs, limit: Optional[int] = None, log=print):
    """Samples (x [n,3,ng], t [n,ng], scale [n]) on the GPU for the pairs of
    every molecule in ``specs`` (first ``limit`` overall)."""
    import torch
    xs, ts, ss = [], [], []
    total = 0
    for spec in specs:
        if limit is not None and total >= limit:
            break
        sysd = inputs.make_system(spec)
        pairs = system_pairs(spec)
        if limit is not None:
            pairs = pairs[:limit - total]
        S = open_system(spec, sysd)
        x = torch.empty((len(pairs), 3, spec.ng), dtype=torch.float32, device="cuda")
        t = torch.empty((len(pairs), spec.ng), dtype=torch.float32, device="cuda")
        sc = torch.empty(len(pairs), dtype=torch.float64, device="cuda")
        t0 = time.perf_counter()
        bse.make_samples(S, pairs, x.data_ptr(), t.data_ptr(), sc.data_ptr())
        torch.cuda.synchronize()
        log(f"[surrogate] seed {spec.seed}: {len(pairs)} samples in {time.perf_counter() - t0:.1f}s")
        S.close()
        xs.append(x)
        ts.append(t)
        ss.append(sc)
        total += len(pairs)
    return torch.cat(xs), torch.cat(ts), torch.cat(ss)


def _cube_symmetry(rng):
    """A random element of the cube's symmetry group: an axis permutation and
    a set of axes to reverse.  On the periodic cubic grid the kinetic and
    Coulomb operators commute with both, so a molecule mapped by one of them
    has the mapped response: 48 molecules per training molecule."""
    return tuple(int(a) for a in rng.permutation(3)), tuple(int(a) for a in np.nonzero(rng.integers(0, 2, 3))[0])


def train(net: "bse.Fno", x, t, epochs: int, batch: int, lr: float, lr_end: float,
          seed: int = 0, log=print, time_limit: Optional[float] = None, augment: bool = True):
    """Adam with a cosine learning-rate decay; returns the per-epoch mean
    training loss.  With augment, each batch goes through a random symmetry
    of the cube (fields [batch][channel][x][y][z], targets [batch][x][y][z])."""
    import torch
    rng = np.random.default_rng(seed)
    n = x.shape[0]
    steps = epochs * (n // batch)
    hist = []
    k = 0
    t_start = time.perf_counter()
    xb = torch.empty((batch,) + tuple(x.shape[1:]), dtype=x.dtype, device=x.device)
    tb = torch.empty((batch,) + tuple(t.shape[1:]), dtype=t.dtype, device=t.device)
    for ep in range(epochs):
        perm = rng.permutation(n)
        losses = []
        for j in range(n // batch):
            # the batch's samples, under a random symmetry of the cube when
            # augmenting, assembled by the library's gather kernel
            sym_axes, flips = _cube_symmetry(rng) if augment else ((0, 1, 2), ())
            net.gather(perm[j * batch:(j + 1) * batch], n, x.data_ptr(), t.data_ptr(), sym_axes,
                       sum(1 << a for a in flips), xb.data_ptr(), tb.data_ptr())
            a = lr_end + 0.5 * (lr - lr_end) * (1 + math.cos(math.pi * k / max(steps, 1)))
            losses.append(net.train_step(batch, xb.data_ptr(), tb.data_ptr(), a))
            k += 1
        hist.append(float(np.mean(losses)))
        log(f"[surrogate] epoch {ep}: loss {hist[-1]:.5f} ({time.perf_counter() - t_start:.0f}s)")
        if time_limit is not None and time.perf_counter() - t_start > time_limit:
            break
    return hist


def predict(net: "bse.Fno", x, batch: int):
    import torch
    y = torch.empty((x.shape[0],) + tuple(x.shape[2:]), dtype=torch.float32, device="cuda")
    for j in range(0, x.shape[0], batch):
        b = min(batch, x.shape[0] - j)
        xb = x[j:j + b].contiguous()
        yb = torch.empty((b,) + tuple(x.shape[2:]), dtype=torch.float32, device="cuda")
        net.forward(b, xb.data_ptr(), yb.data_ptr())
        y[j:j + b] = yb
    return y
