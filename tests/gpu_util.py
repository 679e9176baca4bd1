"""Shared helpers of the GPU tests: cached synthetic systems and the
oracle's W for them (oracle runs on the CPU)."""
import functools
import math
import sys

import numpy as np

from paper_2205_06690_amd import inputs
from oracle.grid import Grid
from oracle import tdh


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=None)
def system(name: str):
    spec = inputs.CONFIGS[name]
    return spec, inputs.make_system(spec)


def small_spec(n=16, h=0.6, wells=5, seed=7, n_occ=6, n_o=2, n_c=3, n_steps=60, n_stoch=4):
    return inputs.SystemSpec(n=n, h=h, n_wells=wells, seed=seed, n_occ=n_occ, n_o=n_o, n_c=n_c,
                             n_stoch=n_stoch, dt=0.05, n_steps=n_steps)


def oracle_w(spec, sysd, pairs, n_stoch=None, xi=None):
    """(W, W^pol) of the oracle for ``pairs`` with the system's signs."""
    grid = Grid(spec.shape, spec.h)
    phi = sysd["phi"].reshape((-1,) + spec.shape)
    L = spec.n_stoch if n_stoch is None else n_stoch
    if L == 0:
        eta0 = phi[:spec.n_occ]
    else:
        xi = sysd["xi"] if xi is None else xi
        eta0 = tdh.stochastic_orbitals(phi[:spec.n_occ], xi)
    return tdh.apply_w(grid, sysd["v_ext"], phi, spec.n_occ, pairs, eta0, dt=spec.dt,
                       n_steps=spec.n_steps, gamma=spec.gamma_eff,
                       clean_every=spec.clean_every)


def gpu_system(spec, sysd, precision, max_batch=4, n_stoch=None, xi=None):
    from paper_2205_06690_amd import bse
    L = spec.n_stoch if n_stoch is None else n_stoch
    s = bse.System(spec.n, spec.h, sysd["v_ext"], n_occ=spec.n_occ, n_stoch=L, seed=spec.seed,
                   dt=spec.dt, n_steps=spec.n_steps, gamma=spec.gamma_eff,
                   clean_every=spec.clean_every, precision=precision, max_batch=max_batch)
    if L > 0:
        s.set_signs(sysd["xi"] if xi is None else xi)
    s.set_orbitals(sysd["phi"], sysd["eps"])
    return s


def rel(a, b):
    return np.linalg.norm(a - b, axis=-1) / np.linalg.norm(b, axis=-1)
