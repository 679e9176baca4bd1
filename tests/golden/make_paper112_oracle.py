"""Writes paper112_oracle_pair.npz beside this script: the FP64 oracle's
W-action for one valence pair of the paper-scale molecule at its full length
(112^3 grid, h = 0.5, 220 wells on a ring plus a sphere, N_occ = 260, L = 10
stochastic orbitals, dt = 0.05, 600 steps, cleaning every 10 steps), which
is too slow to recompute inside a test (about half an hour on 8 cores).

It calls only the oracle and the seeded input generator.  Stored:

* the pair (i, j) and the propagation parameters;
* W and W^pol at 8192 grid points drawn with numpy's default_rng(2205) and
  sorted; the L2 norms and max |.| of W and W^pol over the whole grid;
* the direct-term integrals h^3 sum_r phi_k phi_l W for a few valence pairs
  (k, l), the numbers Eq. 1 takes from this W;
* a fingerprint of the inputs: every eigenvalue, and the integral of each
  orbital against a fixed Gaussian, so that a test built on inputs solved
  elsewhere (another device, another library) can tell whether they agree.

    python tests/golden/make_paper112_oracle.py [out.npz]

The inputs come from the same generator as the tests' (on a machine with a
GPU its eigensolve runs through torch there), so the fixture is made where
the tests run.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from paper_2205_06690_amd import inputs  # noqa: E402
from oracle.grid import Grid  # noqa: E402
from oracle import tdh  # noqa: E402

OUT = os.path.join(HERE, "paper112_oracle_pair.npz")
PAIR = (258, 259)
PROJ = [(258, 259), (258, 258), (259, 259), (257, 259), (250, 255)]
N_SAMPLE = 8192


def fingerprint(spec, phi):
    """Integral of each orbital against a Gaussian of width 6 bohr centred
    at (0.3, 0.4, 0.55) of the box: insensitive to rounding, sensitive to a
    sign or a rotation among nearly degenerate orbitals."""
    x = np.arange(spec.n) * spec.h
    c = np.array([0.3, 0.4, 0.55]) * spec.n * spec.h
    g = (np.exp(-((x - c[0]) ** 2) / 72.0)[:, None, None] * np.exp(-((x - c[1]) ** 2) / 72.0)[None, :, None]
         * np.exp(-((x - c[2]) ** 2) / 72.0)[None, None, :]).reshape(-1)
    return (phi @ g) * spec.h ** 3


def main():
    spec = inputs.CONFIGS["paper112"]
    t0 = time.perf_counter()
    sysd = inputs.make_system(spec)
    print(f"inputs ready in {time.perf_counter() - t0:.0f}s", flush=True)
    grid = Grid(spec.shape, spec.h)
    phi = sysd["phi"].reshape((-1,) + spec.shape)
    eta0 = tdh.stochastic_orbitals(phi[:spec.n_occ], sysd["xi"])
    t1 = time.perf_counter()

    def report(n):
        if n % 30 == 0:
            print(f"oracle step {n}/{spec.n_steps}, {time.perf_counter() - t1:.0f}s", flush=True)

    w, wp = tdh.apply_w(grid, sysd["v_ext"], phi, spec.n_occ, [PAIR], eta0, dt=spec.dt,
                        n_steps=spec.n_steps, gamma=spec.gamma_eff, clean_every=spec.clean_every,
                        progress=report)
    out = sys.argv[1] if len(sys.argv) > 1 else OUT
    w, wp = w.reshape(-1), wp.reshape(-1)
    idx = np.sort(np.random.default_rng(2205).choice(spec.ng, size=N_SAMPLE, replace=False))
    ph2 = sysd["phi"]
    proj = np.array([np.dot(ph2[k] * ph2[l], w) * spec.h ** 3 for k, l in PROJ])
    np.savez(out, pair=np.array(PAIR, dtype=np.int32), n_steps=spec.n_steps, dt=spec.dt,
             gamma=spec.gamma_eff, clean_every=spec.clean_every, n_stoch=spec.n_stoch,
             idx=idx, w=w[idx], wpol=wp[idx], w_norm=np.linalg.norm(w), wpol_norm=np.linalg.norm(wp),
             w_max=np.abs(w).max(), wpol_max=np.abs(wp).max(), proj_pairs=np.array(PROJ, dtype=np.int32),
             proj=proj, eps=sysd["eps"], fingerprint=fingerprint(spec, ph2))
    print(f"wrote {out} after {time.perf_counter() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main()
