"""Plain FP64 CPU oracle of the stochastic-W Bethe-Salpeter hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` use it.  It shares no code with the HIP
library; both receive the same inputs (grid, V_ext, orbitals, eigenvalues,
random signs) from ``paper_2205_06690_amd.inputs``.

Modules
-------
grid  -- periodic grid, spectral kinetic operator, FFT Poisson solver.
tdh   -- linear-response TD-Hartree action of the screened interaction W on a
         pair density (Method: "Stochastic evaluation of the action of W",
         Eqs. 10-15), deterministic or stochastic, linearised or finite alpha.
bse   -- Tamm-Dancoff matrix A (Eq. 1), lowest excitons and the absorption
         cross section with dipole oscillator strengths (Eq. 7).

Every function is written for clarity, not speed: whole-field FFTs with
numpy/scipy, no blocking or fusion.

Parity status: every function is pinned by the ``-m "not gpu"`` tests
(closed forms, sum-over-states and Casida limits, Hadamard-sign exactness,
finite-alpha limit, symmetry and sign invariants); none is "parity
unpinned".
"""
