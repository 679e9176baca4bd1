"""ctypes binding of libbse (include/bse.h): argument marshalling only.

Every step of the computation runs in the HIP library; this module copies
numpy arrays in and out, or passes device pointers of torch tensors for the
device variants.  Importing it raises if the library is not built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np
# torch is loaded before libbse so that the HIP runtime torch brings is the
# process's only one: libbse then binds to it by soname.  Loading libbse
# first pulls in a second runtime, and whichever of the two initialises the
# device second finds none.
import torch  # noqa: F401

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libbse.so")

BSE_OK, BSE_ERR_ARG, BSE_ERR_STATE, BSE_ERR_OOM, BSE_ERR_DEVICE, BSE_ERR_NUMERIC = 0, -1, -2, -3, -4, -5
BSE_FP64, BSE_MIXED = 0, 1
BSE_F64, BSE_F32 = 0, 1

# every symbol declared in include/bse.h
EXPORTS = (
    "bse_create_system", "bse_set_orbitals", "bse_set_signs", "bse_apply_W",
    "bse_apply_W_device", "bse_build_A", "bse_spectrum", "bse_set_stream",
    "bse_generate_signs", "bse_kernel_times", "bse_set_timing", "bse_set_lanczos_path",
    "bse_last_error",
    "bse_version", "bse_destroy_system", "bse_apply_W_batch", "bse_autotune",
    "bse_tuned_shape", "bse_fno_create", "bse_fno_num_params", "bse_fno_set_params",
    "bse_fno_get_params", "bse_fno_set_stream", "bse_fno_forward", "bse_fno_loss_grad",
    "bse_fno_train_step", "bse_fno_gather", "bse_fno_last_error", "bse_fno_destroy", "bse_fno_max_batch",
    "bse_fno_make_samples", "bse_apply_W_surrogate", "bse_chebyshev_spectrum",
    "bse_apply_A_mixed", "bse_chebyshev_mixed", "bse_exciton_states", "bse_exciton_states_mixed",
    "bse_boundary_potential", "bse_fit_box_correction", "bse_inject_fault", "bse_valence_W",
    "bse_chebyshev_spectrum_noalloc", "bse_fno_set_mix_path", "bse_batch_plan_create",
    "bse_batch_plan_run", "bse_batch_plan_destroy", "bse_set_launch_order",
    "bse_set_yz_schedule",
)


class BseConfig(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("h", C.c_double),
        ("n_occ", C.c_int32), ("n_stoch", C.c_int32), ("seed", C.c_uint64),
        ("dt", C.c_double), ("n_steps", C.c_int32), ("gamma", C.c_double),
        ("clean_every", C.c_int32), ("alpha", C.c_double), ("scissors", C.c_double),
        ("precision", C.c_int32), ("device", C.c_int32), ("max_batch", C.c_int32),
    ]


class FnoConfig(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("cin", C.c_int32), ("width", C.c_int32), ("modes", C.c_int32),
        ("layers", C.c_int32), ("max_batch", C.c_int32), ("device", C.c_int32),
        ("bf16_weights", C.c_int32), ("seed", C.c_uint64),
    ]


class BseError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libbse error {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"libbse is not built ({_LIB_PATH} missing); run "
                          "python -m paper_2205_06690_amd.build")
    lib = C.CDLL(_LIB_PATH)
    P = C.c_void_p
    dp = C.POINTER(C.c_double)
    ip = C.POINTER(C.c_int32)
    lib.bse_create_system.argtypes = [C.POINTER(BseConfig), dp, C.POINTER(P)]
    lib.bse_set_orbitals.argtypes = [P, C.c_int32, dp, dp]
    lib.bse_set_signs.argtypes = [P, C.c_int32, C.c_int32, C.POINTER(C.c_int8)]
    lib.bse_apply_W.argtypes = [P, C.c_int32, ip, dp, dp, ip]
    lib.bse_apply_W_device.argtypes = [P, C.c_int32, P, P, C.c_int32]
    lib.bse_inject_fault.argtypes = [P, C.c_int32, C.c_int32, C.c_int64, C.c_double]
    lib.bse_build_A.argtypes = [P, C.c_int32, C.c_int32, dp]
    lib.bse_valence_W.argtypes = [P, dp]
    lib.bse_spectrum.argtypes = [P, C.c_int32, dp, dp, C.c_int32, dp, C.c_double, dp]
    lib.bse_chebyshev_spectrum.argtypes = [P, C.c_int32, C.c_double, C.c_double, C.c_int32, dp,
                                           C.c_double, dp, dp, dp]
    lib.bse_chebyshev_spectrum_noalloc.argtypes = [P, C.c_int32, C.c_double, C.c_double, C.c_int32, dp,
                                                   C.c_double, dp, dp, dp]
    lib.bse_apply_A_mixed.argtypes = [P, C.c_int32, dp, dp]
    lib.bse_exciton_states.argtypes = [P, C.c_int32, C.c_double, C.c_double, C.c_int32, dp, C.c_double,
                                       dp, dp, dp]
    lib.bse_exciton_states_mixed.argtypes = [P, C.c_int32, C.c_double, C.c_double, C.c_int32, dp,
                                             C.c_double, C.c_int32, dp, dp]
    lib.bse_chebyshev_mixed.argtypes = [P, C.c_int32, C.c_double, C.c_double, C.c_int32, dp,
                                        C.c_double, dp, dp]
    lib.bse_boundary_potential.argtypes = [P, dp]
    lib.bse_fit_box_correction.argtypes = [C.c_int32, C.c_int32, dp, dp, dp, dp, dp]
    lib.bse_set_stream.argtypes = [P, P]
    lib.bse_generate_signs.argtypes = [C.c_uint64, C.c_int32, C.c_int32, C.POINTER(C.c_int8)]
    lib.bse_kernel_times.argtypes = [P, C.c_int32, C.POINTER(C.c_char_p), dp, ip]
    lib.bse_kernel_times.restype = C.c_int32
    lib.bse_set_timing.argtypes = [P, C.c_int32]
    lib.bse_set_lanczos_path.argtypes = [P, C.c_int32]
    lib.bse_set_launch_order.argtypes = [P, C.c_int32]
    lib.bse_set_yz_schedule.argtypes = [P, C.c_int32]
    lib.bse_apply_W_batch.argtypes = [C.c_int32, C.POINTER(P), ip, C.POINTER(ip), C.POINTER(P),
                                      C.c_int32]
    lib.bse_batch_plan_create.argtypes = [C.c_int32, C.POINTER(P), ip, C.POINTER(ip), C.POINTER(P),
                                          C.POINTER(P)]
    lib.bse_batch_plan_run.argtypes = [P]
    lib.bse_batch_plan_destroy.argtypes = [P]
    lib.bse_batch_plan_destroy.restype = None
    lib.bse_autotune.argtypes = [P, C.c_int32, C.c_char_p]
    lib.bse_tuned_shape.argtypes = [P, ip, ip]
    lib.bse_tuned_shape.restype = C.c_int32
    fp = C.POINTER(C.c_float)
    lib.bse_fno_create.argtypes = [C.POINTER(FnoConfig), C.POINTER(P)]
    lib.bse_fno_num_params.argtypes = [P]
    lib.bse_fno_num_params.restype = C.c_int64
    lib.bse_fno_set_params.argtypes = [P, fp]
    lib.bse_fno_get_params.argtypes = [P, fp, C.c_int32]
    lib.bse_fno_set_stream.argtypes = [P, P]
    lib.bse_fno_set_mix_path.argtypes = [P, C.c_int32]
    lib.bse_fno_forward.argtypes = [P, C.c_int32, P, P]
    lib.bse_fno_loss_grad.argtypes = [P, C.c_int32, P, P, dp, fp]
    lib.bse_fno_train_step.argtypes = [P, C.c_int32, P, P, C.c_double, dp]
    lib.bse_fno_gather.argtypes = [P, C.c_int32, ip, C.c_int32, P, P, ip, C.c_int32, P, P]
    lib.bse_fno_last_error.restype = C.c_char_p
    lib.bse_fno_max_batch.argtypes = [P]
    lib.bse_fno_max_batch.restype = C.c_int32
    lib.bse_fno_make_samples.argtypes = [P, C.c_int32, ip, P, P, P]
    lib.bse_apply_W_surrogate.argtypes = [P, P, C.c_int32, ip, P, C.c_double, C.c_int32, ip, dp]
    lib.bse_fno_destroy.argtypes = [P]
    lib.bse_fno_destroy.restype = None
    lib.bse_last_error.restype = C.c_char_p
    lib.bse_version.restype = C.c_char_p
    lib.bse_destroy_system.argtypes = [P]
    lib.bse_destroy_system.restype = None
    for name in EXPORTS:
        getattr(lib, name)
    return lib


LIB = _load()


def _check(rc: int):
    if rc != BSE_OK:
        raise BseError(rc, LIB.bse_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def apply_w_batch(systems, pair_lists, w_dev_ptrs, use_graph: bool = True, work_list: bool = False):
    """W-action for several systems at once (bse_apply_W_batch); outputs go to
    the device buffers whose pointers are given.  use_graph: captured into
    one HIP graph; work_list: the lockstep schedule whose propagation passes
    walk the items of every system in one launch each per time step."""
    n = len(systems)
    hs = (C.c_void_p * n)(*[s._h for s in systems])
    pqs = [np.ascontiguousarray(np.asarray(p, dtype=np.int32).reshape(-1, 2)) for p in pair_lists]
    npairs = np.array([p.shape[0] for p in pqs], dtype=np.int32)
    pq_ptrs = (C.POINTER(C.c_int32) * n)(*[_iptr(p) for p in pqs])
    w_ptrs = (C.c_void_p * n)(*[C.c_void_p(p) for p in w_dev_ptrs])
    mode = (1 if use_graph else 0) | (2 if work_list else 0)
    _check(LIB.bse_apply_W_batch(n, hs, _iptr(npairs), pq_ptrs, w_ptrs, mode))


class BatchPlan:
    """A captured uneven batch (bse_batch_plan_*): create once, run many
    times; outputs go to the device buffers given at creation."""

    def __init__(self, systems, pair_lists, w_dev_ptrs):
        n = len(systems)
        self._systems = list(systems)          # the plan uses their workspaces
        hs = (C.c_void_p * n)(*[s._h for s in systems])
        self._pqs = [np.ascontiguousarray(np.asarray(p, dtype=np.int32).reshape(-1, 2)) for p in pair_lists]
        npairs = np.array([p.shape[0] for p in self._pqs], dtype=np.int32)
        pq_ptrs = (C.POINTER(C.c_int32) * n)(*[_iptr(p) for p in self._pqs])
        w_ptrs = (C.c_void_p * n)(*[C.c_void_p(p) for p in w_dev_ptrs])
        h = C.c_void_p()
        _check(LIB.bse_batch_plan_create(n, hs, _iptr(npairs), pq_ptrs, w_ptrs, C.byref(h)))
        self._h = h

    def run(self):
        _check(LIB.bse_batch_plan_run(self._h))

    def close(self):
        if getattr(self, "_h", None):
            LIB.bse_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


def fit_box_correction(omega, v_bndry):
    """Inverse-dielectric fit of the W(k->0) correction over several boxes
    (bse_fit_box_correction): omega[n_box][n_exc] lowest excitation
    energies, v_bndry[n_box] boundary potentials -> (eps_inv, c[n_exc],
    w_k0[n_box])."""
    om = np.ascontiguousarray(omega, dtype=np.float64)
    v = np.ascontiguousarray(v_bndry, dtype=np.float64)
    if om.ndim != 2 or v.shape != (om.shape[0],):
        raise ValueError("omega must be [n_box][n_exc] and v_bndry [n_box]")
    e = C.c_double()
    c = np.empty(om.shape[1])
    wk = np.empty(om.shape[0])
    _check(LIB.bse_fit_box_correction(om.shape[0], om.shape[1], _dptr(om), _dptr(v), C.byref(e),
                                      _dptr(c), _dptr(wk)))
    return e.value, c, wk


def generate_signs(seed: int, n_stoch: int, n_occ: int) -> np.ndarray:
    xi = np.empty((n_stoch, n_occ), dtype=np.int8)
    _check(LIB.bse_generate_signs(seed, n_stoch, n_occ, xi.ctypes.data_as(C.POINTER(C.c_int8))))
    return xi


class System:
    """One periodic system on one device (a bse_system handle)."""

    def __init__(self, n: int, h: float, v_ext: np.ndarray, *, n_occ: int, n_stoch: int = 10,
                 seed: int = 0, dt: float = 0.05, n_steps: int = 200, gamma: float = 0.5,
                 clean_every: int = 10, scissors: float = 0.0, precision: int = BSE_MIXED,
                 device: int = 0, max_batch: int = 16):
        cfg = BseConfig(n, n, n, h, n_occ, n_stoch, seed, dt, n_steps, gamma, clean_every,
                        0.0, scissors, precision, device, max_batch)
        self.cfg = cfg
        self.n = n
        self.ng = n ** 3
        v = np.ascontiguousarray(v_ext, dtype=np.float64).reshape(-1)
        if v.size != self.ng:
            raise ValueError("v_ext size does not match the grid")
        h_ = C.c_void_p()
        _check(LIB.bse_create_system(C.byref(cfg), _dptr(v), C.byref(h_)))
        self._h = h_

    def close(self):
        # LIB is None once the interpreter is tearing the module down
        if getattr(self, "_h", None) and LIB is not None:
            LIB.bse_destroy_system(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def set_signs(self, xi: np.ndarray):
        x = np.ascontiguousarray(xi, dtype=np.int8)
        _check(LIB.bse_set_signs(self._h, x.shape[0], x.shape[1], x.ctypes.data_as(C.POINTER(C.c_int8))))

    def set_orbitals(self, phi: np.ndarray, eps: np.ndarray):
        p = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1, self.ng)
        e = np.ascontiguousarray(eps, dtype=np.float64).reshape(-1)
        if e.size != p.shape[0]:
            raise ValueError("eps and phi disagree on the orbital count")
        _check(LIB.bse_set_orbitals(self._h, p.shape[0], _dptr(p), _dptr(e)))

    def set_stream(self, stream_ptr: int):
        _check(LIB.bse_set_stream(self._h, C.c_void_p(stream_ptr)))

    def apply_w(self, pairs, want_wpol: bool = False, return_status: bool = False):
        pq = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
        B = pq.shape[0]
        w = np.empty((B, self.ng))
        wp = np.empty((B, self.ng)) if want_wpol else None
        st = np.zeros(B, dtype=np.int32)
        rc = LIB.bse_apply_W(self._h, B, _iptr(pq), _dptr(w), _dptr(wp) if wp is not None else None,
                             _iptr(st))
        if rc != BSE_OK and not (return_status and rc == BSE_ERR_NUMERIC):
            _check(rc)
        out = (w, wp) if want_wpol else (w,)
        if return_status:
            out = out + (st,)
        return out if len(out) > 1 else out[0]

    def apply_w_device(self, pq_dev, w_dev):
        """bse_apply_W_device: pq_dev a contiguous int32 device tensor [n][2],
        w_dev a contiguous float64 (BSE_F64) or float32 (BSE_F32) device
        tensor [n][ng]; stream-ordered on the stream of set_stream."""
        if pq_dev.dtype != torch.int32 or pq_dev.dim() != 2 or pq_dev.shape[1] != 2 or not pq_dev.is_contiguous():
            raise ValueError("pq_dev must be a contiguous int32 tensor [n][2]")
        n = pq_dev.shape[0]
        if tuple(w_dev.shape) != (n, self.ng) or not w_dev.is_contiguous():
            raise ValueError("w_dev must be a contiguous tensor [n][ng]")
        if w_dev.dtype == torch.float64:
            dt = BSE_F64
        elif w_dev.dtype == torch.float32:
            dt = BSE_F32
        else:
            raise ValueError("w_dev must be float64 or float32")
        _check(LIB.bse_apply_W_device(self._h, n, C.c_void_p(pq_dev.data_ptr()), C.c_void_p(w_dev.data_ptr()),
                                      dt))

    def inject_fault(self, index: int, point: int, value: float, unperturbed: bool = False):
        """bse_inject_fault: one value of the device copy of orbital ``index``
        (or of the t = 0 unperturbed stochastic orbital ``index``), bypassing
        the input checks (tests of the failure path)."""
        _check(LIB.bse_inject_fault(self._h, 1 if unperturbed else 0, int(index), int(point), float(value)))

    def build_a(self, n_o: int, n_c: int) -> np.ndarray:
        A = np.empty((n_o * n_c, n_o * n_c))
        _check(LIB.bse_build_A(self._h, n_o, n_c, _dptr(A)))
        self.a_window = (n_o, n_c)
        return A

    def valence_w(self) -> np.ndarray:
        """bse_valence_W: the W_ij of the last build_a, [n_o(n_o+1)/2][ng]."""
        n_o = getattr(self, "a_window", (0, 0))[0]
        w = np.empty((n_o * (n_o + 1) // 2, self.ng))
        _check(LIB.bse_valence_W(self._h, _dptr(w)))
        return w

    def apply_a_mixed(self, f: np.ndarray) -> np.ndarray:
        """A f in the mixed representation; f [n_vec][n_o][ng] or [n_o][ng]."""
        x = np.ascontiguousarray(f, dtype=np.float64)
        one = x.ndim == 2
        if one:
            x = x[None]
        out = np.empty_like(x)
        _check(LIB.bse_apply_A_mixed(self._h, x.shape[0], _dptr(x), _dptr(out)))
        return out[0] if one else out

    def chebyshev_mixed(self, n_mom: int, bounds, w_grid=None,
                        sigma: float = 0.08 / 27.211386245988):
        """(sigma on w_grid or None, residues [3][n_mom]) of the mixed
        representation; bounds = (e_min, e_max) of A on the virtual space."""
        res = np.empty((3, n_mom))
        lo, hi = float(bounds[0]), float(bounds[1])
        if w_grid is None:
            _check(LIB.bse_chebyshev_mixed(self._h, n_mom, lo, hi, 0, None, sigma, None, _dptr(res)))
            return None, res
        wg = np.ascontiguousarray(w_grid, dtype=np.float64)
        sg = np.empty(wg.size)
        _check(LIB.bse_chebyshev_mixed(self._h, n_mom, lo, hi, wg.size, _dptr(wg), sigma, _dptr(sg),
                                       _dptr(res)))
        return sg, res

    def exciton_states(self, n_mom: int, w_list, sigma: float = 0.08 / 27.211386245988, bounds=None,
                       densities: bool = True):
        """Frequency-resolved exciton states (Eq. 8) of the last A:
        (F [n_w][3][n_o n_c], densities [n_w][3][nx, ny, nz] or None,
        interval used)."""
        wl = np.ascontiguousarray(w_list, dtype=np.float64).reshape(-1)
        n_o, n_c = getattr(self, "a_window", (0, 0))
        F = np.empty((wl.size, 3, max(1, n_o * n_c)))
        dn = np.empty((wl.size, 3, self.n, self.n, self.n)) if densities else None
        bo = np.empty(2)
        lo, hi = (0.0, 0.0) if bounds is None else bounds
        _check(LIB.bse_exciton_states(self._h, n_mom, lo, hi, wl.size, _dptr(wl), sigma, _dptr(F),
                                      _dptr(dn) if densities else None, _dptr(bo)))
        return F, dn, bo

    def exciton_states_mixed(self, n_mom: int, bounds, w_list, sigma: float = 0.08 / 27.211386245988,
                             n_a: int = 0, densities: bool = True):
        """Exciton states of the mixed representation (Eq. 8 with Eq. 6):
        (amplitudes [n_w][3][n_o][n_a] or None, densities [n_w][3][nx, ny, nz]
        or None); bounds = (e_min, e_max) of A on the virtual space."""
        wl = np.ascontiguousarray(w_list, dtype=np.float64).reshape(-1)
        n_o = getattr(self, "a_window", (1, 0))[0]
        amp = np.empty((wl.size, 3, n_o, n_a)) if n_a > 0 else None
        dn = np.empty((wl.size, 3, self.n, self.n, self.n)) if densities else None
        _check(LIB.bse_exciton_states_mixed(self._h, n_mom, float(bounds[0]), float(bounds[1]), wl.size,
                                            _dptr(wl), sigma, n_a, _dptr(amp) if amp is not None else None,
                                            _dptr(dn) if dn is not None else None))
        return amp, dn

    def chebyshev_spectrum(self, n_mom: int, w_grid=None, sigma: float = 0.08 / 27.211386245988,
                           bounds=None):
        """(sigma on w_grid or None, residues [3][n_mom], interval used)."""
        res = np.empty((3, n_mom))
        bo = np.empty(2)
        lo, hi = (0.0, 0.0) if bounds is None else (float(bounds[0]), float(bounds[1]))
        if w_grid is None:
            _check(LIB.bse_chebyshev_spectrum(self._h, n_mom, lo, hi, 0, None, sigma, None,
                                              _dptr(res), _dptr(bo)))
            return None, res, bo
        wg = np.ascontiguousarray(w_grid, dtype=np.float64)
        sg = np.empty(wg.size)
        _check(LIB.bse_chebyshev_spectrum(self._h, n_mom, lo, hi, wg.size, _dptr(wg), sigma, _dptr(sg),
                                          _dptr(res), _dptr(bo)))
        return sg, res, bo

    def chebyshev_spectrum_noalloc(self, n_mom: int, w_grid=None, sigma: float = 0.08 / 27.211386245988,
                                   bounds=None):
        """bse_chebyshev_spectrum_noalloc: as chebyshev_spectrum, with the
        library's fixed device scratch instead of allocations."""
        res = np.empty((3, n_mom))
        bo = np.empty(2)
        lo, hi = (0.0, 0.0) if bounds is None else (float(bounds[0]), float(bounds[1]))
        if w_grid is None:
            _check(LIB.bse_chebyshev_spectrum_noalloc(self._h, n_mom, lo, hi, 0, None, sigma, None,
                                                      _dptr(res), _dptr(bo)))
            return None, res, bo
        wg = np.ascontiguousarray(w_grid, dtype=np.float64)
        sg = np.empty(wg.size)
        _check(LIB.bse_chebyshev_spectrum_noalloc(self._h, n_mom, lo, hi, wg.size, _dptr(wg), sigma,
                                                  _dptr(sg), _dptr(res), _dptr(bo)))
        return sg, res, bo

    def spectrum(self, n_exc: int, w_grid=None, sigma: float = 0.08 / 27.211386245988):
        om = np.empty(n_exc)
        d2 = np.empty((n_exc, 3))
        if w_grid is None:
            _check(LIB.bse_spectrum(self._h, n_exc, _dptr(om), _dptr(d2), 0, None, sigma, None))
            return om, d2
        wg = np.ascontiguousarray(w_grid, dtype=np.float64)
        sg = np.empty(wg.size)
        _check(LIB.bse_spectrum(self._h, n_exc, _dptr(om), _dptr(d2), wg.size, _dptr(wg), sigma,
                                _dptr(sg)))
        return om, d2, sg

    def autotune(self, n_pairs: int, cache_path: Optional[str] = None):
        _check(LIB.bse_autotune(self._h, n_pairs, cache_path.encode() if cache_path else None))
        tc, nt = C.c_int32(), C.c_int32()
        LIB.bse_tuned_shape(self._h, C.byref(tc), C.byref(nt))
        return tc.value, nt.value

    def set_timing(self, on=True):
        """False/0 off; 1 the propagation passes and contractions; True/2 all."""
        level = 2 if on is True else (0 if on is False else int(on))
        _check(LIB.bse_set_timing(self._h, level))

    def boundary_potential(self) -> float:
        """v_bndry of this box (bse_boundary_potential)."""
        v = C.c_double()
        _check(LIB.bse_boundary_potential(self._h, C.byref(v)))
        return v.value

    def set_launch_order(self, order: int):
        """bse_set_launch_order: bit 0 XCD-grouped x pass, bit 1 y-line pass, bit 2 fused y-z pass."""
        _check(LIB.bse_set_launch_order(self._h, int(order)))

    def set_yz_schedule(self, schedule: int):
        """bse_set_yz_schedule: 2 (default) plane pass, DFT16 per lane; 0 cross-lane DFT16; 1 two line passes."""
        _check(LIB.bse_set_yz_schedule(self._h, int(schedule)))

    def set_lanczos_path(self, path):
        """0: single-workgroup launches up to each convergence check where A
        pays (n <= 384); 1: a chip-wide launch per operation."""
        _check(LIB.bse_set_lanczos_path(self._h, int(path)))

    def kernel_times(self):
        cap = 32
        names = (C.c_char_p * cap)()
        avg = np.zeros(cap)
        calls = np.zeros(cap, dtype=np.int32)
        k = LIB.bse_kernel_times(self._h, cap, names, _dptr(avg), _iptr(calls))
        if k < 0:
            raise BseError(BSE_ERR_DEVICE, LIB.bse_last_error().decode())
        return {names[i].decode(): (float(avg[i]), int(calls[i])) for i in range(k)}


def _fcheck(rc: int):
    if rc != BSE_OK:
        raise BseError(rc, LIB.bse_fno_last_error().decode())


class Fno:
    """The screening surrogate (bse_fno handle); buffers are device pointers."""

    def __init__(self, n: int, cin: int = 3, width: int = 32, modes: int = 8, layers: int = 4,
                 max_batch: int = 8, device: int = 0, bf16_weights: bool = True, seed: int = 0):
        cfg = FnoConfig(n, cin, width, modes, layers, max_batch, device, 1 if bf16_weights else 0, seed)
        h = C.c_void_p()
        _fcheck(LIB.bse_fno_create(C.byref(cfg), C.byref(h)))
        self._h = h
        self.cfg = cfg
        self.n_params = int(LIB.bse_fno_num_params(h))

    def close(self):
        if getattr(self, "_h", None) and LIB is not None:
            LIB.bse_fno_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def set_params(self, flat: np.ndarray):
        f = np.ascontiguousarray(flat, dtype=np.float32)
        if f.size != self.n_params:
            raise ValueError("parameter vector size")
        _fcheck(LIB.bse_fno_set_params(self._h, f.ctypes.data_as(C.POINTER(C.c_float))))

    def get_params(self, compute: bool = False) -> np.ndarray:
        f = np.empty(self.n_params, dtype=np.float32)
        _fcheck(LIB.bse_fno_get_params(self._h, f.ctypes.data_as(C.POINTER(C.c_float)), 1 if compute else 0))
        return f

    def set_stream(self, stream_ptr: int):
        _fcheck(LIB.bse_fno_set_stream(self._h, C.c_void_p(stream_ptr)))

    def set_mix_path(self, path: int):
        """bse_fno_set_mix_path: 0 matrix cores, 1 vector FMA."""
        _fcheck(LIB.bse_fno_set_mix_path(self._h, int(path)))

    def forward(self, B: int, x_ptr: int, y_ptr: int):
        _fcheck(LIB.bse_fno_forward(self._h, B, C.c_void_p(x_ptr), C.c_void_p(y_ptr)))

    def loss_grad(self, B: int, x_ptr: int, t_ptr: int, want_grad: bool = True):
        loss = C.c_double()
        g = np.empty(self.n_params, dtype=np.float32) if want_grad else None
        _fcheck(LIB.bse_fno_loss_grad(self._h, B, C.c_void_p(x_ptr), C.c_void_p(t_ptr), C.byref(loss),
                                      g.ctypes.data_as(C.POINTER(C.c_float)) if g is not None else None))
        return loss.value, g

    def gather(self, idx, n_src: int, x_src_ptr: int, t_src_ptr: int, perm, flip_mask: int,
               x_dst_ptr: int, t_dst_ptr: int):
        """bse_fno_gather: samples idx of the source batch under a symmetry of
        the cube (output axis k = input axis perm[k], axes in flip_mask
        reversed) into the destination buffers."""
        ix = np.ascontiguousarray(np.asarray(idx, dtype=np.int32))
        pm = np.ascontiguousarray(np.asarray(perm, dtype=np.int32))
        _fcheck(LIB.bse_fno_gather(self._h, int(ix.shape[0]), _iptr(ix), int(n_src), C.c_void_p(x_src_ptr),
                                   C.c_void_p(t_src_ptr), _iptr(pm), int(flip_mask), C.c_void_p(x_dst_ptr),
                                   C.c_void_p(t_dst_ptr)))

    def train_step(self, B: int, x_ptr: int, t_ptr: int, lr: float) -> float:
        loss = C.c_double()
        _fcheck(LIB.bse_fno_train_step(self._h, B, C.c_void_p(x_ptr), C.c_void_p(t_ptr), lr, C.byref(loss)))
        return loss.value


def make_samples(system: "System", pairs, x_ptr: int, t_ptr: Optional[int] = None,
                 scale_ptr: Optional[int] = None):
    """Surrogate inputs (and propagated targets) for a system's pairs
    (bse_fno_make_samples)."""
    pq = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    _check(LIB.bse_fno_make_samples(system._h, pq.shape[0], _iptr(pq), C.c_void_p(x_ptr),
                                    C.c_void_p(t_ptr) if t_ptr else None,
                                    C.c_void_p(scale_ptr) if scale_ptr else None))


def apply_w_surrogate(system: "System", net: "Fno", pairs, w_ptr: int, tol: float = 1e-3, n_judge: int = 4):
    """Surrogate W-action judged by the propagation (bse_apply_W_surrogate):
    returns (accepted flags [n_pairs], measured errors of the judged pairs)."""
    pq = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    acc = np.zeros(pq.shape[0], dtype=np.int32)
    err = np.zeros(max(int(n_judge), 1))
    _check(LIB.bse_apply_W_surrogate(system._h, net._h, pq.shape[0], _iptr(pq), C.c_void_p(w_ptr),
                                     float(tol), int(n_judge), _iptr(acc), _dptr(err)))
    return acc, err[:int(n_judge)]
