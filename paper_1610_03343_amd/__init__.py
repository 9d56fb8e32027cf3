"""Python binding of libmbmd (include/mbmd.h): argument marshalling only.

Every step of the force path runs in the HIP kernels of libmbmd.so; this
module only checks tensor shapes/dtypes/devices, passes raw device pointers
and the current torch stream, and turns status codes into exceptions.  It
raises at import time if the library has not been built: there is no CPU
fallback.

Device arrays are torch tensors of dtype float64 on a HIP device, in the
library's structure-of-arrays layout: positions/velocities/forces/heat
current (3, n), energy (n,), virial (9, n) with row 3*alpha + beta.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmbmd.so")

MBMD_OK, MBMD_EINVAL, MBMD_ENOMEM, MBMD_EDEVICE, MBMD_EBOX = 0, 1, 2, 3, 4
MBMD_ENEIGH, MBMD_ESKIN, MBMD_ENONFINITE, MBMD_ENOPOT, MBMD_EBUSY = 5, 6, 7, 8, 9
MBMD_FP64, MBMD_MIXED = 0, 1
STATUS_NAMES = {0: "MBMD_OK", 1: "MBMD_EINVAL", 2: "MBMD_ENOMEM", 3: "MBMD_EDEVICE",
                4: "MBMD_EBOX", 5: "MBMD_ENEIGH", 6: "MBMD_ESKIN", 7: "MBMD_ENONFINITE",
                8: "MBMD_ENOPOT", 9: "MBMD_EBUSY"}
THERMO_COLS = 16
MBMD_REBUILD_FIXED, MBMD_REBUILD_ON_SKIN = 0, 1


class MbmdError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {message}")
        self.code = code


class mbmd_tersoff_params(C.Structure):
    _fields_ = [(k, C.c_double) for k in
                ("A", "B", "lambda_", "mu", "beta", "n", "c", "d", "h", "R", "S")]


class mbmd_sw_params(C.Structure):
    _fields_ = [(k, C.c_double) for k in
                ("epsilon", "sigma", "a", "lambda_", "gamma", "A", "B", "p", "q")]


class mbmd_run_stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("rebuilds", C.c_int64), ("rollbacks", C.c_int64),
                ("max_displacement", C.c_double)]


class mbmd_berendsen(C.Structure):
    _fields_ = [(k, C.c_double) for k in
                ("T0_K", "tau_T_fs", "P0_GPa", "tau_P_fs", "beta_per_GPa")]


class mbmd_kernel_time(C.Structure):
    _fields_ = [("name", C.c_char_p), ("launches", C.c_int64), ("total_ms", C.c_double)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python paper_1610_03343_amd/build.py` (hipcc, gfx950)")
    lib = C.CDLL(LIB_PATH)
    P, I64, D, I = C.c_void_p, C.c_int64, C.c_double, C.c_int
    sig = {
        "mbmd_create": ([C.POINTER(P), I, P], I),
        "mbmd_destroy": ([P], None),
        "mbmd_last_error": ([P], C.c_char_p),
        "mbmd_set_tersoff": ([P, C.POINTER(mbmd_tersoff_params)], I),
        "mbmd_set_sw": ([P, C.POINTER(mbmd_sw_params)], I),
        "mbmd_set_tersoff_multi": ([P, I, P, P], I),
        "mbmd_set_type_masses": ([P, I, P], I),
        "mbmd_set_neighbor": ([P, D, I], I),
        "mbmd_get_max_neighbors": ([P, C.POINTER(I)], I),
        "mbmd_set_rebuild_policy": ([P, I], I),
        "mbmd_get_run_stats": ([P, C.POINTER(mbmd_run_stats)], I),
        "mbmd_set_profiling": ([P, I], I),
        "mbmd_reset_profile": ([P], I),
        "mbmd_get_profile": ([P, C.POINTER(mbmd_kernel_time), I, C.POINTER(I)], I),
        "mbmd_workspace_size": ([P, I64, C.POINTER(C.c_size_t)], I),
        "mbmd_bind_workspace": ([P, P, C.c_size_t], I),
        "mbmd_neighbors": ([P, I64, P, P, P, P, P], I),
        "mbmd_compute": ([P, I, I64, P, P, P, P, P, P, P, P], I),
        "mbmd_compute_noalloc": ([P, I, I64, P, P, P, P, P, P, P, P], I),
        "mbmd_nve_run": ([P, I, I64, P, D, P, P, P, D, I, I, P, P, P, P, P], I),
        "mbmd_nve_continue": ([P, I, I64, P, D, P, P, P, D, I, I, P, P, P, P, P], I),
        "mbmd_npt_run": ([P, I, I64, P, D, P, P, P, D, I, I, C.POINTER(mbmd_berendsen), P, P,
                          P, P, P, P], I),
        "mbmd_green_kubo": ([P, P, I64, I, I, D, D, D, P, P], I),
        "mbmd_batch_open": ([P, I64, I, I], I),
        "mbmd_batch_workspace_size": ([P, I64, I, C.POINTER(C.c_size_t)], I),
        "mbmd_batch_capacity": ([P, C.POINTER(I64), C.POINTER(I), C.POINTER(I64)], I),
        "mbmd_batch_add": ([P, I64, P, P, P, D, D, I, P, C.POINTER(I)], I),
        "mbmd_batch_step": ([P, I, C.POINTER(I)], I),
        "mbmd_batch_finished": ([P, C.POINTER(I), I, C.POINTER(I)], I),
        "mbmd_batch_retire": ([P, I, P, P, P, P, P, P, P], I),
        "mbmd_batch_sync": ([P], I),
        "mbmd_sync": ([P], I),
        "mbmd_batch_close": ([P], I),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()


def lib():
    return _lib


def _dptr(t, shape, name, dtype=torch.float64):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or not t.is_cuda:
        raise TypeError(f"{name} must be a {dtype} tensor on a HIP device")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


def _box(box):
    b = (C.c_double * 3)(*[float(x) for x in box])
    return b


def tersoff_struct(p: dict) -> mbmd_tersoff_params:
    return mbmd_tersoff_params(p["A"], p["B"], p["lam"], p["mu"], p["beta"], p["n"], p["c"],
                               p["d"], p["h"], p["R"], p["S"])


def sw_struct(p: dict) -> mbmd_sw_params:
    return mbmd_sw_params(p["epsilon"], p["sigma"], p["a"], p["lam"], p["gamma"], p["A"], p["B"],
                          p["p"], p["q"])


def _prec(precision) -> int:
    if precision in ("fp64", MBMD_FP64):
        return MBMD_FP64
    if precision in ("mixed", MBMD_MIXED):
        return MBMD_MIXED
    raise ValueError(f"precision must be 'fp64' or 'mixed', not {precision!r}")


class Context:
    """One mbmd_ctx on a device, enqueuing on a torch stream."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        self._check(_lib.mbmd_create(C.byref(h), device, C.c_void_p(self.stream.cuda_stream)),
                    "mbmd_create", ctx=None)
        self._h = h
        self._ws = None

    def close(self):
        # at interpreter exit the module's globals may already be gone
        if getattr(self, "_h", None) and _lib is not None:
            _lib.mbmd_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, code, what, ctx="self"):
        if code != MBMD_OK:
            msg = what
            if ctx is not None and getattr(self, "_h", None):
                msg = f"{what}: {_lib.mbmd_last_error(self._h).decode()}"
            raise MbmdError(code, msg)

    # -- configuration ------------------------------------------------------
    def set_tersoff(self, params: dict):
        st = tersoff_struct(params)
        self._check(_lib.mbmd_set_tersoff(self._h, C.byref(st)), "mbmd_set_tersoff")

    def set_tersoff_multi(self, elems, chi=None):
        """Multicomponent Tersoff: elems = [param dict per type], chi an
        (ntypes, ntypes) symmetric array or None (all 1)."""
        nt = len(elems)
        arr = (mbmd_tersoff_params * nt)(*[tersoff_struct(e) for e in elems])
        ch = None
        if chi is not None:
            flat = [float(x) for row in chi for x in row]
            if len(flat) != nt * nt:
                raise ValueError("chi must be ntypes x ntypes")
            ch = (C.c_double * (nt * nt))(*flat)
        self._check(_lib.mbmd_set_tersoff_multi(self._h, nt, C.cast(arr, C.c_void_p),
                                                C.cast(ch, C.c_void_p) if ch else None),
                    "mbmd_set_tersoff_multi")

    def set_type_masses(self, masses):
        """Per-type masses (amu) for runs with mass 0; None or [] clears."""
        m = [float(x) for x in (masses or [])]
        arr = (C.c_double * max(len(m), 1))(*m) if m else None
        self._check(_lib.mbmd_set_type_masses(self._h, len(m),
                                              C.cast(arr, C.c_void_p) if arr else None),
                    "mbmd_set_type_masses")

    def set_sw(self, params: dict):
        st = sw_struct(params)
        self._check(_lib.mbmd_set_sw(self._h, C.byref(st)), "mbmd_set_sw")

    def set_neighbor(self, skin: float = 0.5, max_neighbors: int = 0):
        self._check(_lib.mbmd_set_neighbor(self._h, float(skin), int(max_neighbors)),
                    "mbmd_set_neighbor")

    def set_rebuild_policy(self, policy):
        """'fixed' (every rebuild_every steps only) or 'skin' (also when an
        atom moved more than skin/2 since the last build)."""
        code = {"fixed": MBMD_REBUILD_FIXED, "skin": MBMD_REBUILD_ON_SKIN}.get(policy, policy)
        self._check(_lib.mbmd_set_rebuild_policy(self._h, int(code)), "mbmd_set_rebuild_policy")

    def run_stats(self) -> dict:
        st = mbmd_run_stats()
        self._check(_lib.mbmd_get_run_stats(self._h, C.byref(st)), "mbmd_get_run_stats")
        return dict(steps=st.steps, rebuilds=st.rebuilds, rollbacks=st.rollbacks,
                    max_displacement=st.max_displacement)

    def set_profiling(self, enable: bool = True):
        self._check(_lib.mbmd_set_profiling(self._h, int(bool(enable))), "mbmd_set_profiling")

    def reset_profile(self):
        self._check(_lib.mbmd_reset_profile(self._h), "mbmd_reset_profile")

    def profile(self) -> dict:
        """{kernel class: (launches, total device ms)} from HIP events."""
        arr = (mbmd_kernel_time * 16)()
        cnt = C.c_int()
        self._check(_lib.mbmd_get_profile(self._h, arr, 16, C.byref(cnt)), "mbmd_get_profile")
        return {arr[k].name.decode(): (arr[k].launches, arr[k].total_ms)
                for k in range(min(cnt.value, 16))}

    @property
    def max_neighbors(self) -> int:
        v = C.c_int()
        self._check(_lib.mbmd_get_max_neighbors(self._h, C.byref(v)), "mbmd_get_max_neighbors")
        return v.value

    def workspace_size(self, n: int) -> int:
        v = C.c_size_t()
        self._check(_lib.mbmd_workspace_size(self._h, int(n), C.byref(v)), "mbmd_workspace_size")
        return v.value

    def bind_workspace(self, buf: torch.Tensor | None):
        """Bind a caller-owned uint8 device tensor as workspace (None unbinds)."""
        if buf is None:
            self._check(_lib.mbmd_bind_workspace(self._h, None, 0), "mbmd_bind_workspace")
            self._ws = None
            return
        if buf.dtype != torch.uint8 or not buf.is_cuda or not buf.is_contiguous():
            raise TypeError("workspace must be a contiguous uint8 tensor on a HIP device")
        self._check(_lib.mbmd_bind_workspace(self._h, C.c_void_p(buf.data_ptr()), buf.numel()),
                    "mbmd_bind_workspace")
        self._ws = buf

    # -- calls --------------------------------------------------------------
    def neighbors(self, pos: torch.Tensor, box, types=None, allow_overflow=False):
        """(nn, nl) of mbmd_neighbors.  A list longer than max_neighbors
        raises MBMD_ENEIGH, unless allow_overflow: then the arrays are
        returned as the call left them (true counts, the first entries)."""
        n = pos.shape[1]
        M = self.max_neighbors
        nn = torch.zeros(n, dtype=torch.int32, device=self.device)
        nl = torch.full((M, n), -1, dtype=torch.int32, device=self.device)
        code = _lib.mbmd_neighbors(self._h, n, _box(box), _dptr(pos, (3, n), "pos"),
                                   _dptr(types, (n,), "types", torch.int32),
                                   _dptr(nn, (n,), "nn", torch.int32),
                                   _dptr(nl, (M, n), "nl", torch.int32))
        if not (allow_overflow and code == MBMD_ENEIGH):
            self._check(code, "mbmd_neighbors")
        return nn, nl

    def _outputs(self, n, out):
        if out is None:
            z = lambda *s: torch.empty(*s, dtype=torch.float64, device=self.device)
            out = dict(U=z(n), F=z(3, n), W=z(9, n), J=z(3, n))
        return out

    def compute(self, pos, box, vel=None, types=None, precision="fp64", out=None):
        n = pos.shape[1]
        out = self._outputs(n, out)
        self._check(_lib.mbmd_compute(
            self._h, _prec(precision), n, _box(box), _dptr(pos, (3, n), "pos"),
            _dptr(vel, (3, n), "vel"), _dptr(types, (n,), "types", torch.int32),
            _dptr(out["U"], (n,), "U"), _dptr(out["F"], (3, n), "F"),
            _dptr(out["W"], (9, n), "W"), _dptr(out["J"], (3, n), "J")), "mbmd_compute")
        return out

    def compute_noalloc(self, pos, box, out, vel=None, types=None, precision="fp64"):
        """mbmd_compute_noalloc: the single point of compute() with the
        workspace in the library's static device scratch; allocates nothing,
        so the caller passes the outputs (dict U, F, W, J)."""
        n = pos.shape[1]
        self._check(_lib.mbmd_compute_noalloc(
            self._h, _prec(precision), n, _box(box), _dptr(pos, (3, n), "pos"),
            _dptr(vel, (3, n), "vel"), _dptr(types, (n,), "types", torch.int32),
            _dptr(out["U"], (n,), "U"), _dptr(out["F"], (3, n), "F"),
            _dptr(out["W"], (9, n), "W"), _dptr(out["J"], (3, n), "J")),
            "mbmd_compute_noalloc")
        return out

    def nve_run(self, pos, vel, box, mass, dt, n_steps, rebuild_every=20, types=None,
                precision="fp64", thermo=True, out=None, cont=False):
        """Advances pos/vel in place; returns dict(U, F, W, J[, thermo]).
        cont=True continues the previous run on this context
        (mbmd_nve_continue): the same pos, vel, types and out["F"] tensors,
        box, mass, dt, rebuild_every and precision."""
        n = pos.shape[1]
        out = self._outputs(n, out)
        th = None
        if thermo is True:
            th = torch.empty(n_steps + 1, THERMO_COLS, dtype=torch.float64, device=self.device)
        elif isinstance(thermo, torch.Tensor):
            th = thermo
        fn = _lib.mbmd_nve_continue if cont else _lib.mbmd_nve_run
        self._check(fn(
            self._h, _prec(precision), n, _box(box), float(mass), _dptr(pos, (3, n), "pos"),
            _dptr(vel, (3, n), "vel"), _dptr(types, (n,), "types", torch.int32), float(dt),
            int(n_steps), int(rebuild_every), _dptr(out["U"], (n,), "U"),
            _dptr(out["F"], (3, n), "F"), _dptr(out["W"], (9, n), "W"),
            _dptr(out["J"], (3, n), "J"),
            _dptr(th, (n_steps + 1, THERMO_COLS), "thermo") if th is not None else None),
            "mbmd_nve_continue" if cont else "mbmd_nve_run")
        if th is not None:
            out["thermo"] = th
        return out

    def npt_run(self, pos, vel, box, mass, dt, n_steps, rebuild_every=20, T0=300.0,
                tau_T=100.0, P0_GPa=0.0, tau_P=1000.0, beta_per_GPa=0.0102, types=None,
                precision="fp64", thermo=None, box_traj=True, out=None):
        """Velocity-Verlet with Berendsen weak coupling (mbmd_npt_run); tau <= 0
        switches a coupling off.  Advances pos/vel in place; returns dict(U, F,
        W, J, thermo, box (final edges, numpy)[, box_traj])."""
        import numpy as np
        n = pos.shape[1]
        out = self._outputs(n, out)
        th = thermo if isinstance(thermo, torch.Tensor) else torch.empty(
            n_steps + 1, THERMO_COLS, dtype=torch.float64, device=self.device)
        bt = None
        if box_traj is True:
            bt = torch.empty(n_steps + 1, 3, dtype=torch.float64, device=self.device)
        elif isinstance(box_traj, torch.Tensor):
            bt = box_traj
        k = mbmd_berendsen(float(T0), float(tau_T), float(P0_GPa), float(tau_P),
                           float(beta_per_GPa))
        b = _box(box)
        self._check(_lib.mbmd_npt_run(
            self._h, _prec(precision), n, b, float(mass), _dptr(pos, (3, n), "pos"),
            _dptr(vel, (3, n), "vel"), _dptr(types, (n,), "types", torch.int32), float(dt),
            int(n_steps), int(rebuild_every), C.byref(k), _dptr(out["U"], (n,), "U"),
            _dptr(out["F"], (3, n), "F"), _dptr(out["W"], (9, n), "W"),
            _dptr(out["J"], (3, n), "J"), _dptr(th, (n_steps + 1, THERMO_COLS), "thermo"),
            _dptr(bt, (n_steps + 1, 3), "box_traj") if bt is not None else None),
            "mbmd_npt_run")
        out["thermo"] = th
        out["box"] = np.array([b[0], b[1], b[2]])
        if bt is not None:
            out["box_traj"] = bt
        return out

    def green_kubo(self, thermo, sample_every, max_lag, dt, volume, T, kappa=True):
        """Heat-current autocorrelation and running Green-Kubo conductivity
        (mbmd_green_kubo) from thermo rows on the device; returns dict(hac,
        kappa) of (max_lag, 3) device tensors."""
        n_rows = thermo.shape[0]
        hac = torch.empty(max_lag, 3, dtype=torch.float64, device=self.device)
        kap = torch.empty(max_lag, 3, dtype=torch.float64, device=self.device) if kappa else None
        self._check(_lib.mbmd_green_kubo(
            self._h, _dptr(thermo, (n_rows, THERMO_COLS), "thermo"), int(n_rows),
            int(sample_every), int(max_lag), float(dt), float(volume), float(T),
            _dptr(hac, (max_lag, 3), "hac"),
            _dptr(kap, (max_lag, 3), "kappa") if kap is not None else None), "mbmd_green_kubo")
        out = {"hac": hac}
        if kap is not None:
            out["kappa"] = kap
        return out

    # -- serving batch --------------------------------------------------------
    def batch_workspace_size(self, max_atoms: int, max_structures: int) -> int:
        v = C.c_size_t()
        self._check(_lib.mbmd_batch_workspace_size(self._h, int(max_atoms), int(max_structures),
                                                   C.byref(v)), "mbmd_batch_workspace_size")
        return v.value

    def batch_open(self, max_atoms: int, max_structures: int, rebuild_every: int = 10):
        self._check(_lib.mbmd_batch_open(self._h, int(max_atoms), int(max_structures),
                                         int(rebuild_every)), "mbmd_batch_open")
        self._batch_keep = {}
        self._batch_fin = (C.c_int * int(max_structures))()

    def batch_close(self):
        self._check(_lib.mbmd_batch_close(self._h), "mbmd_batch_close")
        self._batch_keep = {}

    def batch_capacity(self):
        """(free atoms, free structure slots, largest contiguous free range)."""
        fa, fs, lr = C.c_int64(), C.c_int(), C.c_int64()
        self._check(_lib.mbmd_batch_capacity(self._h, C.byref(fa), C.byref(fs), C.byref(lr)),
                    "mbmd_batch_capacity")
        return fa.value, fs.value, lr.value

    def batch_add(self, pos, vel, box, mass, dt, n_steps, thermo=None) -> int:
        """Admit a structure; returns its handle (raises MbmdError EBUSY if no room)."""
        n = pos.shape[1]
        th = thermo
        h = C.c_int()
        self._check(_lib.mbmd_batch_add(
            self._h, n, _box(box), _dptr(pos, (3, n), "pos"), _dptr(vel, (3, n), "vel"),
            float(mass), float(dt), int(n_steps),
            _dptr(th, (n_steps + 1, THERMO_COLS), "thermo") if th is not None else None,
            C.byref(h)), "mbmd_batch_add")
        if th is not None:
            self._batch_keep[h.value] = th      # the library writes into it while it runs
        return h.value

    def batch_step(self, precision="fp64") -> int:
        a = C.c_int()
        self._check(_lib.mbmd_batch_step(self._h, _prec(precision), C.byref(a)), "mbmd_batch_step")
        return a.value

    def batch_finished(self):
        cnt = C.c_int()
        arr = self._batch_fin
        self._check(_lib.mbmd_batch_finished(self._h, arr, len(arr), C.byref(cnt)),
                    "mbmd_batch_finished")
        if cnt.value > len(arr):
            arr = self._batch_fin = (C.c_int * cnt.value)()
            self._check(_lib.mbmd_batch_finished(self._h, arr, len(arr), C.byref(cnt)),
                        "mbmd_batch_finished")
        return list(arr[: cnt.value])

    def sync(self):
        """Wait for the context's stream; raises MbmdError on a device status."""
        self._check(_lib.mbmd_sync(self._h), "mbmd_sync")

    def batch_sync(self):
        """Wait for the stream; raises MbmdError on a batch-wide error status."""
        self._check(_lib.mbmd_batch_sync(self._h), "mbmd_batch_sync")

    def batch_retire(self, handle: int, n: int, out=None, status=None):
        """Enqueue the copy of a finished structure's final pos, vel, U, F, W,
        J into `out` (allocated if None) and free its slot; the values are
        there once the stream reaches this point (batch_sync).  `status` (an
        int32 device tensor of one element, allocated if None, returned as
        out["status"]) receives the structure's own status code at the same
        point (MBMD_OK, MBMD_ENONFINITE, MBMD_ENEIGH or MBMD_ESKIN)."""
        if out is None:
            z = lambda *s: torch.empty(*s, dtype=torch.float64, device=self.device)
            out = dict(pos=z(3, n), vel=z(3, n), U=z(n), F=z(3, n), W=z(9, n), J=z(3, n))
        if status is None:
            status = torch.empty(1, dtype=torch.int32, device=self.device)
        self._check(_lib.mbmd_batch_retire(
            self._h, int(handle), _dptr(out["pos"], (3, n), "pos"), _dptr(out["vel"], (3, n), "vel"),
            _dptr(out["U"], (n,), "U"), _dptr(out["F"], (3, n), "F"), _dptr(out["W"], (9, n), "W"),
            _dptr(out["J"], (3, n), "J"), _dptr(status, (1,), "status", torch.int32)),
            "mbmd_batch_retire")
        out["status"] = status
        th = self._batch_keep.pop(handle, None)
        if th is not None:
            out["thermo"] = th
        return out

