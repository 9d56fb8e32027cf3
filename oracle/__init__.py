"""ctypes binding of the CPU FP64 oracle.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the HIP product path never does.
Arrays here are row-major per atom (positions (N, 3), virials (N, 9) with
component 3*alpha + beta), independent of the HIP library's SoA layout.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from .build import ensure_built

OK, EINVAL, ENEIGH, EBOX, ENOMEM = 0, 1, 2, 3, 4
_ERR = {EINVAL: "invalid argument", ENEIGH: "neighbour list overflow",
        EBOX: "box shorter than 2 r_list", ENOMEM: "out of memory"}


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle error {code}: {_ERR.get(code, '?')}")
        self.code = code


class _Tersoff(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("A", "B", "lam", "mu", "beta", "n", "c", "d", "h", "R", "S")]


class _TersoffMulti(C.Structure):
    _fields_ = [("ntypes", C.c_int), ("types", C.c_void_p), ("elem", C.c_void_p),
                ("chi", C.c_void_p)]


class _SW(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("epsilon", "sigma", "a", "lam", "gamma", "A", "B", "p", "q")]


_lib = None
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def _load():
    global _lib
    if _lib is None:
        lib = C.CDLL(ensure_built())
        P = C.c_void_p
        lib.ora_neighbors_brute.argtypes = [C.c_long, _dp, _dp, C.c_double, C.c_int, _ip, _ip]
        lib.ora_neighbors_cells.argtypes = [C.c_long, _dp, _dp, C.c_double, C.c_int, _ip, _ip]
        lib.ora_neighbors_brute_typed.argtypes = [C.c_long, _dp, _dp, _ip, C.c_int, _dp, C.c_int,
                                                  _ip, _ip]
        for name, st in (("ora_tersoff", _Tersoff), ("ora_sw", _SW)):
            fn = getattr(lib, name)
            fn.argtypes = [C.c_long, _dp, _dp, P, _ip, _ip, C.c_int, C.POINTER(st),
                           _dp, _dp, _dp, _dp, P, P, P, P]
            fn.restype = C.c_int
        lib.ora_nve.argtypes = [C.c_int, P, C.c_long, _dp, C.c_double, P, _dp, _dp, C.c_int,
                                C.c_double, C.c_double, C.c_double, C.c_int, C.c_int, C.c_int,
                                _dp, _dp, _dp, _dp, P, C.POINTER(C.c_long)]
        D = C.c_double
        lib.ora_npt.argtypes = [C.c_int, P, C.c_long, _dp, D, P, _dp, _dp, C.c_int, D, D,
                                C.c_int, C.c_int, D, D, D, D, D, _dp, _dp, _dp, _dp, _dp, _dp,
                                C.POINTER(C.c_long)]
        lib.ora_tersoff_multi.argtypes = [C.c_long, _dp, _dp, P, _ip, C.c_int, P, P, _ip, _ip,
                                          C.c_int, _dp, _dp, _dp, _dp, P, P, P, P]
        lib.ora_tersoff_multi.restype = C.c_int
        lib.ora_npt.restype = C.c_int
        lib.ora_wrap.argtypes = [C.c_long, _dp, _dp]
        lib.ora_wrap.restype = None
        lib.ora_set_threads.argtypes = [C.c_int]
        lib.ora_set_threads.restype = None
        lib.ora_threads.argtypes = []
        lib.ora_threads.restype = C.c_int
        for name in ("ora_tersoff_g", "ora_tersoff_g_literal", "ora_tersoff_b", "ora_tersoff_db"):
            getattr(lib, name).argtypes = [C.POINTER(_Tersoff), C.c_double]
            getattr(lib, name).restype = C.c_double
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def tersoff_params(p: dict) -> _Tersoff:
    return _Tersoff(**{k: float(p[k]) for k in ("A", "B", "lam", "mu", "beta", "n", "c", "d", "h", "R", "S")})


def sw_params(p: dict) -> _SW:
    return _SW(**{k: float(p[k]) for k in ("epsilon", "sigma", "a", "lam", "gamma", "A", "B", "p", "q")})


def set_threads(n: int) -> int:
    """Host threads for the loops over atoms (OpenMP; 1 = serial, the
    default).  Forces (scattered to neighbours) are summed over per-thread
    buffers in thread order, so they round differently with more than one
    thread; every other output is the same bit for bit.  Returns the count
    in effect."""
    lib = _load()
    lib.ora_set_threads(int(n))
    return lib.ora_threads()


def wrap(pos, box):
    lib = _load()
    out = _f64(pos).copy()
    lib.ora_wrap(out.shape[0], _f64(box), out)
    return out


def neighbors(pos, box, rlist: float, maxnb: int, method: str = "cells", allow_overflow=False):
    """Sorted neighbour lists: returns (nn (N,), nl (N, maxnb), padded with -1)."""
    lib = _load()
    pos = _f64(pos)
    n = pos.shape[0]
    nn = np.zeros(n, dtype=np.int32)
    nl = np.full((max(n, 1), maxnb), -1, dtype=np.int32)
    fn = lib.ora_neighbors_brute if method == "brute" else lib.ora_neighbors_cells
    st = fn(n, _f64(box), pos, float(rlist), int(maxnb), nn, nl)
    if st and not (allow_overflow and st == ENEIGH):
        raise OracleError(st)
    return nn, nl[:n]


def neighbors_typed(pos, box, types, rpair, maxnb: int):
    """Sorted neighbour lists with a radius per pair of types (rpair (nt, nt),
    symmetric): j is listed for i iff r_ij < rpair[t_i, t_j].  Brute force.
    Returns (nn (N,), nl (N, maxnb), padded with -1)."""
    lib = _load()
    pos = _f64(pos)
    n = pos.shape[0]
    rp = np.ascontiguousarray(rpair, dtype=np.float64)
    nt = rp.shape[0]
    if rp.shape != (nt, nt) or not np.array_equal(rp, rp.T):
        raise ValueError("rpair must be a symmetric (nt, nt) array")
    t = np.ascontiguousarray(types, dtype=np.int32)
    if t.shape != (n,):
        raise ValueError("one type per atom")
    nn = np.zeros(n, dtype=np.int32)
    nl = np.full((max(n, 1), maxnb), -1, dtype=np.int32)
    st = lib.ora_neighbors_brute_typed(n, _f64(box), pos, t if n else np.zeros(1, np.int32), nt,
                                       rp.reshape(-1), int(maxnb), nn, nl)
    if st:
        raise OracleError(st)
    return nn, nl[:n]


def _force(name, params, pos, box, nn, nl, vel=None, want_g=False):
    lib = _load()
    pos = _f64(pos)
    n = pos.shape[0]
    maxnb = nl.shape[1] if n else 1
    nl = np.ascontiguousarray(nl, dtype=np.int32)
    if n == 0:
        nl = np.zeros((1, maxnb), dtype=np.int32)
    nn = np.ascontiguousarray(nn, dtype=np.int32)
    velc = None if vel is None else _f64(vel)
    U = np.zeros(max(n, 1))
    F = np.zeros((max(n, 1), 3))
    W = np.zeros((max(n, 1), 9))
    J = np.zeros((max(n, 1), 3))
    Fp = np.zeros((max(n, 1), 3))
    WL = np.zeros((max(n, 1), 9))
    JL = np.zeros((max(n, 1), 3))
    G = np.zeros((max(n, 1), maxnb, 3)) if want_g else None
    pr = tersoff_params(params) if name == "ora_tersoff" else sw_params(params)
    st = getattr(lib, name)(n, _f64(box), pos if n else np.zeros((1, 3)), _ptr(velc), nn if n else np.zeros(1, np.int32),
                            nl, maxnb, C.byref(pr), U, F, W, J, _ptr(Fp), _ptr(WL), _ptr(JL), _ptr(G))
    if st:
        raise OracleError(st)
    out = dict(U=U[:n], F=F[:n], W=W[:n], J=J[:n], Fpair=Fp[:n], WL=WL[:n], JL=JL[:n])
    if want_g:
        out["G"] = G[:n]
    return out


class _MultiArgs:
    """Keeps the ctypes arrays of a multicomponent parameter set alive."""

    def __init__(self, multi):
        elems = multi["elems"]
        nt = len(elems)
        self.types = np.ascontiguousarray(multi["types"], dtype=np.int32)
        self.elem = (_Tersoff * nt)(*[tersoff_params(e) for e in elems])
        chi = multi.get("chi")
        self.chi = None if chi is None else np.ascontiguousarray(chi, dtype=np.float64).reshape(nt, nt)
        self.nt = nt
        self.struct = _TersoffMulti(nt, self.types.ctypes.data_as(C.c_void_p),
                                    C.cast(self.elem, C.c_void_p), _ptr(self.chi))


def tersoff_multi(multi, pos, box, nn, nl, vel=None, want_g=False):
    """Multicomponent Tersoff (ora_tersoff_multi).  multi = dict(elems=[param
    dicts], chi=(nt, nt) array or None, types=(n,) ints).  Returns the outputs
    of tersoff()."""
    lib = _load()
    pos = _f64(pos)
    n = pos.shape[0]
    m = _MultiArgs(multi)
    maxnb = nl.shape[1]
    nl = np.ascontiguousarray(nl, dtype=np.int32)
    nn = np.ascontiguousarray(nn, dtype=np.int32)
    velc = None if vel is None else _f64(vel)
    U, F, W, J = np.zeros(n), np.zeros((n, 3)), np.zeros((n, 9)), np.zeros((n, 3))
    Fp, WL, JL = np.zeros((n, 3)), np.zeros((n, 9)), np.zeros((n, 3))
    G = np.zeros((n, maxnb, 3)) if want_g else None
    st = lib.ora_tersoff_multi(n, _f64(box), pos, _ptr(velc), m.types, m.nt, C.cast(m.elem, C.c_void_p),
                               _ptr(m.chi), nn, nl, maxnb, U, F, W, J, _ptr(Fp), _ptr(WL),
                               _ptr(JL), _ptr(G))
    if st:
        raise OracleError(st)
    out = dict(U=U, F=F, W=W, J=J, Fpair=Fp, WL=WL, JL=JL)
    if want_g:
        out["G"] = G
    return out


def _potential(potential, params):
    """(id, ctypes parameter struct, keep-alive) for the integrators."""
    if potential == "tersoff":
        pr = tersoff_params(params)
        return 0, pr, None
    if potential == "tersoff_multi":
        m = _MultiArgs(params)
        return 2, m.struct, m
    return 1, sw_params(params), None


def tersoff(params, pos, box, nn, nl, vel=None, want_g=False):
    """Per-atom U, F (Algorithm 1 scatter), W, J (pairwise), Fpair, WL, JL[, G]."""
    return _force("ora_tersoff", params, pos, box, nn, nl, vel, want_g)


def sw(params, pos, box, nn, nl, vel=None, want_g=False):
    return _force("ora_sw", params, pos, box, nn, nl, vel, want_g)


def nve(potential: str, params, pos, vel, box, mass: float, n_steps: int, dt: float,
        rlist: float, rebuild_every: int, maxnb: int, skin: float = 0.5,
        check_skin: bool = True, masses=None):
    """Velocity-Verlet NVE.  Returns dict(pos, vel, U, F, W, J,
    thermo[n_steps+1, 16], builds).  The list is rebuilt every rebuild_every
    steps and, with check_skin, before any step whose positions moved more
    than skin/2 from the last build.  potential: "tersoff", "sw" or
    "tersoff_multi" (params as for tersoff_multi); masses: per-atom masses
    replacing `mass`."""
    lib = _load()
    pos = _f64(pos).copy()
    vel = _f64(vel).copy()
    n = pos.shape[0]
    U = np.zeros(n)
    F = np.zeros((n, 3))
    W = np.zeros((n, 9))
    J = np.zeros((n, 3))
    thermo = np.zeros((n_steps + 1, 16))
    pid, pr, keep = _potential(potential, params)
    mz = None if masses is None else _f64(masses)
    builds = C.c_long(0)
    st = lib.ora_nve(pid, C.cast(C.byref(pr), C.c_void_p), n, _f64(box), float(mass), _ptr(mz),
                     pos, vel,
                     int(n_steps), float(dt), float(rlist), float(skin), int(rebuild_every),
                     int(bool(check_skin)), int(maxnb), U, F, W, J, _ptr(thermo),
                     C.byref(builds))
    if st:
        raise OracleError(st)
    return dict(pos=pos, vel=vel, U=U, F=F, W=W, J=J, thermo=thermo, builds=builds.value)


# 1 eV/A^3 in GPa
EV_PER_A3_IN_GPA = 160.21766208


def npt(potential: str, params, pos, vel, box, mass: float, n_steps: int, dt: float,
        rlist: float, rebuild_every: int, maxnb: int, T0: float, tau_T: float, P0_GPa: float,
        tau_P: float, beta_per_GPa: float, masses=None):
    """Velocity-Verlet with Berendsen weak coupling (see ora_npt).  P0 in GPa,
    compressibility beta in 1/GPa; tau_T, tau_P in fs (<= 0: that coupling
    off); potential and masses as for nve().  Returns dict(pos, vel, box, U,
    F, W, J, thermo[n_steps+1, 16], box_traj[n_steps+1, 3], builds)."""
    lib = _load()
    pos = _f64(pos).copy()
    vel = _f64(vel).copy()
    boxc = _f64(box).copy()
    n = pos.shape[0]
    U = np.zeros(n)
    F = np.zeros((n, 3))
    W = np.zeros((n, 9))
    J = np.zeros((n, 3))
    thermo = np.zeros((n_steps + 1, 16))
    box_traj = np.zeros((n_steps + 1, 3))
    pid, pr, keep = _potential(potential, params)
    mz = None if masses is None else _f64(masses)
    builds = C.c_long(0)
    st = lib.ora_npt(pid, C.cast(C.byref(pr), C.c_void_p), n, boxc, float(mass), _ptr(mz), pos,
                     vel,
                     int(n_steps), float(dt), float(rlist), int(rebuild_every), int(maxnb),
                     float(T0), float(tau_T), float(P0_GPa) / EV_PER_A3_IN_GPA, float(tau_P),
                     float(beta_per_GPa) * EV_PER_A3_IN_GPA, U, F, W, J, thermo, box_traj,
                     C.byref(builds))
    if st:
        raise OracleError(st)
    return dict(pos=pos, vel=vel, box=boxc, U=U, F=F, W=W, J=J, thermo=thermo,
                box_traj=box_traj, builds=builds.value)


def pressure_GPa(thermo_row, box):
    """Pressure of a thermo row in a box: (2 E_kin + tr W) / (3 V), in GPa."""
    row = np.asarray(thermo_row)
    v = float(np.prod(box))
    return (2.0 * row[1] + row[2] + row[6] + row[10]) / (3.0 * v) * EV_PER_A3_IN_GPA


def tersoff_g(params, cs: float, literal: bool = False) -> float:
    lib = _load()
    fn = lib.ora_tersoff_g_literal if literal else lib.ora_tersoff_g
    return fn(C.byref(tersoff_params(params)), float(cs))


def tersoff_b(params, zeta: float) -> float:
    return _load().ora_tersoff_b(C.byref(tersoff_params(params)), float(zeta))


def tersoff_db(params, zeta: float) -> float:
    return _load().ora_tersoff_db(C.byref(tersoff_params(params)), float(zeta))
