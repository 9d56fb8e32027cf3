"""Seeded synthetic inputs for the many-body force path.

This module draws and lays out inputs only: diamond-lattice silicon
crystals, Gaussian displacements, vacancies, Maxwell-Boltzmann velocities,
isolated clusters, published potential parameter sets and the serving
request trace.  It holds none of the force method's arithmetic, so both the
HIP path (tests, bench) and the CPU oracle can consume what it produces
without sharing any of the method's code.

The test system follows the paper's performance section: silicon crystal
in a cubic periodic domain, N = 8 n^3 atoms, 300 K.

Units (metal units): Angstrom, eV, amu, fs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# eV/(Angstrom*amu) expressed in Angstrom/fs^2.
KAPPA = 9.64853321567e-3
# Boltzmann constant in eV/K.
K_B = 8.617333262e-5
# Silicon atomic mass in amu.
M_SI = 28.0855
# Diamond-silicon conventional lattice constant used by the paper's test system.
A_SI = 5.43

# Tersoff (1989) silicon parameters, the single-element form the paper states
# in its Tersoff-potential subsection (no lambda_3 term, no chi mixing).
TERSOFF_SI_1989 = dict(
    A=1830.8, B=471.18, lam=2.4799, mu=1.7322, beta=1.1e-6, n=0.78734,
    c=100390.0, d=16.217, h=-0.59825, R=2.7, S=3.0,
)

# Tersoff's multicomponent parameter sets (Tersoff 1989, Table I), with the
# chi of each unlike pair; the silicon set is the one above.
TERSOFF_C_1989 = dict(
    A=1393.6, B=346.74, lam=3.4879, mu=2.2119, beta=1.5724e-7, n=0.72751,
    c=38049.0, d=4.3484, h=-0.57058, R=1.8, S=2.1,
)
TERSOFF_GE_1989 = dict(
    A=1769.0, B=419.23, lam=2.4451, mu=1.7047, beta=9.0166e-7, n=0.75627,
    c=106430.0, d=15.652, h=-0.43884, R=2.8, S=3.1,
)
CHI_SI_C_1989 = 0.9776
CHI_SI_GE_1989 = 1.00061
M_C = 12.011
M_GE = 72.630

# Stillinger-Weber (1985) silicon parameters; cutoff a*sigma = 3.77118 A.
SW_SI_1985 = dict(
    epsilon=2.1683, sigma=2.0951, a=1.80, lam=21.0, gamma=1.20,
    A=7.049556277, B=0.6022245584, p=4.0, q=0.0,
)

# The 8-atom conventional diamond basis in units of the lattice constant.
_DIAMOND_BASIS = np.array([
    [0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0],
    [0.25, 0.25, 0.25], [0.25, 0.75, 0.75], [0.75, 0.25, 0.75], [0.75, 0.75, 0.25],
])


def diamond_lattice(nx: int, ny: int, nz: int, a: float = A_SI):
    """Perfect diamond crystal of nx*ny*nz conventional cells.

    Atoms are ordered by (cell z, cell y, cell x, basis index).  Returns
    positions as an (N, 3) float64 array and the orthorhombic box (3,).
    """
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cells = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    pos = (cells[:, None, :] + _DIAMOND_BASIS[None, :, :]).reshape(-1, 3) * a
    box = np.array([nx * a, ny * a, nz * a], dtype=np.float64)
    return np.ascontiguousarray(pos), box


def wrap_positions(pos: np.ndarray, box: np.ndarray) -> np.ndarray:
    """Fold positions into [0, L) per axis (input preparation only)."""
    out = pos - box * np.floor(pos / box)
    out[out >= box] -= np.broadcast_to(box, out.shape)[out >= box]
    out[out < 0] = 0.0
    return out


def maxwell_boltzmann(n: int, temperature: float, rng: np.random.Generator,
                      mass=M_SI) -> np.ndarray:
    """Velocities (Angstrom/fs) at exactly `temperature`.

    Per-component Gaussian with sigma = sqrt(k_B T kappa / m), centre-of-mass
    velocity removed, then rescaled so that the kinetic temperature with
    3N - 3 degrees of freedom equals `temperature`.  `mass` is a scalar or
    one mass per atom.
    """
    if n == 0:
        return np.zeros((0, 3))
    m = np.broadcast_to(np.asarray(mass, dtype=np.float64), (n,))
    uniform = bool(np.all(m == m[0]))
    if uniform:
        sig = math.sqrt(K_B * temperature * KAPPA / float(m[0]))
        v = rng.normal(0.0, sig, size=(n, 3))
    else:
        v = rng.normal(0.0, 1.0, size=(n, 3)) * np.sqrt(K_B * temperature * KAPPA / m)[:, None]
    if n > 1:
        dof = 3 * n - 3
        if uniform:
            v -= v.mean(axis=0)
            ekin = 0.5 * float(m[0]) * float(np.sum(v * v)) / KAPPA
        else:
            v -= (m[:, None] * v).sum(axis=0) / m.sum()
            ekin = 0.5 * float(np.sum(m[:, None] * v * v)) / KAPPA
        t_now = 2.0 * ekin / (dof * K_B)
        if t_now > 0:
            v *= math.sqrt(temperature / t_now)
    else:
        v[:] = 0.0
    return v


@dataclass
class System:
    """One synthetic structure: positions (N,3), velocities (N,3), box (3,)."""
    pos: np.ndarray
    vel: np.ndarray
    box: np.ndarray
    seed: int
    meta: dict = field(default_factory=dict)
    type_ids: np.ndarray | None = None     # None: every atom type 0

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def types(self) -> np.ndarray:
        if self.type_ids is None:
            return np.zeros(self.n, dtype=np.int32)
        return self.type_ids


def silicon_crystal(cells, seed: int, sigma: float = 0.05, temperature: float = 300.0,
                    vacancy_fraction: float = 0.0, a: float = A_SI) -> System:
    """Diamond Si supercell with seeded Gaussian displacements and velocities.

    `cells` is an int or an (nx, ny, nz) triple.  Draw order from a single
    numpy PCG64 stream seeded with `seed`: vacancy choice, displacements,
    velocities.
    """
    if isinstance(cells, int):
        cells = (cells, cells, cells)
    nx, ny, nz = (int(c) for c in cells)
    pos, box = diamond_lattice(nx, ny, nz, a)
    rng = np.random.default_rng(seed)
    if vacancy_fraction > 0.0:
        n_vac = int(round(vacancy_fraction * pos.shape[0]))
        if n_vac > 0:
            drop = rng.choice(pos.shape[0], size=n_vac, replace=False)
            keep = np.ones(pos.shape[0], dtype=bool)
            keep[drop] = False
            pos = pos[keep]
    if sigma > 0.0:
        pos = pos + rng.normal(0.0, sigma, size=pos.shape)
    pos = wrap_positions(pos, box)
    vel = maxwell_boltzmann(pos.shape[0], temperature, rng)
    return System(np.ascontiguousarray(pos), np.ascontiguousarray(vel), box, seed,
                  dict(cells=(nx, ny, nz), sigma=sigma, temperature=temperature,
                       vacancy_fraction=vacancy_fraction, a=a))


def binary_crystal(cells, seed: int, a: float, masses=(M_SI, M_C), arrangement="zincblende",
                   fraction: float = 0.5, sigma: float = 0.05,
                   temperature: float = 300.0) -> System:
    """Two-element crystal on the diamond lattice, types 0 and 1.

    zincblende: basis sites 0-3 (the fcc sublattice) type 0, sites 4-7 type 1;
    random: each site type 1 with probability `fraction`.  Draw order from
    one PCG64 stream seeded with `seed`: types (random only), displacements,
    velocities (Maxwell-Boltzmann with each atom's mass).
    """
    if isinstance(cells, int):
        cells = (cells, cells, cells)
    nx, ny, nz = (int(c) for c in cells)
    pos, box = diamond_lattice(nx, ny, nz, a)
    rng = np.random.default_rng(seed)
    if arrangement == "zincblende":
        types = np.tile(np.array([0, 0, 0, 0, 1, 1, 1, 1], dtype=np.int32), nx * ny * nz)
    elif arrangement == "random":
        types = (rng.uniform(size=pos.shape[0]) < fraction).astype(np.int32)
    else:
        raise ValueError(arrangement)
    if sigma > 0.0:
        pos = pos + rng.normal(0.0, sigma, size=pos.shape)
    pos = wrap_positions(pos, box)
    m = np.asarray(masses, dtype=np.float64)[types]
    vel = maxwell_boltzmann(pos.shape[0], temperature, rng, mass=m)
    return System(np.ascontiguousarray(pos), np.ascontiguousarray(vel), box, seed,
                  dict(cells=(nx, ny, nz), a=a, arrangement=arrangement, sigma=sigma,
                       temperature=temperature, masses=tuple(masses)), type_ids=types)


def cluster(n: int, seed: int, box_side: float = 60.0, min_dist: float = 2.05,
            radius: float | None = None, temperature: float = 300.0) -> System:
    """Isolated random cluster centred in a large periodic box.

    Atoms are placed uniformly in a sphere by rejection sampling with a
    minimum pair distance, which puts many pairs inside the Tersoff taper
    (R, S) and the SW three-body range.  The box is large enough that no
    periodic image interacts.
    """
    rng = np.random.default_rng(seed)
    if radius is None:
        radius = 1.45 * (n ** (1.0 / 3.0)) + 1.0
    pts = []
    tries = 0
    while len(pts) < n:
        tries += 1
        if tries > 200000:
            raise RuntimeError("cluster placement failed; raise radius")
        p = rng.uniform(-radius, radius, size=3)
        if p @ p > radius * radius:
            continue
        if all(np.linalg.norm(p - q) >= min_dist for q in pts):
            pts.append(p)
    pos = np.array(pts) + box_side / 2.0
    box = np.array([box_side] * 3, dtype=np.float64)
    vel = maxwell_boltzmann(n, temperature, rng)
    return System(np.ascontiguousarray(pos), np.ascontiguousarray(vel), box, seed,
                  dict(kind="cluster", min_dist=min_dist, radius=radius))


# Named workloads: the small parity case and the large single-GPU cases.
def tersoff_small() -> System:
    """Tersoff Si, 4x4x4 cells = 512 atoms, sigma 0.05 A, 300 K, seed 1001."""
    return silicon_crystal(4, seed=1001)


def tersoff_512k() -> System:
    """Tersoff Si, 40x40x40 cells = 512,000 atoms, sigma 0.05 A, 300 K, seed 1002."""
    return silicon_crystal(40, seed=1002)


def sw_1m() -> System:
    """SW Si, 50x50x50 cells = 1,000,000 atoms, sigma 0.05 A, 300 K, seed 1003."""
    return silicon_crystal(50, seed=1003)


@dataclass
class Request:
    """One serving request: a structure and what to do with it."""
    rid: int
    arrival_s: float
    system: System
    kind: str          # "single" or "nve"
    n_steps: int


def serving_trace(n_requests: int, rate_hz: float, seed: int = 2001,
                  min_cells: int = 2, max_cells: int = 16,
                  nve_fraction: float = 0.3, nve_steps: int = 200):
    """Poisson-arrival request trace of uneven diamond-Si supercells.

    Cell counts per axis are drawn i.i.d. log-uniform in [min_cells,
    max_cells] (64 to 32,768 atoms at 2..16), vacancy fraction U(0, 0.05),
    displacement sigma U(0.05, 0.15) A, 300 K velocities; a fraction
    `nve_fraction` asks for `nve_steps` NVE steps, the rest for a single
    point.  Each structure gets its own derived seed.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    lo, hi = math.log(min_cells), math.log(max_cells + 1)
    for rid in range(n_requests):
        t += float(rng.exponential(1.0 / rate_hz))
        cells = tuple(int(min(max_cells, math.floor(math.exp(rng.uniform(lo, hi)))))
                      for _ in range(3))
        vac = float(rng.uniform(0.0, 0.05))
        sig = float(rng.uniform(0.05, 0.15))
        kind = "nve" if rng.uniform() < nve_fraction else "single"
        sub_seed = int(rng.integers(0, 2**31 - 1))
        sysm = silicon_crystal(cells, seed=sub_seed, sigma=sig, vacancy_fraction=vac)
        reqs.append(Request(rid, t, sysm, kind, nve_steps if kind == "nve" else 0))
    return reqs


def soa(x: np.ndarray) -> np.ndarray:
    """(N, k) row-major -> (k, N) contiguous (the library's SoA layout)."""
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).T)
