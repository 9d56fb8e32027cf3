"""Pins of the oracle's Stillinger-Weber three-body term.

The published SW properties of the diamond crystal (cohesive energy, bulk
modulus) are blind to the three-body term: at the tetrahedral angle
cos theta = -1/3 it vanishes, and isotropic strain keeps every angle.  These
tests evaluate configurations whose angles are not tetrahedral, in 50-digit
mpmath, from Stillinger and Weber's own statement of the potential (the
SW potential the paper names in Section 2.4), written here independently
of the oracle in the 1985 reduced form:

    Phi = sum_{i<j} v2(r_ij) + sum_{i<j<k} v3(r_i, r_j, r_k)
    v2(r)  = eps f2(r / sigma),  f2(x) = A (B x^-p - x^-q) exp(1 / (x - a)), x < a
    v3     = eps [h(x_ij, x_ik, theta_jik) + h(x_ji, x_jk, theta_ijk)
                  + h(x_ki, x_kj, theta_ikj)]
    h(x1, x2, theta) = lambda exp(gamma / (x1 - a) + gamma / (x2 - a)) (cos theta + 1/3)^2,
                       both x < a.

Each triplet is visited once, as an unordered set, and contributes one h per
vertex whose two bonds are inside the cutoff.  The per-atom energy is the
vertex partition the oracle states (half of each pair term to each end, each
h to its vertex atom), and the forces are minus the 50-digit derivative of
Phi.  A three-body term counted over ordered partner pairs, a wrong
eps*lambda prefactor, gamma on the wrong factor or a wrong angle offset
changes the per-atom and total energies or the forces beyond the bound.
"""
import math

import numpy as np
import pytest

import workload as wl
from conftest import rel_err

SP = wl.SW_SI_1985
RL_S = SP["a"] * SP["sigma"] + 0.5

mp = pytest.importorskip("mpmath")
mp.mp.dps = 50


def _P():
    return {k: mp.mpf(repr(float(v))) for k, v in SP.items()}


def _min_image(d, box):
    return [d[c] - box[c] * mp.nint(d[c] / box[c]) for c in range(3)]


def _f2(P, x):
    if not x < P["a"]:
        return mp.mpf(0)
    return P["A"] * (P["B"] * x ** (-P["p"]) - x ** (-P["q"])) * mp.exp(1 / (x - P["a"]))


def _h(P, x1, x2, cos_t):
    if not (x1 < P["a"] and x2 < P["a"]):
        return mp.mpf(0)
    return P["lam"] * mp.exp(P["gamma"] / (x1 - P["a"]) + P["gamma"] / (x2 - P["a"])) * \
        (cos_t + mp.mpf(1) / 3) ** 2


class Config:
    """Positions (mp) and box (mp) with the candidate pairs found once in
    float64 (pairs closer than the cutoff plus a margin)."""

    def __init__(self, pos, box):
        self.box = [mp.mpf(repr(float(b))) for b in box]
        self.pos = [[mp.mpf(repr(float(x))) for x in p] for p in pos]
        n = len(pos)
        cut = SP["a"] * SP["sigma"] + 0.3
        self.cand = [[] for _ in range(n)]
        for i in range(n):
            for j in range(n):
                if i == j:
                    continue
                d = np.asarray(pos[j], float) - np.asarray(pos[i], float)
                d -= box * np.rint(d / box)
                if d @ d < cut * cut:
                    self.cand[i].append(j)

    def bonds(self, P, pos, i):
        """(j, x_ij, vector) for every j within a sigma of i."""
        out = []
        for j in self.cand[i]:
            d = _min_image([pos[j][c] - pos[i][c] for c in range(3)], self.box)
            r = mp.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
            x = r / P["sigma"]
            if x < P["a"]:
                out.append((j, x, d, r))
        return out

    def site_energies(self, pos=None):
        """Vertex partition: U_i = 1/2 sum_j v2 + eps sum_{j<k} h(x_ij, x_ik, theta_jik)."""
        P = _P()
        pos = self.pos if pos is None else pos
        U = []
        for i in range(len(pos)):
            b = self.bonds(P, pos, i)
            u = mp.mpf(0)
            for (_, x, _, _) in b:
                u += P["epsilon"] * _f2(P, x) / 2
            for s in range(len(b)):
                for t in range(s + 1, len(b)):
                    _, x1, d1, r1 = b[s]
                    _, x2, d2, r2 = b[t]
                    cs = (d1[0] * d2[0] + d1[1] * d2[1] + d1[2] * d2[2]) / (r1 * r2)
                    u += P["epsilon"] * _h(P, x1, x2, cs)
            U.append(u)
        return U

    def total_energy_triplets(self, pos=None):
        """Phi written as the 1985 sum over pairs i<j and unordered triplets
        i<j<k, each triplet's three vertex terms (a separate transcription of
        the same definition, cross-checking site_energies)."""
        P = _P()
        pos = self.pos if pos is None else pos
        n = len(pos)
        vec = {}
        for i in range(n):
            for (j, x, d, r) in self.bonds(P, pos, i):
                vec[(i, j)] = (x, d, r)
        e = mp.mpf(0)
        for (i, j), (x, _, _) in vec.items():
            if i < j:
                e += P["epsilon"] * _f2(P, x)

        def vertex(v, a, b):
            if (v, a) not in vec or (v, b) not in vec:
                return mp.mpf(0)
            x1, d1, r1 = vec[(v, a)]
            x2, d2, r2 = vec[(v, b)]
            cs = (d1[0] * d2[0] + d1[1] * d2[1] + d1[2] * d2[2]) / (r1 * r2)
            return _h(P, x1, x2, cs)

        for i in range(n):
            for j in range(i + 1, n):
                for k in range(j + 1, n):
                    t = vertex(i, j, k) + vertex(j, i, k) + vertex(k, i, j)
                    e += P["epsilon"] * t
        return e

    def force(self, a, c):
        """-dPhi/dx_{a,c} in 50 digits."""
        def energy(xc):
            pos = [list(p) for p in self.pos]
            pos[a][c] = xc
            return mp.fsum(self.site_energies(pos))
        return -mp.diff(energy, self.pos[a][c])


def _oracle(oracle_mod, pos, box):
    nn, nl = oracle_mod.neighbors(pos, box, RL_S, 48)
    return oracle_mod.sw(SP, pos, box, nn, nl)


def _trimer(theta_deg, r1=2.35, r2=2.50, box_side=40.0):
    """Vertex atom 0, atom 1 along x at r1, atom 2 at r2 and angle theta."""
    t = math.radians(theta_deg)
    c = box_side / 2.0
    pos = np.array([[c, c, c], [c + r1, c, c],
                    [c + r2 * math.cos(t), c + r2 * math.sin(t), c]])
    return pos, np.full(3, box_side)


def _check_cluster(oracle_mod, pos, box, atoms=None):
    cfg = Config(pos, box)
    ref_U = np.array([float(u) for u in cfg.site_energies()])
    total_tri = float(cfg.total_energy_triplets())
    o = _oracle(oracle_mod, pos, box)
    # the two transcriptions of the definition agree to the working digits
    assert abs(math.fsum(ref_U) - total_tri) <= 1e-15 * max(1.0, abs(total_tri))
    assert rel_err(o["U"], ref_U) <= 1e-13
    assert abs(o["U"].sum() - total_tri) <= 1e-13 * max(1.0, abs(total_tri))
    atoms = range(len(pos)) if atoms is None else atoms
    ref_F = np.array([[float(cfg.force(a, c)) for c in range(3)] for a in atoms])
    assert rel_err(o["F"][list(atoms)], ref_F) <= 1e-13
    return o, ref_U, total_tri


@pytest.mark.parametrize("theta", [60.0, 75.0, 90.0, 120.0, 150.0, 180.0])
def test_sw_trimer_three_body_against_definition(oracle_mod, theta):
    """Isolated trimers: angles far from tetrahedral, with (60-90 degrees)
    and without (120-180 degrees) the 1-2 bond inside the cutoff."""
    pos, box = _trimer(theta)
    o, ref_U, total = _check_cluster(oracle_mod, pos, box)
    # the three-body part of the vertex atom is not negligible
    P = {k: float(v) for k, v in SP.items()}
    pair_half = [0.5 * P["epsilon"] * float(_f2(_P(), mp.mpf(r) / _P()["sigma"]))
                 for r in (2.35, 2.50)]
    three = ref_U[0] - sum(pair_half)
    assert three > 1e-3


def test_sw_equilateral_triangle(oracle_mod):
    """Equilateral triangle of side 2.4 A: every vertex carries the same h at
    cos theta = 1/2, and U_i = v2(r) + eps lambda exp(2 gamma / (x - a)) (5/6)^2."""
    s = 2.4
    c = 20.0
    pos = np.array([[c, c, c], [c + s, c, c], [c + s / 2, c + s * math.sqrt(3) / 2, c]])
    box = np.full(3, 40.0)
    o, ref_U, _ = _check_cluster(oracle_mod, pos, box)
    P = _P()
    x = mp.mpf(repr(s)) / P["sigma"]
    closed = P["epsilon"] * _f2(P, x) + P["epsilon"] * P["lam"] * \
        mp.exp(2 * P["gamma"] / (x - P["a"])) * (mp.mpf(1) / 2 + mp.mpf(1) / 3) ** 2
    assert np.all(np.abs(o["U"] - float(closed)) <= 1e-13 * abs(float(closed)))
    # equal and opposite: net force zero, each force along its median
    assert np.abs(o["F"].sum(axis=0)).max() <= 1e-13 * np.abs(o["F"]).max()


def test_sw_strained_diamond_cell(oracle_mod):
    """A 2x2x2 diamond cell under an orthorhombic strain (x +4 %, y -3 %)
    with its second fcc sublattice shifted by (0.05, 0.03, -0.02) A (an
    orthorhombic box admits no shear, so the internal shift breaks the
    symmetry that keeps forces at zero): the bond angles leave the
    tetrahedral value, so every site carries a three-body energy; per-atom
    energies, the total and forces on a few atoms against the definition."""
    pos, box = wl.diamond_lattice(2, 2, 2, a=5.43)
    strain = np.array([1.04, 0.97, 1.0])
    pos, box = pos * strain, box * strain
    second = np.tile(np.arange(8) >= 4, 8)
    pos[second] += np.array([0.05, 0.03, -0.02])
    o, ref_U, _ = _check_cluster(oracle_mod, pos, box, atoms=[0, 5])
    # non-tetrahedral: the site energy differs from the pair-only value
    P = _P()
    cfg = Config(pos, box)
    pair_only = mp.fsum(P["epsilon"] * _f2(P, x) / 2 for (_, x, _, _) in cfg.bonds(P, cfg.pos, 0))
    assert abs(ref_U[0] - float(pair_only)) > 1e-2


def test_sw_displaced_cell_and_cluster(oracle_mod):
    """Generic geometries: a 64-atom cell with 0.15 A displacements and an
    18-atom cluster (many bonds near the cutoff, angles of every kind)."""
    c = wl.silicon_crystal(2, seed=31, sigma=0.15)
    _check_cluster(oracle_mod, c.pos, c.box, atoms=[3, 40])
    k = wl.cluster(12, seed=32, min_dist=2.1, box_side=30.0)
    _check_cluster(oracle_mod, k.pos, k.box, atoms=[0, 7])
