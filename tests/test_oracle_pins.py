"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test names the passage of the paper (or the cited parameter source) it
checks.  Together they cover the energy functional, every force term, the
per-atom partials dU_i/dr_ij behind the paper's pairwise force, the per-atom
virial and heat current, the neighbour lists and the integrator, so that a
dropped term, a wrong sign or index or a transposed operand in the oracle
fails at least one of them.  All run on the CPU.
"""
import math
import os

import numpy as np
import pytest

import workload as wl
from conftest import rel_err
from coupling_law import berendsen_law, ideal_gas

TP = wl.TERSOFF_SI_1989
SP = wl.SW_SI_1985
RL_T = 3.5                  # Tersoff S = 3.0 plus 0.5 skin
RL_S = 3.77118 + 0.5        # SW a*sigma plus 0.5 skin
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden_properties():
    out = {}
    with open(os.path.join(GOLDEN, "published_si_properties.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, val, tol, _unit = line.split()
            out[key] = (float(val), float(tol))
    return out


def evaluate(oracle, pot, pos, box, nn, nl, vel=None, want_g=False):
    fn = oracle.tersoff if pot == "tersoff" else oracle.sw
    return fn(TP if pot == "tersoff" else SP, pos, box, nn, nl, vel=vel, want_g=want_g)


def lists(oracle, pot, pos, box, maxnb=32):
    return oracle.neighbors(pos, box, RL_T if pot == "tersoff" else RL_S, maxnb)


def systems():
    """Small structures exercising distinct regimes of the potentials."""
    c64 = wl.silicon_crystal(2, seed=11, sigma=0.1)
    # Lattice expanded so first neighbours (2.79 A) sit in the taper (R, S).
    exp64 = wl.silicon_crystal(2, seed=12, sigma=0.08, a=6.45)
    vac = wl.silicon_crystal(2, seed=14, sigma=0.15, vacancy_fraction=0.1)
    clu = wl.cluster(18, seed=13, min_dist=2.1, box_side=40.0)
    return dict(crystal=c64, expanded=exp64, vacancies=vac, cluster=clu)


SYSTEMS = systems()
CASES = [(pot, name) for pot in ("tersoff", "sw") for name in SYSTEMS]


# ------------------------------------------------------------ energy functional

def _crystal_energy(oracle, pot, a):
    pos, box = wl.diamond_lattice(2, 2, 2, a=a)
    nn, nl = lists(oracle, pot, pos, box)
    return evaluate(oracle, pot, pos, box, nn, nl)


def test_tersoff_published_crystal_properties(oracle_mod):
    """Tersoff (1989) Si fit: E_c = 4.63 eV, a = 5.432 A, B = 0.98 Mbar."""
    from scipy.optimize import minimize_scalar
    g = golden_properties()
    e = lambda a: _crystal_energy(oracle_mod, "tersoff", a)["U"].mean()
    r = minimize_scalar(e, bracket=(5.40, 5.432, 5.46), tol=1e-12)
    a0 = r.x
    assert abs(a0 - g["tersoff_lattice_constant"][0]) < g["tersoff_lattice_constant"][1]
    assert abs(r.fun - g["tersoff_cohesive_energy"][0]) < g["tersoff_cohesive_energy"][1]
    v0 = a0 ** 3 / 8.0
    h = 1e-3 * v0
    ev = lambda v: e((8.0 * v) ** (1.0 / 3.0))
    bulk = v0 * (ev(v0 + h) - 2 * ev(v0) + ev(v0 - h)) / h ** 2 * 1.602176634
    assert abs(bulk - g["tersoff_bulk_modulus"][0]) < g["tersoff_bulk_modulus"][1]


def test_sw_published_crystal_properties(oracle_mod):
    """SW (1985): diamond at r_nn = 2^(1/6) sigma has -2 epsilon per atom."""
    g = golden_properties()
    a_sw = 4.0 * 2 ** (1.0 / 6.0) * SP["sigma"] / math.sqrt(3.0)
    o = _crystal_energy(oracle_mod, "sw", a_sw)
    assert np.all(np.abs(o["U"] - g["sw_cohesive_energy"][0]) < g["sw_cohesive_energy"][1])
    assert np.abs(o["F"]).max() < 1e-12
    v0 = a_sw ** 3 / 8.0
    h = 1e-3 * v0
    ev = lambda v: _crystal_energy(oracle_mod, "sw", (8.0 * v) ** (1.0 / 3.0))["U"].mean()
    bulk = v0 * (ev(v0 + h) - 2 * ev(v0) + ev(v0 - h)) / h ** 2 * 1.602176634
    assert abs(bulk - g["sw_bulk_modulus"][0]) < g["sw_bulk_modulus"][1]


def test_tersoff_closed_form_crystal(oracle_mod):
    """Perfect diamond reduces the Tersoff sums to a closed form: four bonds
    of length a sqrt(3)/4, three partners each at cos theta = -1/3, so
    U_i = 2 f_R(r0) - 2 b(3 g(-1/3)) f_A(r0); evaluated in 50-digit mpmath."""
    import mpmath as mp
    mp.mp.dps = 50
    a = mp.mpf("5.43")
    r0 = a * mp.sqrt(3) / 4
    fr = mp.mpf(TP["A"]) * mp.exp(-mp.mpf(TP["lam"]) * r0)
    fa = mp.mpf(TP["B"]) * mp.exp(-mp.mpf(TP["mu"]) * r0)
    c2, d2, h = mp.mpf(TP["c"]) ** 2, mp.mpf(TP["d"]) ** 2, mp.mpf(TP["h"])
    g = 1 + c2 / d2 - c2 / (d2 + (h + mp.mpf(1) / 3) ** 2)
    zeta = 3 * g
    n, beta = mp.mpf(TP["n"]), mp.mpf(TP["beta"])
    b = (1 + (beta * zeta) ** n) ** (-1 / (2 * n))
    u_ref = float(2 * fr - 2 * b * fa)
    o = _crystal_energy(oracle_mod, "tersoff", 5.43)
    assert rel_err(o["U"], np.full(64, u_ref)) < 1e-14
    # Perfect crystal: no force, identical isotropic virial, zero J at v = 0.
    assert np.abs(o["F"]).max() < 1e-12
    w = o["W"]
    assert np.allclose(w, w[0], rtol=0, atol=1e-14)
    assert abs(w[0, 0] - w[0, 4]) < 1e-14 and abs(w[0, 0] - w[0, 8]) < 1e-14
    assert np.abs(w[0, [1, 2, 3, 5, 6, 7]]).max() < 1e-14
    assert np.abs(o["J"]).max() == 0.0


def test_g_stable_form_matches_printed_form(oracle_mod):
    """The oracle evaluates g_ijk (Section 2.1) as 1 + c^2 t^2/(d^2 (d^2+t^2)),
    algebraically the printed 1 + c^2/d^2 - c^2/(d^2+t^2); check both
    against a 50-digit evaluation of the printed form."""
    import mpmath as mp
    mp.mp.dps = 50
    c2, d2, h = mp.mpf(TP["c"]) ** 2, mp.mpf(TP["d"]) ** 2, mp.mpf(TP["h"])
    worst_stable = worst_literal = 0.0
    for cs in np.linspace(-1.0, 1.0, 41):
        exact = 1 + c2 / d2 - c2 / (d2 + (h - mp.mpf(float(cs))) ** 2)
        st = oracle_mod.tersoff_g(TP, cs)
        li = oracle_mod.tersoff_g(TP, cs, literal=True)
        worst_stable = max(worst_stable, abs(float((st - exact) / exact)))
        worst_literal = max(worst_literal, abs(float((li - exact) / exact)))
    assert worst_stable < 2e-15
    assert worst_literal > worst_stable  # the printed form cancels ~3.8e7-size terms


def test_bond_order_function(oracle_mod):
    """b = (1 + beta^n zeta^n)^(-1/(2n)) and its zeta derivative."""
    import mpmath as mp
    mp.mp.dps = 40
    n, beta = mp.mpf(TP["n"]), mp.mpf(TP["beta"])
    for z in (1e-3, 0.5, 7.0, 3.0e4, 1e6):
        ref = (1 + (beta * mp.mpf(z)) ** n) ** (-1 / (2 * n))
        assert abs(oracle_mod.tersoff_b(TP, z) - float(ref)) <= 2e-15 * float(ref)
        dref = mp.diff(lambda x: (1 + (beta * x) ** n) ** (-1 / (2 * n)), mp.mpf(z))
        assert abs(oracle_mod.tersoff_db(TP, z) - float(dref)) <= 1e-13 * abs(float(dref))
    # zeta = 0 (no third atom): b = 1 and db/dzeta is taken as 0.
    assert oracle_mod.tersoff_b(TP, 0.0) == 1.0
    assert oracle_mod.tersoff_db(TP, 0.0) == 0.0


# ------------------------------------------------------------------ forces

def _total_energy(oracle, pot, pos, box, nn, nl):
    return float(np.sum(evaluate(oracle, pot, pos, box, nn, nl)["U"]))


def _fd_grad(fun, x, h):
    """Fourth-order central difference of a scalar function of an array."""
    g = np.zeros_like(x)
    it = np.nditer(x, flags=["multi_index"])
    for _ in it:
        idx = it.multi_index
        vals = []
        for s in (-2, -1, 1, 2):
            xp = x.copy()
            xp[idx] += s * h
            vals.append(fun(xp))
        g[idx] = (vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * h)
    return g


@pytest.mark.parametrize("pot,name", CASES)
def test_forces_are_minus_energy_gradient(oracle_mod, pot, name):
    """F_i = -dU/dr_i (Algorithm 1 scatter), against finite differences of the
    total energy U = sum_i U_i."""
    s = SYSTEMS[name]
    nn, nl = lists(oracle_mod, pot, s.pos, s.box)
    o = evaluate(oracle_mod, pot, s.pos, s.box, nn, nl)
    fd = -_fd_grad(lambda x: _total_energy(oracle_mod, pot, x, s.box, nn, nl), s.pos.copy(), 1e-4)
    assert np.abs(o["F"]).max() > 0.1
    assert np.abs(o["F"] - fd).max() < 2e-7


@pytest.mark.parametrize("pot,name", CASES)
def test_pairwise_equals_conventional(oracle_mod, pot, name):
    """Section 2.3: sum_j F_ij with F_ij = dU_i/dr_ij - dU_j/dr_ji equals the
    conventional scatter force; the net force vanishes."""
    s = SYSTEMS[name]
    nn, nl = lists(oracle_mod, pot, s.pos, s.box)
    o = evaluate(oracle_mod, pot, s.pos, s.box, nn, nl)
    assert rel_err(o["Fpair"], o["F"]) < 1e-13
    assert np.abs(o["F"].sum(axis=0)).max() < 1e-12 * np.abs(o["F"]).max()


def _per_atom_partials_fd(oracle, pot, s, nn, nl, h=1e-4):
    """dU_i/dr_j for every i and j by 4th-order differences in r_j."""
    n = s.n
    out = np.zeros((n, n, 3))
    for j in range(n):
        for a in range(3):
            us = []
            for st in (-2, -1, 1, 2):
                x = s.pos.copy()
                x[j, a] += st * h
                us.append(evaluate(oracle, pot, x, s.box, nn, nl)["U"])
            out[:, j, a] = (us[0] - 8 * us[1] + 8 * us[2] - us[3]) / (12 * h)
    return out


@pytest.mark.parametrize("pot,name", CASES)
def test_per_atom_partials(oracle_mod, pot, name):
    """The captured G[i][m] equals dU_i/dr_{NL_im} = dU_i/dr_ij (the quantity
    behind the pairwise force, Section 2.3), U_i depends on no atom outside
    its list, and dU_i/dr_i = -sum_j dU_i/dr_ij."""
    s = SYSTEMS[name]
    nn, nl = lists(oracle_mod, pot, s.pos, s.box)
    o = evaluate(oracle_mod, pot, s.pos, s.box, nn, nl, want_g=True)
    fd = _per_atom_partials_fd(oracle_mod, pot, s, nn, nl)
    G = o["G"]
    scale = np.abs(fd).max()
    for i in range(s.n):
        nbrs = set(nl[i, :nn[i]].tolist())
        for j in range(s.n):
            if j == i:
                ref = -G[i, :nn[i]].sum(axis=0)
            elif j in nbrs:
                ref = G[i, list(nl[i, :nn[i]]).index(j)]
            else:
                ref = np.zeros(3)
            assert np.abs(fd[i, j] - ref).max() < 1e-7 * max(scale, 1.0), (i, j)


@pytest.mark.parametrize("pot,name", CASES)
def test_per_atom_virial_and_heat_current_definitions(oracle_mod, pot, name):
    """W_i = -1/2 sum_j r_ij (x) F_ij and J_i = sum_j r_ij (dU_j/dr_ji . v_i)
    (Section 2.3), rebuilt from finite-difference partials (not from the
    oracle's capture), component order W[3*alpha + beta]."""
    s = SYSTEMS[name]
    nn, nl = lists(oracle_mod, pot, s.pos, s.box)
    o = evaluate(oracle_mod, pot, s.pos, s.box, nn, nl, vel=s.vel)
    fd = _per_atom_partials_fd(oracle_mod, pot, s, nn, nl)
    W = np.zeros((s.n, 3, 3))
    J = np.zeros((s.n, 3))
    for i in range(s.n):
        for j in nl[i, :nn[i]]:
            d = s.pos[j] - s.pos[i]
            d -= s.box * np.rint(d / s.box)
            fij = fd[i, j] - fd[j, i]
            W[i] += -0.5 * np.outer(d, fij)
            J[i] += d * np.dot(fd[j, i], s.vel[i])
    assert np.abs(o["W"] - W.reshape(s.n, 9)).max() < 1e-6 * max(np.abs(W).max(), 1.0)
    assert np.abs(o["J"] - J).max() < 1e-6 * max(np.abs(J).max(), 1e-3)


@pytest.mark.parametrize("pot,name", CASES)
def test_heat_current_directional_derivative(oracle_mod, pot, name):
    """J_i = sum_j r_ij (d/d delta) U_j(r_i + delta v_i): the velocity
    projection of dU_j/dr_ji, by moving atom i alone along v_i."""
    s = SYSTEMS[name]
    nn, nl = lists(oracle_mod, pot, s.pos, s.box)
    o = evaluate(oracle_mod, pot, s.pos, s.box, nn, nl, vel=s.vel)
    for i in range(0, s.n, 3):
        v = s.vel[i]
        h = 1e-4 / np.linalg.norm(v)
        us = []
        for st in (-2, -1, 1, 2):
            x = s.pos.copy()
            x[i] += st * h * v
            us.append(evaluate(oracle_mod, pot, x, s.box, nn, nl)["U"])
        du = (us[0] - 8 * us[1] + 8 * us[2] - us[3]) / (12 * h)
        ji = np.zeros(3)
        for j in nl[i, :nn[i]]:
            d = s.pos[j] - s.pos[i]
            d -= s.box * np.rint(d / s.box)
            ji += d * du[j]
        assert np.abs(o["J"][i] - ji).max() < 1e-7 * max(np.abs(o["J"]).max(), 1e-3)


@pytest.mark.parametrize("pot", ["tersoff", "sw"])
def test_total_heat_current_energy_identity(oracle_mod, pot):
    """For an isolated cluster the potential heat current obeys
    J = sum_i r_i (F_i . v_i + dU_i/dt); the stress-based sum_i W_i . v_i of
    Section 2.3 does not (negative control)."""
    s = SYSTEMS["cluster"]
    nn, nl = lists(oracle_mod, pot, s.pos, s.box)
    o = evaluate(oracle_mod, pot, s.pos, s.box, nn, nl, vel=s.vel)
    h = 1e-2
    us = []
    for st in (-2, -1, 1, 2):
        us.append(evaluate(oracle_mod, pot, s.pos + st * h * s.vel, s.box, nn, nl)["U"])
    dudt = (us[0] - 8 * us[1] + 8 * us[2] - us[3]) / (12 * h)
    ref = np.sum(s.pos * (np.sum(o["F"] * s.vel, axis=1) + dudt)[:, None], axis=0)
    tot = o["J"].sum(axis=0)
    assert np.abs(tot - ref).max() < 1e-7 * np.abs(ref).max()
    stress = o["JL"].sum(axis=0)
    assert np.abs(stress - ref).max() > 1e-3 * np.abs(ref).max()


# ------------------------------------------------------------------ virial

@pytest.mark.parametrize("pot", ["tersoff", "sw"])
@pytest.mark.parametrize("name", ["crystal", "expanded", "vacancies"])
def test_virial_diagonal_finite_strain(oracle_mod, pot, name):
    """Total virial W = sum_i W_i (Section 2.3): W^aa = -dU/d eps_aa under a
    uniform periodic strain of box and positions along axis a."""
    s = SYSTEMS[name]
    nn, nl = lists(oracle_mod, pot, s.pos, s.box)
    o = evaluate(oracle_mod, pot, s.pos, s.box, nn, nl)
    W = o["W"].sum(axis=0).reshape(3, 3)
    for a in range(3):
        def u_of(e):
            x = s.pos.copy()
            b = s.box.copy()
            x[:, a] *= 1 + e
            b[a] *= 1 + e
            return _total_energy(oracle_mod, pot, x, b, nn, nl)
        h = 1e-5
        du = (u_of(-2 * h) - 8 * u_of(-h) + 8 * u_of(h) - u_of(2 * h)) / (12 * h)
        assert abs(W[a, a] + du) < 1e-6 * max(abs(du), 1.0)


@pytest.mark.parametrize("pot", ["tersoff", "sw"])
def test_virial_full_tensor_on_cluster(oracle_mod, pot):
    """Isolated cluster: W = sum_i r_i (x) F_i (the definition in Section 2.3)
    equals sum_i W_i, and W^{ab} = -dU/d eps_{ba} for r^b += eps r^a; the
    LAMMPS-form per-atom virial has the same total but other per-atom values."""
    s = SYSTEMS["cluster"]
    nn, nl = lists(oracle_mod, pot, s.pos, s.box)
    o = evaluate(oracle_mod, pot, s.pos, s.box, nn, nl)
    W = o["W"].sum(axis=0).reshape(3, 3)
    direct = np.einsum("ia,ib->ab", s.pos, o["F"])
    assert np.abs(W - direct).max() < 1e-10 * np.abs(W).max()
    for a in range(3):
        for b in range(3):
            def u_of(e):
                x = s.pos.copy()
                x[:, b] += e * s.pos[:, a]
                return _total_energy(oracle_mod, pot, x, s.box, nn, nl)
            h = 1e-6
            du = (u_of(-2 * h) - 8 * u_of(-h) + 8 * u_of(h) - u_of(2 * h)) / (12 * h)
            assert abs(W[a, b] + du) < 1e-5 * np.abs(W).max(), (a, b)
    assert np.abs(o["WL"].sum(axis=0) - o["W"].sum(axis=0)).max() < 1e-12 * np.abs(W).max()
    assert np.abs(o["WL"] - o["W"]).max() > 1e-3 * np.abs(o["W"]).max()


# ----------------------------------------------------------- invariances

@pytest.mark.parametrize("pot,name", CASES)
def test_translation_invariance(oracle_mod, pot, name):
    s = SYSTEMS[name]
    nn, nl = lists(oracle_mod, pot, s.pos, s.box)
    o = evaluate(oracle_mod, pot, s.pos, s.box, nn, nl, vel=s.vel)
    shift = np.random.default_rng(5).uniform(-7, 7, size=3)
    x2 = oracle_mod.wrap(s.pos + shift, s.box)
    nn2, nl2 = lists(oracle_mod, pot, x2, s.box)
    o2 = evaluate(oracle_mod, pot, x2, s.box, nn2, nl2, vel=s.vel)
    for k in ("U", "F", "W", "J"):
        assert rel_err(o2[k], o[k]) < 1e-12, k


@pytest.mark.parametrize("pot", ["tersoff", "sw"])
def test_rotation_covariance_cluster(oracle_mod, pot):
    """U invariant, F -> R F, W_i -> R W_i R^T, J_i -> R J_i (with v -> R v)."""
    s = SYSTEMS["cluster"]
    nn, nl = lists(oracle_mod, pot, s.pos, s.box)
    o = evaluate(oracle_mod, pot, s.pos, s.box, nn, nl, vel=s.vel)
    q, _ = np.linalg.qr(np.random.default_rng(7).normal(size=(3, 3)))
    R = q * np.sign(np.linalg.det(q))
    c = s.box / 2
    x2 = (s.pos - c) @ R.T + c
    v2 = s.vel @ R.T
    o2 = evaluate(oracle_mod, pot, x2, s.box, nn, nl, vel=v2)
    assert rel_err(o2["U"], o["U"]) < 1e-12
    assert rel_err(o2["F"], o["F"] @ R.T) < 1e-12
    Wr = np.einsum("ab,ibc,dc->iad", R, o["W"].reshape(-1, 3, 3), R).reshape(-1, 9)
    assert rel_err(o2["W"], Wr) < 1e-12
    assert rel_err(o2["J"], o["J"] @ R.T) < 1e-12


@pytest.mark.parametrize("pot,name", CASES)
def test_relabelling_permutes_outputs(oracle_mod, pot, name):
    s = SYSTEMS[name]
    nn, nl = lists(oracle_mod, pot, s.pos, s.box)
    o = evaluate(oracle_mod, pot, s.pos, s.box, nn, nl, vel=s.vel)
    perm = np.random.default_rng(9).permutation(s.n)
    x2, v2 = s.pos[perm], s.vel[perm]
    nn2, nl2 = lists(oracle_mod, pot, x2, s.box)
    o2 = evaluate(oracle_mod, pot, x2, s.box, nn2, nl2, vel=v2)
    for k in ("U", "F", "W", "J"):
        assert rel_err(o2[k], o[k][perm]) < 1e-13, k


def test_cubic_axis_permutation_and_reflection(oracle_mod):
    """Swapping x and y and reflecting z -> L - z are symmetries of a cubic
    periodic box: forces permute / flip, virial components follow."""
    s = SYSTEMS["crystal"]
    for pot in ("tersoff", "sw"):
        nn, nl = lists(oracle_mod, pot, s.pos, s.box)
        o = evaluate(oracle_mod, pot, s.pos, s.box, nn, nl, vel=s.vel)
        P = np.array([[0, 1, 0], [1, 0, 0], [0, 0, -1.0]])
        x2 = s.pos @ P.T
        x2[:, 2] += s.box[2]
        x2 = oracle_mod.wrap(x2, s.box)
        v2 = s.vel @ P.T
        nn2, nl2 = lists(oracle_mod, pot, x2, s.box)
        o2 = evaluate(oracle_mod, pot, x2, s.box, nn2, nl2, vel=v2)
        assert rel_err(o2["U"], o["U"]) < 1e-12
        assert rel_err(o2["F"], o["F"] @ P.T) < 1e-12
        Wp = np.einsum("ab,ibc,dc->iad", P, o["W"].reshape(-1, 3, 3), P).reshape(-1, 9)
        assert rel_err(o2["W"], Wp) < 1e-12
        assert rel_err(o2["J"], o["J"] @ P.T) < 1e-12


# -------------------------------------------------------- special cases

def test_dimer_and_isolated_atoms(oracle_mod):
    """zeta = 0 for a dimer (no third atom): U_ij = f_C (f_R - f_A), a pure
    pair potential; an atom with no neighbour has U = F = W = J = 0."""
    box = np.array([30.0, 30.0, 30.0])
    for r in (2.3, 2.85):       # below R and inside the taper (R, S)
        pos = np.array([[10.0, 10.0, 10.0], [10.0 + r, 10.0, 10.0], [25.0, 25.0, 25.0]])
        vel = np.array([[1e-3, 2e-3, -1e-3], [0.0, 1e-3, 0.0], [1e-3, 1e-3, 1e-3]])
        nn, nl = lists(oracle_mod, "tersoff", pos, box)
        o = evaluate(oracle_mod, "tersoff", pos, box, nn, nl, vel=vel)
        fc = 1.0 if r < TP["R"] else 0.5 + 0.5 * math.cos(math.pi * (r - TP["R"]) / (TP["S"] - TP["R"]))
        u = fc * (TP["A"] * math.exp(-TP["lam"] * r) - TP["B"] * math.exp(-TP["mu"] * r))
        assert abs(o["U"][0] - 0.5 * u) < 1e-13 * abs(u)
        assert abs(o["U"][1] - 0.5 * u) < 1e-13 * abs(u)
        assert o["U"][2] == 0 and np.all(o["F"][2] == 0) and np.all(o["W"][2] == 0)
        assert np.all(o["J"][2] == 0)
        fd = -_fd_grad(lambda x: _total_energy(oracle_mod, "tersoff", x, box, nn, nl), pos.copy(), 1e-5)
        assert np.abs(o["F"] - fd).max() < 1e-7


def test_third_atom_beyond_cutoff_contributes_nothing(oracle_mod):
    """A neighbour-list entry with S <= r < r_list leaves everything unchanged."""
    box = np.array([30.0, 30.0, 30.0])
    base = np.array([[10.0, 10.0, 10.0], [12.3, 10.0, 10.0], [10.0, 12.35, 10.0]])
    far = np.vstack([base, [[7.0, 10.0, 10.1]]])     # 3.0017 A from atom 0
    nn, nl = lists(oracle_mod, "tersoff", base, box)
    nn2, nl2 = lists(oracle_mod, "tersoff", far, box)
    assert nn2[0] == nn[0] + 1
    o = evaluate(oracle_mod, "tersoff", base, box, nn, nl)
    o2 = evaluate(oracle_mod, "tersoff", far, box, nn2, nl2)
    for k in ("U", "F", "W"):
        assert np.array_equal(o2[k][:3], o[k]), k


# ------------------------------------------------------------ neighbours

def _lists_numpy(pos, box, rlist):
    """Definition of the list with numpy: every j != i with minimum-image
    squared distance below r_list^2, ascending."""
    d = pos[None, :, :] - pos[:, None, :]
    d = d - box * np.rint(d / box)
    r2 = d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1] + d[..., 2] * d[..., 2]
    np.fill_diagonal(r2, np.inf)
    return [np.flatnonzero(row < rlist * rlist) for row in r2]


@pytest.mark.parametrize("rlist", [RL_T, RL_S])
@pytest.mark.parametrize("cells,sigma,vac,seed", [
    (2, 0.05, 0.0, 1), (2, 0.15, 0.05, 2), (3, 0.1, 0.02, 3), ((2, 3, 4), 0.15, 0.0, 4)])
def test_neighbor_lists_brute_cells_definition(oracle_mod, rlist, cells, sigma, vac, seed):
    s = wl.silicon_crystal(cells, seed=seed, sigma=sigma, vacancy_fraction=vac)
    nnb, nlb = oracle_mod.neighbors(s.pos, s.box, rlist, 48, method="brute")
    nnc, nlc = oracle_mod.neighbors(s.pos, s.box, rlist, 48, method="cells")
    assert np.array_equal(nnb, nnc) and np.array_equal(nlb, nlc)
    ref = _lists_numpy(s.pos, s.box, rlist)
    for i in range(s.n):
        assert np.array_equal(nlb[i, :nnb[i]], ref[i])


def test_neighbor_overflow_and_box_checks(oracle_mod):
    s = wl.silicon_crystal(2, seed=3)
    with pytest.raises(oracle_mod.OracleError) as e:
        oracle_mod.neighbors(s.pos, s.box, RL_S, 8)
    assert e.value.code == oracle_mod.ENEIGH
    with pytest.raises(oracle_mod.OracleError) as e:
        oracle_mod.neighbors(s.pos, s.box, 5.5, 64)     # 10.86 < 2 * 5.5
    assert e.value.code == oracle_mod.EBOX


# ------------------------------------------------------------ integrator

def test_nve_energy_conservation_and_dt2_order(oracle_mod):
    """Velocity-Verlet NVE (Section 3) on the 512-atom crystal: bounded energy
    error with no drift, shrinking ~dt^2 (ratio near 4 at half the step)."""
    s = wl.tersoff_small()
    r1 = oracle_mod.nve("tersoff", TP, s.pos, s.vel, s.box, wl.M_SI, 100, 1.0, RL_T, 20, 32)
    r2 = oracle_mod.nve("tersoff", TP, s.pos, s.vel, s.box, wl.M_SI, 200, 0.5, RL_T, 20, 32)
    e1 = r1["thermo"][:, 14]
    e2 = r2["thermo"][::2, 14]
    dev1 = np.abs(e1 - e1[0]).max() / s.n
    dev2 = np.abs(e2 - e2[0]).max() / s.n
    assert dev1 < 1e-4
    assert 3.0 < dev1 / dev2 < 5.0
    # thermo columns follow their definitions
    th = r1["thermo"][-1]
    assert abs(th[0] - r1["U"].sum()) < 1e-9
    assert abs(th[1] - 0.5 * wl.M_SI * np.sum(r1["vel"] ** 2) / wl.KAPPA) < 1e-12
    assert np.allclose(th[2:11], r1["W"].sum(axis=0), rtol=0, atol=1e-9)
    assert np.allclose(th[11:14], r1["J"].sum(axis=0), rtol=0, atol=1e-12)
    assert abs(th[15] - 2 * th[1] / ((3 * s.n - 3) * wl.K_B)) < 1e-9
    # starting temperature is the generator's 300 K
    assert abs(r1["thermo"][0, 15] - 300.0) < 1e-9


def test_nve_time_reversibility(oracle_mod):
    s = wl.tersoff_small()
    fw = oracle_mod.nve("tersoff", TP, s.pos, s.vel, s.box, wl.M_SI, 30, 1.0, RL_T, 10, 32)
    bw = oracle_mod.nve("tersoff", TP, fw["pos"], -fw["vel"], s.box, wl.M_SI, 30, 1.0, RL_T, 10, 32)
    d = bw["pos"] - s.pos
    d -= s.box * np.rint(d / s.box)
    assert np.abs(d).max() < 1e-9
    assert np.abs(bw["vel"] + s.vel).max() < 1e-11


def test_nve_rebuild_schedule_does_not_change_trajectory(oracle_mod):
    """List entries beyond the cutoff contribute nothing and the ascending
    order keeps the summation order, so the rebuild schedule cannot change
    the trajectory while the skin holds."""
    s = wl.tersoff_small()
    a = oracle_mod.nve("tersoff", TP, s.pos, s.vel, s.box, wl.M_SI, 25, 1.0, RL_T, 1, 32)
    b = oracle_mod.nve("tersoff", TP, s.pos, s.vel, s.box, wl.M_SI, 25, 1.0, RL_T, 20, 32)
    assert np.array_equal(a["pos"], b["pos"]) and np.array_equal(a["vel"], b["vel"])


def test_sw_nve_conserves_energy(oracle_mod):
    s = wl.silicon_crystal(3, seed=21)
    r = oracle_mod.nve("sw", SP, s.pos, s.vel, s.box, wl.M_SI, 60, 1.0, RL_S, 20, 48)
    e = r["thermo"][:, 14]
    assert np.abs(e - e[0]).max() / s.n < 1e-4


# ---- NPT with Berendsen weak coupling (the paper's benchmark ensemble) ----

@pytest.mark.parametrize("pot", ["tersoff", "sw"])
def test_npt_without_coupling_is_nve(oracle_mod, pot):
    """Both couplings off: the NPT run is the NVE run operation for
    operation (scaling by exactly 1), so every output matches bit for bit."""
    s = wl.silicon_crystal(3, seed=5, sigma=0.05)
    p, rl = (TP, RL_T) if pot == "tersoff" else (SP, RL_S)
    a = oracle_mod.nve(pot, p, s.pos, s.vel, s.box, wl.M_SI, 30, 1.0, rl, 10, 48,
                       check_skin=False)
    b = oracle_mod.npt(pot, p, s.pos, s.vel, s.box, wl.M_SI, 30, 1.0, rl, 10, 48,
                       300.0, 0.0, 0.0, 0.0, 0.0)
    for k in ("pos", "vel", "U", "F", "W", "J", "thermo"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(b["box"], s.box)
    assert np.array_equal(b["box_traj"], np.tile(s.box, (31, 1)))


@pytest.mark.parametrize("pot,a", [("tersoff", 5.40), ("tersoff", 5.47), ("sw", 5.45)])
def test_npt_pressure_is_minus_dU_dV(oracle_mod, pot, a):
    """At rest, the pressure the coupling uses, (2 E_kin + tr W) / (3 V),
    equals -dU/dV of the total energy under isotropic scaling of the
    positions and the box (central difference)."""
    s = wl.silicon_crystal(3, seed=6, sigma=0.04, a=a)
    p, rl = (TP, RL_T) if pot == "tersoff" else (SP, RL_S)
    zero = np.zeros_like(s.vel)
    r = oracle_mod.npt(pot, p, s.pos, zero, s.box, wl.M_SI, 0, 1.0, rl, 10, 48,
                       300.0, 0.0, 0.0, 0.0, 0.0)
    p_row = oracle_mod.pressure_GPa(r["thermo"][0], s.box)

    def energy(scale):
        pos, box = s.pos * scale, s.box * scale
        nn, nl = lists(oracle_mod, pot, pos, box, 48)
        return evaluate(oracle_mod, pot, pos, box, nn, nl)["U"].sum()

    h = 1e-5
    v0 = float(np.prod(s.box))
    dU = energy(1 + h) - energy(1 - h)
    dV = v0 * ((1 + h) ** 3 - (1 - h) ** 3)
    p_fd = -dU / dV * oracle_mod.EV_PER_A3_IN_GPA
    assert abs(p_row - p_fd) < 1e-6 * max(1.0, abs(p_fd)), (p_row, p_fd)


@pytest.mark.parametrize("t0", [150.0, 300.0])
def test_npt_thermostat_relaxes_temperature(oracle_mod, t0):
    """A crystal started at 600 K (it settles near 500 K uncoupled), coupled
    to t0 with a 20 fs time constant and no barostat, ends near t0."""
    s = wl.silicon_crystal(3, seed=7, sigma=0.05, temperature=600.0)
    r = oracle_mod.npt("tersoff", TP, s.pos, s.vel, s.box, wl.M_SI, 400, 1.0, RL_T, 10, 48,
                       t0, 20.0, 0.0, 0.0, 0.0)
    t_end = r["thermo"][-150:, 15].mean()
    assert abs(t_end - t0) < 0.1 * t0, t_end
    free = oracle_mod.npt("tersoff", TP, s.pos, s.vel, s.box, wl.M_SI, 400, 1.0, RL_T, 10, 48,
                          t0, 0.0, 0.0, 0.0, 0.0)
    assert free["thermo"][-150:, 15].mean() > 400.0


@pytest.mark.parametrize("a", [5.38, 5.49])
def test_npt_barostat_moves_toward_target_pressure(oracle_mod, a):
    """Compressed (positive pressure) and expanded (negative pressure)
    crystals coupled to 0 GPa: the box grows or shrinks accordingly and the
    pressure magnitude falls."""
    s = wl.silicon_crystal(3, seed=8, sigma=0.03, temperature=50.0, a=a)
    r = oracle_mod.npt("tersoff", TP, s.pos, s.vel, s.box, wl.M_SI, 300, 1.0, RL_T, 10, 48,
                       50.0, 100.0, 0.0, 100.0, 0.01)
    p0 = oracle_mod.pressure_GPa(r["thermo"][0], r["box_traj"][0])
    p_end = np.mean([oracle_mod.pressure_GPa(r["thermo"][k], r["box_traj"][k])
                     for k in range(250, 301)])
    grew = r["box_traj"][-1, 0] > r["box_traj"][0, 0]
    assert grew == (p0 > 0), (p0, r["box_traj"][[0, -1], 0])
    assert abs(p_end) < 0.5 * abs(p0), (p0, p_end)
    # isotropic: the three edges keep their ratios
    assert np.allclose(r["box_traj"][-1] / r["box_traj"][0], r["box"][0] / s.box[0], rtol=1e-12)


# Berendsen's coupling law, pinned on atoms that never interact: with every
# force zero the velocity-Verlet kicks add nothing, so the kinetic
# temperature and the volume follow the weak-coupling relations exactly,
#   T_{s+1} - T_s = (dt / tau_T) (T0 - T_s),
#   V_{s+1} / V_s - 1 = -(beta dt / tau_P) (P0 - P_s),  P_s = 2 E_kin,s / (3 V_s),
# which the recursions below integrate with no square or cube root: a
# velocity factor without its square root, or a box factor without its cube
# root, misses them at the first step.

@pytest.mark.parametrize("T0,tau_T,P0_GPa,tau_P,beta_GPa", [
    (150.0, 10.0, 0.0, 0.0, 0.0),      # thermostat only, cooling
    (900.0, 7.0, 0.0, 0.0, 0.0),       # thermostat only, heating
    (0.0, 0.0, 0.0, 20.0, 1.0),        # barostat only, ideal-gas pressure: expands
    (0.0, 0.0, 0.2, 100.0, 1.0),       # barostat only, target above: compresses
    (500.0, 15.0, 0.1, 50.0, 2.0),     # both
])
def test_npt_follows_berendsen_law_on_free_atoms(oracle_mod, T0, tau_T, P0_GPa, tau_P,
                                                 beta_GPa):
    pos, vel, box = ideal_gas(seed=41)
    steps = 60
    r = oracle_mod.npt("tersoff", TP, pos, vel, box, wl.M_SI, steps, 1.0, RL_T, 10, 16,
                       T0, tau_T, P0_GPa, tau_P, beta_GPa)
    th = r["thermo"]
    # the premise: nothing interacted
    assert np.all(th[:, 0] == 0.0) and np.all(th[:, 2:11] == 0.0)
    ev = oracle_mod.EV_PER_A3_IN_GPA
    T, V = berendsen_law(th[0, 15], th[0, 1], float(np.prod(box)), steps, 1.0, T0, tau_T,
                         P0_GPa / ev, tau_P, beta_GPa * ev)
    assert rel_err(th[:, 15], T) <= 1e-12
    vol = np.prod(r["box_traj"], axis=1)
    assert rel_err(vol, V) <= 1e-12
    # isotropic: the edges keep their ratios
    assert np.allclose(r["box_traj"] / r["box_traj"][0], (vol / vol[0])[:, None] ** (1 / 3),
                       rtol=1e-12, atol=0)
    # the coupling actually moved something
    moved = max(np.abs(T - T[0]).max() / T[0], np.abs(V - V[0]).max() / V[0])
    assert moved > 1e-2


@pytest.mark.parametrize("pot", ["tersoff", "sw"])
def test_threaded_oracle_matches_serial(oracle_mod, pot):
    """The all-cores timing baseline: with several threads the per-atom
    energies, lists and pairwise W, J are the same bits (each written by its
    own atom's iteration) and the scattered forces differ only by the order
    of the per-thread sums."""
    s = wl.silicon_crystal(4, seed=51, sigma=0.1, vacancy_fraction=0.02)
    p, rl = (TP, RL_T) if pot == "tersoff" else (SP, RL_S)
    outs = []
    try:
        for t in (1, 4):
            assert oracle_mod.set_threads(t) == t
            nn, nl = oracle_mod.neighbors(s.pos, s.box, rl, 48)
            o = evaluate(oracle_mod, pot, s.pos, s.box, nn, nl, vel=s.vel)
            r = oracle_mod.nve(pot, p, s.pos, s.vel, s.box, wl.M_SI, 5, 1.0, rl, 3, 48)
            outs.append((nn, nl, o, r))
    finally:
        oracle_mod.set_threads(1)
    (nn1, nl1, o1, r1), (nn4, nl4, o4, r4) = outs
    assert np.array_equal(nn1, nn4) and np.array_equal(nl1, nl4)
    for k in ("U", "W", "J", "Fpair"):
        assert np.array_equal(o1[k], o4[k]), k
    assert rel_err(o4["F"], o1["F"]) <= 1e-14
    assert rel_err(r4["pos"], r1["pos"]) <= 1e-13
