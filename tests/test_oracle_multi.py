"""Pins of the oracle's multicomponent Tersoff form (ora_tersoff_multi, and
the integrators with per-atom masses) against facts that do not come from
the oracle: Tersoff's published zincblende SiC properties, a 50-digit closed
form of the perfect zincblende crystal, reductions to the single-element
form, finite differences of the energy for forces and every per-atom
partial, the paper's pairwise-equals-scatter identity, the affine
dependence of the energy on chi, and energy conservation at second order in
the time step.  All run on the CPU."""
import math
import os

import numpy as np
import pytest

import workload as wl
from conftest import rel_err

SI, C, GE = wl.TERSOFF_SI_1989, wl.TERSOFF_C_1989, wl.TERSOFF_GE_1989
CHI_SIC = np.array([[1.0, wl.CHI_SI_C_1989], [wl.CHI_SI_C_1989, 1.0]])
CHI_SIGE = np.array([[1.0, wl.CHI_SI_GE_1989], [wl.CHI_SI_GE_1989, 1.0]])
RL_SIC = 3.0 + 0.5          # largest S (Si-Si) plus skin
RL_SIGE = 3.1 + 0.5
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden_properties():
    out = {}
    with open(os.path.join(GOLDEN, "published_sic_properties.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, val, tol, _unit = line.split()
            out[key] = (float(val), float(tol))
    return out


def multi(elems, chi, types):
    return dict(elems=elems, chi=chi, types=types)


def eval_multi(oracle, elems, chi, s, rl, vel=None, want_g=False, pos=None):
    pos = s.pos if pos is None else pos
    nn, nl = oracle.neighbors(pos, s.box, rl, 48)
    return oracle.tersoff_multi(multi(elems, chi, s.types), pos, s.box, nn, nl, vel=vel,
                                want_g=want_g)


def systems():
    """SiC and SiGe structures with bonds inside and across the tapers."""
    zb = wl.binary_crystal(2, seed=41, a=4.36, sigma=0.08)
    # expanded so Si-C first neighbours (2.47 A) sit in the (2.20, 2.51) taper
    zb_taper = wl.binary_crystal(2, seed=42, a=5.7, sigma=0.05)
    alloy = wl.binary_crystal(2, seed=43, a=5.0, arrangement="random", fraction=0.4,
                              sigma=0.15)
    sige = wl.binary_crystal(2, seed=44, a=5.54, arrangement="random", masses=(wl.M_SI, wl.M_GE),
                             sigma=0.1)
    return dict(zincblende=(zb, [SI, C], CHI_SIC, RL_SIC),
                zincblende_taper=(zb_taper, [SI, C], CHI_SIC, RL_SIC),
                sic_alloy=(alloy, [SI, C], CHI_SIC, RL_SIC),
                sige_alloy=(sige, [SI, GE], CHI_SIGE, RL_SIGE))


SYSTEMS = systems()


def _perfect_zb_energy(oracle, a):
    pos, box = wl.diamond_lattice(2, 2, 2, a=a)
    s = wl.System(pos, np.zeros_like(pos), box, 0,
                  type_ids=np.tile(np.array([0, 0, 0, 0, 1, 1, 1, 1], np.int32), 8))
    return eval_multi(oracle, [SI, C], CHI_SIC, s, RL_SIC)


def test_sic_published_crystal_properties(oracle_mod):
    """Tersoff (1989) zincblende SiC: E_c = 6.165 eV, a = 4.32 A, B = 2.24 Mbar."""
    from scipy.optimize import minimize_scalar
    g = golden_properties()
    e = lambda a: _perfect_zb_energy(oracle_mod, a)["U"].mean()
    r = minimize_scalar(e, bracket=(4.28, 4.32, 4.36), tol=1e-12)
    assert abs(r.x - g["sic_lattice_constant"][0]) < g["sic_lattice_constant"][1]
    assert abs(r.fun - g["sic_cohesive_energy"][0]) < g["sic_cohesive_energy"][1]
    v0 = r.x ** 3 / 8.0
    h = 1e-3 * v0
    ev = lambda v: e((8.0 * v) ** (1.0 / 3.0))
    bulk = v0 * (ev(v0 + h) - 2 * ev(v0) + ev(v0 - h)) / h ** 2 * 1.602176634
    assert abs(bulk - g["sic_bulk_modulus"][0]) < g["sic_bulk_modulus"][1]


@pytest.mark.parametrize("a", ["4.36", "5.7"])
def test_zincblende_closed_form(oracle_mod, a):
    """Perfect zincblende: each atom has four unlike neighbours at a sqrt(3)/4
    and three partners each at cos theta = -1/3, so U_i = 2 f_C (f_R - b_i f_A)
    with the mixed pair constants and b_i = chi (1 + (beta_i zeta_i)^n_i)^(-1/2n_i),
    zeta_i = 3 f_C g_i(-1/3), g_i with atom i's own c, d, h; at a = 5.7 the
    bond lies in the taper.  50-digit mpmath."""
    import mpmath as mp
    mp.mp.dps = 50
    si, cc = (lambda k: mp.mpf(SI[k])), (lambda k: mp.mpf(C[k]))
    A, B = mp.sqrt(si("A") * cc("A")), mp.sqrt(si("B") * cc("B"))
    lam, mu = (si("lam") + cc("lam")) / 2, (si("mu") + cc("mu")) / 2
    R, S = mp.sqrt(si("R") * cc("R")), mp.sqrt(si("S") * cc("S"))
    chi = mp.mpf(wl.CHI_SI_C_1989)

    def site(e, r0):
        fc = mp.mpf(1) if r0 < R else mp.mpf("0.5") + mp.cos(mp.pi * (r0 - R) / (S - R)) / 2
        fr, fa = A * mp.exp(-lam * r0), B * mp.exp(-mu * r0)
        c2, d2, h = e("c") ** 2, e("d") ** 2, e("h")
        g = 1 + c2 / d2 - c2 / (d2 + (h + mp.mpf(1) / 3) ** 2)
        b = chi * (1 + (e("beta") * 3 * fc * g) ** e("n")) ** (-1 / (2 * e("n")))
        return 2 * fc * (fr - b * fa)

    r0 = mp.mpf(a) * mp.sqrt(3) / 4
    u = [float(site(e, r0)) for e in (si, cc)]
    # the double-precision lattice puts every bond within a few ulp of the box
    # edge of r0: the bound is |dU_i/dr| times that, plus rounding
    box = 2 * float(a)
    slope = max(abs(float(mp.diff(lambda r: site(e, r), r0))) for e in (si, cc))
    tol = slope * 4 * np.finfo(float).eps * box + 1e-14 * max(abs(x) for x in u)
    o = _perfect_zb_energy(oracle_mod, float(a))
    ref = np.where(np.tile(np.array([0, 0, 0, 0, 1, 1, 1, 1]), 8) == 0, u[0], u[1])
    assert np.max(np.abs(o["U"] - ref)) < tol
    assert np.abs(o["F"]).max() < 1e-12


def test_one_type_through_multi_is_single_element(oracle_mod):
    """nt = 1 with chi = 1 is the single-element form, bit for bit."""
    s = wl.silicon_crystal(2, seed=11, sigma=0.1)
    nn, nl = oracle_mod.neighbors(s.pos, s.box, 3.5, 48)
    a = oracle_mod.tersoff(SI, s.pos, s.box, nn, nl, vel=s.vel)
    b = oracle_mod.tersoff_multi(multi([SI], [[1.0]], s.types), s.pos, s.box, nn, nl, vel=s.vel)
    for k in ("U", "F", "W", "J", "Fpair"):
        assert np.array_equal(a[k], b[k]), k


def test_identical_elements_reduce_to_single_element(oracle_mod):
    """Two types carrying the same parameters with chi = 1: the mixing rules
    return those parameters exactly, so any type assignment gives the
    single-element result bit for bit."""
    s = wl.binary_crystal(2, seed=45, a=5.3, arrangement="random", sigma=0.12)
    nn, nl = oracle_mod.neighbors(s.pos, s.box, 3.5, 48)
    a = oracle_mod.tersoff(SI, s.pos, s.box, nn, nl, vel=s.vel)
    b = oracle_mod.tersoff_multi(multi([SI, SI], None, s.types), s.pos, s.box, nn, nl,
                                 vel=s.vel)
    assert 0 < s.types.sum() < s.n
    for k in ("U", "F", "W", "J"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("name", list(SYSTEMS))
def test_multi_forces_are_minus_energy_gradient(oracle_mod, name):
    s, elems, chi, rl = SYSTEMS[name]
    o = eval_multi(oracle_mod, elems, chi, s, rl)
    rng = np.random.default_rng(7)
    h = 1e-5
    for i in rng.choice(s.n, size=8, replace=False):
        for c in range(3):
            p = s.pos.copy()
            p[i, c] += h
            ep = eval_multi(oracle_mod, elems, chi, s, rl, pos=p)["U"].sum()
            p[i, c] -= 2 * h
            em = eval_multi(oracle_mod, elems, chi, s, rl, pos=p)["U"].sum()
            fd = -(ep - em) / (2 * h)
            assert abs(fd - o["F"][i, c]) < 1e-6 * max(1.0, np.abs(o["F"]).max()), (i, c)


@pytest.mark.parametrize("name", list(SYSTEMS))
def test_multi_per_atom_partials(oracle_mod, name):
    """The captured dU_i/dr_j against central differences of U_i alone."""
    s, elems, chi, rl = SYSTEMS[name]
    nn, nl = oracle_mod.neighbors(s.pos, s.box, rl, 48)
    o = oracle_mod.tersoff_multi(multi(elems, chi, s.types), s.pos, s.box, nn, nl, want_g=True)
    rng = np.random.default_rng(8)
    h = 1e-5
    for i in rng.choice(s.n, size=4, replace=False):
        for m in range(nn[i]):
            j = nl[i, m]
            for c in range(3):
                p = s.pos.copy()
                p[j, c] += h
                up = oracle_mod.tersoff_multi(multi(elems, chi, s.types), p, s.box, nn, nl)["U"][i]
                p[j, c] -= 2 * h
                um = oracle_mod.tersoff_multi(multi(elems, chi, s.types), p, s.box, nn, nl)["U"][i]
                fd = (up - um) / (2 * h)
                assert abs(fd - o["G"][i, m, c]) < 1e-6 * max(1.0, np.abs(o["G"]).max())


@pytest.mark.parametrize("name", list(SYSTEMS))
def test_multi_pairwise_equals_scatter(oracle_mod, name):
    """Section 2.3: sum_j F_ij equals the conventional scatter force."""
    s, elems, chi, rl = SYSTEMS[name]
    o = eval_multi(oracle_mod, elems, chi, s, rl)
    assert rel_err(o["Fpair"], o["F"]) < 1e-12
    assert np.abs(o["F"].sum(axis=0)).max() < 1e-10


def test_energy_is_affine_in_chi(oracle_mod):
    """chi multiplies b_ij of unlike bonds only, so the total energy is an
    affine function of chi(Si-C): equal steps in chi give equal energy
    steps, and chi enters nothing for a pure-Si system."""
    s, elems, _chi, rl = SYSTEMS["sic_alloy"]
    e = []
    for x in (0.9, 0.95, 1.0):
        chi = np.array([[1.0, x], [x, 1.0]])
        e.append(eval_multi(oracle_mod, elems, chi, s, rl)["U"].sum())
    assert abs((e[2] - e[1]) - (e[1] - e[0])) < 1e-10 * abs(e[1])
    assert abs(e[2] - e[1]) > 1e-3
    pure = wl.System(s.pos, s.vel, s.box, 0, type_ids=np.zeros(s.n, np.int32))
    a = eval_multi(oracle_mod, elems, np.array([[1.0, 0.5], [0.5, 1.0]]), pure, rl)["U"]
    b = eval_multi(oracle_mod, elems, None, pure, rl)["U"]
    assert np.array_equal(a, b)


def test_sublattice_swap_symmetry(oracle_mod):
    """Swapping the two elements of perfect zincblende maps the crystal onto
    itself by inversion: same total energy, per-type energies exchanged."""
    pos, box = wl.diamond_lattice(2, 2, 2, a=4.5)
    t = np.tile(np.array([0, 0, 0, 0, 1, 1, 1, 1], np.int32), 8)
    a = eval_multi(oracle_mod, [SI, C], CHI_SIC, wl.System(pos, 0 * pos, box, 0, type_ids=t),
                   RL_SIC)["U"]
    b = eval_multi(oracle_mod, [SI, C], CHI_SIC, wl.System(pos, 0 * pos, box, 0, type_ids=1 - t),
                   RL_SIC)["U"]
    assert abs(a.sum() - b.sum()) < 1e-12 * abs(a.sum())
    assert abs(a[t == 0].mean() - b[t == 1].mean()) < 1e-12


def test_multi_nve_energy_conservation_second_order(oracle_mod):
    """Per-atom masses in the integrator: the total-energy excursion of a SiC
    alloy falls as dt^2 (ratio 4 for half the step)."""
    s, elems, chi, rl = SYSTEMS["sic_alloy"]
    masses = np.array([wl.M_SI, wl.M_C])[s.types]
    spread = []
    for dt, steps in ((0.5, 200), (0.25, 400)):
        r = oracle_mod.nve("tersoff_multi", multi(elems, chi, s.types), s.pos, s.vel, s.box, 0.0,
                           steps, dt, rl, 10, 48, check_skin=False, masses=masses)
        e = r["thermo"][:, 14]
        spread.append(e.max() - e.min())
    assert 3.0 < spread[0] / spread[1] < 5.0
    # the same run with every mass equal to the scalar mass is the scalar run
    m = np.full(s.n, wl.M_SI)
    a = oracle_mod.nve("tersoff_multi", multi(elems, chi, s.types), s.pos, s.vel, s.box, wl.M_SI,
                       20, 1.0, rl, 10, 48, check_skin=False)
    b = oracle_mod.nve("tersoff_multi", multi(elems, chi, s.types), s.pos, s.vel, s.box, 0.0,
                       20, 1.0, rl, 10, 48, check_skin=False, masses=m)
    assert np.array_equal(a["pos"], b["pos"]) and np.array_equal(a["thermo"], b["thermo"])


def test_trimer_closed_form_pair_selection(oracle_mod):
    """Si(i) at the origin, C(j) at 1.9 A and Si(k) at 2.6 A, 100 degrees
    apart, in a large box.  zeta_ij takes f_C of the Si-Si pair at 2.6 A (1,
    below R_SiSi = 2.7) while the Si-C cutoff (S = 2.51) would give 0; j-k is
    3.48 A, outside both.  Site energies by hand (50-digit mpmath):
      U_i = 1/2 [f_C^SiC(r_ij) (f_R^SiC - chi b(zeta_ij) f_A^SiC)
                 + f_C^SiSi(r_ik) (f_R^SiSi - b(zeta_ik) f_A^SiSi)],
      zeta_ij = f_C^SiSi(r_ik) g_Si(cos), zeta_ik = f_C^SiC(r_ij) g_Si(cos),
      U_j = 1/2 f_C^SiC (f_R^SiC - chi f_A^SiC)  (no partner: b = chi),
      U_k = 1/2 f_C^SiSi (f_R^SiSi - f_A^SiSi)."""
    import mpmath as mp
    mp.mp.dps = 50
    th = mp.pi * 100 / 180
    rij, rik = mp.mpf("1.9"), mp.mpf("2.6")
    si, cc = (lambda k: mp.mpf(SI[k])), (lambda k: mp.mpf(C[k]))

    def pair(x, y):
        return dict(A=mp.sqrt(x("A") * y("A")), B=mp.sqrt(x("B") * y("B")),
                    lam=(x("lam") + y("lam")) / 2, mu=(x("mu") + y("mu")) / 2,
                    R=mp.sqrt(x("R") * y("R")), S=mp.sqrt(x("S") * y("S")))

    def fc(p, r):
        if r < p["R"]:
            return mp.mpf(1)
        if r >= p["S"]:
            return mp.mpf(0)
        return mp.mpf("0.5") + mp.cos(mp.pi * (r - p["R"]) / (p["S"] - p["R"])) / 2

    def bond(p, r, b):
        return fc(p, r) * (p["A"] * mp.exp(-p["lam"] * r) - b * p["B"] * mp.exp(-p["mu"] * r))

    def bo(e, z):
        return (1 + (e("beta") * z) ** e("n")) ** (-1 / (2 * e("n"))) if z > 0 else mp.mpf(1)

    chi = mp.mpf(wl.CHI_SI_C_1989)
    psc, pss = pair(si, cc), pair(si, si)
    c2, d2, h = si("c") ** 2, si("d") ** 2, si("h")
    g = 1 + c2 / d2 - c2 / (d2 + (h - mp.cos(th)) ** 2)
    zij, zik = fc(pss, rik) * g, fc(psc, rij) * g
    ui = (bond(psc, rij, chi * bo(si, zij)) + bond(pss, rik, bo(si, zik))) / 2
    uj = bond(psc, rij, chi) / 2
    uk = bond(pss, rik, mp.mpf(1)) / 2
    L = 30.0
    pos = np.array([[10.0, 10.0, 10.0],
                    [10.0 + 1.9, 10.0, 10.0],
                    [10.0 + 2.6 * math.cos(math.radians(100)), 10.0 + 2.6 * math.sin(math.radians(100)), 10.0]])
    s = wl.System(pos, np.zeros_like(pos), np.full(3, L), 0, type_ids=np.array([0, 1, 0], np.int32))
    assert abs(np.linalg.norm(pos[2] - pos[1]) - 3.48) < 0.01
    o = eval_multi(oracle_mod, [SI, C], CHI_SIC, s, RL_SIC)
    ref = np.array([float(ui), float(uj), float(uk)])
    assert np.max(np.abs(o["U"] - ref)) < 1e-12 * np.max(np.abs(ref))
    assert float(zij) > 0 and float(fc(psc, rik)) == 0.0


def pair_radii(elems, skin=0.5):
    """List radius of each type pair: the pair's cutoff sqrt(S_a S_b) (the
    mixing rule of the multicomponent form) plus the skin."""
    return np.array([[math.sqrt(a["S"] * b["S"]) + skin for b in elems] for a in elems])


@pytest.mark.parametrize("name", list(SYSTEMS))
def test_typed_lists_match_a_periodic_kd_tree(oracle_mod, name):
    """The oracle's per-pair-radius lists against scipy's periodic k-d tree:
    every pair within the largest radius, kept when closer than its own
    pair's radius; and the same lists as the one-radius brute force when
    every pair gets the largest radius."""
    from scipy.spatial import cKDTree
    s, elems, _chi, _rl = SYSTEMS[name]
    rp = pair_radii(elems)
    nn, nl = oracle_mod.neighbors_typed(s.pos, s.box, s.types, rp, 48)
    pos = np.mod(s.pos, s.box)
    tree = cKDTree(pos, boxsize=s.box)
    dm = tree.sparse_distance_matrix(tree, rp.max(), output_type="ndarray")
    i, j, r = dm["i"], dm["j"], dm["v"]
    keep = (i != j) & (r < rp[s.types[i], s.types[j]])
    want = [np.sort(j[keep & (i == a)]) for a in range(s.n)]
    for a in range(s.n):
        assert np.array_equal(nl[a, :nn[a]], want[a]), a
    if name in ("zincblende", "sic_alloy"):
        # the radii change these lists (C-C pairs between 2.6 and 3.5 A)
        assert sum(len(w) for w in want) < int(np.sum((i != j) & (r < rp.max())))
    full = np.full_like(rp, rp.max())
    nn1, nl1 = oracle_mod.neighbors_typed(s.pos, s.box, s.types, full, 48)
    nn2, nl2 = oracle_mod.neighbors(s.pos, s.box, rp.max(), 48, method="brute")
    assert np.array_equal(nn1, nn2) and np.array_equal(nl1, nl2)


def test_typed_lists_reject_bad_input(oracle_mod):
    s, elems, _chi, _rl = SYSTEMS["zincblende"]
    rp = pair_radii(elems)
    with pytest.raises(ValueError):
        oracle_mod.neighbors_typed(s.pos, s.box, s.types, np.array([[3.0, 2.0], [2.5, 3.0]]), 48)
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.neighbors_typed(s.pos, s.box, s.types + 1, rp, 48)
