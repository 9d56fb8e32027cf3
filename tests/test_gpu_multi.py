"""Tersoff's multicomponent form on the GPU (mbmd_set_tersoff_multi) against
the oracle's ora_tersoff_multi.

FP64: U, F, W, J within 1e-12 of the oracle (norm-wise per output) on SiC
and SiGe crystals and alloys, bonds inside and across the tapers, several
tiles with ragged tails, and atoms served by the overflow pass; mixed path
forces within 1e-4 eV/A; one type through the multi-type entry point equals
the single-element path bit for bit; NVE and NPT trajectories with per-type
masses within ten times the oracle's own one-ulp divergence.
"""
import numpy as np
import pytest
import torch

import workload as wl
from gpu_util import TOL_FP64, TOL_MIXED_F, min_image, rel, to_dev

pytestmark = pytest.mark.gpu

SI, C, GE = wl.TERSOFF_SI_1989, wl.TERSOFF_C_1989, wl.TERSOFF_GE_1989
CHI_SIC = [[1.0, wl.CHI_SI_C_1989], [wl.CHI_SI_C_1989, 1.0]]
CHI_SIGE = [[1.0, wl.CHI_SI_GE_1989], [wl.CHI_SI_GE_1989, 1.0]]
SKIN = 0.5


def _systems():
    return {
        # name: (system, elements, chi, list capacity)
        "sic_zincblende": (wl.binary_crystal(2, seed=41, a=4.36, sigma=0.08), [SI, C], CHI_SIC, 32),
        "sic_taper": (wl.binary_crystal(2, seed=42, a=5.7, sigma=0.05), [SI, C], CHI_SIC, 16),
        "sic_alloy": (wl.binary_crystal(2, seed=43, a=5.0, arrangement="random", fraction=0.4,
                                        sigma=0.15), [SI, C], CHI_SIC, 32),
        "sige_alloy": (wl.binary_crystal(2, seed=44, a=5.54, arrangement="random",
                                         masses=(wl.M_SI, wl.M_GE), sigma=0.1),
                       [SI, GE], CHI_SIGE, 16),
        "sic_ragged_480": (wl.binary_crystal((3, 4, 5), seed=46, a=4.36, sigma=0.1), [SI, C],
                           CHI_SIC, 32),
        "sic_4096": (wl.binary_crystal(8, seed=47, a=4.36, sigma=0.1), [SI, C], CHI_SIC, 32),
        # compressed Si-rich alloy: Si-Si second neighbours (2.97 A) fall
        # inside S_SiSi = 3.0, so Si atoms hold up to 16 bonds (overflow pass)
        "sic_compressed": (wl.binary_crystal(2, seed=48, a=4.2, arrangement="random",
                                             fraction=0.2, sigma=0.03), [SI, C], CHI_SIC, 48),
    }


SYSTEMS = _systems()


def rlist(elems):
    """The oracle's one list radius: the largest pair cutoff plus the skin.
    Its lists contain the library's per-pair lists, and the oracle's sums
    run over in-cutoff pairs only, so its results do not depend on it."""
    return max(e["S"] for e in elems) + SKIN


class multi_context:
    def __init__(self, elems, chi, M):
        import paper_1610_03343_amd as mb
        self.ctx = mb.Context(0)
        self.ctx.set_tersoff_multi(elems, chi)
        self.ctx.set_neighbor(SKIN, M)

    def __enter__(self):
        return self.ctx

    def __exit__(self, *exc):
        self.ctx.close()


def _types(s):
    return torch.tensor(s.types, dtype=torch.int32, device="cuda:0")


def _oracle(s, elems, chi, M, vel=True):
    import oracle
    nn, nl = oracle.neighbors(s.pos, s.box, rlist(elems), M)
    return oracle.tersoff_multi(dict(elems=elems, chi=np.array(chi), types=s.types), s.pos,
                                s.box, nn, nl, vel=s.vel if vel else None)


def _gpu(ctx, s, precision="fp64"):
    out = ctx.compute(to_dev(s.pos), s.box, vel=to_dev(s.vel), types=_types(s),
                      precision=precision)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy().T.copy() if v.dim() == 2 else v.cpu().numpy().copy()
            for k, v in out.items()}


@pytest.mark.parametrize("name", list(SYSTEMS))
def test_multi_fp64_parity(name):
    s, elems, chi, M = SYSTEMS[name]
    ref = _oracle(s, elems, chi, M)
    with multi_context(elems, chi, M) as ctx:
        got = _gpu(ctx, s)
    errs = {k: rel(got[k], ref[k]) for k in ("U", "F", "W", "J")}
    print(name, {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= TOL_FP64, (k, v)


@pytest.mark.parametrize("name", ["sic_zincblende", "sic_alloy", "sige_alloy", "sic_compressed"])
def test_multi_mixed_forces(name):
    """Crystals and alloys near equilibrium: within 1e-4 eV/A.  The
    compressed alloy (Si-Si pairs at 1.8 A, forces of tens of eV/A) is held
    to a relative bound instead: FP32 rounds each operation to 2^-24, and a
    partial sums a few hundred terms that partly cancel, so 1e-5 of the
    largest force (~100 roundings) bounds it."""
    s, elems, chi, M = SYSTEMS[name]
    ref = _oracle(s, elems, chi, M)
    with multi_context(elems, chi, M) as ctx:
        got = _gpu(ctx, s, "mixed")
    df = np.max(np.abs(got["F"] - ref["F"]))
    fmax = np.max(np.abs(ref["F"]))
    print(f"{name}: mixed max|dF| = {df:.2e} eV/A (max |F| {fmax:.2f} eV/A)")
    if name == "sic_compressed":
        assert df <= 1e-5 * fmax
    else:
        assert df <= TOL_MIXED_F


def test_one_type_equals_single_element_path():
    """ntypes = 1 through mbmd_set_tersoff_multi runs the single-element
    kernels: identical bits to mbmd_set_tersoff.  Two identical elements on a
    random type pattern run the multi-type kernels and agree to FP64 parity."""
    import paper_1610_03343_amd as mb
    s = wl.binary_crystal(3, seed=49, a=5.43, arrangement="random", sigma=0.1)
    pos, vel = to_dev(s.pos), to_dev(s.vel)
    with mb.Context(0) as ctx:
        ctx.set_tersoff(SI)
        ctx.set_neighbor(SKIN, 16)
        a = ctx.compute(pos, s.box, vel=vel)
        torch.cuda.synchronize()
        ctx.set_tersoff_multi([SI])
        b = ctx.compute(pos, s.box, vel=vel)
        torch.cuda.synchronize()
        for k in ("U", "F", "W", "J"):
            assert torch.equal(a[k], b[k]), k
        ctx.set_tersoff_multi([SI, SI])
        c = ctx.compute(pos, s.box, vel=vel, types=_types(s))
        torch.cuda.synchronize()
        for k in ("U", "F", "W", "J"):
            assert rel(c[k].cpu().numpy(), a[k].cpu().numpy()) <= TOL_FP64, k


def _chaos(run, s):
    a = run(s.pos, s.vel)
    rng = np.random.default_rng(99)
    p2 = np.nextafter(s.pos, np.where(rng.uniform(size=s.pos.shape) < 0.5, -np.inf, np.inf))
    v2 = np.nextafter(s.vel, np.where(rng.uniform(size=s.vel.shape) < 0.5, -np.inf, np.inf))
    b = run(p2, v2)
    tol = dict(x=max(10 * np.max(np.abs(min_image(a["pos"] - b["pos"], a.get("box", s.box)))),
                     1e-13),
               v=max(10 * np.max(np.abs(a["vel"] - b["vel"])), 1e-15),
               th=np.maximum(10 * np.max(np.abs(a["thermo"] - b["thermo"]), axis=0),
                             1e-12 * np.max(np.abs(a["thermo"]), axis=0)))
    return a, tol


@pytest.mark.parametrize("name,steps", [("sic_alloy", 100), ("sige_alloy", 100)])
def test_multi_nve_trajectory_with_type_masses(name, steps):
    import oracle
    s, elems, chi, M = SYSTEMS[name]
    tm = list(s.meta["masses"])
    masses = np.array(tm)[s.types]
    par = dict(elems=elems, chi=np.array(chi), types=s.types)
    run = lambda p, v: oracle.nve("tersoff_multi", par, p, v, s.box, 0.0, steps, 1.0,
                                  rlist(elems), 10, M, check_skin=True, masses=masses)
    ref, tol = _chaos(run, s)
    # These disordered starts move atoms up to 0.85 A in ten steps, beyond
    # any list's skin, so both sides rebuild early once an atom has moved
    # more than skin/2 (the library's default policy, the oracle's
    # check_skin); with every list complete the trajectory does not depend
    # on when each side rebuilds.
    with multi_context(elems, chi, M) as ctx:
        ctx.set_type_masses(tm)
        pos, vel = to_dev(s.pos), to_dev(s.vel)
        out = ctx.nve_run(pos, vel, s.box, 0.0, 1.0, steps, rebuild_every=10, types=_types(s))
        torch.cuda.synchronize()
        st = ctx.run_stats()
        assert 0.0 <= st["max_displacement"] <= SKIN / 2, st
        gp, gv, th = pos.cpu().numpy().T, vel.cpu().numpy().T, out["thermo"].cpu().numpy()
    print(f"{name}: tolerances x {tol['x']:.2e} A, v {tol['v']:.2e} A/fs")
    assert rel(th[0], ref["thermo"][0]) <= 1e-12
    assert np.max(np.abs(min_image(gp - ref["pos"], s.box))) <= tol["x"]
    assert np.max(np.abs(gv - ref["vel"])) <= tol["v"]
    assert np.all(np.abs(th - ref["thermo"]) <= tol["th"][None, :])


def test_multi_npt_trajectory_with_type_masses():
    import oracle
    s, elems, chi, M = SYSTEMS["sic_alloy"]
    tm = list(s.meta["masses"])
    masses = np.array(tm)[s.types]
    par = dict(elems=elems, chi=np.array(chi), types=s.types)
    k = dict(T0=600.0, tau_T=20.0, P0_GPa=0.0, tau_P=50.0, beta_per_GPa=0.005)
    run = lambda p, v: oracle.npt("tersoff_multi", par, p, v, s.box, 0.0, 60, 1.0, rlist(elems),
                                  1, M, k["T0"], k["tau_T"], k["P0_GPa"], k["tau_P"],
                                  k["beta_per_GPa"], masses=masses)
    ref, tol = _chaos(run, s)
    # NPT rebuilds on its schedule only: every step on both sides, since this
    # disordered start moves atoms ~0.1 A per step
    with multi_context(elems, chi, M) as ctx:
        ctx.set_type_masses(tm)
        pos, vel = to_dev(s.pos), to_dev(s.vel)
        out = ctx.npt_run(pos, vel, s.box, 0.0, 1.0, 60, rebuild_every=1, types=_types(s), **k)
        torch.cuda.synchronize()
        gp, gv = pos.cpu().numpy().T, vel.cpu().numpy().T
        bt = out["box_traj"].cpu().numpy()
    assert np.max(np.abs(bt - ref["box_traj"])) <= max(1e-13 * s.box[0],
                                                       10 * tol["x"])
    assert np.max(np.abs(min_image(gp - ref["pos"], ref["box"]))) <= tol["x"]
    assert np.max(np.abs(gv - ref["vel"])) <= tol["v"]


def _pair_cutoffs(elems):
    return np.array([[np.sqrt(a["S"] * b["S"]) for b in elems] for a in elems])


@pytest.mark.parametrize("name", list(SYSTEMS))
def test_typed_neighbor_lists_bitexact(name):
    """Per-pair list radii S_ab + skin: the GPU lists against the oracle's
    brute-force typed lists as exact index sets, ordered as stated (pairs
    inside their own cutoff S_ab first, then the others, each by index)."""
    import oracle
    s, elems, chi, M = SYSTEMS[name]
    S = _pair_cutoffs(elems)
    with multi_context(elems, chi, M) as ctx:
        nn, nl = ctx.neighbors(to_dev(s.pos), s.box, types=_types(s))
        torch.cuda.synchronize()
        nn, nl = nn.cpu().numpy(), nl.cpu().numpy()
    onn, onl = oracle.neighbors_typed(s.pos, s.box, s.types, S + SKIN, M)
    assert np.array_equal(nn, onn)
    for i in range(s.n):
        got = nl[:nn[i], i]
        assert np.array_equal(np.sort(got), onl[i, :onn[i]]), i
        d = min_image(s.pos[got] - s.pos[i], s.box)
        inside = np.sum(d * d, axis=1) < S[s.types[i], s.types[got]] ** 2
        k = int(inside.sum())
        assert inside[:k].all() and not inside[k:].any(), i
        assert np.all(np.diff(got[:k]) > 0) and np.all(np.diff(got[k:]) > 0), i


def test_typed_lists_without_types_use_the_first_pair():
    """types = NULL under a multi-element potential: every atom is type 0, so
    every list has the radius S_00 + skin.  Element 0 is carbon here, whose
    cutoff (2.1 A) is below silicon's, so the lists differ from those of the
    largest radius."""
    import oracle
    s, _elems, _chi, M = SYSTEMS["sic_alloy"]
    elems, chi = [C, SI], CHI_SIC
    with multi_context(elems, chi, M) as ctx:
        nn, nl = ctx.neighbors(to_dev(s.pos), s.box)
        torch.cuda.synchronize()
        nn, nl = nn.cpu().numpy(), nl.cpu().numpy()
    onn, onl = oracle.neighbors(s.pos, s.box, elems[0]["S"] + SKIN, M, method="brute")
    assert np.array_equal(nn, onn)
    for i in range(s.n):
        assert np.array_equal(np.sort(nl[:nn[i], i]), onl[i, :onn[i]]), i
    wide, _ = oracle.neighbors(s.pos, s.box, rlist(elems), M, method="brute")
    assert np.sum(wide) > np.sum(onn)


def test_multi_errors():
    import paper_1610_03343_amd as mb
    s, elems, chi, M = SYSTEMS["sic_alloy"]
    with mb.Context(0) as ctx:
        with pytest.raises(mb.MbmdError):
            ctx.set_tersoff_multi([SI] * 5)
        with pytest.raises(mb.MbmdError):
            ctx.set_tersoff_multi([SI, C], [[1.0, 0.9], [0.95, 1.0]])   # not symmetric
        with pytest.raises(mb.MbmdError):
            ctx.set_type_masses([28.0, -1.0])
        ctx.set_tersoff_multi(elems, chi)
        ctx.set_neighbor(SKIN, M)
        bad = _types(s).clone()
        bad[5] = 2
        with pytest.raises(mb.MbmdError) as e:
            ctx.compute(to_dev(s.pos), s.box, types=bad)
        assert e.value.code == mb.MBMD_EINVAL
        # mass 0 without type masses
        with pytest.raises(mb.MbmdError) as e:
            ctx.nve_run(to_dev(s.pos), to_dev(s.vel), s.box, 0.0, 1.0, 2, types=_types(s))
        assert e.value.code == mb.MBMD_EINVAL
        ctx.set_type_masses([wl.M_SI])       # one type short
        with pytest.raises(mb.MbmdError) as e:
            ctx.nve_run(to_dev(s.pos), to_dev(s.vel), s.box, 0.0, 1.0, 2, types=_types(s))
        assert e.value.code == mb.MBMD_EINVAL
        # SW knows one type only
        ctx.set_sw(wl.SW_SI_1985)
        with pytest.raises(mb.MbmdError) as e:
            ctx.compute(to_dev(s.pos), s.box, types=_types(s))
        assert e.value.code == mb.MBMD_EINVAL


def test_multi_full_size_sic_512k():
    """Every atom of the 512,000-atom zincblende SiC input the bench times
    (seed 1006, a = 4.32 A, list capacity 32) against the oracle, FP64."""
    s = wl.binary_crystal(40, seed=1006, a=4.32, sigma=0.05, masses=(wl.M_SI, wl.M_C))
    ref = _oracle(s, [SI, C], CHI_SIC, 32)
    with multi_context([SI, C], CHI_SIC, 32) as ctx:
        got = _gpu(ctx, s)
    errs = {k: rel(got[k], ref[k]) for k in ("U", "F", "W", "J")}
    print("sic 512k", {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= TOL_FP64, (k, v)


def test_sic_512k_fixed_schedule_misses_no_pair():
    """The benchmark's schedule on its 512,000-atom SiC input (lists rebuilt
    every 20 steps, per-pair radii S_ab + 0.5 A, no displacement check):
    60 NVE steps agree with the run that rebuilds before every step, whose
    lists are complete at every step.  A pair missed for even one step
    changes forces by far more than the rounding-level differences that
    the two list orders leave."""
    s = wl.binary_crystal(40, seed=1006, a=4.32, sigma=0.05, masses=(wl.M_SI, wl.M_C))
    res = {}
    for every in (20, 1):
        with multi_context([SI, C], CHI_SIC, 32) as ctx:
            ctx.set_rebuild_policy("fixed")
            ctx.set_type_masses([wl.M_SI, wl.M_C])
            pos, vel = to_dev(s.pos), to_dev(s.vel)
            out = ctx.nve_run(pos, vel, s.box, 0.0, 1.0, 60, rebuild_every=every,
                              types=_types(s))
            torch.cuda.synchronize()
            res[every] = (pos.cpu().numpy().T, vel.cpu().numpy().T,
                          out["thermo"].cpu().numpy())
    dx = np.max(np.abs(min_image(res[20][0] - res[1][0], s.box)))
    dv = np.max(np.abs(res[20][1] - res[1][1]))
    de = np.max(np.abs(res[20][2][:, 14] - res[1][2][:, 14])) / s.n
    print(f"sic 512k, fixed 20 vs every step: dx {dx:.2e} A, dv {dv:.2e} A/fs, "
          f"dE {de:.2e} eV/atom")
    assert dx <= 1e-9 and dv <= 1e-10 and de <= 1e-12, (dx, dv, de)
