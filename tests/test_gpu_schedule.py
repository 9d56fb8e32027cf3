"""The fixed rebuild schedule the benchmark times, and resuming a run.

Section 3 of the paper times runs whose neighbour list is built once (or
every 5 steps) with the four-neighbour argument of the silicon crystal.  The
benchmark rebuilds every 20 steps with a 0.5 A skin and tracks no
displacement (MBMD_REBUILD_FIXED).  Atoms move up to ~0.37 A within one
such interval at 300 K, more than skin/2, so the textbook Verlet argument
does not cover it.  These tests show, on the benchmark's own inputs, that
the schedule misses no pair: the run agrees with one that rebuilds before
every step, whose lists are complete at every step.  A pair missed for one
step changes a force by ~0.1 eV/A and a position by ~1e-4 A within a few
steps; the two list orders alone leave rounding-level differences.

Resuming: a run of 40 steps equals, bit for bit, 20 steps followed by 20
more from the saved positions and velocities (and box), when the rebuild
schedule is in the same phase (the second run builds at its step 0, which
is a build step of the first).
"""
import numpy as np
import pytest
import torch

import workload as wl
from gpu_util import context, min_image, to_dev

pytestmark = pytest.mark.gpu


def _state(pos, vel):
    torch.cuda.synchronize()
    return pos.cpu().numpy().T.copy(), vel.cpu().numpy().T.copy()


def _advance(ctx, s, pos, vel, steps, every):
    out = ctx.nve_run(pos, vel, s.box, wl.M_SI, 1.0, steps, rebuild_every=every)
    torch.cuda.synchronize()
    return out["thermo"].cpu().numpy()


def _one_ulp(x):
    return torch.tensor(wl.soa(np.nextafter(x, np.inf)), device="cuda:0")


@pytest.mark.parametrize("pot,system", [("tersoff", "tersoff_512k"), ("sw", "sw_1m")])
def test_fixed_schedule_misses_no_pair(pot, system):
    """The benchmark's inputs (512,000-atom Tersoff Si, 1,000,000-atom SW Si)
    under its schedule (fixed, every 20 steps, 0.5 A skin) for the 1,000
    steps it times, against rebuilding before every step.  Over the first 60
    steps (three intervals) the positions agree within 1e-12 A; over the
    full 1,000 steps, within ten times the divergence that a one-ulp change
    of every coordinate grows into under the every-step schedule (a rounding
    difference grows with the dynamics' own instability, while a missed
    pair would leave ~1e-4 A)."""
    s = getattr(wl, system)()
    with context(pot) as ctx:
        ctx.set_rebuild_policy("fixed")
        runs = {}
        for every in (20, 1):
            pos, vel = to_dev(s.pos), to_dev(s.vel)
            th = _advance(ctx, s, pos, vel, 60, every)
            runs[every] = [pos, vel, th]
        x20, v20 = _state(runs[20][0], runs[20][1])
        x1, v1 = _state(runs[1][0], runs[1][1])
        dx60 = np.abs(min_image(x20 - x1, s.box)).max()
        dv60 = np.abs(v20 - v1).max()
        print(f"{system} 60 steps, fixed 20 vs every step: dx {dx60:.2e} A, dv {dv60:.2e} A/fs")
        assert dx60 <= 1e-12 and dv60 <= 1e-13, (dx60, dv60)
        # the rest of the 1,000 steps, from step 60 (a build step of both),
        # with a third run perturbed by one ulp
        pos_p, vel_p = _one_ulp(x1), runs[1][1].clone()
        _advance(ctx, s, runs[20][0], runs[20][1], 940, 20)
        _advance(ctx, s, runs[1][0], runs[1][1], 940, 1)
        _advance(ctx, s, pos_p, vel_p, 940, 1)
        xa, _ = _state(runs[20][0], runs[20][1])
        xb, _ = _state(runs[1][0], runs[1][1])
        xc, _ = _state(pos_p, vel_p)
        d_sched = np.abs(min_image(xa - xb, s.box)).max()
        d_ulp = np.abs(min_image(xc - xb, s.box)).max()
        print(f"{system} 1000 steps: fixed 20 vs every step {d_sched:.2e} A, "
              f"one-ulp divergence {d_ulp:.2e} A")
        assert d_sched <= 10.0 * d_ulp + 1e-12, (d_sched, d_ulp)
        assert d_sched <= 1e-8, d_sched


@pytest.mark.parametrize("pot", ["tersoff", "sw"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("policy", ["fixed", "skin"])
def test_nve_resume_is_bitwise(pot, precision, policy):
    """40 NVE steps equal 20 + 20 from the saved state, bit for bit: x, v,
    the last step's U, F, W, J and the thermo rows (row 20 appears in both
    halves)."""
    s = wl.silicon_crystal(5, seed=61, sigma=0.05)          # 1,000 atoms
    with context(pot) as ctx:
        ctx.set_rebuild_policy(policy)
        pa, va = to_dev(s.pos), to_dev(s.vel)
        full = ctx.nve_run(pa, va, s.box, wl.M_SI, 1.0, 40, rebuild_every=10,
                           precision=precision)
        torch.cuda.synchronize()
        st_full = ctx.run_stats()
        full = {k: v.cpu().numpy() for k, v in full.items()}
        pb, vb = to_dev(s.pos), to_dev(s.vel)
        first = ctx.nve_run(pb, vb, s.box, wl.M_SI, 1.0, 20, rebuild_every=10,
                            precision=precision)
        th1 = first["thermo"].cpu().numpy()
        saved_x, saved_v = pb.clone(), vb.clone()     # the checkpoint
        second = ctx.nve_run(saved_x, saved_v, s.box, wl.M_SI, 1.0, 20, rebuild_every=10,
                             precision=precision)
        torch.cuda.synchronize()
        second = {k: v.cpu().numpy() for k, v in second.items()}
    if policy == "skin":
        assert st_full["rollbacks"] == 0    # the premise: the schedule has one phase
    assert torch.equal(pa, saved_x) and torch.equal(va, saved_v)
    for k in ("U", "F", "W", "J"):
        assert np.array_equal(full[k], second[k]), k
    assert np.array_equal(full["thermo"][:21], th1)
    assert np.array_equal(full["thermo"][20:], second["thermo"])


@pytest.mark.parametrize("pot", ["tersoff", "sw"])
def test_npt_resume_is_bitwise(pot):
    """Berendsen NPT: 40 steps equal 20 + 20 from the saved positions,
    velocities and box, bit for bit, box path included."""
    s = wl.silicon_crystal(5, seed=62, sigma=0.05, a=5.45)
    kw = dict(T0=350.0, tau_T=50.0, P0_GPa=0.5, tau_P=200.0, beta_per_GPa=0.02)
    with context(pot) as ctx:
        pa, va = to_dev(s.pos), to_dev(s.vel)
        full = ctx.npt_run(pa, va, s.box.copy(), wl.M_SI, 1.0, 40, rebuild_every=10, **kw)
        pb, vb = to_dev(s.pos), to_dev(s.vel)
        first = ctx.npt_run(pb, vb, s.box.copy(), wl.M_SI, 1.0, 20, rebuild_every=10, **kw)
        second = ctx.npt_run(pb, vb, first["box"].copy(), wl.M_SI, 1.0, 20, rebuild_every=10,
                             **kw)
        torch.cuda.synchronize()
    assert torch.equal(pa, pb) and torch.equal(va, vb)
    assert np.array_equal(full["box"], second["box"])
    ft, fb = full["thermo"].cpu().numpy(), full["box_traj"].cpu().numpy()
    assert np.array_equal(ft[:21], first["thermo"].cpu().numpy())
    assert np.array_equal(ft[20:], second["thermo"].cpu().numpy())
    assert np.array_equal(fb[20:], second["box_traj"].cpu().numpy())
    for k in ("U", "F", "W", "J"):
        assert torch.equal(full[k], second[k]), k


def _drifting(seed, drift):
    """1,000-atom crystal at 300 K with a uniform drift (A/fs) added to
    every velocity: under the skin policy it outruns the skin every few
    steps, so runs rebuild off the fixed schedule too."""
    s = wl.silicon_crystal(5, seed=seed, sigma=0.05)
    s.vel = s.vel + np.asarray(drift)
    return s


@pytest.mark.parametrize("pot", ["tersoff", "sw"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("policy", ["fixed", "skin"])
def test_nve_continue_is_bitwise(pot, precision, policy):
    """mbmd_nve_continue: 40 steps equal 13 continued by 0, 14 and 13 steps,
    bit for bit: x, v, the last step's U, F, W, J, the thermo rows (row 0 of
    a continuation is the last row of the run it continues) and the number
    of list builds.  Under the skin policy the drift makes the runs rebuild
    off the schedule, on both sides of the splits."""
    s = _drifting(71, [0.03, -0.02, 0.015])
    every = 10
    with context(pot) as ctx:
        ctx.set_rebuild_policy(policy)
        pa, va = to_dev(s.pos), to_dev(s.vel)
        full = ctx.nve_run(pa, va, s.box, wl.M_SI, 1.0, 40, rebuild_every=every,
                           precision=precision)
        torch.cuda.synchronize()
        st_full = ctx.run_stats()
        full = {k: v.cpu().numpy() for k, v in full.items()}
        pb, vb = to_dev(s.pos), to_dev(s.vel)
        out = None
        rows, builds = [], 0
        for k, steps in enumerate((13, 0, 14, 13)):
            r = ctx.nve_run(pb, vb, s.box, wl.M_SI, 1.0, steps, rebuild_every=every,
                            precision=precision, out=out, cont=k > 0)
            out = {key: r[key] for key in ("U", "F", "W", "J")}
            torch.cuda.synchronize()
            rows.append(r["thermo"].cpu().numpy())
            builds += ctx.run_stats()["rebuilds"]
    if policy == "skin":
        # builds off the schedule (which alone builds at 0, 10, ..., 40)
        assert st_full["rebuilds"] > 5 and st_full["rollbacks"] >= 1, st_full
    assert builds == st_full["rebuilds"]
    assert torch.equal(pa, pb) and torch.equal(va, vb)
    for k in ("U", "F", "W", "J"):
        assert np.array_equal(full[k], out[k].cpu().numpy()), k
    th = full["thermo"]
    assert np.array_equal(rows[0], th[:14])
    assert np.array_equal(rows[1], th[13:14])
    assert np.array_equal(rows[2], th[13:28])
    assert np.array_equal(rows[3], th[27:41])


def test_nve_continue_errors():
    """A continuation names the run it continues: anything else is refused
    with MBMD_EINVAL, and a refused call leaves the run continuable."""
    import paper_1610_03343_amd as mb
    s = wl.silicon_crystal(3, seed=72)
    with context("tersoff") as ctx:
        p, v = to_dev(s.pos), to_dev(s.vel)
        with pytest.raises(mb.MbmdError) as e:                # nothing ran yet
            ctx.nve_run(p, v, s.box, wl.M_SI, 1.0, 5, cont=True)
        assert e.value.code == mb.MBMD_EINVAL
        out = ctx.nve_run(p, v, s.box, wl.M_SI, 1.0, 5, thermo=None)
        for kw in (dict(box=s.box * 1.01), dict(dt=0.5), dict(every=7), dict(prec="mixed"),
                   dict(F=True), dict(thermo=True)):
            o = dict(out)
            if kw.get("F"):
                o["F"] = out["F"].clone()
            with pytest.raises(mb.MbmdError) as e:
                ctx.nve_run(p, v, kw.get("box", s.box), wl.M_SI, kw.get("dt", 1.0), 5,
                            rebuild_every=kw.get("every", 20), precision=kw.get("prec", "fp64"),
                            thermo=kw.get("thermo", None), out=o, cont=True)
            assert e.value.code == mb.MBMD_EINVAL, kw
        ctx.nve_run(p, v, s.box, wl.M_SI, 1.0, 5, thermo=None, out=out, cont=True)
        ctx.compute(to_dev(s.pos), s.box)                      # reuses the workspace
        with pytest.raises(mb.MbmdError) as e:
            ctx.nve_run(p, v, s.box, wl.M_SI, 1.0, 5, thermo=None, out=out, cont=True)
        assert e.value.code == mb.MBMD_EINVAL


@pytest.mark.parametrize("pot,system", [("tersoff", "tersoff_512k"), ("sw", "sw_1m")])
def test_npt_list_built_once_misses_no_pair(pot, system):
    """The protocol of the paper's size sweep (Section 3): Berendsen NPT at
    300 K and 0 Pa for 1,000 steps with the list built once and never
    rebuilt.  On the benchmark's inputs the run agrees with one that rebuilds
    before every step (complete lists at every step, on each step's box)
    within ten times the divergence a one-ulp change of every coordinate
    grows into, and within 1e-8 A: no pair was missed."""
    s = getattr(wl, system)()
    kw = dict(T0=300.0, tau_T=100.0, P0_GPa=0.0, tau_P=1000.0, beta_per_GPa=0.0102)
    steps = 1000
    runs = {}
    with context(pot) as ctx:
        for name, every, x0 in (("once", steps + 1, s.pos), ("every", 1, s.pos),
                                ("every_ulp", 1, np.nextafter(s.pos, np.inf))):
            pos, vel = to_dev(x0), to_dev(s.vel)
            out = ctx.npt_run(pos, vel, s.box.copy(), wl.M_SI, 1.0, steps, every, **kw)
            torch.cuda.synchronize()
            runs[name] = (pos.cpu().numpy().T.copy(), out["box"].copy(), ctx.run_stats())
    assert runs["once"][2]["rebuilds"] == 1 and runs["every"][2]["rebuilds"] == steps + 1
    box = runs["every"][1]
    d_sched = np.abs(min_image(runs["once"][0] - runs["every"][0], box)).max()
    d_ulp = np.abs(min_image(runs["every_ulp"][0] - runs["every"][0], box)).max()
    d_box = np.abs(runs["once"][1] - runs["every"][1]).max()
    print(f"{system} NPT {steps} steps: list once vs every step {d_sched:.2e} A (box "
          f"{d_box:.2e} A), one-ulp divergence {d_ulp:.2e} A")
    assert d_sched <= 10.0 * d_ulp + 1e-12, (d_sched, d_ulp)
    assert d_sched <= 1e-8 and d_box <= 1e-9, (d_sched, d_box)
