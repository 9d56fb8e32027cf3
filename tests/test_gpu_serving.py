"""Serving batch: structures advanced together in shared launches give, bit
for bit, the results they give alone; admission works while others run;
the batch results match the CPU oracle."""
import numpy as np
import pytest

import workload as wl
from gpu_util import PARAMS, RLIST, TOL_FP64, context, min_image, oracle_compute, rel, to_dev

pytestmark = pytest.mark.gpu

MIX = [  # (cells, seed, sigma, vacancy fraction, n_steps)
    ((2, 2, 3), 201, 0.10, 0.03, 0),
    ((3, 2, 2), 202, 0.05, 0.00, 12),
    ((4, 4, 4), 203, 0.15, 0.05, 25),
    ((2, 3, 2), 204, 0.08, 0.02, 7),
    ((5, 3, 4), 205, 0.12, 0.00, 0),
    ((3, 3, 3), 206, 0.05, 0.04, 18),
]


def _systems():
    return [wl.silicon_crystal(c, seed=s, sigma=sg, vacancy_fraction=v) for c, s, sg, v, _ in MIX]


def _alone(ctx, s, n_steps, precision, rebuild_every):
    import torch
    pos, vel = to_dev(s.pos), to_dev(s.vel)
    if n_steps == 0:
        out = ctx.compute(pos, s.box, vel=vel, precision=precision)
        th = None
    else:
        out = ctx.nve_run(pos, vel, s.box, wl.M_SI, 1.0, n_steps, rebuild_every,
                          precision=precision)
        th = out["thermo"]
    torch.cuda.synchronize()
    res = {k: out[k].cpu().numpy() for k in ("U", "F", "W", "J")}
    res["pos"], res["vel"] = pos.cpu().numpy(), vel.cpu().numpy()
    if th is not None:
        res["thermo"] = th.cpu().numpy()
    return res


@pytest.mark.parametrize("pot", ["tersoff", "sw"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_equals_alone_bitwise(pot, precision):
    """Staggered admission (three structures first, the others after a few
    batch steps) and retirement as they finish; every output equals the same
    structure computed alone through mbmd_compute / mbmd_nve_run."""
    import torch
    systems = _systems()
    every = 5
    alone = []
    with context(pot) as ctx:
        ctx.set_rebuild_policy("fixed")
        for s, (_, _, _, _, k) in zip(systems, MIX):
            alone.append(_alone(ctx, s, k, precision, every))
    got = {}
    with context(pot) as ctx:
        ctx.batch_open(6000, 8, every)
        handles = {}
        thermo = {}

        def admit(idx):
            s, k = systems[idx], MIX[idx][4]
            th = torch.empty(k + 1, 16, dtype=torch.float64, device="cuda:0")
            h = ctx.batch_add(to_dev(s.pos), to_dev(s.vel), s.box, wl.M_SI, 1.0, k, thermo=th)
            handles[h] = idx
            thermo[idx] = th

        for idx in (0, 1, 2):
            admit(idx)
        step = 0
        while handles or len(got) < len(systems):
            if step == 3:
                for idx in (3, 4, 5):
                    admit(idx)
            ctx.batch_step(precision)
            step += 1
            for h in ctx.batch_finished():
                idx = handles.pop(h)
                n = systems[idx].n
                out = ctx.batch_retire(h, n)
                ctx.batch_sync()
                got[idx] = {k: v.cpu().numpy() for k, v in out.items()}
            assert step < 200
        ctx.batch_close()
    for idx, (a, b) in enumerate(zip(alone, [got[i] for i in range(len(systems))])):
        for k in ("U", "F", "W", "J", "pos", "vel"):
            assert np.array_equal(a[k], b[k]), (idx, k)
        if "thermo" in a:
            assert np.array_equal(a["thermo"], b["thermo"]), idx


@pytest.mark.parametrize("pot", ["tersoff", "sw"])
def test_build_lane_split_does_not_change_lists(pot):
    """The list build takes four lanes per atom in launches of at most 512
    blocks of 256 atoms and one lane above; the lists, and so every force,
    are the same either way.  Five 32,768-atom structures alone (four lanes)
    and in one batch of 163,840 atoms (one lane) give the same bits."""
    import torch
    systems = [wl.silicon_crystal(16, seed=260 + k, sigma=0.08) for k in range(5)]
    assert all(s.n <= 512 * 256 for s in systems) and sum(s.n for s in systems) > 512 * 256
    with context(pot) as ctx:
        alone = [_alone(ctx, s, 0, "fp64", 5) for s in systems]
    got = {}
    with context(pot) as ctx:
        ctx.batch_open(sum(s.n for s in systems), len(systems), 5)
        handles = {ctx.batch_add(to_dev(s.pos), to_dev(s.vel), s.box, wl.M_SI, 1.0, 0): k
                   for k, s in enumerate(systems)}
        ctx.batch_step("fp64")
        for h in ctx.batch_finished():
            k = handles.pop(h)
            out = ctx.batch_retire(h, systems[k].n)
            ctx.batch_sync()
            got[k] = {key: v.cpu().numpy() for key, v in out.items()}
        ctx.batch_close()
        torch.cuda.synchronize()
    assert sorted(got) == list(range(len(systems)))
    for k, a in enumerate(alone):
        for key in ("U", "F", "W", "J"):
            assert np.array_equal(a[key], got[k][key]), (k, key)


@pytest.mark.parametrize("pot", ["tersoff", "sw"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_pairwise_form_does_not_change_results(pot, precision):
    """The pairwise pass takes four lanes per atom in launches of at most 64
    blocks of 256 atoms and one thread per atom above, with the same bits:
    twenty 4,096-atom structures run 25 NVE steps alone (four lanes) and in
    one 81,920-atom batch (one thread), and every output and thermo row
    agrees."""
    import torch
    systems = [wl.silicon_crystal(8, seed=280 + k, sigma=0.1) for k in range(20)]
    n_steps, every = 25, 5
    assert systems[0].n <= 64 * 256 < sum(s.n for s in systems)
    with context(pot) as ctx:
        ctx.set_rebuild_policy("fixed")
        alone = [_alone(ctx, s, n_steps, precision, every) for s in systems]
    got = {}
    with context(pot) as ctx:
        ctx.batch_open(sum(s.n for s in systems), len(systems), every)
        handles, thermo = {}, {}
        for k, s in enumerate(systems):
            th = torch.empty(n_steps + 1, 16, dtype=torch.float64, device="cuda:0")
            h = ctx.batch_add(to_dev(s.pos), to_dev(s.vel), s.box, wl.M_SI, 1.0, n_steps,
                              thermo=th)
            handles[h], thermo[k] = k, th
        steps = 0
        while handles:
            ctx.batch_step(precision)
            steps += 1
            for h in ctx.batch_finished():
                k = handles.pop(h)
                out = ctx.batch_retire(h, systems[k].n)
                ctx.batch_sync()
                got[k] = {key: v.cpu().numpy() for key, v in out.items()}
                got[k]["thermo"] = thermo[k].cpu().numpy()
            assert steps < 100
        ctx.batch_close()
    for k, a in enumerate(alone):
        for key in ("U", "F", "W", "J", "pos", "vel", "thermo"):
            assert np.array_equal(a[key], got[k][key]), (k, key)


@pytest.mark.parametrize("pot", ["tersoff", "sw"])
def test_batch_single_points_match_oracle(pot):
    import torch
    systems = _systems()
    with context(pot) as ctx:
        ctx.batch_open(6000, 8, 10)
        hs = {}
        for idx, s in enumerate(systems):
            hs[ctx.batch_add(to_dev(s.pos), to_dev(s.vel), s.box, wl.M_SI, 1.0, 0)] = idx
        assert ctx.batch_step("fp64") == len(systems)
        fin = ctx.batch_finished()
        assert sorted(fin) == sorted(hs)
        for h in fin:
            s = systems[hs[h]]
            out = ctx.batch_retire(h, s.n)
            ctx.batch_sync()
            ref = oracle_compute(pot, s)
            for k in ("U", "F", "W", "J"):
                g = out[k].cpu().numpy()
                g = g.T if g.ndim == 2 else g
                assert rel(g, ref[k]) <= TOL_FP64, (k, rel(g, ref[k]))
        ctx.batch_close()


@pytest.mark.parametrize("pot,M", [("tersoff", 32), ("sw", 64)])
def test_batch_with_overflow_structures_bitwise(pot, M):
    """Compressed lattices, whose atoms exceed the fast site path, share the
    batch with ordinary crystals: the batch's overflow pass (always enqueued
    there) serves them, and every result equals the same structure alone."""
    import torch
    c = 2 if pot == "tersoff" else 3
    systems = [wl.silicon_crystal(c, seed=51, sigma=0.05, a=4.2),
               wl.silicon_crystal((3, 3, 2), seed=52, sigma=0.1),
               wl.silicon_crystal(c, seed=53, sigma=0.05, a=4.4)]
    nsteps = [3, 5, 0]
    every = 5
    alone = []
    with context(pot, max_neighbors=M) as ctx:
        ctx.set_rebuild_policy("fixed")
        for s, k in zip(systems, nsteps):
            alone.append(_alone(ctx, s, k, "fp64", every))
    got = {}
    with context(pot, max_neighbors=M) as ctx:
        ctx.batch_open(4000, 4, every)
        handles = {}
        for idx, (s, k) in enumerate(zip(systems, nsteps)):
            th = torch.empty(k + 1, 16, dtype=torch.float64, device="cuda:0")
            handles[ctx.batch_add(to_dev(s.pos), to_dev(s.vel), s.box, wl.M_SI, 1.0, k,
                                  thermo=th)] = idx
        steps = 0
        while handles:
            ctx.batch_step("fp64")
            steps += 1
            for h in ctx.batch_finished():
                idx = handles.pop(h)
                out = ctx.batch_retire(h, systems[idx].n)
                ctx.batch_sync()
                got[idx] = {k: v.cpu().numpy() for k, v in out.items()}
            assert steps < 50
        ctx.batch_close()
    for idx, a in enumerate(alone):
        for k in ("U", "F", "W", "J", "pos", "vel"):
            assert np.array_equal(a[k], got[idx][k]), (idx, k)
        if "thermo" in a:
            assert np.array_equal(a["thermo"], got[idx]["thermo"]), idx


def test_batch_admission_limits_and_errors():
    import paper_1610_03343_amd as mb
    s = wl.silicon_crystal(2, seed=7)
    with context("tersoff") as ctx:
        ctx.batch_open(150, 2, 10)
        h1 = ctx.batch_add(to_dev(s.pos), to_dev(s.vel), s.box, wl.M_SI, 1.0, 3)
        assert ctx.batch_capacity() == (150 - 64, 1, 150 - 64)
        h2 = ctx.batch_add(to_dev(s.pos), to_dev(s.vel), s.box, wl.M_SI, 1.0, 1)
        with pytest.raises(mb.MbmdError) as e:         # no slot left
            ctx.batch_add(to_dev(s.pos), to_dev(s.vel), s.box, wl.M_SI, 1.0, 1)
        assert e.value.code == mb.MBMD_EBUSY
        with pytest.raises(mb.MbmdError) as e:         # not finished
            ctx.batch_retire(h1, s.n)
        assert e.value.code == mb.MBMD_EBUSY
        with pytest.raises(mb.MbmdError):              # single calls refused while open
            ctx.compute(to_dev(s.pos), s.box)
        ctx.batch_step()
        ctx.batch_step()
        assert ctx.batch_finished() == [h2]
        ctx.batch_retire(h2, s.n)
        big = wl.silicon_crystal(3, seed=8)            # 216 atoms: no range that large
        with pytest.raises(mb.MbmdError) as e:
            ctx.batch_add(to_dev(big.pos), to_dev(big.vel), big.box, wl.M_SI, 1.0, 0)
        assert e.value.code == mb.MBMD_EBUSY
        ctx.batch_step()
        ctx.batch_step()
        assert ctx.batch_finished() == [h1]
        ctx.batch_retire(h1, s.n)
        ctx.batch_sync()
        assert ctx.batch_capacity() == (150, 2, 150)
        # a non-finite position is reported by the next sync, once
        bad = s.pos.copy()
        bad[3, 1] = np.nan
        h3 = ctx.batch_add(to_dev(bad), to_dev(s.vel), s.box, wl.M_SI, 1.0, 0)
        ctx.batch_step()
        with pytest.raises(mb.MbmdError) as e:
            ctx.batch_sync()
        assert e.value.code == mb.MBMD_ENONFINITE
        ctx.batch_sync()
        assert ctx.batch_finished() == [h3]
        ctx.batch_retire(h3, s.n)
        ctx.sync()
        ctx.batch_close()
        ctx.sync()


def test_serving_loop_trace_and_identity():
    """A short Poisson trace through the request loop: every request is
    served, latencies are recorded, and the results equal the
    one-structure-per-launch baseline bit for bit.  Several of these
    disordered requests (sigma up to 0.15 A, vacancies) outrun the skin
    within 10 steps: the batch reports them and the loop serves them again
    under the rebuild-on-skin policy, which the baseline uses throughout."""
    import paper_1610_03343_amd as mb
    from paper_1610_03343_amd import serving
    reqs = wl.serving_trace(24, rate_hz=400.0, seed=2001, max_cells=6, nve_steps=20)
    jobs = serving.jobs_from_requests(reqs)
    with context("tersoff") as ctx, context("tersoff") as rctx:
        res_b, st_b = serving.serve_batched(ctx, jobs, hbm_budget_bytes=256 << 20,
                                            max_structures=16, rebuild_every=10,
                                            keep_results=True, rerun_ctx=rctx)
    assert st_b.skin_reruns >= 1
    with context("tersoff") as ctx:
        res_s, st_s = serving.serve_sequential(ctx, jobs, rebuild_every=10, keep_results=True)
    assert len(res_b) == len(jobs) == len(res_s)
    sb, ss = st_b.summary(), st_s.summary()
    assert sb["requests"] == len(jobs) and sb["p99_ms"] >= sb["p50_ms"] > 0
    assert sb["max_in_flight"] >= 2
    for rid in res_b:
        for k in ("U", "F", "W", "J", "pos", "vel"):
            a = res_b[rid][k].cpu().numpy()
            b = res_s[rid][k].cpu().numpy()
            assert np.array_equal(a, b), (rid, k)
    assert mb.MBMD_OK == 0


def test_serving_loop_reports_device_errors():
    """The request loop checks the batch status once, at the end: a request
    with a non-finite position still surfaces as MBMD_ENONFINITE."""
    import paper_1610_03343_amd as mb
    from paper_1610_03343_amd import serving
    reqs = wl.serving_trace(8, rate_hz=400.0, seed=2002, max_cells=4, nve_steps=10)
    jobs = serving.jobs_from_requests(reqs)
    bad = jobs[3]
    pos = bad.pos.copy()
    pos[0, 1] = np.nan
    jobs[3] = serving.Job(bad.rid, bad.arrival_s, pos, bad.vel, bad.box, bad.n_steps)
    with context("tersoff") as ctx:
        with pytest.raises(mb.MbmdError) as e:
            serving.serve_batched(ctx, jobs, hbm_budget_bytes=128 << 20, max_structures=8,
                                  rebuild_every=5)
        assert e.value.code == mb.MBMD_ENONFINITE
        ctx.sync()


def _hot_and_cool(seed):
    """Two 216-atom crystals at 300 K; the hot one also drifts uniformly at
    0.08 A/fs, so its atoms move more than skin/2 = 0.25 A from their build
    positions within four steps, while the cool one's stay within ~0.1 A."""
    cool = wl.silicon_crystal(3, seed=seed, sigma=0.05)
    hot = wl.silicon_crystal(3, seed=seed + 1, sigma=0.05)
    hot.vel = hot.vel + np.array([0.06, -0.04, 0.03])
    return cool, hot


@pytest.mark.parametrize("pot", ["tersoff", "sw"])
def test_batch_reports_skin_violation_per_structure(pot):
    """Lists are rebuilt every 10 batch steps; the drifting structure outruns
    the skin in between and its retire call reports MBMD_ESKIN, the other
    structure of the same batch reports MBMD_OK and still equals its run
    alone bit for bit (the check only reads positions)."""
    import paper_1610_03343_amd as mb
    import torch
    cool, hot = _hot_and_cool(310)
    with context(pot) as ctx:
        ctx.set_rebuild_policy("fixed")
        alone = _alone(ctx, cool, 25, "fp64", 10)
    with context(pot) as ctx:
        ctx.batch_open(1000, 4, 10)
        hc = ctx.batch_add(to_dev(cool.pos), to_dev(cool.vel), cool.box, wl.M_SI, 1.0, 25)
        hh = ctx.batch_add(to_dev(hot.pos), to_dev(hot.vel), hot.box, wl.M_SI, 1.0, 25)
        outs = {}
        while len(outs) < 2:
            ctx.batch_step()
            for h in ctx.batch_finished():
                outs[h] = ctx.batch_retire(h, cool.n)
        ctx.batch_sync()          # skin violations are not batch-wide errors
        torch.cuda.synchronize()
        ctx.batch_close()
    assert int(outs[hh]["status"][0]) == mb.MBMD_ESKIN
    assert int(outs[hc]["status"][0]) == mb.MBMD_OK
    for k in ("U", "F", "W", "J", "pos", "vel"):
        assert np.array_equal(outs[hc][k].cpu().numpy(), alone[k]), k


def test_batch_reports_list_overflow_per_structure():
    """With room for 4 list entries, a compressed crystal overflows its
    lists and is reported MBMD_ENEIGH by its retire call (and by the batch
    sync), while a crystal at the equilibrium lattice constant, whose lists
    hold exactly its 4 bonds, is reported MBMD_OK."""
    import paper_1610_03343_amd as mb
    ok = wl.silicon_crystal(3, seed=320, sigma=0.03)
    squeezed = wl.silicon_crystal(3, seed=321, sigma=0.03, a=4.9)
    with context("tersoff", max_neighbors=4) as ctx:
        ctx.batch_open(1000, 4, 10)
        h_ok = ctx.batch_add(to_dev(ok.pos), to_dev(ok.vel), ok.box, wl.M_SI, 1.0, 3)
        h_sq = ctx.batch_add(to_dev(squeezed.pos), to_dev(squeezed.vel), squeezed.box, wl.M_SI,
                             1.0, 3)
        outs = {}
        while len(outs) < 2:
            ctx.batch_step()
            for h in ctx.batch_finished():
                outs[h] = ctx.batch_retire(h, ok.n)
        with pytest.raises(mb.MbmdError) as e:
            ctx.batch_sync()
        assert e.value.code == mb.MBMD_ENEIGH
        ctx.batch_close()
    assert int(outs[h_sq]["status"][0]) == mb.MBMD_ENEIGH
    assert int(outs[h_ok]["status"][0]) == mb.MBMD_OK


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_serving_loop_reruns_skin_violations(precision):
    """The request loop serves a structure reported with MBMD_ESKIN again
    alone under the rebuild-on-skin policy: its results equal that run bit
    for bit, and the other requests still equal their runs alone on the
    batch's fixed schedule.  Without a context to rerun on, the loop raises
    MBMD_ESKIN."""
    import paper_1610_03343_amd as mb
    from paper_1610_03343_amd import serving
    cool, hot = _hot_and_cool(330)
    jobs = [serving.Job(0, 0.0, cool.pos, cool.vel, cool.box, 30),
            serving.Job(1, 0.0, hot.pos, hot.vel, hot.box, 30),
            serving.Job(2, 0.0, cool.pos, cool.vel, cool.box, 0)]
    with context("tersoff") as ctx, context("tersoff") as rctx:
        res, st = serving.serve_batched(ctx, jobs, precision=precision,
                                        hbm_budget_bytes=64 << 20, max_structures=4,
                                        rebuild_every=10, keep_results=True, saturate=True,
                                        rerun_ctx=rctx)
        with pytest.raises(mb.MbmdError) as e:
            serving.serve_batched(ctx, jobs, precision=precision, hbm_budget_bytes=64 << 20,
                                  max_structures=4, rebuild_every=10, saturate=True)
        assert e.value.code == mb.MBMD_ESKIN
        ctx.sync()
    assert st.skin_reruns == 1 and len(res) == 3 and not st.failed
    with context("tersoff") as ctx:
        ctx.set_rebuild_policy("skin")
        hot_alone = _alone(ctx, hot, 30, precision, 10)
        assert ctx.run_stats()["rollbacks"] >= 1
        ctx.set_rebuild_policy("fixed")
        cool_alone = _alone(ctx, cool, 30, precision, 10)
        cool_single = _alone(ctx, cool, 0, precision, 10)
    for rid, want in ((1, hot_alone), (0, cool_alone), (2, cool_single)):
        for k in ("U", "F", "W", "J", "pos", "vel"):
            assert np.array_equal(res[rid][k].numpy(), want[k]), (rid, k)
    assert np.array_equal(res[1]["thermo"].numpy(), hot_alone["thermo"])
