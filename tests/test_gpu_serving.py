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
    one-structure-per-launch baseline bit for bit."""
    import paper_1610_03343_amd as mb
    from paper_1610_03343_amd import serving
    reqs = wl.serving_trace(24, rate_hz=400.0, seed=2001, max_cells=6, nve_steps=20)
    jobs = serving.jobs_from_requests(reqs)
    with context("tersoff") as ctx:
        res_b, st_b = serving.serve_batched(ctx, jobs, hbm_budget_bytes=256 << 20,
                                            max_structures=16, rebuild_every=10,
                                            keep_results=True)
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
