"""Request loop for the serving batch (continuous batching).

Requests (structures with a single-point or short-MD job) arrive over time.
The loop admits waiting requests in arrival order whenever the batch has a
free structure slot and a contiguous free atom range large enough, so new
work joins structures that are already mid-run; every loop iteration is one
mbmd_batch_step over all unfinished structures; finished structures are
retired at once, their results are copied to the host, and their latency
(arrival to results on the host) is recorded.  The batch's atom capacity is
set from an HBM budget, so admission is by free device memory.

The loop never drains the stream while it runs: a retirement's copies to
pinned host memory are followed by an event that later iterations poll, and
the host stays at most MAX_STEPS_AHEAD batch steps ahead of the GPU (it waits
on the event of an older step), so the GPU always has queued work while the
host admits and retires.  A request's latency ends when the host sees its
copy complete.  Each retired structure's own status comes back with its
results: a structure whose atoms outran the skin between two scheduled list
builds (MBMD_ESKIN) is served again alone under the rebuild-on-skin policy,
whose results then stand (and its latency ends when they are on the host);
a structure with any other error is dropped (its rid and code are kept in
the statistics) while the loop serves the rest.  At the end the batch's
device status is checked, and the loop raises if a request failed.

The one-structure-per-launch path serves the same trace in arrival order
through mbmd_compute / mbmd_nve_run, one structure at a time, rebuilding on
the skin: a run that never outruns the skin rebuilds only on the fixed
schedule, so every request gets the same bits on both paths.

All arithmetic runs in libmbmd; this module only schedules.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import THERMO_COLS, Context, MbmdError, MBMD_EBUSY, MBMD_ESKIN, MBMD_OK

# rows of the stacked per-request result: U, F (3), W (9), J (3), pos (3), vel (3)
RESULT_ROWS = 22
# batch steps the host may enqueue ahead of the GPU
MAX_STEPS_AHEAD = 3


@dataclass
class Job:
    """One request as the loop sees it."""
    rid: int
    arrival_s: float
    pos: np.ndarray           # (n, 3)
    vel: np.ndarray           # (n, 3)
    box: np.ndarray           # (3,)
    n_steps: int              # 0: single point
    mass: float = 28.0855
    dt: float = 1.0

    @property
    def n(self) -> int:
        return self.pos.shape[0]


@dataclass
class ServeStats:
    latencies_s: dict = field(default_factory=dict)   # rid -> latency
    makespan_s: float = 0.0
    atom_steps: int = 0
    loop_steps: int = 0
    max_in_flight: int = 0
    capacity_atoms: int = 0
    skin_reruns: int = 0
    failed: dict = field(default_factory=dict)        # rid -> mbmd_status code

    def summary(self) -> dict:
        lat = np.array(sorted(self.latencies_s.values()))
        ok = lat.size > 0
        return {
            "requests": int(lat.size),
            "p50_ms": float(1e3 * np.percentile(lat, 50)) if ok else None,
            "p99_ms": float(1e3 * np.percentile(lat, 99)) if ok else None,
            "mean_ms": float(1e3 * lat.mean()) if ok else None,
            "makespan_s": self.makespan_s,
            "atom_steps_per_s": self.atom_steps / self.makespan_s if self.makespan_s > 0 else None,
            "loop_steps": self.loop_steps,
            "max_in_flight": self.max_in_flight,
            "capacity_atoms": self.capacity_atoms or None,
            "skin_reruns": self.skin_reruns,
            "failed": len(self.failed),
        }


def jobs_from_requests(requests, time_scale: float = 1.0):
    """Jobs from workload Requests; arrival times multiplied by time_scale."""
    return [Job(r.rid, r.arrival_s * time_scale, r.system.pos, r.system.vel, r.system.box,
                r.n_steps if r.kind == "nve" else 0) for r in requests]


def _dev(a, device):
    return torch.tensor(np.ascontiguousarray(np.asarray(a, dtype=np.float64).T), device=device)


def _dev_async(a, device):
    """(n, 3) host array -> (3, n) device tensor through pinned memory, without
    waiting for the copy (it is ordered before later work on the stream)."""
    host = torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float64).T))
    return host.pin_memory().to(device, non_blocking=True)


def _result_views(buf):
    return {"U": buf[0], "F": buf[1:4], "W": buf[4:13], "J": buf[13:16], "pos": buf[16:19],
            "vel": buf[19:22]}


def _unstack(host):
    return _result_views(host)


def batch_capacity_atoms(ctx: Context, hbm_budget_bytes: int, max_structures: int) -> int:
    """Largest batch atom capacity whose workspace fits the HBM budget."""
    lo, hi = 1, 1 << 28
    if ctx.batch_workspace_size(lo, max_structures) > hbm_budget_bytes:
        raise ValueError("HBM budget below the workspace of a one-atom batch")
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if ctx.batch_workspace_size(mid, max_structures) <= hbm_budget_bytes:
            lo = mid
        else:
            hi = mid - 1
    return lo


def rerun_alone(ctx: Context, job: Job, precision, rebuild_every):
    """One structure on its own under the rebuild-on-skin policy; returns
    the stacked result rows on the host and its thermo rows (or None)."""
    dev = ctx.device
    ctx.set_rebuild_policy("skin")
    buf = torch.empty(RESULT_ROWS, job.n, dtype=torch.float64, device=dev)
    out = _result_views(buf)
    out["pos"].copy_(_dev(job.pos, dev))
    out["vel"].copy_(_dev(job.vel, dev))
    th = None
    if job.n_steps == 0:
        ctx.compute(out["pos"], job.box, vel=out["vel"], precision=precision, out=out)
    else:
        th = torch.empty(job.n_steps + 1, THERMO_COLS, dtype=torch.float64, device=dev)
        ctx.nve_run(out["pos"], out["vel"], job.box, job.mass, job.dt, job.n_steps,
                    rebuild_every, precision=precision, thermo=th, out=out)
    return buf.cpu(), (th.cpu() if th is not None else None)


def serve_batched(ctx: Context, jobs, precision="fp64", hbm_budget_bytes=None,
                  max_structures=256, rebuild_every=10, keep_results=False, saturate=False,
                  rerun_ctx: Context | None = None, clock=time.perf_counter):
    """Continuous batching over the arrival trace `jobs`.

    hbm_budget_bytes: device memory the batch may use (default: half of the
    free memory, but no more than max_structures of the largest request need).
    saturate: every request is taken as arrived at time 0 (capacity runs).
    rerun_ctx: a context with the same potential and skin, on which a
    structure reported with MBMD_ESKIN is served again alone (rebuilding on
    the skin); without one such a structure fails.
    """
    dev = ctx.device
    largest_job = max(j.n for j in jobs)
    if hbm_budget_bytes is None:
        free, _total = torch.cuda.mem_get_info(dev)
        need = ctx.batch_workspace_size(max_structures * largest_job, max_structures)
        hbm_budget_bytes = min(int(0.5 * free), need)
    cap = batch_capacity_atoms(ctx, hbm_budget_bytes, max_structures)
    if cap < largest_job:
        raise ValueError(f"HBM budget admits {cap} atoms, less than the largest request "
                         f"({largest_job})")
    ctx.batch_open(cap, max_structures, rebuild_every)
    stats = ServeStats(capacity_atoms=cap)
    results = {}
    order = sorted(jobs, key=lambda j: (0.0 if saturate else j.arrival_s, j.rid))
    pending = collections.deque(order)
    waiting = collections.deque()
    in_flight = {}
    copies = collections.deque()     # (event, [(job, host, thermo host)]) not yet seen complete
    steps_ahead = collections.deque()
    stream = ctx.stream
    free_atoms, free_slots, largest = ctx.batch_capacity()
    t0 = clock()

    def collect(block):
        """Record every retirement whose copies have completed (the oldest
        first; with block, wait for all of them)."""
        while copies and (block or copies[0][0].query()):
            ev, done = copies.popleft()
            ev.synchronize()
            now = clock() - t0
            for job, host, th_host, st_host in done:
                code = int(st_host[0])
                if code == MBMD_ESKIN and rerun_ctx is not None:
                    host, th_alone = rerun_alone(rerun_ctx, job, precision, rebuild_every)
                    th_host = th_alone if th_host is not None else None
                    stats.skin_reruns += 1
                    now = clock() - t0
                elif code != MBMD_OK:
                    stats.failed[job.rid] = code
                    continue
                stats.latencies_s[job.rid] = now - (0.0 if saturate else job.arrival_s)
                stats.atom_steps += job.n * max(1, job.n_steps)
                if keep_results:
                    r = _unstack(host)
                    if th_host is not None:
                        r["thermo"] = th_host
                    results[job.rid] = r

    try:
        while pending or waiting or in_flight or copies:
            collect(False)
            now = clock() - t0
            while pending and (saturate or pending[0].arrival_s <= now):
                waiting.append(pending.popleft())
            admitted = False
            while waiting and free_slots > 0 and largest >= waiting[0].n:
                job = waiting[0]
                th = torch.empty(job.n_steps + 1, THERMO_COLS, dtype=torch.float64, device=dev)
                try:
                    h = ctx.batch_add(_dev_async(job.pos, dev), _dev_async(job.vel, dev), job.box,
                                      job.mass, job.dt, job.n_steps, thermo=th)
                except MbmdError as e:
                    if e.code != MBMD_EBUSY:
                        raise
                    break
                in_flight[h] = job
                waiting.popleft()
                admitted = True
                free_atoms, free_slots, largest = ctx.batch_capacity()
            stats.max_in_flight = max(stats.max_in_flight, len(in_flight))
            if not in_flight:
                if copies:
                    collect(True)
                elif pending and not admitted:
                    delay = pending[0].arrival_s - (clock() - t0)
                    if delay > 2e-3:
                        time.sleep(delay - 1e-3)
                continue
            ctx.batch_step(precision)
            stats.loop_steps += 1
            ev = torch.cuda.Event()
            ev.record(stream)
            steps_ahead.append(ev)
            if len(steps_ahead) > MAX_STEPS_AHEAD:
                steps_ahead.popleft().synchronize()
            fin = ctx.batch_finished()
            if not fin:
                continue
            # retire every finished structure: asynchronous copies into pinned
            # host buffers, marked by one event that later iterations poll
            done = []
            st = torch.empty(len(fin), dtype=torch.int32, device=dev)
            for k, h in enumerate(fin):
                job = in_flight.pop(h)
                buf = torch.empty(RESULT_ROWS, job.n, dtype=torch.float64, device=dev)
                th = ctx.batch_retire(h, job.n, _result_views(buf), status=st[k:k + 1]).get("thermo")
                host = torch.empty(RESULT_ROWS, job.n, dtype=torch.float64, pin_memory=True)
                host.copy_(buf, non_blocking=True)
                th_host = None
                if keep_results and th is not None:
                    th_host = torch.empty(th.shape, dtype=torch.float64, pin_memory=True)
                    th_host.copy_(th, non_blocking=True)
                done.append((job, host, th_host, k))
            st_host = torch.empty(len(fin), dtype=torch.int32, pin_memory=True)
            st_host.copy_(st, non_blocking=True)
            done = [(job, host, th_host, st_host[k:k + 1]) for job, host, th_host, k in done]
            ev = torch.cuda.Event()
            ev.record(stream)
            copies.append((ev, done))
            free_atoms, free_slots, largest = ctx.batch_capacity()
        collect(True)
        stats.makespan_s = clock() - t0
        ctx.batch_sync()
        if stats.failed:
            rid, code = next(iter(stats.failed.items()))
            raise MbmdError(code, f"{len(stats.failed)} request(s) failed in the batch "
                                  f"(request {rid} first)")
    finally:
        ctx.batch_close()
    return results, stats


def serve_sequential(ctx: Context, jobs, precision="fp64", rebuild_every=10, keep_results=False,
                     saturate=False, clock=time.perf_counter):
    """The same trace, one structure per launch sequence, in arrival order
    (lists rebuilt every rebuild_every steps and whenever an atom has moved
    skin/2 since the last build)."""
    dev = ctx.device
    stats = ServeStats()
    results = {}
    ctx.set_rebuild_policy("skin")
    order = sorted(jobs, key=lambda j: (0.0 if saturate else j.arrival_s, j.rid))
    t0 = clock()
    for job in order:
        arrival = 0.0 if saturate else job.arrival_s
        delay = arrival - (clock() - t0)
        if delay > 2e-3:
            time.sleep(delay - 1e-3)
        while clock() - t0 < arrival:
            pass
        buf = torch.empty(RESULT_ROWS, job.n, dtype=torch.float64, device=dev)
        out = _result_views(buf)
        out["pos"].copy_(_dev(job.pos, dev))
        out["vel"].copy_(_dev(job.vel, dev))
        th = None
        if job.n_steps == 0:
            ctx.compute(out["pos"], job.box, vel=out["vel"], precision=precision, out=out)
        else:
            th = torch.empty(job.n_steps + 1, THERMO_COLS, dtype=torch.float64, device=dev)
            ctx.nve_run(out["pos"], out["vel"], job.box, job.mass, job.dt, job.n_steps,
                        rebuild_every, precision=precision, thermo=th, out=out)
        host = buf.cpu()
        stats.latencies_s[job.rid] = clock() - t0 - arrival
        stats.atom_steps += job.n * max(1, job.n_steps)
        stats.loop_steps += max(1, job.n_steps)
        if keep_results:
            r = _unstack(host)
            if th is not None:
                r["thermo"] = th.cpu()
            results[job.rid] = r
    stats.makespan_s = clock() - t0
    return results, stats
