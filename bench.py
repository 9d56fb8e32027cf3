#!/usr/bin/env python3
"""Benchmark of the many-body force path on one MI355X.

Workload (the headline configuration): Tersoff (1989) silicon, diamond
40x40x40 conventional cells = 512,000 atoms, a = 5.43 A, periodic, seeded
Gaussian displacements sigma = 0.05 A, 300 K velocities (seed 1002); NVE
velocity-Verlet at dt = 1 fs; cell-list neighbour rebuild every 20 steps
with a 0.5 A skin; per-atom energy, force, 9-component virial and heat
current computed and stored every step; a thermo row per step.

One "step" is one MD step of the whole path (list build when due, site-local
partials, pairwise forces with the fused integrator, thermo reduction).
Inputs are resident in HBM before the timed region; the timed region is one
mbmd_nve_run of --steps steps (plus the force evaluation at its start),
bracketed by device synchronisation.

Prints ONE JSON line.  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "atom-steps/s, Tersoff Si 512k atoms (FP64 vs mixed); p50/p99 batched latency"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(kernel: str, k_cut: float, l_list: float, dsize: int) -> float:
    """Compulsory HBM bytes per atom of one launch (unique data only).

    k_cut: mean in-cutoff neighbours, l_list: mean list length, dsize: bytes
    of one stored partial component (8 FP64, 4 mixed).
    """
    part = 3 * dsize * k_cut            # dU_i/dr_ij per in-cutoff neighbour
    if kernel == "site_partials":
        # read x_i (24), list count (4), list (4 l); write mask (8), U (8), partials
        return 24 + 4 + 4 * l_list + 8 + 8 + part
    if kernel == "pair_gather":
        # read x (24), mask (8), count (4), list + reverse slots (8 l), own partials,
        # U (8), v (24); write F (24), W (72), J (24), v (24), x_next (24)
        return 24 + 8 + 4 + 8 * l_list + part + 8 + 24 + 24 + 72 + 24 + 24 + 24
    if kernel == "neighbor_build":
        return 24 + 4 + 8 * l_list
    return 0.0


def run_cpu_baseline(sysm, steps):
    import oracle
    import workload as wl
    log(f"cpu baseline: oracle NVE, {sysm.n} atoms, {steps} steps, 1 thread")
    t0 = time.perf_counter()
    oracle.nve("tersoff", wl.TERSOFF_SI_1989, sysm.pos, sysm.vel, sysm.box, wl.M_SI, steps, 1.0,
               3.5, 20, 16, check_skin=False)
    dt = time.perf_counter() - t0
    return {"value": sysm.n * steps / dt, "unit": "atom-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{sysm.n}-atom Tersoff Si, {steps} NVE steps (one list build, "
                      f"{steps + 1} force evaluations), single thread, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--cpu-steps", type=int, default=10, help="oracle sample length")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=200,
                    help="steps of the HIP-event profiled pass used for the roofline")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1610_03343_amd as mb
    import workload as wl

    dev = torch.device("cuda", 0)
    log("generating the 512,000-atom Tersoff Si input (seed 1002)")
    s = wl.tersoff_512k()
    n = s.n
    pos0 = torch.tensor(wl.soa(s.pos), device=dev)
    vel0 = torch.tensor(wl.soa(s.vel), device=dev)
    every, skin, dt = 20, 0.5, 1.0

    ctx = mb.Context(0)
    ctx.set_tersoff(wl.TERSOFF_SI_1989)
    ctx.set_neighbor(skin, 16)
    ctx.set_rebuild_policy("fixed")

    # list statistics for the byte accounting (host numpy on the GPU-built list)
    nn, nl = ctx.neighbors(pos0, s.box)
    nn_h = nn.cpu().numpy()
    nl_h = nl.cpu().numpy()
    l_list = float(nn_h.mean())
    idx = np.arange(n)
    kc = 0
    for m in range(int(nn_h.max())):
        have = nn_h > m
        j = nl_h[m, have]
        d = s.pos[j] - s.pos[idx[have]]
        d -= s.box * np.rint(d / s.box)
        kc += int(np.sum(np.sum(d * d, axis=1) < wl.TERSOFF_SI_1989["S"] ** 2))
    k_cut = kc / n

    out = {k: torch.empty(sh, dtype=torch.float64, device=dev)
           for k, sh in (("U", (n,)), ("F", (3, n)), ("W", (9, n)), ("J", (3, n)))}
    thermo = torch.empty(args.steps + 1, mb.THERMO_COLS, dtype=torch.float64, device=dev)

    def timed(precision, steps, warmup):
        pos, vel = pos0.clone(), vel0.clone()
        if warmup > 0:
            th_w = torch.empty(warmup + 1, mb.THERMO_COLS, dtype=torch.float64, device=dev)
            ctx.nve_run(pos, vel, s.box, wl.M_SI, dt, warmup, every, precision=precision,
                        thermo=th_w, out=out)
        pos.copy_(pos0)
        vel.copy_(vel0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.nve_run(pos, vel, s.box, wl.M_SI, dt, steps, every, precision=precision,
                    thermo=thermo[: steps + 1], out=out)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        th = thermo[: steps + 1].cpu().numpy()
        stats = ctx.run_stats()
        drift = float((th[-1, 14] - th[0, 14]) / n)
        return t1 - t0, stats, drift

    log(f"timed FP64 run: {args.warmup} warmup + {args.steps} steps")
    t64, st64, drift64 = timed("fp64", args.steps, args.warmup)
    value = n * args.steps / t64
    log(f"FP64: {t64:.3f} s, {value:.4e} atom-steps/s, rebuilds {st64['rebuilds']}")

    mixed = None
    if not args.no_mixed:
        log(f"timed mixed run: {args.warmup} warmup + {args.steps} steps")
        tmx, stmx, driftmx = timed("mixed", args.steps, args.warmup)
        mixed = {"value": n * args.steps / tmx, "unit": "atom-steps/s",
                 "ms_per_step": 1e3 * tmx / args.steps,
                 "energy_change_eV_per_atom": driftmx, "rebuilds": stmx["rebuilds"]}
        log(f"mixed: {tmx:.3f} s, {mixed['value']:.4e} atom-steps/s")

    # HIP-event profiled pass of the same workload: per-kernel durations
    psteps = min(args.profile_steps, args.steps)
    log(f"profiled FP64 pass: {psteps} steps with HIP events per kernel launch")
    ctx.set_profiling(True)
    ctx.reset_profile()
    pos, vel = pos0.clone(), vel0.clone()
    ctx.nve_run(pos, vel, s.box, wl.M_SI, dt, psteps, every, thermo=thermo[: psteps + 1], out=out)
    prof = ctx.profile()
    ctx.set_profiling(False)
    kernels = {}
    for name, (launches, ms) in prof.items():
        if launches == 0:
            continue
        avg_us = 1e3 * ms / launches
        b = algorithmic_bytes(name, k_cut, l_list, 8)
        kernels[name] = {"launches": launches, "avg_us": round(avg_us, 3),
                         "algorithmic_bytes_per_atom": round(b, 1),
                         "achieved_GBs": round(b * n / (avg_us * 1e-6) / 1e9, 1) if b else None}
    dom = max(("site_partials", "pair_gather"), key=lambda k: prof[k][1])
    dk = kernels[dom]
    achieved = dk["achieved_GBs"]
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": dom, "avg_us": dk["avg_us"],
                "algorithmic_bytes_per_launch": round(dk["algorithmic_bytes_per_atom"] * n)}
    log(f"dominant kernel {dom}: {dk['avg_us']} us, {achieved} GB/s")

    if args.calib_copy_mib > 0:
        nbytes = args.calib_copy_mib * (1 << 20)
        a = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calib_copy_mib} MiB read + {args.calib_copy_mib} MiB written, x5")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = run_cpu_baseline(s, args.cpu_steps)
        log(f"cpu baseline: {cpu['value']:.4e} atom-steps/s")

    ctx.close()
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t64 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "tersoff_si_diamond_40x40x40_512000_atoms_nve",
                   "atoms": n, "potential": "Tersoff 1989 Si (R=2.7, S=3.0)", "dt_fs": dt,
                   "rebuild_every": every, "skin_A": skin, "rebuild_policy": "fixed",
                   "per_step_outputs": "U, F, W(9), J(3) per atom + thermo row",
                   "seed": 1002, "parallelism": "single_gpu",
                   "mean_list_length": round(l_list, 4), "mean_in_cutoff": round(k_cut, 4)},
        "fp64_run": {"rebuilds": st64["rebuilds"], "energy_change_eV_per_atom": drift64},
        "mixed": mixed,
        "roofline": roofline,
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
