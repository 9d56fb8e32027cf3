#!/usr/bin/env python3
"""Benchmark of the many-body force path on one MI355X.

Headline workload: Tersoff (1989) silicon, diamond 40x40x40 conventional
cells = 512,000 atoms, a = 5.43 A, periodic, seeded Gaussian displacements
sigma = 0.05 A, 300 K velocities (seed 1002); NVE velocity-Verlet at
dt = 1 fs; cell-list neighbour rebuild every 20 steps with a 0.5 A skin;
per-atom energy, force, 9-component virial and heat current computed and
stored every step; a thermo row per step.  FP64.

One "step" is one MD step of the whole path (list build when due, site-local
partials, pairwise forces with the fused integrator, thermo reduction).
Inputs are resident in HBM before the timed region.  --warmup steps run
first (an mbmd_nve_run from the input); the timed region is the
mbmd_nve_continue of that run by --steps steps, bracketed by device
synchronisation: each timed step has its one force evaluation, and the list
builds are those the 20-step schedule puts among the timed steps (with
--warmup 0 the timed run starts from the input instead, and its initial
list build and step-0 force evaluation fall inside the time).  The default
--warmup of 500 steps (about 40 ms of sustained work) covers the rise of the
GPU's clock under load: in kernel traces the site pass takes ~43 us in the
first milliseconds of a run and ~36 us from about 30 ms on, so a short
warm-up times the rise (the 20-step figure with --warmup 5 is mostly that).

Also measured, as extra fields of the same line:
  mixed    the same input with FP32 bond-order/force arithmetic, --mixed-steps
           steps: throughput, max |dF| and per-atom energy error against the
           FP64 path at step 0 and on the mixed trajectory every
           --mixed-check steps, total-energy drift of both paths
           (eV/atom/ps, linear fit)
  npt      the same input under Berendsen weak coupling (300 K, 0 Pa), both
           precisions
  sic_512k Tersoff's multicomponent form on 512,000-atom zincblende SiC
  green_kubo  heat-current autocorrelation and running conductivity of an
           8,000-atom NVE run, and the correlation kernel at 10^6 samples
  repeats  further timed FP64 runs: median/min/max and whether the outputs
           (x, v, F, W, J, thermo) are the same bits every time
  sw_1m    Stillinger-Weber (1985) Si, 50x50x50 cells = 1,000,000 atoms, FP64
  speed_vs_n  throughput of both potentials and precisions for crystals of
           5^3 to 70^3 cells (1,000 to 2,744,000 atoms), and Tersoff FP64
           with the list rebuilt every 5 steps
  serving  a Poisson request trace through the continuous-batching loop and
           through one structure per launch, p50/p99 latency to results on
           the host, both precisions, and an HBM-capped batch; the batched
           loop serves the trace --serve-runs times and reports its
           median-p99 run
  roofline the dominant kernel against its bound, timed with HIP events: the
           Tersoff site pass against the FP64 vector peak (algorithmic
           FLOPs), the pairwise pass against HBM bandwidth (algorithmic bytes)
  cpu_baseline  the CPU oracle on a bounded sample of the headline workload

Prints ONE JSON line.  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "atom-steps/s, Tersoff Si 512k atoms (FP64 vs mixed); p50/p99 batched latency"
HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
FP32_VECTOR_PEAK_TFLOPS = 157.3
PROFILES = os.path.join(ROOT, "profiles")
# Compulsory HBM bytes per atom-step of a whole MD step (read x, v, F and the
# lists, write and read the bond data, write U, F, W, J and v), NN = 4 for
# the Tersoff crystal and 16 list entries for SW: FP64 Tersoff 517, mixed
# Tersoff (bond data in FP32) 453, FP64 SW (no bond-order pass) 390.
STEP_BYTES_PER_ATOM = {"tersoff_fp64": 517.0, "tersoff_mixed": 453.0, "sw_fp64": 390.0}


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
        # read x (24), mask (8), list (4) + reverse slot (1) of each in-cutoff
        # entry, own partials, U (8), v (24); write F (24), W (72), J (24),
        # v (24), x_next (24)
        return 24 + 8 + 5 * k_cut + part + 8 + 24 + 24 + 72 + 24 + 24 + 24
    if kernel == "neighbor_build":
        return 24 + 4 + 5 * l_list
    return 0.0


# FP64 operations (FMA = 2) of the special functions as hipcc compiles them
# for gfx950 (read from the kernels' assembly), used as their weights; the
# unweighted count takes each special function as one operation
FP64_WEIGHTS = {"exp": 30, "log": 80, "rcp": 9, "rsqrt": 13}
UNWEIGHTED = {"exp": 1, "log": 1, "rcp": 1, "rsqrt": 1}


def tersoff_site_flops(mean_L, mean_K, mean_KK, w=FP64_WEIGHTS):
    """Algorithmic FP64 operations per atom of the Tersoff site pass.

    mean_L: list entries, mean_K: in-cutoff bonds K, mean_KK: mean of K(K-1)
    (ordered angles).  Per list entry: minimum-image displacement and r^2 (20).
    Per bond: length and unit vector (rsqrt + 4), f_R and f_A (exp + 2 each),
    bond order b and db/dzeta (log + exp + 14 for the series and the
    reciprocal + 1), energy and pair-derivative terms (17).  Per unordered
    angle: cosine (5) and g, g' (10 + rcp).  Per ordered angle: the zeta
    term (2) and the partial-derivative accumulation (27).  Bonds in the
    cutoff taper (none in the 300 K crystal) would add a sincos each.
    """
    per_bond = ((w["rsqrt"] + 4) + 2 * (w["exp"] + 2) + (w["log"] + w["exp"] + 14 + w["rcp"] + 2)
                + 17)
    per_pair = 5 + 10 + w["rcp"]
    per_ordered = 2 + 27
    return 20 * mean_L + per_bond * mean_K + per_pair * mean_KK / 2 + per_ordered * mean_KK


def sw_site_flops(mean_L, mean_K, mean_KK, w=FP64_WEIGHTS):
    """Algorithmic FP64 operations per atom of the SW site pass (FMA = 2;
    special functions weighted as for Tersoff).  Per list entry: displacement
    and r^2 (20).  Per bond: length and unit vector (rsqrt + 4), the two-body
    term and its derivative with E = exp(gamma sigma/(r - a sigma)) (two exp,
    a reciprocal and 21), its share of U_i (2), the radial factor of the
    partial (rcp + 4).  Per unordered angle: the three-body energy (11).  Per
    ordered angle: the three-body part of the partial (28)."""
    per_bond = (w["rsqrt"] + 4) + (2 * w["exp"] + w["rcp"] + 21) + 2 + (w["rcp"] + 4)
    return 20 * mean_L + per_bond * mean_K + 11 * mean_KK / 2 + 28 * mean_KK


def profile_value(fname, pattern):
    """A machine-read value from a committed profile summary, or None if the
    file is missing, has no such line, or was taken on other kernel sources."""
    try:
        text = open(os.path.join(PROFILES, fname)).read()
    except OSError:
        return None
    m = re.search(r"^source_sha256:\s*([0-9a-f]{64})", text, re.M)
    if not m or m.group(1) != kernel_source_hash():
        return None
    m = re.search(pattern, text, re.M)
    return m.groups() if m else None


def path_roofline(path, n, ms_per_step, kernels, site_flops_atom, site_peak_tflops,
                  bytes_pair_atom, bytes_site_atom):
    """Roofline figures of one path: the whole step against HBM with its
    compulsory bytes, the site pass against the vector peak of its precision
    (algorithmic FLOP) and its VALU issue share (counters), the pairwise pass
    against HBM (algorithmic bytes) and its counted traffic.  Durations are
    the HIP-event averages of the bench's profiled pass; where a committed
    rocprofv3 summary of the same kernel sources exists, its average and the
    fractions it gives are reported beside them."""
    sb = STEP_BYTES_PER_ATOM[path]
    step_gbs = sb * n / (ms_per_step * 1e-3) / 1e9
    out = {"step": {"bound": "hbm", "bytes_per_atom_step": sb, "achieved": round(step_gbs, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(step_gbs / HBM_PEAK_GBS, 4),
                    "ms_per_step": ms_per_step}}
    stats = f"{path.replace('tersoff', 'tersoff_512k').replace('sw', 'sw_1m')}"
    for kind, unit in (("site_partials", "TFLOP/s"), ("pair_gather", "GB/s")):
        k = kernels.get(kind)
        if not k:
            continue
        us = k["avg_us"]
        rp = profile_value(f"{stats}_kernel_stats.md", rf"^avg_us\s+{kind}:\s*([0-9.]+)")
        us_rp = float(rp[0]) if rp else None
        d = {"avg_us": us, "avg_us_rocprof": us_rp}
        if kind == "site_partials":
            if site_flops_atom:
                f = site_flops_atom * n
                d.update({"bound": "alu", "algorithmic_flops_per_atom": round(site_flops_atom, 1),
                          "achieved": round(f / (us * 1e-6) / 1e12, 3), "peak": site_peak_tflops,
                          "unit": "TFLOP/s"})
                d["frac"] = round(d["achieved"] / site_peak_tflops, 4)
                if us_rp:
                    d["frac_rocprof"] = round(f / (us_rp * 1e-6) / 1e12 / site_peak_tflops, 4)
            d["bytes_per_atom"] = bytes_site_atom
            d["hbm_GBs"] = round(bytes_site_atom * n / (us * 1e-6) / 1e9, 1)
            v = profile_value(f"{stats}_valu_counters.md",
                              r"^valu\s+site_partials:\s*insts_per_launch=([0-9.e+]+)")
            if v:
                d["valu_issue_frac"] = round(float(v[0]) / VALU_ISSUE_PER_S /
                                             ((us_rp or us) * 1e-6), 4)
        else:
            b = bytes_pair_atom * n
            d.update({"bound": "hbm", "algorithmic_bytes_per_atom": round(bytes_pair_atom, 1),
                      "achieved": round(b / (us * 1e-6) / 1e9, 1), "peak": HBM_PEAK_GBS,
                      "unit": "GB/s"})
            d["frac"] = round(d["achieved"] / HBM_PEAK_GBS, 4)
            if us_rp:
                d["frac_rocprof"] = round(b / (us_rp * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
        t = profile_value(f"{stats}_hbm_traffic.md",
                          rf"^traffic\s+{kind}:\s*fetch_bytes=([0-9.e+]+)\s+write_bytes=([0-9.e+]+)")
        if t:
            tb = float(t[0]) + float(t[1])
            d["traffic"] = tb
            d["traffic_over_algorithmic"] = round(
                tb / ((bytes_pair_atom if kind == "pair_gather" else bytes_site_atom) * n), 3)
            d["traffic_GBs"] = round(tb / ((us_rp or us) * 1e-6) / 1e9, 1)
        out[kind] = d
    return out


def kernel_source_hash() -> str:
    """SHA-256 over the sources that define the kernels and their launch
    shapes (every csrc file but the host-side C ABI, capi.hip, which only
    sequences launches)."""
    h = hashlib.sha256()
    files = sorted(f for f in glob.glob(os.path.join(ROOT, "paper_1610_03343_amd", "csrc", "*"))
                   if os.path.basename(f) != "capi.hip")
    for f in files:
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()


# wave64 VALU instruction issue: 4 cycles per instruction on each of
# 256 CUs x 4 SIMDs at 2.4 GHz
VALU_ISSUE_PER_S = 256 * 4 * 2.4e9 / 4


def list_statistics(ctx, pos_dev, sysm, cutoff):
    """Mean list length, mean in-cutoff count K and mean K(K-1) of the
    GPU-built list at the input positions."""
    import numpy as np
    nn, nl = ctx.neighbors(pos_dev, sysm.box)
    nn_h = nn.cpu().numpy()
    nl_h = nl.cpu().numpy()
    n = sysm.n
    idx = np.arange(n)
    k = np.zeros(n, dtype=np.int64)
    for m in range(int(nn_h.max())):
        have = nn_h > m
        j = nl_h[m, have]
        d = sysm.pos[j] - sysm.pos[idx[have]]
        d -= sysm.box * np.rint(d / sysm.box)
        k[have] += np.sum(d * d, axis=1) < cutoff ** 2
    return float(nn_h.mean()), float(k.mean()), float((k * (k - 1)).mean())


def drift_per_ps(thermo, n, dt_fs):
    """Slope of the total energy per atom against time, eV/atom/ps."""
    import numpy as np
    t = np.arange(thermo.shape[0]) * dt_fs * 1e-3
    e = thermo[:, 14] / n
    return float(np.polyfit(t, e, 1)[0])


class Workload:
    """A resident input and the nve timing around it."""

    def __init__(self, mb, wl, torch, sysm, pot, every, skin, max_nb):
        self.mb, self.wl, self.torch = mb, wl, torch
        self.s = sysm
        self.n = sysm.n
        self.dev = torch.device("cuda", 0)
        self.pos0 = torch.tensor(wl.soa(sysm.pos), device=self.dev)
        self.vel0 = torch.tensor(wl.soa(sysm.vel), device=self.dev)
        self.every = every
        self.ctx = mb.Context(0)
        if pot == "tersoff":
            self.ctx.set_tersoff(wl.TERSOFF_SI_1989)
        else:
            self.ctx.set_sw(wl.SW_SI_1985)
        self.ctx.set_neighbor(skin, max_nb)
        self.ctx.set_rebuild_policy("fixed")
        z = lambda *sh: torch.empty(*sh, dtype=torch.float64, device=self.dev)
        self.out = dict(U=z(self.n), F=z(3, self.n), W=z(9, self.n), J=z(3, self.n))

    def run(self, precision, steps, pos=None, vel=None, thermo=None, cont=False):
        torch, mb = self.torch, self.mb
        if pos is None:
            pos, vel = self.pos0.clone(), self.vel0.clone()
        if thermo is None:
            thermo = torch.empty(steps + 1, mb.THERMO_COLS, dtype=torch.float64, device=self.dev)
        self.ctx.nve_run(pos, vel, self.s.box, self.wl.M_SI, 1.0, steps, self.every,
                         precision=precision, thermo=thermo, out=self.out, cont=cont)
        return pos, vel, thermo

    def timed(self, precision, steps, warmup):
        """Times `steps` MD steps that continue a `warmup`-step run from the
        input (mbmd_nve_continue): steps warmup + 1 ... warmup + steps of one
        trajectory, each with its force evaluation, per-atom outputs and
        thermo row, and the list builds the 20-step schedule puts among them.
        With warmup 0 the timed run starts from the input, so its step-0
        force evaluation and list build fall inside the time."""
        torch = self.torch
        pos, vel = self.pos0.clone(), self.vel0.clone()
        if warmup > 0:
            self.run(precision, warmup, pos, vel)
        thermo = torch.empty(steps + 1, self.mb.THERMO_COLS, dtype=torch.float64, device=self.dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        self.run(precision, steps, pos, vel, thermo, cont=warmup > 0)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return dt, self.ctx.run_stats(), thermo.cpu().numpy(), pos, vel

    def close(self):
        self.ctx.close()


def bench_mixed(W, args):
    """Mixed path on the headline input: throughput, errors, drift.  Errors
    are taken against the FP64 path, which the parity tests hold to the
    oracle within 1e-12 on this same input (the oracle itself runs here only
    in the CPU-baseline leg)."""
    torch, wl = W.torch, W.wl
    n = W.n
    steps = args.mixed_steps
    log(f"mixed: timed {steps} steps (+{args.warmup} warmup)")
    tmx, stmx, th_mx, pos_mx, vel_mx = W.timed("mixed", steps, args.warmup)
    log(f"mixed: {tmx:.3f} s, {n * steps / tmx:.4e} atom-steps/s")
    log(f"fp64 reference run: {steps} steps")
    t64, _, th_64, _, _ = W.timed("fp64", steps, args.warmup)

    # error checks on a second context, so that the trajectory's context
    # keeps its run continuable
    chk = W.mb.Context(0)
    chk.set_tersoff(wl.TERSOFF_SI_1989)
    chk.set_neighbor(0.5, 16)

    def errors(step, pos, vel):
        o64 = chk.compute(pos, W.s.box, vel=vel, precision="fp64")
        omx = chk.compute(pos, W.s.box, vel=vel, precision="mixed")
        return {"step": step, "against": "fp64 path",
                "max_abs_dF_eV_per_A": float((omx["F"] - o64["F"]).abs().max()),
                "max_abs_dU_i_eV": float((omx["U"] - o64["U"]).abs().max())}

    # step 0: both paths on the input positions; then the mixed trajectory of
    # the timed run again, its warm-up continued in chunks (the chunks
    # reproduce the one continuation bit for bit), FP64 and mixed evaluated
    # on its positions after each
    checks = [errors(0, W.pos0, W.vel0)]
    pos, vel = W.pos0.clone(), W.vel0.clone()
    done = 0
    if args.warmup > 0:
        W.run("mixed", args.warmup, pos, vel)
    chunk = args.mixed_check
    while done < steps:
        k = min(chunk, steps - done)
        W.run("mixed", k, pos, vel, cont=args.warmup > 0 or done > 0)
        done += k
        checks.append(errors(args.warmup + done, pos, vel))
    chk.close()
    same = bool(torch.equal(pos, pos_mx) and torch.equal(vel, vel_mx))
    # per-kernel durations of the mixed path (HIP events, separate pass)
    W.ctx.set_profiling(True)
    W.ctx.reset_profile()
    W.run("mixed", min(args.profile_steps, steps))
    prof = W.ctx.profile()
    W.ctx.set_profiling(False)
    kernels = {k: {"launches": c, "avg_us": round(1e3 * ms / c, 3)}
               for k, (c, ms) in prof.items() if c}
    # FP32 arithmetic: the algorithmic count with each special function as one
    # operation, against the FP32 vector peak
    roof = path_roofline("tersoff_mixed", n, 1e3 * tmx / steps, kernels,
                         tersoff_site_flops(W.l_list, W.k_cut, W.k_kk, UNWEIGHTED),
                         FP32_VECTOR_PEAK_TFLOPS,
                         algorithmic_bytes("pair_gather", W.k_cut, W.l_list, 4),
                         algorithmic_bytes("site_partials", W.k_cut, W.l_list, 4))
    return {
        "roofline": roof,
        "value": n * steps / tmx, "unit": "atom-steps/s", "steps": steps,
        "ms_per_step": 1e3 * tmx / steps, "rebuilds": stmx["rebuilds"],
        "fp64_same_steps_s": t64,
        "max_abs_dF_eV_per_A": max(c["max_abs_dF_eV_per_A"] for c in checks),
        "max_abs_dU_i_eV": max(c["max_abs_dU_i_eV"] for c in checks),
        "checkpoints": checks,
        "energy_drift_eV_per_atom_per_ps": {"mixed": drift_per_ps(th_mx, n, 1.0),
                                            "fp64": drift_per_ps(th_64, n, 1.0)},
        "energy_change_eV_per_atom": {"mixed": float((th_mx[-1, 14] - th_mx[0, 14]) / n),
                                      "fp64": float((th_64[-1, 14] - th_64[0, 14]) / n)},
        "chunked_run_bitwise_equal": same,
        "kernels": kernels,
    }


# Berendsen constants of the NPT timing (the paper gives none): 300 K and
# 0 Pa as in its timings, tau_T = 100 fs, tau_P = 1 ps, silicon's isothermal
# compressibility 1 / (98 GPa)
NPT_COUPLING = dict(T0=300.0, tau_T=100.0, P0_GPa=0.0, tau_P=1000.0, beta_per_GPa=0.0102)


def bench_npt(W, args, nve_ms_per_step):
    """The paper's own benchmark ensemble on the headline input: Berendsen
    NPT at 300 K and 0 Pa, both precisions."""
    torch, mb, wl = W.torch, W.mb, W.wl
    n, steps = W.n, args.npt_steps

    def pressure_gpa(row, box):
        # (2 E_kin + tr W) / (3 V), eV/A^3 -> GPa
        return (2.0 * row[1] + row[2] + row[6] + row[10]) / (3.0 * float(box.prod())) * 160.21766208

    res = {}
    for prec in ("fp64", "mixed"):
        run = lambda k, pos, vel: W.ctx.npt_run(pos, vel, W.s.box, wl.M_SI, 1.0, k, W.every,
                                                precision=prec, out=W.out, **NPT_COUPLING)
        if args.warmup > 0:
            run(args.warmup, W.pos0.clone(), W.vel0.clone())
        pos, vel = W.pos0.clone(), W.vel0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = run(steps, pos, vel)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        st = W.ctx.run_stats()
        th = out["thermo"].cpu().numpy()
        bt = out["box_traj"].cpu().numpy()
        p_gpa = [pressure_gpa(th[k], bt[k]) for k in (0, steps)]
        log(f"NPT {prec}: {t:.3f} s, {n * steps / t:.4e} atom-steps/s")
        res[prec] = {"value": n * steps / t, "unit": "atom-steps/s", "steps": steps,
                     "ms_per_step": 1e3 * t / steps, "rebuilds": st["rebuilds"],
                     "T_K": [round(float(th[0, 15]), 3), round(float(th[-1, 15]), 3)],
                     "P_GPa": [round(p, 5) for p in p_gpa],
                     "box_edge_A": [float(bt[0, 0]), float(bt[-1, 0])]}
    psteps = min(args.profile_steps, steps)
    W.ctx.set_profiling(True)
    W.ctx.reset_profile()
    W.ctx.npt_run(W.pos0.clone(), W.vel0.clone(), W.s.box, wl.M_SI, 1.0, psteps, W.every,
                  out=W.out, **NPT_COUPLING)
    prof = W.ctx.profile()
    W.ctx.set_profiling(False)
    res["kernels"] = {k: {"launches": c, "avg_us": round(1e3 * ms / c, 3)}
                      for k, (c, ms) in prof.items() if c}
    res["fp64_vs_nve_time"] = round(res["fp64"]["ms_per_step"] / nve_ms_per_step, 4)
    res["coupling"] = NPT_COUPLING
    res["config"] = {"workload": "tersoff_si_diamond_40x40x40_512000_atoms_npt_berendsen",
                     "atoms": n, "rebuild_every": W.every, "dt_fs": 1.0}
    return res


def bench_green_kubo(mb, wl, torch, args):
    """Green-Kubo from the per-step heat current: an NVE run of an 8000-atom
    crystal, its running conductivity, and the correlation kernel timed on
    a 1,000,000-sample synthetic series with 10,000 lags."""
    import numpy as np
    log("green-kubo: generating the 8,000-atom Tersoff Si input (seed 1004)")
    s = wl.silicon_crystal(10, seed=1004)
    W = Workload(mb, wl, torch, s, "tersoff", 20, 0.5, 16)
    steps, every, lags = args.gk_steps, 5, 2000
    t, st, _, _, _ = W.timed("fp64", steps, 1000)
    thermo = torch.empty(steps + 1, mb.THERMO_COLS, dtype=torch.float64, device=W.dev)
    W.run("fp64", steps, thermo=thermo)
    th_host = thermo.cpu().numpy()
    T = float(th_host[:, 15].mean())
    V = float(np.prod(s.box))
    gk_t = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = W.ctx.green_kubo(thermo, every, lags, 1.0, V, T)
        gk_t.append(time.perf_counter() - t0)
    kap = out["kappa"].cpu().numpy()
    tail = kap[int(0.8 * lags):]
    log(f"green-kubo: NVE {steps} steps in {t:.2f} s; kappa(last 20% of 10 ps) "
        f"{tail.mean(axis=0)} W/(m K)")
    W.close()
    # the correlation kernel at a larger size
    S, K = 1_000_000, 10_000
    g = torch.Generator(device=W.dev).manual_seed(1005)
    big = torch.randn(S, mb.THERMO_COLS, dtype=torch.float64, device=W.dev, generator=g)
    ctx = mb.Context(0)
    ctx.green_kubo(big, 1, K, 1.0, 1.0, 300.0)
    big_t = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.green_kubo(big, 1, K, 1.0, 1.0, 300.0)
        big_t.append(time.perf_counter() - t0)
    ctx.close()
    del big
    fma = 3 * (K * S - K * (K - 1) // 2)
    tb = min(big_t)
    log(f"green-kubo: {S} samples x {K} lags in {1e3 * tb:.2f} ms, "
        f"{2 * fma / tb / 1e12:.2f} TFLOP/s")
    return {"md": {"workload": "tersoff_si_diamond_10x10x10_8000_atoms_nve", "atoms": s.n,
                   "steps": steps, "dt_fs": 1.0, "seed": 1004, "seconds": t,
                   "atom_steps_per_s": s.n * steps / t, "rebuilds": st["rebuilds"],
                   "mean_T_K": T},
            "analysis": {"sample_every": every, "lags": lags, "window_ps": lags * every * 1e-3,
                         "call_ms": round(1e3 * min(gk_t), 3),
                         "kappa_last20pct_W_per_mK": [float(x) for x in tail.mean(axis=0)],
                         "note": "one short run: a statistical estimate, not a converged value"},
            "correlator": {"samples": S, "lags": K, "call_ms": round(1e3 * tb, 3),
                           "algorithmic_fma": fma,
                           "achieved_TFLOPs": round(2 * fma / tb / 1e12, 3),
                           "peak_fp64_TFLOPs": FP64_VECTOR_PEAK_TFLOPS}}


def bench_sic(mb, wl, torch, args, si_ms_per_step):
    """Tersoff's multicomponent form: zincblende SiC, 40^3 cells = 512,000
    atoms at a = 4.32 A (the potential's own lattice constant), per-type
    masses, NVE, both precisions."""
    import numpy as np
    log("SiC: generating the 512,000-atom zincblende input (seed 1006)")
    s = wl.binary_crystal(40, seed=1006, a=4.32, sigma=0.05, masses=(wl.M_SI, wl.M_C))
    dev = torch.device("cuda", 0)
    ctx = mb.Context(0)
    chi = [[1.0, wl.CHI_SI_C_1989], [wl.CHI_SI_C_1989, 1.0]]
    ctx.set_tersoff_multi([wl.TERSOFF_SI_1989, wl.TERSOFF_C_1989], chi)
    ctx.set_neighbor(0.5, 32)
    ctx.set_rebuild_policy("fixed")
    ctx.set_type_masses([wl.M_SI, wl.M_C])
    pos0 = torch.tensor(wl.soa(s.pos), device=dev)
    vel0 = torch.tensor(wl.soa(s.vel), device=dev)
    types = torch.tensor(s.types, dtype=torch.int32, device=dev)
    z = lambda *sh: torch.empty(*sh, dtype=torch.float64, device=dev)
    out = dict(U=z(s.n), F=z(3, s.n), W=z(9, s.n), J=z(3, s.n))
    steps = args.sic_steps
    res = {}
    for prec in ("fp64", "mixed"):
        # the timed steps continue a warm-up run (as Workload.timed)
        pos, vel = pos0.clone(), vel0.clone()
        if args.warmup > 0:
            ctx.nve_run(pos, vel, s.box, 0.0, 1.0, args.warmup, 20, types=types,
                        precision=prec, out=out)
        th = z(steps + 1, mb.THERMO_COLS)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.nve_run(pos, vel, s.box, 0.0, 1.0, steps, 20, types=types, precision=prec,
                    thermo=th, out=out, cont=args.warmup > 0)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        thh = th.cpu().numpy()
        log(f"SiC {prec}: {t:.3f} s, {s.n * steps / t:.4e} atom-steps/s")
        res[prec] = {"value": s.n * steps / t, "unit": "atom-steps/s", "steps": steps,
                     "ms_per_step": 1e3 * t / steps,
                     "energy_change_eV_per_atom": float((thh[-1, 14] - thh[0, 14]) / s.n),
                     "E_pot_eV_per_atom_step0": float(thh[0, 0] / s.n)}
    ctx.set_profiling(True)
    ctx.reset_profile()
    ctx.nve_run(pos0.clone(), vel0.clone(), s.box, 0.0, 1.0, min(args.profile_steps, steps), 20,
                types=types, out=out)
    prof = ctx.profile()
    ctx.close()
    res["kernels"] = {k: {"launches": c, "avg_us": round(1e3 * ms / c, 3)}
                      for k, (c, ms) in prof.items() if c}
    res["fp64_vs_si_time"] = round(res["fp64"]["ms_per_step"] / si_ms_per_step, 4)
    res["config"] = {"workload": "tersoff_sic_zincblende_40x40x40_512000_atoms_nve",
                     "atoms": s.n, "a_A": 4.32, "chi_SiC": wl.CHI_SI_C_1989, "seed": 1006,
                     "rebuild_every": 20, "skin_A": 0.5, "masses": [wl.M_SI, wl.M_C]}
    return res


def bench_sw(mb, wl, torch, args):
    log("generating the 1,000,000-atom SW Si input (seed 1003)")
    s = wl.sw_1m()
    W = Workload(mb, wl, torch, s, "sw", 20, 0.5, 32)
    steps = args.sw_steps
    log(f"SW 1M: timed {steps} steps (+{args.warmup} warmup)")
    t, st, th, _, _ = W.timed("fp64", steps, args.warmup)
    l_list, k_cut, k_kk = list_statistics(W.ctx, W.pos0, s,
                                          wl.SW_SI_1985["a"] * wl.SW_SI_1985["sigma"])
    psteps = min(args.profile_steps, steps)
    W.ctx.set_profiling(True)
    W.ctx.reset_profile()
    W.run("fp64", psteps)
    prof = W.ctx.profile()
    W.ctx.set_profiling(False)
    kernels = {k: {"launches": c, "avg_us": round(1e3 * ms / c, 3)}
               for k, (c, ms) in prof.items() if c}
    W.close()
    log(f"SW 1M: {t:.3f} s, {s.n * steps / t:.4e} atom-steps/s")
    roof = path_roofline("sw_fp64", s.n, 1e3 * t / steps, kernels,
                         sw_site_flops(l_list, k_cut, k_kk), FP64_VECTOR_PEAK_TFLOPS,
                         algorithmic_bytes("pair_gather", k_cut, l_list, 8),
                         algorithmic_bytes("site_partials", k_cut, l_list, 8))
    roof["site_partials"]["flop_weights"] = FP64_WEIGHTS
    return {"roofline": roof,
            "value": s.n * steps / t, "unit": "atom-steps/s", "dtype": "f64", "steps": steps,
            "ms_per_step": 1e3 * t / steps, "rebuilds": st["rebuilds"],
            "energy_change_eV_per_atom": float((th[-1, 14] - th[0, 14]) / s.n),
            "kernels": kernels,
            "config": {"workload": "sw_si_diamond_50x50x50_1000000_atoms_nve", "atoms": s.n,
                       "rebuild_every": 20, "skin_A": 0.5, "seed": 1003,
                       "mean_list_length": round(l_list, 4), "mean_in_cutoff": round(k_cut, 4),
                       "mean_ordered_angles": round(k_kk, 4)}}


def bench_serving(mb, wl, torch, args):
    from paper_1610_03343_amd import serving
    log(f"serving: generating {args.serve_requests} requests (seed 2001)")
    reqs = wl.serving_trace(args.serve_requests, rate_hz=1.0, seed=2001)
    base = serving.jobs_from_requests(reqs)
    atoms = [j.n for j in base]
    every = 5

    def ctx():
        c = mb.Context(0)
        c.set_tersoff(wl.TERSOFF_SI_1989)
        c.set_neighbor(0.5, 16)
        return c

    c = ctx()
    rc = ctx()     # structures reported with MBMD_ESKIN are served again here, alone
    # warm-up and capacity: the first requests all present at time 0
    sub = base[: args.serve_calib]
    serving.serve_batched(c, sub[:32], saturate=True, rebuild_every=every, rerun_ctx=rc)
    _, st = serving.serve_batched(c, sub, saturate=True, rebuild_every=every, rerun_ctx=rc)
    cap_rps = len(sub) / st.makespan_s
    rate = args.serve_load * cap_rps
    log(f"serving: batched capacity {cap_rps:.1f} requests/s; arrival rate {rate:.1f}/s")
    jobs = serving.jobs_from_requests(reqs, time_scale=1.0 / rate)
    res = {"requests": len(jobs), "arrival_rate_per_s": rate,
           "batched_capacity_requests_per_s": cap_rps, "load_fraction": args.serve_load,
           "atoms_per_request": {"min": min(atoms), "median": float(sorted(atoms)[len(atoms) // 2]),
                                 "max": max(atoms)},
           "nve_fraction": sum(1 for j in jobs if j.n_steps) / len(jobs),
           "rebuild_every": every, "latency": "arrival to results (U, F, W, J, x, v) on the host"}
    for prec in ("fp64", "mixed"):
        # The tail of one trace moves from run to run (the host loop's timing
        # and the GPU clock): the batched loop serves the same trace
        # --serve-runs times, and the run with the median p99 is reported,
        # every run's p50/p99 beside it.
        runs = []
        for k in range(max(1, args.serve_runs)):
            log(f"serving: batched {prec}, run {k + 1}")
            _, sb = serving.serve_batched(c, jobs, precision=prec, rebuild_every=every,
                                          rerun_ctx=rc)
            runs.append(sb.summary())
        order = sorted(range(len(runs)), key=lambda k: runs[k]["p99_ms"])
        sb_sum = runs[order[len(runs) // 2]]
        log(f"serving: one structure per launch {prec}")
        _, ss = serving.serve_sequential(c, jobs, precision=prec, rebuild_every=every)
        res[prec] = {"batched": sb_sum, "one_per_launch": ss.summary(),
                     "batched_runs_p50_p99_ms": [[round(r["p50_ms"], 3), round(r["p99_ms"], 3)]
                                                 for r in runs]}
        log(f"serving {prec}: batched p50/p99 {sb_sum['p50_ms']:.2f}/"
            f"{sb_sum['p99_ms']:.2f} ms (median-p99 run of {len(runs)}); one per launch "
            f"{ss.summary()['p50_ms']:.2f}/{ss.summary()['p99_ms']:.2f} ms")
    log(f"serving: batched fp64 with a {args.serve_cap_mib} MiB HBM budget")
    _, sc = serving.serve_batched(c, jobs, precision="fp64", rebuild_every=every,
                                  hbm_budget_bytes=args.serve_cap_mib << 20, rerun_ctx=rc)
    res["fp64_hbm_capped"] = dict(sc.summary(), hbm_budget_mib=args.serve_cap_mib)
    c.close()
    rc.close()
    return res


def bench_sweep(mb, wl, torch, args):
    """Throughput against system size: diamond crystals of n^3 cells
    (N = 8 n^3), 300 K, sigma 0.05 A, both potentials and precisions.

    speed_vs_n: NVE, list rebuilt every 20 steps, plus the Tersoff FP64 case
    rebuilt every 5 (the paper's rebuild-every-5 comparison).
    speed_vs_n_npt: the protocol of the paper's size sweep (Section 3):
    Berendsen NPT at 300 K and 0 Pa, the list built once before the run and
    never rebuilt, --sweep-npt-steps steps (1,000 in the paper); the time
    includes that one build and the step-0 force evaluation."""
    rows, npt_rows = [], []
    sizes = [int(x) for x in args.sweep_cells.split(",") if x]
    for n in sizes:
        sysm = wl.silicon_crystal(n, seed=1100 + n, sigma=0.05)
        for pot, prec, every in (("tersoff", "fp64", 20), ("tersoff", "mixed", 20),
                                 ("sw", "fp64", 20), ("sw", "mixed", 20), ("tersoff", "fp64", 5)):
            W = Workload(mb, wl, torch, sysm, pot, every, 0.5, 16 if pot == "tersoff" else 32)
            t, _, _, _, _ = W.timed(prec, args.sweep_steps, args.sweep_steps // 10)
            W.close()
            rows.append({"cells": n, "atoms": sysm.n, "potential": pot, "precision": prec,
                         "rebuild_every": every,
                         "atom_steps_per_s": sysm.n * args.sweep_steps / t,
                         "us_per_step": 1e6 * t / args.sweep_steps})
        steps = args.sweep_npt_steps
        if steps > 0:
            for pot, prec in (("tersoff", "fp64"), ("tersoff", "mixed"), ("sw", "fp64"),
                              ("sw", "mixed")):
                W = Workload(mb, wl, torch, sysm, pot, steps + 1, 0.5,
                             16 if pot == "tersoff" else 32)
                run = lambda k, pos, vel: W.ctx.npt_run(pos, vel, sysm.box, wl.M_SI, 1.0, k,
                                                        k + 1, precision=prec, out=W.out,
                                                        **NPT_COUPLING)
                run(20, W.pos0.clone(), W.vel0.clone())          # warm-up
                pos, vel = W.pos0.clone(), W.vel0.clone()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                out = run(steps, pos, vel)
                torch.cuda.synchronize()
                t = time.perf_counter() - t0
                st = W.ctx.run_stats()
                th = out["thermo"][-1].cpu().numpy()
                W.close()
                npt_rows.append({"cells": n, "atoms": sysm.n, "potential": pot,
                                 "precision": prec, "rebuilds": st["rebuilds"],
                                 "atom_steps_per_s": sysm.n * steps / t,
                                 "us_per_step": 1e6 * t / steps,
                                 "T_end_K": round(float(th[15]), 2),
                                 "box_end_A": round(float(out["box"][0]), 5)})
        log(f"sweep: {n}^3 cells ({sysm.n} atoms) done")
    res = {"nve": {"steps": args.sweep_steps, "rows": rows}}
    if npt_rows:
        res["npt_list_built_once"] = {
            "steps": args.sweep_npt_steps, "ensemble": "Berendsen NPT", "coupling": NPT_COUPLING,
            "rebuilds_per_run": 1, "rows": npt_rows}
    return res


def host_cpu():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


def run_cpu_baseline(sysm, steps, steps_all):
    """The oracle on the headline input: single-threaded for `steps` NVE
    steps, and with OpenMP over atoms on every host CPU this process may use
    for `steps_all` steps (per-thread force buffers summed in thread order).
    The all-cores figure is the reported baseline; the single-thread one is
    kept beside it."""
    import oracle
    import workload as wl

    def run(threads, k):
        used = oracle.set_threads(threads)
        log(f"cpu baseline: oracle NVE, {sysm.n} atoms, {k} steps, {used} thread(s)")
        t0 = time.perf_counter()
        oracle.nve("tersoff", wl.TERSOFF_SI_1989, sysm.pos, sysm.vel, sysm.box, wl.M_SI, k, 1.0,
                   3.5, 20, 16, check_skin=False)
        dt = time.perf_counter() - t0
        oracle.set_threads(1)
        return used, dt

    model, ncpu = host_cpu()
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = ncpu or 1
    one_used, one_dt = run(1, steps)
    all_used, all_dt = run(avail, steps_all)
    single = {"value": sysm.n * steps / one_dt, "unit": "atom-steps/s", "cores": one_used,
              "sample": f"{sysm.n}-atom Tersoff Si, {steps} NVE steps (one list build, "
                        f"{steps + 1} force evaluations), {one_dt:.1f} s"}
    return {"value": sysm.n * steps_all / all_dt, "unit": "atom-steps/s", "cores": all_used,
            "kind": "oracle",
            "sample": f"{sysm.n}-atom Tersoff Si, {steps_all} NVE steps "
                      f"({1 + steps_all // 20} list build(s), {steps_all + 1} force "
                      f"evaluations), OpenMP over atoms on {all_used} threads, {all_dt:.1f} s",
            "single_thread": single, "host_cpu": model, "host_logical_cpus": ncpu,
            "cpus_available": avail}


def main():
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=500,
                    help="untimed steps before each timed run (the clock's rise under load)")
    ap.add_argument("--cpu-steps", type=int, default=10,
                    help="oracle sample length, single thread")
    ap.add_argument("--cpu-steps-all", type=int, default=20,
                    help="oracle sample length on all host cores")
    ap.add_argument("--mixed-steps", type=int, default=10000)
    ap.add_argument("--mixed-check", type=int, default=1000)
    ap.add_argument("--sw-steps", type=int, default=1000)
    ap.add_argument("--npt-steps", type=int, default=1000)
    ap.add_argument("--gk-steps", type=int, default=100000)
    ap.add_argument("--sic-steps", type=int, default=1000)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-calib", type=int, default=400)
    ap.add_argument("--serve-load", type=float, default=0.7)
    ap.add_argument("--serve-cap-mib", type=int, default=64)
    ap.add_argument("--serve-runs", type=int, default=3,
                    help="batched serving runs of the same trace; the median-p99 run is reported")
    ap.add_argument("--repeats", type=int, default=5,
                    help="further timed FP64 runs for median/min/max and an output check")
    ap.add_argument("--sweep-cells", default="5,10,15,20,30,40,50,60,70",
                    help="cells per axis of the size sweep (empty: no sweep)")
    ap.add_argument("--sweep-steps", type=int, default=200)
    ap.add_argument("--sweep-npt-steps", type=int, default=1000,
                    help="steps of each run of the NPT, list-built-once size sweep (0: none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-sw", action="store_true")
    ap.add_argument("--no-npt", action="store_true")
    ap.add_argument("--no-gk", action="store_true")
    ap.add_argument("--no-sic", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=200,
                    help="steps of the HIP-event profiled pass used for the roofline")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1610_03343_amd as mb
    import workload as wl

    log("generating the 512,000-atom Tersoff Si input (seed 1002)")
    s = wl.tersoff_512k()
    n = s.n
    every, skin = 20, 0.5
    W = Workload(mb, wl, torch, s, "tersoff", every, skin, 16)
    l_list, k_cut, k_kk = list_statistics(W.ctx, W.pos0, s, wl.TERSOFF_SI_1989["S"])
    W.l_list, W.k_cut, W.k_kk = l_list, k_cut, k_kk

    log(f"timed FP64 run: {args.warmup} warmup + {args.steps} steps")
    t64, st64, th64, _, _ = W.timed("fp64", args.steps, args.warmup)
    value = n * args.steps / t64
    log(f"FP64: {t64:.3f} s, {value:.4e} atom-steps/s, rebuilds {st64['rebuilds']}")
    # repetitions: spread of the timing, and the same bits every time
    rep_ms, digests = [1e3 * t64 / args.steps], []
    for _ in range(args.repeats):
        tr, _, thr, pr, vr = W.timed("fp64", args.steps, args.warmup)
        rep_ms.append(1e3 * tr / args.steps)
        h = hashlib.sha256()
        for a in (pr, vr, W.out["F"], W.out["W"], W.out["J"]):
            h.update(a.cpu().numpy().tobytes())
        h.update(thr.tobytes())
        digests.append(h.hexdigest())
    repeats = {"ms_per_step": [round(x, 4) for x in rep_ms],
               "median_ms_per_step": round(sorted(rep_ms)[len(rep_ms) // 2], 4),
               "min_ms_per_step": round(min(rep_ms), 4), "max_ms_per_step": round(max(rep_ms), 4),
               "outputs_identical": len(set(digests)) <= 1}
    log(f"repeats: {repeats}")

    # HIP-event profiled pass of the same workload: per-kernel durations
    psteps = min(args.profile_steps, args.steps)
    log(f"profiled FP64 pass: {psteps} steps with HIP events per kernel launch")
    W.ctx.set_profiling(True)
    W.ctx.reset_profile()
    W.run("fp64", psteps)
    prof = W.ctx.profile()
    W.ctx.set_profiling(False)
    kernels = {}
    for name, (launches, ms) in prof.items():
        if launches == 0:
            continue
        avg_us = 1e3 * ms / launches
        b = algorithmic_bytes(name, k_cut, l_list, 8)
        kernels[name] = {"launches": launches, "avg_us": round(avg_us, 3),
                         "algorithmic_bytes_per_atom": round(b, 1),
                         "achieved_GBs": round(b * n / (avg_us * 1e-6) / 1e9, 1) if b else None}
    flops_atom = tersoff_site_flops(l_list, k_cut, k_kk)
    flops_unw = tersoff_site_flops(l_list, k_cut, k_kk, UNWEIGHTED)
    sk = kernels["site_partials"]
    sk["algorithmic_flops_per_atom"] = round(flops_atom, 1)
    sk["achieved_TFLOPs"] = round(flops_atom * n / (sk["avg_us"] * 1e-6) / 1e12, 3)
    ms_step = 1e3 * t64 / args.steps
    paths = {"tersoff_fp64": path_roofline(
        "tersoff_fp64", n, ms_step, kernels, flops_atom, FP64_VECTOR_PEAK_TFLOPS,
        algorithmic_bytes("pair_gather", k_cut, l_list, 8),
        algorithmic_bytes("site_partials", k_cut, l_list, 8))}
    # the dominant kernel of the headline path (longest total time)
    dom = max(("site_partials", "pair_gather"), key=lambda k: prof[k][1])
    pr = paths["tersoff_fp64"][dom]
    roofline = {k: pr[k] for k in ("bound", "achieved", "peak", "unit", "frac")}
    roofline["traffic"] = pr.get("traffic")
    roofline.update({"kernel": dom, "avg_us": pr["avg_us"], "avg_us_rocprof": pr["avg_us_rocprof"],
                     "frac_rocprof": pr.get("frac_rocprof")})
    if dom == "site_partials":
        # bound by FP64 vector arithmetic (transcendentals), not by HBM; the
        # special functions weighted by the FP64 operations of their
        # implementation, and, beside it, each taken as one operation
        roofline.update({
            "algorithmic_flops_per_launch": round(flops_atom * n), "flop_weights": FP64_WEIGHTS,
            "achieved_unweighted": round(flops_unw * n / (pr["avg_us"] * 1e-6) / 1e12, 3),
            "hbm_achieved_GBs": pr["hbm_GBs"]})
        roofline["frac_unweighted"] = round(roofline["achieved_unweighted"] /
                                            FP64_VECTOR_PEAK_TFLOPS, 4)
        if "valu_issue_frac" in pr:
            roofline["valu_issue_frac"] = pr["valu_issue_frac"]
    else:
        roofline["algorithmic_bytes_per_launch"] = round(pr["algorithmic_bytes_per_atom"] * n)
    t = profile_value("tersoff_512k_fp64_hbm_traffic.md",
                      rf"^traffic\s+{dom}:\s*fetch_bytes=([0-9.e+]+)\s+write_bytes=([0-9.e+]+)")
    if t:
        roofline["traffic_parts"] = {"fetch": float(t[0]), "write": float(t[1])}
    log(f"dominant kernel {dom}: {pr['avg_us']} us, {pr['achieved']} {pr['unit']}")

    if args.calib_copy_mib > 0:
        nbytes = args.calib_copy_mib * (1 << 20)
        a = torch.empty(nbytes // 8, dtype=torch.float64, device=W.dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calib_copy_mib} MiB read + {args.calib_copy_mib} MiB "
            f"written, x5")
        del a, b

    mixed = None if args.no_mixed else bench_mixed(W, args)
    npt = None if args.no_npt else bench_npt(W, args, 1e3 * t64 / args.steps)
    W.close()
    sic = None if args.no_sic else bench_sic(mb, wl, torch, args, 1e3 * t64 / args.steps)
    sw = None if args.no_sw else bench_sw(mb, wl, torch, args)
    serve = None if args.no_serving else bench_serving(mb, wl, torch, args)
    gkr = None if args.no_gk else bench_green_kubo(mb, wl, torch, args)
    sweep = bench_sweep(mb, wl, torch, args) if args.sweep_cells else None

    cpu = None
    if not args.no_cpu_baseline:
        cpu = run_cpu_baseline(s, args.cpu_steps, args.cpu_steps_all)
        log(f"cpu baseline: {cpu['value']:.4e} atom-steps/s")

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
                   "atoms": n, "potential": "Tersoff 1989 Si (R=2.7, S=3.0)", "dt_fs": 1.0,
                   "rebuild_every": every, "skin_A": skin, "rebuild_policy": "fixed",
                   "per_step_outputs": "U, F, W(9), J(3) per atom + thermo row",
                   "seed": 1002, "parallelism": "single_gpu",
                   "mean_list_length": round(l_list, 4), "mean_in_cutoff": round(k_cut, 4),
                   "mean_ordered_angles": round(k_kk, 4)},
        "repeats": repeats,
        "fp64_run": {"rebuilds": st64["rebuilds"],
                     "energy_change_eV_per_atom": float((th64[-1, 14] - th64[0, 14]) / n)},
        "mixed": mixed,
        "npt": npt,
        "green_kubo": gkr,
        "sic_512k": sic,
        "sw_1m": sw,
        "serving": serve,
        "speed_vs_n": sweep["nve"] if sweep else None,
        "speed_vs_n_npt": sweep.get("npt_list_built_once") if sweep else None,
        "roofline": roofline,
        "paths": dict(paths, **({"tersoff_mixed": mixed["roofline"]} if mixed else {}),
                      **({"sw_fp64": sw["roofline"]} if sw else {})),
        "kernels": kernels,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
