"""Helpers shared by the GPU tests: run the HIP path through the C ABI and
the oracle on the same seeded input, and compare."""
from __future__ import annotations

import numpy as np

import workload as wl

RLIST = {"tersoff": 3.0 + 0.5, "sw": 3.77118 + 0.5}
PARAMS = {"tersoff": wl.TERSOFF_SI_1989, "sw": wl.SW_SI_1985}
DEFAULT_M = {"tersoff": 16, "sw": 32}

# FP64 parity bound: max |gpu - oracle| <= TOL_FP64 * max |oracle| per output.
TOL_FP64 = 1e-12
# Mixed path: force error bound in eV/A.
TOL_MIXED_F = 1e-4


def context(pot: str, max_neighbors: int | None = None, skin: float = 0.5):
    import paper_1610_03343_amd as mb
    ctx = mb.Context(0)
    if pot == "tersoff":
        ctx.set_tersoff(PARAMS[pot])
    else:
        ctx.set_sw(PARAMS[pot])
    ctx.set_neighbor(skin, max_neighbors or DEFAULT_M[pot])
    return ctx


def to_dev(a):
    import torch
    return torch.tensor(wl.soa(a), device="cuda:0")


def gpu_compute(ctx, s, precision="fp64", with_vel=True):
    import torch
    pos = to_dev(s.pos)
    vel = to_dev(s.vel) if with_vel else None
    out = ctx.compute(pos, s.box, vel=vel, precision=precision)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy().T.copy() if v.dim() == 2 else v.cpu().numpy().copy()
            for k, v in out.items()}


def oracle_compute(pot, s, maxnb=64, with_vel=True):
    import oracle
    nn, nl = oracle.neighbors(s.pos, s.box, RLIST[pot], maxnb)
    fn = oracle.tersoff if pot == "tersoff" else oracle.sw
    return fn(PARAMS[pot], s.pos, s.box, nn, nl, vel=s.vel if with_vel else None)


def rel(a, b):
    scale = np.max(np.abs(b))
    d = np.max(np.abs(a - b))
    return d / scale if scale > 0 else d


def min_image(d, box):
    return d - box * np.rint(d / box)
