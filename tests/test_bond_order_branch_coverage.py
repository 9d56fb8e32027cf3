"""The FP64 parity inputs of the Tersoff site pass reach every branch of its
bond order b = (1 + u)^(-1/2n), u = (beta zeta)^n (Tersoff 1989, the bond
order of the potential's subsection): the binomial series for u < 2^-9, the
Taylor polynomial about u0 = 7/64 on [1/32, 3/16], and exp/log elsewhere, on
both sides of the polynomial's interval.  The GPU parity tests compare those
inputs with the oracle to 1e-12, so each branch is checked there; this test
keeps the inputs from drifting away from a branch.  CPU only: zeta is formed
here with numpy from the published parameters."""
import numpy as np

import workload as wl

SERIES_BELOW = 2.0 ** -9
POLY_LO, POLY_HI = 1.0 / 32.0, 3.0 / 16.0


def bond_u(s, p):
    """u of every bond (i, j) with r_ij < S and zeta_ij > 0, by brute force."""
    x, L = s.pos, s.box
    c2, d2, h = p["c"] ** 2, p["d"] ** 2, p["h"]
    R, S = p["R"], p["S"]
    out = []
    for i in range(len(x)):
        dv = x - x[i]
        dv -= L * np.round(dv / L)
        r = np.linalg.norm(dv, axis=1)
        nb = np.where((r > 0) & (r < S))[0]
        if len(nb) < 2:
            continue
        u = dv[nb] / r[nb, None]
        rk = r[nb]
        fc = np.where(rk < R, 1.0, 0.5 + 0.5 * np.cos(np.pi * (rk - R) / (S - R)))
        cos = u @ u.T
        g = 1.0 + c2 / d2 - c2 / (d2 + (h - cos) ** 2)
        np.fill_diagonal(g, 0.0)
        zeta = g @ fc
        zeta = zeta[zeta > 0]
        out.append((p["beta"] * zeta) ** p["n"])
    return np.concatenate(out)


def test_parity_inputs_reach_every_bond_order_branch():
    p = wl.TERSOFF_SI_1989
    inputs = [
        wl.silicon_crystal(2, seed=12, sigma=0.08, a=6.45),
        wl.silicon_crystal(4, seed=14, sigma=0.15, vacancy_fraction=0.05),
        wl.cluster(18, seed=13, min_dist=2.1, box_side=40.0),
    ]
    u = np.concatenate([bond_u(s, p) for s in inputs])
    assert np.sum(u < SERIES_BELOW) > 0
    assert np.sum((u >= SERIES_BELOW) & (u < POLY_LO)) > 0
    assert np.sum((u >= POLY_LO) & (u <= POLY_HI)) > 0
    assert np.sum(u > POLY_HI) > 0
