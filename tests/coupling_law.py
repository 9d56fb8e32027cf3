"""Berendsen's weak-coupling relations for atoms that never interact, and
such a system: test infrastructure shared by the oracle's pins and the GPU
tests of the coupled integrator.

With every force zero the velocity-Verlet kicks add nothing, so the kinetic
temperature and the volume of a coupled run follow
    T_{s+1} - T_s = (dt / tau_T) (T0 - T_s),
    V_{s+1} / V_s - 1 = -(beta dt / tau_P) (P0 - P_s),  P_s = 2 E_kin,s / (3 V_s),
integrated below with no square or cube root.
"""
import numpy as np

import workload as wl


def ideal_gas(seed, temperature=300.0, spacing=4.5, cells=4):
    """A simple-cubic arrangement 4.5 A apart: beyond the Tersoff list radius
    (3.5 A), so every list is empty and every force zero."""
    g = np.stack(np.meshgrid(*[np.arange(cells)] * 3, indexing="ij"), -1).reshape(-1, 3)
    pos = (g + 0.5) * spacing
    box = np.full(3, cells * spacing)
    rng = np.random.default_rng(seed)
    vel = wl.maxwell_boltzmann(pos.shape[0], temperature, rng)
    return pos, vel, box


def berendsen_law(T_init, ekin_init, V_init, steps, dt, T0, tau_T, P0, tau_P, beta):
    """(T_s, V_s) of the weak-coupling relations for non-interacting atoms
    (P0 in eV/A^3, beta in A^3/eV)."""
    T, E, V = [T_init], [ekin_init], [V_init]
    for _ in range(steps):
        t, e, v = T[-1], E[-1], V[-1]
        t_next = t + dt / tau_T * (T0 - t) if tau_T > 0 else t
        v_next = v * (1.0 - beta * dt / tau_P * (P0 - 2.0 * e / (3.0 * v))) if tau_P > 0 else v
        E.append(e * t_next / t)
        T.append(t_next)
        V.append(v_next)
    return np.array(T), np.array(V)
