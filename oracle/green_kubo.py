"""Green-Kubo heat-current autocorrelation and running conductivity (numpy).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the HIP product path never does.

The paper computes the per-atom heat current J_i (Section 2.3) because its
sum J = sum_i J_i feeds Green-Kubo thermal-conductivity calculations (the
applications of Section 3); the Green-Kubo relation itself is the textbook
one, which the paper leaves to its references.  Written out plainly:

  HCACF    C_a(k) = 1/(S - k) sum_{t=0}^{S-k-1} J_a(t) J_a(t + k)
           for samples J(0) .. J(S-1) taken every `sample_every` steps
           (every available time origin, each lag averaged over its own
           number of origins), a = x, y, z;
  running  kappa_a(K) = dtau / (k_B T^2 V) * [C_a(0)/2 + C_a(1) + ...
  kappa      + C_a(K-1) + C_a(K)/2]   (trapezoid rule, kappa_a(0) = 0),
           dtau = sample_every * dt, converted from eV/(fs A K) to W/(m K).
"""
from __future__ import annotations

import numpy as np

K_B_EV = 8.617333262e-5                 # eV/K
EV_PER_FS_A_K_IN_W_PER_M_K = 1.602176634e6


def hcacf(J, max_lag: int):
    """C[k, a] for k = 0 .. max_lag-1 from the sample series J (S, 3), each
    lag a plain dot product over its S - k origins."""
    J = np.asarray(J, dtype=np.float64)
    S = J.shape[0]
    if not 1 <= max_lag <= S:
        raise ValueError("need 1 <= max_lag <= number of samples")
    C = np.zeros((max_lag, J.shape[1]))
    for k in range(max_lag):
        for a in range(J.shape[1]):
            C[k, a] = np.dot(J[:S - k, a], J[k:, a]) / (S - k)
    return C


def hcacf_lags(J, lags):
    """C[k, a] for the listed lags only (the same per-lag dot products as
    hcacf, for sampling long series)."""
    J = np.asarray(J, dtype=np.float64)
    S = J.shape[0]
    out = np.zeros((len(lags), J.shape[1]))
    for r, k in enumerate(lags):
        if not 0 <= k < S:
            raise ValueError("lag out of range")
        for a in range(J.shape[1]):
            out[r, a] = np.dot(J[:S - k, a], J[k:, a]) / (S - k)
    return out


def running_kappa(C, dtau_fs: float, volume_A3: float, T_K: float):
    """Trapezoid running integral of the HCACF scaled to W/(m K); row K is
    the integral up to lag K (row 0 is zero)."""
    C = np.asarray(C, dtype=np.float64)
    if not (dtau_fs > 0 and volume_A3 > 0 and T_K > 0):
        raise ValueError("need dtau, volume and temperature > 0")
    scale = dtau_fs / (K_B_EV * T_K * T_K * volume_A3) * EV_PER_FS_A_K_IN_W_PER_M_K
    kappa = np.zeros_like(C)
    for K in range(1, C.shape[0]):
        kappa[K] = kappa[K - 1] + 0.5 * (C[K - 1] + C[K])
    return scale * kappa


def samples_from_thermo(thermo, sample_every: int):
    """Total heat current (thermo columns 11..13) of rows 0, e, 2e, ..."""
    th = np.asarray(thermo, dtype=np.float64)
    return th[::sample_every, 11:14].copy()
