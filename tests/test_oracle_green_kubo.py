"""Pins of the oracle's Green-Kubo functions (oracle/green_kubo.py) against
an independent algorithm (the Wiener-Khinchin FFT autocorrelation), closed
forms of the lag sums and of the trapezoid integral, and the SI units of
the Green-Kubo relation.  All run on the CPU."""
import math

import numpy as np
import pytest

from oracle import green_kubo as gk


def _fft_lag_sums(x, max_lag):
    """Lag sums sum_t x(t) x(t + k) through the zero-padded FFT (a different
    algorithm from the oracle's per-lag dot products)."""
    S = x.shape[0]
    f = np.fft.rfft(x, n=2 * S, axis=0)
    return np.fft.irfft(f * np.conj(f), n=2 * S, axis=0)[:max_lag]


@pytest.mark.parametrize("S,max_lag", [(1, 1), (7, 7), (1000, 100), (4099, 4099)])
def test_hcacf_equals_wiener_khinchin(S, max_lag):
    """The lag sums (C times its origin count S - k) against the FFT, to
    1e-12 of the largest sum (the FFT's own rounding is ~1e-15 of it); the
    per-lag normalisation is pinned by the cosine closed form below."""
    rng = np.random.default_rng(S)
    J = rng.normal(size=(S, 3)) * np.array([1.0, 3.0, 0.2])
    C = gk.hcacf(J, max_lag)
    raw = C * (S - np.arange(max_lag))[:, None]
    ref = _fft_lag_sums(J, max_lag)
    scale = np.max(np.abs(ref), axis=0)
    assert np.all(np.max(np.abs(raw - ref), axis=0) <= 1e-12 * scale)
    # lag 0 is the mean square
    assert np.allclose(C[0], np.mean(J * J, axis=0), rtol=1e-13, atol=0)


def test_hcacf_cosine_closed_form():
    """x(t) = cos(w t): sum_{t<n} cos(w t) cos(w (t + k)) =
    n/2 cos(w k) + sin(n w) cos(w k + (n - 1) w) / (2 sin w), n = S - k."""
    S, w = 2000, 0.0137
    t = np.arange(S)
    J = np.stack([np.cos(w * t), np.cos(2 * w * t), np.cos(3 * w * t)], axis=1)
    C = gk.hcacf(J, 600)
    for a, ww in enumerate((w, 2 * w, 3 * w)):
        k = np.arange(600)
        n = S - k
        exact = 0.5 * np.cos(ww * k) + np.sin(n * ww) * np.cos(ww * k + (n - 1) * ww) / (
            2 * n * np.sin(ww))
        assert np.max(np.abs(C[:, a] - exact)) <= 1e-12


def test_running_kappa_trapezoid_of_an_exponential():
    """C(k) = C0 r^k integrates by the trapezoid rule to
    (1 - r^(K+1))/(1 - r) - (1 + r^K)/2 in units of C0 dtau."""
    r, C0, K = 0.995, 2.5, 3000
    C = np.repeat((C0 * r ** np.arange(K))[:, None], 3, axis=1)
    dtau, V, T = 2.0, 1000.0, 300.0
    kap = gk.running_kappa(C, dtau, V, T)
    scale = dtau / (gk.K_B_EV * T * T * V) * gk.EV_PER_FS_A_K_IN_W_PER_M_K
    k = np.arange(K)
    exact = C0 * ((1 - r ** (k + 1)) / (1 - r) - 0.5 * (1 + r ** k)) * scale
    assert kap[0, 0] == 0.0
    assert np.max(np.abs(kap[:, 1] - exact)) <= 1e-12 * np.max(np.abs(exact))


def test_running_kappa_si_units():
    """Against the Green-Kubo relation evaluated in SI units: kappa =
    dtau C / (k_B T^2 V) with k_B = 1.380649e-23 J/K and J in J m/s."""
    C = np.full((2, 3), 1.7)                # (eV A / fs)^2, constant
    dtau, V, T = 5.0, 2.0e4, 500.0          # fs, A^3, K
    kap = gk.running_kappa(C, dtau, V, T)
    ev, ang, fs = 1.602176634e-19, 1e-10, 1e-15
    c_si = 1.7 * (ev * ang / fs) ** 2
    kappa_si = (dtau * fs) * c_si / (1.380649e-23 * T * T * V * ang ** 3)
    assert math.isclose(kap[1, 0], kappa_si, rel_tol=1e-9)


def test_samples_from_thermo_and_argument_checks():
    th = np.arange(10 * 16, dtype=float).reshape(10, 16)
    s = gk.samples_from_thermo(th, 3)
    assert np.array_equal(s, th[[0, 3, 6, 9]][:, 11:14])
    with pytest.raises(ValueError):
        gk.hcacf(np.zeros((5, 3)), 6)
    with pytest.raises(ValueError):
        gk.hcacf(np.zeros((5, 3)), 0)
    with pytest.raises(ValueError):
        gk.running_kappa(np.zeros((5, 3)), 1.0, 1.0, 0.0)


def test_hcacf_lags_equals_hcacf():
    rng = np.random.default_rng(5)
    J = rng.normal(size=(3000, 3))
    full = gk.hcacf(J, 3000)
    lags = [0, 1, 17, 1024, 2999]
    assert np.array_equal(gk.hcacf_lags(J, lags), full[lags])
    with pytest.raises(ValueError):
        gk.hcacf_lags(J, [3000])
