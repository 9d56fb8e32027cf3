"""Green-Kubo analysis on the GPU (mbmd_green_kubo) against the oracle's
plain per-lag dot products and trapezoid integral.

Bar: per component, max |gpu - oracle| <= 1e-12 max |oracle| for the
autocorrelation and for the running conductivity (the two differ only in
summation order).  Cases span one sample, lag counts below, at and past a
64-lag tile, every lag of the series, several 1024-origin tiles with a
ragged tail, sampling intervals above one, and a heat-current series from
an MD run.
"""
import numpy as np
import pytest

import workload as wl
from gpu_util import context, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _oracle(th, every, max_lag, dt, V, T):
    from oracle import green_kubo as gk
    C = gk.hcacf(gk.samples_from_thermo(th, every), max_lag)
    return C, gk.running_kappa(C, every * dt, V, T)


def _compare(got, ref):
    scale = np.max(np.abs(ref), axis=0)
    err = np.max(np.abs(got - ref), axis=0)
    assert np.all(err <= TOL * np.maximum(scale, 1e-300)), (err, scale)


@pytest.mark.parametrize("n_rows,every,max_lag", [
    (1, 1, 1), (5, 1, 5), (3001, 1, 1000), (4096, 1, 4096), (5000, 2, 65),
    (10001, 3, 3334), (70000, 7, 2000)])
def test_green_kubo_matches_oracle(n_rows, every, max_lag):
    import torch
    rng = np.random.default_rng(n_rows + every)
    th = rng.normal(size=(n_rows, 16))
    th[:, 11:14] *= np.array([1.0, 0.3, 2.0])
    dt, V, T = 1.0, 1.2e4, 310.0
    with context("tersoff") as ctx:
        out = ctx.green_kubo(torch.tensor(th, device="cuda:0"), every, max_lag, dt, V, T)
        torch.cuda.synchronize()
        hac, kap = out["hac"].cpu().numpy(), out["kappa"].cpu().numpy()
    C, K = _oracle(th, every, max_lag, dt, V, T)
    _compare(hac, C)
    _compare(kap, K)
    assert np.all(kap[0] == 0.0)


def test_green_kubo_on_an_md_heat_current():
    """J from 3000 NVE steps of the 512-atom crystal, sampled every 2 steps,
    correlated over 500 lags; also the same bits on a second call."""
    import torch
    s = wl.tersoff_small()
    with context("tersoff") as ctx:
        out = ctx.nve_run(to_dev(s.pos), to_dev(s.vel), s.box, wl.M_SI, 1.0, 3000,
                          rebuild_every=20)
        th_dev = out["thermo"]
        T = float(th_dev[:, 15].mean())
        V = float(np.prod(s.box))
        a = ctx.green_kubo(th_dev, 2, 500, 1.0, V, T)
        b = ctx.green_kubo(th_dev, 2, 500, 1.0, V, T)
        torch.cuda.synchronize()
        assert torch.equal(a["hac"], b["hac"]) and torch.equal(a["kappa"], b["kappa"])
        hac, kap = a["hac"].cpu().numpy(), a["kappa"].cpu().numpy()
        th = th_dev.cpu().numpy()
    C, K = _oracle(th, 2, 500, 1.0, V, T)
    _compare(hac, C)
    _compare(kap, K)
    assert np.all(hac[0] > 0)
    print(f"512-atom crystal, 3000 steps: C(0) = {hac[0]} (eV A/fs)^2, "
          f"kappa(1 ps) = {kap[-1]} W/(m K)")


def test_green_kubo_errors():
    import torch
    import paper_1610_03343_amd as mb
    th = torch.zeros(10, 16, dtype=torch.float64, device="cuda:0")
    with context("tersoff") as ctx:
        for args in [(1, 11, 1.0, 1.0, 300.0),    # more lags than samples
                     (3, 5, 1.0, 1.0, 300.0),     # 4 samples at every = 3
                     (1, 0, 1.0, 1.0, 300.0),
                     (0, 1, 1.0, 1.0, 300.0),
                     (1, 5, 1.0, 1.0, 0.0),
                     (1, 5, 1.0, -2.0, 300.0),
                     (1, 5, float("nan"), 1.0, 300.0)]:
            with pytest.raises(mb.MbmdError) as e:
                ctx.green_kubo(th, *args)
            assert e.value.code == mb.MBMD_EINVAL, args
        # hac alone (no conductivity) is allowed
        out = ctx.green_kubo(th, 3, 4, 1.0, 1.0, 300.0, kappa=False)
        torch.cuda.synchronize()
        assert "kappa" not in out and torch.equal(out["hac"], torch.zeros_like(out["hac"]))


def test_green_kubo_full_size_sampled_lags():
    """The correlator at the size the bench times (10^6 samples, 10^4 lags):
    sampled lags against the oracle's per-lag dot products."""
    import torch
    from oracle import green_kubo as gk
    S, K = 1_000_000, 10_000
    rng = np.random.default_rng(1005)
    th = rng.normal(size=(S, 16))
    with context("tersoff") as ctx:
        out = ctx.green_kubo(torch.tensor(th, device="cuda:0"), 1, K, 1.0, 1.0, 300.0,
                             kappa=False)
        torch.cuda.synchronize()
        hac = out["hac"].cpu().numpy()
    lags = [0, 1, 63, 64, 65, 1023, 1024, 5000, K - 1]
    ref = gk.hcacf_lags(th[:, 11:14], lags)
    scale = np.max(np.abs(ref), axis=0)
    assert np.all(np.max(np.abs(hac[lags] - ref), axis=0) <= TOL * scale)
