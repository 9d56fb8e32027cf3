"""The single point that allocates nothing (mbmd_compute_noalloc): through
the C ABI it gives the bits of mbmd_compute on the same inputs, on calls in a
row that share the static device scratch (the second one smaller), and it
refuses a structure whose workspace exceeds the scratch."""
import numpy as np
import pytest
import torch

import workload as wl
from gpu_util import context, to_dev

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 64 << 20


def _outs(n):
    z = lambda *s: torch.full(s, np.nan, dtype=torch.float64, device="cuda:0")
    return dict(U=z(n), F=z(3, n), W=z(9, n), J=z(3, n))


def _host(out):
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("pot,M", [("tersoff", 32), ("sw", 64)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_equals_compute_twice(pot, M, precision):
    """Two calls in a row, the second on a smaller structure, each against
    mbmd_compute on its own context and workspace: U, F, W, J equal bit for
    bit.  The first input (4,032 atoms: many blocks and a ragged tail) is a
    compressed lattice whose 16 (Tersoff) or 28 (SW) bonds per atom send
    every site to the overflow pass; the second is a hot vacancy crystal of
    a few blocks on the fast path."""
    big = wl.silicon_crystal((9, 8, 7), seed=401, sigma=0.05, a=4.2)
    small = wl.silicon_crystal(3, seed=402, sigma=0.15, vacancy_fraction=0.04,
                               temperature=900.0)
    with context(pot, max_neighbors=M) as ref, context(pot, max_neighbors=M) as ctx:
        for s in (big, small):
            assert ctx.workspace_size(s.n) <= SCRATCH_BYTES
            pos, vel = to_dev(s.pos), to_dev(s.vel)
            want = _host(ref.compute(pos, s.box, vel=vel, precision=precision,
                                     out=_outs(s.n)))
            got = _host(ctx.compute_noalloc(pos, s.box, _outs(s.n), vel=vel,
                                            precision=precision))
            for k in ("U", "F", "W", "J"):
                assert np.array_equal(got[k], want[k]), (s.n, k)
        # an ordinary call on the same context afterwards uses its own
        # workspace again and still agrees
        again = _host(ctx.compute(to_dev(big.pos), big.box, vel=to_dev(big.vel),
                                  precision=precision))
        want = _host(ref.compute(to_dev(big.pos), big.box, vel=to_dev(big.vel),
                                 precision=precision))
        for k in ("U", "F", "W", "J"):
            assert np.array_equal(again[k], want[k]), k


def test_noalloc_refuses_structures_beyond_the_scratch():
    import paper_1610_03343_amd as mb
    s = wl.silicon_crystal((22, 22, 22), seed=403)      # 85,184 atoms
    with context("tersoff") as ctx:
        assert ctx.workspace_size(s.n) > SCRATCH_BYTES
        with pytest.raises(mb.MbmdError) as e:
            ctx.compute_noalloc(to_dev(s.pos), s.box, _outs(s.n))
        assert e.value.code == mb.MBMD_ENOMEM
        assert "static scratch" in str(e.value)
        ok = wl.silicon_crystal(2, seed=404)              # the context still works
        out = ctx.compute_noalloc(to_dev(ok.pos), ok.box, _outs(ok.n))
        torch.cuda.synchronize()
        assert torch.isfinite(out["F"]).all()
