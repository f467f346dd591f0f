"""The allocation-free collision entry point (ephx_collision_noalloc) against
ephx_collision, through the C ABI: two calls in a row on one table, then a
call on a smaller table (the static work array keeps the previous call's
contents), on FP64 and FP32 tables; bit-identical results are expected, since
the two entry points run the same kernels on the same plan.  Before
ephx_collision_setup there is no plan, and the call is refused."""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import grid, interp

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _states(m, n, count):
    eps, _ = interp.bands(m, grid.grid_points(n))
    return grid.lowest_states(eps.numpy(), m.nw // 2, count)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_collision_noalloc_matches_collision(prec):
    import paper_2002_02045_amd as px
    m = synth.make_config_model("tiny")
    dm = px.Model(m)
    par = px.Params(temp=300.0, sigma=0.02, n_q=1728.0)
    big = px.PairTable(dm, (12, 12, 12), *_states(m, (12, 12, 12), 1030), precision=prec)
    small = px.PairTable(dm, (6, 6, 6), *_states(m, (6, 6, 6), 60), precision=prec)
    big.setup(par)
    small.setup(px.Params(temp=300.0, sigma=0.02, n_q=216.0))
    rng = np.random.default_rng(41)
    for t, label in ((big, "S=1030"), (big, "S=1030 again"), (small, "S=60 after S=1030")):
        _say("collision_noalloc %s %s" % (prec, label))
        f = torch.as_tensor(rng.random(t.S) * 0.4, device="cuda")
        ref = t.collision(f)
        out = torch.full((t.S,), float("nan"), dtype=torch.float64, device="cuda")
        t.collision_noalloc(f, out)
        torch.cuda.synchronize()
        assert torch.isfinite(out).all()
        assert torch.equal(out, ref)
    small.close()
    big.close()


def test_collision_noalloc_needs_setup():
    import paper_2002_02045_amd as px
    m = synth.make_config_model("tiny")
    dm = px.Model(m)
    t = px.PairTable(dm, (6, 6, 6), *_states(m, (6, 6, 6), 60), precision="fp64")
    f = torch.zeros(t.S, dtype=torch.float64, device="cuda")
    out = torch.zeros_like(f)
    with pytest.raises(px.EphxError):
        t.collision_noalloc(f, out)           # no setup yet
    t.close()
