"""Models whose g(Re,Rp) is drawn on the device by the counter scheme
(Philox4x32-10, Irwin-Hall variates, complex-float storage) instead of being
uploaded: needed for the large cell at its named shape (6^3 real-space sets,
120 modes, 64 functions: 183 GB of complex float).

- The draws: device entries read back equal the host's counter_coupling bit
  for bit, at the small shapes and at sampled indices of the full large-cell
  tensor (1.1e10 entries).
- Parity: a drawn tiny model (Nw = 4, 6 modes) and a drawn wide model (Nw = 20,
  15 modes, batched-GEMM path) against the oracle run on the host-drawn g:
  |g|^2 group sums and rates, as for uploaded models.
- At the large-cell shape: |g|^2 of the reduced precisions against the FP64
  path on a few pairs (a property that holds at any size), finite rates."""
import gc
import sys

import numpy as np
import pytest
import torch

import synth
from helpers import g2_error, group_sums_g2, rate_error
from oracle import eph

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import paper_2002_02045_amd as px
    return px


@pytest.mark.parametrize("name,kw", [("tiny", {}), ("wide", {})])
def test_drawn_model_parity(lib, name, kw):
    m, env, seed = synth.make_counter_model(name, **kw)
    _say("drawn-g model %s: nw=%d modes=%d, %d x %d vectors" % (name, m.nw, m.nmodes, len(m.re_g), len(m.rp_g)))
    dm = lib.Model(m, drawn=(seed, env))
    rng = np.random.default_rng(7)
    idx = np.unique(np.concatenate([[0, m.g.size - 1], rng.integers(0, m.g.size, 200)]))
    got = dm.g_entries(idx)
    assert np.array_equal(got, m.g.reshape(-1)[idx])
    k = synth.random_points(201, 3)
    q = synth.random_points(202, 37)
    blk = eph.eph_pipeline(m, k, q)
    ref = group_sums_g2(blk["g"].abs() ** 2, blk["eps_k"], blk["eps_kq"], blk["omega"])
    for prec, tol in (("fp64", 1e-10), ("fp32", 1e-5), ("fp16x3", 1e-5)):
        g2 = lib.gkq(dm, k, q, precision=prec)
        got2 = group_sums_g2(g2.double().cpu().numpy(), blk["eps_k"], blk["eps_kq"], blk["omega"])
        emax, _ = g2_error(got2, ref)
        _say("  |g|^2 error %s: %.3e" % (prec, emax))
        assert emax <= tol
    par = dict(temp=300.0, mu=0.0, sigma=0.05)
    go, _ = eph.rates(m, k, q, **par)
    for prec, tol in (("fp64", 1e-10), ("fp32", 1e-4)):
        g, _ = lib.rates(dm, k, q, lib.Params(**par), precision=prec)
        err = rate_error(g.cpu().numpy(), go.numpy())
        _say("  rates error %s: %.3e" % (prec, err))
        assert err <= tol
    with pytest.raises(lib.EphxError):
        lib.rates_vjp(dm, k, q, lib.Params(**par), np.ones((3, m.nw)))
    with pytest.raises(lib.EphxError):
        dm.set_g(torch.zeros(dm.g_shape, dtype=torch.complex128, device="cuda"))
    dm.close()


def test_large_cell_named_shape(lib):
    """The large cell on its 6^3 sets: g drawn on the device (183 GB), the
    draws checked at sampled indices, |g|^2 of FP32 and FP16x3 against the
    FP64 path on 2 k x 8 q, and finite rates on them."""
    gc.collect()
    torch.cuda.empty_cache()
    m, env, seed = synth.make_counter_model("cell", n_grid=6, full=False)
    per = m.nmodes * m.nw * m.nw
    total = len(m.re_g) * len(m.rp_g) * per
    _say("large cell 6^3: %d Re x %d Rp, %d entries (%.0f GB complex float)" % (
        len(m.re_g), len(m.rp_g), total, total * 8 / 1e9))
    dm = lib.Model(m, drawn=(seed, env))
    rng = np.random.default_rng(11)
    idx = np.unique(np.concatenate([[0, total - 1, total // 2], rng.integers(0, total, 300)]))
    host = synth.counter_coupling(env, per, seed, entries=idx).astype(np.complex128)
    assert np.array_equal(dm.g_entries(idx), host)
    k = synth.random_points(211, 2)
    q = synth.random_points(212, 8)
    ref = lib.gkq(dm, k, q, precision="fp64").cpu()
    ek, _, _ = lib.bands(dm, k, want_u=False)
    kq = (k[:, None, :] + q[None, :, :]).reshape(-1, 3)
    ekq, _, _ = lib.bands(dm, kq, want_u=False)
    om, _ = lib.phonons(dm, q, want_evec=False)
    ek, ekq, om = ek.cpu().numpy(), ekq.cpu().numpy().reshape(2, 8, -1), om.cpu().numpy()
    rs = group_sums_g2(ref.numpy(), ek, ekq, om)
    assert float(rs.max()) > 0
    for prec in ("fp32", "fp16x3"):
        got = group_sums_g2(lib.gkq(dm, k, q, precision=prec).double().cpu().numpy(), ek, ekq, om)
        emax, _ = g2_error(got, rs)
        _say("  6^3 large cell |g|^2 error %s vs FP64: %.3e" % (prec, emax))
        assert emax <= 1e-5
    g, _ = lib.rates(dm, k, q, lib.Params(temp=300.0, mu=0.0, sigma=0.005), precision="fp16x3")
    assert bool(torch.isfinite(g).all())
    dm.close()
    gc.collect()
    torch.cuda.empty_cache()
