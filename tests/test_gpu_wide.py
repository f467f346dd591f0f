"""GPU parity of the large-model path (nw > 16, more than 12 modes) against the
FP64 oracle: the workgroup eigensolver (bands, phonons) and the batched-GEMM
rotation / mode projection behind |g|^2 and the rates, through the C ABI.

Model: simple-cubic cell, 5 atoms (15 modes), 20 Wannier functions, 3^3 sets.
Tolerances as for the small models: FP64 1e-10 relative; FP32 / BF16x6 |g|^2
1e-5 of the pair's block maximum (degenerate-group sums); rates 1e-4.
"""
import sys

import numpy as np
import pytest
import torch

import synth
from helpers import g2_error, group_sums_g2, rate_error
from oracle import eph, interp

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import paper_2002_02045_amd as px
    return px


@pytest.fixture(scope="module")
def wide(lib):
    m = synth.make_config_model("wide")
    return m, lib.Model(m)


def test_wide_bands_parity(lib, wide):
    _say("bands parity, nw=20 (workgroup eigensolver)")
    m, dm = wide
    k = np.vstack([np.zeros((1, 3)), synth.random_points(201, 40)])
    eps, u, _ = lib.bands(dm, k, want_u=True)
    eo, _ = interp.bands(m, k)
    scale = float(eo.abs().max())
    assert float((eps.cpu() - eo).abs().max()) <= 1e-10 * scale
    hk = interp.hamiltonian_k(m, k)
    uc = u.cpu()
    assert float((hk @ uc - uc * eps.cpu()[:, None, :]).abs().max()) <= 1e-10 * scale
    eye = torch.eye(m.nw, dtype=torch.complex128)
    assert float((uc.mH @ uc - eye).abs().max()) <= 1e-12
    with pytest.raises(lib.EphxError) as ei:
        lib.bands(dm, k, want_vel=True)
    assert ei.value.code == -6


def test_wide_phonons_parity(lib, wide):
    _say("phonons parity, 15 modes (workgroup eigensolver)")
    m, dm = wide
    q = np.vstack([np.zeros((1, 3)), synth.random_points(202, 45)])
    om, ev = lib.phonons(dm, q)
    oo, _ = interp.phonons(m, q)
    wmax = float(oo.abs().max())
    assert float((om.cpu()[1:] - oo[1:]).abs().max()) <= 1e-10 * wmax
    assert float(om.cpu()[0, :3].abs().max()) <= 1e-6 * wmax
    d = interp.dynamical_matrix(m, q)
    evc = ev.cpu()
    lam = om.cpu().sign() * om.cpu() ** 2 / 0.004180159280496722
    res = d @ evc - evc * lam[:, None, :]
    assert float(res.abs().max()) <= 1e-10 * float(lam.abs().max())


def test_eig_order_64_bands_and_120_modes(lib):
    """The two sizes at the ends of the workgroup eigensolver's range: H(k) of
    order 64 (the largest kept in LDS with its eigenvectors) and D(q) of order
    120 (the large cell's 40 atoms, above the LDS range)."""
    _say("bands parity, nw=64; phonons parity, 120 modes")
    m = synth.make_config_model("wide", nw=64)
    dm = lib.Model(m)
    k = np.vstack([np.zeros((1, 3)), synth.random_points(205, 11)])
    eps, u, _ = lib.bands(dm, k, want_u=True)
    eo, _ = interp.bands(m, k)
    scale = float(eo.abs().max())
    assert float((eps.cpu() - eo).abs().max()) <= 1e-10 * scale
    hk = interp.hamiltonian_k(m, k)
    uc = u.cpu()
    assert float((hk @ uc - uc * eps.cpu()[:, None, :]).abs().max()) <= 1e-10 * scale
    assert float((uc.mH @ uc - torch.eye(64, dtype=torch.complex128)).abs().max()) <= 1e-12
    del dm
    mc = synth.make_config_model("cell", nw=2)
    dc = lib.Model(mc)
    q = np.vstack([np.zeros((1, 3)), synth.random_points(206, 7)])
    om, ev = lib.phonons(dc, q)
    oo, _ = interp.phonons(mc, q)
    wmax = float(oo.abs().max())
    assert float((om.cpu()[1:] - oo[1:]).abs().max()) <= 1e-10 * wmax
    d = interp.dynamical_matrix(mc, q)
    evc = ev.cpu()
    lam = om.cpu().sign() * om.cpu() ** 2 / 0.004180159280496722
    assert float((d @ evc - evc * lam[:, None, :]).abs().max()) <= 1e-10 * float(lam.abs().max())
    assert float((evc.mH @ evc - torch.eye(120, dtype=torch.complex128)).abs().max()) <= 1e-12


@pytest.fixture(scope="module")
def wide_case(wide):
    m, _ = wide
    k = synth.random_points(203, 3)
    q = synth.random_points(204, 37)
    blk = eph.eph_pipeline(m, k, q)
    ref = group_sums_g2(blk["g"].abs() ** 2, blk["eps_k"], blk["eps_kq"], blk["omega"])
    return k, q, blk, ref


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5), ("bf16x6", 1e-5), ("fp16x3", 1e-5)])
def test_wide_gkq_parity(lib, wide, wide_case, prec, tol):
    _say("gkq parity nw=20, 15 modes, prec=%s" % prec)
    m, dm = wide
    k, q, blk, ref = wide_case
    g2 = lib.gkq(dm, k, q, precision=prec)
    got = group_sums_g2(g2.double().cpu().numpy(), blk["eps_k"], blk["eps_kq"], blk["omega"])
    emax, e99 = g2_error(got, ref)
    _say("  |g|^2 error %s: max %.3e  p99 %.3e" % (prec, emax, e99))
    assert emax <= tol


def test_wide_rates_parity(lib, wide):
    _say("rates parity nw=20, 15 modes")
    m, dm = wide
    k = synth.random_points(205, 4)
    q = synth.random_points(206, 90)
    go, gmo = eph.rates(m, k, q, temp=300.0, mu=0.0, sigma=0.1)
    p = lib.Params(temp=300.0, mu=0.0, sigma=0.1, omega_cut=1e-4)
    for prec, tol in (("fp64", 1e-10), ("fp32", 1e-4), ("bf16x6", 1e-4), ("fp16x3", 1e-4)):
        g, gm = lib.rates(dm, k, q, p, precision=prec)
        err = rate_error(g.cpu().numpy(), go.numpy())
        errm = rate_error(gm.cpu().numpy(), gmo.numpy())
        _say("  rates error %s: %.3e (per mode %.3e)" % (prec, err, errm))
        assert err <= tol and errm <= tol


def test_wide_polar_parity(lib):
    """Long-range term on the large-model path (overlap U(k+q)^dag U(k) by GEMM)."""
    _say("polar gkq/rates parity, nw=20, 15 modes")
    m = synth.make_config_model("wide")
    z = 1.5
    m.zstar = np.stack([(z if a % 2 == 0 else -z) * np.eye(3) for a in range(m.nat)])
    m.eps_inf = 8.0 * np.eye(3)
    a = synth.CONFIGS["wide"]["a"]
    pol = dict(alpha_ewald=(2 * np.pi / a) ** 2, gcut=4 * 2 * np.pi / a)
    dm = lib.Model(m, polar=pol)
    k = synth.random_points(207, 2)
    q = np.vstack([synth.random_points(208, 20), 1e-3 * np.array([[0.3, -0.2, 0.1]])])
    blk = eph.eph_pipeline(m, k, q, polar=pol)
    ref = group_sums_g2(blk["g"].abs() ** 2, blk["eps_k"], blk["eps_kq"], blk["omega"])
    g2 = lib.gkq(dm, k, q, precision="fp64")
    got = group_sums_g2(g2.double().cpu().numpy(), blk["eps_k"], blk["eps_kq"], blk["omega"])
    emax, _ = g2_error(got, ref)
    _say("  polar |g|^2 error fp64: %.3e" % emax)
    assert emax <= 1e-10
    go, _ = eph.rates(m, k, q, temp=300.0, mu=0.0, sigma=0.1, polar=pol)
    g, _ = lib.rates(dm, k, q, lib.Params(temp=300.0, mu=0.0, sigma=0.1))
    assert rate_error(g.cpu().numpy(), go.numpy()) <= 1e-10


def test_wide_rates_vjp_parity(lib, wide):
    """Adjoint of the rates w.r.t. g(Re,Rp) on the batched-GEMM path (per pair:
    the rates derivative, the conjugate-transposed projection, U(k+q)) vs the
    oracle's autograd gradient, 1e-10 relative."""
    from oracle import grad
    m, dm = wide
    _say("rates VJP w.r.t. g(Re,Rp), nw=20, 15 modes")
    k = synth.random_points(141, 2)
    q = synth.random_points(142, 21)
    lam = np.random.default_rng(143).random((2, m.nw))
    _, gref = grad.rates_grad_g(m, k, q, lam, temp=300.0, mu=0.0, sigma=0.1)
    gb = lib.rates_vjp(dm, k, q, lib.Params(temp=300.0, mu=0.0, sigma=0.1), lam).cpu()
    err = float((gb - gref).abs().max() / gref.abs().max())
    _say("  adjoint vs oracle autograd: %.3e" % err)
    assert err <= 1e-10


def test_wide_unsupported_calls(lib, wide):
    m, dm = wide
    with pytest.raises(lib.EphxError) as ei:
        lib.PairTable(dm, (2, 2, 2), np.array([0, 1], np.int32), np.array([10, 10], np.int32))
    assert ei.value.code == -6
