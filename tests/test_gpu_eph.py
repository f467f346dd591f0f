"""GPU parity of the g(k,q) path against the FP64 oracle: bands, phonons,
|g|^2 (FP64, FP32, BF16x3) and scattering rates, through the C ABI.

Tolerances (per result, metric in tests/helpers.py):
  FP64 path: 1e-10 relative; FP32 / BF16x3 |g|^2: 1e-5 of the pair's block
  maximum (group sums over degenerate bands/modes); rates 1e-4 relative.
"""
import sys

import numpy as np
import pytest
import torch

import synth
from helpers import g2_error, group_labels, group_sums_g2, rate_error
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
def tiny(lib):
    m = synth.make_config_model("tiny")
    return m, lib.Model(m)


def test_bands_parity(lib, tiny):
    _say("bands parity tiny model")
    m, dm = tiny
    k = synth.random_points(101, 333)                        # ragged vs 64-row tiles
    eps, u, v = lib.bands(dm, k, want_u=True, want_vel=True)
    eo, uo, vo = interp.bands(m, k, velocity=True)
    scale = float(eo.abs().max())
    assert float((eps.cpu() - eo).abs().max()) <= 1e-10 * scale
    # eigenvectors: H(k) U = U diag(eps) with the oracle's H(k), and U unitary
    hk = interp.hamiltonian_k(m, k)
    uc = u.cpu()
    res = hk @ uc - uc * eps.cpu()[:, None, :]
    assert float(res.abs().max()) <= 1e-10 * scale
    eye = torch.eye(m.nw, dtype=torch.complex128)
    assert float((uc.mH @ uc - eye).abs().max()) <= 1e-12
    vmax = float(vo.abs().max())
    assert float((v.cpu() - vo).abs().max()) <= 1e-9 * vmax


def test_phonons_parity(lib, tiny):
    _say("phonons parity tiny model")
    m, dm = tiny
    q = np.vstack([np.zeros((1, 3)), synth.random_points(102, 130)])
    om, ev = lib.phonons(dm, q)
    oo, eo = interp.phonons(m, q)
    wmax = float(oo.abs().max())
    # Gamma acoustic modes are ~1e-9 eV: compare omega^2 (the eigenvalues) there
    assert float((om.cpu()[1:] - oo[1:]).abs().max()) <= 1e-10 * wmax
    assert float((om.cpu()[0, :3].abs()).max()) <= 1e-6 * wmax
    d = interp.dynamical_matrix(m, q)
    lam = (oo.sign() * oo ** 2 / 0.004180159280496722)
    evc = ev.cpu()
    lam_g = om.cpu().sign() * om.cpu() ** 2 / 0.004180159280496722
    res = d @ evc - evc * lam_g[:, None, :]
    assert float(res.abs().max()) <= 1e-10 * float(lam.abs().max())


def _oracle_g2_groups(m, k, q):
    blk = eph.eph_pipeline(m, k, q)
    g2 = blk["g"].abs() ** 2
    ref = group_sums_g2(g2, blk["eps_k"], blk["eps_kq"], blk["omega"])
    return blk, ref


@pytest.fixture(scope="module")
def gkq_case(tiny):
    m, _ = tiny
    k = synth.random_points(103, 24)      # 16 + 8 k batches
    q = synth.random_points(104, 100)     # ragged q tail
    blk, ref = _oracle_g2_groups(m, k, q)
    return k, q, blk, ref


# BF16x3 (two bf16 parts, three products) carries a representation error of
# ~3*2^-18 per product; its measured |g|^2 error on this case is 1.02e-5
# (p99 8e-6): it misses the 1e-5 contract, which is recorded as an expected
# failure, and a separate regression bound of 2e-5 guards it.  BF16x6 and
# FP16x3 meet 1e-5 with margin.
@pytest.mark.parametrize("prec,tol", [
    ("fp64", 1e-10), ("fp32", 1e-5),
    pytest.param("bf16x3", 1e-5, marks=pytest.mark.xfail(
        strict=True, reason="two bf16 parts per operand: measured 1.02e-5 here, 1.1-1.3e-5 elsewhere")),
    ("bf16x6", 1e-5), ("fp16x3", 1e-5)])
def test_gkq_parity(lib, tiny, gkq_case, prec, tol):
    _say("gkq parity tiny model prec=%s" % prec)
    m, dm = tiny
    k, q, blk, ref = gkq_case
    g2 = lib.gkq(dm, k, q, precision=prec)
    got = group_sums_g2(g2.double().cpu().numpy(), blk["eps_k"], blk["eps_kq"], blk["omega"])
    emax, e99 = g2_error(got, ref)
    _say("  |g|^2 error %s: max %.3e  p99 %.3e" % (prec, emax, e99))
    assert emax <= tol


def test_gkq_bf16x3_regression_bound(lib, tiny, gkq_case):
    """BF16x3 below the 1e-5 contract is not met (see test_gkq_parity); this
    holds it to its measured level so that a regression still fails."""
    test_gkq_parity(lib, tiny, gkq_case, "bf16x3", 2e-5)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5), ("bf16x6", 1e-5), ("fp16x3", 1e-5)])
def test_gkq_parity_one_sided_rp(lib, prec, tol):
    """An Rp list without any +/-R pair (R = 0 and the vectors that are
    lexicographically positive) leaves the half-set form nothing to gain, so the
    library sums over the list with complex phases; parity of that path."""
    import dataclasses
    m = synth.make_config_model("tiny")
    keep = [i for i, r in enumerate(m.rp_g.tolist()) if tuple(r) >= (0, 0, 0)]
    m = dataclasses.replace(m, rp_g=m.rp_g[keep], w_rp_g=m.w_rp_g[keep], g=m.g[:, keep])
    v = {tuple(r) for r in m.rp_g.tolist()}
    assert not any(tuple(-c for c in r) in v for r in v if r != (0, 0, 0))
    _say("gkq parity one-sided Rp list (%d vectors) prec=%s" % (len(keep), prec))
    k = synth.random_points(131, 5)
    q = synth.random_points(132, 70)
    blk, ref = _oracle_g2_groups(m, k, q)
    g2 = lib.gkq(lib.Model(m), k, q, precision=prec)
    got = group_sums_g2(g2.double().cpu().numpy(), blk["eps_k"], blk["eps_kq"], blk["omega"])
    emax, e99 = g2_error(got, ref)
    _say("  |g|^2 error %s: max %.3e  p99 %.3e" % (prec, emax, e99))
    assert emax <= tol


@pytest.mark.parametrize("factor", [1e-6, 1e6])
def test_fp16x3_scale_of_g(lib, factor):
    """FP16x3 scales the g(k,Rp) operand into fp16's range by a power of two
    fixed per model: a coupling tensor a million times smaller or larger than
    the tiny model's must give the same relative |g|^2 error (no underflow to
    zero, no overflow to inf)."""
    import dataclasses
    m = synth.make_config_model("tiny")
    m = dataclasses.replace(m, g=m.g * factor)
    _say("FP16x3 with g scaled by %g" % factor)
    k = synth.random_points(151, 5)
    q = synth.random_points(152, 60)
    blk, ref = _oracle_g2_groups(m, k, q)
    g2 = lib.gkq(lib.Model(m), k, q, precision="fp16x3")
    assert bool(torch.isfinite(g2).all())
    got = group_sums_g2(g2.double().cpu().numpy(), blk["eps_k"], blk["eps_kq"], blk["omega"])
    emax, e99 = g2_error(got, ref)
    _say("  |g|^2 error: max %.3e  p99 %.3e" % (emax, e99))
    assert emax <= 1e-5


def test_rates_parity(lib, tiny):
    _say("rates parity tiny model")
    m, dm = tiny
    c = synth.CONFIGS["tiny"]
    k = synth.random_points(105, 10)
    q = synth.random_points(106, 300)
    par = dict(temp=c["T"], mu=c["mu"], sigma=0.05)
    go, gmo = eph.rates(m, k, q, **par)
    p = lib.Params(temp=c["T"], mu=c["mu"], sigma=0.05, omega_cut=1e-4)
    for prec, tol in (("fp64", 1e-10), ("fp32", 1e-4), ("bf16x3", 1e-4), ("bf16x6", 1e-4), ("fp16x3", 1e-4)):
        g, gm = lib.rates(dm, k, q, p, precision=prec)
        err = rate_error(g.cpu().numpy(), go.numpy())
        errm = rate_error(gm.cpu().numpy(), gmo.numpy())
        _say("  rates error %s: %.3e (per mode %.3e)" % (prec, err, errm))
        assert err <= tol and errm <= tol


def test_rates_with_weights_and_empty_q(lib, tiny):
    m, dm = tiny
    k = synth.random_points(107, 3)
    q = synth.random_points(108, 70)
    w = np.random.default_rng(0).random(70)
    w /= w.sum()
    go, _ = eph.rates(m, k, q, temp=300.0, mu=0.0, sigma=0.05, q_weights=w)
    p = lib.Params(temp=300.0, mu=0.0, sigma=0.05)
    g, _ = lib.rates(dm, k, q, p, q_weights=w)
    assert rate_error(g.cpu().numpy(), go.numpy()) <= 1e-10
    g0, _ = lib.rates(dm, k, np.zeros((0, 3)), p)
    assert float(g0.abs().max()) == 0.0


def test_error_paths(lib, tiny):
    m, dm = tiny
    with pytest.raises(lib.EphxError) as ei:
        lib.gkq(dm, synth.random_points(1, 2), synth.random_points(2, 2), precision=7)
    assert ei.value.code == -1
    bad = synth.make_config_model("tiny")
    bad.h = bad.h.copy()
    bad.h[5] += 0.1                      # breaks H(-R) = H(R)^dagger
    with pytest.raises(lib.EphxError) as ei:
        lib.Model(bad)
    assert ei.value.code == -4
    nan = synth.make_config_model("tiny")
    nan.g = nan.g.copy()
    nan.g[0, 0, 0, 0, 0] = np.nan
    with pytest.raises(lib.EphxError) as ei:
        lib.Model(nan)
    assert ei.value.code == -5
    e0, _, _ = lib.bands(dm, np.zeros((0, 3)))
    assert e0.shape == (0, m.nw)


def test_polar_gkq_and_rates_parity(lib):
    """GaAs-like polar model: the Froehlich term (Eq. e_ph_long, smooth-phase
    bra-ket) is added in the Wannier gauge before the rotation."""
    _say("polar gkq/rates parity (GaAs-like, 4^3 set, nw=4)")
    m = synth.make_config_model("gaas", n_grid=4, nw=4)
    a = synth.models.A_GAAS
    pol = dict(alpha_ewald=(2 * np.pi / a) ** 2, gcut=4 * 2 * np.pi / a)
    dm = lib.Model(m, polar=pol)
    k = synth.random_points(111, 12)
    q = np.vstack([synth.random_points(112, 70), 1e-3 * np.array([[0.3, -0.2, 0.1]])])   # includes small q
    blk = eph.eph_pipeline(m, k, q, polar=pol)
    ref = group_sums_g2(blk["g"].abs() ** 2, blk["eps_k"], blk["eps_kq"], blk["omega"])
    for prec, tol in (("fp64", 1e-10), ("fp32", 1e-5)):
        g2 = lib.gkq(dm, k, q, precision=prec)
        got = group_sums_g2(g2.double().cpu().numpy(), blk["eps_k"], blk["eps_kq"], blk["omega"])
        emax, _ = g2_error(got, ref)
        _say("  polar |g|^2 error %s: %.3e" % (prec, emax))
        assert emax <= tol
    go, _ = eph.rates(m, k, q, temp=300.0, mu=0.0, sigma=0.05, polar=pol)
    g, _ = lib.rates(dm, k, q, lib.Params(temp=300.0, mu=0.0, sigma=0.05))
    assert rate_error(g.cpu().numpy(), go.numpy()) <= 1e-10


def test_rates_vjp_parity_and_finite_difference(lib, tiny):
    """Hand-written adjoint of the rates w.r.t. g(Re,Rp) vs the oracle's autograd
    gradient (1e-10) and vs a central difference of the GPU rates along a random
    direction (1e-6)."""
    import copy
    from oracle import grad
    _say("rates VJP w.r.t. g(Re,Rp), tiny model")
    m, dm = tiny
    k = synth.random_points(121, 3)
    q = synth.random_points(122, 45)
    lam = np.random.default_rng(123).random((3, m.nw))
    kw = dict(temp=300.0, mu=0.0, sigma=0.08)
    p = lib.Params(temp=300.0, mu=0.0, sigma=0.08)
    _, gref = grad.rates_grad_g(m, k, q, lam, **kw)
    gb = lib.rates_vjp(dm, k, q, p, lam).cpu()
    err = float((gb - gref).abs().max() / gref.abs().max())
    _say("  adjoint vs oracle autograd: %.3e" % err)
    assert err <= 1e-10
    # directional central difference of the GPU rates
    direc = np.random.default_rng(124).standard_normal(m.g.shape) + 1j * np.random.default_rng(125).standard_normal(m.g.shape)
    h = 1e-6 * float(np.abs(m.g).max())
    vals = []
    for sgn in (1.0, -1.0):
        mm = copy.deepcopy(m)
        mm.g = m.g + sgn * h * direc
        g_s, _ = lib.rates(lib.Model(mm), k, q, p, mode_resolved=False)
        vals.append(float((g_s.cpu().numpy() * lam).sum()))
    fd = (vals[0] - vals[1]) / (2 * h)
    ad = float((gb.numpy().real * direc.real + gb.numpy().imag * direc.imag).sum())
    _say("  directional FD %.9e vs adjoint %.9e" % (fd, ad))
    assert abs(fd - ad) <= 1e-6 * abs(ad)
    # the autograd Function computes from the g it is given and routes its
    # backward through the same entry point
    gt = torch.as_tensor(m.g, dtype=torch.complex128, device="cuda").requires_grad_(True)
    gam = lib.RatesFunction.apply(gt, dm, k, q, p)
    g0, _ = lib.rates(dm, k, q, p, mode_resolved=False)
    assert torch.equal(gam.detach(), g0)
    (gam * torch.as_tensor(lam, device="cuda")).sum().backward()
    assert torch.allclose(gt.grad.cpu(), gb)


def test_lo_to_phonons_gkq_rates_parity(lib):
    """Dipole-dipole (LO-TO) part of D(q) on the GPU vs the oracle: phonons
    (including Gamma and a small q, where the splitting is non-analytic), and
    |g|^2 and rates, which see it through omega and e."""
    _say("LO-TO parity (GaAs-like, 4^3 set, nw=4)")
    m = synth.make_config_model("gaas", n_grid=4, nw=4)
    a = synth.models.A_GAAS
    pol = dict(alpha_ewald=(2 * np.pi / a) ** 2, gcut=4 * 2 * np.pi / a, lo_to=True)
    dip = dict(alpha_ewald=pol["alpha_ewald"], gcut=pol["gcut"])
    dm = lib.Model(m, polar=pol)
    q = np.vstack([np.zeros((1, 3)), 1e-3 * np.array([[0.3, -0.2, 0.1]]), synth.random_points(131, 60)])
    om, ev = lib.phonons(dm, q)
    oo, _ = interp.phonons(m, q, dipole=dip)
    wmax = float(oo.abs().max())
    assert float((om.cpu()[1:] - oo[1:]).abs().max()) <= 1e-10 * wmax
    assert float(om.cpu()[0, :3].abs().max()) <= 1e-6 * wmax
    assert float((om.cpu()[0, 3:] - oo[0, 3:]).abs().max()) <= 1e-10 * wmax
    d = interp.dynamical_matrix(m, q, dipole=dip)
    lam = om.cpu().sign() * om.cpu() ** 2 / 0.004180159280496722
    res = d @ ev.cpu() - ev.cpu() * lam[:, None, :]
    assert float(res.abs().max()) <= 1e-10 * float(lam.abs().max())
    k = synth.random_points(132, 6)
    qq = q[1:40]
    blk = eph.eph_pipeline(m, k, qq, polar=pol)
    ref = group_sums_g2(blk["g"].abs() ** 2, blk["eps_k"], blk["eps_kq"], blk["omega"])
    g2 = lib.gkq(dm, k, qq, precision="fp64")
    got = group_sums_g2(g2.double().cpu().numpy(), blk["eps_k"], blk["eps_kq"], blk["omega"])
    emax, _ = g2_error(got, ref)
    _say("  LO-TO |g|^2 error fp64: %.3e" % emax)
    assert emax <= 1e-10
    go, _ = eph.rates(m, k, qq, temp=300.0, mu=0.0, sigma=0.05, polar=pol)
    g, _ = lib.rates(dm, k, qq, lib.Params(temp=300.0, mu=0.0, sigma=0.05))
    assert rate_error(g.cpu().numpy(), go.numpy()) <= 1e-10


def test_cauchy_sampled_rates(lib):
    """Importance sampling of the q sum (Sec. 4.3): Cauchy points around Gamma
    with weights 1/(n p(q)).  Parity of the weighted polar rates vs the oracle,
    then agreement of the Cauchy and uniform Monte Carlo estimates over
    independent seeds (both unbiased) on the GPU alone."""
    _say("Cauchy-sampled rates (GaAs-like with LO-TO, nw=4)")
    m = synth.make_config_model("gaas", n_grid=4, nw=4)
    a = synth.models.A_GAAS
    pol = dict(alpha_ewald=(2 * np.pi / a) ** 2, gcut=4 * 2 * np.pi / a, lo_to=True)
    dm = lib.Model(m, polar=pol)
    k = np.array([[0.01, 0.02, -0.015], [0.05, 0.0, 0.0], [0.1, 0.1, 0.1]])
    par = dict(temp=300.0, mu=0.0, sigma=0.05)
    p = lib.Params(omega_cut=1e-4, **par)
    q, w = synth.cauchy_points(141, 60, 0.05)
    go, _ = eph.rates(m, k, q, q_weights=w, polar=pol, **par)
    for prec, tol in (("fp64", 1e-10), ("fp32", 1e-4)):
        g, _ = lib.rates(dm, k, q, p, precision=prec, q_weights=w)
        err = rate_error(g.cpu().numpy(), go.numpy())
        _say("  weighted rates error %s: %.3e" % (prec, err))
        assert err <= tol
    n, seeds = 16384, 6
    est_c, est_u = [], []
    for s in range(seeds):
        qc, wc = synth.cauchy_points(1000 + s, n, 0.05)
        est_c.append(lib.rates(dm, k, qc, p, q_weights=wc, mode_resolved=False)[0].cpu().numpy())
        est_u.append(lib.rates(dm, k, synth.random_points(2000 + s, n), p, mode_resolved=False)[0].cpu().numpy())
    est_c, est_u = np.array(est_c), np.array(est_u)
    mc, mu_ = est_c.mean(0), est_u.mean(0)
    se = np.sqrt(est_c.var(0, ddof=1) / seeds + est_u.var(0, ddof=1) / seeds)
    live = mu_ > 1e-3 * mu_.max()
    assert live.any()
    z = np.abs(mc - mu_)[live] / np.maximum(se[live], 1e-12 * mu_.max())
    ratio = est_u.var(0, ddof=1)[live] / np.maximum(est_c.var(0, ddof=1)[live], 1e-300)
    _say("  states %d, max |z| %.2f, variance ratio uniform/Cauchy median %.2f"
         % (int(live.sum()), float(z.max()), float(np.median(ratio))))
    assert float(z.max()) <= 5.0


def test_polar_split_rates(lib):
    """Polar split of the q sum: the long-range part |g_L|^2 and the rest
    |g|^2 - |g_L|^2 against the oracle (FP64 1e-10, FP32 1e-4 on the rates
    above the floor, the rest compared as a difference of full and long-range
    rates since it can change sign); the split estimator (rest on uniform q,
    long-range part on Cauchy q) agrees with the uniform estimate of the full
    rates over independent seeds (both unbiased), with a smaller spread."""
    _say("polar split (GaAs-like with LO-TO, nw=4)")
    m = synth.make_config_model("gaas", n_grid=4, nw=4)
    a = synth.models.A_GAAS
    pol = dict(alpha_ewald=(2 * np.pi / a) ** 2, gcut=4 * 2 * np.pi / a, lo_to=True)
    dm = lib.Model(m, polar=pol)
    k = np.array([[0.01, 0.02, -0.015], [0.05, 0.0, 0.0], [0.1, 0.1, 0.1]])
    par = dict(temp=300.0, mu=0.0, sigma=0.05)
    p = lib.Params(omega_cut=1e-4, **par)
    q, w = synth.cauchy_points(151, 50, 0.05)
    full_o, _ = eph.rates(m, k, q, q_weights=w, polar=pol, **par)
    lr_o, lrm_o = eph.rates(m, k, q, q_weights=w, polar=pol, part="polar", **par)
    rest_o, _ = eph.rates(m, k, q, q_weights=w, polar=pol, part="rmpol", **par)
    scale = float(full_o.abs().max())
    for prec, tol in (("fp64", 1e-10), ("fp32", 1e-4)):
        lr, lrm = lib.rates_part(dm, k, q, p, "polar", precision=prec, q_weights=w)
        rest, _ = lib.rates_part(dm, k, q, p, "rmpol", precision=prec, q_weights=w)
        e_lr = rate_error(lr.cpu().numpy(), lr_o.numpy())
        e_lrm = rate_error(lrm.cpu().numpy(), lrm_o.numpy())
        e_rest = float((rest.cpu() - rest_o).abs().max()) / scale
        _say("  polar part error %s: %.3e (per mode %.3e), rest %.3e of the full scale" % (prec, e_lr, e_lrm, e_rest))
        assert e_lr <= tol and e_lrm <= tol and e_rest <= tol
        sp, _ = lib.rates_polar_split(dm, k, q, q, p, precision=prec, w_uniform=w, w_cauchy=w)
        assert float((sp.cpu() - full_o).abs().max()) <= tol * scale
    with pytest.raises(lib.EphxError):
        lib.rates_part(lib.Model(m), k, q, p, "polar")          # no Froehlich term
    n, seeds = 8192, 6
    est_s, est_u = [], []
    for s in range(seeds):
        qc, wc = synth.cauchy_points(3000 + s, n, 0.05)
        qu = synth.random_points(4000 + s, n)
        est_s.append(lib.rates_polar_split(dm, k, qu, qc, p, w_cauchy=wc, mode_resolved=False)[0].cpu().numpy())
        est_u.append(lib.rates(dm, k, synth.random_points(5000 + s, n), p, mode_resolved=False)[0].cpu().numpy())
    est_s, est_u = np.array(est_s), np.array(est_u)
    ms_, mu_ = est_s.mean(0), est_u.mean(0)
    se = np.sqrt(est_s.var(0, ddof=1) / seeds + est_u.var(0, ddof=1) / seeds)
    live = mu_ > 1e-3 * mu_.max()
    assert live.any()
    z = np.abs(ms_ - mu_)[live] / np.maximum(se[live], 1e-12 * mu_.max())
    ratio = est_u.var(0, ddof=1)[live] / np.maximum(est_s.var(0, ddof=1)[live], 1e-300)
    _say("  split vs uniform: %d states, max |z| %.2f, variance ratio uniform/split median %.2f"
         % (int(live.sum()), float(z.max()), float(np.median(ratio))))
    assert float(z.max()) <= 5.0


def test_gkq_pairs_parity(lib, tiny):
    """The pair-list form of |g|^2: arbitrary (k, q) pairs, repeated k and q,
    unsorted, against the oracle pair by pair."""
    m, dm = tiny
    k = synth.random_points(151, 5)
    q = synth.random_points(152, 40)
    rng = np.random.default_rng(153)
    ik = rng.integers(0, 5, 70).astype(np.int32)
    iq = rng.integers(0, 40, 70).astype(np.int32)
    blk = eph.eph_pipeline(m, k, q)
    g = blk["g"].abs() ** 2                                   # [k][q][nu][m][n]
    ref_all = group_sums_g2(g, blk["eps_k"], blk["eps_kq"], blk["omega"])
    for prec, tol in (("fp64", 1e-10), ("fp32", 1e-5), ("bf16x6", 1e-5)):
        got = lib.gkq_pairs(dm, k, q, ik, iq, precision=prec).double().cpu()
        # place each pair's block in an outer-product array to reuse the group sums
        full = torch.zeros_like(g)
        full[torch.as_tensor(ik, dtype=torch.long), torch.as_tensor(iq, dtype=torch.long)] = got
        gs = group_sums_g2(full, blk["eps_k"], blk["eps_kq"], blk["omega"])
        sel = (torch.as_tensor(ik, dtype=torch.long), torch.as_tensor(iq, dtype=torch.long))
        d = (gs[sel] - ref_all[sel]).abs().flatten(1).max(dim=1).values
        s = ref_all[sel].abs().flatten(1).max(dim=1).values
        err = float((d / s.clamp_min(1e-300)).max())
        _say("  gkq_pairs error %s: %.3e" % (prec, err))
        assert err <= tol
    with pytest.raises(lib.EphxError):
        lib.gkq_pairs(dm, k, q, np.array([5], np.int32), np.array([0], np.int32))


def test_workspace_query(lib, tiny):
    m, dm = tiny
    b1 = lib.workspace_query(dm, "gkq", 4, 1000, "fp32")
    b2 = lib.workspace_query(dm, "gkq", 4, 100000, "fp32")
    br = lib.workspace_query(dm, "rates", 4, 100000, "fp32")
    bb = lib.workspace_query(dm, "gkq", 4, 100000, "bf16x6")
    assert 0 < b1 < b2 <= br
    assert bb > 0
    assert lib.workspace_query(dm, "gkq", 0, 10, "fp64") == 0
    with pytest.raises(lib.EphxError):
        lib.workspace_query(dm, "gkq", -1, 10, "fp64")
