"""GPU parity of the transport path on the polar (GaAs-like) model and of the
iterative BTE run to its stopping threshold, through the C ABI:

- the symmetrised pair table with the Froehlich term of Eq. e_ph_long (and with
  the LO-TO part of D(q) as well) against the oracle, FP64 and reduced precisions;
- the iterative BTE (Eq. BTE_iter) run until F changes by less than tol, against
  the oracle's iteration with the same rule and against the dense solution of
  (1 - diag(tau/N_q) W) F = tau v with sum_s F_s = 0;
- the mobility (Eq. cond) from FP32 and split-precision tables against the FP64
  oracle (contract 1e-4 per diagonal component);
- the mobility adjoint w.r.t. g(Re,Rp) on the polar model against the oracle's
  autograd (1e-10) and a GPU central difference (1e-6);
- the autograd Functions compute from the g tensor they are given.

Model: GaAs-like (Z* = +-2.1, eps_inf = 10.9, real H, C and g, so time reversal
holds and F^0 is odd), 4^3 real-space sets, Nw = 4; states of the conduction
bands in a 0.9 eV window on an 8^3 grid (160 states)."""
import dataclasses
import sys

import numpy as np
import pytest
import torch

import synth
from helpers import group_labels
from oracle import bte, grad, grid, interp

pytestmark = pytest.mark.gpu

A = synth.models.A_GAAS
POL = dict(alpha_ewald=(2 * np.pi / A) ** 2, gcut=4 * 2 * np.pi / A)
GRID = (8, 8, 8)
T, SIG = 300.0, 0.02


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import paper_2002_02045_amd as px
    return px


def _states(m, n, window):
    eps_g, _ = interp.bands(m, grid.grid_points(n))
    cbm = float(eps_g[:, m.nw // 2].min())
    kk, bb = grid.window_states(eps_g.numpy(), m.nw // 2, m.nw, cbm - 0.01, cbm + window)
    _, _, v = interp.bands(m, bte.state_points(kk, n), velocity=True)
    vel = v[torch.arange(len(bb)), torch.as_tensor(bb)]
    return kk, bb, vel, cbm


@pytest.fixture(scope="module")
def polar(lib):
    m = synth.make_config_model("gaas", n_grid=4, nw=4)
    kk, bb, vel, cbm = _states(m, GRID, 0.9)
    _say("polar oracle pair table S=%d" % len(kk))
    g2s, om = bte.pair_table(m, GRID, kk, bb, polar=POL)
    eps = bte.state_energies(m, kk, bb, GRID)
    return dict(m=m, dm=lib.Model(m, polar=POL), kk=kk, bb=bb, vel=vel, g2s=g2s, om=om, eps=eps,
                mu=cbm - 0.3, nq=float(np.prod(GRID)))


def _mode_group_sums(g2, omega):
    lab = group_labels(np.asarray(omega))                 # (s, t, nu)
    oh = torch.nn.functional.one_hot(torch.as_tensor(lab), g2.shape[0]).double()
    return torch.einsum("vst,stva->ast", torch.as_tensor(np.asarray(g2), dtype=torch.float64), oh)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5), ("fp16x3", 1e-5), ("bf16x6", 1e-5)])
def test_polar_table_parity(lib, polar, prec, tol):
    c = polar
    _say("polar pair table S=%d prec=%s" % (len(c["kk"]), prec))
    t = lib.PairTable(c["dm"], GRID, c["kk"], c["bb"], precision=prec)
    g, e = t.g2()
    ref = _mode_group_sums(c["g2s"].permute(2, 0, 1).numpy(), c["om"].numpy())
    got = _mode_group_sums(g.double().cpu().numpy(), c["om"].numpy())
    err = float((got - ref).abs().max() / ref.abs().max())
    _say("  polar table error %s: %.3e" % (prec, err))
    assert err <= tol
    assert float((e.cpu() - c["eps"]).abs().max()) <= 1e-12 * float(c["eps"].abs().max())
    # the long-range term is not negligible on this table
    m_sr = dataclasses.replace(c["m"])
    t_sr = lib.PairTable(lib.Model(m_sr), GRID, c["kk"], c["bb"], precision="fp64")
    g_sr, _ = t_sr.g2()
    assert float((g_sr.double().cpu() - g.double().cpu()).abs().max()) > 1e-3 * float(g.abs().max())


def test_polar_lo_to_table_parity(lib, polar):
    c = polar
    pol = dict(POL, lo_to=True)
    _say("polar + LO-TO pair table S=%d fp64" % len(c["kk"]))
    g2s, om = bte.pair_table(c["m"], GRID, c["kk"], c["bb"], polar=pol)
    t = lib.PairTable(lib.Model(c["m"], polar=pol), GRID, c["kk"], c["bb"], precision="fp64")
    g, _ = t.g2()
    ref = _mode_group_sums(g2s.permute(2, 0, 1).numpy(), om.numpy())
    got = _mode_group_sums(g.double().cpu().numpy(), om.numpy())
    err = float((got - ref).abs().max() / ref.abs().max())
    _say("  LO-TO table error %.3e" % err)
    assert err <= 1e-10


def _partners(kk, bb, n):
    """Index of the state at -k with the same band, for every state."""
    pos = {(int(k), int(b)): i for i, (k, b) in enumerate(zip(kk, bb))}
    mk = grid.grid_index((-grid.grid_coords(kk, n)) % np.asarray(n), n)
    return np.array([pos[(int(mk[i]), int(bb[i]))] for i in range(len(kk))])


def _oracle_w(c, g2s=None):
    return bte.transport_matrix(c["eps"], c["g2s"] if g2s is None else g2s, c["om"], temp=T, mu=c["mu"], sigma=SIG)


def test_polar_ita_to_threshold(lib, polar):
    """Eq. BTE_iter to a threshold: the GPU stops where the oracle does (the
    relative change first below tol) and its F is the dense solution; n_iter_max
    = 0 is the RTA and a cap below the count stops there."""
    c = polar
    t = lib.PairTable(c["dm"], GRID, c["kk"], c["bb"], precision="fp64")
    par = lib.Params(temp=T, mu=c["mu"], sigma=SIG, n_q=c["nq"])
    w = _oracle_w(c)
    tol = 1e-12
    fo, tau_o, n_o, chg_o = bte.ita_converged(w, c["vel"], c["nq"], 1000, tol)
    ff, tau, mob, n, chg = t.ita(par, c["vel"].numpy(), 1000, tol)
    _say("  ITA to %.0e: GPU %d updates (change %.2e), oracle %d (%.2e)" % (tol, n, chg, n_o, chg_o))
    assert abs(n - n_o) <= 1 and n < 1000 and chg < tol
    assert float((ff.cpu() - fo).abs().max()) <= 1e-10 * float(fo.abs().max())
    # dense: (1 - M) F = tau v is singular (M 1 = 1); time reversal makes W
    # invariant under k -> -k and v odd, and the odd solution is unique
    dense, _ = bte.ita_dense_odd(w, c["vel"], c["nq"], _partners(c["kk"], c["bb"], GRID))
    assert float((ff.cpu() - dense).abs().max()) <= 1e-10 * float(dense.abs().max())
    assert float((tau.cpu() - tau_o).abs().max()) <= 1e-10 * float(tau_o.abs().max())
    mob_o = bte.mobility(c["eps"], c["vel"], dense, mu=c["mu"], temp=T)
    assert float((mob.cpu() - mob_o).abs().max()) <= 1e-10 * float(mob_o.abs().max())
    f0, _, _, n0, c0 = t.ita(par, c["vel"].numpy(), 0, tol)
    assert n0 == 0 and c0 == -1.0
    assert float((f0.cpu() - tau_o[:, None] * c["vel"]).abs().max()) <= 1e-10 * float(f0.abs().max())
    f3, _, _, n3, c3 = t.ita(par, c["vel"].numpy(), 3, tol)
    f3o, _ = bte.ita(w, c["vel"], c["nq"], 3)
    assert n3 == 3 and c3 >= tol
    assert float((f3.cpu() - f3o).abs().max()) <= 1e-10 * float(f3o.abs().max())


@pytest.mark.parametrize("prec", ["fp32", "fp16x3", "bf16x6", "bf16x3"])
def test_polar_mobility_reduced_precision(lib, polar, prec):
    """Mobility (Eq. cond) from a reduced-precision table against the FP64
    oracle's converged value, per diagonal component (contract 1e-4).  The
    table's rounding breaks the exact k -> -k symmetry at its precision, so
    the run takes the FP64 run's number of updates rather than a threshold
    below that level."""
    c = polar
    par = lib.Params(temp=T, mu=c["mu"], sigma=SIG, n_q=c["nq"])
    fo, _, n_o, _ = bte.ita_converged(_oracle_w(c), c["vel"], c["nq"], 1000, 1e-12)
    mob_o = bte.mobility(c["eps"], c["vel"], fo, mu=c["mu"], temp=T)
    t = lib.PairTable(c["dm"], GRID, c["kk"], c["bb"], precision=prec)
    _, _, mob = t.mobility(par, c["vel"].numpy(), n_o)
    d_o = torch.diagonal(mob_o)
    err = float(((torch.diagonal(mob.cpu()) - d_o).abs() / d_o.abs()).max())
    _say("  mobility error %s vs FP64 oracle: %.3e (mu_xx %.6e)" % (prec, err, float(mob[0, 0])))
    assert err <= 1e-4


def test_polar_mobility_vjp(lib, polar):
    """d mu / d g(Re,Rp) through the polar table (the Froehlich term is part of
    the recomputed g): oracle autograd 1e-10; GPU central difference 1e-6."""
    c = polar
    kw = dict(mu=c["mu"], temp=T, sigma=SIG, n_q=c["nq"], n_iter=4, polar=POL)
    lam = np.random.default_rng(91).standard_normal((3, 3))
    _say("polar mobility adjoint vs oracle autograd, S=%d" % len(c["kk"]))
    _, g_ref = grad.mobility_grad_g(c["m"], GRID, c["kk"], c["bb"], c["vel"], lam, **kw)
    par = lib.Params(temp=T, mu=c["mu"], sigma=SIG, n_q=c["nq"])
    t = lib.PairTable(c["dm"], GRID, c["kk"], c["bb"], precision="fp64")
    g_bar = t.mobility_vjp(par, c["vel"].numpy(), 4, lam).cpu()
    err = float((g_bar - g_ref).abs().max() / g_ref.abs().max())
    _say("  max rel err %.2e" % err)
    assert err <= 1e-10
    rng = np.random.default_rng(92)
    d = rng.standard_normal(c["m"].g.shape) + 1j * rng.standard_normal(c["m"].g.shape)
    h = 2e-6          # the central difference's own error is O(h^2): 8e-7 at h = 1e-5
    vals = []
    for sgn in (1.0, -1.0):
        mm = dataclasses.replace(c["m"], g=c["m"].g + sgn * h * d)
        tt = lib.PairTable(lib.Model(mm, polar=POL), GRID, c["kk"], c["bb"], precision="fp64")
        _, _, mob = tt.mobility(par, c["vel"].numpy(), 4)
        vals.append(float((mob.cpu() * torch.as_tensor(lam)).sum()))
    fd = (vals[0] - vals[1]) / (2 * h)
    ad = float((g_bar.conj() * torch.as_tensor(d)).real.sum())
    _say("  fd %.10e adjoint %.10e" % (fd, ad))
    assert abs(fd - ad) <= 1e-6 * abs(ad)


def test_autograd_functions_use_the_g_they_are_given(lib, polar):
    """RatesFunction and MobilityFunction load the g they receive: doubling g
    multiplies the rates by 4 and changes the mobility to that of a model
    created with 2g; the gradients are the adjoints at that g."""
    c = polar
    m = c["m"]
    dm = lib.Model(m, polar=POL)
    k = synth.random_points(93, 3)
    q = synth.random_points(94, 40)
    p = lib.Params(temp=T, mu=0.0, sigma=0.05)
    g1 = torch.as_tensor(m.g, dtype=torch.complex128, device="cuda")
    g2 = (2.0 * g1).requires_grad_(True)
    m2 = dataclasses.replace(m, g=2.0 * m.g)
    dm2 = lib.Model(m2, polar=POL)
    ref2, _ = lib.rates(dm2, k, q, p, mode_resolved=False)
    gam2 = lib.RatesFunction.apply(g2, dm, k, q, p)
    assert float((gam2.detach() - ref2).abs().max()) <= 1e-12 * float(ref2.abs().max())
    lam = torch.as_tensor(np.random.default_rng(95).random((3, m.nw)), device="cuda")
    (gam2 * lam).sum().backward()
    vjp2 = lib.rates_vjp(dm2, k, q, p, lam)
    assert float((g2.grad - vjp2).abs().max()) <= 1e-12 * float(vjp2.abs().max())
    # the model now holds 2g: the rates without the Function see it
    gam_now, _ = lib.rates(dm, k, q, p, mode_resolved=False)
    assert float((gam_now - ref2).abs().max()) <= 1e-12 * float(ref2.abs().max())
    # the fp16 scale follows the values: FP16x3 rates of 2g vs FP64
    g16, _ = lib.rates(dm, k, q, p, precision="fp16x3", mode_resolved=False)
    assert float(((g16 - ref2).abs() / ref2.abs().clamp_min(1e-6 * float(ref2.abs().max()))).max()) <= 1e-4
    # mobility from the g given
    par = lib.Params(temp=T, mu=c["mu"], sigma=SIG, n_q=c["nq"])
    mob = lib.MobilityFunction.apply(g2.detach().clone().requires_grad_(True), dm, GRID, c["kk"], c["bb"], par,
                                     c["vel"].numpy(), 3)
    t2 = lib.PairTable(dm2, GRID, c["kk"], c["bb"], precision="fp64")
    _, _, mob_ref = t2.mobility(par, c["vel"].numpy(), 3)
    assert float((mob.detach() - mob_ref).abs().max()) <= 1e-12 * float(mob_ref.abs().max())
    # a non-finite g is refused and the model keeps its values
    bad = g1.clone()
    bad[0, 0, 0, 0, 0] = float("nan")
    with pytest.raises(lib.EphxError):
        dm.set_g(bad)
    gam_after, _ = lib.rates(dm, k, q, p, mode_resolved=False)
    assert torch.equal(gam_after, gam_now)
