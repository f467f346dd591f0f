"""Pins of the oracle gradients (autograd through the FP64 oracle) against
central finite differences of the oracle's forward values."""
import copy

import numpy as np
import torch

import synth
from oracle import bte, eph, grad, grid, interp


def test_rates_gradient_wrt_g_matches_finite_differences(tiny_model):
    k = synth.random_points(50, 2)
    q = synth.random_points(51, 6)
    lam = np.random.default_rng(52).random((2, tiny_model.nw))
    kw = dict(temp=300.0, mu=0.0, sigma=0.08)
    loss, g_bar = grad.rates_grad_g(tiny_model, k, q, lam, **kw)
    rng = np.random.default_rng(53)
    h = 1e-6
    for _ in range(6):
        idx = tuple(int(rng.integers(0, s)) for s in tiny_model.g.shape)
        for part, unit in (("re", 1.0), ("im", 1j)):
            mp = copy.deepcopy(tiny_model)
            mm = copy.deepcopy(tiny_model)
            mp.g[idx] += h * unit
            mm.g[idx] -= h * unit
            lp = float((eph.rates(mp, k, q, **kw)[0] * torch.as_tensor(lam)).sum())
            lm = float((eph.rates(mm, k, q, **kw)[0] * torch.as_tensor(lam)).sum())
            fd = (lp - lm) / (2 * h)
            ad = float(g_bar[idx].real if part == "re" else g_bar[idx].imag)
            assert abs(fd - ad) <= 1e-6 * max(abs(ad), 1e-3 * float(g_bar.abs().max()))


def test_dynamics_gradient_matches_finite_differences():
    rng = np.random.default_rng(54)
    s, nm = 16, 3
    eps = torch.as_tensor(np.sort(rng.random(s) * 0.25))
    g2s = torch.as_tensor(rng.random((s, s, nm)))
    g2s = 0.5 * (g2s + g2s.transpose(0, 1))
    om = torch.as_tensor(0.01 + 0.05 * rng.random((s, s, nm)))
    om = 0.5 * (om + om.transpose(0, 1))
    f0 = torch.as_tensor(0.1 * rng.random(s))
    kw = dict(dt=1.0, n_steps=15, e_ref=0.0, temp=300.0, sigma=0.01, n_q=2000.0)
    e, df0, ds = grad.dynamics_grad(f0, eps, g2s, om, **kw)
    h = 1e-6
    for i in (0, 5, 11):
        fp, fm = f0.clone(), f0.clone()
        fp[i] += h
        fm[i] -= h
        ep = float(grad.dynamics_mean_energy(fp, eps, g2s, om, torch.ones(nm, dtype=torch.float64), **kw))
        em = float(grad.dynamics_mean_energy(fm, eps, g2s, om, torch.ones(nm, dtype=torch.float64), **kw))
        assert abs((ep - em) / (2 * h) - float(df0[i])) <= 1e-6 * float(df0.abs().max())
    for nu in range(nm):
        sp = torch.ones(nm, dtype=torch.float64)
        sm = sp.clone()
        sp[nu] += h
        sm[nu] -= h
        ep = float(grad.dynamics_mean_energy(f0, eps, g2s, om, sp, **kw))
        em = float(grad.dynamics_mean_energy(f0, eps, g2s, om, sm, **kw))
        assert abs((ep - em) / (2 * h) - float(ds[nu])) <= 1e-6 * float(ds.abs().max())


def _mobility_case():
    m = synth.make_config_model("tiny", real=True)
    n = (4, 4, 4)
    eps_g, _ = interp.bands(m, grid.grid_points(n))
    cbm = float(eps_g[:, m.nw // 2].min())
    kk, bb = grid.window_states(eps_g.numpy(), m.nw // 2, m.nw, cbm - 0.01, cbm + 1.0)
    _, _, v = interp.bands(m, bte.state_points(kk, n), velocity=True)
    vel = v[torch.arange(len(bb)), torch.as_tensor(bb)]
    kw = dict(mu=cbm - 0.3, temp=300.0, sigma=0.1, n_q=float(np.prod(n)), n_iter=3)
    return m, n, kk, bb, vel, kw


def test_mobility_gradient_wrt_g_matches_finite_differences():
    m, n, kk, bb, vel, kw = _mobility_case()
    assert len(kk) >= 8
    lam = np.random.default_rng(55).standard_normal((3, 3))
    loss, g_bar = grad.mobility_grad_g(m, n, kk, bb, vel, lam, **kw)
    assert np.isfinite(loss) and float(g_bar.abs().max()) > 0
    rng = np.random.default_rng(56)
    h = 1e-6
    # random directions over the whole tensor and single entries
    dirs = [rng.standard_normal(m.g.shape) + 1j * rng.standard_normal(m.g.shape) for _ in range(2)]
    for _ in range(3):
        d = np.zeros(m.g.shape, dtype=np.complex128)
        d[tuple(int(rng.integers(0, s)) for s in m.g.shape)] = 1.0 if rng.random() < 0.5 else 1j
        dirs.append(d)
    for d in dirs:
        mp = copy.deepcopy(m)
        mm = copy.deepcopy(m)
        mp.g = m.g + h * d
        mm.g = m.g - h * d
        lp = float((grad.mobility_of(mp, n, kk, bb, vel, **kw) * torch.as_tensor(lam)).sum())
        lm = float((grad.mobility_of(mm, n, kk, bb, vel, **kw) * torch.as_tensor(lam)).sum())
        fd = (lp - lm) / (2 * h)
        ad = float((g_bar.conj() * torch.as_tensor(d)).real.sum())
        assert abs(fd - ad) <= 1e-6 * max(abs(ad), 1e-3 * float(g_bar.abs().sum()))
