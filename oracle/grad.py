"""Oracle gradients by PyTorch autograd through the plain FP64 oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Complex convention: the gradient of a real loss L with respect to a complex
array z is returned as dL/dRe(z) + i dL/dIm(z) (PyTorch's convention; for
L = |z|^2 it gives 2z).
"""
from __future__ import annotations

import copy

import numpy as np
import torch

from . import bte, eph
from .interp import t64


def rates_grad_g(model, k, q, lam, **rate_kw):
    """dL/dg(Re,Rp) for L = sum_nk lam_nk Gamma_nk (Eq. scatter_rate); the
    eigenvectors of H and D do not depend on g, so only the linear chain
    g(Re,Rp) -> g^W -> g^H -> g_mn,nu -> |g|^2 -> Gamma is differentiated."""
    m = copy.copy(model)
    gt = torch.as_tensor(model.g, dtype=torch.complex128).clone().requires_grad_(True)
    m.g = gt
    gamma, _ = eph.rates(m, k, q, **rate_kw)
    loss = (gamma * t64(lam)).sum()
    loss.backward()
    return float(loss.detach()), gt.grad


def mobility_of(model, n_grid, k_idx, band, vel, *, mu, temp, sigma, n_q, n_iter, omega_cut=1e-4, polar=None):
    """Mobility tensor (Eq. cond over e n_c) after n_iter iterations of the
    linearised BTE (Eqs. BTE_W, BTE_iter) on the symmetrised pair table of the
    given grid states; differentiable in model.g."""
    g2s, om = bte.pair_table(model, n_grid, k_idx, band, omega_cut=omega_cut, polar=polar)
    eps = bte.state_energies(model, k_idx, band, n_grid)
    w = bte.transport_matrix(eps, g2s, om, temp=temp, mu=mu, sigma=sigma, omega_cut=omega_cut)
    ff, _ = bte.ita(w, vel, n_q, n_iter)
    return bte.mobility(eps, vel, ff, mu=mu, temp=temp)


def mobility_grad_g(model, n_grid, k_idx, band, vel, lam, **kw):
    """dL/dg(Re,Rp) for L = sum_ab lam_ab mu_ab with mu from mobility_of: the
    chain g -> |g|^2 table -> W -> (tau, F) -> mu, by autograd."""
    m = copy.copy(model)
    gt = torch.as_tensor(model.g, dtype=torch.complex128).clone().requires_grad_(True)
    m.g = gt
    mob = mobility_of(m, n_grid, k_idx, band, vel, **kw)
    loss = (mob * t64(lam)).sum()
    loss.backward()
    return float(loss.detach()), gt.grad


def dynamics_mean_energy(f0, eps, g2s, omega, mode_scale, *, dt, n_steps, e_ref, **coll_kw):
    """Mean carrier energy sum_s (eps_s - e_ref) f_s / sum_s f_s after n_steps RK4
    steps of df/dt = I[f] (Eq. BTE_E with E = 0)."""
    rhs = lambda x: bte.collision(x, eps, g2s, omega, mode_scale=mode_scale, **coll_kw)
    f = bte.integrate(f0, dt, n_steps, rhs)
    e = t64(eps) - e_ref
    return (e * f).sum() / f.sum()


def dynamics_grad(f0, eps, g2s, omega, *, dt, n_steps, e_ref, **coll_kw):
    """(E, dE/df0, dE/ds_nu at s_nu = 1) for the mean energy above."""
    f0t = t64(f0).clone().requires_grad_(True)
    s = torch.ones(g2s.shape[-1], dtype=torch.float64, requires_grad=True)
    e = dynamics_mean_energy(f0t, eps, g2s, omega, s, dt=dt, n_steps=n_steps, e_ref=e_ref, **coll_kw)
    e.backward()
    return float(e.detach()), f0t.grad, s.grad
