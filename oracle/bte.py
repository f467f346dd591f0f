"""Boltzmann-equation work on grid states (paper Sec. 2.1): the stored |g|^2
pair table, the e-ph collision integral, RK4 time stepping, the iterative
linearised BTE and the mobility.

TEST INFRASTRUCTURE ONLY (see the package docstring).

States s = (k_s, n_s) live on a Gamma-centred grid; the transition s -> t
absorbs or emits a phonon of wavevector q = k_t - k_s (Sec. 4.3).
"""
from __future__ import annotations

import numpy as np
import torch

from .eph import eph_pipeline
from .grid import grid_coords
from .interp import F64, bands, bose, fermi, gauss_delta, t64
from .units import HBAR_EV_FS, KB_EV, TWO_PI


def state_points(k_idx, n_grid):
    return grid_coords(k_idx, n_grid) / np.asarray(n_grid, dtype=np.float64)


def state_energies(model, k_idx, band, n_grid):
    eps, _ = bands(model, state_points(k_idx, n_grid))
    return eps[torch.arange(len(band)), torch.as_tensor(band)]


def pair_table(model, n_grid, k_idx, band, *, omega_cut=1e-4, polar=None):
    """|g|^2 of every ordered pair of states and the phonon energies of its q.

    Returns (g2s, omega) of shape (S, S, nmodes):
      g2s[s,t,nu]   = 1/2 (|g_{n_t n_s nu}(k_s, k_t-k_s)|^2 + |g_{n_s n_t nu}(k_t, k_s-k_t)|^2)
      omega[s,t,nu] = hbar omega_nu(k_t - k_s)
    The symmetrisation makes |g(s->t)|^2 = |g(t->s)|^2, which carrier-number
    conservation of the collision integral needs and which a synthetic
    g(Re,Rp) does not satisfy by itself."""
    n_grid = np.asarray(n_grid)
    ks = state_points(k_idx, n_grid)
    cs = grid_coords(k_idx, n_grid)
    S = len(k_idx)
    nm = model.nmodes
    raw = torch.zeros((S, S, nm), dtype=F64)
    om = torch.zeros((S, S, nm), dtype=F64)
    bt = torch.as_tensor(band)
    for s in range(S):
        q = ((cs - cs[s]) % n_grid) / n_grid                 # q for every target t
        blk = eph_pipeline(model, ks[s:s + 1], q, polar, omega_cut)
        g = blk["g"][0]                                      # (t, nu, m, n)
        raw[s] = g[torch.arange(S), :, bt, int(band[s])].abs() ** 2
        om[s] = blk["omega"]
    return 0.5 * (raw + raw.transpose(0, 1)), om


def pair_entries(model, n_grid, k_idx, band, pairs, *, omega_cut=1e-4, polar=None):
    """Entries of `pair_table` at the listed ordered pairs (s, t) only, each
    evaluated from its definition (for sampling tables too large to build
    here).  Returns (g2s [P, nmodes], omega [P, nmodes])."""
    n_grid = np.asarray(n_grid)
    ks = state_points(k_idx, n_grid)
    cs = grid_coords(k_idx, n_grid)
    nm = model.nmodes
    g2s = torch.zeros((len(pairs), nm), dtype=F64)
    om = torch.zeros((len(pairs), nm), dtype=F64)
    for i, (s, t) in enumerate(pairs):
        q_st = ((cs[t] - cs[s]) % n_grid) / n_grid
        q_ts = ((cs[s] - cs[t]) % n_grid) / n_grid
        a = eph_pipeline(model, ks[s:s + 1], q_st[None], polar, omega_cut)
        b = eph_pipeline(model, ks[t:t + 1], q_ts[None], polar, omega_cut)
        g_st = a["g"][0, 0, :, int(band[t]), int(band[s])].abs() ** 2
        g_ts = b["g"][0, 0, :, int(band[s]), int(band[t])].abs() ** 2
        g2s[i] = 0.5 * (g_st + g_ts)
        om[i] = a["omega"][0]
    return g2s, om


def collision(f, eps, g2s, omega, *, temp, sigma, n_q, omega_cut=1e-4, mode_scale=None):
    """e-ph collision integral, Eq. e_ph_scattering with F_abs and F_em:

      I_s = -(2 pi/hbar)(1/N_q) sum_{t,nu} s_nu |g|^2 [ delta(eps_s - hw - eps_t) F_em
                                                       + delta(eps_s + hw - eps_t) F_abs ]
      F_abs = f_s(1-f_t) N - f_t(1-f_s)(N+1),   F_em = f_s(1-f_t)(N+1) - f_t(1-f_s) N

    N = Bose-Einstein occupations at the (fixed) phonon temperature; modes with
    omega <= omega_cut contribute nothing.  Returns I in 1/fs.  Works with
    autograd in f and mode_scale."""
    f = t64(f) if not torch.is_tensor(f) else f
    eps = t64(eps)
    nb = bose(omega, temp, omega_cut)
    fs = f[:, None, None]
    ft = f[None, :, None]
    f_abs = fs * (1 - ft) * nb - ft * (1 - fs) * (nb + 1)
    f_em = fs * (1 - ft) * (nb + 1) - ft * (1 - fs) * nb
    d = eps[:, None, None] - eps[None, :, None]
    keep = omega > omega_cut
    term = g2s * (gauss_delta(d - omega, sigma) * f_em + gauss_delta(d + omega, sigma) * f_abs)
    term = torch.where(keep, term, torch.zeros_like(term))
    if mode_scale is not None:
        term = term * mode_scale[None, None, :]
    return -(TWO_PI / HBAR_EV_FS) / n_q * term.sum(dim=(1, 2))


def collision_rows(rows, f, eps, g2_rows, omega_rows, *, temp, sigma, n_q, omega_cut=1e-4, mode_scale=None):
    """The entries `rows` of the collision integral of `collision` (Eq.
    e_ph_scattering), from those rows of the table alone: g2_rows and
    omega_rows are (len(rows), S, nmodes), the rows s of g2s and omega.  For
    tables too large to hold whole; the terms are those of `collision`."""
    f = t64(f)
    eps = t64(eps)
    rows = torch.as_tensor(np.asarray(rows), dtype=torch.long)
    g2_rows, omega_rows = t64(g2_rows), t64(omega_rows)
    nb = bose(omega_rows, temp, omega_cut)
    fs = f[rows][:, None, None]
    ft = f[None, :, None]
    f_abs = fs * (1 - ft) * nb - ft * (1 - fs) * (nb + 1)
    f_em = fs * (1 - ft) * (nb + 1) - ft * (1 - fs) * nb
    d = eps[rows][:, None, None] - eps[None, :, None]
    term = g2_rows * (gauss_delta(d - omega_rows, sigma) * f_em + gauss_delta(d + omega_rows, sigma) * f_abs)
    term = torch.where(omega_rows > omega_cut, term, torch.zeros_like(term))
    if mode_scale is not None:
        term = term * t64(mode_scale)[None, None, :]
    return -(TWO_PI / HBAR_EV_FS) / n_q * term.sum(dim=(1, 2))


def rk4_step(f, dt, rhs):
    """Classic four-stage Runge-Kutta step (the paper's default integrator)."""
    k1 = rhs(f)
    k2 = rhs(f + 0.5 * dt * k1)
    k3 = rhs(f + 0.5 * dt * k2)
    k4 = rhs(f + dt * k3)
    return f + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


def euler_step(f, dt, rhs):
    return f + dt * rhs(f)


def integrate(f0, dt, n_steps, rhs, step=rk4_step, keep_every=0):
    f = f0
    saved = [f0] if keep_every else []
    for i in range(n_steps):
        f = step(f, dt, rhs)
        if keep_every and (i + 1) % keep_every == 0:
            saved.append(f)
    return (f, saved) if keep_every else f


# ---------------------------------------------------------------- transport

def transport_matrix(eps, g2s, omega, *, temp, mu, sigma, omega_cut=1e-4):
    """Scattering probabilities W_{s,t} of Eq. BTE_W between grid states with
    equilibrium occupations f0 = Fermi-Dirac(mu, T), summed over modes (1/fs):
      W_st = (2 pi/hbar) sum_nu |g|^2 [ delta(eps_s - hw - eps_t)(1 + N - f0_t)
                                       + delta(eps_s + hw - eps_t)(N + f0_t) ]"""
    eps = t64(eps)
    nb = bose(omega, temp, omega_cut)
    f0 = fermi(eps, mu, temp)[None, :, None]
    d = eps[:, None, None] - eps[None, :, None]
    w = g2s * (gauss_delta(d - omega, sigma) * (1 + nb - f0) + gauss_delta(d + omega, sigma) * (nb + f0))
    w = torch.where(omega > omega_cut, w, torch.zeros_like(w))
    return (TWO_PI / HBAR_EV_FS) * w.sum(dim=2)


def ita(w, vel, n_q, n_iter, gamma=None):
    """Iterative solution of the linearised BTE (Eqs. BTE_lin, BTE_iter):
      Gamma_s = (1/N_q) sum_t W_st (unless given),  tau = 1/Gamma,  F^0 = tau v,
      F^{i+1} = F^0 + (tau/N_q) sum_t W_st F^i_t.
    n_iter = 0 gives the RTA.  Returns (F (S,3), tau (S,)).

    When Gamma is the row sum of the same W, (tau/N_q) W is row-stochastic and
    the iteration converges only on the subspace that excludes its unit
    eigenvector, e.g. for inversion-symmetric models where F^0 = tau v is odd."""
    w = t64(w)
    vel = t64(vel)
    if gamma is None:
        gamma = w.sum(dim=1) / n_q
    tau = 1.0 / gamma
    f0 = tau[:, None] * vel
    f = f0
    for _ in range(n_iter):
        f = f0 + (tau / n_q)[:, None] * (w @ f)
    return f, tau


def ita_converged(w, vel, n_q, n_iter_max, tol, gamma=None):
    """The iteration of `ita` run until F stops changing (Eq. BTE_iter): after
    each update F^{i+1}, stop if max_{s,a} |F^{i+1} - F^i| < tol max_{s,a} |F^{i+1}|,
    and in any case after n_iter_max updates.  Returns (F, tau, number of updates,
    relative change of the last update; -1 if none was made)."""
    w = t64(w)
    vel = t64(vel)
    if gamma is None:
        gamma = w.sum(dim=1) / n_q
    tau = 1.0 / gamma
    f0 = tau[:, None] * vel
    f = f0
    change = -1.0
    n = 0
    for i in range(n_iter_max):
        fn = f0 + (tau / n_q)[:, None] * (w @ f)
        amax = float(fn.abs().max())
        change = float((fn - f).abs().max()) / amax if amax > 0 else 0.0
        f = fn
        n = i + 1
        if change < tol:
            break
    return f, tau, n, change


def ita_dense_odd(w, vel, n_q, partner, gamma=None):
    """The fixed point of Eq. BTE_iter, F = tau v + (tau/N_q) W F, by a dense
    solve on the odd vectors, F_partner[s] = -F_s, where partner[s] is the state
    at -k_s with the same band (a permutation, partner[s] = s at k = -k).  When
    W and tau are invariant under s -> partner[s] and v is odd, the iteration
    stays among odd vectors and converges there, even though (1 - diag(tau/N_q)
    W) itself is singular (its rows sum to zero, more than once if the states
    fall into groups that do not scatter into each other).  Returns (F, tau)."""
    w = t64(w)
    vel = t64(vel)
    partner = np.asarray(partner)
    if gamma is None:
        gamma = w.sum(dim=1) / n_q
    tau = 1.0 / gamma
    m = (tau / n_q)[:, None] * w
    rep = np.array([s for s in range(len(partner)) if s < partner[s]], dtype=np.int64)
    # F on the representatives x; F[partner[rep]] = -x; F = 0 where partner[s] = s
    a = torch.eye(len(rep), dtype=F64) - (m[rep][:, rep] - m[rep][:, partner[rep]])
    x = torch.linalg.solve(a, tau[rep, None] * vel[rep])
    f = torch.zeros_like(vel)
    f[rep] = x
    f[partner[rep]] = -x
    return f, tau


def mobility(eps, vel, ff, *, mu, temp):
    """Mobility tensor mu_ab = sigma_ab / (e n_c) with sigma from Eq. cond and
    n_c = (S/(N_k Omega)) sum f0 over the same states; the prefactors cancel:
      mu_ab = e sum_s v^a F^b (-df0/deps) / sum_s f0.
    With v in Angstrom/fs, F in Angstrom and energies in eV the value is in
    Angstrom^2/(V fs) = 0.1 cm^2/(V s); returned in cm^2/(V s)."""
    eps = t64(eps)
    f0 = fermi(eps, mu, temp)
    mdf = f0 * (1 - f0) / (KB_EV * temp)
    num = torch.einsum("sa,sb,s->ab", t64(vel), t64(ff), mdf)
    return 0.1 * num / f0.sum()


def carrier_density(eps, mu, temp, n_k, omega_cell, spin=2.0):
    """n_c = (S/(N_k Omega)) sum_s f0_s, in cm^-3 (Omega in Angstrom^3)."""
    return spin / (n_k * omega_cell) * float(fermi(eps, mu, temp).sum()) * 1e24


def chemical_potential(eps, n_c, temp, n_k, omega_cell, spin=2.0, lo=-10.0, hi=10.0, iters=200):
    """Bisection for the mu that gives carrier density n_c (cm^-3)."""
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if carrier_density(eps, mid, temp, n_k, omega_cell, spin) < n_c:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)
