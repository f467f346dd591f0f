"""Wannier interpolation of the e-ph matrix elements and scattering rates
(paper Sec. 2.2.3, 2.3 and Eqs. scatter_rate / BTE_W).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Array layouts (shared with the library only as a documented convention):
  g^W, g^H : (nk, nq, nmodes[kappa alpha], nw[i or m], nw[j or n])
  |g|^2    : (nk, nq, nmodes[nu], nw[m, final band at k+q], nw[n, initial band at k])
"""
from __future__ import annotations

import copy
import math

import torch

from .interp import C128, F64, bands, bose, fermi, gauss_delta, phases, phonons, t64
from .units import E2_4PIEPS0, HBAR2_AMU_A2, HBAR_EV_FS, TWO_PI


def _g(model):
    return torch.as_tensor(model.g, dtype=C128)


def g_wannier_direct(model, k, q):
    """Literal double sum of Eq. eph_mat_wann2 (inner part), term by term over
    every (Re, Rp) pair: sum_{Re,Rp} e^{i(k.Re + q.Rp)} g(Re,Rp).  Tiny inputs
    only."""
    k, q = t64(k), t64(q)
    g = _g(model)
    we, wp = t64(model.w_re_g), t64(model.w_rp_g)
    out = torch.zeros((k.shape[0], q.shape[0]) + tuple(g.shape[2:]), dtype=C128)
    for a in range(k.shape[0]):
        for b in range(q.shape[0]):
            acc = torch.zeros(g.shape[2:], dtype=C128)
            for e in range(g.shape[0]):
                pe = phases(k[a:a + 1], model.re_g[e:e + 1])[0, 0] * we[e]
                for p in range(g.shape[1]):
                    pp = phases(q[b:b + 1], model.rp_g[p:p + 1])[0, 0] * wp[p]
                    acc += pe * pp * g[e, p]
            out[a, b] = acc
    return out


def g_k_rp(model, k):
    """First factor of Eq. eph_mat_wann2: g(k,Rp) = sum_Re e^{ik.Re} g(Re,Rp)."""
    p = phases(k, model.re_g) * t64(model.w_re_g)
    return torch.einsum("ke,epxij->kpxij", p, _g(model))


def g_wannier(model, k, q, gk=None):
    """Factored form: g^W(k,q) = sum_Rp e^{iq.Rp} g(k,Rp)."""
    if gk is None:
        gk = g_k_rp(model, k)
    p = phases(q, model.rp_g) * t64(model.w_rp_g)
    return torch.einsum("qp,kpxij->kqxij", p, gk)


def frohlich(model, q, alpha_ewald, gcut):
    """Long-range (Froehlich) coupling in the Wannier gauge, Eq. e_ph_long with
    the smooth-phase bra-ket of Eq. smooth_phase (delta_ij in the Wannier gauge):

      C^{kappa a}(q) = i e^2/(eps0 Omega) sum_{G, q+G != 0, |q+G| < gcut}
            [(q+G).Z*_kappa]_a e^{-i tau_kappa.(q+G)} e^{-(q+G).eps.(q+G)/(4 Lambda)}
            / ((q+G).eps.(q+G))

    The sum runs over q+G, so q is first brought to [-1/2,1/2)^3 (a relabelling
    of G).  Returns (nq, 3 nat) complex, in eV/Angstrom."""
    q = t64(q)
    lat = t64(model.lattice)
    bvec = TWO_PI * torch.linalg.inv(lat).T                   # rows b_i
    zs = t64(model.zstar)                                     # (nat, beta, alpha)
    eps = t64(model.eps_inf)
    tau = t64(model.tau)
    omega_cell = abs(float(torch.linalg.det(lat)))
    pref = 4.0 * math.pi * E2_4PIEPS0 / omega_cell            # e^2/(eps0 Omega)
    qr = q - torch.round(q)
    mmax = int(math.ceil((gcut + float(torch.linalg.norm(bvec, dim=1).sum())) *
                         float(torch.linalg.norm(lat, dim=1).max()) / TWO_PI)) + 1
    rng = torch.arange(-mmax, mmax + 1, dtype=F64)
    mgrid = torch.stack(torch.meshgrid(rng, rng, rng, indexing="ij"), -1).reshape(-1, 3)
    gvec = mgrid @ bvec                                       # (nG,3)
    nat = tau.shape[0]
    out = torch.zeros((q.shape[0], 3 * nat), dtype=C128)
    for iq in range(q.shape[0]):
        qg = (qr[iq] @ bvec)[None, :] + gvec                  # (nG,3)
        norm = torch.linalg.norm(qg, dim=1)
        keep = (norm < gcut) & (norm > 1e-12)
        qg = qg[keep]
        qeq = torch.einsum("ga,ab,gb->g", qg, eps, qg)
        damp = torch.exp(-qeq / (4.0 * alpha_ewald)) / qeq
        for kap in range(nat):
            qz = qg @ zs[kap]                                 # [(q+G).Z*]_a
            ph = torch.polar(torch.ones_like(qeq), -(qg @ tau[kap]))
            out[iq, 3 * kap:3 * kap + 3] = 1j * pref * torch.einsum(
                "g,ga->a", (damp * ph), qz.to(C128))
    return out


def band_basis(gw, u_kq, u_k):
    """Rotation of Eq. eph_mat_wann2: g^H = U^dag(k+q) g^W U(k).
    u_kq: (nk,nq,nw,nw), u_k: (nk,nw,nw)."""
    return torch.einsum("kqim,kqxij,kjn->kqxmn", u_kq.conj(), gw, u_k)


def mode_project(gh, omega, evec, mass, omega_cut):
    """Mode projection of Eq. eph_mat:
       g_mn,nu = sqrt(hbar/(2 omega_nu)) sum_{kappa a} e^{kappa a}_nu / sqrt(M_kappa) g^{kappa a}_mn
    (e not conjugated).  Modes with omega <= omega_cut are set to zero.
    omega: (nq,nm) eV, evec: (nq,nm,nm) columns; returns (nk,nq,nu,m,n)."""
    m = t64(mass).repeat_interleave(3)
    keep = omega > omega_cut
    safe = torch.where(keep, omega, torch.ones_like(omega))
    amp = torch.where(keep, torch.sqrt(HBAR2_AMU_A2 / (2.0 * safe)), torch.zeros_like(omega))
    e_scaled = evec / torch.sqrt(m)[None, :, None]
    g = torch.einsum("qxv,kqxmn->kqvmn", e_scaled, gh)
    return g * amp[None, :, :, None, None].to(C128)


def eph_pipeline(model, k, q, polar=None, omega_cut=1e-4):
    """All quantities of one (k-list x q-list) block: returns a dict with eps_k
    (nk,nw), eps_kq (nk,nq,nw), omega (nq,nm), g (nk,nq,nu,m,n) complex."""
    k, q = t64(k), t64(q)
    nk, nq = k.shape[0], q.shape[0]
    eps_k, u_k = bands(model, k)
    kq = (k[:, None, :] + q[None, :, :]).reshape(-1, 3)
    eps_kq, u_kq = bands(model, kq)
    nw = model.nw
    eps_kq = eps_kq.reshape(nk, nq, nw)
    u_kq = u_kq.reshape(nk, nq, nw, nw)
    # polar = dict(alpha_ewald, gcut[, lo_to]): the Froehlich term, and with
    # lo_to the dipole-dipole part of D(q) as well
    ew = None if polar is None else dict(alpha_ewald=polar["alpha_ewald"], gcut=polar["gcut"])
    omega, evec = phonons(model, q, dipole=ew if polar is not None and polar.get("lo_to") else None)
    gw = g_wannier(model, k, q)
    if polar is not None:
        lr = frohlich(model, q, **ew)                            # (nq, nm)
        eye = torch.eye(nw, dtype=C128)
        gw = gw + lr[None, :, :, None, None] * eye
    gh = band_basis(gw, u_kq, u_k)
    g = mode_project(gh, omega, evec, model.mass, omega_cut)
    return dict(eps_k=eps_k, eps_kq=eps_kq, omega=omega, evec=evec, g=g, u_k=u_k, u_kq=u_kq)


def g2(model, k, q, polar=None, omega_cut=1e-4):
    """|g_mn,nu(k,q)|^2 in eV^2, layout (nk, nq, nu, m, n)."""
    return eph_pipeline(model, k, q, polar, omega_cut)["g"].abs() ** 2


def g_abs_modes(g2v):
    """Gauge-invariant |g_nu| = sqrt(sum_mn |g_mn,nu|^2 / N_b)  (Eq. g_abs)."""
    nb = g2v.shape[-1]
    return torch.sqrt(g2v.sum(dim=(-1, -2)) / nb)


def rates(model, k, q, *, temp, mu, sigma, omega_cut=1e-4, q_weights=None,
          polar=None, chunk=64, part="full"):
    """Scattering rates (Eq. scatter_rate with W of Eq. BTE_W), in 1/fs:

      Gamma_nk = sum_q w_q sum_{m,nu} (2 pi/hbar) |g_mn,nu(k,q)|^2
                 [ delta(eps_nk - hw - eps_mk+q)(1 + N - f_m) + delta(eps_nk + hw - eps_mk+q)(N + f_m) ]

    w_q = 1/N_q unless given.  Returns (gamma (nk,nw), gamma_mode (nk,nw,nm)).

    part (polar models): "full" uses |g|^2; "polar" the long-range coupling
    alone, |g_L|^2, with g_L the Froehlich term of Eq. e_ph_long taken through
    the same rotation and mode projection (the pipeline with g(Re,Rp) = 0);
    "rmpol" the rest, |g|^2 - |g_L|^2.  The rates are linear in |g|^2, so the
    two parts add up to the full rates for any q set, and each part's q sum
    can be estimated with its own sampling (the polar split of Sec. 5.2)."""
    if part not in ("full", "polar", "rmpol"):
        raise ValueError("part must be full, polar or rmpol")
    if part != "full" and polar is None:
        raise ValueError("the polar and rmpol parts need a polar model")
    k, q = t64(k), t64(q)
    nq = q.shape[0]
    w = torch.full((nq,), 1.0 / nq, dtype=F64) if q_weights is None else t64(q_weights)
    nk, nw, nm = k.shape[0], model.nw, model.nmodes
    gmode = torch.zeros((nk, nw, nm), dtype=F64)
    m_lr = None
    if part != "full":
        m_lr = copy.copy(model)
        m_lr.g = torch.zeros_like(torch.as_tensor(model.g, dtype=C128))
    for s in range(0, nq, chunk):
        blk = eph_pipeline(model, k, q[s:s + chunk], polar, omega_cut)
        gg = blk["g"].abs() ** 2                                  # (k,q,nu,m,n)
        if part != "full":
            gl = eph_pipeline(m_lr, k, q[s:s + chunk], polar, omega_cut)["g"].abs() ** 2
            gg = gl if part == "polar" else gg - gl
        om = blk["omega"]                                         # (q,nu)
        nb = bose(om, temp, omega_cut)
        fm = fermi(blk["eps_kq"], mu, temp)                       # (k,q,m)
        ek = blk["eps_k"][:, None, None, None, :]
        ekq = blk["eps_kq"][:, :, None, :, None]
        hw = om[None, :, :, None, None]
        nn = nb[None, :, :, None, None]
        ff = fm[:, :, None, :, None]
        term = (gauss_delta(ek - hw - ekq, sigma) * (1.0 + nn - ff)
                + gauss_delta(ek + hw - ekq, sigma) * (nn + ff))
        wgt = (TWO_PI / HBAR_EV_FS) * gg * term * w[s:s + chunk][None, :, None, None, None]
        gmode += wgt.sum(dim=(1, 3)).transpose(1, 2)              # sum q, m -> (k, n, nu)
    return gmode.sum(dim=2), gmode
