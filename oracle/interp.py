"""Band and phonon interpolation (paper Sec. 2.2.1 and 2.2.2).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import math

import torch

from .units import E2_4PIEPS0, HBAR_EV_FS, HBAR2_AMU_A2, KB_EV, SQRT_PI, TWO_PI

F64 = torch.float64
C128 = torch.complex128


def t64(x):
    return torch.as_tensor(x, dtype=F64)


def phases(x, n):
    """exp(i k.R) = exp(2 pi i x.n) for reduced points x (...,3) and integer
    vectors n (K,3).  The argument t = x.n is formed in FP64 and reduced to
    r = t - rint(t) before the exponential (phase convention of Eqs. wannier_3,
    IFC2 and eph_mat_wann2: e^{+ik.R})."""
    t = t64(x) @ t64(n).T
    r = t - torch.round(t)
    return torch.polar(torch.ones_like(r), TWO_PI * r)


# ---------------------------------------------------------------- electrons

def hamiltonian_k(model, k):
    """H^(W)(k) = sum_Re w_Re e^{ik.Re} H(Re)   (Eq. wannier_3)."""
    p = phases(k, model.re) * t64(model.w_re)
    return torch.einsum("kr,rij->kij", p, torch.as_tensor(model.h, dtype=C128))


def degenerate_groups(e, tol):
    """Consecutive runs of ascending eigenvalues closer than tol."""
    groups, start = [], 0
    for i in range(1, len(e) + 1):
        if i == len(e) or float(e[i] - e[i - 1]) >= tol:
            groups.append(list(range(start, i)))
            start = i
    return groups


def bands(model, k, velocity=False, deg_tol=1e-4):
    """Band energies eps_nk (eV, ascending), eigenvectors U(k) (columns, so that
    H^(W) = U diag(eps) U^dagger, Eq. wannier_3) and optionally band velocities
    v (Angstrom/fs) from hbar v^a_n = [U^dag dH/dk_a U]_nn (Eqs. velocity,
    wannier_4).  Within degenerate groups (gaps below deg_tol) the velocity is
    taken as the eigenvalues, in ascending order, of the group block of
    U^dag dH/dk_a U -- the degenerate extension the paper cites (Yates 2007)."""
    hk = hamiltonian_k(model, k)
    hk = 0.5 * (hk + hk.mH)
    eps, u = torch.linalg.eigh(hk)
    if not velocity:
        return eps, u
    rc = t64(model.re).to(F64) @ t64(model.lattice)            # Cartesian R, (nR,3)
    p = phases(k, model.re) * t64(model.w_re)
    dh = torch.einsum("kr,ra,rij->kaij", p, 1j * rc.to(C128),
                      torch.as_tensor(model.h, dtype=C128))
    m = torch.einsum("kim,kaij,kjn->kamn", u.conj(), dh, u)
    v = torch.diagonal(m, dim1=-2, dim2=-1).real.clone()        # (nk,3,nw)
    for ik in range(eps.shape[0]):
        for grp in degenerate_groups(eps[ik], deg_tol):
            if len(grp) < 2:
                continue
            idx = torch.tensor(grp)
            for a in range(3):
                blk = m[ik, a][idx][:, idx]
                blk = 0.5 * (blk + blk.mH)
                v[ik, a, idx] = torch.linalg.eigvalsh(blk)
    return eps, u, v.transpose(1, 2) / HBAR_EV_FS               # (nk,nw,3)


# ---------------------------------------------------------------- phonons

def dipole_matrix(model, q, alpha_ewald, gcut):
    """Long-range dipole-dipole part of the force constants in reciprocal space
    (the polar correction the paper takes from Gonze & Lee 1997, Sec. 2.3),
    eV/Angstrom^2, no mass factor:

      D^dd_{ka,k'b}(q) = (4 pi e^2/(4 pi eps0) / Omega) [
            sum_{G, q+G != 0, |q+G| < gcut} T_kk'(q+G)_ab e^{i (q+G).(tau_k - tau_k')}
          - delta_kk' sum_k'' sum_{G != 0, |G| < gcut} T_kk''(G)_ab e^{i G.(tau_k - tau_k'')} ],
      T_kk'(K)_ab = [K.Z*_k]_a [K.Z*_k']_b e^{-K.eps.K/(4 Lambda)} / (K.eps.K).

    The phase (q+G).(tau_k - tau_k') is the one of D(q) = sum_R e^{iq.R} C(R)
    with C_kk'(R) coupling kappa in cell 0 to kappa' in cell R.  q is brought to
    [-1/2,1/2)^3 first, as for the Froehlich term; the subtracted q = 0 sum keeps
    the acoustic sum rule."""
    q = t64(q)
    lat = t64(model.lattice)
    bvec = TWO_PI * torch.linalg.inv(lat).T
    zs = t64(model.zstar)
    eps = t64(model.eps_inf)
    tau = t64(model.tau)
    nat = tau.shape[0]
    omega_cell = abs(float(torch.linalg.det(lat)))
    pref = 4.0 * math.pi * E2_4PIEPS0 / omega_cell
    mmax = int(math.ceil((gcut + float(torch.linalg.norm(bvec, dim=1).sum())) *
                         float(torch.linalg.norm(lat, dim=1).max()) / TWO_PI)) + 1
    rng = torch.arange(-mmax, mmax + 1, dtype=F64)
    gvec = torch.stack(torch.meshgrid(rng, rng, rng, indexing="ij"), -1).reshape(-1, 3) @ bvec

    def block_sum(kv):
        # sum over the vectors kv of T_kk'(K) e^{i K.(tau_k - tau_k')}, (nat,3,nat,3)
        norm = torch.linalg.norm(kv, dim=1)
        keep = (norm < gcut) & (norm > 1e-12)
        kv = kv[keep]
        kek = torch.einsum("ga,ab,gb->g", kv, eps, kv)
        damp = torch.exp(-kek / (4.0 * alpha_ewald)) / kek
        kz = torch.einsum("gb,kba->gka", kv, zs)                  # [K.Z*_k]_a
        ph = torch.exp(1j * (kv @ tau.T))                         # e^{i K.tau_k}
        kzc = kz.to(C128) * ph[:, :, None]
        return torch.einsum("g,gka,glb->kalb", damp.to(C128), kzc, kzc.conj())

    corr = block_sum(gvec).sum(dim=2)                             # (nat,3,3): sum over k''
    qr = q - torch.round(q)
    out = torch.zeros((q.shape[0], 3 * nat, 3 * nat), dtype=C128)
    for iq in range(q.shape[0]):
        blk = block_sum((qr[iq] @ bvec)[None, :] + gvec)
        for k in range(nat):
            blk[k, :, k, :] -= corr[k]
        out[iq] = pref * blk.reshape(3 * nat, 3 * nat)
    return out


def dynamical_matrix(model, q, dipole=None):
    """D(q) = sum_Rp w e^{iq.Rp} C(Rp) / sqrt(M_kappa M_kappa')  (Eq. IFC2, with
    the mass factor the force constants of Eq. IFC1 leave out), plus the
    dipole-dipole part when dipole = dict(alpha_ewald, gcut) is given."""
    p = phases(q, model.rp_ph) * t64(model.w_rp_ph)
    m = t64(model.mass).repeat_interleave(3)
    c = torch.as_tensor(model.ifc, dtype=F64).to(C128)
    d = torch.einsum("qr,rab->qab", p, c)
    if dipole is not None:
        d = d + dipole_matrix(model, q, **dipole)
    return d / torch.sqrt(m[:, None] * m[None, :])


def phonons(model, q, dipole=None):
    """Phonon energies hbar*omega_nu (eV, ascending in omega^2; a negative
    omega^2 gives a negative value) and eigenvectors e_nu (columns) of D(q)."""
    d = dynamical_matrix(model, q, dipole)
    d = 0.5 * (d + d.mH)
    lam, e = torch.linalg.eigh(d)
    hw2 = HBAR2_AMU_A2 * lam
    return torch.sign(hw2) * torch.sqrt(torch.abs(hw2)), e


# ---------------------------------------------------------------- occupations

def fermi(eps, mu, temp):
    return 1.0 / (torch.exp((t64(eps) - mu) / (KB_EV * temp)) + 1.0)


def bose(omega, temp, omega_cut):
    """Bose-Einstein occupation; zero for excluded modes (omega <= omega_cut)."""
    omega = t64(omega)
    keep = omega > omega_cut
    safe = torch.where(keep, omega, torch.ones_like(omega))
    return torch.where(keep, 1.0 / torch.expm1(safe / (KB_EV * temp)), torch.zeros_like(omega))


def gauss_delta(x, sigma):
    """Gaussian-smeared delta function exp(-(x/s)^2)/(sqrt(pi) s)."""
    return torch.exp(-(x / sigma) ** 2) / (SQRT_PI * sigma)
