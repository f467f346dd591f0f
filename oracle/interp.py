"""Band and phonon interpolation (paper Sec. 2.2.1 and 2.2.2).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import torch

from .units import HBAR_EV_FS, HBAR2_AMU_A2, KB_EV, SQRT_PI, TWO_PI

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

def dynamical_matrix(model, q):
    """D(q) = sum_Rp w e^{iq.Rp} C(Rp) / sqrt(M_kappa M_kappa')  (Eq. IFC2, with
    the mass factor the force constants of Eq. IFC1 leave out)."""
    p = phases(q, model.rp_ph) * t64(model.w_rp_ph)
    m = t64(model.mass).repeat_interleave(3)
    c = torch.as_tensor(model.ifc, dtype=F64).to(C128)
    d = torch.einsum("qr,rab->qab", p, c)
    return d / torch.sqrt(m[:, None] * m[None, :])


def phonons(model, q):
    """Phonon energies hbar*omega_nu (eV, ascending in omega^2; a negative
    omega^2 gives a negative value) and eigenvectors e_nu (columns) of D(q)."""
    d = dynamical_matrix(model, q)
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
