"""Pins of the dipole-dipole (LO-TO) part of the dynamical matrix in the
oracle (oracle.interp.dipole_matrix), against what the method fixes."""
import math

import numpy as np
import torch

import synth
from oracle import interp
from oracle.units import E2_4PIEPS0


def _case():
    m = synth.make_config_model("gaas", n_grid=4, nw=4)
    a = synth.models.A_GAAS
    return m, dict(alpha_ewald=(2 * np.pi / a) ** 2, gcut=4 * 2 * np.pi / a)


def test_acoustic_sum_rule_kept_at_gamma():
    m, dip = _case()
    om, _ = interp.phonons(m, np.zeros((1, 3)), dipole=dip)
    wmax = float(interp.phonons(m, np.array([[0.5, 0.0, 0.0]]), dipole=dip)[0].abs().max())
    assert float(om[0, :3].abs().max()) <= 1e-6 * wmax
    d0 = interp.dipole_matrix(m, np.zeros((1, 3)), **dip)[0]
    # sum over kappa' of every (kappa alpha, kappa' beta) block vanishes
    blocks = d0.reshape(m.nat, 3, m.nat, 3).sum(dim=2)
    assert float(blocks.abs().max()) <= 1e-12 * float(d0.abs().max())


def test_hermitian_and_time_reversal():
    m, dip = _case()
    q = synth.random_points(300, 5)
    d = interp.dipole_matrix(m, q, **dip)
    dm = interp.dipole_matrix(m, -q, **dip)
    assert float((d - d.mH).abs().max()) <= 1e-12 * float(d.abs().max())
    assert float((dm - d.conj()).abs().max()) <= 1e-12 * float(d.abs().max())


def test_nonanalytic_limit_at_small_q():
    # D^dd(s qhat) - D^dd(0) -> (4 pi e^2/Omega) [qhat.Z_k]_a [qhat.Z_k']_b / (qhat.eps.qhat), linearly in s
    m, dip = _case()
    omega_cell = m.volume()
    qhat_red = np.array([0.3, -0.2, 0.7])
    bvec = 2 * np.pi * np.linalg.inv(m.lattice).T
    qhat = qhat_red @ bvec
    qhat /= np.linalg.norm(qhat)
    zq = np.einsum("b,kba->ka", qhat, m.zstar).reshape(-1)
    na = 4 * math.pi * E2_4PIEPS0 / omega_cell * np.outer(zq, zq) / (qhat @ m.eps_inf @ qhat)
    d0 = interp.dipole_matrix(m, np.zeros((1, 3)), **dip)[0].numpy()
    errs = []
    for s in (1e-3, 1e-4):
        d = interp.dipole_matrix(m, (s * qhat_red)[None, :], **dip)[0].numpy()
        errs.append(np.abs(d - d0 - na).max() / np.abs(na).max())
    assert errs[1] <= 2e-3 and errs[0] / errs[1] > 5.0


def test_continuous_across_the_zone_boundary():
    # with D(q) = sum_R e^{iq.R} C(R) the sum is periodic in q: the values just
    # inside either face of the zone agree (a tau-dependent phase convention would jump)
    m, dip = _case()
    for axis in range(3):
        lo = np.array([0.13, -0.21, 0.07])
        hi = lo.copy()
        lo[axis], hi[axis] = 0.5 - 1e-6, -0.5 + 1e-6
        d = interp.dipole_matrix(m, np.stack([lo, hi]), **dip)
        assert float((d[0] - d[1]).abs().max()) <= 1e-4 * float(d[0].abs().max())
