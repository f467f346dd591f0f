"""Pins of the oracle's phase, band and phonon interpolation (paper Sec. 2.2.1,
2.2.2) against textbook closed forms, calculus and symmetry -- not against the
oracle itself."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import interp
from oracle.units import HBAR2_AMU_A2, HBAR_EV_FS


def _model_from(lattice, tau, mass, re, h, rp=None, ifc=None, nw=None):
    nr = len(re)
    nat = len(tau)
    if rp is None:
        rp = np.zeros((1, 3), np.int32)
        ifc = np.zeros((1, 3 * nat, 3 * nat))
    return synth.Model(
        lattice=np.asarray(lattice, float), tau=np.asarray(tau, float), mass=np.asarray(mass, float),
        nw=nw or h.shape[1], wf_centres=np.zeros((h.shape[1], 3)),
        re=np.asarray(re, np.int32), w_re=np.ones(nr), h=np.asarray(h, complex),
        rp_ph=np.asarray(rp, np.int32), w_rp_ph=np.ones(len(rp)), ifc=np.asarray(ifc, float),
        re_g=np.zeros((1, 3), np.int32), w_re_g=np.ones(1), rp_g=np.zeros((1, 3), np.int32),
        w_rp_g=np.ones(1), g=np.zeros((1, 1, 3 * nat, h.shape[1], h.shape[1]), complex))


def test_phase_is_periodic_and_multiplicative():
    x = synth.random_points(3, 7)
    n = synth.ws_vectors(synth.fcc_lattice(1.0), 4)
    p = interp.phases(x, n)
    assert torch.allclose(p.abs(), torch.ones_like(p.abs()), atol=1e-15)
    # exact lattice periodicity: x -> x + integer vector
    shifted = interp.phases(x + np.array([3.0, -2.0, 5.0]), n)
    assert torch.allclose(shifted, p, atol=1e-13)
    # e^{ik.(R1+R2)} = e^{ik.R1} e^{ik.R2}
    s = interp.phases(x, n[3:4] + n[5:6])
    assert torch.allclose(s[:, 0], p[:, 3] * p[:, 5], atol=1e-14)


def test_phase_sign_with_a_complex_chain_hopping():
    """One hopping t e^{i phi} along a_1: with the e^{+ik.R} convention of
    Eq. wannier_3 the band is eps0 + 2 t cos(2 pi x_1 + phi)."""
    t, phi, eps0 = 0.3, 0.7, 0.1
    re = [[0, 0, 0], [1, 0, 0], [-1, 0, 0]]
    h = np.array([[[eps0]], [[t * np.exp(1j * phi)]], [[t * np.exp(-1j * phi)]]])
    m = _model_from(np.eye(3), [[0, 0, 0]], [1.0], re, h)
    x = np.array([[0.1, 0.37, 0.9], [0.33, 0.0, 0.0], [0.8, 0.5, 0.5]])
    eps, _ = interp.bands(m, x)
    ref = eps0 + 2 * t * np.cos(2 * np.pi * x[:, 0] + phi)
    assert np.allclose(eps[:, 0].numpy(), ref, atol=1e-14)
    wrong = eps0 + 2 * t * np.cos(2 * np.pi * x[:, 0] - phi)
    assert not np.allclose(eps[:, 0].numpy(), wrong, atol=1e-6)


def _fcc_nn_vectors():
    lat = synth.fcc_lattice(1.0)
    vecs = synth.ws_vectors(lat, 4)
    d = np.linalg.norm(vecs @ lat, axis=1)
    nn = vecs[np.abs(d - d[d > 0].min()) < 1e-9]
    assert len(nn) == 12
    return nn


def test_fcc_nearest_neighbour_s_band_textbook():
    """fcc s band with NN hopping t (Ashcroft-Mermin):
    eps = eps0 + 4t [cos(kx a/2)cos(ky a/2) + cos(ky a/2)cos(kz a/2) + cos(kz a/2)cos(kx a/2)]."""
    a, t, eps0 = 5.389, -0.4, 1.0
    lat = synth.fcc_lattice(a)
    nn = _fcc_nn_vectors()
    re = np.vstack([[0, 0, 0], nn])
    h = np.array([[[eps0]]] + [[[t]]] * 12, dtype=complex)
    m = _model_from(lat, [[0, 0, 0]], [1.0], re, h)
    x = synth.random_points(11, 50)
    eps, _ = interp.bands(m, x)
    kc = x @ (2 * np.pi * np.linalg.inv(lat).T)              # Cartesian k
    c = np.cos(kc * a / 2)
    ref = eps0 + 4 * t * (c[:, 0] * c[:, 1] + c[:, 1] * c[:, 2] + c[:, 2] * c[:, 0])
    assert np.allclose(eps[:, 0].numpy(), ref, atol=1e-13)


def test_band_periodicity_and_hermitian_spectrum(tiny_model):
    x = synth.random_points(5, 20)
    e1, _ = interp.bands(tiny_model, x)
    e2, _ = interp.bands(tiny_model, x + np.array([1.0, -1.0, 2.0]))
    assert torch.allclose(e1, e2, atol=1e-12)
    hk = interp.hamiltonian_k(tiny_model, x)
    assert torch.allclose(hk, hk.mH, atol=1e-13)           # Hermitian before symmetrising


def test_velocity_matches_finite_difference(tiny_model):
    """hbar v = grad_k eps (Hellmann-Feynman), checked by central differences
    of the interpolated eigenvalues along Cartesian directions."""
    lat = tiny_model.lattice
    x = synth.random_points(7, 6)
    eps, _, v = interp.bands(tiny_model, x, velocity=True)
    h = 1e-5
    for a in range(3):
        dx = h * lat[:, a] / (2 * np.pi)                     # Cartesian step -> reduced
        ep, _ = interp.bands(tiny_model, x + dx)
        em, _ = interp.bands(tiny_model, x - dx)
        fd = (ep - em) / (2 * h) / HBAR_EV_FS
        assert torch.allclose(v[:, :, a], fd, rtol=1e-6, atol=1e-8)


def test_degenerate_velocity_on_doubled_model(tiny_model):
    """H1 (x) I2 has every band exactly doubly degenerate; the degenerate
    extension must give both copies the velocity of the single model."""
    m = tiny_model
    h2 = np.kron(m.h, np.eye(2))
    md = _model_from(m.lattice, m.tau, m.mass, m.re, h2.reshape(len(m.re), 2 * m.nw, 2 * m.nw))
    x = synth.random_points(9, 5)
    _, _, v1 = interp.bands(m, x, velocity=True)
    _, _, v2 = interp.bands(md, x, velocity=True)
    assert torch.allclose(v2[:, 0::2], v1, atol=1e-9)
    assert torch.allclose(v2[:, 1::2], v1, atol=1e-9)


def test_acoustic_sum_rule_and_stability():
    for name in ("tiny", "si"):
        m = synth.make_config_model(name) if name == "tiny" else _si_small()
        om, _ = interp.phonons(m, np.zeros((1, 3)))
        q = synth.random_points(13, 40)
        omq, _ = interp.phonons(m, q)
        wmax = float(omq.max())
        assert float(om[0, :3].abs().max()) <= 1e-6 * wmax
        assert float(omq.min()) > 0.0                          # omega^2 > 0 off Gamma


def _si_small():
    # Si-like geometry on a 4^3 set (the spring construction does not depend on set size)
    return synth.make_config_model("si", n_grid=4)


def test_fcc_central_force_phonons_at_x_textbook():
    """Monatomic fcc, NN central springs K: omega_L(X) = sqrt(8K/M),
    omega_T(X) = sqrt(4K/M) (two-fold), omega(Gamma) = 0."""
    a, kspring, mass = 4.0, 2.5, 30.0
    lat = synth.fcc_lattice(a)
    nn = _fcc_nn_vectors()
    re = np.vstack([[0, 0, 0], nn])
    ifc = np.zeros((13, 3, 3))
    for i, n in enumerate(nn):
        r = n @ lat
        rr = np.outer(r, r) / (r @ r)
        ifc[1 + i] = -kspring * rr
        ifc[0] += kspring * rr
    h = np.zeros((13, 1, 1), complex)
    m = _model_from(lat, [[0, 0, 0]], [mass], re, h, rp=re, ifc=ifc)
    xpt = np.array([[0.0, 0.5, 0.5]])                         # X = (2pi/a)(1,0,0) in fcc reduced coords
    kc = xpt @ (2 * np.pi * np.linalg.inv(lat).T)
    assert np.allclose(kc, [[2 * np.pi / a, 0, 0]])
    om, _ = interp.phonons(m, xpt)
    ref = np.sqrt(HBAR2_AMU_A2 * np.array([4, 4, 8]) * kspring / mass)
    assert np.allclose(om[0].numpy(), ref, rtol=1e-12)
    om0, _ = interp.phonons(m, np.zeros((1, 3)))
    assert float(om0.abs().max()) < 1e-7


def test_occupations_and_delta():
    x = torch.linspace(-0.05, 0.05, 20001, dtype=torch.float64)
    d = interp.gauss_delta(x, 0.005)
    assert abs(float(torch.trapezoid(d, x)) - 1.0) < 1e-12   # unit weight
    assert abs(float(interp.fermi(torch.tensor([0.3], dtype=torch.float64), 0.3, 300.0)) - 0.5) < 1e-15
    om = torch.tensor([0.05, 1e-5], dtype=torch.float64)
    n = interp.bose(om, 300.0, 1e-4)
    kt = 8.617333262e-5 * 300.0
    assert abs(float(n[0]) - 1.0 / (math.exp(0.05 / kt) - 1.0)) < 1e-15
    assert float(n[1]) == 0.0
