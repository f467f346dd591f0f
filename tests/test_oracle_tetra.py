"""Pins of the linear tetrahedron integration (oracle/tetra.py) against what
the method fixes: closed-form energy moments of the corner weights, Monte
Carlo sampling of one tetrahedron, the exact count rule on a complete band,
and the density of states of a chain."""
import math

import numpy as np
import pytest

from oracle import grid, tetra


def _integrate_weights(e, n=6001):
    E = np.linspace(min(e) - 1e-9, max(e) + 1e-9, n)
    c = np.array([tetra.delta_weights(e, x) for x in E])
    return E, c


@pytest.mark.parametrize("e", [[0.1, 0.35, 0.6, 0.9], [0.7, -0.2, 0.3, 0.1], [0.0, 0.5, 0.5, 1.0], [0.2, 0.2, 0.9, 0.4]])
def test_weight_moments_closed_form(e):
    # (1/V_T) int lambda_j = 1/4 and (1/V_T) int eps lambda_j = (e_j + sum e)/20
    E, c = _integrate_weights(e)
    m0 = np.trapezoid(c, E, axis=0)
    m1 = np.trapezoid(c * E[:, None], E, axis=0)
    assert np.allclose(m0, 0.25, atol=1e-5)
    assert np.allclose(m1, (np.asarray(e) + sum(e)) / 20.0, atol=1e-5)


def test_weights_match_monte_carlo():
    rng = np.random.default_rng(90)
    e = np.array([0.1, 0.45, 0.55, 1.0])
    lam = rng.dirichlet(np.ones(4), size=4_000_000)
    eps = lam @ e
    h = 2e-3
    for E in (0.3, 0.5, 0.8):          # one energy in each case
        sel = np.abs(eps - E) < h
        mc = lam[sel].sum(axis=0) / (2 * h * len(lam))
        got = tetra.delta_weights(e, E)
        assert np.allclose(got, mc, rtol=0.03, atol=2e-3), (E, got, mc)


def test_complete_band_counts_every_state_once():
    # every grid point is a corner of 24 tetrahedra, each giving it 1/4 of its
    # weight integral over 1/6: the energy integral of sum X delta is sum X
    n = (3, 3, 3)
    pts = grid.grid_points(n)
    # any corner energies obey the rule; distinct ones keep p(E) continuous for the quadrature
    eps = np.random.default_rng(92).random(len(pts))
    k_idx = np.arange(len(pts))
    band = np.zeros(len(pts), dtype=np.int64)
    tets = tetra.tetrahedra(k_idx, band, n)
    assert len(tets) == 6 * len(pts)
    x = np.random.default_rng(91).random(len(pts))
    E = np.linspace(eps.min() - 1e-6, eps.max() + 1e-6, 801)
    p = tetra.population(eps, x, tets, E)
    assert abs(np.trapezoid(p, E) - x.sum()) <= 1e-4 * x.sum()


def test_chain_density_of_states():
    # eps = -2t cos(2 pi k_x): per grid point the DOS is 1/(pi sqrt(4t^2 - E^2));
    # the linear interpolation converges to it as the grid is refined
    n = (240, 1, 1)
    pts = grid.grid_points(n)
    t = 0.5
    eps = -2 * t * np.cos(2 * np.pi * pts[:, 0])
    k_idx = np.arange(len(pts))
    tets = tetra.tetrahedra(k_idx, np.zeros(len(pts), dtype=np.int64), n)
    E = np.array([-0.6, -0.2, 0.05, 0.45])
    dos = tetra.population(eps, np.ones(len(pts)), tets, E) / len(pts)
    exact = 1.0 / (np.pi * np.sqrt(4 * t * t - E * E))
    assert np.allclose(dos, exact, rtol=1e-2)


def test_transport_integrals_mott_formula():
    # Sigma(E) = a + b (E - mu) on a wide grid: sigma = e^2 a (S/m units of
    # SIGMA_UNIT) and, by the Sommerfeld expansion (exact for a linear TDF),
    # S = -(pi^2/3) k_B^2 T b / a (Mott formula; electron charge -e)
    mu, temp = 0.1, 300.0
    E = np.linspace(mu - 1.5, mu + 1.5, 30001)
    a = np.diag([2.0, 3.0, 4.0])
    b = np.diag([0.5, -1.0, 2.0])
    sig = a[None] + (E - mu)[:, None, None] * b[None]
    sigma, seebeck = tetra.transport_from_tdf(E, sig, mu, temp)
    kt = 8.617333262e-5 * temp
    assert np.allclose(sigma, tetra.SIGMA_UNIT * a, rtol=1e-9)
    mott = -(math.pi ** 2 / 3.0) * kt * kt * np.diag(b) / np.diag(a) / temp
    assert np.allclose(np.diag(seebeck), mott, rtol=1e-6)
