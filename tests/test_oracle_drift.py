"""Pins of the field-drift oracle (Eq. BTE_E with E != 0) and of Euler stepping.

The drift term is checked against the analytic gradient of a plane wave on a
non-orthogonal (fcc) grid, with second-order convergence; against number
conservation on a complete band; against the empty-neighbour rule at a window
edge; and against the physics it encodes: a packet of electrons moves in k at
-|e|E/hbar.  Euler stepping is pinned by its closed form on a linear equation
and by first-order convergence (RK4 by fourth order).
"""
import numpy as np
import pytest

import synth
from oracle import bte, drift
from oracle.grid import grid_points
from oracle.units import HBAR_EV_FS

LAT = synth.fcc_lattice(5.4)
B = 2 * np.pi * np.linalg.inv(LAT).T        # rows b_i, a_i . b_j = 2 pi delta_ij
E = np.array([0.003, -0.001, 0.002])         # V/Angstrom


def _full_band(n):
    ng = n ** 3
    return np.arange(ng), np.zeros(ng, dtype=np.int64)


def _cart(n):
    kr = grid_points((n, n, n))
    kr = kr - np.floor(kr + 0.5)              # reduced coordinates in [-1/2, 1/2)
    return kr @ B


def test_plane_wave_gradient_converges_at_second_order():
    m = np.array([1, -2, 1])
    G = m @ LAT                               # cos(G.k) is periodic over the zone
    errs = []
    for n in (8, 16, 32):
        k_idx, band = _full_band(n)
        nbr = drift.neighbours(k_idx, band, (n, n, n))
        k = _cart(n)
        f = np.cos(k @ G)
        exact = -(E @ G) * np.sin(k @ G) / HBAR_EV_FS
        got = drift.drift(f, nbr, LAT, (n, n, n), E)
        errs.append(np.abs(got - exact).max() / np.abs(exact).max())
    assert errs[-1] < 0.04
    assert 3.6 < errs[0] / errs[1] < 4.4 and 3.6 < errs[1] / errs[2] < 4.4


def test_complete_band_conserves_number():
    n = 6
    k_idx, band = _full_band(n)
    k_idx = np.concatenate([k_idx, k_idx])
    band = np.concatenate([band, band + 1])
    nbr = drift.neighbours(k_idx, band, (n, n, n))
    f = np.random.default_rng(3).random(len(k_idx))
    d = drift.drift(f, nbr, LAT, (n, n, n), E)
    assert abs(d.sum()) <= 1e-12 * np.abs(d).sum()
    assert np.abs(d).max() > 0


def test_window_edge_reads_empty_states():
    # a distribution that vanishes outside a window: the drift on the window's
    # states is the complete band's drift restricted to them
    n = 8
    k_idx, band = _full_band(n)
    k = _cart(n)
    inside = (k ** 2).sum(axis=1) < (0.45 * np.linalg.norm(B[0])) ** 2
    f_all = np.where(inside, 1.0 + np.random.default_rng(5).random(len(k)), 0.0)
    full = drift.drift(f_all, drift.neighbours(k_idx, band, (n,) * 3), LAT, (n,) * 3, E)
    win = drift.drift(f_all[inside], drift.neighbours(k_idx[inside], band[inside], (n,) * 3), LAT, (n,) * 3, E)
    assert np.allclose(win, full[inside], rtol=0, atol=1e-12 * np.abs(full).max())
    assert inside.sum() < len(k)


def test_packet_moves_against_the_field():
    # hbar dk/dt = -|e| E: the centroid of a packet near Gamma moves by -E t/hbar
    n = 24
    k_idx, band = _full_band(n)
    nbr = drift.neighbours(k_idx, band, (n,) * 3)
    k = _cart(n)
    w = 0.15 * np.linalg.norm(B[0])
    f0 = np.exp(-(k ** 2).sum(axis=1) / w ** 2)
    t, steps = 30.0, 60
    f = bte.integrate(f0, t / steps, steps, lambda y: drift.drift(y, nbr, LAT, (n,) * 3, E))
    shift = (f[:, None] * k).sum(0) / f.sum() - (f0[:, None] * k).sum(0) / f0.sum()
    expect = -E * t / HBAR_EV_FS
    assert np.linalg.norm(shift - expect) <= 0.03 * np.linalg.norm(expect)
    assert abs(f.sum() - f0.sum()) <= 1e-6 * f0.sum()


@pytest.mark.parametrize("lam", [0.02, 0.3])
def test_euler_closed_form_and_orders(lam):
    f0 = np.array([1.0, 0.5])
    rhs = lambda y: -lam * y
    dt, n = 0.5, 40
    got = bte.integrate(f0, dt, n, rhs, step=bte.euler_step)
    assert np.allclose(got, f0 * (1 - lam * dt) ** n, rtol=1e-14)
    exact = f0 * np.exp(-lam * dt * n)
    e1 = np.abs(bte.integrate(f0, dt, n, rhs, step=bte.euler_step) - exact).max()
    e2 = np.abs(bte.integrate(f0, dt / 2, 2 * n, rhs, step=bte.euler_step) - exact).max()
    r1 = np.abs(bte.integrate(f0, dt, n, rhs) - exact).max()
    r2 = np.abs(bte.integrate(f0, dt / 2, 2 * n, rhs) - exact).max()
    assert 1.8 < e1 / e2 < 2.2
    assert 14.0 < r1 / r2 < 18.0
