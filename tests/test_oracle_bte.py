"""Pins of the oracle's grid machinery, collision integral, RK4, iterative BTE
and mobility (paper Sec. 2.1, 4.3) against brute force, conservation laws,
exact detailed balance, closed forms and linear algebra."""
import math

import numpy as np
import pytest
import scipy.linalg
import torch

import synth
from oracle import bte, eph, grid, interp
from oracle.units import HBAR2_AMU_A2, HBAR_EV_FS, KB_EV


# --------------------------------------------------------------- grids and pairs

def test_grid_index_roundtrip_and_pairs_bruteforce():
    n = (4, 5, 3)
    idx = np.arange(60)
    c = grid.grid_coords(idx, n)
    assert (grid.grid_index(c, n) == idx).all()
    pts = grid.grid_points(n)
    rng = np.random.default_rng(0)
    ks, kt = rng.integers(0, 60, 200), rng.integers(0, 60, 200)
    iq = grid.pair_q_index(ks, kt, n)
    for a, b, q in zip(ks, kt, iq):
        # brute force: the grid point q with k_s + q = k_t modulo reciprocal vectors
        found = [j for j in range(60) if np.allclose(((pts[a] + pts[j] - pts[b]) + 0.5) % 1.0 - 0.5, 0)]
        assert found == [q]
    back = grid.pair_q_index(kt, ks, n)
    assert (grid.minus_q_index(iq, n) == back).all()


def test_window_states_bruteforce():
    rng = np.random.default_rng(1)
    eps = rng.random((300, 5))
    kk, bb = grid.window_states(eps, 1, 4, 0.2, 0.6)
    ref = [(k, b) for k in range(300) for b in range(1, 4) if 0.2 < eps[k, b] < 0.6]
    assert list(zip(kk.tolist(), bb.tolist())) == ref
    k2, b2 = grid.lowest_states(eps, 2, 37)
    order = sorted(range(300), key=lambda k: (eps[k, 2], k))[:37]
    assert k2.tolist() == sorted(order)


# --------------------------------------------------------------- collision

def _random_table(s, nm, seed):
    rng = np.random.default_rng(seed)
    eps = torch.as_tensor(np.sort(rng.random(s) * 0.3))
    g2 = torch.as_tensor(rng.random((s, s, nm)))
    g2 = 0.5 * (g2 + g2.transpose(0, 1))
    om = torch.as_tensor(0.01 + 0.05 * rng.random((s, s, nm)))
    om = 0.5 * (om + om.transpose(0, 1))                  # omega(q) = omega(-q)
    return eps, g2, om


def test_collision_conserves_carriers_for_any_f():
    eps, g2, om = _random_table(40, 3, 2)
    f = torch.as_tensor(np.random.default_rng(3).random(40))
    i = bte.collision(f, eps, g2, om, temp=300.0, sigma=0.01, n_q=1000)
    assert abs(float(i.sum())) <= 1e-13 * float(i.abs().sum())
    assert float(i.abs().max()) > 0


def test_resonant_ladder_exact_detailed_balance():
    """Energies on a ladder eps_s in hw0*Z with a dispersionless mode hw0 and
    sigma = hw0/10: every non-resonant Gaussian weight is <= e^{-100}, and on
    resonance F_em = F_abs = 0 for Fermi-Dirac f and Bose-Einstein N, so
    I[f_FD] vanishes (exact detailed balance, Eq. e_ph_scattering)."""
    hw0, s, temp, mu = 0.04, 30, 300.0, 0.05
    rng = np.random.default_rng(4)
    eps = torch.as_tensor(hw0 * rng.integers(0, 8, s).astype(float))
    g2 = torch.as_tensor(rng.random((s, s, 1)))
    g2 = 0.5 * (g2 + g2.transpose(0, 1))
    om = torch.full((s, s, 1), hw0, dtype=torch.float64)
    ffd = interp.fermi(eps, mu, temp)
    i_eq = bte.collision(ffd, eps, g2, om, temp=temp, sigma=hw0 / 10, n_q=100)
    f_hot = interp.fermi(eps, mu, 3000.0)
    i_hot = bte.collision(f_hot, eps, g2, om, temp=temp, sigma=hw0 / 10, n_q=100)
    assert float(i_eq.abs().max()) <= 1e-14 * float(i_hot.abs().max())
    assert float(i_hot.abs().max()) > 0


def test_two_state_closed_form_and_stationary_point():
    """Two states with eps2 - eps1 = hw0, one mode: I_1 = -(2pi/hbar)(1/Nq) G
    delta(0) [f1(1-f2) N - f2(1-f1)(N+1)] (absorption 1->2), I_2 = -I_1, and the
    stationary point satisfies f2/(1-f2) = f1/(1-f1) * N/(N+1)."""
    hw0, temp, sig, gg, nq = 0.03, 300.0, 0.003, 0.7, 10000
    eps = torch.tensor([0.1, 0.1 + hw0], dtype=torch.float64)
    g2 = torch.full((2, 2, 1), gg, dtype=torch.float64)
    om = torch.full((2, 2, 1), hw0, dtype=torch.float64)
    f = torch.tensor([0.4, 0.1], dtype=torch.float64)
    i = bte.collision(f, eps, g2, om, temp=temp, sigma=sig, n_q=nq)
    nb = 1.0 / (math.exp(hw0 / (KB_EV * temp)) - 1.0)
    d0 = 1.0 / (math.sqrt(math.pi) * sig)
    off = math.exp(-(2 * hw0 / sig) ** 2) / (math.sqrt(math.pi) * sig)     # emission 1->2
    f1, f2 = 0.4, 0.1
    # self-pairs (s,s): delta(-hw) F_em + delta(+hw) F_abs = delta(hw) [f(1-f) - f(1-f)] = 0
    i1 = -(2 * math.pi / HBAR_EV_FS) / nq * gg * (
        d0 * (f1 * (1 - f2) * nb - f2 * (1 - f1) * (nb + 1))
        + off * (f1 * (1 - f2) * (nb + 1) - f2 * (1 - f1) * nb))
    assert abs(float(i[0]) - i1) <= 1e-12 * abs(i1)
    assert abs(float(i[0] + i[1])) <= 1e-14 * abs(i1)
    # integrate to the stationary point
    rhs = lambda x: bte.collision(x, eps, g2, om, temp=temp, sigma=sig, n_q=nq)
    x = bte.integrate(f, 1.0, 600, rhs)
    r1, r2 = float(x[0] / (1 - x[0])), float(x[1] / (1 - x[1]))
    assert abs(r2 / r1 - nb / (nb + 1)) < 1e-8
    assert abs(float(x.sum()) - 0.5) < 1e-13


def test_rk4_fourth_order_on_linear_system():
    """RK4 applied to the linearisation J = dI/df at f = 0 of a random table,
    against scipy.linalg.expm: error falls by ~16x when dt halves."""
    eps, g2, om = _random_table(12, 2, 5)
    par = dict(temp=300.0, sigma=0.02, n_q=20000)
    jac = torch.autograd.functional.jacobian(
        lambda x: bte.collision(x, eps, g2, om, **par), torch.zeros(12, dtype=torch.float64))
    f0 = torch.as_tensor(np.random.default_rng(6).random(12))
    t_end = 40.0
    exact = torch.as_tensor(scipy.linalg.expm(jac.numpy() * t_end) @ f0.numpy())
    errs = []
    for nsteps in (20, 40, 80):
        dt = t_end / nsteps
        y = bte.integrate(f0, dt, nsteps, lambda x: jac @ x)
        errs.append(float((y - exact).abs().max()))
    assert 12.0 < errs[0] / errs[1] < 20.0
    assert 12.0 < errs[1] / errs[2] < 20.0


def test_carrier_number_conserved_over_many_steps():
    eps, g2, om = _random_table(30, 3, 7)
    f = 0.2 * torch.as_tensor(np.random.default_rng(8).random(30))
    rhs = lambda x: bte.collision(x, eps, g2, om, temp=300.0, sigma=0.01, n_q=50000)
    y = bte.integrate(f, 1.0, 1000, rhs)
    assert abs(float(y.sum() - f.sum())) <= 1e-12 * float(f.sum())
    assert not torch.allclose(y, f, atol=1e-6)


# --------------------------------------------------------------- transport

def test_ita_converges_to_dense_solve_and_zero_iterations_is_rta():
    """With a total rate above the in-set row sum the iteration map is a
    contraction and its limit is the dense solution of (1 - diag(tau/Nq) W) F = tau v."""
    eps, g2, om = _random_table(25, 2, 9)
    w = bte.transport_matrix(eps, g2, om, temp=300.0, mu=-0.2, sigma=0.02)
    v = torch.as_tensor(np.random.default_rng(10).standard_normal((25, 3)))
    nq = 1000.0
    gam = 1.3 * w.sum(dim=1) / nq
    f_rta, tau = bte.ita(w, v, nq, 0, gamma=gam)
    assert torch.allclose(f_rta, tau[:, None] * v)
    f_it, _ = bte.ita(w, v, nq, 300, gamma=gam)
    a = torch.eye(25, dtype=torch.float64) - (tau / nq)[:, None] * w
    f_dense = torch.linalg.solve(a, tau[:, None] * v)
    assert torch.allclose(f_it, f_dense, rtol=1e-12, atol=1e-14)


def test_ita_converges_on_inversion_symmetric_table():
    """States in +/-k pairs with W invariant under the pairing and odd velocities:
    the in-set iteration (Gamma = row sum) converges to the dense solution
    restricted to odd vectors."""
    half = 12
    rng = np.random.default_rng(11)
    e_half = np.sort(rng.random(half) * 0.2)
    eps = torch.as_tensor(np.concatenate([e_half, e_half]))
    perm = np.concatenate([np.arange(half, 2 * half), np.arange(half)])   # s -> -s
    g = rng.random((2 * half, 2 * half, 2))
    g = g + g[perm][:, perm]
    g = g + g.transpose(1, 0, 2)
    om = 0.02 + 0.03 * rng.random((2 * half, 2 * half, 2))
    om = om + om[perm][:, perm]
    om = 0.5 * (om + om.transpose(1, 0, 2))
    w = bte.transport_matrix(eps, torch.as_tensor(g), torch.as_tensor(om), temp=300.0, mu=-0.2, sigma=0.03)
    vh = rng.standard_normal((half, 3))
    v = torch.as_tensor(np.concatenate([vh, -vh]))
    nq = 50.0
    f_it, tau = bte.ita(w, v, nq, 400)
    f_prev, _ = bte.ita(w, v, nq, 399)
    assert float((f_it - f_prev).abs().max()) < 1e-12 * float(f_it.abs().max())
    m = (tau / nq)[:, None] * w
    assert torch.allclose(f_it, tau[:, None] * v + m @ f_it, rtol=1e-10, atol=1e-12)
    assert torch.allclose(f_it[:half], -f_it[half:], atol=1e-12)


def test_mobility_drude_limit_parabolic_band():
    """Isotropic parabolic band eps = hbar^2 k^2/(2 m*), v = hbar k/m*, constant
    tau, Boltzmann statistics: mu = e tau / m* (equipartition).  Constants in
    this test are independent of the oracle's: hbar/m_e = 11.5767636 A^2/fs,
    hbar^2/(2 m_e) = 3.80998208 eV A^2, e/m_e * 1 fs = 1.75882001e-4 m^2/(V s)."""
    mstar, tau, temp = 0.3, 12.0, 300.0
    h2m = 3.80998208 / mstar
    hm = 11.5767636 / mstar
    kmax = math.sqrt(12 * KB_EV * temp / h2m)          # ~12 kT of the tail
    n = 81
    ax = np.linspace(-kmax, kmax, n)
    kx, ky, kz = np.meshgrid(ax, ax, ax, indexing="ij")
    kv = np.stack([kx.ravel(), ky.ravel(), kz.ravel()], 1)
    eps = h2m * (kv ** 2).sum(1)
    vel = hm * kv
    ff = tau * vel
    mu_t = bte.mobility(torch.as_tensor(eps), torch.as_tensor(vel), torch.as_tensor(ff), mu=-0.3, temp=temp)
    drude = 1.75882001e-4 * tau / mstar * 1e4          # cm^2/(V s)
    assert abs(float(mu_t[0, 0]) / drude - 1) < 2e-3
    assert abs(float(mu_t[0, 1])) < 1e-6 * drude


def test_chemical_potential_bisection():
    eps = torch.as_tensor(np.linspace(1.0, 1.3, 500))
    mu = bte.chemical_potential(eps, 1e17, 300.0, 1000, 40.0)
    n = bte.carrier_density(eps, mu, 300.0, 1000, 40.0)
    assert abs(n / 1e17 - 1) < 1e-10


# --------------------------------------------------------------- pair table on a model

def test_pair_table_symmetric_and_matches_direct_pairs(tiny_model):
    n_grid = (4, 4, 4)
    pts = grid.grid_points(n_grid)
    eps, _ = interp.bands(tiny_model, pts)
    kk, bb = grid.lowest_states(eps.numpy(), tiny_model.nw // 2, 10)
    g2s, om = bte.pair_table(tiny_model, n_grid, kk, bb)
    assert torch.allclose(g2s, g2s.transpose(0, 1))
    # spot-check one ordered pair against the pipeline at (k_s, q)
    from oracle import eph
    s, t = 2, 7
    q = ((grid.grid_coords(kk[t], n_grid) - grid.grid_coords(kk[s], n_grid)) % 4) / 4.0
    ga = eph.g2(tiny_model, pts[kk[s]][None], q[None])[0, 0, :, bb[t], bb[s]]
    gb = eph.g2(tiny_model, pts[kk[t]][None], -q[None])[0, 0, :, bb[s], bb[t]]
    assert torch.allclose(g2s[s, t], 0.5 * (ga + gb), rtol=1e-10)


def test_pair_entries_match_the_table():
    """The per-pair evaluation used to sample large tables gives the entries of
    the full table (same definition, evaluated two ways)."""
    m = synth.make_config_model("tiny")
    n = (4, 4, 4)
    eps, _ = interp.bands(m, grid.grid_points(n))
    kk, bb = grid.lowest_states(eps.numpy(), m.nw // 2, 12)
    g2s, om = bte.pair_table(m, n, kk, bb)
    pairs = [(0, 0), (0, 5), (5, 0), (3, 11), (11, 7), (6, 6)]
    e2, eo = bte.pair_entries(m, n, kk, bb, pairs)
    for i, (s, t) in enumerate(pairs):
        assert torch.allclose(e2[i], g2s[s, t], rtol=1e-12, atol=1e-300)
        assert torch.allclose(eo[i], om[s, t], rtol=1e-12, atol=1e-300)


def test_transport_matrix_two_state_closed_form():
    """Eq. BTE_W for two states eps_2 - eps_1 = hw0 and one mode, every delta
    term kept (sigma is not small against hw0):
      W_st = (2 pi/hbar) G [delta(eps_s - hw - eps_t)(1 + N - f0_t) + delta(eps_s + hw - eps_t)(N + f0_t)]
    The occupation is the final state's; mu is placed so that f0_1 and f0_2
    differ by a factor ~2."""
    hw0, temp, sig, gg, mu = 0.03, 300.0, 0.02, 0.7, 0.12
    eps = torch.tensor([0.1, 0.1 + hw0], dtype=torch.float64)
    g2 = torch.full((2, 2, 1), gg, dtype=torch.float64)
    om = torch.full((2, 2, 1), hw0, dtype=torch.float64)
    w = bte.transport_matrix(eps, g2, om, temp=temp, mu=mu, sigma=sig)
    kt = KB_EV * temp
    nb = 1.0 / (math.exp(hw0 / kt) - 1.0)
    f0 = [1.0 / (math.exp((float(e) - mu) / kt) + 1.0) for e in eps]
    assert 1.5 < f0[0] / f0[1] < 2.5

    def delta(x):
        return math.exp(-(x / sig) ** 2) / (math.sqrt(math.pi) * sig)

    c = 2 * math.pi / HBAR_EV_FS * gg
    for s in range(2):
        for t in range(2):
            d = float(eps[s] - eps[t])
            ref = c * (delta(d - hw0) * (1 + nb - f0[t]) + delta(d + hw0) * (nb + f0[t]))
            assert abs(float(w[s, t]) - ref) <= 1e-12 * ref


def test_transport_matrix_row_sums_are_the_rates():
    """On a complete grid (every k, every band a state) the row sum of W over
    the final states, divided by N_q, is the scattering rate of Eq. scatter_rate
    with the grid as the q set: the flat-band Einstein model, whose rates are
    pinned in closed form, with a coupling gamma^a_mn Hermitian in (m, n) so
    that the symmetrised table has the same mode sums as |g(s->t)|^2."""
    hw, mass, sig, temp, mu = 0.05, 20.0, 0.02, 300.0, 0.02
    lev = [0.0, 0.05]
    rng = np.random.default_rng(11)
    gam = rng.standard_normal((3, 2, 2)) + 1j * rng.standard_normal((3, 2, 2))
    gam = 0.5 * (gam + gam.conj().transpose(0, 2, 1))
    z = np.zeros((1, 3), np.int32)
    m = synth.Model(
        lattice=synth.fcc_lattice(5.0), tau=np.zeros((1, 3)), mass=np.array([mass]), nw=2,
        wf_centres=np.zeros((2, 3)), re=z, w_re=np.ones(1), h=np.diag(lev).astype(complex)[None],
        rp_ph=z, w_rp_ph=np.ones(1), ifc=(hw ** 2 * mass / HBAR2_AMU_A2) * np.eye(3)[None],
        re_g=z, w_re_g=np.ones(1), rp_g=z, w_rp_g=np.ones(1), g=gam[None, None])
    n = (2, 2, 2)
    nk = 8
    kk = np.repeat(np.arange(nk), 2).astype(np.int32)
    bb = np.tile(np.arange(2), nk).astype(np.int32)
    g2s, om = bte.pair_table(m, n, kk, bb)
    eps = bte.state_energies(m, kk, bb, n)
    w = bte.transport_matrix(eps, g2s, om, temp=temp, mu=mu, sigma=sig)
    pts = grid.grid_points(n)
    gamma, _ = eph.rates(m, pts, pts, temp=temp, mu=mu, sigma=sig)
    ref = gamma[torch.as_tensor(kk), torch.as_tensor(bb)]
    assert float(ref.min()) > 0
    assert torch.allclose(w.sum(dim=1) / nk, ref, rtol=1e-12)


def _symmetric_pair_table(half, seed):
    """States in +/-k pairs: W invariant under the pairing, odd velocities."""
    rng = np.random.default_rng(seed)
    e_half = np.sort(rng.random(half) * 0.2)
    eps = torch.as_tensor(np.concatenate([e_half, e_half]))
    perm = np.concatenate([np.arange(half, 2 * half), np.arange(half)])
    g = rng.random((2 * half, 2 * half, 2))
    g = g + g[perm][:, perm]
    g = g + g.transpose(1, 0, 2)
    om = 0.02 + 0.03 * rng.random((2 * half, 2 * half, 2))
    om = om + om[perm][:, perm]
    om = 0.5 * (om + om.transpose(1, 0, 2))
    w = bte.transport_matrix(eps, torch.as_tensor(g), torch.as_tensor(om), temp=300.0, mu=-0.2, sigma=0.03)
    vh = rng.standard_normal((half, 3))
    return w, torch.as_tensor(np.concatenate([vh, -vh]))


def test_ita_dense_odd_with_decoupled_groups():
    """Two groups of states that do not scatter into each other: (1 - M) has a
    two-dimensional null space, yet the odd fixed point is unique and is what
    the iteration converges to; the dense odd solve gives it, with self-partnered
    states (k = -k) at F = 0."""
    w1, v1 = _symmetric_pair_table(6, 31)
    w2, v2 = _symmetric_pair_table(5, 32)
    s1, s2 = len(v1), len(v2)
    w = torch.zeros((s1 + s2 + 1, s1 + s2 + 1), dtype=torch.float64)
    w[:s1, :s1] = w1
    w[s1:s1 + s2, s1:s1 + s2] = w2
    w[-1, -1] = 1.0                       # a state at k = -k scattering only into itself
    v = torch.cat([v1, v2, torch.zeros((1, 3), dtype=torch.float64)])
    partner = np.concatenate([np.arange(6, 12), np.arange(6), s1 + np.arange(5, 10), s1 + np.arange(5),
                              [s1 + s2]])
    nq = 40.0
    f_it, _, n, _ = bte.ita_converged(w, v, nq, 5000, 1e-13)
    f_d, _ = bte.ita_dense_odd(w, v, nq, partner)
    assert n < 5000
    assert float((f_it - f_d).abs().max()) <= 1e-10 * float(f_d.abs().max())
    assert float(f_d[-1].abs().max()) == 0.0


def test_ita_stopping_rule_and_converged_value():
    """The converged iterate (Eq. BTE_iter run to a threshold) solves
    (1 - M) F = tau v, M = diag(tau/N_q) W: that system is singular here (the
    rows of M sum to one, M 1 = 1), and F is its solution with sum_s F_s = 0,
    as odd vectors have; that solution is also the one of the regular system
    (1 - M + 1 1^T / S) F = tau v, and the minimum-norm least-squares one.
    The count is the first update whose relative change is below tol, found
    by brute force over fixed-count runs."""
    w, v = _symmetric_pair_table(14, 12)
    nq, tol = 50.0, 1e-12
    f, tau, n, chg = bte.ita_converged(w, v, nq, 5000, tol)
    assert 0 < n < 5000 and 0 <= chg < tol
    S = len(v)
    a = torch.eye(S, dtype=torch.float64) - (tau / nq)[:, None] * w
    ref = torch.linalg.solve(a + 1.0 / S, tau[:, None] * v)
    assert float((f - ref).abs().max()) <= 1e-10 * float(ref.abs().max())
    lsq = torch.linalg.lstsq(a, tau[:, None] * v, rcond=1e-12, driver="gelsd").solution
    assert float((lsq - ref).abs().max()) <= 1e-9 * float(ref.abs().max())
    half = S // 2
    partner = np.concatenate([np.arange(half, S), np.arange(half)])
    odd, _ = bte.ita_dense_odd(w, v, nq, partner)
    assert float((odd - ref).abs().max()) <= 1e-10 * float(ref.abs().max())
    prev, _ = bte.ita(w, v, nq, 0)
    for i in range(1, n + 1):
        cur, _ = bte.ita(w, v, nq, i)
        rel = float((cur - prev).abs().max()) / float(cur.abs().max())
        assert (rel < tol) == (i == n)
        prev = cur
    assert torch.equal(f, prev)
    # n_iter_max = 0 is the RTA; a cap below the count stops there
    f0, _, n0, c0 = bte.ita_converged(w, v, nq, 0, tol)
    assert n0 == 0 and c0 == -1.0 and torch.equal(f0, tau[:, None] * v)
    f3, _, n3, c3 = bte.ita_converged(w, v, nq, 3, tol)
    assert n3 == 3 and c3 >= tol and torch.equal(f3, bte.ita(w, v, nq, 3)[0])


def test_collision_rows_are_rows_of_the_collision_integral():
    """collision_rows on a subset of rows equals those entries of the pinned
    collision integral (any f, mode scales included)."""
    eps, g2, om = _random_table(30, 3, 21)
    f = torch.as_tensor(np.random.default_rng(22).random(30))
    sc = torch.as_tensor([1.0, 0.3, 2.0])
    par = dict(temp=300.0, sigma=0.02, n_q=500.0)
    full = bte.collision(f, eps, g2, om, mode_scale=sc, **par)
    rows = np.array([0, 7, 8, 29])
    part = bte.collision_rows(rows, f, eps, g2[rows], om[rows], mode_scale=sc, **par)
    assert torch.allclose(part, full[rows], rtol=1e-13, atol=0)
