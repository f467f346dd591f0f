"""Pins of the oracle's e-ph interpolation, Froehlich term and rates (paper
Sec. 2.2.3, 2.3, Eqs. eph_mat, eph_mat_wann2, e_ph_long, scatter_rate, BTE_W)
against closed forms, unitary invariants, gauge/time-reversal symmetry and
hand-reducible special cases."""
import copy
import math

import numpy as np
import pytest
import torch

import synth
from oracle import eph, interp
from oracle.units import E2_4PIEPS0, HBAR2_AMU_A2, HBAR_EV_FS, KB_EV


def test_direct_double_sum_equals_factored(tiny_model):
    k = synth.random_points(21, 2)
    q = synth.random_points(22, 2)
    direct = eph.g_wannier_direct(tiny_model, k, q)
    fact = eph.g_wannier(tiny_model, k, q)
    scale = float(fact.abs().max())
    assert float((direct - fact).abs().max()) <= 1e-13 * scale


def test_single_re_rp_closed_form(tiny_model):
    """With g nonzero at one (Re,Rp) only, g^W(k,q) = e^{i(k.Re+q.Rp)} g(Re,Rp)."""
    m = copy.deepcopy(tiny_model)
    e0, p0 = 17, 41
    keep = m.g[e0, p0].copy()
    m.g[:] = 0
    m.g[e0, p0] = keep
    k = synth.random_points(23, 3)
    q = synth.random_points(24, 4)
    gw = eph.g_wannier(m, k, q).numpy()
    ph = np.exp(2j * np.pi * (k @ m.re_g[e0])[:, None] + 2j * np.pi * (q @ m.rp_g[p0])[None, :])
    assert np.allclose(gw, ph[:, :, None, None, None] * keep[None, None], atol=1e-14)


def test_rotation_commutator_model_has_zero_diagonal(tiny_model):
    """If g^{x}(Re,0) = c_x [H(Re) A - A H(Re)] then g^W(k,q) = c_x [H(k), A]-like
    and, at q = 0, U^dag(k) [H(k) A - A H(k)] U(k) = (eps_m - eps_n) (U^dag A U)_mn:
    the band-diagonal vanishes.  A wrong side or conjugation of U breaks it."""
    m = copy.deepcopy(tiny_model)
    rng = np.random.default_rng(5)
    a = rng.standard_normal((m.nw, m.nw)) + 1j * rng.standard_normal((m.nw, m.nw))
    c = rng.standard_normal(m.nmodes) + 1j * rng.standard_normal(m.nmodes)
    m.g[:] = 0
    ip0 = int(np.nonzero((m.rp_g == 0).all(axis=1))[0][0])
    assert (m.re_g == m.re).all()
    for e in range(len(m.re_g)):
        comm = m.h[e] @ a - a @ m.h[e]
        m.g[e, ip0] = c[:, None, None] * comm[None]
    k = synth.random_points(25, 4)
    blk = eph.eph_pipeline(m, k, np.zeros((1, 3)), omega_cut=1e-4)   # optical modes at Gamma
    g = blk["g"][:, 0]                                           # (k, nu, m, n)
    diag = torch.diagonal(g, dim1=-2, dim2=-1).abs()
    assert float(diag.max()) < 1e-12 * float(g.abs().max())
    assert float(g.abs().max()) > 1e-3


def test_unitary_free_identity(tiny_model):
    """sum_mn |g_mn,nu|^2 = hbar/(2 omega) || sum_x e^{x}_nu/sqrt(M_x) g^{W,x} ||_F^2:
    the band rotation is unitary, so it cannot change the Frobenius norm."""
    k = synth.random_points(26, 3)
    q = synth.random_points(27, 5)
    blk = eph.eph_pipeline(tiny_model, k, q)
    gw = eph.g_wannier(tiny_model, k, q)
    minv = 1.0 / np.sqrt(np.repeat(tiny_model.mass, 3))
    proj = torch.einsum("qxv,kqxij->kqvij", blk["evec"] * torch.as_tensor(minv)[None, :, None], gw)
    lhs = (blk["g"].abs() ** 2).sum(dim=(-1, -2))
    rhs = (proj.abs() ** 2).sum(dim=(-1, -2)) * HBAR2_AMU_A2 / (2 * blk["omega"])[None]
    assert torch.allclose(lhs, rhs, rtol=1e-12)


def test_eigenvector_free_identity(tiny_model):
    """sum_nu 2 omega_nu |g_mn,nu|^2 / hbar = sum_x |g^{H,x}_mn|^2 / M_x over all
    3 nat modes (the mode-eigenvector matrix is unitary)."""
    k = synth.random_points(28, 3)
    q = synth.random_points(29, 4)
    blk = eph.eph_pipeline(tiny_model, k, q, omega_cut=-1.0)
    gw = eph.g_wannier(tiny_model, k, q)
    gh = eph.band_basis(gw, blk["u_kq"], blk["u_k"])
    lhs = (2 * blk["omega"][None, :, :, None, None] / HBAR2_AMU_A2 * blk["g"].abs() ** 2).sum(dim=2)
    m = torch.as_tensor(np.repeat(tiny_model.mass, 3))
    rhs = (gh.abs() ** 2 / m[None, None, :, None, None]).sum(dim=2)
    assert torch.allclose(lhs, rhs, rtol=1e-11)


def test_gauge_invariance_random_eigenvector_phases(tiny_model):
    k = synth.random_points(30, 2)
    q = synth.random_points(31, 3)
    blk = eph.eph_pipeline(tiny_model, k, q)
    gw = eph.g_wannier(tiny_model, k, q)
    rng = np.random.default_rng(0)
    ph_k = torch.as_tensor(np.exp(2j * np.pi * rng.random(blk["u_k"].shape[:-2] + (tiny_model.nw,))))
    ph_kq = torch.as_tensor(np.exp(2j * np.pi * rng.random(blk["u_kq"].shape[:-2] + (tiny_model.nw,))))
    gh1 = eph.band_basis(gw, blk["u_kq"], blk["u_k"])
    gh2 = eph.band_basis(gw, blk["u_kq"] * ph_kq[..., None, :], blk["u_k"] * ph_k[..., None, :])
    assert torch.allclose(gh1.abs(), gh2.abs(), atol=1e-13)


def test_gauge_invariance_in_degenerate_subspaces(tiny_model):
    """Doubled model H1 (x) I2, g1 (x) I2: every band is two-fold degenerate; a
    random U(2) rotation inside each degenerate pair leaves the group sums of
    |g|^2 (Eq. g_abs over the group) unchanged."""
    m = tiny_model
    md = copy.deepcopy(m)
    md.nw = 2 * m.nw
    md.h = np.stack([np.kron(x, np.eye(2)) for x in m.h])
    md.g = np.kron(m.g, np.eye(2))
    k = synth.random_points(32, 2)
    q = synth.random_points(33, 3)
    blk = eph.eph_pipeline(md, k, q)
    gw = eph.g_wannier(md, k, q)
    rng = np.random.default_rng(1)

    def rand_u2(shape):
        z = rng.standard_normal(shape + (2, 2)) + 1j * rng.standard_normal(shape + (2, 2))
        qm, _ = np.linalg.qr(z)
        return qm

    def rotate(u):
        r = rand_u2(u.shape[:-2] + (m.nw,))
        out = u.clone()
        for b in range(m.nw):
            out[..., 2 * b:2 * b + 2] = u[..., 2 * b:2 * b + 2] @ torch.as_tensor(r[..., b, :, :])
        return out

    def group_sums(gh):
        g2 = gh.abs() ** 2
        return g2.reshape(g2.shape[:-2] + (m.nw, 2, m.nw, 2)).sum(dim=(-1, -3))

    gh1 = eph.band_basis(gw, blk["u_kq"], blk["u_k"])
    gh2 = eph.band_basis(gw, rotate(blk["u_kq"]), rotate(blk["u_k"]))
    assert torch.allclose(group_sums(gh1), group_sums(gh2), atol=1e-12)
    assert not torch.allclose(gh1.abs(), gh2.abs(), atol=1e-6)


def _group_sum_modes(model, k, q):
    """Gauge-invariant |g_nu|^2 summed over degenerate band groups at k, k+q and
    degenerate mode groups at q (thresholds 1e-4 eV)."""
    blk = eph.eph_pipeline(model, k, q)
    g2 = blk["g"].abs() ** 2
    return g2.sum(dim=(-1, -2))                                # sum over all bands


def test_time_reversal_real_model(tiny_real_model, tiny_model):
    """Real H(R), C(R), g(Re,Rp): |g_nu|(-k,-q) = |g_nu|(k,q) (Sec. 4.1 symmetry
    argument, time reversal).  The complex model must fail (negative control)."""
    k = synth.random_points(34, 3)
    q = synth.random_points(35, 3)
    a = eph.g_abs_modes(eph.g2(tiny_real_model, k, q))
    b = eph.g_abs_modes(eph.g2(tiny_real_model, -k, -q))
    assert torch.allclose(a, b, rtol=1e-11)
    a = eph.g_abs_modes(eph.g2(tiny_model, k, q))
    b = eph.g_abs_modes(eph.g2(tiny_model, -k, -q))
    assert not torch.allclose(a, b, rtol=1e-3)


# --------------------------------------------------------------- Froehlich

def _polar_model():
    m = synth.make_config_model("gaas", n_grid=4, nw=4)
    a = synth.models.A_GAAS
    return m, dict(alpha_ewald=(2 * np.pi / a) ** 2, gcut=4 * 2 * np.pi / a)


def test_frohlich_small_q_limit():
    """As q -> 0 the G = 0 term dominates: |q| C^{kappa a}(q) ->
    i e^2/(eps0 Omega) [qhat.Z*_kappa]_a / (qhat.eps.qhat), with O(|q|) corrections."""
    m, pol = _polar_model()
    lat = m.lattice
    bvec = 2 * np.pi * np.linalg.inv(lat).T
    qhat = np.array([0.3, -0.5, 0.81])
    qhat /= np.linalg.norm(qhat)
    omega_cell = abs(np.linalg.det(lat))
    lim = np.zeros(6, complex)
    for kap in range(2):
        lim[3 * kap:3 * kap + 3] = 1j * 4 * np.pi * E2_4PIEPS0 / omega_cell * (qhat @ m.zstar[kap]) / (qhat @ m.eps_inf @ qhat)
    errs = []
    for t in (1e-3, 1e-4):
        qc = t * qhat
        qred = (qc @ np.linalg.inv(bvec))[None, :]
        c = eph.frohlich(m, qred, **pol)[0].numpy()
        errs.append(np.abs(c * t - lim).max() / np.abs(lim).max())
    assert errs[1] < 2e-3
    assert errs[1] < 0.2 * errs[0]                                # linear convergence


def test_frohlich_periodic_and_time_reversal():
    m, pol = _polar_model()
    q = synth.random_points(36, 4)
    c = eph.frohlich(m, q, **pol)
    c_shift = eph.frohlich(m, q + np.array([1.0, -2.0, 1.0]), **pol)
    assert torch.allclose(c, c_shift, rtol=1e-12, atol=1e-14)
    c_minus = eph.frohlich(m, -q, **pol)
    assert torch.allclose(c_minus, c.conj(), rtol=1e-12, atol=1e-14)


# --------------------------------------------------------------- rates

def _flat_model(eps_levels, omega0, mass, gamma):
    """Flat bands (only H(0) nonzero), Einstein phonons (only C(0) nonzero),
    coupling only at (Re,Rp) = (0,0): every (k,q) pair is the same."""
    nw = len(eps_levels)
    kspring = omega0 ** 2 * mass / HBAR2_AMU_A2
    z = np.zeros((1, 3), np.int32)
    return synth.Model(
        lattice=synth.fcc_lattice(5.0), tau=np.zeros((1, 3)), mass=np.array([mass]), nw=nw,
        wf_centres=np.zeros((nw, 3)), re=z, w_re=np.ones(1), h=np.diag(eps_levels).astype(complex)[None],
        rp_ph=z, w_rp_ph=np.ones(1), ifc=kspring * np.eye(3)[None],
        re_g=z, w_re_g=np.ones(1), rp_g=z, w_rp_g=np.ones(1), g=gamma[None, None].astype(complex))


def test_rates_flat_band_einstein_closed_form():
    """Two flat levels 0 and 0.05 eV, Einstein phonons at 0.05 eV (three
    degenerate modes), constant coupling gamma^{a}_{mn}.  The q-sum collapses:
    Gamma_n = (2pi/hbar) sum_m hbar^2/(2 M hw) sum_a |gamma^a_mn|^2
              [delta(e_n - hw - e_m)(1 + N - f_m) + delta(e_n + hw - e_m)(N + f_m)]."""
    hw, mass, sigma, temp, mu = 0.05, 20.0, 0.004, 300.0, -0.3
    rng = np.random.default_rng(3)
    gam = rng.standard_normal((3, 2, 2)) + 1j * rng.standard_normal((3, 2, 2))
    m = _flat_model([0.0, 0.05], hw, mass, gam)
    k = synth.random_points(40, 2)
    q = synth.random_points(41, 7)
    gamma, gmode = eph.rates(m, k, q, temp=temp, mu=mu, sigma=sigma)
    kt = KB_EV * temp
    nb = 1.0 / (math.exp(hw / kt) - 1.0)
    lev = [0.0, 0.05]
    f = [1.0 / (math.exp((e - mu) / kt) + 1.0) for e in lev]

    def delta(x):
        return math.exp(-(x / sigma) ** 2) / (math.sqrt(math.pi) * sigma)

    for n in range(2):
        tot = 0.0
        for mm in range(2):
            c2 = sum(abs(gam[a, mm, n]) ** 2 for a in range(3))
            amp = HBAR2_AMU_A2 / (2 * mass * hw) * c2
            tot += amp * (delta(lev[n] - hw - lev[mm]) * (1 + nb - f[mm]) + delta(lev[n] + hw - lev[mm]) * (nb + f[mm]))
        ref = 2 * math.pi / HBAR_EV_FS * tot
        assert np.allclose(gamma[:, n].numpy(), ref, rtol=1e-12)
    assert torch.allclose(gmode.sum(dim=2), gamma, rtol=1e-14)


def test_rates_positive_and_quadratic_in_g(tiny_model):
    k = synth.random_points(42, 3)
    q = synth.random_points(43, 40)
    par = dict(temp=300.0, mu=0.0, sigma=0.05)
    g1, gm1 = eph.rates(tiny_model, k, q, **par)
    assert float(gm1.min()) >= 0.0
    assert float(g1.max()) > 0.0
    m2 = copy.deepcopy(tiny_model)
    m2.g = 2.0 * m2.g
    g2v, _ = eph.rates(m2, k, q, **par)
    assert torch.allclose(g2v, 4.0 * g1, rtol=1e-12)


# --------------------------------------------------------------- atom relabelling

def _relabel_atom(model, kap, t):
    """The same crystal with atom kap taken from the neighbouring cell:
    tau'_kap = tau_kap + T, T = t . (a_1, a_2, a_3).  Atom (kap, cell R) of the
    new labels is atom (kap, cell R + T) of the old ones, so the tensors that
    index an atomic displacement by its cell are re-indexed (Sec. 2.2.2, 2.2.3):
      C'_{k k'}(R) = C_{k k'}(R + T_k' - T_k),   g'^{k a}(Re, Rp) = g^{k a}(Re, Rp + T_k),
    with T_k = T for k = kap and 0 otherwise.  The R lists grow by the shifted
    vectors (the oracle takes any list); entries with no source stay zero."""
    t = np.asarray(t, dtype=np.int64)
    nat = model.nat
    shift = [t if k == kap else np.zeros(3, np.int64) for k in range(nat)]
    m = copy.deepcopy(model)
    m.tau = model.tau.copy()
    m.tau[kap] = model.tau[kap] + t @ model.lattice

    def union(vecs, extra):
        seen = {tuple(int(x) for x in v): None for v in vecs}
        for e in extra:
            for v in vecs:
                seen.setdefault(tuple(int(x) for x in (v + e)), None)
        return np.array(list(seen), dtype=np.int32)

    old_ph = {tuple(int(x) for x in v): i for i, v in enumerate(model.rp_ph)}
    rp_ph = union(model.rp_ph, [t, -t])
    ifc = np.zeros((len(rp_ph),) + model.ifc.shape[1:])
    for i, r in enumerate(rp_ph):
        for k in range(nat):
            for kk in range(nat):
                src = old_ph.get(tuple(int(x) for x in (r + shift[kk] - shift[k])))
                if src is not None:
                    ifc[i, 3 * k:3 * k + 3, 3 * kk:3 * kk + 3] = model.ifc[src, 3 * k:3 * k + 3, 3 * kk:3 * kk + 3]
    m.rp_ph, m.w_rp_ph, m.ifc = rp_ph, np.ones(len(rp_ph)), ifc
    old_g = {tuple(int(x) for x in v): i for i, v in enumerate(model.rp_g)}
    rp_g = union(model.rp_g, [-t])
    g = np.zeros((model.g.shape[0], len(rp_g)) + model.g.shape[2:], dtype=complex)
    for i, r in enumerate(rp_g):
        for k in range(nat):
            src = old_g.get(tuple(int(x) for x in (r + shift[k])))
            if src is not None:
                g[:, i, 3 * k:3 * k + 3] = model.g[:, src, 3 * k:3 * k + 3]
    m.rp_g, m.w_rp_g, m.g = rp_g, np.ones(len(rp_g)), g
    return m


def _mode_group_sums(blk):
    """|g|^2 summed over all bands and over degenerate mode groups (1e-4 eV)."""
    g2 = (blk["g"].abs() ** 2).sum(dim=(-1, -2))                # (k, q, nu)
    om = blk["omega"].numpy()
    out = torch.zeros_like(g2)
    for iq in range(om.shape[0]):
        grp = interp.degenerate_groups(om[iq], 1e-4)
        for gi in grp:
            out[:, iq, gi[0]] = g2[:, iq, gi].sum(dim=-1)
    return out


@pytest.mark.parametrize("long_range_only", [False, True])
def test_atom_relabelling_leaves_coupling_unchanged(long_range_only):
    """Moving atom kappa by a lattice vector T (and re-indexing the force
    constants and g(Re,Rp) to match) describes the same crystal: D(q) becomes
    L D(q) L^dag with L = diag(e^{iq.T_kappa}), the eigenvectors pick up
    e^{iq.T_kappa} on atom kappa, the short-range g^W picks up e^{-iq.T_kappa},
    and so must the Froehlich term through its phase e^{-i tau_kappa.(q+G)}
    (Eq. e_ph_long).  |g_mn,nu| is then unchanged; the opposite sign of that
    phase would leave a factor e^{2iq.T} on atom kappa's long-range part.
    Checked with the short- and long-range parts together and with the
    long-range part alone (g(Re,Rp) = 0), and with the LO-TO part of D(q) on,
    whose phase e^{i(q+G).(tau_k - tau_k')} must follow the same relabelling."""
    m, pol = _polar_model()
    if long_range_only:
        m = copy.deepcopy(m)
        m.g[:] = 0
    k = synth.random_points(90, 2)
    q = synth.random_points(91, 5)
    for lo_to in (False, True):
        polar = dict(pol, lo_to=lo_to)
        ref = eph.eph_pipeline(m, k, q, polar)
        for kap, t in ((1, (1, 0, 0)), (0, (0, -1, 2))):
            mr = _relabel_atom(m, kap, t)
            got = eph.eph_pipeline(mr, k, q, polar)
            assert torch.allclose(got["omega"], ref["omega"], rtol=1e-10, atol=1e-12)
            a, b = _mode_group_sums(got), _mode_group_sums(ref)
            assert float(b.max()) > 0
            assert float((a - b).abs().max()) <= 1e-10 * float(b.max())
            # the relabelled model really differs: its long-range term alone
            # changes by the phase e^{-iq.T} on atom kappa
            c0 = eph.frohlich(m, q, **pol)
            c1 = eph.frohlich(mr, q, **pol)
            assert not torch.allclose(c0, c1, atol=1e-6 * float(c0.abs().max()))


# --------------------------------------------------------------- polar split

def test_polar_split_parts_add_up_and_reduce_correctly():
    """The rates are linear in |g|^2: the long-range part and the remainder
    add up to the full rates for the same q set (each weighted sum of the
    polar split estimates its own part).  The long-range part equals the full
    rates of the model with g(Re,Rp) = 0; on a model without Born charges'
    effect (Z* = 0) it vanishes and the remainder is the full rate."""
    m, pol = _polar_model()
    k = synth.random_points(95, 3)
    q = synth.random_points(96, 40)
    par = dict(temp=300.0, mu=0.0, sigma=0.06, polar=pol)
    full, fm = eph.rates(m, k, q, **par)
    lr, lm = eph.rates(m, k, q, part="polar", **par)
    rest, rm = eph.rates(m, k, q, part="rmpol", **par)
    assert float(full.max()) > 0 and float(lr.max()) > 0
    assert torch.allclose(lr + rest, full, rtol=1e-12, atol=1e-14 * float(full.max()))
    assert torch.allclose(lm + rm, fm, rtol=1e-12, atol=1e-14 * float(fm.max()))
    m0 = copy.deepcopy(m)
    m0.g[:] = 0
    lr0, _ = eph.rates(m0, k, q, **par)
    assert torch.allclose(lr, lr0, rtol=1e-13)
    mz = copy.deepcopy(m)
    mz.zstar = 0.0 * m.zstar
    lz, _ = eph.rates(mz, k, q, part="polar", **par)
    fz, _ = eph.rates(mz, k, q, **par)
    rz, _ = eph.rates(mz, k, q, part="rmpol", **par)
    assert float(lz.abs().max()) == 0.0
    assert torch.allclose(rz, fz, rtol=1e-14)
