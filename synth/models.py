"""Synthetic Wannier models: seeded draws of H(R), C(R) and g(Re,Rp).

Conventions shared by every consumer (they are conventions of the *inputs*,
not steps of the method):

* Lengths in Angstrom, masses in amu, energies in eV.
* ``lattice`` rows are the primitive vectors a_1, a_2, a_3 (Cartesian).
* Real-space vectors are integer triples n, R = n_1 a_1 + n_2 a_2 + n_3 a_3.
* k and q are given in reduced (crystal) coordinates, k = sum_i x_i b_i.
* ``h[r, i, j]``   = H_ij(R_r)                         complex,   [nR][nw][nw]
* ``ifc[r, a, b]`` = C_{a b}(R_r), a = 3*kappa+alpha  real,      [nR][3nat][3nat]
  (force constants *without* the mass factor, paper Eq. IFC1)
* ``g[e, p, a, i, j]`` = g^{a}_{ij}(Re_e, Rp_p)        complex,  [nRe][nRp][3nat][nw][nw]
  (paper Eq. eph_mat_wann, units eV/Angstrom)

Readings of the paper's silent points that shape these draws (Sec. "Wigner-Seitz
supercell", Eq. wann_ws): one least-distance image per Born-von Karman cell, ties
broken by the lexicographically smallest integer triple, unit weights; H and C
are left zero on vectors whose inverse is not in the set so that H(k) and D(q)
stay Hermitian.
"""
from __future__ import annotations

import dataclasses
import itertools
from typing import Optional

import numpy as np

A_SI = 5.389      # Angstrom, silicon lattice constant of the Sec. 5.4 example
A_GAAS = 5.556    # Angstrom, GaAs lattice constant of the Sec. 5.1 example
M_SI = 28.0855
M_GA = 69.723
M_AS = 74.9216


@dataclasses.dataclass
class Model:
    lattice: np.ndarray            # (3,3) rows a_i, Angstrom
    tau: np.ndarray                # (nat,3) Cartesian atom positions, Angstrom
    mass: np.ndarray               # (nat,) amu
    nw: int
    wf_centres: np.ndarray         # (nw,3) Cartesian, Angstrom (informational)
    re: np.ndarray                 # (nRe,3) int32, vectors of H(R)
    w_re: np.ndarray               # (nRe,) weights
    h: np.ndarray                  # (nRe,nw,nw) complex128
    rp_ph: np.ndarray              # (nRph,3) int32, vectors of C(R)
    w_rp_ph: np.ndarray
    ifc: np.ndarray                # (nRph,3nat,3nat) float64
    re_g: np.ndarray               # (nReg,3) int32
    w_re_g: np.ndarray
    rp_g: np.ndarray               # (nRpg,3) int32
    w_rp_g: np.ndarray
    g: np.ndarray                  # (nReg,nRpg,3nat,nw,nw) complex128
    zstar: Optional[np.ndarray] = None   # (nat,3,3) Born charges, Z*[kappa, beta, alpha]
    eps_inf: Optional[np.ndarray] = None  # (3,3) high-frequency dielectric tensor
    name: str = "model"

    @property
    def nat(self) -> int:
        return int(self.tau.shape[0])

    @property
    def nmodes(self) -> int:
        return 3 * self.nat

    def volume(self) -> float:
        return float(abs(np.linalg.det(self.lattice)))


def fcc_lattice(a: float) -> np.ndarray:
    return 0.5 * a * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])


def sc_lattice(a: float) -> np.ndarray:
    return a * np.eye(3)


def ws_vectors(lattice: np.ndarray, n_grid) -> np.ndarray:
    """One least-distance lattice vector per Born-von Karman cell of an
    n1 x n2 x n3 supercell (paper Sec. "Wigner-Seitz supercell", Eq. wann_ws,
    with all Wannier centres taken at the origin).  Ties go to the
    lexicographically smallest integer triple.  Returns int32 (N,3) in cell
    enumeration order."""
    n_grid = tuple(int(x) for x in np.broadcast_to(np.asarray(n_grid), (3,)))
    out = []
    shifts = list(itertools.product(range(-2, 3), repeat=3))
    scale = float(np.max(np.linalg.norm(lattice, axis=1)))
    for cell in itertools.product(*(range(n) for n in n_grid)):
        best = None
        best_d = None
        for s in shifts:
            cand = tuple(cell[i] + n_grid[i] * s[i] for i in range(3))
            d = float(np.linalg.norm(np.asarray(cand, float) @ lattice))
            if best is None or d < best_d - 1e-9 * scale or (
                abs(d - best_d) <= 1e-9 * scale and cand < best
            ):
                best, best_d = cand, d
        out.append(best)
    return np.asarray(out, dtype=np.int32)


def _cnormal(rng, shape, real=False):
    if real:
        return rng.standard_normal(shape)
    z = rng.standard_normal(shape + (2,))
    return (z[..., 0] + 1j * z[..., 1]) / np.sqrt(2.0)


def _index(vecs: np.ndarray) -> dict:
    return {tuple(int(x) for x in v): i for i, v in enumerate(vecs)}


def hermitian_hoppings(rng, vecs, lattice, nw, amp, decay, onsite=None, real=False,
                       nn_hop=None):
    """H(R) = onsite*delta_R0 + nn_hop*delta_{R in NN} + amp * X(R) * exp(-|R|/decay),
    with X(-R) = X(R)^H drawn once per +/-R pair; zero where -R is not in the
    set.  nn_hop (length nw, real) is a diagonal nearest-neighbour hopping that
    gives each band a smooth, parabolic-like extremum."""
    idx = _index(vecs)
    h = np.zeros((len(vecs), nw, nw), dtype=np.complex128)
    draws = _cnormal(rng, (len(vecs), nw, nw), real=real)
    dists = np.linalg.norm(vecs.astype(float) @ lattice, axis=1)
    dnn = np.min(dists[dists > 1e-9])
    for i, v in enumerate(vecs):
        j = idx.get(tuple(-int(x) for x in v))
        if j is None or j < i:
            continue
        dist = float(np.linalg.norm(v.astype(float) @ lattice))
        x = amp * np.exp(-dist / decay) * draws[i]
        if i == j:
            x = 0.5 * (x + x.conj().T)
            if onsite is not None:
                x = x + np.diag(onsite)
            h[i] = x
        else:
            if nn_hop is not None and abs(dist - dnn) < 1e-6 * dnn:
                x = x + np.diag(np.asarray(nn_hop, dtype=float))
            h[i] = x
            h[j] = x.conj().T
    return h


def spring_ifc(rng, vecs, lattice, tau, amp, decay):
    """Force constants as a sum of random positive semi-definite 3x3 springs,
    one per unordered bond (kappa@0, kappa'@R).  Each spring K adds
    -K to C_{kk'}(R) and C_{k'k}(-R), +K to C_kk(0) and C_k'k'(0), so the
    acoustic sum rule and Hermiticity of D(q) hold by construction."""
    nat = tau.shape[0]
    idx = _index(vecs)
    zero = idx[(0, 0, 0)]
    c = np.zeros((len(vecs), 3 * nat, 3 * nat))
    for i, v in enumerate(vecs):
        tv = tuple(int(x) for x in v)
        j = idx.get(tuple(-x for x in tv))
        if j is None:
            continue
        for ka in range(nat):
            for kb in range(nat):
                if ka > kb:
                    continue
                if ka == kb and not (tv > tuple(-x for x in tv)):
                    continue  # self-bonds: count each +/-R once, never R=0
                b = rng.standard_normal((3, 3))
                d = float(np.linalg.norm(v.astype(float) @ lattice + tau[kb] - tau[ka]))
                k = amp * np.exp(-d / decay) * (b @ b.T) / 3.0
                sa, sb = slice(3 * ka, 3 * ka + 3), slice(3 * kb, 3 * kb + 3)
                c[i, sa, sb] -= k
                c[j, sb, sa] -= k.T
                c[zero, sa, sa] += k
                c[zero, sb, sb] += k
    return c


def coupling_tensor(rng, re, rp, lattice, nm, nw, amp, decay, real=False):
    """g(Re,Rp) = amp * Z * exp(-(|Re|+|Rp|)/decay), Z complex (or real) normal."""
    de = np.linalg.norm(re.astype(float) @ lattice, axis=1)
    dp = np.linalg.norm(rp.astype(float) @ lattice, axis=1)
    z = _cnormal(rng, (len(re), len(rp), nm, nw, nw), real=real)
    env = amp * np.exp(-(de[:, None] + dp[None, :]) / decay)
    return z * env[:, :, None, None, None]


def make_model(
    *,
    lattice,
    tau,
    mass,
    nw,
    n_grid,
    seed,
    a_h,
    a_g,
    s_k,
    decay,
    gap_onsite=3.0,
    band_step=0.5,
    nn_hop=0.12,
    real=False,
    zstar=None,
    eps_inf=None,
    name="model",
    draw_g=True,
):
    """Draw a complete synthetic model on the least-distance set of an
    n_grid^3 supercell (the same set for H, C, Re and Rp).  draw_g=False
    leaves g empty (it is drawn last, so H and C are unchanged)."""
    lattice = np.asarray(lattice, float)
    tau = np.asarray(tau, float)
    mass = np.asarray(mass, float)
    nat = tau.shape[0]
    rng = np.random.default_rng(seed)
    vecs = ws_vectors(lattice, n_grid)
    nr = len(vecs)
    nv = nw // 2
    lev = np.arange(max(nv, nw - nv), dtype=float)
    # valence levels below -gap_onsite, conduction levels above +gap_onsite;
    # NN hopping of opposite signs puts the VB maximum and CB minimum at Gamma
    onsite = np.concatenate([-(gap_onsite + band_step * lev[:nv])[::-1],
                             gap_onsite + band_step * lev[:nw - nv]])
    hop = np.concatenate([(nn_hop * (1 + 0.25 * lev[:nv]))[::-1],
                          -nn_hop * (1 + 0.25 * lev[:nw - nv])])
    h = hermitian_hoppings(rng, vecs, lattice, nw, a_h, decay, onsite=onsite, real=real,
                           nn_hop=hop)
    ifc = spring_ifc(rng, vecs, lattice, tau, s_k, decay)
    g = (coupling_tensor(rng, vecs, vecs, lattice, 3 * nat, nw, a_g, decay, real=real) if draw_g
         else np.zeros((0,), dtype=np.complex128))
    wf = np.repeat(tau, int(np.ceil(nw / nat)), axis=0)[:nw]
    ones = np.ones(nr)
    return Model(
        lattice=lattice, tau=tau, mass=mass, nw=nw, wf_centres=wf,
        re=vecs, w_re=ones, h=h, rp_ph=vecs.copy(), w_rp_ph=ones.copy(), ifc=ifc,
        re_g=vecs.copy(), w_re_g=ones.copy(), rp_g=vecs.copy(), w_rp_g=ones.copy(), g=g,
        zstar=None if zstar is None else np.asarray(zstar, float),
        eps_inf=None if eps_inf is None else np.asarray(eps_inf, float),
        name=name,
    )


def random_points(seed: int, n: int) -> np.ndarray:
    """n uniform random points in reduced coordinates [0,1)^3 (NumPy PCG64)."""
    return np.random.default_rng(seed).random((n, 3))


def random_positions(seed: int, nat: int, a: float, min_sep: float) -> np.ndarray:
    """nat atoms at uniform random positions in a simple-cubic cell of side a,
    drawn one at a time and redrawn while closer than min_sep (minimum image) to
    an earlier atom."""
    rng = np.random.default_rng(seed)
    pos = []
    while len(pos) < nat:
        x = rng.random(3) * a
        ok = True
        for y in pos:
            d = x - y
            d -= a * np.round(d / a)
            if np.linalg.norm(d) < min_sep:
                ok = False
                break
        if ok:
            pos.append(x)
    return np.array(pos)


def cauchy_points(seed: int, n: int, gamma: float):
    """n q points concentrated near Gamma for importance sampling of the q sum
    (Sec. 4.3): each reduced coordinate from a Cauchy distribution of scale
    gamma wrapped onto [-1/2, 1/2).  Returns (q, w) with w = 1/(n p(q)), p the
    product of the wrapped densities p(x) = sinh(2 pi gamma)/(cosh(2 pi gamma) -
    cos(2 pi x)), so that sum_q w f(q) estimates the zone average of f."""
    rng = np.random.default_rng(seed)
    u = rng.random((n, 3))
    x = gamma * np.tan(np.pi * (u - 0.5))
    x = x - np.floor(x + 0.5)
    s, c = np.sinh(2 * np.pi * gamma), np.cosh(2 * np.pi * gamma)
    p = np.prod(s / (c - np.cos(2 * np.pi * x)), axis=1)
    return x, 1.0 / (n * p)


# ---------------------------------------------------------------- counter-based coupling draws
# For models too large to draw on the host (the 6^3 large cell's g(Re,Rp) is
# 1.1e10 complex entries), the coupling tensor is drawn from a counter-based
# generator that the device reproduces bit for bit: Philox4x32-10 (Salmon,
# Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC11),
# and an exact integer Irwin-Hall sum of twelve uniform 32-bit words as the
# (approximately) normal variate.  Complex entry t (flat index over
# [Re][Rp][3nat][nw][nw]) takes the six blocks with 64-bit counter 6t + b
# (b = 0..5, words 2 and 3 of the counter zero) under the key (seed mod 2^32,
# seed div 2^32): blocks 0-2 give the real part, blocks 3-5 the imaginary part,
#   x = (sum of the 12 words) * 2^-32 - 6      (exact in double),
# and the stored value is float(env[Re][Rp] * x) (complex64; env is a given
# amplitude per (Re, Rp), so both sides round the same product).

_PHILOX_M = (np.uint64(0xD2511F53), np.uint64(0xCD9E8D57))
_PHILOX_W = (np.uint32(0x9E3779B9), np.uint32(0xBB67AE85))


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32 with 10 rounds on uint32 arrays (counter words c0..c3, key
    words k0, k1); returns the four output words."""
    c = [np.asarray(x, dtype=np.uint32) for x in (c0, c1, c2, c3)]
    k0 = np.asarray(k0, dtype=np.uint32).copy()
    k1 = np.asarray(k1, dtype=np.uint32).copy()
    lo32 = np.uint64(0xFFFFFFFF)
    with np.errstate(over="ignore"):
        for _ in range(10):
            p0 = _PHILOX_M[0] * c[0].astype(np.uint64)
            p1 = _PHILOX_M[1] * c[2].astype(np.uint64)
            hi0, lo0 = (p0 >> np.uint64(32)).astype(np.uint32), (p0 & lo32).astype(np.uint32)
            hi1, lo1 = (p1 >> np.uint64(32)).astype(np.uint32), (p1 & lo32).astype(np.uint32)
            c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
            k0 = k0 + _PHILOX_W[0]
            k1 = k1 + _PHILOX_W[1]
    return c


def counter_normals(t, seed):
    """The real and imaginary variates of complex entries t (int64 array) under
    the scheme above: two float64 arrays, each an Irwin-Hall(12) - 6 value."""
    t = np.asarray(t, dtype=np.uint64)
    k0 = np.uint32(seed & 0xFFFFFFFF)
    k1 = np.uint32((seed >> 32) & 0xFFFFFFFF)
    out = []
    for half in range(2):
        acc = np.zeros(t.shape, dtype=np.uint64)
        for b in range(3 * half, 3 * half + 3):
            ctr = t * np.uint64(6) + np.uint64(b)
            words = philox4x32_10((ctr & np.uint64(0xFFFFFFFF)).astype(np.uint32),
                                  (ctr >> np.uint64(32)).astype(np.uint32), 0, 0, k0, k1)
            for w in words:
                acc += w.astype(np.uint64)
        out.append(acc.astype(np.float64) * 2.0 ** -32 - 6.0)
    return out[0], out[1]


def coupling_envelope(re, rp, lattice, amp, decay):
    """env[Re][Rp] = amp exp(-(|Re| + |Rp|)/decay) / sqrt(2): the amplitude of
    the counter-drawn g (a complex variate of unit variance per entry)."""
    de = np.linalg.norm(np.asarray(re, float) @ lattice, axis=1)
    dp = np.linalg.norm(np.asarray(rp, float) @ lattice, axis=1)
    return amp * np.exp(-(de[:, None] + dp[None, :]) / decay) / np.sqrt(2.0)


def counter_coupling(env, per, seed, entries=None):
    """Complex64 g from the counter scheme: the whole tensor [nRe][nRp][per]
    (small models), or, with entries (flat complex indices), those entries."""
    n_re, n_rp = env.shape
    t = np.arange(n_re * n_rp * per, dtype=np.int64) if entries is None else np.asarray(entries, dtype=np.int64)
    xr, xi = counter_normals(t, seed)
    a = env.reshape(-1)[t // per]
    g = (a * xr).astype(np.float32) + 1j * (a * xi).astype(np.float32)
    return g.astype(np.complex64) if entries is not None else g.astype(np.complex64).reshape(n_re, n_rp, per)


def make_counter_model(name: str, *, n_grid=None, nw=None, seed=None, full=True):
    """The model of a workload with g(Re,Rp) drawn by the counter scheme instead
    of NumPy's generator; returns (model, env, seed).  With full=False the
    model's g is left empty (the device draws it; the host evaluates chosen
    entries with counter_coupling)."""
    c = CONFIGS[name]
    m = make_config_model(name, n_grid=n_grid, nw=nw, draw_g=False)
    a = c["a"]
    env = coupling_envelope(m.re_g, m.rp_g, m.lattice, c["a_g"], 1.5 * a)
    seed = int(c["seed"] + 500 if seed is None else seed)
    per = m.nmodes * m.nw * m.nw
    if full:
        g = counter_coupling(env, per, seed).astype(np.complex128)
        m = dataclasses.replace(m, g=g.reshape(len(m.re_g), len(m.rp_g), m.nmodes, m.nw, m.nw))
    return m, env, seed


SEED_BASE = 20020205

# Workload definitions.  Physical parameters follow the readings listed in the
# design notes: Gaussian delta exp(-(x/s)^2)/(sqrt(pi) s), mu at the midpoint of
# the onsite levels (0 eV, inside the gap), omega_cut = 1e-4 eV.  The coupling
# amplitude a_g of the Si-like models gives |g| of tens of meV and relaxation
# rates of ~0.1/fs near the band edge, so RK4 with dt = 1 fs is stable.
CONFIGS = {
    "tiny": dict(
        lattice="fcc", a=A_SI, nat=2, masses=(M_SI, M_SI), nw=4, n_grid=4,
        a_h=0.05, nn_hop=0.12, a_g=0.5, s_k=0.375, seed=SEED_BASE + 1,
        nk=200, nq=500, T=300.0, sigma=0.010, mu=0.0, omega_cut=1e-4,
    ),
    "si": dict(
        lattice="fcc", a=A_SI, nat=2, masses=(M_SI, M_SI), nw=8, n_grid=8,
        a_h=0.015, nn_hop=0.1, a_g=0.09, s_k=0.1, seed=SEED_BASE + 2,
        nk=5000, nq=1_000_000, window=0.3, T=300.0, sigma=0.005, mu=0.0, omega_cut=1e-4,
    ),
    "gaas": dict(
        lattice="fcc", a=A_GAAS, nat=2, masses=(M_GA, M_AS), nw=8, n_grid=8,
        a_h=0.015, nn_hop=0.1, a_g=0.09, s_k=0.1, seed=SEED_BASE + 3,
        real=True, zstar=2.1, eps_inf=10.9, k_grid=100, window=0.2, T=300.0, sigma=0.005,
        n_c=1e17, omega_cut=1e-4,
    ),
    # just past the per-pair register kernels (nw > 16, 3nat > 12): the
    # batched-GEMM path at a size the oracle handles
    "wide": dict(
        lattice="sc", a=6.0, nat=5, masses=(12.0, 14.0, 16.0, 28.0), nw=20, n_grid=3,
        a_h=0.05, nn_hop=0.12, a_g=0.3, s_k=0.3, seed=SEED_BASE + 4, positions="random", min_sep=1.8,
        T=300.0, sigma=0.02, mu=0.0, omega_cut=1e-4,
    ),
    # large cell: 40 atoms (120 modes), 64 Wannier functions on a simple-cubic
    # 10 Angstrom cell; the real-space sets default to the 3^3 supercell (the
    # 6^3 set's g(Re,Rp) alone is 183 GB in complex64)
    "cell": dict(
        lattice="sc", a=10.0, nat=40, masses=(12.0, 14.0, 16.0, 28.0), nw=64, n_grid=3,
        a_h=0.015, nn_hop=0.1, a_g=0.05, s_k=0.1, seed=SEED_BASE + 5, positions="random", min_sep=1.8,
        nk=2000, nq=200_000, window=0.3, T=300.0, sigma=0.005, mu=0.0, omega_cut=1e-4,
    ),
    "dyn": dict(
        lattice="fcc", a=A_SI, nat=2, masses=(M_SI, M_SI), nw=8, n_grid=8,
        a_h=0.015, nn_hop=0.1, a_g=0.09, s_k=0.1, seed=SEED_BASE + 2,
        k_grid=80, n_states=20_000, T=300.0, sigma=0.008, dt=1.0, n_steps=1000,
        ckpt_every=50, f0_peak=0.1, f0_centre=0.3, f0_width=0.05, omega_cut=1e-4,
    ),
}


def make_config_model(name: str, *, real=None, n_grid=None, nw=None, draw_g=True) -> Model:
    c = CONFIGS[name]
    if real is None:
        real = bool(c.get("real", False))
    a = c["a"]
    lat = fcc_lattice(a) if c["lattice"] == "fcc" else sc_lattice(a)
    if c.get("positions") == "random":
        tau = random_positions(c["seed"] + 17, c["nat"], a, c["min_sep"])
        masses = np.resize(np.asarray(c["masses"], float), c["nat"])
    else:
        tau = np.array([[0.0, 0.0, 0.0], [0.25 * a, 0.25 * a, 0.25 * a]])[: c["nat"]]
        masses = np.array(c["masses"])
    zstar = eps = None
    if "zstar" in c:
        z = c["zstar"]
        zstar = np.stack([z * np.eye(3), -z * np.eye(3)])
        eps = c["eps_inf"] * np.eye(3)
    return make_model(
        lattice=lat, tau=tau, mass=masses,
        nw=nw or c["nw"], n_grid=n_grid or c["n_grid"], seed=c["seed"],
        a_h=c["a_h"], a_g=c["a_g"], s_k=c["s_k"], nn_hop=c["nn_hop"], decay=1.5 * a, real=real,
        zstar=zstar, eps_inf=eps, name=name, draw_g=draw_g,
    )
